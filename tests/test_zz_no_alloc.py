"""The allocation-free entry point against abip_setup + abip_solve, via the C ABI.

abip_solve_noalloc carves every device buffer out of the library's fixed scratch
region.  It runs the same kernels on the same data layout as abip_setup followed
by abip_solve, so its results must equal theirs bitwise.  Two calls in a row
(the second on a smaller LP) check that a call leaves nothing behind that the
next one reads: the region keeps the previous call's contents.
"""
import math

import numpy as np
import pytest
import torch

import lpgen

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _reference(lp, settings):
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], settings)
    x, y, s, info = abip.abip_solve(w)
    w.free()
    return _np(x), _np(y), _np(s), info


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_setup_and_solve_twice(prec):
    p = abip.ABIP_PREC_FP32_POLISH if prec == "fp32" else abip.ABIP_PREC_FP64
    st = abip.abip_default_settings(precision=p)
    # the first call is the largest allowed shape class in use here, the second smaller
    for lp in [lpgen.dense_planted(200, 900, 11), lpgen.dense_planted(30, 70, 12)]:
        print(f"noalloc {prec} m={lp['m']} n={lp['n']}", flush=True)
        x, y, s, info = abip.abip_solve_noalloc(lp["A"], lp["b"], lp["c"], st)
        xr, yr, sr, ir = _reference(lp, st)
        print("  status", info["status_name"], ir["status_name"], "iters", info["admm_iters"], ir["admm_iters"],
              flush=True)
        assert info["status"] == ir["status"] == abip.ABIP_SOLVED
        assert info["admm_iters"] == ir["admm_iters"]
        assert info["admm_iters_fp64"] == ir["admm_iters_fp64"]
        np.testing.assert_array_equal(_np(x), xr)
        np.testing.assert_array_equal(_np(y), yr)
        np.testing.assert_array_equal(_np(s), sr)
        assert info["err_vs_fp64"] == ir["err_vs_fp64"] and info["err_vs_fp64"] <= 1e-6
        assert math.isnan(info["kernel_ms"])


def test_noalloc_infeasible_then_feasible():
    """A certificate first, then a feasible LP: the second call must not see the first's state."""
    st = abip.abip_default_settings()
    for lp in [lpgen.dense_farkas_infeasible(40, 100, 3), lpgen.toy_two_var()]:
        x, y, s, info = abip.abip_solve_noalloc(lp["A"], lp["b"], lp["c"], st)
        xr, yr, sr, ir = _reference(lp, st)
        assert info["status"] == ir["status"]
        assert info["admm_iters"] == ir["admm_iters"]
        np.testing.assert_array_equal(np.nan_to_num(_np(y), nan=7.0), np.nan_to_num(yr, nan=7.0))
        np.testing.assert_array_equal(np.nan_to_num(_np(x), nan=7.0), np.nan_to_num(xr, nan=7.0))


def test_noalloc_rejects_what_it_cannot_hold():
    big = lpgen.dense_planted(257, 600, 1)
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_solve_noalloc(big["A"], big["b"], big["c"])
    assert e.value.code == abip.ABIP_E_DIM
    wide = lpgen.dense_planted(10, 1025, 1)
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_solve_noalloc(wide["A"], wide["b"], wide["c"])
    assert e.value.code == abip.ABIP_E_DIM
    lp = lpgen.dense_planted(10, 30, 1)
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_solve_noalloc(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID))
    assert e.value.code == abip.ABIP_E_INVALID
    # still usable after the rejections
    x, y, s, info = abip.abip_solve_noalloc(lp["A"], lp["b"], lp["c"])
    assert info["status"] == abip.ABIP_SOLVED


def test_noalloc_largest_shape():
    """m = 256, n = 1024: the scratch region's sizing case."""
    lp = lpgen.dense_planted(256, 1024, 5)
    st = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
    x, y, s, info = abip.abip_solve_noalloc(lp["A"], lp["b"], lp["c"], st)
    xr, yr, sr, ir = _reference(lp, st)
    assert info["status"] == ir["status"] == abip.ABIP_SOLVED
    np.testing.assert_array_equal(_np(x), xr)
    torch.cuda.synchronize()
