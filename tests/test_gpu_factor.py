"""The cached factorization (Section 4.4) on the matrix cores, via the C ABI.

G = I + A A^T, its blocked Cholesky factor and G^{-1} = W^T W are formed with
64 x 64 tiles on v_mfma_f64_16x16x4f64 for every LP of a handle at once.  The
tile edges are where such code goes wrong: m below, at and just past multiples
of 64, and LPs of different tile counts in one batch.  Each LP's linear step
(I+Q)^{-1} w (which uses G^{-1} and the border built from it) is compared with
the oracle's dense solve of the assembled I + Q.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.abip import Problem

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


EDGE_M = [1, 2, 5, 63, 64, 65, 127, 128, 129, 191, 192, 257, 400]


def test_factor_tile_edges_in_one_batch():
    lps = [lpgen.dense_planted(m, max(2 * m, 3), 100 + m) for m in EDGE_M]
    w = abip.abip_setup_batch([lp["A"] for lp in lps], [lp["b"] for lp in lps], [lp["c"] for lp in lps])
    rng = np.random.default_rng(7)
    for k, lp in enumerate(lps):
        m, n = lp["m"], lp["n"]
        win = rng.standard_normal(m + n + 2)
        ref = oracle.DenseIQSolver(Problem(lp["A"], lp["b"], lp["c"])).solve(win)
        got = _np(abip.abip_apply_iq(w, k, win))
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"m={m} n={n} rel err {err:.2e}", flush=True)
        assert err < 1e-11, (m, err)
        got_t = _np(abip.abip_apply_iq(w, k, win, transpose=True))
        Q = oracle.assemble_Q(Problem(lp["A"], lp["b"], lp["c"]))
        ref_t = np.linalg.solve(np.eye(m + n + 2) - Q, win)
        assert np.abs(got_t - ref_t).max() <= 1e-10 * np.abs(ref_t).max(), m
    w.free()


@pytest.mark.parametrize("m,n,seed", [(2100, 4600, 3), (4200, 9000, 4)])
def test_factor_grid_engine_linear_step(m, n, seed):
    """One large LP (grid engine): the same factorization over many tiles and the
    border's products over the whole GPU."""
    lp = lpgen.dense_planted(m, n, seed)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID))
    win = np.random.default_rng(seed).standard_normal(m + n + 2)
    ref = oracle.SchurIQSolver(Problem(lp["A"], lp["b"], lp["c"])).solve(win)
    got = _np(abip.abip_apply_iq(w, 0, win))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"grid m={m} n={n} rel err {err:.2e}", flush=True)
    assert err < 1e-10, err
    w.free()
