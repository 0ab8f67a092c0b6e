"""Full solves with the restart of Algorithm 2 itself on every engine, against the oracle.

The restart rule of Algorithm 2 (eq. update-next-iterate) multiplies every one of
(y, x, s, tau, kappa, theta) by sqrt(gamma) when the inner test passes.  Each
engine applies it in its own code (the LDS-resident loop, the streamed
one-workgroup loop, the grid engine's column kernel, the sparse engine), so each
one runs a whole solve here with restart_rule = ABIP_RESTART_SQRT and is compared
with oracle.solve(restart_rule="sqrt"): the same status, the same number of outer
steps, the ADMM count within 1%, and the returned x element by element.  FP32
bulk runs are compared by status and by the FP64 recheck of their result.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.abip import Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


ENGINES = {
    "lds": dict(),
    "streamed": dict(lds_resident=0),
    "grid": dict(engine=2),
}


_CACHE = {}


def _ref(lp, A=None):
    """oracle.solve with the sqrt restart, cached per instance across the parametrisations."""
    A = lp["A"] if A is None else A
    key = (A.shape, float(np.asarray(A).sum()), float(lp["b"].sum()), float(lp["c"].sum()))
    if key not in _CACHE:
        _CACHE[key] = oracle.solve(A, lp["b"], lp["c"], Settings(restart_rule="sqrt"))
    return _CACHE[key]


def _check_fp64(lp, A, ref, x, y, s, info):
    assert info["status"] == ref["status"], (info["status_name"], ref["status_name"])
    assert info["ipm_iters"] == ref["ipm_iters"], (info["ipm_iters"], ref["ipm_iters"])
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"]), \
        (info["admm_iters"], ref["admm_iters"])
    if ref["status"] == oracle.SOLVED:
        kk = oracle.kkt_relative(A, lp["b"], lp["c"], x, y, s)
        assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
        np.testing.assert_allclose(x, ref["x"], atol=1e-6 * (1 + np.abs(ref["x"]).max()))
        np.testing.assert_allclose(y, ref["y"], atol=1e-6 * (1 + np.abs(ref["y"]).max()))


@pytest.mark.parametrize("engine", list(ENGINES))
@pytest.mark.parametrize("seed", [4, 5])
def test_sqrt_restart_solve_matches_oracle(engine, seed):
    print(f"sqrt restart solve engine={engine} seed={seed}", flush=True)
    lp = lpgen.config0(seed)
    ref = _ref(lp)
    kw = dict(ENGINES[engine])
    if "engine" in kw:
        kw["engine"] = abip.ABIP_ENGINE_GRID
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        abip.abip_default_settings(restart_rule=abip.ABIP_RESTART_SQRT, **kw))
    x, y, s, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], ref["admm_iters"], info["ipm_iters"], ref["ipm_iters"],
          flush=True)
    _check_fp64(lp, lp["A"], ref, _np(x), _np(y), _np(s), info)
    w.free()


@pytest.mark.parametrize("engine", list(ENGINES))
def test_sqrt_restart_certificate(engine):
    """A planted Farkas LP: the restart scales y too, and the certificate must survive it."""
    lp = lpgen.dense_farkas_infeasible(20, 50, 3)
    ref = _ref(lp)
    kw = dict(ENGINES[engine])
    if "engine" in kw:
        kw["engine"] = abip.ABIP_ENGINE_GRID
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        abip.abip_default_settings(restart_rule=abip.ABIP_RESTART_SQRT, **kw))
    x, y, s, info = abip.abip_solve(w)
    print(engine, info["status_name"], info["admm_iters"], ref["admm_iters"], flush=True)
    assert info["status"] == ref["status"] == oracle.PRIMAL_INFEASIBLE
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"])
    yv = _np(y)
    assert abs(lp["b"] @ yv - 1.0) < 1e-9
    assert np.linalg.norm(lp["A"].T @ yv + _np(s)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001
    w.free()


@pytest.mark.parametrize("lds", [1, 0])
def test_sqrt_restart_batch(lds):
    """Feasible and infeasible LPs in one batched launch, LDS-resident and streamed."""
    lps = [lpgen.dense_planted(12, 30, 2), lpgen.dense_planted(50, 100, 5), lpgen.dense_farkas_infeasible(20, 50, 3)]
    w = abip.abip_setup_batch([lp["A"] for lp in lps], [lp["b"] for lp in lps], [lp["c"] for lp in lps],
                              abip.abip_default_settings(restart_rule=abip.ABIP_RESTART_SQRT, lds_resident=lds))
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    for lp, x, y, s, info in zip(lps, xs, ys, ss, infos):
        ref = _ref(lp)
        print(lp["m"], lp["n"], info["status_name"], info["admm_iters"], ref["admm_iters"], flush=True)
        assert info["status"] == ref["status"]
        assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"])
        if ref["status"] == oracle.SOLVED:
            _check_fp64(lp, lp["A"], ref, _np(x), _np(y), _np(s), info)
    w.free()


@pytest.mark.parametrize("engine", ["lds", "streamed", "grid"])
def test_sqrt_restart_fp32_bulk(engine):
    """FP32 bulk + FP64 polish under the sqrt restart: same status, and the returned
    point meets the tolerance in an FP64 recheck and sits at the planted optimum."""
    lp = lpgen.config0(7)
    kw = dict(ENGINES[engine])
    if "engine" in kw:
        kw["engine"] = abip.ABIP_ENGINE_GRID
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        abip.abip_default_settings(restart_rule=abip.ABIP_RESTART_SQRT,
                                                   precision=abip.ABIP_PREC_FP32_POLISH, **kw))
    x, y, s, info = abip.abip_solve(w)
    print(engine, info["status_name"], info["admm_iters"], info["admm_iters_fp64"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
    w.free()


@pytest.mark.parametrize("lds", [1, 0])
def test_sqrt_restart_sparse_matches_oracle(lds):
    lp = lpgen.sparse_planted(60, 150, 1, density=0.05)
    Ac = lp["A_csr"]
    A = sp.csr_matrix((Ac["data"], Ac["indices"], Ac["indptr"]), shape=Ac["shape"])
    ref = _ref(lp, A.toarray())
    w = abip.abip_setup(A, lp["b"], lp["c"],
                        abip.abip_default_settings(cg_tol=1e-13, cg_max_iters=2000, cg_rule=1, lds_resident=lds,
                                                   restart_rule=abip.ABIP_RESTART_SQRT))
    x, y, s, info = abip.abip_solve(w)
    print("sparse", lds, info["status_name"], info["admm_iters"], ref["admm_iters"], flush=True)
    _check_fp64(lp, A.toarray(), ref, _np(x), _np(y), _np(s), info)
    w.free()
