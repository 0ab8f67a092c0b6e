"""The sparse, basis-pursuit and differentiable workloads at their full sizes, in the launch
configuration bench.py times, checked through what holds at any size (status, the Section 4.1
residuals recomputed on the host, the objective against the planted optimum, finite gradients
and converged adjoint solves) and, where the oracle computes it in seconds, against the oracle
on a sample.  All through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import lpgen
import oracle

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _check_solution(A, lp, x, y, s, obj_bar):
    x, y, s = _np(x), _np(y), _np(s)
    kk = oracle.kkt_relative(A, lp["b"], lp["c"], x, y, s)
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6 * (1 + 1e-9), kk
    assert np.all(x >= 0) and np.all(s >= 0)
    assert abs(lp["c"] @ x - lp["pstar"]) <= obj_bar * (1 + abs(lp["pstar"]))


def test_sparse_10000_by_30000_cg_engine():
    print("sparse 10000 x 30000", flush=True)
    lp = lpgen.sparse_planted(10000, 30000, 1, density=1e-3)
    A = lp["A_csr"]
    As = sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])
    w = abip.abip_setup(As, lp["b"], lp["c"], abip.abip_default_settings())
    x, y, s, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], info["cg_iters"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    _check_solution(As.toarray(), lp, x, y, s, 1e-5)      # the pinned checker takes a dense A (2.4 GB)


@pytest.mark.parametrize("mirror", [1, 0])
def test_basis_pursuit_2000_by_16000_grid_engine_fp32_bulk(mirror):
    """Both column passes of the bench: A0 read once per pair (the default for A = [A0, -A0])
    and every column streamed."""
    print(f"basis pursuit 2000 x 16000 grid_mirror={mirror}", flush=True)
    lp = lpgen.basis_pursuit(2000, 8000, 400, 2)
    A = torch.tensor(lp["A"], device="cuda")
    w = abip.abip_setup(A, lp["b"], lp["c"], abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH,
                                                                         grid_mirror=mirror))
    x, y, s, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], info["admm_iters_fp64"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    assert info["grid_mirror"] == mirror
    _check_solution(lp["A"], lp, x, y, s, 1e-5)
    # the planted sparse signal is recovered: x+ - x- against x_true
    xv = _np(x)
    xr = xv[:8000] - xv[8000:]
    assert np.linalg.norm(xr - lp["x_true"]) <= 1e-3 * (1 + np.linalg.norm(lp["x_true"]))


def test_differentiable_batch_64_of_200_by_500():
    print("differentiable 64 x (200 x 500)", flush=True)
    lps = lpgen.diff_batch(64, 200, 500, 4)
    As = [torch.tensor(lp["A"], device="cuda") for lp in lps]
    bs = [torch.tensor(lp["b"], device="cuda") for lp in lps]
    cs = [torch.tensor(lp["c"], device="cuda") for lp in lps]
    ws = [torch.tensor(lp["w"], device="cuda") for lp in lps]
    w = abip.abip_setup_batch(As, bs, cs, abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    assert all(i["status"] == abip.ABIP_SOLVED for i in infos)
    dcs, dbs, _ = abip.abip_backward_batch(w, ws)
    for k in range(len(lps)):
        assert np.all(np.isfinite(_np(dcs[k]))) and np.all(np.isfinite(_np(dbs[k])))
        it, rr = abip.abip_backward_stats(w, k)
        assert rr <= 1e-11, (k, it, rr)
    # a sample against the dense KKT adjoint at the same final iterate (measured about 1e-11;
    # the system is ill conditioned at mu ~ 1e-8, so the bar leaves room for other draws)
    for k in (0, 31, 63):
        lp = lps[k]
        yv, xv, sv, sc = abip.abip_get_state(w, k)
        st = oracle.State(_np(yv), _np(xv), sc["tau"], sc["theta"], _np(sv), sc["kappa"], sc["mu"])
        lam = oracle.kkt_adjoint(lp["A"], lp["b"], lp["c"], st, lp["w"])
        ref = oracle.contract_adjoint(lp["A"], lp["b"], lp["c"], st, lam)
        e = np.abs(_np(dbs[k]) - ref["db"]).max() / (1 + np.abs(ref["db"]).max())
        print(k, "db vs KKT adjoint", e, flush=True)
        assert e <= 1e-7


def test_paper_random_4000_by_20000_scaled_grid_engine():
    """The largest size of the paper's random-LP table (eps 1e-3) as the bench runs it: FP64 after
    10 Ruiz rounds; the solve must pass the Section 4.1 tests on the LP as given (host recheck)."""
    print("paper random 4000 x 20000, scaled", flush=True)
    lp = lpgen.paper_random(4000, 20000, 1)
    A = torch.tensor(lp["A"], device="cuda")
    s = abip.abip_default_settings(eps=1e-3, engine=abip.ABIP_ENGINE_GRID, precision=abip.ABIP_PREC_FP64,
                                   scale_iters=10)
    w = abip.abip_setup(A, lp["b"], lp["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], info["err_vs_fp64"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-3 * (1 + 1e-9), kk
    assert np.all(_np(x) >= 0) and np.all(_np(sv) >= 0)
    assert info["err_vs_fp64"] <= 1e-3 * (1 + 1e-9)
    pobj = float(lp["c"] @ _np(x))
    assert abs(pobj - lp["pstar"]) <= 1e-2 * (1 + abs(lp["pstar"])), (pobj, lp["pstar"])
    w.free()
