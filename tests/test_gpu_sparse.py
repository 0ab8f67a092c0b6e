"""Sparse engine (A in CSR, CG on I + A A^T) against the FP64 oracle, via the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.abip import Problem, Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _csr(lp):
    A = lp["A_csr"]
    return sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])


def _tight(**kw):
    return abip.abip_default_settings(cg_tol=1e-13, cg_max_iters=2000, cg_rule=1, **kw)


@pytest.mark.parametrize("m,n,seed,density", [(40, 90, 1, 0.08), (150, 420, 2, 0.02), (600, 1700, 3, 0.004)])
@pytest.mark.parametrize("rule", ["heuristic", "sqrt"])
@pytest.mark.parametrize("lds,gram", [(1, 0), (0, 0), (1, 1)])
def test_sparse_iterations_match_oracle(m, n, seed, density, rule, lds, gram):
    """Fixed updates from the same restarted iterate: the CG-based step equals the exact one,
    with the CSR rows held in LDS (lds=1) and read from global memory (lds=0), or with the CG
    multiplying by the explicit G~ = A A^T (gram=1)."""
    print(f"sparse iterate m={m} n={n} seed={seed} rule={rule} lds={lds} gram={gram}", flush=True)
    lp = lpgen.sparse_planted(m, n, seed, density=density)
    A = _csr(lp)
    prob = Problem(A.toarray(), lp["b"], lp["c"])
    s = Settings(restart_rule=rule)
    st = oracle.initial_state(prob, s)
    st = oracle.restart(st, s.gamma, rule)
    w = abip.abip_setup(A, lp["b"], lp["c"], _tight(restart_rule=0 if rule == "heuristic" else 1, lds_resident=lds,
                                                    sparse_gram=gram))
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    solver = oracle.SchurIQSolver(prob)
    N = 25
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    abip.abip_iterate(w, 0, N)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    scale = 1.0 + np.abs(st.u()).max()
    assert np.abs(_np(y) - st.y).max() <= 1e-9 * scale
    assert np.abs(_np(x) - st.x).max() <= 1e-9 * scale
    assert np.abs(_np(sv) - st.s).max() <= 1e-9 * scale
    for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
        assert abs(sc[key] - ref) <= 1e-9 * scale, (key, sc[key], ref)
    np.testing.assert_allclose(_np(x) * _np(sv), st.mu, rtol=1e-8)


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("lds,gram", [(1, 0), (0, 0), (1, 1)])
def test_sparse_solve_matches_oracle(seed, lds, gram):
    lp = lpgen.sparse_planted(60, 150, seed, density=0.05)
    A = _csr(lp)
    ref = oracle.solve(A.toarray(), lp["b"], lp["c"], Settings())
    w = abip.abip_setup(A, lp["b"], lp["c"], _tight(lds_resident=lds, sparse_gram=gram))
    x, y, s, info = abip.abip_solve(w)
    print(info, ref["admm_iters"], flush=True)
    G = (A @ A.T).tocsr()
    G.eliminate_zeros()
    if gram == 1:
        assert info["gram_nnz"] >= G.nnz          # structural entries (exact cancellations kept)
    else:
        assert info["gram_nnz"] == 0
    assert info["status"] == abip.ABIP_SOLVED == ref["status"]
    kk = oracle.kkt_relative(A.toarray(), lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"])
    assert info["cg_iters"] > 0


def test_sparse_matches_dense_engine():
    lp = lpgen.dense_planted(30, 70, 6)
    A = sp.csr_matrix(lp["A"])
    wd = abip.abip_setup(lp["A"], lp["b"], lp["c"])
    xd, yd, sd, infod = abip.abip_solve(wd)
    ws = abip.abip_setup(A, lp["b"], lp["c"], _tight())
    xs, ys, ss, infos = abip.abip_solve(ws)
    print(infod["admm_iters"], infos["admm_iters"], infos["cg_iters"], flush=True)
    assert infos["status"] == infod["status"] == abip.ABIP_SOLVED
    assert abs(infos["admm_iters"] - infod["admm_iters"]) <= max(3, 0.01 * infod["admm_iters"])
    np.testing.assert_allclose(_np(xs), _np(xd), atol=1e-6 * (1 + np.abs(_np(xd)).max()))


def test_sparse_certificates():
    for lp in [lpgen.dense_farkas_infeasible(20, 50, 3), lpgen.toy_dual_infeasible()]:
        A = sp.csr_matrix(lp["A"])
        ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
        w = abip.abip_setup(A, lp["b"], lp["c"], _tight())
        x, y, s, info = abip.abip_solve(w)
        print(lp["status"], info["status_name"], info["admm_iters"], ref["admm_iters"], flush=True)
        assert info["status"] == ref["status"]
        if info["status"] == abip.ABIP_PRIMAL_INFEASIBLE:
            yv = _np(y)
            assert abs(lp["b"] @ yv - 1.0) < 1e-9
            assert np.linalg.norm(lp["A"].T @ yv + _np(s)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001
        else:
            xv = _np(x)
            assert abs(lp["c"] @ xv + 1.0) < 1e-9 and np.all(xv >= 0)


def test_sparse_boundary_errors():
    lp = lpgen.sparse_planted(30, 60, 4, density=0.1)
    A = lp["A_csr"]
    bad = dict(A, indptr=A["indptr"].copy())
    bad["indptr"][5] = bad["indptr"][6] + 1            # decreasing row pointer
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(bad, lp["b"], lp["c"])
    assert e.value.code == abip.ABIP_E_INVALID
    bad = dict(A, indices=A["indices"].copy())
    bad["indices"][3] = 60                              # column out of range
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(bad, lp["b"], lp["c"])
    assert e.value.code == abip.ABIP_E_INVALID
    bad = dict(A, data=A["data"].copy())
    bad["data"][7] = np.nan
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(bad, lp["b"], lp["c"])
    assert e.value.code == abip.ABIP_E_NONFINITE
    w = abip.abip_setup(A, lp["b"], lp["c"])
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_backward(w, np.ones(60))
    assert e.value.code == abip.ABIP_E_STATE


def test_sparse_lds_and_global_passes_agree():
    """A CSR LP spread over many workgroups (several CG passes per update, default CG
    schedule): the LDS-resident and global-memory passes reach the same status, KKT
    tolerance and objective, with iteration counts within a few percent."""
    lp = lpgen.sparse_planted(3000, 9000, 11, density=3e-3)
    A = _csr(lp)
    res = {}
    for lds in (1, 0):
        w = abip.abip_setup(A, lp["b"], lp["c"], abip.abip_default_settings(lds_resident=lds))
        x, y, s, info = abip.abip_solve(w)
        print("lds", lds, info["admm_iters"], info["cg_iters"], info["kernel_ms"], flush=True)
        assert info["status"] == abip.ABIP_SOLVED
        xh, yh, sh = _np(x), _np(y), _np(s)
        pres = np.linalg.norm(A @ xh - lp["b"]) / (1 + np.linalg.norm(lp["b"]))
        dres = np.linalg.norm(A.T @ yh + sh - lp["c"]) / (1 + np.linalg.norm(lp["c"]))
        assert max(pres, dres) <= 1e-6 * 1.01, (pres, dres)
        assert abs(lp["c"] @ xh - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
        res[lds] = info["admm_iters"]
        w.free()
    assert abs(res[1] - res[0]) <= max(5, 0.05 * res[0]), res
