"""The triangular-solve form of the linear step (ABIP_LIN_TRSV) against the oracle.

With lin_solver = ABIP_LIN_TRSV the one-workgroup engine keeps the Cholesky
factor L of G = I + A A^T (Section 4.4's cached factorization) and solves
L z = t, L^T a = z by blocked substitution on every update instead of
multiplying by G^{-1}.  Fixed updates are compared element by element with the
oracle's Schur solve (which uses a Cholesky solve per application) on shapes
whose m falls below, on and past the 64-row blocks and spans one to four
256-row chunks; full solves take the oracle's iteration count; the FP32 phase
agrees with the G^{-1} form run on the same FP32 data to the FP32 model's level.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.abip import Problem, Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _iterate(lp, st, N, lin, fp32=False):
    s = abip.abip_default_settings(lin_solver=lin, precision=abip.ABIP_PREC_FP32_POLISH if fp32 else
                                   abip.ABIP_PREC_FP64)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    abip.abip_iterate(w, 0, N, use_fp32=fp32)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    w.free()
    return _np(y), _np(x), _np(sv), sc


@pytest.mark.parametrize("m,n,seed", [(20, 45, 1), (63, 140, 2), (64, 150, 3), (65, 150, 4), (200, 450, 5),
                                      (400, 900, 6), (700, 1500, 7)])
def test_trsv_updates_match_oracle(m, n, seed):
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings()
    st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, "heuristic")
    solver = oracle.SchurIQSolver(prob)
    N = 30
    st = st0.copy()
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    y, x, sv, sc = _iterate(lp, st0, N, abip.ABIP_LIN_TRSV)
    scale = 1.0 + np.abs(st.u()).max()
    err = max(np.abs(y - st.y).max(), np.abs(x - st.x).max(), np.abs(sv - st.s).max()) / scale
    print(f"{m}x{n}: trsv vs oracle {err:.2e}", flush=True)
    assert err <= 1e-10
    assert abs(sc["tau"] - st.tau) <= 1e-10 * scale and abs(sc["theta"] - st.theta) <= 1e-10 * scale


@pytest.mark.parametrize("m,n,seed", [(64, 150, 3), (400, 900, 6)])
def test_trsv_fp32_phase_matches_inverse_form(m, n, seed):
    """FP32 data: L (FP32) by substitution and G^{-1} (FP32) by a product round
    differently; both stay within the FP32-data model's distance of the FP64 step."""
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings()
    st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, "heuristic")
    N = 20
    st = st0.copy()
    solver = oracle.SchurIQSolver(prob)
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    scale = 1.0 + np.abs(st.u()).max()
    a = _iterate(lp, st0, N, abip.ABIP_LIN_TRSV, fp32=True)
    b = _iterate(lp, st0, N, abip.ABIP_LIN_AUTO, fp32=True)
    ea = max(np.abs(a[0] - st.y).max(), np.abs(a[1] - st.x).max()) / scale
    eb = max(np.abs(b[0] - st.y).max(), np.abs(b[1] - st.x).max()) / scale
    print(f"{m}x{n}: FP32 trsv {ea:.2e}, FP32 inverse {eb:.2e}", flush=True)
    assert ea <= 1e-3 and eb <= 1e-3
    assert ea <= 10 * eb + 1e-6


@pytest.mark.parametrize("m,n,seed", [(50, 100, 1), (300, 650, 3)])
def test_trsv_full_solve(m, n, seed):
    lp = lpgen.dense_planted(m, n, seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"])
    s = abip.abip_default_settings(lin_solver=abip.ABIP_LIN_TRSV)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    print(f"{m}x{n}: trsv {info['status_name']} iters {info['admm_iters']} oracle {ref['admm_iters']}, "
          f"lds_mode {info['lds_mode']}", flush=True)
    assert info["status_name"] == ref["status_name"] == "solved"
    assert info["lds_mode"] == 0
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(5, ref["admm_iters"] // 100)
    k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    w.free()


def test_trsv_batch_and_rejections():
    lps = lpgen.batch(10, 12, m_lo=20, m_hi=300)
    s = abip.abip_default_settings(lin_solver=abip.ABIP_LIN_TRSV, precision=abip.ABIP_PREC_FP32_POLISH)
    w = abip.abip_setup_batch([l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps], s)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    w0 = abip.abip_setup_batch([l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps],
                               abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    _, _, _, infos0 = abip.abip_solve_batch(w0)
    for lp, info, i0 in zip(lps, infos, infos0):
        assert info["status"] == i0["status"]
    w.free()
    w0.free()
    lp = lpgen.dense_planted(300, 900, 1)
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(
            lin_solver=abip.ABIP_LIN_TRSV, engine=abip.ABIP_ENGINE_GRID))
    assert e.value.code == abip.ABIP_E_INVALID
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(lin_solver=abip.ABIP_LIN_TRSV, bb=1))
    assert e.value.code == abip.ABIP_E_INVALID
