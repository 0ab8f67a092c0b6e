"""LDS-resident variant of the batched engine: A and G^{-1} held in LDS, or A
alone held in LDS with G^{-1} read from device memory on every pass (LPs whose
A fits but not together with G^{-1}).

The same iteration as the streamed variant, with sums formed in another order:
fixed-iteration iterates are compared with the FP64 oracle and with the
streamed variant (lds_resident=0) on the same LP; full solves are compared with
the oracle's status and the KKT tolerance.  Shapes cover one and two columns
per thread, FP64 data that fits and FP64 data that does not (the FP32 phase then
hands over to the streamed variant).
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


# (m, n, seed, FP64 data fits in LDS); 90 x 180: the FP64 phase holds only A in LDS
# (G^{-1} read from the pool); 128 x 256: the FP32 phase does, and FP64 data does not fit
SHAPES = [(39, 97, 21, True), (76, 159, 23, True), (23, 400, 13, True), (100, 200, 14, False),
          (90, 180, 17, True), (128, 256, 16, False)]


def _iterate(lp, st, N, lds, fp32, rule):
    s = abip.abip_default_settings(restart_rule=0 if rule == "heuristic" else 1, lds_resident=lds,
                                   precision=abip.ABIP_PREC_FP32_POLISH if fp32 else abip.ABIP_PREC_FP64)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    abip.abip_iterate(w, 0, N, use_fp32=fp32)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    return _np(y), _np(x), _np(sv), sc


@pytest.mark.parametrize("m,n,seed,fits64", SHAPES)
@pytest.mark.parametrize("rule", ["heuristic", "sqrt"])
def test_lds_iterations_match_oracle_and_streamed(m, n, seed, fits64, rule):
    print(f"lds iterate m={m} n={n} seed={seed} rule={rule}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings(alpha=1.8, gamma=0.5, restart_rule=rule)
    st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, rule)
    solver = oracle.SchurIQSolver(prob)
    N = 60
    st = st0.copy()
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    scale = 1.0 + np.abs(st.u()).max()
    # FP64 data: LDS-resident (when it fits) and streamed against the oracle
    for lds in (1, 0):
        y, x, sv, sc = _iterate(lp, st0, N, lds, False, rule)
        for got, ref in [(y, st.y), (x, st.x), (sv, st.s)]:
            assert np.abs(got - ref).max() <= 1e-10 * scale, lds
        for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
            assert abs(sc[key] - ref) <= 1e-10 * scale, (lds, key, sc[key], ref)
        np.testing.assert_allclose(x * sv, st.mu, rtol=1e-9)     # Theorem 3.1: x o s = mu / beta
    # FP32 data: both variants round A and G^{-1} the same way, so they agree far
    # below the FP32 rounding of the data itself
    a = _iterate(lp, st0, N, 1, True, rule)
    b = _iterate(lp, st0, N, 0, True, rule)
    for ga, gb in zip(a[:3], b[:3]):
        assert np.abs(ga - gb).max() <= 1e-9 * scale
    for key in ("tau", "kappa", "theta"):
        assert abs(a[3][key] - b[3][key]) <= 1e-9 * scale, key
    # and they stay at the FP32 distance from the FP64 oracle
    assert np.abs(a[1] - st.x).max() <= 1e-3 * scale


def _check_solution(lp, x, y, s, info):
    if lp["status"] == "solved":
        assert info["status"] == abip.ABIP_SOLVED
        k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
        assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6, k
    else:
        assert info["status"] == abip.ABIP_PRIMAL_INFEASIBLE
        yv = _np(y)
        assert abs(lp["b"] @ yv - 1.0) < 1e-9
        assert np.linalg.norm(lp["A"].T @ yv + _np(s)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001


@pytest.mark.parametrize("m,n,seed,fits64", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_lds_solve_matches_oracle(m, n, seed, fits64, prec):
    print(f"lds solve m={m} n={n} seed={seed} prec={prec}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"])
    assert ref["status_name"] == "solved"
    p = abip.ABIP_PREC_FP32_POLISH if prec == "fp32" else abip.ABIP_PREC_FP64
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(precision=p))
    x, y, s, info = abip.abip_solve(w)
    print(" iters", info["admm_iters"], "fp64", info["admm_iters_fp64"], "oracle", ref["admm_iters"], flush=True)
    _check_solution(lp, x, y, s, info)
    np.testing.assert_allclose(_np(x), ref["x"], atol=1e-4 * (1 + np.abs(ref["x"]).max()))
    if prec == "fp64":
        # the same iteration in the same precision: the counts agree up to the
        # iterations where rounding order decides a test
        assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(5, ref["admm_iters"] // 50)


def test_lds_batch_matches_streamed_and_kkt():
    """A mixed batch (LDS-resident and streamed LPs, feasible and infeasible):
    both variants give the planted status and the KKT tolerance."""
    lps = lpgen.batch(40, 21, m_lo=20, m_hi=160)
    As, bs, cs = [l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps]
    for lds in (1, 0):
        w = abip.abip_setup_batch(As, bs, cs, abip.abip_default_settings(
            precision=abip.ABIP_PREC_FP32_POLISH, lds_resident=lds))
        xs, ys, ss, infos = abip.abip_solve_batch(w)
        its = [i["admm_iters"] for i in infos]
        print("lds", lds, "iters", sum(its), "max", max(its), flush=True)
        for k, lp in enumerate(lps):
            _check_solution(lp, xs[k], ys[k], ss[k], infos[k])
        w.free()


# edge shapes of the LDS-resident layout: one row, one column, the column-pair
# boundary (ceil(n/4) = 32 / 33), two columns per lane (n > 256), rows per lane
# 2 and 3, FP64 data that does and does not fit
EDGE = [(1, 1, 31), (1, 7, 32), (3, 3, 33), (4, 128, 34), (4, 129, 35), (5, 300, 40), (64, 100, 45),
        (65, 70, 38), (129, 140, 42)]


@pytest.mark.parametrize("m,n,seed", EDGE)
def test_lds_edge_shapes_match_oracle_and_streamed(m, n, seed):
    print(f"lds edge m={m} n={n} seed={seed}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings(alpha=1.8, gamma=0.5, restart_rule="heuristic")
    st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, "heuristic")
    solver = oracle.SchurIQSolver(prob)
    N = 30
    st = st0.copy()
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    scale = 1.0 + np.abs(st.u()).max()
    got = {}
    for lds in (1, 0):
        for fp32 in (False, True):
            got[(lds, fp32)] = _iterate(lp, st0, N, lds, fp32, "heuristic")
    for lds in (1, 0):
        y, x, sv, sc = got[(lds, False)]
        for g, ref in [(y, st.y), (x, st.x), (sv, st.s)]:
            assert np.abs(g - ref).max() <= 1e-10 * scale, (lds, m, n)
        assert abs(sc["tau"] - st.tau) <= 1e-10 * scale
    a, b = got[(1, True)], got[(0, True)]
    for ga, gb in zip(a[:3], b[:3]):
        assert np.abs(ga - gb).max() <= 1e-9 * scale
    # full solve, default settings (LDS-resident where it fits), against the oracle's status
    ref = oracle.solve(lp["A"], lp["b"], lp["c"])
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, sv, info = abip.abip_solve(w)
    assert info["status_name"] == ref["status_name"]
    if ref["status_name"] == "solved":
        k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
        assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6, k


class _ExplicitInverseIQ(oracle.SchurIQSolver):
    """The oracle's Schur linear step with G^{-1} formed once (numpy's inverse)
    instead of a Cholesky solve per application: the same mathematics, another
    FP64 rounding, used to measure how far FP64 arithmetic alone spreads an
    iterate of an ill-conditioned LP."""

    def __init__(self, prob):
        A = prob.A
        self.Gi = np.linalg.inv(np.eye(A.shape[0]) + A @ A.T)
        super().__init__(prob)

    def apply_Minv(self, w):
        m, A = self.m, self.prob.A
        a = self.Gi @ (w[:m] - A @ w[m:])
        return np.concatenate([a, w[m:] + A.T @ a])


def _tall(m_planted, n, extra, seed):
    """A planted m_planted x n LP stacked with `extra` random combinations of its
    rows: more rows than columns, rank m_planted, consistent b, same optimum."""
    lp = lpgen.dense_planted(m_planted, n, seed)
    R = np.random.default_rng(seed + 1).standard_normal((extra, m_planted))
    A = np.vstack([lp["A"], R @ lp["A"]])
    b = np.concatenate([lp["b"], R @ lp["b"]])
    return dict(A=A, b=b, c=lp["c"], pstar=lp["pstar"], status="solved", m=A.shape[0], n=n)


def test_lds_tall_a_only_fp32_held_as_doubles():
    """160 x 90 (m > n): G^{-1} (160 x 160) does not fit beside A in either precision,
    so both phases hold A alone in LDS, and the FP32 phase holds its FP32-rounded A as
    doubles (the FP64 A-only layout fits).  Fixed updates in both precisions against the
    streamed variant and the oracle, then full FP32-bulk and FP64 solves."""
    lp = _tall(40, 90, 120, 51)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings(alpha=1.8, gamma=0.5, restart_rule="heuristic")
    st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, "heuristic")
    N = 40

    def run(solver):
        st = st0.copy()
        for _ in range(N):
            st = oracle.admm_iteration(prob, solver, st, s)
        return st

    st = run(oracle.SchurIQSolver(prob))
    scale = 1.0 + np.abs(st.u()).max()
    # G = I + A A^T has condition number ~4e4 here, so FP64 rounding alone moves the
    # 40-update iterate by ~1e-10 relative: the bar is 1e-10 plus four times the
    # spread between the oracle's Cholesky-solve linear step and the same step through
    # an explicitly formed G^{-1} (the form Section 4.4's cached inverse takes)
    st_inv = run(_ExplicitInverseIQ(prob))
    spread = max(np.abs(st_inv.u() - st.u()).max(), np.abs(st_inv.v() - st.v()).max())
    tol = (1e-10 + 4 * spread / scale) * scale
    print(f"tall: oracle FP64 spread {spread / scale:.2e} relative, bar {tol / scale:.2e}", flush=True)
    got = {(lds, fp32): _iterate(lp, st0, N, lds, fp32, "heuristic") for lds in (1, 0) for fp32 in (False, True)}
    for lds in (1, 0):
        y, x, sv, sc = got[(lds, False)]
        for g, ref in [(y, st.y), (x, st.x), (sv, st.s)]:
            assert np.abs(g - ref).max() <= tol, lds
        for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
            assert abs(sc[key] - ref) <= tol, (lds, key)
    a, b = got[(1, True)], got[(0, True)]
    for ga, gb in zip(a[:3], b[:3]):
        assert np.abs(ga - gb).max() <= 1e-9 * scale
    assert np.abs(a[1] - st.x).max() <= 1e-3 * scale
    ref = oracle.solve(lp["A"], lp["b"], lp["c"])
    assert ref["status_name"] == "solved"
    for prec in (abip.ABIP_PREC_FP32_POLISH, abip.ABIP_PREC_FP64):
        w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(precision=prec))
        x, y, sv, info = abip.abip_solve(w)
        print("tall", prec, info["status_name"], info["admm_iters"], info["admm_iters_fp64"], "oracle",
              ref["admm_iters"], "lds_mode", info["lds_mode"], flush=True)
        assert info["lds_mode"] == 4 | 8           # A alone in LDS in both phases
        assert info["colpass_lds_fp32"] + info["colpass_lds_fp64"] > 0
        _check_solution(lp, x, y, sv, info)
        k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
        assert abs(k["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
        if prec == abip.ABIP_PREC_FP64:
            assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(5, ref["admm_iters"] // 50)
        w.free()
