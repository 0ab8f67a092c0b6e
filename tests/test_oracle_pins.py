"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests compares the oracle with itself: each one checks it
against a closed form, an invariant the paper proves, an independent
derivation (Algorithm 1, Newton on the central-path system, the first form of
the projection formula), a library routine (HiGHS) or brute force.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import lpgen
import oracle
from oracle.abip import Problem, Settings

FAST = [(3, 6, 1), (3, 6, 4), (4, 8, 4), (4, 8, 6), (12, 30, 2), (12, 30, 4)]


def _prob(lp):
    return Problem(lp["A"], lp["b"], lp["c"])


# --------------------------------------------------------------------------
# HSD embedding (Section 3.1)
# --------------------------------------------------------------------------

def test_Q_is_skew_symmetric_and_matches_implicit_apply():
    lp = lpgen.dense_planted(7, 13, 0)
    prob = _prob(lp)
    Q = oracle.assemble_Q(prob)
    assert np.array_equal(Q, -Q.T)
    rng = np.random.default_rng(1)
    for _ in range(5):
        u = rng.standard_normal(7 + 13 + 2)
        Qu = oracle.apply_Q(prob, u)
        np.testing.assert_allclose(Qu, Q @ u, rtol=0, atol=1e-12 * np.abs(Q).max() * np.abs(u).sum())
        assert abs(u @ Qu) <= 1e-13 * (u @ u) * np.linalg.norm(Q, 2)


def test_hsd_constants_closed_form():
    A = np.array([[1.0, 2.0, 0.0], [0.0, -1.0, 3.0]])
    b = np.array([4.0, 5.0])
    c = np.array([1.0, -2.0, 0.5])
    bbar, cbar, zbar = oracle.hsd_constants(Problem(A, b, c))
    np.testing.assert_array_equal(bbar, [4.0 - 3.0, 5.0 - 2.0])
    np.testing.assert_array_equal(cbar, [0.0, -3.0, -0.5])
    assert zbar == 1.0 - 2.0 + 0.5 + 1.0


def test_initial_point_is_central_and_inner_test_passes_at_once():
    """Q u0 = v0 exactly at (y,x,tau,theta) = (0,e,1,1), (s,kappa,xi) = (e,1,-(n+1)),
    so the first inner test passes and N_0 = 0 (Algorithm 2; Lemma 3.3's proof)."""
    lp = lpgen.dense_planted(6, 11, 3)
    prob = _prob(lp)
    st = oracle.initial_state(prob, Settings())
    r = oracle.apply_Q(prob, st.u()) - st.v()
    assert np.abs(r).max() <= 1e-12 * (1 + np.abs(lp["A"]).sum())
    out = oracle.solve(prob, settings=Settings(max_admm_iters=3))
    assert out["inner_counts"][0] == 0


# --------------------------------------------------------------------------
# The affine step (eq. Simple-Update:Affine, Section 4.4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(1, 2), (5, 9), (20, 45)])
def test_schur_solver_equals_projection_definition(m, n):
    lp = lpgen.dense_planted(m, n, m + n)
    prob = _prob(lp)
    Q = oracle.assemble_Q(prob)
    N = m + n + 2
    rng = np.random.default_rng(5)
    w = rng.standard_normal(N)
    ut = oracle.SchurIQSolver(prob).solve(w)
    ud = oracle.DenseIQSolver(prob).solve(w)
    # (I + Q) u~ = w  <=>  u~ + Q u~ = u + v  (Theorem 3.1, step 1)
    assert np.linalg.norm(ut + Q @ ut - w) <= 1e-12 * np.linalg.norm(w) * (1 + np.linalg.norm(Q, 2))
    np.testing.assert_allclose(ut, ud, rtol=0, atol=1e-11 * np.linalg.norm(w))
    # first form of eq. (Simple-Update:Affine): projection of (w, w) onto {Qu = v}
    up = np.linalg.solve(np.eye(N) + Q.T @ Q, (np.eye(N) - Q) @ w)
    np.testing.assert_allclose(ut, up, rtol=0, atol=1e-9 * np.linalg.norm(w))
    assert abs(ut @ (Q @ ut)) <= 1e-12 * (ut @ ut) * np.linalg.norm(Q, 2)


# --------------------------------------------------------------------------
# The barrier prox (eqs. Simple-Update:Barrier-X / -tau)
# --------------------------------------------------------------------------

def _bisect_prox(w, t):
    """argmin_{z>0} -t log z + (z-w)^2/2 by bisection on the derivative z - w - t/z."""
    lo, hi = 1e-300, max(1.0, abs(w)) * 4 + 4 * math.sqrt(t) + 1
    for _ in range(2000):
        mid = 0.5 * (lo + hi) if hi / lo < 4 else math.sqrt(lo * hi)
        if mid - w - t / mid > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-16 * hi:
            break
    return 0.5 * (lo + hi)


def _decimal_root(w, t):
    """Positive root of z^2 - w z - t = 0 in 60-digit decimal arithmetic."""
    import decimal
    ctx = decimal.Context(prec=60)
    W = decimal.Decimal(float(w))
    T = decimal.Decimal(float(t))
    r = ctx.sqrt(W * W + 4 * T)
    z = (W + r) / 2 if W >= 0 else (2 * T) / (r - W)
    return float(z)


def test_prox_is_positive_root_and_minimiser():
    rng = np.random.default_rng(0)
    ws = np.concatenate([rng.standard_normal(50) * 10, [0.0, -1e8, 1e8, -3e-3]])
    for t in [1.0, 1e-4, 1e-10]:
        z = oracle.barrier_prox(ws, t)
        assert np.all(z > 0)
        for w, zz in zip(ws, z):
            assert abs(zz - _decimal_root(w, t)) <= 4e-16 * zz
        for w, zz in zip(ws[:10], z[:10]):
            assert abs(zz - _bisect_prox(w, t)) <= 1e-12 * max(1.0, zz) + 1e-15
    # far in the tail the root is t/|w| to first order; the naive form rounds to 0
    z = oracle.barrier_prox(np.array([-1e8]), 1e-10)[0]
    assert abs(z - 1e-18) <= 1e-24


# --------------------------------------------------------------------------
# Theorem 3.1 and Algorithm 1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alpha", [1.0, 1.8])
@pytest.mark.parametrize("rule", ["heuristic", "sqrt"])
def test_theorem31_invariants_along_iterations(alpha, rule):
    lp = lpgen.dense_planted(6, 14, 2)
    prob = _prob(lp)
    s = Settings(alpha=alpha, restart_rule=rule, gamma=0.5)
    solver = oracle.SchurIQSolver(prob)
    st = oracle.initial_state(prob, s)
    n = prob.n
    for k in range(4):
        for i in range(25):
            st, v = oracle.admm_iteration(prob, solver, st, s, return_v=True)
            t = st.mu / s.beta
            np.testing.assert_allclose(st.x * st.s, t, rtol=1e-10)
            assert abs(st.tau * st.kappa - t) <= 1e-10 * t
            assert np.abs(v[:prob.m]).max() <= 1e-12 * (1 + np.abs(st.y).max())
            assert abs(v[-1] + (n + 1)) <= 1e-12 * (n + 1)
            assert np.all(st.x > 0) and np.all(st.s > 0) and st.tau > 0 and st.kappa > 0
        st = oracle.restart(st, s.gamma, rule)
        np.testing.assert_allclose(st.x * st.s, st.mu / s.beta, rtol=1e-12)
        assert abs(st.tau * st.kappa - st.mu / s.beta) <= 1e-12 * st.mu


def test_algorithm1_equals_algorithm2():
    """Theorem 3.1: with p0 = v0, q0 = u0 the explicit-multiplier ADMM produces
    the same (u, v) as the simplified iteration (alpha = 1), including after a
    sqrt(gamma) restart that re-initialises p = v, q = u."""
    lp = lpgen.dense_planted(3, 7, 11)
    prob = _prob(lp)
    s = Settings(alpha=1.0, gamma=0.5, restart_rule="sqrt")
    solver = oracle.DenseIQSolver(prob)
    st = oracle.initial_state(prob, s)
    for stage in range(2):
        z = oracle.alg1_initial(st)
        for i in range(40):
            st = oracle.admm_iteration(prob, solver, st, s)
            z = oracle.alg1_iteration(prob, z, st.mu, s.beta)
            np.testing.assert_allclose(z["u"], st.u(), rtol=1e-8, atol=1e-10)
            np.testing.assert_allclose(z["v"], st.v(), rtol=1e-8, atol=1e-10)
            np.testing.assert_allclose(z["p"], st.v(), rtol=1e-8, atol=1e-10)
            np.testing.assert_allclose(z["q"], st.u(), rtol=1e-8, atol=1e-10)
        st = oracle.restart(st, s.gamma, "sqrt")


# --------------------------------------------------------------------------
# Inner loop at fixed mu: central point, Lemma 3.2
# --------------------------------------------------------------------------

def test_central_point_solves_hsd_log_kkt():
    lp = lpgen.dense_planted(5, 12, 1)
    prob = _prob(lp)
    t = 0.05
    cp = oracle.central_point(prob, t=t)
    r = oracle.apply_Q(prob, cp.u()) - cp.v()
    assert np.abs(r).max() < 1e-10
    np.testing.assert_allclose(cp.x * cp.s, t, rtol=1e-10)
    assert abs(cp.tau * cp.kappa - t) < 1e-12
    assert abs(cp.theta - t) < 1e-10          # theta = mu/beta on the central path


def test_inner_loop_converges_monotonically_to_central_point():
    """Lemma 3.2 (alpha = 1): ||u_i - u*||^2 + ||v_i - v*||^2 is non-increasing
    and tends to 0; theta_i tends to mu/beta."""
    lp = lpgen.dense_planted(5, 12, 1)
    prob = _prob(lp)
    s = Settings(alpha=1.0, gamma=0.2, restart_rule="heuristic")
    solver = oracle.SchurIQSolver(prob)
    st = oracle.initial_state(prob, s)
    st = oracle.restart(st, s.gamma, s.restart_rule)       # mu^1 = gamma * beta
    t = st.mu / s.beta
    cp = oracle.central_point(prob, t=t)
    dist = []
    for i in range(3000):
        d = np.sum((st.u() - cp.u()) ** 2) + np.sum((st.v() - cp.v()) ** 2)
        dist.append(d)
        st = oracle.admm_iteration(prob, solver, st, s)
    dist = np.array(dist)
    assert np.all(np.diff(dist) <= 1e-12 * dist[:-1] + 1e-28)
    assert dist[-1] < 1e-16 * dist[0] + 1e-20
    assert abs(st.theta - t) < 1e-8


def test_outer_count_in_mu_stop_mode():
    """With the outer loop stopped once mu^k < eps, the number of outer
    iterations is ceil(log(mu0/eps)/log(1/gamma)) (proof of Theorem 3.5)."""
    lp = lpgen.dense_planted(4, 8, 4)
    for gamma, eps in [(0.5, 3e-3), (0.3, 1e-4), (0.9, 0.2)]:
        s = Settings(gamma=gamma, mu_stop=eps, beta=1.0)
        out = oracle.solve(lp["A"], lp["b"], lp["c"], s)
        assert out["status"] == oracle.MU_STOP
        expect = math.ceil(math.log(1.0 / eps) / math.log(1.0 / gamma))
        assert out["ipm_iters"] == expect


# --------------------------------------------------------------------------
# End to end: LP optimum and certificates (Theorems 2.1-2.3, Section 4.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,seed", FAST[:4])
def test_solution_matches_vertex_enumeration(m, n, seed):
    lp = lpgen.dense_planted(m, n, seed)
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-7))
    assert out["status"] == oracle.SOLVED
    pstar, xstar = oracle.vertex_enumeration(lp["A"], lp["b"], lp["c"])
    assert abs(out["info"]["pobj"] - pstar) <= 1e-5 * (1 + abs(pstar))
    np.testing.assert_allclose(out["x"], xstar, atol=1e-4)
    np.testing.assert_allclose(out["x"], lp["x0"], atol=1e-4)     # planted, unique
    np.testing.assert_allclose(out["y"], lp["y0"], atol=1e-4)


@pytest.mark.parametrize("m,n,seed", FAST[4:])
def test_solution_matches_highs(m, n, seed):
    lp = lpgen.dense_planted(m, n, seed)
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-7))
    assert out["status"] == oracle.SOLVED
    ref = scipy.optimize.linprog(lp["c"], A_eq=lp["A"], b_eq=lp["b"], bounds=(0, None), method="highs")
    assert ref.status == 0
    assert abs(out["info"]["pobj"] - ref.fun) <= 1e-6 * (1 + abs(ref.fun))
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], out["x"], out["y"], out["s"])
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-7


def test_toy_two_var_closed_form():
    lp = lpgen.toy_two_var()
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-8))
    assert out["status"] == oracle.SOLVED
    np.testing.assert_allclose(out["x"], lp["xstar"], atol=1e-6)
    np.testing.assert_allclose(out["y"], lp["ystar"], atol=1e-6)
    np.testing.assert_allclose(out["s"], lp["sstar"], atol=1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_toy_simplex_closed_form(seed):
    lp = lpgen.toy_simplex(6, seed)
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-8))
    assert out["status"] == oracle.SOLVED
    assert abs(out["info"]["pobj"] - lp["pstar"]) <= 1e-6
    np.testing.assert_allclose(out["x"], lp["xstar"], atol=1e-5)


def test_toy_primal_infeasible_certificate():
    lp = lpgen.toy_primal_infeasible()
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
    assert out["status"] == oracle.PRIMAL_INFEASIBLE
    np.testing.assert_allclose(out["y"], lp["certificate"], atol=1e-9)   # y / (b^T y)
    st = out["state"]
    assert st.kappa > st.tau            # Theorem 2.2 (ii): tau -> 0, kappa > 0


def test_toy_dual_infeasible_certificate():
    lp = lpgen.toy_dual_infeasible()
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
    assert out["status"] == oracle.DUAL_INFEASIBLE
    x = out["x"]
    assert abs(lp["c"] @ x + 1.0) < 1e-12           # -x / (c^T x) has c^T x = -1
    np.testing.assert_allclose(x / np.linalg.norm(x), lp["ray"], atol=1e-6)


def test_planted_farkas_infeasible():
    lp = lpgen.dense_farkas_infeasible(20, 50, 3)
    A, b = lp["A"], lp["b"]
    assert np.all(A.T @ lp["farkas"] < 0) and abs(b @ lp["farkas"] - 1) < 1e-9   # generator check
    out = oracle.solve(A, b, lp["c"], Settings())
    assert out["status"] == oracle.PRIMAL_INFEASIBLE
    y, s = out["y"], out["s"]
    assert abs(b @ y - 1.0) < 1e-12
    assert np.linalg.norm(A.T @ y + s) <= 1e-6 / np.linalg.norm(b) * 1.0000001
    assert np.all(s >= 0)


def test_basis_pursuit_recovers_l1_optimum():
    lp = lpgen.basis_pursuit(20, 40, 3, 7)
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-7))
    assert out["status"] == oracle.SOLVED
    assert abs(out["info"]["pobj"] - lp["pstar"]) <= 1e-5 * (1 + lp["pstar"])
    N = lp["n"] // 2
    np.testing.assert_allclose(out["x"][:N] - out["x"][N:], lp["x_true"], atol=1e-4)


# --------------------------------------------------------------------------
# Derivative references
# --------------------------------------------------------------------------

def test_kkt_adjoint_matches_finite_differences_of_central_point():
    """The dense adjoint at a central point equals central differences of the
    central point itself (an independent Newton solve per perturbation)."""
    lp = lpgen.dense_planted(3, 7, 2)
    A, b, c = lp["A"], lp["b"], lp["c"]
    w = np.random.default_rng(9).standard_normal(7)
    t = 1e-3
    cp = oracle.central_point(A, b, c, t=t)
    lam = oracle.kkt_adjoint(A, b, c, cp, w)
    g = oracle.contract_adjoint(A, b, c, cp, lam, want_A=True)

    def L(A_, b_, c_):
        p = oracle.central_point(A_, b_, c_, t=t)
        return w @ p.x / p.tau

    h = 1e-6
    for k in range(7):
        e = np.zeros(7)
        e[k] = h
        fd = (L(A, b, c + e) - L(A, b, c - e)) / (2 * h)
        assert abs(fd - g["dc"][k]) <= 1e-5 * (1 + abs(fd))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (L(A, b + e, c) - L(A, b - e, c)) / (2 * h)
        assert abs(fd - g["db"][i]) <= 1e-5 * (1 + abs(fd))
    for (i, j) in [(0, 0), (1, 3), (2, 6)]:
        E = np.zeros_like(A)
        E[i, j] = h
        fd = (L(A + E, b, c) - L(A - E, b, c)) / (2 * h)
        assert abs(fd - g["dA"][i, j]) <= 1e-5 * (1 + abs(fd))


def test_basis_gradients_match_finite_differences_and_small_t_adjoint():
    lp = lpgen.dense_planted(4, 9, 5)
    A, b, c = lp["A"], lp["b"], lp["c"]
    w = np.random.default_rng(2).standard_normal(9)
    bg = oracle.basis_gradients(A, b, lp["basis"], w)
    h = 1e-5

    def Lb(b_):
        return w @ oracle.basis_gradients(A, b_, lp["basis"], w)["x"]

    for i in range(4):
        e = np.zeros(4)
        e[i] = h
        assert abs((Lb(b + e) - Lb(b - e)) / (2 * h) - bg["db"][i]) < 1e-8
    # as t -> 0 the central-path derivative tends to the basis derivative
    cp = oracle.central_point(A, b, c, t=1e-10)
    g = oracle.contract_adjoint(A, b, c, cp, oracle.kkt_adjoint(A, b, c, cp, w), want_A=True)
    np.testing.assert_allclose(g["db"], bg["db"], atol=1e-6 * (1 + np.abs(bg["db"]).max()))
    np.testing.assert_allclose(g["dc"], 0.0, atol=1e-6 * np.linalg.norm(w))
    np.testing.assert_allclose(g["dA"], bg["dA"], atol=1e-6 * (1 + np.abs(bg["dA"]).max()))


# --------------------------------------------------------------------------
# Planted mistakes: each pin above must notice a plausible bug in the oracle
# --------------------------------------------------------------------------

def test_planted_mistakes_are_caught(monkeypatch):
    lp = lpgen.dense_planted(3, 7, 11)
    prob = _prob(lp)
    # (1) wrong sign of zbar in Q: the central start point is no longer central
    orig = oracle.abip.hsd_constants
    monkeypatch.setattr(oracle.abip, "hsd_constants",
                        lambda p: (lambda bb, cb, zb: (bb, cb, -zb))(*orig(p)))
    st = oracle.initial_state(prob, Settings())
    r = oracle.apply_Q(prob, st.u()) - st.v()
    assert np.abs(r).max() > 1e-3
    monkeypatch.setattr(oracle.abip, "hsd_constants", orig)
    # (2) prox root with the wrong sign of the square root: Algorithm 1 disagrees
    good = oracle.abip.barrier_prox
    monkeypatch.setattr(oracle.abip, "barrier_prox",
                        lambda w, t: np.abs(0.5 * (w - np.sqrt(w * w + 4 * t))))
    s = Settings(alpha=1.0)
    st = oracle.initial_state(prob, s)
    st.mu = 0.5
    st.x = st.x * np.sqrt(0.5)
    st.s = st.s * np.sqrt(0.5)
    st.tau = st.kappa = np.sqrt(0.5)
    z = oracle.alg1_initial(st)
    st2 = oracle.admm_iteration(prob, oracle.DenseIQSolver(prob), st, s)
    monkeypatch.setattr(oracle.abip, "barrier_prox", good)
    z2 = oracle.alg1_iteration(prob, z, st.mu, s.beta)
    assert np.abs(z2["u"] - st2.u()).max() > 1e-3


# ---------------------------------------------------------------------------
# FP32-data model of the linear step (precision extension)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,seed", [(5, 11, 1), (30, 70, 2), (60, 150, 3)])
def test_fp32_data_model_without_rounding_is_the_exact_solve(m, n, seed):
    """With nothing rounded the model is the Section 4.4 solve: equal to the dense LU of
    the assembled I + Q (not only to the Schur solver it borrows its border from)."""
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    w = np.random.default_rng(seed).standard_normal(m + n + 2)
    got = oracle.Fp32DataSchurSolver(prob, dtype=np.float64).solve(w)
    ref = oracle.DenseIQSolver(prob).solve(w)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("m,n,seed", [(30, 70, 2), (60, 150, 3), (120, 300, 4)])
def test_fp32_data_model_within_the_rounding_bound(m, n, seed):
    """Rounding A and G^{-1} to FP32 (unit roundoff u = 2^-24) moves the step by at most
    the first-order bound propagated through a = G^{-1}(y - A f), d = f + A^T a and the
    rank-2 border:  |da| <= u (||G^{-1}||_F ||t|| + ||A||_F ||f||),
    |dd| <= u ||A||_F ||a|| + ||A||_2 |da|,  |dq| <= (||A c - b|| + ||bbar - A cbar||) |da|,
    |du| <= |da| + |dd| + (||Z||_2 + 1) ||K^{-1}||_2 |dq|  (twice that, for second-order
    terms).  The deviation must also be above the FP64 level, i.e. the rounding happened."""
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    A = lp["A"]
    w = np.random.default_rng(seed + 7).standard_normal(m + n + 2)
    exact = oracle.SchurIQSolver(prob)
    ref = exact.solve(w)
    got = oracle.Fp32DataSchurSolver(prob).solve(w)
    u = 2.0 ** -24
    bbar, cbar, _ = oracle.hsd_constants(prob)
    Ginv = np.linalg.inv(np.eye(m) + A @ A.T)
    y, f = w[:m], w[m:m + n]
    t = y - A @ f
    a = Ginv @ t
    nA_F, nA_2 = np.linalg.norm(A), np.linalg.norm(A, 2)
    da = u * (np.linalg.norm(Ginv) * np.linalg.norm(t) + nA_F * np.linalg.norm(f))
    dd = u * nA_F * np.linalg.norm(a) + nA_2 * da
    dq = (np.linalg.norm(A @ lp["c"] - lp["b"]) + np.linalg.norm(bbar - A @ cbar)) * da
    bound = 2.0 * (da + dd + (np.linalg.norm(exact.Z, 2) + 1.0) * np.linalg.norm(np.linalg.inv(exact.K), 2) * dq)
    dev = np.linalg.norm(got - ref)
    assert dev <= bound, (dev, bound)
    assert dev >= 1e-6 * bound, (dev, bound)


@pytest.mark.parametrize("sparse", [False, True])
def test_cg_solver_equals_direct_solve(sparse):
    """The indirect variant of Section 4.4 (CG on G = I + A A^T, A and A^T products
    only) converges to the direct solve; a warm-started second solve agrees too."""
    import scipy.sparse as sps
    lp = lpgen.sparse_planted(80, 200, 3, density=0.05)
    Ac = lp["A_csr"]
    A = sps.csr_matrix((Ac["data"], Ac["indices"], Ac["indptr"]), shape=Ac["shape"])
    prob_d = Problem(A.toarray(), lp["b"], lp["c"])
    prob = oracle.abip._as_problem(A if sparse else A.toarray(), lp["b"], lp["c"])
    cg = oracle.CGIQSolver(prob, tol=1e-14, max_iters=2000)
    ref = oracle.DenseIQSolver(prob_d)
    rng = np.random.default_rng(0)
    for _ in range(2):
        w = rng.standard_normal(80 + 200 + 2)
        got, want = cg.solve(w), ref.solve(w)
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    assert cg.cg_iters > 0


def test_cg_solver_full_solve_matches_direct():
    """Algorithm 2 with the CG step (tight tolerance) takes the direct path's iterations."""
    import scipy.sparse as sps
    lp = lpgen.sparse_planted(40, 90, 1, density=0.08)
    Ac = lp["A_csr"]
    A = sps.csr_matrix((Ac["data"], Ac["indices"], Ac["indptr"]), shape=Ac["shape"])
    prob = oracle.abip._as_problem(A, lp["b"], lp["c"])
    out_cg = oracle.solve(prob, settings=Settings(), solver=oracle.CGIQSolver(prob, tol=1e-13, max_iters=2000))
    out_d = oracle.solve(A.toarray(), lp["b"], lp["c"], Settings())
    assert out_cg["status"] == out_d["status"] == oracle.SOLVED
    assert abs(out_cg["admm_iters"] - out_d["admm_iters"]) <= max(3, out_d["admm_iters"] // 100)
    np.testing.assert_allclose(out_cg["x"], out_d["x"], atol=1e-7 * (1 + np.abs(out_d["x"]).max()))


# ---------------------------------------------------------------------------
# Barzilai-Borwein choice of beta (Section 4.3)
# ---------------------------------------------------------------------------

def _bb_from_pairs(rng, dvh, dut, du, alpha=1.8):
    """Iterates (u0, v0, ut1, u1, v1, ut2, u2, v2) whose curvature pairs of Section 4.3
    are the given (dvh, dut, du): u0, v0, ut1, u1, v2 are drawn, u2 follows from du,
    ut2 from dut and v1 from dvh."""
    N = dvh.size
    u0, v0, ut1, u1, v2 = (rng.standard_normal(N) for _ in range(5))
    u2 = u1 - du
    ut2 = ut1 + (dut - (1 - alpha) * (u1 - u0)) / alpha
    vh1 = v0 - alpha * ut1 - (1 - alpha) * u0 + alpha * u1
    v1 = dvh + vh1 + alpha * ut2 + (1 - alpha) * u1 - alpha * u2
    return [u0, v0, ut1, u1, v1, ut2, u2, v2]


def test_bb_sd_at_least_mg_by_cauchy_schwarz():
    rng = np.random.default_rng(0)
    seen = 0
    for _ in range(200):
        dvh, dut, du = (rng.standard_normal(9) for _ in range(3))
        dut = dut + rng.uniform(0.1, 3.0) * dvh            # positive correlations
        du = du + rng.uniform(0.1, 3.0) * dvh
        _, d = oracle.bb_estimate(*_bb_from_pairs(rng, dvh, dut, du), 1.8, 1.0, eps_cor=0.0)
        for k in ("phi", "psi"):
            assert d[k + "_cor"] <= 1 + 1e-12
            if d[k + "_cor"] > 0:
                assert d[k + "_sd"] >= d[k + "_mg"] * (1 - 1e-12)
                seen += 1
    assert seen > 300


@pytest.mark.parametrize("cst", [0.3, 2.5])
def test_bb_exact_curvature_gives_that_step(cst):
    """dvh = c dut and dvh = d du exactly: SD = MG for both, correlations 1, the
    hybrid picks MG, and the estimate is sqrt(c d)."""
    rng = np.random.default_rng(1)
    dvh = rng.standard_normal(9)
    d2 = 1.7
    vs = _bb_from_pairs(rng, dvh, dvh / cst, dvh / d2)
    bh, d = oracle.bb_estimate(*vs, 1.8, 1.0, eps_cor=0.2)
    assert abs(d["phi_cor"] - 1.0) < 1e-12 and abs(d["psi_cor"] - 1.0) < 1e-12
    assert abs(d["phi_sd"] - cst) < 1e-10 * cst and abs(d["phi_mg"] - cst) < 1e-10 * cst
    assert abs(d["phi"] - cst) < 1e-10 * cst and abs(d["psi"] - d2) < 1e-10 * d2
    assert abs(bh - np.sqrt(cst * d2)) < 1e-10


def test_bb_hybrid_branches():
    assert oracle.abip._hybrid(3.0, 2.0) == 2.0            # 2 MG > SD: MG
    assert oracle.abip._hybrid(5.0, 2.0) == 4.0            # otherwise SD - MG / 2
    assert oracle.abip._hybrid(4.0, 2.0) == 3.0            # tie 2 MG == SD: the second branch


def test_bb_safeguard_branches():
    """Every branch of the correlation safeguard: both estimates reliable (geometric
    mean), one of them (that one), neither (beta kept)."""
    rng = np.random.default_rng(2)
    beta = 1.7
    dvh, e1, e2 = (rng.standard_normal(9) for _ in range(3))
    dut = dvh + 0.3 * e1            # correlation near 0.96
    du = dvh + 2.0 * e2             # correlation near 0.45
    vs = _bb_from_pairs(rng, dvh, dut, du)
    _, d0 = oracle.bb_estimate(*vs, 1.8, beta, 0.0)
    pc, sc = d0["phi_cor"], d0["psi_cor"]
    assert 0.0 < sc < pc < 1.0
    bh, d = oracle.bb_estimate(*vs, 1.8, beta, 0.5 * sc)            # both reliable
    assert abs(bh - np.sqrt(d["phi"] * d["psi"])) <= 1e-12 * bh
    bh, d = oracle.bb_estimate(*vs, 1.8, beta, 0.5 * (sc + pc))     # phi only
    assert d["psi"] is None and bh == d["phi"]
    vs2 = _bb_from_pairs(rng, dvh, du, dut)                          # swapped: psi only
    bh, d = oracle.bb_estimate(*vs2, 1.8, beta, 0.5 * (sc + pc))
    assert d["phi"] is None and bh == d["psi"]
    bh, d = oracle.bb_estimate(*vs, 1.8, beta, 0.5 * (pc + 1.0))    # neither: beta kept
    assert d["phi"] is None and d["psi"] is None and bh == beta
    # the Section 5 threshold on these iterates: both reliable
    bh, d = oracle.bb_estimate(*vs, 1.8, beta, 0.2)
    assert d["phi"] is not None and d["psi"] is not None


def test_bb_selection_rule():
    assert oracle.bb_rule(1.0, 1.0, 0.1) == ("keep", 1.0)
    act, b = oracle.bb_rule(1.0, 1.08, 0.1)
    assert act == "average" and abs(b - 1.04) < 1e-15
    assert oracle.bb_rule(1.0, 1.5, 0.1) == ("redo", 1.5)
    assert oracle.bb_rule(1.0, 0.5, 0.1) == ("redo", 0.5)


def test_bb_solve_still_reaches_the_optimum():
    """With the Section 4.3 beta the method still ends SOLVED at the planted optimum."""
    lp = lpgen.config0(4)
    out = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(bb=True))
    assert out["status"] == oracle.SOLVED
    assert out["betas"] and all(b > 0 for _, b, _ in out["betas"])
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], out["x"], out["y"], out["s"])
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))


def test_bb_differences_from_iterate_differences():
    """The curvature differences of Section 4.3, formed as the paper defines them
    (v-hat from v, u-tilde, u; the relaxed u-tilde difference), equal the forms
    built from differences of consecutive iterates alone: with the dual update
    v_k = v_{k-1} - uh_k + u_k and uh_k = alpha ut_k + (1 - alpha) u_{k-1},
        dvh = dv2 - (1 - alpha) du2,  dut = du2 - dv2 + dv1,  du = -du2
    (du2 = u2 - u1, dv2 = v2 - v1, dv1 = v1 - v0).  The GPU accumulates the
    second form, so a wrong sign or a dropped term in either fails here."""
    lp = lpgen.dense_planted(20, 45, 3)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    for alpha in (1.0, 1.8, 0.7):
        s = Settings(alpha=alpha)
        st0 = oracle.restart(oracle.initial_state(prob, s), s.gamma, "heuristic")
        solver = oracle.SchurIQSolver(prob)
        for _ in range(5):                      # a point inside the outer iteration
            st0 = oracle.admm_iteration(prob, solver, st0, s)
        u0, v0 = st0.u(), st0.v()
        st1, v1, ut1 = oracle.admm_iteration(prob, solver, st0, s, return_ut=True)
        st2, v2, ut2 = oracle.admm_iteration(prob, solver, st1, s, return_ut=True)
        u1, u2 = st1.u(), st2.u()
        vh1 = v0 - alpha * ut1 - (1.0 - alpha) * u0 + alpha * u1
        vh2 = v1 - alpha * ut2 - (1.0 - alpha) * u1 + alpha * u2
        dvh, dut, du = vh2 - vh1, alpha * (ut2 - ut1) + (1.0 - alpha) * (u1 - u0), -(u2 - u1)
        du2, dv2, dv1 = u2 - u1, v2 - v1, v1 - v0
        scale = np.abs(u0).max() + np.abs(v0).max()
        assert np.abs(dvh - (dv2 - (1.0 - alpha) * du2)).max() <= 1e-12 * scale
        assert np.abs(dut - (du2 - dv2 + dv1)).max() <= 1e-12 * scale
        assert np.abs(du + du2).max() == 0.0
        # v's y block stays 0 and its theta entry -(n+1)
        m, n = prob.m, prob.n
        assert np.all(v1[:m] == 0.0) and v1[m + n + 1] == -(n + 1.0)
