"""ABIP in plain FP64 NumPy -- the oracle (test infrastructure only).

Notation follows the paper.  The LP pair is (P) min c^T x s.t. Ax = b, x >= 0 and
(D) max b^T y s.t. A^T y + s = c, s >= 0 (Section 2).  The homogeneous self-dual
(HSD) embedding with y0 = 0, x0 = s0 = e is written in Section 3.1 as Q u = v with

        [  0     A    -b    bbar ]        u = (y, x, tau, theta)
    Q = [ -A^T   0     c   -cbar ]        v = (r, s, kappa, xi)
        [  b^T  -c^T   0    zbar ]        r = 0, xi = -(n+1)
        [ -bbar^T cbar^T -zbar 0 ]

with bbar = b - A e, cbar = c - e, zbar = c^T e + 1 (eq. bar-b-c-z-re).

One inner ADMM iteration of Algorithm 2 with the over-relaxation of Section 4.2:
  (1) utilde = (I+Q)^{-1}(u + v)                        eq. (Simple-Update:Affine)
  (2) uhat   = alpha*utilde + (1-alpha)*u                Section 4.2
  (3) y = uhat_y, theta = uhat_theta, x and tau are the positive roots of the
      barrier prox                                      eqs. (Simple-Update:Barrier-*)
  (4) v = v - uhat + u_new                               eq. (Simple-Update:Dual)
The inner loop stops when ||Qu - v||^2 <= mu (eq. inner-stop); the outer loop
multiplies mu by gamma and restarts the iterate (eq. update-next-iterate, or the
per-coordinate heuristic described in Section 5); the whole method stops on the
tests of Section 4.1.

Readings where the paper is silent (each one is listed in the design notes):
  * beta = 1 (mu^0 = beta, Algorithm 2), gamma fixed per solve.
  * the default restart is the per-coordinate heuristic of Section 5; it keeps
    y and theta unchanged and a tie x_j == s_j scales s_j.
  * the final test is applied to the post-update iterate, in the order
    optimal -> primal infeasible -> dual infeasible; the duality-gap test uses
    the tau-scaled candidate; the certificate tests are skipped when their
    denominators vanish or have the wrong sign.
  * the linear system keeps the theta row/column: Section 4.4's Schur/SMW
    reduction with a rank-2 border H = [(-b; c), (bbar; -cbar)].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

SOLVED = 1
PRIMAL_INFEASIBLE = 2
DUAL_INFEASIBLE = 3
MAX_ITERS = 4
MU_STOP = 5          # only in the mu-stop test mode (outer loop ends when mu < eps)

STATUS_NAMES = {SOLVED: "solved", PRIMAL_INFEASIBLE: "primal_infeasible",
                DUAL_INFEASIBLE: "dual_infeasible", MAX_ITERS: "max_iters",
                MU_STOP: "mu_stop"}


@dataclasses.dataclass
class Settings:
    """Run parameters.  eps is used for all five tolerances (Section 5)."""
    eps: float = 1e-6
    alpha: float = 1.8          # over-relaxation (Section 4.2; Section 5 uses 1.8)
    beta: float = 1.0           # penalty parameter; mu^0 = beta (Algorithm 2)
    gamma: float = 0.5          # mu reduction factor (fixed; chosen by a sweep)
    max_admm_iters: int = 1_000_000   # Section 5
    restart_rule: str = "heuristic"   # "heuristic" (Section 5) or "sqrt" (Algorithm 2)
    mu_stop: float | None = None      # if set: stop the outer loop once mu < mu_stop
    keep_history: bool = False
    bb: bool = False                  # Barzilai-Borwein choice of beta per outer iteration (Section 4.3)
    eps_cor: float = 0.2              # Section 5 defaults of the Section 4.3 rule
    eps_penalty: float = 0.1
    bb_max_redo: int = 10             # [reading] bound on the "redo" branch of Section 4.3


@dataclasses.dataclass
class Problem:
    A: np.ndarray
    b: np.ndarray
    c: np.ndarray

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def n(self):
        return self.A.shape[1]


@dataclasses.dataclass
class State:
    """(u, v) with u = (y, x, tau, theta), v = (r = 0, s, kappa, xi = -(n+1))."""
    y: np.ndarray
    x: np.ndarray
    tau: float
    theta: float
    s: np.ndarray
    kappa: float
    mu: float

    def copy(self):
        return State(self.y.copy(), self.x.copy(), self.tau, self.theta,
                     self.s.copy(), self.kappa, self.mu)

    def u(self):
        return np.concatenate([self.y, self.x, [self.tau, self.theta]])

    def v(self):
        n = self.x.size
        return np.concatenate([np.zeros_like(self.y), self.s, [self.kappa, -(n + 1.0)]])


def _as_problem(A, b=None, c=None):
    if isinstance(A, Problem):
        return A
    if hasattr(A, "tocsr"):           # scipy.sparse: kept sparse (CG solver only)
        A = A.tocsr().astype(np.float64)
    else:
        A = np.asarray(A, dtype=np.float64)
    return Problem(A, np.asarray(b, dtype=np.float64), np.asarray(c, dtype=np.float64))


def hsd_constants(prob):
    """bbar = b - A e, cbar = c - e, zbar = c^T e + 1  (eq. bar-b-c-z-re)."""
    e = np.ones(prob.n)
    return prob.b - prob.A @ e, prob.c - e, float(prob.c @ e) + 1.0


def assemble_Q(prob):
    """The dense skew-symmetric (m+n+2) x (m+n+2) matrix Q of Section 3.1."""
    A, b, c = prob.A, prob.b, prob.c
    m, n = A.shape
    bbar, cbar, zbar = hsd_constants(prob)
    N = m + n + 2
    Q = np.zeros((N, N))
    iy, ix, it, ih = slice(0, m), slice(m, m + n), m + n, m + n + 1
    Q[iy, ix] = A
    Q[iy, it] = -b
    Q[iy, ih] = bbar
    Q[ix, iy] = -A.T
    Q[ix, it] = c
    Q[ix, ih] = -cbar
    Q[it, iy] = b
    Q[it, ix] = -c
    Q[it, ih] = zbar
    Q[ih, iy] = -bbar
    Q[ih, ix] = cbar
    Q[ih, it] = -zbar
    return Q


def apply_Q(prob, u):
    """Q u without forming Q, row block by row block (Section 3.1)."""
    A, b, c = prob.A, prob.b, prob.c
    m, n = A.shape
    bbar, cbar, zbar = hsd_constants(prob)
    y, x, tau, theta = u[:m], u[m:m + n], u[m + n], u[m + n + 1]
    return np.concatenate([
        A @ x - b * tau + bbar * theta,
        -A.T @ y + c * tau - cbar * theta,
        [b @ y - c @ x + zbar * theta],
        [-bbar @ y + cbar @ x - zbar * tau],
    ])


class DenseIQSolver:
    """(I+Q)^{-1} w by an LU factorization of the assembled matrix (small sizes)."""

    def __init__(self, prob):
        N = prob.m + prob.n + 2
        self.lu = sla.lu_factor(np.eye(N) + assemble_Q(prob))

    def solve(self, w):
        return sla.lu_solve(self.lu, w)


class SchurIQSolver:
    """(I+Q)^{-1} w through the structure of Section 4.4.

    I + Q = [[M, H], [-H^T, I2 + S]] with M = [[I, A], [-A^T, I]],
    H = [h1 h2], h1 = (-b; c), h2 = (bbar; -cbar), S = [[0, zbar], [-zbar, 0]].
    M^{-1}(e; f) = (a; f + A^T a) with a = (I + A A^T)^{-1}(e - A f); the
    Cholesky factor of G = I + A A^T is computed once.  The border is
    eliminated with the cached Z = M^{-1} H and the 2x2 K = I2 + S + H^T Z
    (the paper caches M^{-1} h for its rank-1 border; the theta column makes
    it rank 2).
    """

    def __init__(self, prob):
        A, b, c = prob.A, prob.b, prob.c
        m, n = A.shape
        self.prob = prob
        self.m, self.n = m, n
        bbar, cbar, zbar = hsd_constants(prob)
        G = np.eye(m) + A @ A.T
        self.cho = sla.cho_factor(G, lower=True)
        H = np.zeros((m + n, 2))
        H[:m, 0] = -b
        H[m:, 0] = c
        H[:m, 1] = bbar
        H[m:, 1] = -cbar
        self.H = H
        self.Z = np.column_stack([self.apply_Minv(H[:, 0]), self.apply_Minv(H[:, 1])])
        S = np.array([[0.0, zbar], [-zbar, 0.0]])
        self.K = np.eye(2) + S + H.T @ self.Z

    def apply_Minv(self, w):
        m = self.m
        A = self.prob.A
        e, f = w[:m], w[m:]
        a = sla.cho_solve(self.cho, e - A @ f)
        return np.concatenate([a, f + A.T @ a])

    def solve(self, w):
        m, n = self.m, self.n
        z = self.apply_Minv(w[:m + n])
        pq = np.linalg.solve(self.K, w[m + n:] + self.H.T @ z)
        return np.concatenate([z - self.Z @ pq, pq])


class CGIQSolver:
    """(I+Q)^{-1} w by the structure of Section 4.4 with the inner solve
    G a = e - A f (G = I + A A^T) done by conjugate gradients, the paper's
    indirect variant: each CG iteration multiplies once by A and once by A^T,
    so A may be a scipy.sparse matrix and G is never formed.

    [reading] Jacobi preconditioner diag(G)_i = 1 + ||A_i,:||^2; CG starts from
    the previous solve's a (warm start) and stops when ||r|| <= tol ||rhs||.
    The border Z = M^{-1} H is solved once to ``border_tol``.  With a tight tol
    the result equals ``SchurIQSolver`` (pinned in the tests).
    """

    def __init__(self, prob, tol=1e-7, max_iters=500, border_tol=1e-14):
        A, b, c = prob.A, prob.b, prob.c
        m, n = A.shape
        self.A = A
        self.m, self.n = m, n
        self.tol, self.max_iters = tol, max_iters
        bbar, cbar, zbar = hsd_constants(prob)
        if hasattr(A, "multiply"):
            self.dinv = 1.0 / (1.0 + np.asarray(A.multiply(A).sum(axis=1)).ravel())
        else:
            self.dinv = 1.0 / (1.0 + np.einsum("ij,ij->i", A, A))
        self.a_prev = np.zeros(m)
        self.cg_iters = 0
        H = np.zeros((m + n, 2))
        H[:m, 0] = -b
        H[m:, 0] = c
        H[:m, 1] = bbar
        H[m:, 1] = -cbar
        self.H = H
        z0 = self._minv(H[:, 0], border_tol, warm=False)
        z1 = self._minv(H[:, 1], border_tol, warm=False)
        self.Z = np.column_stack([z0, z1])
        S = np.array([[0.0, zbar], [-zbar, 0.0]])
        self.K = np.eye(2) + S + H.T @ self.Z

    def _cg(self, rhs, x0, tol):
        A = self.A
        x = x0.copy()
        r = rhs - (x + A @ (A.T @ x))
        z = self.dinv * r
        p = z.copy()
        rz = r @ z
        nrhs = np.linalg.norm(rhs)
        for _ in range(self.max_iters):
            if np.linalg.norm(r) <= tol * nrhs:
                break
            Gp = p + A @ (A.T @ p)
            al = rz / (p @ Gp)
            x += al * p
            r -= al * Gp
            z = self.dinv * r
            rz1 = r @ z
            p = z + (rz1 / rz) * p
            rz = rz1
            self.cg_iters += 1
        return x

    def _minv(self, w, tol, warm=True):
        m = self.m
        e, f = w[:m], w[m:]
        a = self._cg(e - self.A @ f, self.a_prev if warm else np.zeros(m), tol)
        if warm:
            self.a_prev = a
        return np.concatenate([a, f + self.A.T @ a])

    def solve(self, w):
        m, n = self.m, self.n
        z = self._minv(w[:m + n], self.tol)
        pq = np.linalg.solve(self.K, w[m + n:] + self.H.T @ z)
        return np.concatenate([z - self.Z @ pq, pq])


def barrier_prox(w, t):
    """Positive root of z^2 - w z - t = 0, i.e. argmin_z -t log z + (z - w)^2 / 2.

    This is the closed form of eqs. (Simple-Update:Barrier-X/-tau), evaluated in
    the cancellation-free form 2t / (sqrt(w^2 + 4t) - w) when w < 0.
    """
    w = np.asarray(w, dtype=np.float64)
    r = np.sqrt(w * w + 4.0 * t)
    with np.errstate(divide="ignore", invalid="ignore"):
        neg = 2.0 * t / (r - w)
    return np.where(w >= 0.0, 0.5 * (w + r), neg)


def initial_state(prob, settings):
    """Algorithm 2's start: mu^0 = beta, (y, x, tau, theta) = (0, e, 1, 1),
    (r, s, kappa, xi) = (0, e, 1, -(n+1))."""
    m, n = prob.m, prob.n
    return State(np.zeros(m), np.ones(n), 1.0, 1.0, np.ones(n), 1.0, settings.beta)


def admm_iteration(prob, solver, st, settings, return_v=False, beta=None, return_ut=False):
    """One relaxed inner iteration of Algorithm 2 (Section 4.2 form).

    With ``return_v`` the full updated v = (r, s, kappa, xi) is returned too, so
    that Theorem 3.1's claims r = 0 and xi = -(n+1) can be checked; with
    ``return_ut`` also the affine step u~ (before relaxation).  ``beta``
    overrides settings.beta (the outer iteration's beta of Section 4.3).
    """
    n = prob.n
    m = prob.m
    a = settings.alpha
    t = st.mu / (settings.beta if beta is None else beta)
    u = st.u()
    v = st.v()
    ut = solver.solve(u + v)                          # eq. (Simple-Update:Affine)
    uh = a * ut + (1.0 - a) * u                       # Section 4.2
    y_new = uh[:m]                                    # eq. (Simple-Update:Barrier-Y)
    x_new = barrier_prox(uh[m:m + n] - st.s, t)       # eq. (Simple-Update:Barrier-X)
    tau_new = float(barrier_prox(uh[m + n] - st.kappa, t))   # eq. (...-tau)
    theta_new = float(uh[m + n + 1])                  # eq. (...-theta)
    u_new = np.concatenate([y_new, x_new, [tau_new, theta_new]])
    v_new = v - uh + u_new                            # eq. (Simple-Update:Dual)
    out = State(y_new, x_new, tau_new, theta_new, v_new[m:m + n].copy(),
                float(v_new[m + n]), st.mu)
    if return_ut:
        return out, v_new, ut
    return (out, v_new) if return_v else out


def inner_residual(prob, st):
    """||Q u - v||^2, the left side of eq. (inner-stop)."""
    r = apply_Q(prob, st.u()) - st.v()
    return float(r @ r)


def termination(prob, st, eps):
    """Section 4.1.  Returns (status or 0, dict of residuals).

    Optimality is tested on the candidate (x/tau, y/tau, s/tau) when tau > 0;
    then the primal and dual infeasibility certificates.
    """
    A, b, c = prob.A, prob.b, prob.c
    Ax = A @ st.x
    ATy = A.T @ st.y
    nb = float(np.linalg.norm(b))
    nc = float(np.linalg.norm(c))
    info = {}
    if st.tau > 0:
        pres = float(np.linalg.norm(Ax / st.tau - b))
        dres = float(np.linalg.norm(ATy / st.tau + st.s / st.tau - c))
        pobj = float(c @ st.x) / st.tau
        dobj = float(b @ st.y) / st.tau
        gap = abs(pobj - dobj)
        info.update(pres=pres / (1.0 + nb), dres=dres / (1.0 + nc),
                    gap=gap / (1.0 + abs(pobj) + abs(dobj)), pobj=pobj, dobj=dobj)
        if pres <= eps * (1.0 + nb) and dres <= eps * (1.0 + nc) and \
                gap <= eps * (1.0 + abs(pobj) + abs(dobj)):
            return SOLVED, info
    by = float(b @ st.y)
    if nb > 0.0 and by > 0.0:
        if np.linalg.norm(ATy + st.s) <= eps * by / nb:
            return PRIMAL_INFEASIBLE, info
    cx = float(c @ st.x)
    if nc > 0.0 and cx < 0.0:
        if np.linalg.norm(Ax) <= eps * (-cx) / nc:
            return DUAL_INFEASIBLE, info
    return 0, info


def restart(st, gamma, rule):
    """Start of the next outer iteration.

    rule "sqrt": every one of (y, x, s, tau, kappa, theta) times sqrt(gamma)
    (eq. update-next-iterate).  rule "heuristic" (Section 5): in each pair
    (x_j, s_j), if x_j >= s_j scale s_j by gamma, otherwise scale x_j; the
    same for (tau, kappa); y and theta unchanged.
    Both keep x o s = (gamma mu / beta) e and tau kappa = gamma mu / beta.
    """
    st = st.copy()
    if rule == "sqrt":
        g = math.sqrt(gamma)
        st.y *= g
        st.x *= g
        st.s *= g
        st.tau *= g
        st.kappa *= g
        st.theta *= g
    elif rule == "heuristic":
        big_x = st.x >= st.s
        st.s = np.where(big_x, gamma * st.s, st.s)
        st.x = np.where(big_x, st.x, gamma * st.x)
        if st.tau >= st.kappa:
            st.kappa *= gamma
        else:
            st.tau *= gamma
    else:
        raise ValueError(rule)
    st.mu = gamma * st.mu
    return st


def _hybrid(sd, mg):
    """The hybrid spectral step of Section 4.3: MG when 2 MG > SD, else SD - MG/2."""
    return mg if 2.0 * mg > sd else sd - 0.5 * mg


def bb_estimate(u0, v0, ut1, u1, v1, ut2, u2, v2, alpha, beta, eps_cor):
    """Spectral estimate of beta from the first three iterates of an outer
    iteration (Section 4.3): curvature pairs, the steepest-descent and
    minimum-gradient steps, their hybrid, and the correlation safeguard.

    Returns (beta_hat, diagnostics); beta_hat == beta when neither curvature
    estimate is reliable (both correlations <= eps_cor).
    """
    vh1 = v0 - alpha * ut1 - (1.0 - alpha) * u0 + alpha * u1
    vh2 = v1 - alpha * ut2 - (1.0 - alpha) * u1 + alpha * u2
    dvh = vh2 - vh1
    dut = alpha * (ut2 - ut1) + (1.0 - alpha) * (u1 - u0)
    du = -(u2 - u1)
    vv, vt, tt = float(dvh @ dvh), float(dvh @ dut), float(dut @ dut)
    vu, uu = float(dvh @ du), float(du @ du)
    nv, nt, nu = np.sqrt(vv), np.sqrt(tt), np.sqrt(uu)
    phi_cor = vt / (nv * nt) if nv > 0 and nt > 0 else 0.0
    psi_cor = vu / (nv * nu) if nv > 0 and nu > 0 else 0.0
    d = dict(phi_cor=phi_cor, psi_cor=psi_cor)
    phi = psi = None
    if phi_cor > eps_cor:
        d["phi_sd"], d["phi_mg"] = vv / vt, vt / tt
        phi = _hybrid(d["phi_sd"], d["phi_mg"])
    if psi_cor > eps_cor:
        d["psi_sd"], d["psi_mg"] = vv / vu, vu / uu
        psi = _hybrid(d["psi_sd"], d["psi_mg"])
    d["phi"], d["psi"] = phi, psi
    if phi is not None and psi is not None:
        return float(np.sqrt(phi * psi)), d
    if phi is not None:
        return float(phi), d
    if psi is not None:
        return float(psi), d
    return beta, d


def bb_rule(beta, beta_hat, eps_penalty):
    """The heuristic selection of Section 4.3: ("keep", beta) when the estimate
    equals beta, ("average", (beta + beta_hat)/2) when it is within eps_penalty,
    ("redo", beta_hat) otherwise (estimate again from the same initial point)."""
    if beta_hat == beta:
        return "keep", beta
    if abs(beta_hat - beta) <= eps_penalty:
        return "average", 0.5 * (beta + beta_hat)
    return "redo", beta_hat


def bb_select(prob, solver, st0, settings, beta):
    """Choose the beta of an outer iteration (Section 4.3) from its initial point.

    [reading] Each estimate takes two probe iterations from st0 with the current
    beta; the probes are then discarded and the outer iteration starts from st0
    with the chosen beta; st0 is not rescaled (a redo uses the same initial
    point).  At most settings.bb_max_redo redos.  Returns (beta, probe
    iterations, list of (action, beta)).
    """
    probes = 0
    trail = []
    for _ in range(settings.bb_max_redo + 1):
        u0, v0 = st0.u(), st0.v()
        st1, v1, ut1 = admm_iteration(prob, solver, st0, settings, beta=beta, return_ut=True)
        st2, v2, ut2 = admm_iteration(prob, solver, st1, settings, beta=beta, return_ut=True)
        probes += 2
        beta_hat, _ = bb_estimate(u0, v0, ut1, st1.u(), v1, ut2, st2.u(), v2, settings.alpha, beta,
                                  settings.eps_cor)
        action, nb = bb_rule(beta, beta_hat, settings.eps_penalty)
        trail.append((action, nb))
        if action != "redo" or not (nb > 0.0) or not np.isfinite(nb):
            if action == "redo":                      # a non-positive estimate: keep beta
                trail[-1] = ("keep", beta)
                return beta, probes, trail
            return nb, probes, trail
        beta = nb
    return beta, probes, trail


def solve(A, b=None, c=None, settings=None, solver=None, state=None):
    """Algorithm 2 (with Section 4.1-4.2 and the Section 5 restart).

    Returns a dict with status, the candidate solution (x/tau, y/tau, s/tau) or
    the normalised certificate, the final HSD state, and iteration counts.
    """
    prob = _as_problem(A, b, c)
    settings = settings or Settings()
    if solver is None:
        solver = SchurIQSolver(prob)
    st = state.copy() if state is not None else initial_state(prob, settings)
    total = 0
    outer = 0
    inner_counts = []
    history = []
    betas = []
    status = 0
    info = {}
    beta = settings.beta
    while status == 0:
        if settings.mu_stop is not None and st.mu < settings.mu_stop:
            status = MU_STOP
            break
        i = 0
        if settings.bb and inner_residual(prob, st) > st.mu:
            beta, probes, trail = bb_select(prob, solver, st, settings, beta)   # Section 4.3
            total += probes
            betas.append((outer, beta, trail))
        while True:
            res = inner_residual(prob, st)
            if res <= st.mu:                          # eq. (inner-stop)
                break
            if total >= settings.max_admm_iters:
                status = MAX_ITERS
                break
            st = admm_iteration(prob, solver, st, settings, beta=beta)
            total += 1
            i += 1
            if settings.mu_stop is None:
                status, info = termination(prob, st, settings.eps)
                if settings.keep_history:
                    history.append(dict(k=outer, i=i, mu=st.mu, **info))
                if status:
                    break
        inner_counts.append(i)
        if status:
            break
        st = restart(st, settings.gamma, settings.restart_rule)
        outer += 1
    out = dict(status=status, status_name=STATUS_NAMES.get(status, "?"), state=st,
               admm_iters=total, ipm_iters=outer, inner_counts=inner_counts,
               history=history, info=info, betas=betas)
    if status in (SOLVED, MAX_ITERS, MU_STOP) and st.tau > 0:
        out.update(x=st.x / st.tau, y=st.y / st.tau, s=st.s / st.tau)
    elif status == PRIMAL_INFEASIBLE:
        by = float(prob.b @ st.y)
        out.update(y=st.y / by, s=st.s / by, x=np.full(prob.n, np.nan))
    elif status == DUAL_INFEASIBLE:
        cx = float(prob.c @ st.x)
        out.update(x=-st.x / cx, y=np.full(prob.m, np.nan), s=np.full(prob.n, np.nan))
    return out


# ---------------------------------------------------------------------------
# Algorithm 1 (explicit multipliers p, q) -- used only to pin Theorem 3.1
# ---------------------------------------------------------------------------

def alg1_initial(st):
    """Theorem 3.1's initialisation: p = v, q = u."""
    return dict(u=st.u(), v=st.v(), p=st.v(), q=st.u())


def alg1_iteration(prob, z, mu, beta):
    """One iteration of Algorithm 1: eqs. (admm-typical-1/2/3), no relaxation.

    The projection onto {(u, v): Q u = v} is computed from its definition,
    min ||u' - a||^2 + ||Q u' - b||^2, i.e. (I + Q^T Q) u' = a + Q^T b, v' = Q u'.
    The barrier step minimises B(u, v, mu) + beta/2 ||(u,v) - (u~,v~) + (p,q)||^2
    coordinate-wise.
    """
    m, n = prob.m, prob.n
    Q = assemble_Q(prob)
    N = m + n + 2
    a = z["u"] + z["p"]
    bb = z["v"] + z["q"]
    ut = np.linalg.solve(np.eye(N) + Q.T @ Q, a + Q.T @ bb)
    vt = Q @ ut
    t = mu / beta
    p, q = z["p"], z["q"]
    iy, ix, it, ih = slice(0, m), slice(m, m + n), m + n, m + n + 1
    u = np.empty(N)
    v = np.empty(N)
    u[iy] = ut[iy] - p[iy]
    u[ix] = barrier_prox(ut[ix] - p[ix], t)
    u[it] = barrier_prox(ut[it] - p[it], t)
    u[ih] = ut[ih] - p[ih] - (n + 1.0)      # linear term beta (n+1) theta
    v[iy] = 0.0                              # indicator r = 0
    v[ix] = barrier_prox(vt[ix] - q[ix], t)
    v[it] = barrier_prox(vt[it] - q[it], t)
    v[ih] = -(n + 1.0)                       # indicator xi = -(n+1)
    return dict(u=u, v=v, p=p - ut + u, q=q - vt + v)
