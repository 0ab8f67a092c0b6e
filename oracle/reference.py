"""Independent references that pin the oracle (test infrastructure only).

* ``central_point``   -- the unique solution of the central-path system
                         (HSD-log-kkt) of Section 3 at t = mu/beta, by damped
                         Newton continuation.  Pins the inner loop's limit
                         (Lemma 3.2) and the adjoint.
* ``kkt_adjoint``     -- dense FP64 adjoint of the central-path system.
* ``basis_gradients`` -- derivatives of the basic solution x_B = A_B^{-1} b.
* ``vertex_enumeration`` -- brute-force LP optimum over all bases (tiny LPs).
* ``kkt_relative``    -- the relative residuals of Section 4.1 for a returned
                         (x, y, s), recomputed in FP64.
"""
from __future__ import annotations

import itertools

import numpy as np

from .abip import Problem, State, assemble_Q, _as_problem


def _central_residual(prob, Q, z, t):
    m, n = prob.m, prob.n
    y, x = z[:m], z[m:m + n]
    tau, theta = z[m + n], z[m + n + 1]
    s, kappa = z[m + n + 2:m + 2 * n + 2], z[m + 2 * n + 2]
    u = z[:m + n + 2]
    v = np.concatenate([np.zeros(m), s, [kappa, -(n + 1.0)]])
    return np.concatenate([Q @ u - v, x * s - t, [tau * kappa - t]])


def central_point(A, b=None, c=None, t=1.0, tol=1e-13, max_newton=200):
    """Solve (HSD-log-kkt): Q u = v, x o s = t e, tau kappa = t, r = 0, xi = -(n+1).

    Damped Newton on the full (m + 2n + 3)-dimensional system with a
    fraction-to-boundary rule, continued in t from t = 1 (where the
    Algorithm 2 start point is central) down or up to the requested t.
    Returns a State with mu = t (i.e. beta = 1 units).
    """
    prob = _as_problem(A, b, c)
    m, n = prob.m, prob.n
    Q = assemble_Q(prob)
    N = m + n + 2
    dim = m + 2 * n + 3
    z = np.concatenate([np.zeros(m), np.ones(n), [1.0, 1.0], np.ones(n), [1.0]])
    pos = np.concatenate([np.arange(m, m + n + 1), np.arange(N, dim)])

    def jac(z):
        x = z[m:m + n]
        tau = z[m + n]
        s = z[N:N + n]
        kappa = z[N + n]
        J = np.zeros((dim, dim))
        J[:N, :N] = Q
        J[m:m + n, N:N + n] = -np.eye(n)
        J[m + n, N + n] = -1.0
        J[N:N + n, m:m + n] = np.diag(s)
        J[N:N + n, N:N + n] = np.diag(x)
        J[N + n, m + n] = kappa
        J[N + n, N + n] = tau
        return J

    t_cur = 1.0
    ratio = 0.5 if t < 1.0 else 2.0
    while True:
        t_cur = max(t, t_cur * ratio) if t < 1.0 else min(t, t_cur * ratio)
        for _ in range(max_newton):
            F = _central_residual(prob, Q, z, t_cur)
            if np.linalg.norm(F) <= tol * (1.0 + np.linalg.norm(z)):
                break
            dz = np.linalg.solve(jac(z), -F)
            step = 1.0
            neg = dz[pos] < 0
            if np.any(neg):
                step = min(1.0, 0.95 * float(np.min(-z[pos][neg] / dz[pos][neg])))
            z = z + step * dz
        if t_cur == t:
            break
    # final polish at the target
    for _ in range(5):
        F = _central_residual(prob, Q, z, t)
        z = z + np.linalg.solve(jac(z), -F)
    return State(z[:m].copy(), z[m:m + n].copy(), float(z[m + n]), float(z[m + n + 1]),
                 z[N:N + n].copy(), float(z[N + n]), float(t))


def kkt_adjoint(A, b=None, c=None, st=None, w=None):
    """Dense adjoint of the central-path system at the iterate ``st``.

    Eliminating s and kappa through x o s = t e and tau kappa = t, the central
    path is F(u) = Q u - (0, t/x, t/tau, -(n+1)) = 0 with Jacobian Q + D,
    D = diag(0, s/x, kappa/tau, 0) (the linearisation of x o s = const).
    For L = w^T x / tau the adjoint solves (Q + D)^T lam = (D - Q) lam = dL/du,
    dL/du = (0, w/tau, -w^T x / tau^2, 0).
    """
    prob = _as_problem(A, b, c)
    m, n = prob.m, prob.n
    Q = assemble_Q(prob)
    d = np.concatenate([np.zeros(m), st.s / st.x, [st.kappa / st.tau, 0.0]])
    g = np.concatenate([np.zeros(m), w / st.tau, [-(w @ st.x) / st.tau ** 2, 0.0]])
    return np.linalg.solve(np.diag(d) - Q, g)


def contract_adjoint(A, b=None, c=None, st=None, lam=None, want_A=False):
    """dL/dp = -lam^T d(Q u)/dp for p in (c, b, A), including the dependence of
    bbar, cbar and zbar on the data (eq. bar-b-c-z-re)."""
    prob = _as_problem(A, b, c)
    m, n = prob.m, prob.n
    ly, lx, lt, lh = lam[:m], lam[m:m + n], lam[m + n], lam[m + n + 1]
    y, x, tau, theta = st.y, st.x, st.tau, st.theta
    dc = -(lx * (tau - theta) + lt * (theta - x) + lh * (x - tau))
    db = -(ly * (theta - tau) + lt * y - lh * y)
    out = dict(dc=dc, db=db)
    if want_A:
        out["dA"] = -(np.outer(ly, x - theta) - np.outer(y, lx) + lh * np.outer(y, np.ones(n)))
    return out


def basis_gradients(A, b, basis, w):
    """Derivatives of L = w^T x* for the basic solution x*_B = A_B^{-1} b, x*_N = 0.

    dL/db = A_B^{-T} w_B, dL/dc = 0 (a nondegenerate optimal basis is locally
    constant in c), dL/dA = -(A_B^{-T} w_B) x*^T.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    AB = A[:, basis]
    lam = np.linalg.solve(AB.T, w[basis])
    x = np.zeros(n)
    x[basis] = np.linalg.solve(AB, b)
    return dict(db=lam, dc=np.zeros(n), dA=-np.outer(lam, x), x=x)


def vertex_enumeration(A, b, c, tol=1e-10):
    """Brute-force LP optimum: try every basis, keep feasible vertices, take the min.

    Returns (pstar, xstar) or (None, None) if no feasible vertex exists.  Only
    meaningful for bounded LPs of a few variables.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    best = None
    bestx = None
    for B in itertools.combinations(range(n), m):
        AB = A[:, B]
        if abs(np.linalg.det(AB)) < 1e-12:
            continue
        xB = np.linalg.solve(AB, b)
        if np.all(xB >= -tol):
            x = np.zeros(n)
            x[list(B)] = np.maximum(xB, 0.0)
            val = float(c @ x)
            if best is None or val < best - 1e-12:
                best, bestx = val, x
    return best, bestx


def kkt_relative(A, b, c, x, y, s):
    """Relative residuals of Section 4.1 for a candidate (x, y, s), in FP64."""
    A = np.asarray(A, dtype=np.float64)
    pres = np.linalg.norm(A @ x - b) / (1.0 + np.linalg.norm(b))
    dres = np.linalg.norm(A.T @ y + s - c) / (1.0 + np.linalg.norm(c))
    pobj = float(c @ x)
    dobj = float(b @ y)
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    return dict(pres=float(pres), dres=float(dres), gap=float(gap), pobj=pobj, dobj=dobj)
