"""Seeded synthetic LP instances shared by the oracle tests, the GPU tests and the bench.

This module only draws random data and assembles LP data (A, b, c) from planted
primal/dual pairs.  It contains none of the solver's arithmetic, so both the
FP64 oracle and the HIP path can consume its output without sharing any
method code.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and returns a
plain dict.  Dense A is returned row-major float64 (m x n); sparse A is CSR
(``indptr``, ``indices``, ``data``; int32 / float64).

Workloads (the paper's own instances -- NETLIB, UCI -- are not available, so
these synthetic shapes stand in for them):

* ``dense_planted``      -- the random feasible LP family: A ~ N(0,1), a
                            planted strictly complementary (x0, y0, s0).
* ``sparse_planted``     -- a sparse NETLIB-sized LP (random CSR plus a
                            full-rank diagonal block), planted the same way.
* ``basis_pursuit``      -- min ||x||_1 s.t. A0 x = b written as a standard LP
                            with x = x+ - x-.
* ``batch``              -- many dense planted LPs of uneven size, a fraction
                            of them made primal infeasible by a planted
                            Farkas vector.
* ``paper_random``       -- the random dense LP recipe of the paper's random-LP
                            experiments (Section 5): A = U^T D V with sparse
                            Gaussian factors, a planted x split 60/10/30 into
                            zero / ten times larger / ten times smaller entries,
                            complementary s, Gaussian y.
* ``sice``               -- the sparse inverse covariance estimation LPs of
                            Section 5 (one LP per column of Omega) with a
                            synthetic sample covariance standing in for the UCI
                            data.
* toy LPs with closed-form answers.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "dense_planted",
    "dense_farkas_infeasible",
    "sparse_planted",
    "basis_pursuit",
    "batch",
    "diff_batch",
    "toy_simplex",
    "toy_two_var",
    "toy_primal_infeasible",
    "toy_dual_infeasible",
    "config0",
    "paper_random",
    "sice",
]


def _planted_pair(rng, A, n_basic):
    """Draw a strictly complementary (x0, y0, s0) for A with |supp x0| = n_basic.

    x0 is U(0,1) on a random support B, zero elsewhere; s0 is U(0,1) on the
    complement of B and zero on B; y0 ~ N(0,1).
    """
    m, n = A.shape
    perm = rng.permutation(n)
    B = np.sort(perm[:n_basic])
    N = np.sort(perm[n_basic:])
    x0 = np.zeros(n)
    s0 = np.zeros(n)
    x0[B] = rng.uniform(0.0, 1.0, size=B.size)
    s0[N] = rng.uniform(0.0, 1.0, size=N.size)
    y0 = rng.standard_normal(m)
    return x0, y0, s0, B


def dense_planted(m, n, seed, n_basic=None):
    """Dense random feasible LP with a planted optimal pair.

    A_ij ~ N(0,1); x0 has ``n_basic`` coordinates U(0,1) (default m, so the
    planted optimum is a nondegenerate vertex and unique), s0 is U(0,1) on the
    zero set of x0, y0 ~ N(0,1); b = A x0 and c = A^T y0 + s0.
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    if n_basic is None:
        n_basic = m
    x0, y0, s0, B = _planted_pair(rng, A, n_basic)
    b = A @ x0
    c = A.T @ y0 + s0
    return dict(A=A, b=b, c=c, x0=x0, y0=y0, s0=s0, basis=B,
                pstar=float(c @ x0), status="solved", m=m, n=n)


def config0(seed):
    """The small dense workload: m=50, n=100, 50 planted positive x0 coordinates."""
    return dense_planted(50, 100, seed, n_basic=50)


def dense_farkas_infeasible(m, n, seed):
    """Dense LP made primal infeasible by a planted Farkas vector y_c.

    Start from a planted instance, then bend A so that A^T y_c <= -delta < 0 and
    choose b with b^T y_c = 1 > 0: no x >= 0 can satisfy A x = b.
    """
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x0, y0, s0, B = _planted_pair(rng, A, m)
    yc = rng.standard_normal(m)
    g = A.T @ yc
    delta = 0.1 * np.mean(np.abs(g))
    A = A - np.outer(yc, np.maximum(g, 0.0) + delta) / (yc @ yc)
    eta = (1.0 - x0 @ (A.T @ yc)) / (yc @ yc)
    b = A @ x0 + eta * yc
    c = A.T @ y0 + s0
    return dict(A=A, b=b, c=c, farkas=yc, status="primal_infeasible", m=m, n=n)


def sparse_planted(m, n, seed, density=1e-3):
    """Sparse NETLIB-sized feasible LP, CSR.

    A = R + [diag(d) | 0] with R a uniform random sparse pattern of about
    density*m*n entries valued U(-1,1) and d ~ U(1,2) on columns 0..m-1 (the
    full-rank diagonal block).  The planted basis is B = {0..m-1}.
    """
    rng = np.random.default_rng(seed)
    target = int(round(density * m * n))
    flat = np.unique(rng.integers(0, m * n, size=target, dtype=np.int64))
    rows = (flat // n).astype(np.int64)
    cols = (flat % n).astype(np.int64)
    vals = rng.uniform(-1.0, 1.0, size=flat.size)
    d = rng.uniform(1.0, 2.0, size=m)
    rows = np.concatenate([rows, np.arange(m)])
    cols = np.concatenate([cols, np.arange(m)])
    vals = np.concatenate([vals, d])
    # merge duplicates (a random entry landing on the diagonal) by summation
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, rows, cols, vals = key[order], rows[order], cols[order], vals[order]
    uniq, start = np.unique(key, return_index=True)
    vals = np.add.reduceat(vals, start)
    rows = rows[start]
    cols = cols[start]
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    B = np.arange(m)
    x0 = np.zeros(n)
    s0 = np.zeros(n)
    x0[:m] = rng.uniform(0.0, 1.0, size=m)
    s0[m:] = rng.uniform(0.0, 1.0, size=n - m)
    y0 = rng.standard_normal(m)
    csr = dict(indptr=indptr.astype(np.int32), indices=cols.astype(np.int32),
               data=vals.astype(np.float64), shape=(m, n))
    # b = A x0 and c = A^T y0 + s0 assembled entry by entry from the CSR lists
    b = np.zeros(m)
    np.add.at(b, rows, vals * x0[cols])
    c = s0.copy()
    np.add.at(c, cols, vals * y0[rows])
    return dict(A_csr=csr, b=b, c=c, x0=x0, y0=y0, s0=s0, basis=B,
                pstar=float(c @ x0), status="solved", m=m, n=n, nnz=int(vals.size))


def basis_pursuit(m, N, k, seed):
    """Basis pursuit min ||x||_1 s.t. A0 x = b as a standard-form LP.

    A0 is m x N with iid N(0,1)/sqrt(m) entries, x_true has k nonzeros N(0,1)
    at random positions, b = A0 x_true.  LP data: A = [A0, -A0], c = e,
    x = (x+, x-).  When l1 recovery holds the optimum is ||x_true||_1.
    """
    rng = np.random.default_rng(seed)
    A0 = rng.standard_normal((m, N)) / np.sqrt(m)
    x_true = np.zeros(N)
    pos = rng.choice(N, size=k, replace=False)
    x_true[pos] = rng.standard_normal(k)
    b = A0 @ x_true
    A = np.concatenate([A0, -A0], axis=1)
    c = np.ones(2 * N)
    xp = np.maximum(x_true, 0.0)
    xm = np.maximum(-x_true, 0.0)
    return dict(A=A, b=b, c=c, A0=A0, x_true=x_true, x0=np.concatenate([xp, xm]),
                pstar=float(np.abs(x_true).sum()), status="solved", m=m, n=2 * N)


def batch(count, seed, m_lo=20, m_hi=400, infeasible_frac=0.1):
    """Many dense LPs of uneven size: m ~ U{m_lo..m_hi}, n ~ U{2m..3m}.

    Each LP is a planted instance with |supp x0| = m; round(count*frac) of them,
    picked at random, are made primal infeasible with a planted Farkas vector.
    Per-LP seeds are derived from ``seed`` so each LP is reproducible alone.
    """
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = np.array([rng.integers(2 * mm, 3 * mm + 1) for mm in ms])
    n_inf = int(round(count * infeasible_frac))
    infeasible = np.zeros(count, dtype=bool)
    infeasible[rng.choice(count, size=n_inf, replace=False)] = True
    seeds = rng.integers(0, 2**31 - 1, size=count)
    lps = []
    for i in range(count):
        if infeasible[i]:
            lp = dense_farkas_infeasible(int(ms[i]), int(ns[i]), int(seeds[i]))
        else:
            lp = dense_planted(int(ms[i]), int(ns[i]), int(seeds[i]))
        lp["seed"] = int(seeds[i])
        lps.append(lp)
    return lps


def diff_batch(count, m, n, seed):
    """Batch of planted LPs with a random loss weight w ~ N(0, I_n) per LP."""
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    lps = []
    for i in range(count):
        lp = dense_planted(m, n, int(seeds[i]))
        lp["w"] = np.random.default_rng(int(seeds[i]) + 1).standard_normal(n)
        lp["seed"] = int(seeds[i])
        lps.append(lp)
    return lps


# ---------------------------------------------------------------------------
# toy LPs with answers known in closed form
# ---------------------------------------------------------------------------

def toy_simplex(n, seed):
    """min c^T x s.t. e^T x = 1, x >= 0: the optimum is min_j c_j."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1.0, 1.0, size=n)
    A = np.ones((1, n))
    b = np.ones(1)
    j = int(np.argmin(c))
    x = np.zeros(n)
    x[j] = 1.0
    return dict(A=A, b=b, c=c, pstar=float(c[j]), xstar=x, ystar=np.array([c[j]]),
                status="solved", m=1, n=n)


def toy_two_var():
    """min x1 + 2 x2 s.t. x1 + x2 = 1: x* = (1,0), y* = 1, s* = (0,1)."""
    return dict(A=np.array([[1.0, 1.0]]), b=np.array([1.0]), c=np.array([1.0, 2.0]),
                pstar=1.0, xstar=np.array([1.0, 0.0]), ystar=np.array([1.0]),
                sstar=np.array([0.0, 1.0]), status="solved", m=1, n=2)


def toy_primal_infeasible():
    """x1 + x2 = -1, x >= 0 has no solution; y = -1 is a Farkas certificate."""
    return dict(A=np.array([[1.0, 1.0]]), b=np.array([-1.0]), c=np.array([1.0, 1.0]),
                certificate=np.array([-1.0]), status="primal_infeasible", m=1, n=2)


def toy_dual_infeasible():
    """min -x1 s.t. x1 - x2 = 0: unbounded along the ray (1, 1)."""
    return dict(A=np.array([[1.0, -1.0]]), b=np.array([0.0]), c=np.array([-1.0, 0.0]),
                ray=np.array([1.0, 1.0]) / np.sqrt(2.0), status="dual_infeasible", m=1, n=2)


def _sprandn(rng, rows, cols, density):
    """Dense array with a uniform random pattern of about density*rows*cols
    standard normal entries (the rest zero)."""
    mask = rng.random((rows, cols)) < density
    return np.where(mask, rng.standard_normal((rows, cols)), 0.0)


def paper_random(m, n, seed):
    """The random dense LP recipe of the paper's random-LP experiments (Section 5).

    x: Gaussian, split at random into 60% zeros, 10% scaled by 10 and 30%
    scaled by 1/10; s: standard normal on the zero set of x, zero elsewhere, so
    x o s = 0.  The paper's text leaves the signs of x and s free, which would
    break x, s >= 0; absolute values are taken.  A = U^T D V with
    D = diag(N(0,1)), U an m x m and V an m x n sparse Gaussian matrix of
    density 0.2; y ~ N(0,1); b = A x, c = A^T y + s, so (x, y, s) is a planted
    optimal pair (the optimum need not be unique; the optimal value
    c^T x = b^T y is).
    """
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    perm = rng.permutation(n)
    n0, n1 = int(round(0.6 * n)), int(round(0.1 * n))
    zero, big, small = perm[:n0], perm[n0:n0 + n1], perm[n0 + n1:]
    x[zero] = 0.0
    x[big] *= 10.0
    x[small] *= 0.1
    x = np.abs(x)
    s = np.zeros(n)
    s[zero] = np.abs(rng.standard_normal(zero.size))
    D = rng.standard_normal(m)
    U = _sprandn(rng, m, m, 0.2)
    V = _sprandn(rng, m, n, 0.2)
    A = U.T @ (D[:, None] * V)
    y = rng.standard_normal(m)
    b = A @ x
    c = A.T @ y + s
    return dict(A=A, b=b, c=c, x0=x, y0=y, s0=s, pstar=float(c @ x), status="solved", m=m, n=n,
                groups=dict(zero=np.sort(zero), big=np.sort(big), small=np.sort(small)))


def sice(d, N, seed, cols=None):
    """Sparse inverse covariance estimation LPs (Section 5), one per column j
    of Omega: min e^T (beta+ + beta-) s.t. Sigma beta+ - Sigma beta- + w+ =
    lambda e + e_j, w+ + w- = 2 lambda e, all variables >= 0; m = 2d, n = 4d.

    Sigma is the sample covariance of N draws of a d-variate Gaussian with a
    random well-conditioned covariance (a stand-in for the UCI data sets, which
    are not available); lambda = (3/2) sqrt(log(d) / N) as in the paper.
    Returns the shared A (2d x 4d, rows [Sigma, -Sigma, I, 0] and [0, 0, I, I]),
    c, and one b per requested column (all d by default).
    """
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((d, d)) / np.sqrt(d)
    cov = L @ L.T + 0.5 * np.eye(d)
    X = rng.standard_normal((N, d)) @ np.linalg.cholesky(cov).T
    X -= X.mean(axis=0)
    Sigma = X.T @ X / N
    lam = 1.5 * np.sqrt(np.log(d) / N)
    I = np.eye(d)
    Z = np.zeros((d, d))
    A = np.block([[Sigma, -Sigma, I, Z], [Z, Z, I, I]])
    c = np.concatenate([np.ones(2 * d), np.zeros(2 * d)])
    cols = list(range(d)) if cols is None else list(cols)
    bs = []
    for j in cols:
        e = np.zeros(d)
        e[j] = 1.0
        bs.append(np.concatenate([lam * np.ones(d) + e, 2.0 * lam * np.ones(d)]))
    return dict(A=A, c=c, bs=bs, cols=cols, Sigma=Sigma, lam=lam, d=d, N=N, m=2 * d, n=4 * d)
