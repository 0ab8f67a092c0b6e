"""Presolve, postsolve and scaling of Section 4.5 -- oracle (test infrastructure only).

The input LP has the bounded form of Section 4.5,

    min c^T x  s.t.  A x = b,  l <= x <= w     (l_j may be -inf, w_j may be +inf),

and the output is the standard form (P) of Section 2, min c~^T x~ s.t. A~ x~ = b~,
x~ >= 0, that the solver takes, plus a record that maps a solution of the
reduced problem back to the original one (postsolve).

Reductions, in the order of the paper's list (P1-P6), repeated until none
applies, each scan in ascending index order so that the result is unique:
  P3  l_j > w_j: trivially infeasible.
  P4  l_j = w_j: x_j is fixed and substituted out (b -= A_j x_j).
  P1  an empty row: redundant when b_i = 0 (its multiplier is 0), else infeasible.
  P2  an empty column: x_j goes to the bound its cost favours (the lower bound
      for c_j > 0, the upper for c_j < 0, the finite one -- lower first -- or 0
      for c_j = 0); a favoured bound at infinity means the LP is unbounded (when
      feasible), reported as such.
  P6  a singleton row a_ik x_k = b_i fixes x_k = b_i / a_ik (infeasible when
      outside [l_k, w_k]); the row and the column leave together.
Then the reformulation of Section 4.5 on the columns that remain:
  P5  a free variable is split into x+ - x- (two nonnegative columns);
      [reading] a variable with l_j = -inf and finite w_j is reflected,
      x_j = w_j - x'_j, so that every lower bound is finite as the paper
      requires before the shift;
  shift x = x~ + l (b -= A l), and every finite upper bound w_j becomes a row
  x~_j + t_j = w_j - l_j with a slack column t_j >= 0 (cost 0).
[reading] P7 (dependent rows removed by a Dulmage-Mendelsohn decomposition) is
not applied: the linear step works with G = I + A A^T, which is nonsingular
for any A, so dependent consistent rows need no removal.
[reading] "Empty" means exactly zero entries; b_i counts as zero when
|b_i| <= 1e-9 (1 + max|b|), and a singleton's value lies within its bounds up to
1e-9 (1 + |bound|).

Postsolve returns the original x, the multipliers y of the original rows and
the reduced costs r = c - A^T y (r_j > 0 at a lower bound, r_j < 0 at an upper
bound).  Removed empty rows take y_i = 0; a singleton row takes the y_i that
zeroes the reduced cost of the variable it fixed (rows in reverse order of
removal, so every row still present at that removal already has its y).

Scaling (the remark of Section 4.5, which defers to SCS): [reading] Ruiz
equilibration of A in ``iters`` rounds; each round forms the row and column
max-abs of the current scaled matrix (D_i a_ij) E_j and multiplies D_i by
1/sqrt(row max) and E_j by 1/sqrt(column max) (an all-zero row or column keeps
its factor).  The scaled LP is ((D_i a_ij) E_j, D b, E c), and a solution
(x', y', s') of it maps back as x = E x', y = D y', s = s' / E.  The solver's
tests (Section 4.1) are then taken on the scaled LP; the FP64 recheck of the
returned point measures the original one.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INFEASIBLE, UNBOUNDED, REDUCED = "infeasible", "unbounded", "reduced"


@dataclass
class PresolveRecord:
    m: int
    n: int
    A: np.ndarray                 # the original data, for postsolve
    b: np.ndarray
    c: np.ndarray
    rows: list = field(default_factory=list)       # original rows kept, in order
    cols: list = field(default_factory=list)       # original columns kept (before the reformulation)
    fixed: dict = field(default_factory=dict)      # column -> value (P4, P2, P6)
    removed_rows: list = field(default_factory=list)   # (kind, row, col): kind "empty" or "singleton"
    colmap: list = field(default_factory=list)     # per kept column: (kind, first std column, second or -1, l, w)
    n_std: int = 0                # columns of the standard form
    m_std: int = 0                # rows of the standard form (kept rows + upper-bound rows)
    obj_offset: float = 0.0       # c^T x of the fixed part and of the shift


@dataclass
class PresolveResult:
    status: str                   # REDUCED, INFEASIBLE or UNBOUNDED
    A: np.ndarray | None = None
    b: np.ndarray | None = None
    c: np.ndarray | None = None
    record: PresolveRecord | None = None
    reason: str = ""


def presolve(A, b, c, l=None, w=None):
    """Section 4.5's presolve of min c^T x s.t. A x = b, l <= x <= w (dense A).
    Defaults: l = 0, w = +inf (an LP already in standard form)."""
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    b = np.array(b, dtype=np.float64).copy()
    c = np.array(c, dtype=np.float64)
    l = np.zeros(n) if l is None else np.array(l, dtype=np.float64)
    w = np.full(n, np.inf) if w is None else np.array(w, dtype=np.float64)
    rec = PresolveRecord(m=m, n=n, A=A.copy(), b=b.copy(), c=c.copy())
    rowalive = np.ones(m, dtype=bool)
    colalive = np.ones(n, dtype=bool)
    btol = 1e-9 * (1.0 + (np.abs(b).max() if m else 0.0))

    def fix(j, v):
        # substitute x_j = v: b_i -= a_ij v in ascending row order
        for i in range(m):
            if rowalive[i] and A[i, j] != 0.0:
                b[i] -= A[i, j] * v
        rec.obj_offset += c[j] * v
        rec.fixed[j] = v
        colalive[j] = False

    changed = True
    while changed:
        changed = False
        for j in range(n):                                   # P3
            if colalive[j] and l[j] > w[j]:
                return PresolveResult(INFEASIBLE, reason=f"P3: l > w at column {j}")
        for j in range(n):                                   # P4
            if colalive[j] and l[j] == w[j]:
                fix(j, l[j])
                changed = True
        for i in range(m):                                   # P1
            if rowalive[i] and not np.any(A[i, colalive] != 0.0):
                if abs(b[i]) > btol:
                    return PresolveResult(INFEASIBLE, reason=f"P1: empty row {i} with b = {b[i]:.3g}")
                rowalive[i] = False
                rec.removed_rows.append(("empty", i, -1))
                changed = True
        for j in range(n):                                   # P2
            if colalive[j] and not np.any(A[rowalive, j] != 0.0):
                if c[j] > 0.0:
                    if not np.isfinite(l[j]):
                        return PresolveResult(UNBOUNDED, reason=f"P2: empty column {j}, c > 0, l = -inf")
                    v = l[j]
                elif c[j] < 0.0:
                    if not np.isfinite(w[j]):
                        return PresolveResult(UNBOUNDED, reason=f"P2: empty column {j}, c < 0, w = +inf")
                    v = w[j]
                else:
                    v = l[j] if np.isfinite(l[j]) else (w[j] if np.isfinite(w[j]) else 0.0)
                fix(j, v)
                changed = True
        for i in range(m):                                   # P6
            if not rowalive[i]:
                continue
            nz = [j for j in range(n) if colalive[j] and A[i, j] != 0.0]
            if len(nz) != 1:
                continue
            k = nz[0]
            v = b[i] / A[i, k]
            if v < l[k] - 1e-9 * (1.0 + abs(l[k])) or v > w[k] + 1e-9 * (1.0 + abs(w[k])):
                return PresolveResult(INFEASIBLE, reason=f"P6: row {i} fixes x_{k} = {v:.6g} outside its bounds")
            rowalive[i] = False
            rec.removed_rows.append(("singleton", i, k))
            fix(k, v)
            changed = True

    rows = [i for i in range(m) if rowalive[i]]
    cols = [j for j in range(n) if colalive[j]]
    rec.rows, rec.cols = rows, cols
    # reformulation: P5 split, reflection, shift, upper-bound rows
    std_cols = []          # per standard column: (sign, original column)
    ub_rows = []           # (standard column, bound w - l)
    for j in cols:
        lj, wj = l[j], w[j]
        if not np.isfinite(lj) and not np.isfinite(wj):      # P5: free
            p = len(std_cols)
            std_cols.append((1.0, j))
            std_cols.append((-1.0, j))
            rec.colmap.append(("free", p, p + 1, lj, wj))
        elif not np.isfinite(lj):                             # x = w - x'
            p = len(std_cols)
            std_cols.append((-1.0, j))
            rec.colmap.append(("reflect", p, -1, lj, wj))
        else:                                                 # x = l + x~
            p = len(std_cols)
            std_cols.append((1.0, j))
            rec.colmap.append(("shift", p, -1, lj, wj))
            if np.isfinite(wj):
                ub_rows.append((p, wj - lj))
    mk, nk = len(rows), len(std_cols)
    n_std = nk + len(ub_rows)
    m_std = mk + len(ub_rows)
    As = np.zeros((m_std, n_std))
    bs = np.zeros(m_std)
    cs = np.zeros(n_std)
    for r, i in enumerate(rows):
        bs[r] = b[i]
    for p, (sg, j) in enumerate(std_cols):
        As[:mk, p] = sg * A[rows, j]
        cs[p] = sg * c[j]
    # the constant part of each substitution: x = l + x~ (shift) or x = w - x' (reflect)
    for kind, p, q, lj, wj in rec.colmap:
        j = std_cols[p][1]
        if kind == "shift":
            x0 = lj
        elif kind == "reflect":
            x0 = wj
        else:
            continue
        if x0 != 0.0:
            for r, i in enumerate(rows):
                if A[i, j] != 0.0:
                    bs[r] -= A[i, j] * x0
            rec.obj_offset += c[j] * x0
    for t, (p, u) in enumerate(ub_rows):
        As[mk + t, p] = 1.0
        As[mk + t, nk + t] = 1.0
        bs[mk + t] = u
    rec.n_std, rec.m_std = n_std, m_std
    return PresolveResult(REDUCED, As, bs, cs, rec)


def postsolve(rec: PresolveRecord, xs, ys):
    """Original (x, y, r = c - A^T y) from a solution (xs, ys) of the reduced
    standard-form LP."""
    A, b, c = rec.A, rec.b, rec.c
    x = np.zeros(rec.n)
    for j, v in rec.fixed.items():
        x[j] = v
    for j, (kind, p, q, lj, wj) in zip(rec.cols, rec.colmap):
        if kind == "free":
            x[j] = xs[p] - xs[q]
        elif kind == "reflect":
            x[j] = wj - xs[p]
        else:
            x[j] = lj + xs[p]
    y = np.zeros(rec.m)
    for r, i in enumerate(rec.rows):
        y[i] = ys[r]
    for kind, i, k in reversed(rec.removed_rows):
        if kind == "singleton":
            rest = A[:, k] @ y - A[i, k] * y[i]
            y[i] = (c[k] - rest) / A[i, k]
    r = c - A.T @ y
    return x, y, r


def ruiz(A, iters):
    """Ruiz equilibration: returns (D, E).  Each round takes the row and column
    max-abs of (D_i a_ij) E_j formed from the original entries with the factors
    so far, and multiplies D_i by 1/sqrt(row max), E_j by 1/sqrt(column max)
    (both from the same matrix; a zero row or column keeps its factor)."""
    A = np.array(A, dtype=np.float64)
    m, n = A.shape
    D = np.ones(m)
    E = np.ones(n)
    for _ in range(iters):
        S = np.abs((D[:, None] * A) * E[None, :])
        rmax = S.max(axis=1) if n else np.zeros(m)
        cmax = S.max(axis=0) if m else np.zeros(n)
        fr, fc = np.ones(m), np.ones(n)
        fr[rmax > 0.0] = 1.0 / np.sqrt(rmax[rmax > 0.0])
        fc[cmax > 0.0] = 1.0 / np.sqrt(cmax[cmax > 0.0])
        D = D * fr
        E = E * fc
    return D, E


def scaled_problem(A, b, c, iters):
    """((D_i a_ij) E_j, D b, E c, D, E) after ``iters`` Ruiz rounds."""
    D, E = ruiz(A, iters)
    A = np.asarray(A, dtype=np.float64)
    return (D[:, None] * A) * E[None, :], D * np.asarray(b, dtype=np.float64), \
        E * np.asarray(c, dtype=np.float64), D, E


def unscale(D, E, x, y, s):
    """A solution of the scaled LP in the original variables."""
    return E * x, D * y, s / E
