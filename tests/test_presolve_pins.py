"""Pins of the oracle's Section 4.5 presolve / postsolve and Ruiz scaling.

The presolved LP is solved by an independent LP solver (HiGHS through
scipy.optimize.linprog) and postsolved; the result must be an optimal solution
of the original bounded LP, checked by LP duality on the original data:
primal feasibility, the bounded dual's sign conditions on r = c - A^T y
(complementary slackness) and equal objectives.  Each reduction of the list
(P1-P6, the split / reflection / shift / upper-bound rows) is present in the
constructed LP, so a dropped substitution, a wrong sign in the reflection or a
wrong dual recovery for a singleton row fails here.
"""
import numpy as np
import pytest
import scipy.optimize

import oracle.presolve as pre


def _bounded_lp(seed):
    """An LP with every reduction: an empty row, empty columns (c > 0 at its lower
    bound, c < 0 at its upper bound), a fixed variable, a free variable, a variable
    bounded only above, two upper-bounded variables and a singleton row."""
    rng = np.random.default_rng(seed)
    m, n = 9, 14
    A = rng.standard_normal((m, n))
    A[rng.random((m, n)) < 0.2] = 0.0
    A[0, :] = 0.0                       # P1: empty row
    A[:, 3] = 0.0                       # P2: empty column, c > 0
    A[:, 4] = 0.0                       # P2: empty column, c < 0, finite upper bound
    A[5, :] = 0.0
    A[5, 2] = 2.0                       # P6: singleton row fixes x_2
    l = np.zeros(n)
    w = np.full(n, np.inf)
    l[5] = w[5] = 1.5                   # P4: fixed
    l[6], w[6] = -np.inf, np.inf        # P5: free
    l[7], w[7] = -np.inf, 3.0           # bounded above only (reflected)
    w[8], w[9] = 2.0, 4.0               # upper-bound rows
    w[4] = 2.0                          # the c < 0 empty column goes to this bound
    l[10] = -1.0                        # shifted lower bound
    x0 = rng.uniform(0.2, 1.0, n)       # a feasible point
    x0[3], x0[4], x0[5] = 0.0, 2.0, 1.5
    x0[7] = 1.0
    b = A @ x0
    c = rng.standard_normal(n)
    c[3], c[4] = 1.0, -1.0
    # keep the LP bounded: cost in the row space plus a positive part on the
    # unbounded directions
    c = A.T @ rng.standard_normal(m) + np.abs(rng.standard_normal(n)) * (np.isinf(w) & np.isfinite(l))
    c[3], c[4] = 1.0, -1.0
    return A, b, c, l, w


def _linprog_bounds(l, w):
    return [(None if np.isinf(a) else a, None if np.isinf(z) else z) for a, z in zip(l, w)]


def _check_optimal(A, b, c, l, w, x, y, r, obj, tol=1e-7):
    scale = 1.0 + np.abs(x).max()
    assert np.abs(A @ x - b).max() <= tol * (1 + np.abs(b).max())
    assert np.all(x >= l - tol * scale) and np.all(x <= w + tol * scale)
    assert np.allclose(r, c - A.T @ y, atol=1e-12 * (1 + np.abs(c).max()))
    at_l = np.abs(x - l) <= 1e-7 * scale
    at_w = np.abs(x - w) <= 1e-7 * scale
    inner = ~at_l & ~at_w
    rs = 1.0 + np.abs(r).max()
    assert np.all(np.abs(r[inner]) <= 1e-6 * rs)          # interior variables: zero reduced cost
    assert np.all(r[at_l & ~at_w] >= -1e-6 * rs)          # at the lower bound only
    assert np.all(r[at_w & ~at_l] <= 1e-6 * rs)           # at the upper bound only
    assert abs(c @ x - obj) <= 1e-7 * (1 + abs(obj))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_presolve_postsolve_gives_an_optimum_of_the_original(seed):
    A, b, c, l, w = _bounded_lp(seed)
    ref = scipy.optimize.linprog(c, A_eq=A, b_eq=b, bounds=_linprog_bounds(l, w), method="highs")
    assert ref.status == 0, ref.message
    res = pre.presolve(A, b, c, l, w)
    assert res.status == pre.REDUCED
    rec = res.record
    kinds = {k for k, _, _ in rec.removed_rows}
    assert kinds == {"empty", "singleton"}
    assert {3, 4, 5, 2} <= set(rec.fixed)
    red = scipy.optimize.linprog(res.c, A_eq=res.A, b_eq=res.b, bounds=(0, None), method="highs")
    assert red.status == 0, red.message
    # the reduced optimum plus the offset is the original optimum
    assert abs(red.fun + rec.obj_offset - ref.fun) <= 1e-7 * (1 + abs(ref.fun))
    x, y, r = pre.postsolve(rec, red.x, red.eqlin.marginals)
    _check_optimal(A, b, c, l, w, x, y, r, ref.fun)
    # removed empty rows carry a zero multiplier
    assert y[0] == 0.0


def test_presolve_fixed_values():
    A, b, c, l, w = _bounded_lp(1)
    rec = pre.presolve(A, b, c, l, w).record
    assert rec.fixed[3] == 0.0            # c > 0, empty: its lower bound
    assert rec.fixed[4] == w[4]           # c < 0, empty: its upper bound
    assert rec.fixed[5] == 1.5            # fixed variable
    assert rec.fixed[2] == b[5] / A[5, 2]  # singleton row 5


def test_presolve_standard_form_is_untouched():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((5, 9))
    b = A @ rng.uniform(0.5, 1.0, 9)
    c = rng.standard_normal(9)
    res = pre.presolve(A, b, c)
    assert res.status == pre.REDUCED
    np.testing.assert_array_equal(res.A, A)
    np.testing.assert_array_equal(res.b, b)
    np.testing.assert_array_equal(res.c, c)
    assert res.record.obj_offset == 0.0


def test_presolve_detects_infeasible_and_unbounded():
    A = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 1.0, 1.0]])
    c = np.array([1.0, 1.0, 1.0])
    # P1: empty row with b != 0
    assert pre.presolve(A, np.array([1.0, 2.0, 1.0]), c).status == pre.INFEASIBLE
    # P3: l > w
    assert pre.presolve(A, np.array([1.0, 0.0, 1.0]), c, l=np.array([0, 2.0, 0]),
                        w=np.array([np.inf, 1.0, np.inf])).status == pre.INFEASIBLE
    # P6: a singleton row forces x_0 = -1 < 0
    A6 = np.array([[1.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    assert pre.presolve(A6, np.array([-1.0, 1.0]), c).status == pre.INFEASIBLE
    # P2: an empty column with c < 0 and no upper bound
    A2 = np.array([[1.0, 0.0, 1.0]])
    assert pre.presolve(A2, np.array([1.0]), np.array([1.0, -1.0, 1.0])).status == pre.UNBOUNDED


def test_ruiz_equilibrates_and_keeps_the_optimum():
    rng = np.random.default_rng(5)
    m, n = 12, 30
    A = rng.standard_normal((m, n)) * np.exp(rng.uniform(-4, 4, m))[:, None] * np.exp(rng.uniform(-3, 3, n))[None, :]
    x0 = rng.uniform(0.5, 1.0, n)
    b = A @ x0
    c = A.T @ rng.standard_normal(m) + rng.uniform(0.1, 1.0, n)
    As, bs, cs, D, E = pre.scaled_problem(A, b, c, 25)
    S = np.abs(As)
    assert np.abs(S.max(axis=1) - 1.0).max() <= 1e-3
    assert np.abs(S.max(axis=0) - 1.0).max() <= 1e-3
    ref = scipy.optimize.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    sc = scipy.optimize.linprog(cs, A_eq=As, b_eq=bs, bounds=(0, None), method="highs")
    x, y, s = pre.unscale(D, E, sc.x, sc.eqlin.marginals, cs - As.T @ sc.eqlin.marginals)
    assert abs(c @ x - ref.fun) <= 1e-8 * (1 + abs(ref.fun))
    assert np.abs(A @ x - b).max() <= 1e-8 * (1 + np.abs(b).max())
    assert np.allclose(s, c - A.T @ y, atol=1e-9 * (1 + np.abs(c).max()))


def test_ruiz_fixed_point_and_zero_lines():
    # a signed permutation-like matrix is already equilibrated: D = E = 1
    A = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    D, E = pre.ruiz(A, 10)
    assert np.all(D == 1.0) and np.all(E == 1.0)
    # an all-zero row and column keep factor 1; a single entry 16 -> factors 1/4 each
    B = np.zeros((2, 2))
    B[0, 0] = 16.0
    D, E = pre.ruiz(B, 1)
    assert D[1] == 1.0 and E[1] == 1.0 and D[0] == 0.25 and E[0] == 0.25
