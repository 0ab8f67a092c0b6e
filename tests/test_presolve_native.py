"""The library's host presolve / postsolve (Section 4.5) against the oracle's.

Host code only (no GPU): the reductions are integer decisions, compared exactly
(which rows and columns go, in which order, the fixed values); the standard form
is produced by the same element operations in the same order, so A~, b~, c~ and
the objective constant are compared bitwise; postsolve's dot products are summed
in another order, so y and r agree to rounding.
"""
import numpy as np
import pytest
import scipy.optimize

import oracle.presolve as pre
from test_presolve_pins import _bounded_lp, _check_optimal, _linprog_bounds

abip = pytest.importorskip("paper_1805_12344_amd")

VERDICT = {pre.REDUCED: abip.ABIP_PRESOLVE_REDUCED, pre.INFEASIBLE: abip.ABIP_PRESOLVE_INFEASIBLE,
           pre.UNBOUNDED: abip.ABIP_PRESOLVE_UNBOUNDED}


def _compare(A, b, c, l=None, w=None):
    ref = pre.presolve(A, b, c, l, w)
    got = abip.abip_presolve(A, b, c, l, w)
    assert got.status == VERDICT[ref.status], (ref.status, ref.reason, got.status)
    if ref.status != pre.REDUCED:
        return ref, got
    rec = ref.record
    np.testing.assert_array_equal(got.A, ref.A)
    np.testing.assert_array_equal(got.b, ref.b)
    np.testing.assert_array_equal(got.c, ref.c)
    assert got.obj_offset == rec.obj_offset
    assert list(got.rows_kept) == rec.rows and list(got.cols_kept) == rec.cols
    assert got.fixed == list(rec.fixed.items())
    kinds = np.full(len(b), -1)
    for kind, i, _ in rec.removed_rows:
        kinds[i] = 0 if kind == "empty" else 1
    np.testing.assert_array_equal(got.row_kind, kinds)
    return ref, got


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_native_presolve_equals_oracle(seed):
    A, b, c, l, w = _bounded_lp(seed)
    ref, got = _compare(A, b, c, l, w)
    red = scipy.optimize.linprog(got.c, A_eq=got.A, b_eq=got.b, bounds=(0, None), method="highs")
    assert red.status == 0
    x, y, r = abip.abip_postsolve(got, red.x, red.eqlin.marginals)
    xr, yr, rr = pre.postsolve(ref.record, red.x, red.eqlin.marginals)
    np.testing.assert_array_equal(x, xr)
    assert np.abs(y - yr).max() <= 1e-13 * (1 + np.abs(yr).max())
    assert np.abs(r - rr).max() <= 1e-13 * (1 + np.abs(rr).max())
    opt = scipy.optimize.linprog(c, A_eq=A, b_eq=b, bounds=_linprog_bounds(l, w), method="highs")
    _check_optimal(A, b, c, l, w, x, y, r, opt.fun)


def test_native_presolve_random_structures():
    """Many small LPs with random zero patterns, fixed, free, bounded-above and
    boxed variables: the same decisions and the same standard form as the oracle."""
    rng = np.random.default_rng(11)
    verdicts = set()
    for t in range(300):
        m, n = int(rng.integers(1, 8)), int(rng.integers(1, 10))
        A = rng.standard_normal((m, n)) * (rng.random((m, n)) < rng.uniform(0.1, 0.7))
        x0 = rng.uniform(-1, 2, n)
        l = np.where(rng.random(n) < 0.2, -np.inf, rng.uniform(-1, 0.5, n))
        w = np.where(rng.random(n) < 0.5, np.inf, rng.uniform(0.5, 3, n))
        fixed = rng.random(n) < 0.1
        w[fixed] = l[fixed] = np.where(np.isfinite(l[fixed]), l[fixed], 0.0)
        b = A @ np.clip(x0, np.where(np.isfinite(l), l, -5), np.where(np.isfinite(w), w, 5))
        if rng.random() < 0.2:
            b = b + rng.standard_normal(m)                  # often infeasible
        c = rng.standard_normal(n)
        ref, got = _compare(A, b, c, l, w)
        verdicts.add(ref.status)
    assert verdicts == {pre.REDUCED, pre.INFEASIBLE, pre.UNBOUNDED}


def test_native_presolve_rejects_bad_input():
    A = np.ones((2, 3))
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_presolve(A, np.ones(2), np.array([1.0, np.nan, 0.0]))
    assert e.value.code == abip.ABIP_E_NONFINITE
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_presolve(A, np.ones(2), np.ones(3), l=np.array([0.0, np.inf, 0.0]))
    assert e.value.code == abip.ABIP_E_INVALID
    p = abip.abip_presolve(np.zeros((1, 2)), np.ones(1), np.ones(2))
    assert p.status == abip.ABIP_PRESOLVE_INFEASIBLE and p.where == 0
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_postsolve(p, np.zeros(0), np.zeros(0))
    assert e.value.code == abip.ABIP_E_STATE
