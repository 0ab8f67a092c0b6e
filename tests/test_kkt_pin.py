"""The Section 4.1 residual checkers against values worked out by hand.

Three pieces of code compute the relative residuals of the termination criteria
(paper Section 4.1): the oracle's ``kkt_relative`` (used by every GPU KKT
assertion), the oracle's ``termination`` (the stopping test of Algorithm 2, on
the tau-scaled candidate) and the benchmark's host re-check.  None of them may
be pinned by re-typing its own formula, so all three are compared here with the
worked examples in ``tests/golden/kkt_relative_worked.txt``, whose values follow
from closed forms evaluated by hand.  The examples are chosen so that the usual
slips give different numbers: the ``1 +`` in each normaliser, the norm of b or c
in place of its 1 + norm, |pobj - dobj| in place of |pobj| + |dobj| in the gap's
normaliser, and a sign slip in A^T y + s - c.
"""
import os

import numpy as np
import pytest

import bench
import oracle
from oracle.abip import Problem, State

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kkt_relative_worked.txt")


def _cases():
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, dims, A, b, c, x, y, s, want = [p.strip() for p in line.split("|")]
            m, n = (int(v) for v in dims.split())
            arr = lambda t: np.array([float(v) for v in t.split()])
            out.append(dict(name=name, A=arr(A).reshape(m, n), b=arr(b), c=arr(c), x=arr(x), y=arr(y),
                            s=arr(s), want=arr(want)))
    return out


CASES = _cases()


def test_fixture_has_both_cases():
    assert [c["name"] for c in CASES] == ["case1", "case2"]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_kkt_relative_matches_worked_values(case):
    kk = oracle.kkt_relative(case["A"], case["b"], case["c"], case["x"], case["y"], case["s"])
    got = np.array([kk["pres"], kk["dres"], kk["gap"]])
    np.testing.assert_allclose(got, case["want"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("tau", [1.0, 2.5])
def test_termination_residuals_match_worked_values(case, tau):
    """termination() reads the candidate (x/tau, y/tau, s/tau) off the HSD state."""
    prob = Problem(case["A"], case["b"], case["c"])
    st = State(case["y"] * tau, case["x"] * tau, tau, 1.0, case["s"] * tau, 1.0, 1.0)
    status, info = oracle.termination(prob, st, 1e-12)
    assert status == 0
    got = np.array([info["pres"], info["dres"], info["gap"]])
    np.testing.assert_allclose(got, case["want"], rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c["name"])
def test_bench_host_check_matches_worked_values(case):
    got = np.array(bench.host_kkt(case["A"], case["b"], case["c"], case["x"], case["y"], case["s"]))
    np.testing.assert_allclose(got, case["want"], rtol=1e-14, atol=0)


def _variants():
    """Plausible slips in a residual checker; each must miss the worked values."""
    n2 = np.linalg.norm

    def gap_diff_norm(A, b, c, x, y, s):     # |pobj - dobj| in the normaliser
        p, d = c @ x, b @ y
        return n2(A @ x - b) / (1 + n2(b)), n2(A.T @ y + s - c) / (1 + n2(c)), abs(p - d) / (1 + abs(p - d))

    def no_one_pres(A, b, c, x, y, s):       # ||b|| instead of 1 + ||b||
        p, d = c @ x, b @ y
        return n2(A @ x - b) / n2(b), n2(A.T @ y + s - c) / (1 + n2(c)), abs(p - d) / (1 + abs(p) + abs(d))

    def no_one_gap(A, b, c, x, y, s):        # |pobj| + |dobj| without the 1
        p, d = c @ x, b @ y
        return n2(A @ x - b) / (1 + n2(b)), n2(A.T @ y + s - c) / (1 + n2(c)), abs(p - d) / (abs(p) + abs(d))

    def sign_s(A, b, c, x, y, s):            # A^T y - s - c
        p, d = c @ x, b @ y
        return n2(A @ x - b) / (1 + n2(b)), n2(A.T @ y - s - c) / (1 + n2(c)), abs(p - d) / (1 + abs(p) + abs(d))

    def dres_by_b(A, b, c, x, y, s):         # dual residual normalised by b
        p, d = c @ x, b @ y
        return n2(A @ x - b) / (1 + n2(b)), n2(A.T @ y + s - c) / (1 + n2(b)), abs(p - d) / (1 + abs(p) + abs(d))

    return [gap_diff_norm, no_one_pres, no_one_gap, sign_s, dres_by_b]


@pytest.mark.parametrize("variant", _variants(), ids=lambda f: f.__name__)
def test_worked_values_catch_plausible_slips(variant):
    missed = False
    for case in CASES:
        got = np.array(variant(case["A"], case["b"], case["c"], case["x"], case["y"], case["s"]))
        if not np.allclose(got, case["want"], rtol=1e-12, atol=0):
            missed = True
    assert missed, variant.__name__
