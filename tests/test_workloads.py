"""The paper's Section 5 workloads as generated here, and the oracle on them.

Generator checks (what the recipe fixes) and oracle pins against facts
independent of the oracle: the planted optimal value of the random-LP recipe,
HiGHS on the SICE LP, and the SICE constraint ||Sigma beta - e_j||_inf <= lambda
itself (with beta = beta+ - beta-).  CPU only.
"""
import numpy as np
import pytest
import scipy.optimize

import lpgen
import oracle
from oracle.abip import Settings


def test_paper_random_recipe():
    lp = lpgen.paper_random(60, 300, 3)
    A, b, c, x, y, s = lp["A"], lp["b"], lp["c"], lp["x0"], lp["y0"], lp["s0"]
    g = lp["groups"]
    assert (g["zero"].size, g["big"].size, g["small"].size) == (180, 30, 90)
    assert np.all(x[g["zero"]] == 0.0) and np.all(x >= 0.0) and np.all(s >= 0.0)
    assert np.all(s[g["big"]] == 0.0) and np.all(s[g["small"]] == 0.0)
    assert np.all(x * s == 0.0)
    # ten times larger / smaller groups (|N(0,1)| has median ~0.67)
    assert np.median(x[g["big"]]) > 10 * np.median(x[g["small"]])
    np.testing.assert_allclose(A @ x, b, rtol=0, atol=1e-12 * (1 + np.abs(b).max()))
    np.testing.assert_allclose(A.T @ y + s, c, rtol=0, atol=1e-12 * (1 + np.abs(c).max()))
    assert abs(c @ x - b @ y) <= 1e-9 * (1 + abs(c @ x))          # zero duality gap
    # U^T D V with density-0.2 factors: A is dense for m this large
    assert np.mean(A != 0.0) > 0.9


def test_oracle_reaches_planted_value_of_paper_random_lp():
    """The oracle on the paper's random-LP recipe: its objective matches the
    planted optimal value c^T x0 = b^T y0 (and HiGHS) to the accuracy the
    tolerance allows; b carries entries ten times larger than the rest, so the
    relative tests at eps = 1e-5 leave an objective error near 1e-4 relative."""
    lp = lpgen.paper_random(30, 150, 7)
    r = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-5))
    assert r["status_name"] == "solved"
    obj = float(lp["c"] @ r["x"])
    assert abs(obj - lp["pstar"]) <= 1e-3 * (1 + abs(lp["pstar"])), (obj, lp["pstar"])
    ref = scipy.optimize.linprog(lp["c"], A_eq=lp["A"], b_eq=lp["b"], bounds=(0, None), method="highs")
    assert abs(ref.fun - lp["pstar"]) <= 1e-9 * (1 + abs(lp["pstar"]))


def test_sice_structure():
    S = lpgen.sice(20, 300, 1, cols=[0, 7])
    d, A = S["d"], S["A"]
    assert A.shape == (2 * d, 4 * d) and S["m"] == 2 * d and S["n"] == 4 * d
    Sig = S["Sigma"]
    np.testing.assert_allclose(Sig, Sig.T, atol=1e-14)
    assert np.linalg.eigvalsh(Sig).min() > 0
    np.testing.assert_array_equal(A[:d, :d], Sig)
    np.testing.assert_array_equal(A[:d, d:2 * d], -Sig)
    np.testing.assert_array_equal(A[:d, 2 * d:3 * d], np.eye(d))
    np.testing.assert_array_equal(A[d:, 2 * d:], np.hstack([np.eye(d), np.eye(d)]))
    assert np.all(A[d:, :2 * d] == 0.0) and np.all(A[:d, 3 * d:] == 0.0)
    assert abs(S["lam"] - 1.5 * np.sqrt(np.log(d) / 300)) < 1e-15
    e7 = np.zeros(d); e7[7] = 1.0
    np.testing.assert_array_equal(S["bs"][1], np.concatenate([S["lam"] + e7, 2 * S["lam"] * np.ones(d)]))
    # density of the paper's UCI instances: about 1/4 (Sigma dense, two blocks of it in 8 d^2)
    assert abs(np.mean(A != 0) - 0.25) < 0.05


@pytest.mark.parametrize("j", [0, 3, 11])
def test_oracle_solves_sice_column(j):
    """One column of the SICE problem: the oracle's optimum matches HiGHS and
    its beta satisfies the SICE constraint with lambda."""
    S = lpgen.sice(12, 200, 4, cols=[j])
    A, b, c, d = S["A"], S["bs"][0], S["c"], S["d"]
    r = oracle.solve(A, b, c)
    assert r["status_name"] == "solved"
    ref = scipy.optimize.linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert ref.status == 0
    assert abs(c @ r["x"] - ref.fun) <= 1e-5 * (1 + abs(ref.fun))
    beta = r["x"][:d] - r["x"][d:2 * d]
    e = np.zeros(d); e[j] = 1.0
    assert np.abs(S["Sigma"] @ beta - e).max() <= S["lam"] * (1 + 1e-4)
    assert abs(np.abs(beta).sum() - ref.fun) <= 1e-4 * (1 + ref.fun)    # ||beta||_1 is the objective
