"""The paper's Section 5 workloads on the GPU: the sparse inverse covariance
LPs (one batched launch over the columns of Omega) and the random-LP recipe,
against the FP64 oracle, the SICE constraint and the planted optimal value."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.abip import Settings

pytestmark = pytest.mark.gpu

abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sice_batch_matches_oracle(prec):
    S = lpgen.sice(16, 200, 3)
    d, A, c = S["d"], S["A"], S["c"]
    p = abip.ABIP_PREC_FP32_POLISH if prec == "fp32" else abip.ABIP_PREC_FP64
    print(f"sice batch d={d} prec={prec}", flush=True)
    w = abip.abip_setup_batch([A] * d, S["bs"], [c] * d, abip.abip_default_settings(precision=p))
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    for j in range(d):
        assert infos[j]["status"] == abip.ABIP_SOLVED
        x = _np(xs[j])
        k = oracle.kkt_relative(A, S["bs"][j], c, x, _np(ys[j]), _np(ss[j]))
        assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6, (j, k)
        beta = x[:d] - x[d:2 * d]
        e = np.zeros(d); e[j] = 1.0
        assert np.abs(S["Sigma"] @ beta - e).max() <= S["lam"] * (1 + 1e-4)
    for j in (0, 9):
        ref = oracle.solve(A, S["bs"][j], c)
        assert abs(c @ _np(xs[j]) - c @ ref["x"]) <= 1e-5 * (1 + abs(c @ ref["x"]))
    w.free()


@pytest.mark.parametrize("engine", ["wg", "grid"])
def test_paper_random_reaches_planted_value(engine):
    lp = lpgen.paper_random(30, 150, 7)
    eng = abip.ABIP_ENGINE_GRID if engine == "grid" else abip.ABIP_ENGINE_WG
    print(f"paper_random 30x150 engine={engine}", flush=True)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(eps=1e-5, engine=eng))
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED
    obj = float(lp["c"] @ _np(x))
    assert abs(obj - lp["pstar"]) <= 1e-3 * (1 + abs(lp["pstar"])), (obj, lp["pstar"])
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(eps=1e-5))
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(5, ref["admm_iters"] // 50)


def test_paper_random_table_size_at_paper_tolerance():
    """A Table-1-sized instance (500 x 5000) at the paper's 1e-3: the host
    recomputes the Section 4.1 residuals of the returned point."""
    lp = lpgen.paper_random(500, 5000, 1)
    print("paper_random 500x5000 eps=1e-3", flush=True)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(
        eps=1e-3, engine=abip.ABIP_ENGINE_GRID, precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED
    k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-3 * (1 + 1e-6), k
