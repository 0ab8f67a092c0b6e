"""Autotuner: every engine's candidates run, the kept configuration solves correctly."""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _kkt_ok(A, lp, x, y, s):
    kk = oracle.kkt_relative(A, lp["b"], lp["c"], x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy())
    return max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6


@pytest.mark.parametrize("engine", ["wg", "grid"])
def test_autotune_dense(engine):
    lp = lpgen.config0(5)
    eng = abip.ABIP_ENGINE_GRID if engine == "grid" else abip.ABIP_ENGINE_WG
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=eng))
    r = abip.abip_autotune(w, 40)
    print(engine, r, flush=True)
    assert len(r["ms"]) >= (2 if engine == "wg" else 4) and all(t > 0 for t in r["ms"])
    assert r["chosen"] > 0
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED and _kkt_ok(lp["A"], lp, x, y, s)


def test_autotune_sparse():
    lp = lpgen.sparse_planted(300, 800, 7, density=0.01)
    A = lp["A_csr"]
    As = sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])
    w = abip.abip_setup(As, lp["b"], lp["c"])
    r = abip.abip_autotune(w, 20)
    print(r, flush=True)
    assert len(r["ms"]) >= 1 and r["chosen"] > 0
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED and _kkt_ok(As.toarray(), lp, x, y, s)
