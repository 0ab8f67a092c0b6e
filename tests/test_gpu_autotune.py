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
    assert (0 <= r["chosen"] < len(r["ms"])) if engine == "wg" else r["chosen"] > 0
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


def test_autotune_batch_lds_choices():
    """A batch of small and large LPs: the LDS policies and the per-LP mix are all
    timed, the kept one solves every LP as a fresh handle does (same statuses, the
    KKT bar), and a handle tuned to stream everything reports no LDS mode."""
    lps = lpgen.batch(24, 9, m_lo=20, m_hi=300)
    As, bs, cs = [l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps]
    st = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
    w = abip.abip_setup_batch(As, bs, cs, st)
    r = abip.abip_autotune(w, 30)
    print(r, flush=True)
    nfit512 = all(l["m"] <= 256 for l in lps)
    assert len(r["ms"]) == (5 if nfit512 else 4) and all(t > 0 for t in r["ms"])
    assert 0 <= r["chosen"] < len(r["ms"])
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    w2 = abip.abip_setup_batch(As, bs, cs, st)
    _, _, _, infos2 = abip.abip_solve_batch(w2)
    for k, lp in enumerate(lps):
        assert infos[k]["status"] == infos2[k]["status"], k
        if infos[k]["status"] == abip.ABIP_SOLVED:
            assert _kkt_ok(lp["A"], lp, xs[k], ys[k], ss[k]), k
    if r["chosen"] == 2:
        assert all(i["lds_mode"] == 0 for i in infos)
    w.free()
    w2.free()
