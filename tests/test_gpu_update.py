"""abip_update_data: new LPs of the same shapes loaded into an existing handle.

The reload reruns the whole setup in the handle's own buffers and the next
solve replays the batched launch's captured graph, so results must equal those
of a fresh handle bitwise (same kernels, same data layout).
"""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _batch(seed):
    lps = lpgen.batch(12, seed, m_lo=20, m_hi=150)
    return [l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps]


def _solve_fresh(As, bs, cs, st):
    w = abip.abip_setup_batch(As, bs, cs, st)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    out = ([_np(x) for x in xs], [i["admm_iters"] for i in infos], [i["status"] for i in infos])
    w.free()
    return out


def test_update_batch_equals_fresh_handles():
    st = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
    d1, d2 = _batch(41), _batch(42)
    # the same shapes with new values: redraw the second set's values for the first set's shapes
    rng = np.random.default_rng(5)
    shapes = [A.shape for A in d1[0]]
    d2 = ([], [], [])
    for (m, n) in shapes:
        lp = lpgen.dense_planted(m, n, int(rng.integers(1 << 30)))
        d2[0].append(lp["A"]); d2[1].append(lp["b"]); d2[2].append(lp["c"])
    ref1 = _solve_fresh(*d1, st)
    ref2 = _solve_fresh(*d2, st)
    w = abip.abip_setup_batch(*d1, st)
    for data, ref in [(d1, ref1), (d2, ref2), (d1, ref1)]:
        abip.abip_update_data(w, *data)
        xs, ys, ss, infos = abip.abip_solve_batch(w)
        got = ([_np(x) for x in xs], [i["admm_iters"] for i in infos], [i["status"] for i in infos])
        print("iters", sum(got[1]), sum(ref[1]), flush=True)
        assert got[1] == ref[1] and got[2] == ref[2]
        for a, b in zip(got[0], ref[0]):
            np.testing.assert_array_equal(a, b)
    w.free()


def test_update_rejects_other_shapes():
    d1 = _batch(43)
    w = abip.abip_setup_batch(*d1)
    As = list(d1[0])
    As[3] = np.ones((As[3].shape[0] + 1, As[3].shape[1]))
    bs = list(d1[1])
    bs[3] = np.ones(As[3].shape[0])
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_update_data(w, As, bs, d1[2])
    assert e.value.code == abip.ABIP_E_DIM
    w.free()


def test_update_grid_engine():
    lp1 = lpgen.dense_planted(300, 900, 1)
    lp2 = lpgen.dense_planted(300, 900, 2)
    st = abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID)
    w = abip.abip_setup(lp1["A"], lp1["b"], lp1["c"], st)
    abip.abip_update_data(w, [lp2["A"]], [lp2["b"]], [lp2["c"]])
    x, y, s, info = abip.abip_solve(w)
    w2 = abip.abip_setup(lp2["A"], lp2["b"], lp2["c"], st)
    x2, y2, s2, info2 = abip.abip_solve(w2)
    assert info["status"] == info2["status"] == abip.ABIP_SOLVED
    assert info["admm_iters"] == info2["admm_iters"]
    np.testing.assert_array_equal(_np(x), _np(x2))
    w.free()
    w2.free()
