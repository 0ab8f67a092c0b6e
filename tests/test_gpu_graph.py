"""hipGraph replay: every replay equals the plain stream launches, bitwise.

Each engine is run with graphs several times in a row, with eager (plain
launch) solves and host synchronisations in between, and every result is
compared with the eager one."""
import numpy as np
import pytest
import torch

import lpgen

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _run(w):
    x, y, s, info = abip.abip_solve(w)
    torch.cuda.synchronize()
    return x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy(), info


def _same(a, b):
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    for k in ("status", "admm_iters", "ipm_iters", "tau", "kappa", "mu"):
        assert a[3][k] == b[3][k], k


def test_grid_engine_graph_replays_match_eager():
    lp = lpgen.config0(4)
    sg = abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID, use_graph=1)
    se = abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID, use_graph=0)
    wg = abip.abip_setup(lp["A"], lp["b"], lp["c"], sg)
    we = abip.abip_setup(lp["A"], lp["b"], lp["c"], se)
    ref = _run(we)
    print("grid eager", ref[3]["admm_iters"], flush=True)
    for rep in range(3):
        got = _run(wg)
        _same(got, ref)
        _same(_run(we), ref)          # eager work between the replays


def test_batched_graph_replays_match_eager():
    lps = [lpgen.dense_planted(m, n, sd) for (m, n, sd) in [(12, 30, 1), (40, 90, 2), (7, 15, 3), (60, 130, 4)]]
    lps.append(lpgen.dense_farkas_infeasible(20, 50, 3))
    args = ([lp["A"] for lp in lps], [lp["b"] for lp in lps], [lp["c"] for lp in lps])
    for prec in (abip.ABIP_PREC_FP64, abip.ABIP_PREC_FP32_POLISH):
        wg = abip.abip_setup_batch(*args, abip.abip_default_settings(precision=prec, use_graph=1))
        we = abip.abip_setup_batch(*args, abip.abip_default_settings(precision=prec, use_graph=0))
        ref = abip.abip_solve_batch(we)
        torch.cuda.synchronize()
        for rep in range(3):
            got = abip.abip_solve_batch(wg)
            torch.cuda.synchronize()
            for k in range(len(lps)):
                for i in range(3):            # bitwise, NaN (certificate fill) matching NaN
                    assert torch.allclose(got[i][k], ref[i][k], rtol=0, atol=0, equal_nan=True)
                assert got[3][k]["admm_iters"] == ref[3][k]["admm_iters"]
                assert got[3][k]["status"] == ref[3][k]["status"]
            abip.abip_solve_batch(we)     # eager work between the replays
            torch.cuda.synchronize()
