"""The 256-LP batch workload (m ~ U[20, 400], n ~ U[2m, 3m], 10% primal infeasible, seed 3)
in the launch configuration bench.py times: FP32 bulk + FP64 polish, the adaptive beta of
Section 4.3, an autotuned handle reloaded with abip_update_data.  Every LP: the status against
its planted one, the Section 4.1 residuals recomputed on the host, the objective against the
planted optimum, the Farkas certificates of the infeasible ones; a sample the FP64 oracle solves
in seconds: the objective against the oracle's.  All through the C ABI."""
import numpy as np
import pytest
import torch

import lpgen
import oracle
from oracle.abip import Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def test_headline_batch_every_lp_and_a_sample_against_the_oracle():
    lps = lpgen.batch(256, 3)
    As = [torch.tensor(lp["A"], dtype=torch.float64, device="cuda") for lp in lps]
    bs = [torch.tensor(lp["b"], dtype=torch.float64, device="cuda") for lp in lps]
    cs = [torch.tensor(lp["c"], dtype=torch.float64, device="cuda") for lp in lps]
    s = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH, bb=1)
    w = abip.abip_setup_batch(As, bs, cs, s)
    tune = abip.abip_autotune(w, 200)
    print("autotune", tune, flush=True)
    abip.abip_update_data(w, As, bs, cs)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    solved = []
    for k, (lp, x, y, sv, info) in enumerate(zip(lps, xs, ys, ss, infos)):
        if lp["status"] == "solved":
            assert info["status"] == abip.ABIP_SOLVED, (k, info["status_name"])
            x, y, sv = _np(x), _np(y), _np(sv)
            kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], x, y, sv)
            assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6 * (1 + 1e-9), (k, kk)
            assert np.all(x >= 0) and np.all(sv >= 0)
            # a relative KKT of 1e-6 bounds the objective's distance to the optimum through
            # the conditioning of A; the bench reports at most 2e-5 on this batch
            assert abs(lp["c"] @ x - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"])), k
            solved.append(k)
        else:
            assert info["status"] == abip.ABIP_PRIMAL_INFEASIBLE, (k, info["status_name"])
            y = _np(y)
            assert abs(lp["b"] @ y - 1.0) < 1e-9, k
            assert np.linalg.norm(lp["A"].T @ y + _np(sv)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001, k
    assert len(solved) == sum(lp["status"] == "solved" for lp in lps) == 230
    # the FP64 oracle with the same adaptive beta on the solved LPs it finishes quickest
    sample = sorted(solved, key=lambda k: lps[k]["m"] * lps[k]["n"] * infos[k]["admm_iters"])[:4]
    for k in sample:
        lp = lps[k]
        ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(bb=True))
        assert ref["status"] == 1
        p_gpu = float(lp["c"] @ _np(xs[k]))
        p_ref = float(lp["c"] @ ref["x"])
        print(k, lp["m"], lp["n"], "iters gpu", infos[k]["admm_iters"], "oracle", ref["admm_iters"],
              "pobj", p_gpu, p_ref, flush=True)
        assert abs(p_gpu - p_ref) <= 1e-4 * (1 + abs(p_ref)), k
