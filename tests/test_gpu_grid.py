"""Grid engine (one LP over the whole GPU) against the FP64 oracle, via the C ABI."""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.abip import Problem, Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


# up to 2048 rows every lane holds one four-row group per wave; 2100, 4200 and 6200
# rows take the variants with two, three and four such chunks per lane
@pytest.mark.parametrize("m,n,seed,engine", [(50, 100, 1, "grid"), (300, 700, 2, "grid"),
                                             (1100, 2600, 3, "auto"), (2100, 2300, 7, "grid"),
                                             (4200, 4400, 8, "grid"), (6200, 6400, 9, "grid")])
def test_grid_iterations_match_oracle(m, n, seed, engine):
    print(f"grid iterate m={m} n={n}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings()
    st = oracle.restart(oracle.initial_state(prob, s), s.gamma, s.restart_rule)
    eng = abip.ABIP_ENGINE_GRID if engine == "grid" else abip.ABIP_ENGINE_AUTO
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=eng))
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    solver = oracle.SchurIQSolver(prob)
    N = 30
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    abip.abip_iterate(w, 0, N)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    scale = 1.0 + np.abs(st.u()).max()
    assert np.abs(_np(y) - st.y).max() <= 1e-9 * scale
    assert np.abs(_np(x) - st.x).max() <= 1e-9 * scale
    assert np.abs(_np(sv) - st.s).max() <= 1e-9 * scale
    for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
        assert abs(sc[key] - ref) <= 1e-9 * scale, (key, sc[key], ref)


@pytest.mark.parametrize("seed", [4, 5])
def test_grid_solve_matches_oracle(seed):
    lp = lpgen.config0(seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID))
    x, y, s, info = abip.abip_solve(w)
    print(info, flush=True)
    assert info["status"] == abip.ABIP_SOLVED == ref["status"]
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"])


def test_grid_basis_pursuit_fp32_polish():
    lp = lpgen.basis_pursuit(120, 480, 6, 2)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID,
                                                   precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, s, info = abip.abip_solve(w)
    print(info, flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-5 * (1 + lp["pstar"])


@pytest.mark.parametrize("m,n,seed", [(2100, 2300, 7), (4200, 4400, 8)])
def test_grid_multichunk_fp32_polish_solve(m, n, seed):
    """FP32-streamed A and G^{-1} with two and three row chunks per lane: the solve
    reaches the planted optimum at the KKT tolerance (FP64 recheck on the host)."""
    lp = lpgen.dense_planted(m, n, seed)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID,
                                                   precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, s, info = abip.abip_solve(w)
    print(m, n, info["status_name"], info["admm_iters"], info["admm_iters_fp64"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
