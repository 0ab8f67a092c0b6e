"""Adaptive beta (Section 4.3) on the GPU against the oracle's bb_select.

Each outer iteration that starts with ||Q u - v||^2 > mu takes two probe
iterations from its initial point, estimates beta from the three iterates,
keeps / averages / redoes, and restarts from the initial point with the chosen
beta.  The GPU forms the curvature differences from differences of the iterate
(an algebraically equal form, pinned on the CPU in test_oracle_pins.py), so the
estimates agree to rounding.

* First selection: a solve capped at one ADMM update stops right after the
  first outer iteration's choice; beta, the number of estimates (redos
  included), the probe count and the restored initial point equal the oracle's.
* Trajectory: capped at a few hundred updates (several outer iterations, each
  with its own choice), the final beta and iterate equal the oracle's.
* Full solves: status, the KKT bar and the objective against the oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
import oracle
from oracle.abip import Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")

# (m, n, seed): column pairs / one column / two columns per lane in the LDS variant
LPS = [(30, 70, 1), (76, 159, 23), (120, 260, 7)]
ENGINES = ["lds", "streamed", "grid"]


def _np(t):
    return t.detach().cpu().numpy()


def _gpu(lp, lds, **kw):
    if lds == "grid":          # one LP over the whole GPU: the beta steps run while the grid waits
        kw["engine"] = abip.ABIP_ENGINE_GRID
    s = abip.abip_default_settings(bb=1, lds_resident=1 if lds == "lds" else 0, **kw)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    st = abip.abip_get_state(w, 0)
    w.free()
    return x, y, sv, info, st


@pytest.mark.parametrize("lds", ENGINES)
@pytest.mark.parametrize("m,n,seed", LPS)
def test_bb_first_selection_matches_oracle(m, n, seed, lds):
    lp = lpgen.dense_planted(m, n, seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(bb=True, max_admm_iters=1))
    assert ref["status_name"] == "max_iters" and len(ref["betas"]) == 1
    _, beta_ref, trail = ref["betas"][0]
    x, y, sv, info, (gy, gx, gs, sc) = _gpu(lp, lds, max_admm_iters=1)
    print(f"{m}x{n} {lds}: beta {info['beta']:.12g} oracle {beta_ref:.12g}, estimates {info['bb_estimates']} "
          f"oracle {len(trail)} {trail}", flush=True)
    assert info["status"] == abip.ABIP_MAX_ITERS
    assert info["bb_estimates"] == len(trail)
    assert info["bb_probe_iters"] == 2 * len(trail) == info["admm_iters"] == ref["admm_iters"]
    assert abs(info["beta"] - beta_ref) <= 1e-9 * beta_ref
    # the restored initial point of the first outer iteration
    st = ref["state"]
    scale = 1.0 + np.abs(st.u()).max()
    for g, r in [(gy, st.y), (gx, st.x), (gs, st.s)]:
        assert np.abs(_np(g) - r).max() <= 1e-12 * scale
    assert abs(sc["tau"] - st.tau) <= 1e-12 * scale and abs(sc["kappa"] - st.kappa) <= 1e-12 * scale


@pytest.mark.parametrize("lds", ENGINES)
@pytest.mark.parametrize("m,n,seed", LPS)
def test_bb_trajectory_matches_oracle(m, n, seed, lds):
    lp = lpgen.dense_planted(m, n, seed)
    cap = 300
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(bb=True, max_admm_iters=cap))
    x, y, sv, info, (gy, gx, gs, sc) = _gpu(lp, lds, max_admm_iters=cap)
    betas = [b for (_, b, _) in ref["betas"]]
    print(f"{m}x{n} {lds}: status {info['status_name']} iters {info['admm_iters']} oracle {ref['admm_iters']}, "
          f"ipm {info['ipm_iters']} oracle {ref['ipm_iters']}, beta {info['beta']:.10g} oracle {betas[-1]:.10g}, "
          f"estimates {info['bb_estimates']} oracle {sum(len(t) for (_, _, t) in ref['betas'])}", flush=True)
    assert info["status_name"] == ref["status_name"]
    assert info["ipm_iters"] == ref["ipm_iters"] and info["admm_iters"] == ref["admm_iters"]
    assert info["bb_estimates"] == sum(len(t) for (_, _, t) in ref["betas"])
    assert abs(info["beta"] - betas[-1]) <= 1e-7 * betas[-1]
    st = ref["state"]
    scale = 1.0 + np.abs(st.u()).max()
    for g, r in [(gy, st.y), (gx, st.x), (gs, st.s)]:
        assert np.abs(_np(g) - r).max() <= 1e-7 * scale


@pytest.mark.parametrize("lds", ENGINES)
@pytest.mark.parametrize("m,n,seed", [(30, 70, 1), (76, 159, 23)])
def test_bb_full_solve(m, n, seed, lds):
    lp = lpgen.dense_planted(m, n, seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings(bb=True))
    x, y, sv, info, _ = _gpu(lp, lds)
    print(f"{m}x{n} {lds}: {info['status_name']} iters {info['admm_iters']} oracle {ref['admm_iters']} "
          f"(probes {info['bb_probe_iters']}, estimates {info['bb_estimates']}), beta {info['beta']:.6g}",
          flush=True)
    assert info["status_name"] == ref["status_name"] == "solved"
    k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    assert abs(k["pobj"] - lp["pstar"]) <= 1e-5 * (1 + abs(lp["pstar"]))
    # the trajectory follows the oracle's while decisions agree; once a rounding
    # difference flips one, the count may drift: a loose bar on the total
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= 0.25 * ref["admm_iters"]


def test_bb_fp32_bulk_and_batch():
    lps = [lpgen.dense_planted(m, n, s) for (m, n, s) in [(30, 70, 1), (76, 159, 23), (300, 650, 3)]]
    s = abip.abip_default_settings(bb=1, precision=abip.ABIP_PREC_FP32_POLISH)
    w = abip.abip_setup_batch([l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps], s)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    for lp, x, y, sv, info in zip(lps, xs, ys, ss, infos):
        print(lp["m"], lp["n"], info["status_name"], info["admm_iters"], info["bb_estimates"], flush=True)
        assert info["status"] == abip.ABIP_SOLVED and info["bb_estimates"] > 0
        k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
        assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    w.free()


def test_bb_grid_fp32_bulk_basis_pursuit():
    """The grid engine with the adaptive beta and FP32 bulk on a basis-pursuit LP (paired
    column pass): solved, host KKT, the planted l1 value."""
    lp = lpgen.basis_pursuit(120, 480, 6, 2)
    s = abip.abip_default_settings(bb=1, engine=abip.ABIP_ENGINE_GRID, precision=abip.ABIP_PREC_FP32_POLISH)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], info["bb_estimates"], info["beta"], info["grid_mirror"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED and info["bb_estimates"] > 0 and info["grid_mirror"] == 1
    k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    assert abs(k["pobj"] - lp["pstar"]) <= 1e-4 * (1 + lp["pstar"])
    w.free()


def _sparse(sl, **kw):
    A = sl["A_csr"]
    As = sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])
    s = abip.abip_default_settings(bb=1, cg_tol=1e-13, cg_rule=1, cg_max_iters=2000, **kw)
    w = abip.abip_setup(As, sl["b"], sl["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    st = abip.abip_get_state(w, 0)
    w.free()
    return As, x, y, sv, info, st


def test_bb_sparse_first_selection_matches_oracle():
    """The sparse engine (CG on G to 1e-13): the first choice against the oracle's."""
    sl = lpgen.sparse_planted(150, 420, 2, density=0.02)
    As, x, y, sv, info, (gy, gx, gs, sc) = _sparse(sl, max_admm_iters=1)
    ref = oracle.solve(As.toarray(), sl["b"], sl["c"], Settings(bb=True, max_admm_iters=1))
    _, beta_ref, trail = ref["betas"][0]
    print(f"sparse: beta {info['beta']:.12g} oracle {beta_ref:.12g}, estimates {info['bb_estimates']} {len(trail)}",
          flush=True)
    assert info["status"] == abip.ABIP_MAX_ITERS
    assert info["bb_estimates"] == len(trail)
    assert info["bb_probe_iters"] == 2 * len(trail) == info["admm_iters"] == ref["admm_iters"]
    assert abs(info["beta"] - beta_ref) <= 1e-8 * beta_ref
    st = ref["state"]
    scale = 1.0 + np.abs(st.u()).max()
    for g, r in [(gy, st.y), (gx, st.x), (gs, st.s)]:
        assert np.abs(_np(g) - r).max() <= 1e-10 * scale


def test_bb_sparse_trajectory_and_full_solve():
    sl = lpgen.sparse_planted(150, 420, 2, density=0.02)
    As, x, y, sv, info, (gy, gx, gs, sc) = _sparse(sl, max_admm_iters=300)
    ref = oracle.solve(As.toarray(), sl["b"], sl["c"], Settings(bb=True, max_admm_iters=300))
    print(f"sparse 300: {info['status_name']} iters {info['admm_iters']} {ref['admm_iters']} ipm {info['ipm_iters']} "
          f"{ref['ipm_iters']} beta {info['beta']:.10g} {ref['betas'][-1][1]:.10g}", flush=True)
    assert info["status_name"] == ref["status_name"]
    assert info["ipm_iters"] == ref["ipm_iters"] and info["admm_iters"] == ref["admm_iters"]
    assert info["bb_estimates"] == sum(len(t) for (_, _, t) in ref["betas"])
    assert abs(info["beta"] - ref["betas"][-1][1]) <= 1e-6 * ref["betas"][-1][1]
    # a full solve with the default CG rule
    A = sl["A_csr"]
    w = abip.abip_setup(As, sl["b"], sl["c"], abip.abip_default_settings(bb=1))
    x, y, sv, info = abip.abip_solve(w)
    print("sparse full:", info["status_name"], info["admm_iters"], info["bb_estimates"], info["beta"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED and info["bb_estimates"] > 0
    k = oracle.kkt_relative(As.toarray(), sl["b"], sl["c"], _np(x), _np(y), _np(sv))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    w.free()


@pytest.mark.parametrize("engine", ["grid", "streamed", "sparse"])
def test_bb_with_sqrt_restart_matches_oracle(engine):
    """The sqrt(gamma) restart (Algorithm 2) scales y in the pass that precedes the start point
    a beta choice keeps: 300-update trajectories against the oracle under that rule."""
    cap = 300
    if engine == "sparse":
        sl = lpgen.sparse_planted(150, 420, 2, density=0.02)
        As, x, y, sv, info, (gy, gx, gs, sc) = _sparse(sl, max_admm_iters=cap, restart_rule=abip.ABIP_RESTART_SQRT)
        A, b, c = As.toarray(), sl["b"], sl["c"]
    else:
        lp = lpgen.dense_planted(76, 159, 23)
        x, y, sv, info, (gy, gx, gs, sc) = _gpu(lp, engine, max_admm_iters=cap, restart_rule=abip.ABIP_RESTART_SQRT)
        A, b, c = lp["A"], lp["b"], lp["c"]
    ref = oracle.solve(A, b, c, Settings(bb=True, max_admm_iters=cap, restart_rule="sqrt"))
    print(f"{engine} sqrt: iters {info['admm_iters']} {ref['admm_iters']} ipm {info['ipm_iters']} {ref['ipm_iters']} "
          f"beta {info['beta']:.10g} {ref['betas'][-1][1]:.10g}", flush=True)
    assert info["status_name"] == ref["status_name"]
    assert info["ipm_iters"] == ref["ipm_iters"] and info["admm_iters"] == ref["admm_iters"]
    assert info["bb_estimates"] == sum(len(t) for (_, _, t) in ref["betas"])
    assert abs(info["beta"] - ref["betas"][-1][1]) <= 1e-6 * ref["betas"][-1][1]
    st = ref["state"]
    scale = 1.0 + np.abs(st.u()).max()
    for g, r in [(gy, st.y), (gx, st.x), (gs, st.s)]:
        assert np.abs(_np(g) - r).max() <= 1e-6 * scale


def test_bb_grid_two_row_chunks_fp32_bulk():
    """The grid engine's two-chunk variant (2100 rows) with the adaptive beta and FP32 bulk."""
    lp = lpgen.dense_planted(2100, 2300, 7)
    s = abip.abip_default_settings(bb=1, engine=abip.ABIP_ENGINE_GRID, precision=abip.ABIP_PREC_FP32_POLISH)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], s)
    x, y, sv, info = abip.abip_solve(w)
    print(info["status_name"], info["admm_iters"], info["bb_estimates"], info["beta"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED and info["bb_estimates"] > 0
    k = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(sv))
    assert max(k["pres"], k["dres"], k["gap"]) <= 1e-6
    assert abs(k["pobj"] - lp["pstar"]) <= 1e-5 * (1 + abs(lp["pstar"]))
    w.free()
