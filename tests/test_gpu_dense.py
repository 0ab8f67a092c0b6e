"""GPU parity of the dense one-workgroup engine against the FP64 oracle.

Every call goes through the C ABI (libabip.so via the thin binding).
"""
import numpy as np
import pytest
import torch

import lpgen
import oracle
from oracle.abip import Problem, Settings

pytestmark = pytest.mark.gpu

abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _settings(**kw):
    return abip.abip_default_settings(**kw)


# one to four 256-row chunks per lane in the one-workgroup engine (m <= 256, 512, 768, 1024)
SHAPES = [(7, 13, 0), (50, 100, 1), (130, 301, 2), (300, 650, 3), (20, 1000, 4), (600, 1300, 5),
          (1000, 2100, 6)]


@pytest.mark.parametrize("m,n,seed", SHAPES)
def test_apply_iq_matches_oracle(m, n, seed):
    print(f"apply_iq m={m} n={n} seed={seed}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"])
    rng = np.random.default_rng(seed + 100)
    win = rng.standard_normal(m + n + 2)
    ref = oracle.SchurIQSolver(Problem(lp["A"], lp["b"], lp["c"])).solve(win)
    got = _np(abip.abip_apply_iq(w, 0, win))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err
    got32 = _np(abip.abip_apply_iq(w, 0, win, use_fp32=True))
    err32 = np.abs(got32 - ref).max() / np.abs(ref).max()
    assert err32 < 1e-4, err32
    # the adjoint's solve: (I+Q)^{-T} = (I-Q)^{-1}, against a dense solve
    Q = oracle.assemble_Q(Problem(lp["A"], lp["b"], lp["c"]))
    reft = np.linalg.solve(np.eye(m + n + 2) - Q, win)
    gott = _np(abip.abip_apply_iq(w, 0, win, transpose=True))
    errt = np.abs(gott - reft).max() / np.abs(reft).max()
    assert errt < 1e-10, errt


@pytest.mark.parametrize("m,n,seed", SHAPES)
@pytest.mark.parametrize("rule", ["heuristic", "sqrt"])
def test_iterations_match_oracle_elementwise(m, n, seed, rule):
    """Fixed number of relaxed ADMM iterations from the same (restarted) iterate."""
    print(f"iterate m={m} n={n} seed={seed} rule={rule}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings(alpha=1.8, gamma=0.5, restart_rule=rule)
    st = oracle.initial_state(prob, s)
    st = oracle.restart(st, s.gamma, rule)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(restart_rule=0 if rule == "heuristic" else 1))
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    solver = oracle.SchurIQSolver(prob)
    N = 40
    for _ in range(N):
        st = oracle.admm_iteration(prob, solver, st, s)
    abip.abip_iterate(w, 0, N)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    scale = 1.0 + np.abs(st.u()).max()
    assert np.abs(_np(y) - st.y).max() <= 1e-10 * scale
    assert np.abs(_np(x) - st.x).max() <= 1e-10 * scale
    assert np.abs(_np(sv) - st.s).max() <= 1e-10 * scale
    for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
        assert abs(sc[key] - ref) <= 1e-10 * scale, (key, sc[key], ref)
    # Theorem 3.1 invariants on the GPU iterate
    t = st.mu
    np.testing.assert_allclose(_np(x) * _np(sv), t, rtol=1e-9)


@pytest.mark.parametrize("seed", [4, 5, 7])
def test_solve_config0_matches_oracle(seed):
    print(f"solve config0 seed={seed}", flush=True)
    lp = lpgen.config0(seed)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"])
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED == ref["status"]
    x, y, s = _np(x), _np(y), _np(s)
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], x, y, s)
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    # 1e-6 relative KKT bounds the objective error only through ||y*|| ||Ax - b|| etc.
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
    assert abs(kk["pobj"] - ref["info"]["pobj"]) <= 1e-7 * (1 + abs(lp["pstar"]))
    # 1e-6 relative KKT bounds the distance to the planted vertex only up to conditioning
    assert np.linalg.norm(x - lp["x0"]) / (1 + np.linalg.norm(lp["x0"])) <= 1e-4
    # same algorithm in FP64: the trajectories agree and stop together
    assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"]), \
        (info["admm_iters"], ref["admm_iters"])
    np.testing.assert_allclose(x, ref["x"], atol=1e-6 * (1 + np.abs(ref["x"]).max()))


CERT_CFG = {"wg": {}, "wg_streamed": {"lds_resident": 0}, "grid": {"engine": 2},
            "wg_fp32": {"precision": 1}, "grid_fp32": {"engine": 2, "precision": 1}}


@pytest.mark.parametrize("cfg", list(CERT_CFG))
def test_toys_and_certificates(cfg):
    """Toy LPs and Farkas certificates (Section 4.1) on every dense configuration:
    one workgroup LDS-resident / streamed, grid engine, FP32 bulk + FP64 confirmation."""
    kw = dict(CERT_CFG[cfg])
    if "engine" in kw:
        kw["engine"] = abip.ABIP_ENGINE_GRID
    if "precision" in kw:
        kw["precision"] = abip.ABIP_PREC_FP32_POLISH
    for lp in [lpgen.toy_two_var(), lpgen.toy_primal_infeasible(), lpgen.toy_dual_infeasible(),
               lpgen.dense_farkas_infeasible(20, 50, 3)]:
        ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
        w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(**kw))
        x, y, s, info = abip.abip_solve(w)
        print(lp["status"], info["status_name"], info["admm_iters"], ref["admm_iters"], flush=True)
        assert info["status"] == ref["status"]
        if lp["status"] == "primal_infeasible":
            y = _np(y)
            assert abs(lp["b"] @ y - 1.0) < 1e-9
            assert np.linalg.norm(lp["A"].T @ y + _np(s)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001
            assert np.all(np.isnan(_np(x)))
        elif lp["status"] == "dual_infeasible":
            x = _np(x)
            assert abs(lp["c"] @ x + 1.0) < 1e-9 and np.all(x >= 0)
            assert np.linalg.norm(lp["A"] @ x) <= 1e-6 / np.linalg.norm(lp["c"]) * 1.001


def test_batch_uneven_matches_status_and_kkt():
    lps = [lpgen.dense_planted(m, n, sd) for (m, n, sd) in
           [(3, 6, 1), (12, 30, 2), (4, 8, 4), (50, 100, 5), (12, 30, 4)]]
    lps.append(lpgen.dense_farkas_infeasible(20, 50, 3))
    w = abip.abip_setup_batch([lp["A"] for lp in lps], [lp["b"] for lp in lps], [lp["c"] for lp in lps])
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    for lp, x, y, s, info in zip(lps, xs, ys, ss, infos):
        print(lp["m"], lp["n"], info["status_name"], info["admm_iters"], flush=True)
        if lp["status"] == "solved":
            assert info["status"] == abip.ABIP_SOLVED
            kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
            assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
        else:
            assert info["status"] == abip.ABIP_PRIMAL_INFEASIBLE
    # the batch gives the same answers as one-at-a-time solves
    for k in [0, 3]:
        lp = lps[k]
        w1 = abip.abip_setup(lp["A"], lp["b"], lp["c"])
        x1, _, _, info1 = abip.abip_solve(w1)
        assert info1["admm_iters"] == infos[k]["admm_iters"]
        assert torch.equal(x1, xs[k])


@pytest.mark.parametrize("seed", [4, 5])
def test_fp32_bulk_with_fp64_polish(seed):
    lp = lpgen.config0(seed)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, s, info = abip.abip_solve(w)
    print(info, flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))


def test_boundary_errors():
    lp = lpgen.dense_planted(5, 9, 0)
    A = lp["A"].copy()
    A[1, 2] = np.nan
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(A, lp["b"], lp["c"])
    assert e.value.code == abip.ABIP_E_NONFINITE
    b = lp["b"].copy()
    b[0] = np.inf
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(lp["A"], b, lp["c"])
    assert e.value.code == abip.ABIP_E_NONFINITE
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(gamma=1.5))
    assert e.value.code == abip.ABIP_E_INVALID
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(max_admm_iters=5))
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_MAX_ITERS and info["admm_iters"] == 5


def test_out_of_device_memory_is_reported_and_frees_what_it_took():
    """A batch whose pools exceed the GPU's memory (every LP points at the same 1000 x 3000
    A, so the caller holds one copy): ABIP_E_OOM, the allocations made before the failing
    one released, and a normal setup and solve afterwards."""
    m, n = 1000, 3000
    total = torch.cuda.get_device_properties(0).total_memory
    B = int(1.25 * total // (8 * m * n)) + 1          # the FP64 copies of A alone exceed the memory
    print(f"oom batch B={B} of {m}x{n}", flush=True)
    A = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    b = torch.zeros(m, dtype=torch.float64, device="cuda")
    c = torch.ones(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with pytest.raises(abip.ABIPError) as e:
        abip.abip_setup_batch([A] * B, [b] * B, [c] * B)
    assert e.value.code == abip.ABIP_E_OOM, str(e.value)
    assert "out of device memory" in str(e.value) or "hipMalloc" in str(e.value)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20), (free0, free1)
    lp = lpgen.dense_planted(30, 75, 2)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"])
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED


@pytest.mark.parametrize("engine", ["wg", "grid"])
def test_fp32_floor_hands_over_to_fp64(engine):
    """Infeasible LPs whose FP32 inner loop settles above mu: the FP32 phase must
    hand over to FP64 and the Farkas certificate must still be found."""
    lps = lpgen.batch(48, 3)
    picks = [k for k in range(len(lps)) if lps[k]["status"] != "solved"][:3]
    assert picks
    eng = abip.ABIP_ENGINE_GRID if engine == "grid" else abip.ABIP_ENGINE_WG
    for k in picks:
        lp = lps[k]
        w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                            _settings(precision=abip.ABIP_PREC_FP32_POLISH, engine=eng, max_admm_iters=30000))
        x, y, s, info = abip.abip_solve(w)
        print(engine, k, lp["m"], lp["n"], info["status_name"], info["admm_iters"], info["admm_iters_fp64"],
              flush=True)
        assert info["status"] == abip.ABIP_PRIMAL_INFEASIBLE
        y = _np(y)
        assert abs(lp["b"] @ y - 1.0) < 1e-9
        assert np.linalg.norm(lp["A"].T @ y + _np(s)) <= 1e-6 / np.linalg.norm(lp["b"]) * 1.001
        assert info["admm_iters"] - info["admm_iters_fp64"] > 0      # the bulk ran in FP32


@pytest.mark.parametrize("m,n,seed", [(600, 1300, 5), (1000, 2100, 6)])
def test_fp32_polish_solve_three_and_four_chunks(m, n, seed):
    """FP32-streamed A and G^{-1} with three and four 256-row chunks per lane (one
    workgroup): the solve reaches the planted optimum at the KKT tolerance."""
    lp = lpgen.dense_planted(m, n, seed)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(precision=abip.ABIP_PREC_FP32_POLISH))
    x, y, s, info = abip.abip_solve(w)
    print(m, n, info["status_name"], info["admm_iters"], info["admm_iters_fp64"], flush=True)
    assert info["status"] == abip.ABIP_SOLVED
    kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))


def test_zero_row_and_empty_column_every_engine():
    """A planted LP extended by a zero row (b_i = 0: A loses full row rank, G = I + A A^T
    stays nonsingular) and an empty column with cost 1 (its x_j is 0 at the optimum, the
    planted pair stays optimal): the oracle and every engine reach the planted value."""
    import scipy.sparse as sp
    lp = lpgen.dense_planted(40, 90, 12)
    m, n = lp["A"].shape
    A = np.zeros((m + 1, n + 1))
    A[:m, :n] = lp["A"]
    b = np.concatenate([lp["b"], [0.0]])
    c = np.concatenate([lp["c"], [1.0]])
    ref = oracle.solve(A, b, c)
    assert ref["status_name"] == "solved"
    assert abs(c @ ref["x"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"]))
    cases = [("wg", A, _settings()), ("grid", A, _settings(engine=abip.ABIP_ENGINE_GRID)),
             ("sparse lds", sp.csr_matrix(A), _settings(lds_resident=1)),
             ("sparse global", sp.csr_matrix(A), _settings(lds_resident=0))]
    for name, Ain, st in cases:
        w = abip.abip_setup(Ain, b, c, st)
        x, y, s, info = abip.abip_solve(w)
        print(name, info["status_name"], info["admm_iters"], "oracle", ref["admm_iters"], flush=True)
        assert info["status"] == abip.ABIP_SOLVED, name
        kk = oracle.kkt_relative(A, b, c, _np(x), _np(y), _np(s))
        assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, (name, kk)
        assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"])), name
        assert abs(_np(x)[n]) <= 1e-4 * (1 + np.abs(_np(x)).max()), name
        w.free()


def test_more_rows_than_columns_every_engine():
    """m > n: a planted 6 x 12 LP whose rows are repeated as 12 random combinations
    (18 x 12, rank 6, consistent b).  The feasible set and the optimum are the planted
    LP's; G = I + A A^T is nonsingular regardless of rank.  Every engine reaches the
    oracle's iteration count and the planted value."""
    import scipy.sparse as sp
    lp = lpgen.dense_planted(6, 12, 13)
    R = np.random.default_rng(5).standard_normal((12, 6))
    A = np.vstack([lp["A"], R @ lp["A"]])
    b = np.concatenate([lp["b"], R @ lp["b"]])
    c = lp["c"]
    ref = oracle.solve(A, b, c)
    assert ref["status_name"] == "solved"
    cases = [("wg", A, _settings()), ("wg streamed", A, _settings(lds_resident=0)),
             ("grid", A, _settings(engine=abip.ABIP_ENGINE_GRID)),
             # CG to the relative floor, so the step is the exact one the oracle takes
             ("sparse", sp.csr_matrix(A), _settings(cg_tol=1e-13, cg_max_iters=2000, cg_rule=1))]
    for name, Ain, st in cases:
        w = abip.abip_setup(Ain, b, c, st)
        x, y, s, info = abip.abip_solve(w)
        print(name, info["status_name"], info["admm_iters"], "oracle", ref["admm_iters"], flush=True)
        assert info["status"] == abip.ABIP_SOLVED, name
        kk = oracle.kkt_relative(A, b, c, _np(x), _np(y), _np(s))
        assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, (name, kk)
        assert abs(kk["pobj"] - lp["pstar"]) <= 1e-4 * (1 + abs(lp["pstar"])), name
        assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(5, ref["admm_iters"] // 50), name
        w.free()
