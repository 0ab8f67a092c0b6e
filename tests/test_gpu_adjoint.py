"""GPU adjoint (abip_backward) against the dense FP64 KKT adjoint and the
basis-solution derivative.  All calls go through the C ABI."""
import numpy as np
import pytest
import torch

import lpgen
import oracle

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("m,n,seed,t", [(5, 12, 1, 1e-3), (30, 75, 2, 1e-5), (130, 300, 3, 1e-7)])
def test_backward_equals_kkt_adjoint_at_central_point(m, n, seed, t):
    print(f"adjoint central m={m} n={n} t={t}", flush=True)
    lp = lpgen.dense_planted(m, n, seed)
    A, b, c = lp["A"], lp["b"], lp["c"]
    cp = oracle.central_point(A, b, c, t=t)
    w = abip.abip_setup(A, b, c)
    abip.abip_set_state(w, 0, cp.y, cp.x, cp.s, cp.tau, cp.kappa, cp.theta, t)
    g = np.random.default_rng(seed).standard_normal(n)
    dc, db, dA = abip.abip_backward(w, g, want_A=True)
    it, rr = abip.abip_backward_stats(w)
    ref = oracle.contract_adjoint(A, b, c, cp, oracle.kkt_adjoint(A, b, c, cp, g), want_A=True)
    print("bicgstab iters", it, "resid", rr, flush=True)
    # dL/db and dL/dA are O(1); dL/dc tends to 0 at the optimum (a nondegenerate
    # vertex is locally constant in c), so it is compared on the scale of the
    # terms it is made of (|zeta| x |u|, zeta the adjoint), not relative to itself
    for got, want in [(db, ref["db"]), (dA, ref["dA"])]:
        err = np.abs(_np(got) - want).max() / (1e-12 + np.abs(want).max())
        assert err < 1e-7, err
    lam = oracle.kkt_adjoint(A, b, c, cp, g)
    scale = np.abs(lam).max() * (1.0 + np.abs(cp.u()).max())
    assert np.abs(_np(dc) - ref["dc"]).max() <= 1e-9 * scale


def test_backward_after_solve_matches_oracle_and_basis_formula():
    lp = lpgen.dense_planted(30, 75, 11)
    A, b, c = lp["A"], lp["b"], lp["c"]
    g = np.random.default_rng(5).standard_normal(75)
    w = abip.abip_setup(A, b, c, abip.abip_default_settings(eps=1e-7))
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED
    dc, db, dA = abip.abip_backward(w, g, want_A=True)
    yv, xv, sv, sc = abip.abip_get_state(w, 0)
    st = oracle.State(_np(yv), _np(xv), sc["tau"], sc["theta"], _np(sv), sc["kappa"], sc["mu"])
    ref = oracle.contract_adjoint(A, b, c, st, oracle.kkt_adjoint(A, b, c, st, g), want_A=True)
    for got, want in [(db, ref["db"]), (dA, ref["dA"])]:
        assert np.abs(_np(got) - want).max() <= 1e-7 * (1 + np.abs(want).max())
    lam = oracle.kkt_adjoint(A, b, c, st, g)
    assert np.abs(_np(dc) - ref["dc"]).max() <= 1e-9 * np.abs(lam).max() * (1.0 + np.abs(st.u()).max())
    # as mu -> 0 the central point tends to the planted nondegenerate vertex, whose derivative is
    # dL/db = A_B^{-T} w_B and dL/dc = 0 (the fixed point of Algorithm 2 read as a map of (b, c))
    bg = oracle.basis_gradients(A, b, lp["basis"], g)
    assert np.abs(_np(db) - bg["db"]).max() <= 1e-3 * (1 + np.abs(bg["db"]).max())
    assert np.abs(_np(dc)).max() <= 1e-3 * np.linalg.norm(g)


def test_autograd_function_and_batch_backward():
    lp = lpgen.dense_planted(20, 50, 4)
    A = torch.tensor(lp["A"], device="cuda", requires_grad=True)
    b = torch.tensor(lp["b"], device="cuda", requires_grad=True)
    c = torch.tensor(lp["c"], device="cuda", requires_grad=True)
    g = torch.randn(50, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    x = abip.abip_solve_diff(A, b, c)
    (g * x).sum().backward()
    bg = oracle.basis_gradients(lp["A"], lp["b"], lp["basis"], _np(g))
    assert np.abs(_np(b.grad) - bg["db"]).max() <= 1e-3 * (1 + np.abs(bg["db"]).max())
    assert np.abs(_np(A.grad) - bg["dA"]).max() <= 1e-3 * (1 + np.abs(bg["dA"]).max())
    # batch: FP32-bulk forward, FP64 adjoint, each LP against its own single backward
    lps = lpgen.diff_batch(6, 20, 50, 9)
    wb = abip.abip_setup_batch([l["A"] for l in lps], [l["b"] for l in lps], [l["c"] for l in lps],
                               abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    xs, ys, ss, infos = abip.abip_solve_batch(wb)
    dcs, dbs, _ = abip.abip_backward_batch(wb, [l["w"] for l in lps])
    for k, l in enumerate(lps):
        assert infos[k]["status"] == abip.ABIP_SOLVED
        yv, xv, sv, sc = abip.abip_get_state(wb, k)
        st = oracle.State(_np(yv), _np(xv), sc["tau"], sc["theta"], _np(sv), sc["kappa"], sc["mu"])
        ref = oracle.contract_adjoint(l["A"], l["b"], l["c"], st, oracle.kkt_adjoint(l["A"], l["b"], l["c"], st, l["w"]))
        assert np.abs(_np(dbs[k]) - ref["db"]).max() <= 1e-7 * (1 + np.abs(ref["db"]).max())
        lam = oracle.kkt_adjoint(l["A"], l["b"], l["c"], st, l["w"])
        assert np.abs(_np(dcs[k]) - ref["dc"]).max() <= 1e-9 * np.abs(lam).max() * (1.0 + np.abs(st.u()).max())


def test_backward_recovers_from_bicgstab_breakdown():
    """LPs of the 64 x (200 x 500) differentiable batch whose adjoint BiCGSTAB meets a
    breakdown (two-sided recurrence orthogonal / non-finite step): the restarted
    solve must still give the KKT adjoint and the basis-solution derivative."""
    lps = lpgen.diff_batch(64, 200, 500, 4)
    picks = [8, 55, 0]
    sub = [lps[k] for k in picks]
    wb = abip.abip_setup_batch([l["A"] for l in sub], [l["b"] for l in sub], [l["c"] for l in sub],
                               abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    xs, ys, ss, infos = abip.abip_solve_batch(wb)
    dcs, dbs, _ = abip.abip_backward_batch(wb, [l["w"] for l in sub])
    for k, l in enumerate(sub):
        assert infos[k]["status"] == abip.ABIP_SOLVED
        it, rr = abip.abip_backward_stats(wb, k)
        print(picks[k], "bicgstab", it, rr, flush=True)
        assert np.isfinite(rr) and rr <= 1e-11
        yv, xv, sv, sc = abip.abip_get_state(wb, k)
        st = oracle.State(_np(yv), _np(xv), sc["tau"], sc["theta"], _np(sv), sc["kappa"], sc["mu"])
        lam = oracle.kkt_adjoint(l["A"], l["b"], l["c"], st, l["w"])
        ref = oracle.contract_adjoint(l["A"], l["b"], l["c"], st, lam)
        # at mu ~ 1e-8 the adjoint system is ill conditioned (BiCGSTAB stops at a relative
        # residual ~1e-12, the solution error is about cond x residual): a looser bar than
        # the central-point tests, and the LP derivative itself as the real check
        e_kkt = np.abs(_np(dbs[k]) - ref["db"]).max() / (1 + np.abs(ref["db"]).max())
        bg = oracle.basis_gradients(l["A"], l["b"], l["basis"], l["w"])
        e_lp = np.abs(_np(dbs[k]) - bg["db"]).max() / (1 + np.abs(bg["db"]).max())
        print(picks[k], "db vs KKT adjoint", e_kkt, "vs basis formula", e_lp, flush=True)
        # the object differentiated is the fixed point at the final mu; its distance
        # to the vertex derivative depends on how close the planted vertex is to
        # degenerate, so only the KKT adjoint at the same iterate is a bar here
        assert e_kkt <= 1e-3


def _csr(lp):
    import scipy.sparse as sp
    A = lp["A_csr"]
    return sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])


def _one_lp_handle(engine, m, n, seed, **kw):
    """(handle, dense A, b, c, CSR A or None) of a planted LP on the grid or the sparse engine."""
    if engine == "grid":
        lp = lpgen.dense_planted(m, n, seed)
        w = abip.abip_setup(lp["A"], lp["b"], lp["c"], abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID, **kw))
        return w, lp["A"], lp["b"], lp["c"], None
    lp = lpgen.sparse_planted(m, n, seed, density=0.05)
    A = _csr(lp)
    w = abip.abip_setup(A, lp["b"], lp["c"], abip.abip_default_settings(cg_tol=1e-13, cg_max_iters=2000, cg_rule=1,
                                                                         **kw))
    return w, A.toarray(), lp["b"], lp["c"], A


def _check_against_kkt(engine, A, b, c, st, g, dc, db, dA, Acsr, bar):
    lam = oracle.kkt_adjoint(A, b, c, st, g)
    ref = oracle.contract_adjoint(A, b, c, st, lam, want_A=True)
    dA_ref = ref["dA"]
    if Acsr is not None:      # the CSR engine returns dL/dA on the stored entries, in CSR order
        rows = np.repeat(np.arange(Acsr.shape[0]), np.diff(Acsr.indptr))
        dA_ref = ref["dA"][rows, Acsr.indices]
    for got, want in [(db, ref["db"]), (dA, dA_ref)]:
        err = np.abs(_np(got) - want).max() / (1e-12 + np.abs(want).max())
        assert err < bar, (engine, err)
    scale = np.abs(lam).max() * (1.0 + np.abs(st.u()).max())
    assert np.abs(_np(dc) - ref["dc"]).max() <= 1e-2 * bar * scale


@pytest.mark.parametrize("engine", ["grid", "sparse"])
@pytest.mark.parametrize("m,n,seed,t", [(5, 12, 1, 1e-3), (30, 75, 2, 1e-5), (130, 300, 3, 1e-7)])
def test_backward_one_lp_engines_at_central_point(engine, m, n, seed, t):
    """The adjoint driven from the host over the whole GPU (one large dense LP, CSR LP)
    equals the dense KKT adjoint of the central-path system at a central point."""
    print(f"adjoint {engine} central m={m} n={n} t={t}", flush=True)
    w, A, b, c, Acsr = _one_lp_handle(engine, m, n, seed)
    cp = oracle.central_point(A, b, c, t=t)
    abip.abip_set_state(w, 0, cp.y, cp.x, cp.s, cp.tau, cp.kappa, cp.theta, t)
    g = np.random.default_rng(seed).standard_normal(n)
    dc, db, dA = abip.abip_backward(w, g, want_A=True)
    it, rr = abip.abip_backward_stats(w)
    print("bicgstab iters", it, "resid", rr, flush=True)
    assert rr <= 1e-12
    _check_against_kkt(engine, A, b, c, cp, g, dc, db, dA, Acsr, 1e-7)
    # a second call reuses the workspace (and, for CSR, the border of I - Q)
    dc2, db2, _ = abip.abip_backward(w, g)
    assert np.array_equal(_np(dc2), _np(dc)) and np.array_equal(_np(db2), _np(db))


@pytest.mark.parametrize("engine,m,n,seed", [("grid", 300, 700, 5), ("sparse", 150, 420, 6)])
def test_backward_one_lp_engines_after_solve(engine, m, n, seed):
    """After a full solve: against the KKT adjoint at the returned iterate; the grid
    engine's gradients also against the one-workgroup engine's on the same LP."""
    print(f"adjoint {engine} after solve m={m} n={n}", flush=True)
    w, A, b, c, Acsr = _one_lp_handle(engine, m, n, seed, eps=1e-7)
    x, y, s, info = abip.abip_solve(w)
    assert info["status"] == abip.ABIP_SOLVED
    g = np.random.default_rng(seed).standard_normal(n)
    dc, db, dA = abip.abip_backward(w, g, want_A=True)
    it, rr = abip.abip_backward_stats(w)
    print("bicgstab iters", it, "resid", rr, flush=True)
    yv, xv, sv, sc = abip.abip_get_state(w, 0)
    st = oracle.State(_np(yv), _np(xv), sc["tau"], sc["theta"], _np(sv), sc["kappa"], sc["mu"])
    # near the optimum the adjoint system is ill conditioned (see the breakdown test)
    _check_against_kkt(engine, A, b, c, st, g, dc, db, dA, Acsr, 1e-5)
    if engine == "grid":
        w1 = abip.abip_setup(A, b, c, abip.abip_default_settings(engine=abip.ABIP_ENGINE_WG))
        abip.abip_set_state(w1, 0, yv, xv, sv, sc["tau"], sc["kappa"], sc["theta"], sc["mu"])
        dc1, db1, dA1 = abip.abip_backward(w1, g, want_A=True)
        for got, want in [(db, db1), (dA, dA1)]:
            assert np.abs(_np(got) - _np(want)).max() <= 1e-6 * (1 + np.abs(_np(want)).max())
    if engine == "sparse":   # the solve's state is untouched: solving again gives the same point
        x2, _, _, info2 = abip.abip_solve(w)
        assert info2["admm_iters"] == info["admm_iters"]
        assert np.array_equal(_np(x2), _np(x))
