"""Grid engine's paired column pass against the FP64 oracle, via the C ABI.

When A = [A0, -A0] (a free variable split into x+ - x-, as in basis pursuit)
the column pass reads A0 alone: column j + n/2 takes the negated products of
column j, and each pair adds A0 (f_j - f_{j+n/2}) to the row sums.  The ADMM
step (Algorithm 2) is the same map, so the iterates must match the oracle's to
rounding with the pairing on and off; the pairing test itself is checked on
data that is paired, nearly paired, unpaired and of odd width, and across a
reload of the handle's data.
"""
import numpy as np
import pytest

import lpgen
import oracle
from oracle.abip import Problem, Settings

pytestmark = pytest.mark.gpu
abip = pytest.importorskip("paper_1805_12344_amd")


def _np(t):
    return t.detach().cpu().numpy()


def _settings(**kw):
    return abip.abip_default_settings(engine=abip.ABIP_ENGINE_GRID, **kw)


# (m, N): A is m x 2N.  125 pairs leave a ragged last column group; 2100 rows take
# the variant with two four-row chunks per lane.
@pytest.mark.parametrize("mirror", [1, 0])
@pytest.mark.parametrize("m,N,seed", [(50, 125, 1), (300, 700, 2), (2100, 1100, 3)])
def test_paired_iterations_match_oracle(m, N, seed, mirror):
    print(f"paired iterate m={m} N={N} mirror={mirror}", flush=True)
    lp = lpgen.basis_pursuit(m, N, max(2, N // 25), seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings()
    st = oracle.restart(oracle.initial_state(prob, s), s.gamma, s.restart_rule)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(grid_mirror=mirror))
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    solver = oracle.SchurIQSolver(prob)
    N_IT = 30
    for _ in range(N_IT):
        st = oracle.admm_iteration(prob, solver, st, s)
    abip.abip_iterate(w, 0, N_IT)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    scale = 1.0 + np.abs(st.u()).max()
    assert np.abs(_np(y) - st.y).max() <= 1e-9 * scale
    assert np.abs(_np(x) - st.x).max() <= 1e-9 * scale
    assert np.abs(_np(sv) - st.s).max() <= 1e-9 * scale
    for key, ref in [("tau", st.tau), ("kappa", st.kappa), ("theta", st.theta)]:
        assert abs(sc[key] - ref) <= 1e-9 * scale, (key, sc[key], ref)
    w.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32_polish"])
def test_paired_solve_matches_oracle(precision):
    lp = lpgen.basis_pursuit(60, 150, 6, 5)
    ref = oracle.solve(lp["A"], lp["b"], lp["c"], Settings())
    assert ref["status"] == oracle.SOLVED
    ref_obj = float(lp["c"] @ ref["x"])
    prec = abip.ABIP_PREC_FP64 if precision == "fp64" else abip.ABIP_PREC_FP32_POLISH
    for mirror in (1, 0):
        w = abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(grid_mirror=mirror, precision=prec))
        x, y, s, info = abip.abip_solve(w)
        print(precision, mirror, info["status_name"], info["admm_iters"], ref["admm_iters"], info["ipm_iters"],
              ref["ipm_iters"], flush=True)
        assert info["grid_mirror"] == mirror
        assert info["status"] == abip.ABIP_SOLVED
        kk = oracle.kkt_relative(lp["A"], lp["b"], lp["c"], _np(x), _np(y), _np(s))
        assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
        pobj = float(lp["c"] @ _np(x))
        assert abs(pobj - ref_obj) <= 1e-5 * (1 + abs(ref_obj)), (pobj, ref_obj)
        if precision == "fp64":
            assert info["ipm_iters"] == ref["ipm_iters"]
            assert abs(info["admm_iters"] - ref["admm_iters"]) <= max(3, 0.01 * ref["admm_iters"])
        w.free()


def test_pairing_detection_and_reload():
    lp = lpgen.basis_pursuit(40, 90, 4, 7)
    A, b, c = lp["A"], lp["b"], lp["c"]
    w = abip.abip_setup(A, b, c, _settings())
    x1, _, _, info = abip.abip_solve(w)
    assert info["grid_mirror"] == 1 and info["status"] == abip.ABIP_SOLVED
    x1 = _np(x1).copy()
    it1 = info["admm_iters"]
    # one entry of the second half one ulp off: not paired, every column is read
    A2 = A.copy()
    A2[3, 90 + 5] = np.nextafter(A2[3, 90 + 5], np.inf)
    abip.abip_update_data(w, [A2], [b], [c])
    x2, y2, s2, info2 = abip.abip_solve(w)
    assert info2["grid_mirror"] == 0 and info2["status"] == abip.ABIP_SOLVED
    ref2 = oracle.solve(A2, b, c, Settings())
    assert abs(info2["admm_iters"] - ref2["admm_iters"]) <= max(3, 0.01 * ref2["admm_iters"])
    kk = oracle.kkt_relative(A2, b, c, _np(x2), _np(y2), _np(s2))
    assert max(kk["pres"], kk["dres"], kk["gap"]) <= 1e-6, kk
    # the paired data again: the same arithmetic as the first solve, bit for bit
    abip.abip_update_data(w, [A], [b], [c])
    x3, _, _, info3 = abip.abip_solve(w)
    assert info3["grid_mirror"] == 1 and info3["admm_iters"] == it1
    assert np.array_equal(_np(x3), x1)
    w.free()
    # even width but unpaired, and odd width: the pairing test fails or is not taken
    for m, n, seed in [(30, 70, 11), (30, 71, 12)]:
        lp2 = lpgen.dense_planted(m, n, seed)
        w2 = abip.abip_setup(lp2["A"], lp2["b"], lp2["c"], _settings())
        _, _, _, i2 = abip.abip_solve(w2)
        assert i2["grid_mirror"] == 0 and i2["status"] == abip.ABIP_SOLVED
        w2.free()


def test_grid_mirror_setting_is_validated():
    lp = lpgen.basis_pursuit(10, 20, 2, 1)
    with pytest.raises(Exception):
        abip.abip_setup(lp["A"], lp["b"], lp["c"], _settings(grid_mirror=2))


@pytest.mark.parametrize("mirror", [1, 0])
@pytest.mark.parametrize("m,N,seed", [(120, 500, 4), (2100, 2300, 5)])
def test_paired_fp32_data_iterations_match_model(m, N, seed, mirror):
    """FP32 data (the bulk phase): the oracle iterating with its FP32-data model of
    the step (A and G^{-1} rounded to FP32, FP64 arithmetic).  Rounding commutes
    with negation, so the model's A is what the paired pass reads as [A0, -A0]."""
    print(f"paired fp32 iterate m={m} N={N} mirror={mirror}", flush=True)
    lp = lpgen.basis_pursuit(m, N, max(2, N // 25), seed)
    prob = Problem(lp["A"], lp["b"], lp["c"])
    s = Settings()
    st = oracle.restart(oracle.initial_state(prob, s), s.gamma, s.restart_rule)
    w = abip.abip_setup(lp["A"], lp["b"], lp["c"],
                        _settings(grid_mirror=mirror, precision=abip.ABIP_PREC_FP32_POLISH))
    abip.abip_set_state(w, 0, st.y, st.x, st.s, st.tau, st.kappa, st.theta, st.mu)
    model = oracle.Fp32DataSchurSolver(prob)
    exact = oracle.SchurIQSolver(prob)
    N_IT = 30
    st_m, st_e = st.copy(), st.copy()
    for _ in range(N_IT):
        st_m = oracle.admm_iteration(prob, model, st_m, s)
        st_e = oracle.admm_iteration(prob, exact, st_e, s)
    abip.abip_iterate(w, 0, N_IT, use_fp32=True)
    y, x, sv, sc = abip.abip_get_state(w, 0)
    y, x, sv = _np(y), _np(x), _np(sv)
    scale = 1.0 + np.abs(st_m.u()).max()
    dev = max(np.abs(y - st_m.y).max(), np.abs(x - st_m.x).max(), np.abs(sv - st_m.s).max())
    gap32 = max(np.abs(st_m.x - st_e.x).max(), np.abs(st_m.y - st_e.y).max())
    print(f"  |gpu - model| = {dev:.3e}, |model - exact| = {gap32:.3e}", flush=True)
    assert dev <= 1e-9 * scale, dev
    for key, ref in [("tau", st_m.tau), ("kappa", st_m.kappa), ("theta", st_m.theta)]:
        assert abs(sc[key] - ref) <= 1e-9 * scale, (key, sc[key], ref)
    assert gap32 > 10 * dev          # FP32 rounding moves the iterate far more than the bar
    w.free()
