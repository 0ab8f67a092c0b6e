#!/usr/bin/env python3
"""ABIP throughput on one MI355X: many uneven dense LPs solved to 1e-6 relative KKT.

Workload (one "step"): 256 dense random LPs, m ~ U{20..400}, n ~ U{2m..3m},
planted strictly complementary optima, 10% made primal infeasible by a planted
Farkas vector (seed 3).  A step is the whole hot path for the batch: setup
(HSD constants, FP64 SYRK + Cholesky + inverse of I + A A^T, Schur border) and
the batched ABIP solve (FP32 bulk with FP64 checks and FP64 polish) in one
persistent launch, inputs already resident in HBM.

Printed: one JSON line.  value = LP solves/s (LPs ending with the right status,
solved ones re-checked in FP64 on the host at <= 1e-6 relative KKT) over the
end-to-end wall time of the timed steps.  Beside it: the FP64 batched run and
the plain FP64 path (one LP per setup/solve call) on the same 256 LPs, the
error of every FP32-bulk result against the FP64 results and the planted
optimum, the roofline of the solve kernel, the oracle's time on the host cores,
and extra measurements of the other workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM-side traffic of the persistent solve kernel from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of this same default command,
# scaled by what the counters read for a plain copy of known size
# (bench.py --copy-calibration).  Keyed by a hash of the kernel's sources: any
# change to them voids the figure (reported as null until measured again).
PMC_TRAFFIC = {
    # k_solve_wg<2, 256, false, false> (beta fixed) on the 256-LP batch, one step
    "b18b07d907567789:bb0": {"fetch_kib": 1020510046.25, "fetch_scale": 1048576.0 / 524315.3125,
                         "write_kib": 19796195.8125, "write_scale": 1048576.0 / 1048576.0},
    # k_solve_wg<2, 256, true, false> (adaptive beta, the default) on the same batch, one step
    # (profiles/k_solve_wg_batched256_pmc.md)
    "b18b07d907567789:bb1": {"fetch_kib": 1245388554.0, "fetch_scale": 1048576.0 / 524315.3125,
                             "write_kib": 24280125.4375, "write_scale": 1048576.0 / 1048576.0},
}
KERNEL_SOURCES = ["paper_1805_12344_amd/csrc/abip_solve_wg.hip", "paper_1805_12344_amd/csrc/abip_small.h",
                  "paper_1805_12344_amd/csrc/abip_internal.h"]


BB_MODE = [1]   # the run's settings.bb (the kernel variant the counters belong to)


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def copy_calibration(nbytes=1 << 30):
    """One plain device-to-device copy of known size, for scaling the PMC bytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(count, seed):
    import lpgen
    return lpgen.batch(count, seed)


def to_device(lps):
    import torch
    As = [torch.tensor(lp["A"], dtype=torch.float64, device="cuda") for lp in lps]
    bs = [torch.tensor(lp["b"], dtype=torch.float64, device="cuda") for lp in lps]
    cs = [torch.tensor(lp["c"], dtype=torch.float64, device="cuda") for lp in lps]
    torch.cuda.synchronize()
    return As, bs, cs


def host_kkt(A, b, c, x, y, s):
    """The relative residuals of the Section 4.1 tests for a returned (x, y, s),
    recomputed in FP64 on the host: (pres, dres, gap)."""
    pres = np.linalg.norm(A @ x - b) / (1 + np.linalg.norm(b))
    dres = np.linalg.norm(A.T @ y + s - c) / (1 + np.linalg.norm(c))
    pobj, dobj = float(c @ x), float(b @ y)
    gap = abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj))
    return float(pres), float(dres), float(gap)


def _host(ts):
    return [t.cpu().numpy() for t in ts]


def verify(lps, xs, ys, ss, infos, eps=1e-6):
    """Host FP64 re-check: status right, and KKT <= eps for solved LPs.
    Returns (number correct, worst KKT, per-LP host KKT (NaN where not solved))."""
    ok = 0
    worst = 0.0
    per = []
    for lp, x, y, s, info in zip(lps, xs, ys, ss, infos):
        kkt = float("nan")
        if lp["status"] == "solved":
            if info["status"] == 1:
                kkt = max(host_kkt(lp["A"], lp["b"], lp["c"], x, y, s))
                worst = max(worst, kkt)
                if kkt <= eps * (1 + 1e-9):
                    ok += 1
        elif info["status"] == 2:
            ok += 1
        per.append(kkt)
    return ok, worst, per


# ---------------------------------------------------------------------------
# bytes of the solve kernel
# ---------------------------------------------------------------------------

def survey_bytes_per_update(m, n, p):
    """Algorithmic bytes of one ADMM update by the count of the scope table's
    measurement row: A read twice (2 m n p), the factor's two triangular sweeps
    (m^2 p, here one pass over the symmetric G^{-1}) and about ten vectors of
    length m + n in FP64; p = 4 for FP32 data, 8 for FP64."""
    return 2.0 * m * n * p + m * m * p + 80.0 * (m + n)


def launch_bytes(lps, infos):
    """Bytes of one persistent solve launch, from the library's own counters.

    survey: every update priced by survey_bytes_per_update (data precision of
            the update), wherever the data actually lives;
    hbm:    what this design must move through device memory: one read of A
            per pass that streams it (8 doubles per column of vectors with it)
            and one read of G^{-1} per pass that reads it from device memory;
            passes whose A (and G^{-1}) sit in LDS move no HBM bytes.
    """
    survey = hbm = 0.0
    passes = {"lds": 0, "streamed": 0}
    for lp, info in zip(lps, infos):
        m, n = lp["m"], lp["n"]
        it64 = info["admm_iters_fp64"]
        it32 = info["admm_iters"] - it64
        survey += it32 * survey_bytes_per_update(m, n, 4) + it64 * survey_bytes_per_update(m, n, 8)
        s32 = info["colpass_fp32"] - info["colpass_lds_fp32"]
        s64 = info["colpass_fp64"] - info["colpass_lds_fp64"]
        hbm += s32 * (4.0 * m * n + 64.0 * n) + s64 * (8.0 * m * n + 64.0 * n)
        hbm += info["ginv_hbm_fp32"] * 4.0 * m * m + info["ginv_hbm_fp64"] * 8.0 * m * m
        passes["lds"] += info["colpass_lds_fp32"] + info["colpass_lds_fp64"]
        passes["streamed"] += s32 + s64
    return survey, hbm, passes


def traffic_bytes():
    t = PMC_TRAFFIC.get(f"{kernel_hash()}:bb{BB_MODE[0]}")
    if t is None:
        return None
    return t["fetch_kib"] * 1024.0 * t["fetch_scale"] + t["write_kib"] * 1024.0 * t["write_scale"]


def run_batch(abip, As, bs, cs, settings):
    w = abip.abip_setup_batch(As, bs, cs, settings)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    w.free()
    return xs, ys, ss, infos


def _stats(v):
    v = [x for x in v if np.isfinite(x)]
    if not v:
        return None
    return {"max": float(np.max(v)), "median": float(np.median(v)), "count": len(v)}


def error_report(lps, r32, r64):
    """Error of every FP32-bulk result against the FP64 batched result of the
    same LP and against the planted optimum (unique: |supp x0| = m)."""
    e_obj64, e_x64, e_objp, e_xp, lib, lib_cap = [], [], [], [], [], []
    for k, lp in enumerate(lps):
        i32, i64 = r32[3][k], r64[3][k]
        (lib_cap if i32["status"] == 4 else lib).append(i32["err_vs_fp64"])
        if lp["status"] != "solved" or i32["status"] != 1 or i64["status"] != 1:
            continue
        x32, x64 = r32[0][k], r64[0][k]
        p32, p64 = float(lp["c"] @ x32), float(lp["c"] @ x64)
        e_obj64.append(abs(p32 - p64) / (1 + abs(p64)))
        e_x64.append(float(np.linalg.norm(x32 - x64) / (1 + np.linalg.norm(x64))))
        e_objp.append(abs(p32 - lp["pstar"]) / (1 + abs(lp["pstar"])))
        e_xp.append(float(np.linalg.norm(x32 - lp["x0"]) / (1 + np.linalg.norm(lp["x0"]))))
    return {"what": "fp32-bulk results: objective |c^T x - ref| / (1 + |ref|) and solution "
                    "||x - x_ref|| / (1 + ||x_ref||) against the fp64 batched result and the planted optimum; "
                    "err_vs_fp64 = the library's FP64 recheck of each returned point (relative KKT, or the "
                    "certificate test for infeasible LPs)",
            "obj_vs_fp64": _stats(e_obj64), "x_vs_fp64": _stats(e_x64),
            "obj_vs_planted": _stats(e_objp), "x_vs_planted": _stats(e_xp),
            "err_vs_fp64_library": _stats(lib), "err_vs_fp64_library_at_iteration_cap": _stats(lib_cap)}


def per_lp_rows(lps, infos, infos64, kkt):
    rows = []
    for k, (lp, i, j) in enumerate(zip(lps, infos, infos64)):
        rows.append([k, lp["m"], lp["n"], lp["status"], i["status_name"], i["admm_iters"], i["admm_iters_fp64"],
                     i["colpass_fp32"], i["colpass_fp64"], i["colpass_lds_fp32"], i["colpass_lds_fp64"],
                     i["ginv_hbm_fp32"], i["ginv_hbm_fp64"], i["lds_mode"], j["admm_iters"] if j else -1,
                     kkt[k], i["err_vs_fp64"], i["fp32_exit_kkt"],
                     i["ticks_total"] / 100.0 / max(1, i["admm_iters"])])
    return rows


PER_LP_HEADER = ["lp", "m", "n", "planted", "status", "iters", "iters_fp64", "colpass_fp32", "colpass_fp64",
                 "colpass_lds_fp32", "colpass_lds_fp64", "ginv_hbm_fp32", "ginv_hbm_fp64", "lds_mode",
                 "iters_fp64_batched", "host_kkt", "err_vs_fp64", "fp32_exit_kkt", "us_per_update"]


# ---------------------------------------------------------------------------
# the oracle on the host cores (cpu_baseline leg: the only part that runs the oracle)
# ---------------------------------------------------------------------------

def host_info():
    model = "?"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def _oracle_lp_times(A, b, c, cap, bb):
    """(setup seconds, seconds per iteration) of the oracle on one LP, at the
    caller's BLAS thread setting: Schur solver set up once, then `cap` updates."""
    import oracle
    prob = oracle.Problem(A, b, c)
    t0 = time.perf_counter()
    solver = oracle.SchurIQSolver(prob)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    out = oracle.solve(prob, settings=oracle.Settings(max_admm_iters=cap, bb=bb), solver=solver)
    return t_setup, (time.perf_counter() - t0) / max(1, out["admm_iters"])


def _pool_job(args):
    """One oracle job of the process-pool measurement (a worker process, one BLAS thread)."""
    from threadpoolctl import threadpool_limits
    A, b, c, cap, bb = args
    with threadpool_limits(limits=1):
        return _oracle_lp_times(A, b, c, cap, bb)[1]


def cpu_baseline(lps, iters64, correct, budget_iters=1500, bb=False, reps=3):
    """The FP64 oracle as it stands, timed on the host on a stratified sample of
    the batch: at one BLAS thread, at all host cores, and as a process pool.

    Every sampled LP runs its setup (Schur solver: Cholesky of G, border) and
    min(its FP64 iteration count, budget_iters) oracle iterations (tests every
    iteration), `reps` times; the medians are kept.  A least-squares fit of the
    per-iteration time against (1, m n, m^2) and of the setup time against
    (1, m^2 n) over the sample then prices every LP of the batch at its FP64
    iteration count (the same count the oracle takes: the GPU's FP64 path
    matches it to 1%), so the estimate covers the whole batch, including the
    slowest LPs.  bb: the oracle takes the same adaptive beta (Section 4.3) as
    the GPU solves.  Process pool: one worker per host core, one BLAS thread
    each, the LPs spread over the workers; its rate is the one-thread rate times
    the number of workers times their parallel efficiency, measured by running
    one job per worker at once on the sample's median LP.
    """
    from threadpoolctl import threadpool_limits
    model, nproc = host_info()
    order = np.argsort([lp["m"] * lp["n"] for lp in lps])
    sample = sorted(set(int(order[i]) for i in np.linspace(0, len(lps) - 1, 10).round().astype(int)) |
                    {k for k in range(len(lps)) if iters64[k] >= 10 ** 6} |
                    {int(k) for k in np.argsort(iters64)[-2:]})
    out = {}
    per_it_1 = {}
    for label, threads in (("1_thread", 1), ("all_cores", nproc)):
        rows_it, rows_su = [], []
        t_all = time.perf_counter()
        with threadpool_limits(limits=threads):
            for k in sample:
                lp = lps[k]
                cap = int(min(max(1, iters64[k]), budget_iters))
                runs = [_oracle_lp_times(lp["A"], lp["b"], lp["c"], cap, bb) for _ in range(reps)]
                t_setup = float(np.median([r[0] for r in runs]))
                t_it = float(np.median([r[1] for r in runs]))
                if threads == 1:
                    per_it_1[k] = t_it
                rows_it.append((lp["m"] * lp["n"], lp["m"] ** 2, t_it))
                rows_su.append((lp["m"] ** 2 * lp["n"], t_setup))
        wall = time.perf_counter() - t_all
        log(f"cpu_baseline {label}: {wall:.1f} s over {len(sample)} LPs x {reps}")
        X = np.array([[1.0, r[0], r[1]] for r in rows_it])
        ci, *_ = np.linalg.lstsq(X, np.array([r[2] for r in rows_it]), rcond=None)
        Xs = np.array([[1.0, r[0]] for r in rows_su])
        cs, *_ = np.linalg.lstsq(Xs, np.array([r[1] for r in rows_su]), rcond=None)
        total = 0.0
        for k, lp in enumerate(lps):
            m, n = lp["m"], lp["n"]
            t_it = max(ci[0] + ci[1] * m * n + ci[2] * m * m, 1e-7)
            t_su = max(cs[0] + cs[1] * m * m * n, 0.0)
            total += t_su + t_it * iters64[k]
        out[label] = {"value": correct / total, "threads": threads, "batch_seconds_estimated": total,
                      "sample_cpu_seconds": wall}
    # process pool: parallel efficiency of nproc concurrent one-thread jobs
    pool = None
    try:
        import multiprocessing as mp
        kmid = sorted(sample, key=lambda k: lps[k]["m"] * lps[k]["n"])[len(sample) // 2]   # median size
        lp = lps[kmid]
        cap = int(min(max(1, iters64[kmid]), budget_iters))
        t0 = time.perf_counter()
        from concurrent.futures import ProcessPoolExecutor
        # spawned workers (no GPU state), one job each; a failed worker raises instead of hanging
        with ProcessPoolExecutor(max_workers=nproc, mp_context=mp.get_context("spawn")) as ex:
            list(ex.map(_pool_job, [(lp["A"], lp["b"], lp["c"], 50, bb)] * nproc, timeout=600))   # workers warm
            times = list(ex.map(_pool_job, [(lp["A"], lp["b"], lp["c"], cap, bb)] * nproc, timeout=600))
        eff = per_it_1[kmid] / float(np.median(times))
        one_total = out["1_thread"]["batch_seconds_estimated"]
        pool = {"value": correct / (one_total / (nproc * eff)), "workers": nproc, "parallel_efficiency": eff,
                "probe_lp": kmid, "seconds": time.perf_counter() - t0}
        log(f"cpu_baseline process_pool: efficiency {eff:.2f} over {nproc} workers")
    except Exception as exc:          # the pool is a reported extra, never a failure of the bench
        pool = {"error": repr(exc)}
    one = out["1_thread"]
    return {"value": one["value"], "unit": "LP solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample)} LPs of the batch stratified by m n (indices {sample}, including every LP "
                      f"at the iteration cap and the two with the most iterations), setup + min(FP64 count, "
                      f"{budget_iters}) oracle iterations each, median of {reps} runs; "
                      f"per-iteration and setup times fitted against (1, m n, m^2) and (1, m^2 n) and summed "
                      f"over all {len(lps)} LPs at their FP64 iteration counts; {one['sample_cpu_seconds']:.1f} s "
                      f"of CPU work at 1 thread",
            "all_cores": out["all_cores"], "process_pool": pool, "host_cpu": model, "nproc": nproc}


def cpu_time_single(A, b, c, iters_total, sample_iters, solver_fn, threads):
    """Oracle time of one LP: setup once, `sample_iters` iterations, scaled to iters_total."""
    from threadpoolctl import threadpool_limits
    import oracle
    with threadpool_limits(limits=threads):
        prob = oracle.abip._as_problem(A, b, c)
        t0 = time.perf_counter()
        solver = solver_fn(prob)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        out = oracle.solve(prob, settings=oracle.Settings(max_admm_iters=sample_iters), solver=solver)
        t_it = (time.perf_counter() - t0) / max(1, out["admm_iters"])
    return {"threads": threads, "setup_s": t_setup, "s_per_iter": t_it, "iters_timed": out["admm_iters"],
            "solve_s_estimated": t_setup + t_it * iters_total}


# ---------------------------------------------------------------------------
# extra workloads
# ---------------------------------------------------------------------------

def _bp_solve(abip, torch, lp, A, b, c, mirror, bb=0):
    """One timed basis-pursuit solve on a fresh handle (grid engine, FP32 bulk + FP64 polish)."""
    s = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH, grid_mirror=mirror, bb=bb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = abip.abip_setup(A, b, c, s)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    tune = abip.abip_autotune(w, 30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, y, sv, info = abip.abip_solve(w)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    xh, yh, sh = _host((x, y, sv))
    kkt = host_kkt(lp["A"], lp["b"], lp["c"], xh, yh, sh)
    w.free()
    return info, setup_ms, solve_s, tune, kkt, xh


def extra_basis_pursuit(abip, torch, cpu=True):
    """Basis pursuit LP, A = [A0, -A0] with A0 2000 x 8000 Gaussian/sqrt(2000), 5% sparse x_true,
    seed 2: one LP on the whole GPU (grid engine), FP32 bulk + FP64 polish.  The main figures
    stream every column (settings.grid_mirror = 0); `paired_columns` is the same solve with the
    column pass reading A0 alone (the library's default for such data), reported separately."""
    import lpgen
    lp = lpgen.basis_pursuit(2000, 8000, 400, 2)
    A = torch.tensor(lp["A"], device="cuda")
    b = torch.tensor(lp["b"], device="cuda")
    c = torch.tensor(lp["c"], device="cuda")
    m, n = 2000, 16000
    log("basis pursuit 2000 x 16000: every column streamed")
    info, setup_ms, solve_s, tune, kkt, xh = _bp_solve(abip, torch, lp, A, b, c, 0)
    it32 = info["admm_iters"] - info["admm_iters_fp64"]
    it64 = info["admm_iters_fp64"]
    survey = it32 * survey_bytes_per_update(m, n, 4) + it64 * survey_bytes_per_update(m, n, 8)
    # this design: A once per pass, G^{-1} once per update, 8 doubles per column
    design = info["colpass_fp32"] * (4.0 * m * n + 64.0 * n) + info["colpass_fp64"] * (8.0 * m * n + 64.0 * n) \
        + it32 * 4.0 * m * m + it64 * 8.0 * m * m
    ks = info["kernel_ms"] / 1e3
    out = {"workload": "basis pursuit LP 2000 x 16000 (A = [A0, -A0]), seed 2, eps 1e-6, fp32 bulk + fp64 polish",
           "status": info["status_name"], "admm_iters": info["admm_iters"], "admm_iters_fp64": it64,
           "setup_ms": setup_ms, "solve_s": solve_s, "admm_iters_per_s": info["admm_iters"] / solve_s,
           "us_per_iter": info["kernel_ms"] * 1e3 / max(1, info["admm_iters"]),
           "host_kkt": list(kkt), "err_vs_fp64": info["err_vs_fp64"], "fp32_exit_kkt": info["fp32_exit_kkt"],
           "pobj": float(lp["c"] @ xh), "pstar": lp["pstar"],
           "obj_vs_planted": abs(float(lp["c"] @ xh) - lp["pstar"]) / (1 + lp["pstar"]),
           "grid_mirror": info["grid_mirror"], "autotune": tune,
           "roofline": {"bound": "hbm", "achieved": survey / ks / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": survey / ks / 1e9 / HBM_PEAK_GBS,
                        "frac_design_bytes": design / ks / 1e9 / HBM_PEAK_GBS,
                        "bytes_per_update_survey": survey_bytes_per_update(m, n, 4),
                        "kernel": "grid engine (column pass + reduction + G^-1 slice)"}}
    log("basis pursuit 2000 x 16000: paired columns (A0 read once per pass)")
    pinfo, psetup, psolve, ptune, pkkt, pxh = _bp_solve(abip, torch, lp, A, b, c, 1)
    pit32 = pinfo["admm_iters"] - pinfo["admm_iters_fp64"]
    pit64 = pinfo["admm_iters_fp64"]
    pdesign = pinfo["colpass_fp32"] * (2.0 * m * n + 64.0 * n) + pinfo["colpass_fp64"] * (4.0 * m * n + 64.0 * n) \
        + pit32 * 4.0 * m * m + pit64 * 8.0 * m * m
    pks = pinfo["kernel_ms"] / 1e3
    out["paired_columns"] = {
        "grid_mirror": pinfo["grid_mirror"], "status": pinfo["status_name"], "admm_iters": pinfo["admm_iters"],
        "admm_iters_fp64": pit64, "setup_ms": psetup, "solve_s": psolve,
        "admm_iters_per_s": pinfo["admm_iters"] / psolve,
        "us_per_iter": pinfo["kernel_ms"] * 1e3 / max(1, pinfo["admm_iters"]),
        "host_kkt": list(pkkt), "err_vs_fp64": pinfo["err_vs_fp64"],
        "obj_vs_planted": abs(float(lp["c"] @ pxh) - lp["pstar"]) / (1 + lp["pstar"]),
        "autotune": ptune,
        "design_bytes_per_update_fp32": 2.0 * m * n + 64.0 * n + 4.0 * m * m,
        "frac_design_bytes": pdesign / pks / 1e9 / HBM_PEAK_GBS,
        "speedup_per_update": (info["kernel_ms"] / max(1, info["admm_iters"]))
                              / (pinfo["kernel_ms"] / max(1, pinfo["admm_iters"])),
        "note": "A0 (2000 x 8000) is read once per column pass instead of A (2000 x 16000); the method's "
                "byte count of the main line does not apply"}
    log("basis pursuit 2000 x 16000: paired columns, adaptive beta")
    binfo, _, bsolve, _, bkkt, bxh = _bp_solve(abip, torch, lp, A, b, c, 1, bb=1)
    out["paired_columns_adaptive_beta"] = {
        "status": binfo["status_name"], "admm_iters": binfo["admm_iters"],
        "bb_probe_iters": binfo["bb_probe_iters"], "bb_estimates": binfo["bb_estimates"], "beta": binfo["beta"],
        "solve_s": bsolve, "us_per_iter": binfo["kernel_ms"] * 1e3 / max(1, binfo["admm_iters"]),
        "host_kkt": list(bkkt), "obj_vs_planted": abs(float(lp["c"] @ bxh) - lp["pstar"]) / (1 + lp["pstar"]),
        "note": "each step of a beta choice runs in workgroup 0 of the G^-1 kernel of the pass that reaches it"}
    if cpu:
        import oracle
        out["cpu_baseline"] = {
            "kind": "oracle", "what": "dense Schur solve (Cholesky of G), 40 iterations timed, scaled to the "
                                      "GPU's iteration count",
            "runs": [cpu_time_single(lp["A"], lp["b"], lp["c"], info["admm_iters"], 40, oracle.SchurIQSolver, t)
                     for t in (1, host_info()[1])]}
    return out


def extra_sparse(abip, torch, cpu=True):
    """Sparse NETLIB-sized LP 10000 x 30000, ~0.1% U(-1,1) plus a diagonal block, seed 1, CG path, FP64."""
    import lpgen
    import scipy.sparse as sp
    lp = lpgen.sparse_planted(10000, 30000, 1, density=1e-3)
    A = lp["A_csr"]
    As = sp.csr_matrix((A["data"], A["indices"], A["indptr"]), shape=A["shape"])
    s = abip.abip_default_settings()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = abip.abip_setup(As, lp["b"], lp["c"], s)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    x, y, sv, info = abip.abip_solve(w)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    xh, yh, sh = _host((x, y, sv))
    kkt = host_kkt(As, lp["b"], lp["c"], xh, yh, sh)
    it = max(1, info["admm_iters"])
    w.free()
    m, n, nnz = 10000, 30000, lp["nnz"]
    gnnz = info["gram_nnz"]
    if gnnz > 0:
        # algorithmic bytes of one CG iteration with the explicit G~ = A A^T: its CSR rows once
        # (8-byte value + 4-byte index per entry, 4-byte row pointers), the 32-byte record of
        # every row read (the gathers) and written, and p, a, u read and written (48 bytes per row)
        cg_bytes = 12.0 * gnnz + 4.0 * (m + 1) + 32.0 * m + 32.0 * m + 48.0 * m
        count = "12 nnz(G~) + 4 (m + 1) + 112 m"
    else:
        # with the two products: CSR(A^T) and CSR(A) once each (8-byte value + 4-byte index per
        # entry, 4-byte row pointers), the 32-byte CG record of every row read by the column pass,
        # q1 written and read (8 bytes per column), and the row update's reads and writes of r,
        # G u, G p (record) and p, a, u (56 + 32 bytes per row)
        cg_bytes = 24.0 * nnz + 4.0 * (m + n + 2) + 32.0 * m + 16.0 * n + 88.0 * m
        count = "24 nnz(A) + 4 (m + n + 2) + 120 m + 16 n"
    us_cg = info["kernel_ms"] * 1e3 / max(1, info["cg_iters"])
    achieved = cg_bytes / (us_cg * 1e-6) / 1e9
    # the same solve with the explicit G~ = A A^T (one product, one barrier per CG iteration)
    w2 = abip.abip_setup(As, lp["b"], lp["c"], abip.abip_default_settings(sparse_gram=1))
    _, _, _, info2 = abip.abip_solve(w2)
    w2.free()
    two = {"gram_nnz": info2["gram_nnz"], "admm_iters": info2["admm_iters"], "cg_iters": info2["cg_iters"],
           "us_per_iter": info2["kernel_ms"] * 1e3 / max(1, info2["admm_iters"]),
           "us_per_cg_iter": info2["kernel_ms"] * 1e3 / max(1, info2["cg_iters"]), "status": info2["status_name"]}
    out = {"workload": "sparse planted LP 10000 x 30000, nnz %d, seed 1, eps 1e-6, CG on I + A A^T, fp64" % nnz,
           "status": info["status_name"], "admm_iters": info["admm_iters"], "cg_iters": info["cg_iters"],
           "setup_ms": setup_ms, "solve_s": solve_s, "admm_iters_per_s": info["admm_iters"] / solve_s,
           "us_per_iter": info["kernel_ms"] * 1e3 / it, "us_per_cg_iter": us_cg,
           "barrier_ticks_share": info["ticks_check"] / max(1, info["ticks_total"]),
           "host_kkt": list(kkt), "err_vs_fp64": info["err_vs_fp64"], "pobj": float(lp["c"] @ xh),
           "pstar": lp["pstar"], "gram_nnz": gnnz, "explicit_gram_per_cg_iteration": two,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "kernel": "k_sp_solve (per CG iteration)",
                        "algorithmic_bytes_per_cg_iteration": cg_bytes, "count": count,
                        "note": "bound in practice by the grid barriers of each CG iteration, not by HBM"}}
    if cpu:
        import oracle
        out["cpu_baseline"] = {
            "kind": "oracle", "what": "CG step of Section 4.4 on scipy.sparse A (Jacobi, warm start, tol 1e-7), "
                                      "30 iterations timed, scaled to the GPU's iteration count",
            "runs": [cpu_time_single(As, lp["b"], lp["c"], info["admm_iters"], 30,
                                     lambda p: oracle.CGIQSolver(p, tol=1e-7), t) for t in (1, host_info()[1])]}
    return out


def extra_differentiable(abip, torch, cpu=True):
    """64 LPs 200 x 500, seed 4, FP32 forward; adjoint backward of L = w^T x* per LP,
    checked against the LP derivative of the planted basis (dL/db = A_B^{-T} w_B,
    dL/dc = 0), which is what central differences of the basis solution map give."""
    import lpgen
    lps = lpgen.diff_batch(64, 200, 500, 4)
    As = [torch.tensor(lp["A"], device="cuda") for lp in lps]
    bs = [torch.tensor(lp["b"], device="cuda") for lp in lps]
    cs = [torch.tensor(lp["c"], device="cuda") for lp in lps]
    ws = [torch.tensor(lp["w"], device="cuda") for lp in lps]
    s = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = abip.abip_setup_batch(As, bs, cs, s)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    dcs, dbs, _ = abip.abip_backward_batch(w, ws)
    torch.cuda.synchronize()
    bwd = time.perf_counter() - t0
    ok = sum(1 for i in infos if i["status"] == abip.ABIP_SOLVED)
    eb, ec = [], []
    dch, dbh = _host(dcs), _host(dbs)
    for lp, dc, db in zip(lps, dch, dbh):
        B = lp["basis"]
        lam = np.linalg.solve(lp["A"][:, B].T, lp["w"][B])
        eb.append(float(np.linalg.norm(db - lam) / np.linalg.norm(lam)))
        ec.append(float(np.linalg.norm(dc) / np.linalg.norm(lp["w"])))
    adj = [abip.abip_backward_stats(w, k) for k in range(len(lps))]
    # the final iterates of the LPs furthest from and nearest to the basis formula, for the host check
    order = np.argsort(ec)
    probe = [int(order[-1]), int(order[len(order) // 2])]
    states = {k: [t.cpu().numpy() if hasattr(t, "cpu") else t for t in abip.abip_get_state(w, k)] for k in probe}
    w.free()
    out = {"workload": "64 LPs 200 x 500, seed 4, L = w^T x*, fp32 bulk + fp64 polish forward, adjoint backward",
           "solved": ok, "forward_s": fwd, "backward_s": bwd, "backward_over_forward": bwd / fwd,
           "adjoint_iters": _stats([a[0] for a in adj]), "adjoint_rel_resid": _stats([a[1] for a in adj]),
           "db_rel_err_vs_basis_formula": _stats(eb), "dc_norm_over_w_norm": _stats(ec),
           "note": "the adjoint differentiates the central point at the final mu (checked against the dense "
                   "KKT adjoint at the same iterate in cpu_baseline); its distance to the LP derivative of the "
                   "basis shrinks with mu and grows as the vertex nears degeneracy (small reduced costs)"}
    if cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        runs = []
        for threads in (1, host_info()[1]):
            with threadpool_limits(limits=threads):
                t0 = time.perf_counter()
                for lp in lps[:2]:
                    ref = oracle.solve(lp["A"], lp["b"], lp["c"])
                    lam = oracle.kkt_adjoint(lp["A"], lp["b"], lp["c"], ref["state"], lp["w"])
                    oracle.contract_adjoint(lp["A"], lp["b"], lp["c"], ref["state"], lam)
                per = (time.perf_counter() - t0) / 2
            runs.append({"threads": threads, "s_per_lp_forward_backward": per,
                         "batch_s_estimated": per * len(lps)})
        # the GPU gradients against the oracle's dense KKT adjoint at the GPU's own final iterate
        checks = []
        for k in probe:
            y, x, s_, sc = states[k]
            lp = lps[k]
            st = oracle.State(y, x, sc["tau"], sc["theta"], s_, sc["kappa"], sc["mu"])
            lam = oracle.kkt_adjoint(lp["A"], lp["b"], lp["c"], st, lp["w"])
            ref = oracle.contract_adjoint(lp["A"], lp["b"], lp["c"], st, lam)
            checks.append({"lp": k, "dc_rel_err": float(np.linalg.norm(dch[k] - ref["dc"]) / np.linalg.norm(ref["dc"])),
                           "db_rel_err": float(np.linalg.norm(dbh[k] - ref["db"]) / np.linalg.norm(ref["db"]))})
        out["cpu_baseline"] = {"kind": "oracle", "what": "oracle solve + dense KKT adjoint, 2 LPs timed, "
                                                         "scaled to 64", "runs": runs,
                               "gpu_vs_kkt_adjoint_at_gpu_iterate": checks}
    return out


def extra_paper_random(abip, torch, cpu=True):
    """The paper's random-LP recipe (lpgen.paper_random, seed 1) at every Table 1
    size and its tolerance 1e-3: one LP on the whole GPU (grid engine).  Two runs
    per size: FP64 after 10 rounds of Ruiz equilibration (the scaling of Section
    4.5's remark; the KKT is rechecked on the LP as given), and FP32 bulk + FP64
    polish without scaling, capped at 20000 updates.  The paper's own ABIP times
    (a laptop CPU, other instances drawn from the same recipe) are context, not a
    target."""
    import lpgen
    paper_s = {(500, 5000): 10.6, (500, 10000): 25.7, (500, 20000): 61.6, (1000, 5000): 39.9,
               (1000, 10000): 56.0, (1000, 20000): 122.0, (2000, 10000): 889.0, (2000, 20000): 4040.0,
               (4000, 20000): 5670.0}
    runs = (("fp64_scaled", dict(precision=abip.ABIP_PREC_FP64, scale_iters=10)),
            ("fp32_bulk_unscaled", dict(precision=abip.ABIP_PREC_FP32_POLISH, max_admm_iters=20000)))
    out = []
    for (m, n), ps in paper_s.items():
        log(f"paper random LP {m} x {n}")
        lp = lpgen.paper_random(m, n, 1)
        A = torch.tensor(lp["A"], device="cuda")
        b = torch.tensor(lp["b"], device="cuda")
        c = torch.tensor(lp["c"], device="cuda")
        row = {"m": m, "n": n, "pstar": lp["pstar"], "paper_abip_s_laptop_cpu": ps}
        for label, kw in runs:
            torch.cuda.synchronize()
            s = abip.abip_default_settings(eps=1e-3, engine=abip.ABIP_ENGINE_GRID, **kw)
            t0 = time.perf_counter()
            w = abip.abip_setup(A, b, c, s)
            x, y, sv, info = abip.abip_solve(w)
            torch.cuda.synchronize()
            total_s = time.perf_counter() - t0
            xh, yh, sh = _host((x, y, sv))
            w.free()
            row[label] = {"status": info["status_name"], "admm_iters": info["admm_iters"],
                          "setup_plus_solve_s": total_s, "solve_kernel_s": info["kernel_ms"] / 1e3,
                          "host_kkt": list(host_kkt(lp["A"], lp["b"], lp["c"], xh, yh, sh)),
                          "err_vs_fp64": info["err_vs_fp64"], "pobj": float(lp["c"] @ xh)}
        out.append(row)
    return {"workload": "paper's random-LP recipe, seed 1, eps 1e-3, grid engine: FP64 with Ruiz scaling, "
                        "and FP32 bulk + FP64 polish unscaled (20000-update cap)",
            "instances": out}


def extra_sice(abip, torch, d=64, N=1000, cpu=True):
    """Sparse inverse covariance estimation (lpgen.sice: synthetic Sigma, d
    variables, N samples, lambda = 1.5 sqrt(log d / N)): the d column LPs
    (2d x 4d each) in one batched launch, FP32 bulk + FP64 polish."""
    import lpgen
    S = lpgen.sice(d, N, 1)
    A = torch.tensor(S["A"], device="cuda")
    c = torch.tensor(S["c"], device="cuda")
    bs = [torch.tensor(b, device="cuda") for b in S["bs"]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w = abip.abip_setup_batch([A] * d, bs, [c] * d, abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH))
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    X = torch.stack(xs).cpu().numpy()
    B = X[:, :d] - X[:, d:2 * d]
    viol = float(np.abs(S["Sigma"] @ B.T - np.eye(d)).max() / S["lam"])
    its = [i["admm_iters"] for i in infos]
    st = np.bincount([i["status"] for i in infos], minlength=5).tolist()
    w.free()
    return {"workload": f"SICE d={d} (N={N} samples, lambda={S['lam']:.4f}): {d} LPs of {2 * d} x {4 * d}, "
                        "one batched launch, fp32 bulk + fp64 polish, eps 1e-6",
            "statuses": st, "setup_plus_solve_s": total_s, "solve_kernel_s": infos[0]["kernel_ms"] / 1e3,
            "admm_iters_mean": float(np.mean(its)), "admm_iters_max": int(np.max(its)),
            "err_vs_fp64": _stats([i["err_vs_fp64"] for i in infos]),
            "max_constraint_over_lambda": viol, "l1_norm_of_omega": float(np.abs(B).sum())}


def extra_trsv(abip, torch, cpu=True):
    """The linear step by triangular solves with the cached factor L (ABIP_LIN_TRSV)
    against the product with the cached G^{-1} (the default), streamed one-workgroup
    engine, FP64, on dense planted LPs of growing m: time per update and the
    iteration count of the same solve (capped at 3000 updates)."""
    import lpgen
    rows = []
    for m in (100, 200, 400, 700, 1000):
        lp = lpgen.dense_planted(m, int(2.2 * m), 40 + m)
        row = {"m": m, "n": int(2.2 * m)}
        for key, lin in (("inverse", abip.ABIP_LIN_AUTO), ("trsv", abip.ABIP_LIN_TRSV)):
            st = abip.abip_default_settings(lin_solver=lin, lds_resident=0, max_admm_iters=3000)
            w = abip.abip_setup(lp["A"], lp["b"], lp["c"], st)
            x, y, sv, info = abip.abip_solve(w)
            w.free()
            it = max(1, info["admm_iters"])
            row[key] = {"us_per_update": info["kernel_ms"] * 1e3 / it, "admm_iters": info["admm_iters"],
                        "status": info["status_name"]}
        row["trsv_over_inverse"] = row["trsv"]["us_per_update"] / row["inverse"]["us_per_update"]
        rows.append(row)
    return {"workload": "dense planted LPs m = 100 ... 1000, n = 2.2 m, FP64, streamed, one workgroup per LP, "
                        "3000-update cap", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baselines")
    ap.add_argument("--plain-sample", type=int, default=48,
                    help="time the plain FP64 path on this many LPs stratified by m n, plus the two "
                         "slowest (0: all LPs of the batch)")
    ap.add_argument("--per-lp-out", default=None, help="write the per-LP table (TSV) to this file")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra measurements (basis pursuit, sparse CG, differentiable batch, "
                         "the paper's random LPs, SICE, triangular solves vs the inverse)")
    ap.add_argument("--extra-only", default=None,
                    choices=["basis_pursuit", "sparse_cg", "differentiable", "paper_random", "sice", "trsv"],
                    help="run one extra measurement alone, print its JSON object and exit (for profiling)")
    ap.add_argument("--bb", type=int, default=1, choices=[0, 1],
                    help="1 (default): the adaptive beta of Section 4.3 in every solve of the headline, "
                         "its FP64 comparisons and the oracle baseline; 0: beta fixed at settings.beta")
    ap.add_argument("--tune-iters", type=int, default=200,
                    help="updates per autotuner candidate on the batch handle (0: no tuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy (PMC byte-counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the batch would shard "
              f"LP-by-LP across GPUs, which this library does not implement.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1805_12344_amd as abip

    torch.cuda.set_device(0)
    extras = {"trsv": extra_trsv, "basis_pursuit": extra_basis_pursuit, "sparse_cg": extra_sparse,
              "differentiable": extra_differentiable, "paper_random": extra_paper_random, "sice": extra_sice}
    if args.extra_only:
        print(json.dumps({args.extra_only: extras[args.extra_only](abip, torch, cpu=False)}), flush=True)
        return
    lps = make_workload(args.batch, args.seed)
    As, bs, cs = to_device(lps)
    BB_MODE[0] = args.bb
    s32 = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH, bb=args.bb)
    log(f"workload: {len(lps)} LPs, sum m*n = {sum(lp['m'] * lp['n'] for lp in lps):.3e}")

    # one handle for every step: its buffers are allocated once, each step loads the
    # batch into them (the whole setup: copies, the factorization, the border) and
    # solves it, so the batched launch's captured graph is replayed from the second
    # step on
    t0 = time.perf_counter()
    wb = abip.abip_setup_batch(As, bs, cs, s32)
    torch.cuda.synchronize()
    log(f"handle + first setup: {time.perf_counter() - t0:.2f} s")
    tune = None
    if args.tune_iters > 0:
        t0 = time.perf_counter()
        r = abip.abip_autotune(wb, args.tune_iters)
        labels = ["LDS: A and G^-1, else A alone", "LDS: A and G^-1 only", "all streamed"]
        if all(lp["m"] <= 256 for lp in lps):
            labels.append("512 threads, streamed")
        labels.append("per-LP mix of resident and streamed")
        tune = {"iters_per_candidate": args.tune_iters,
                "score": "sum over LPs of each LP's own device-clock time for the candidate's run, ms",
                "candidates": [{"config": labels[i], "score_ms": r["ms"][i]} for i in range(len(r["ms"]))],
                "chosen": labels[r["chosen"]], "seconds": time.perf_counter() - t0}
        log(f"autotune: {tune}")

    def step():
        abip.abip_update_data(wb, As, bs, cs)
        return abip.abip_solve_batch(wb)

    for i in range(args.warmup):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.2f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} step(s): {elapsed:.2f} s")

    xs, ys, ss, infos = results[-1]
    r32 = (_host(xs), _host(ys), _host(ss), infos)
    ok, worst, kkt32 = verify(lps, *r32)
    solves_per_s = ok * args.steps / elapsed
    iters = np.array([i["admm_iters"] for i in infos])
    kernel_ms = infos[0]["kernel_ms"]
    admm_per_s = float(iters.sum()) / (kernel_ms / 1e3)
    survey_b, hbm_b, passes = launch_bytes(lps, infos)
    ks = kernel_ms / 1e3
    statuses = np.bincount([i["status"] for i in infos], minlength=5).tolist()
    tail = sorted(range(len(lps)), key=lambda k: -infos[k]["ticks_total"])[:4]
    line = {
        "metric": "ADMM iters/s and LP solves/s at 1e-6 rel KKT; FP32-batched vs FP64 plain",
        "value": solves_per_s,
        "unit": "LP solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 arithmetic on f32-stored A and G^-1, f64 polish",
        "data": "synthetic",
        "config": {"workload": f"batched dense LPs: {len(lps)} LPs, m~U[20,400], n~U[2m,3m], 10% "
                               f"primal infeasible, seed {args.seed}; eps 1e-6",
                   "global_batch": len(lps), "precision": "fp32 bulk + fp64 polish",
                   "beta": "adaptive (Section 4.3)" if args.bb else "fixed (settings.beta = 1)",
                   "engine": "one workgroup per LP, persistent, largest first; one handle reloaded "
                             "per step (abip_update_data), graph replayed"},
        "autotune": tune,
        "admm_iters_per_s": admm_per_s,
        "admm_iters_total": int(iters.sum()),
        "admm_iters_fp64_total": int(sum(i["admm_iters_fp64"] for i in infos)),
        "correct": ok,
        "statuses": statuses,
        "worst_kkt": worst,
        "solve_kernel_ms": kernel_ms,
        "setup_plus_solve_ms": elapsed / args.steps * 1e3,
        "makespan_lps": [{"lp": k, "m": lps[k]["m"], "n": lps[k]["n"], "iters": infos[k]["admm_iters"],
                          "status": infos[k]["status_name"], "lds_mode": infos[k]["lds_mode"],
                          "ms": infos[k]["ticks_total"] / 1e5,
                          "us_per_update": infos[k]["ticks_total"] / 100.0 / max(1, infos[k]["admm_iters"])}
                         for k in tail],
        "roofline": {"bound": "hbm", "achieved": survey_b / ks / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": survey_b / ks / 1e9 / HBM_PEAK_GBS, "traffic": traffic_bytes(),
                     "kernel": "k_solve_wg (persistent batched solve)", "kernel_src": kernel_hash(),
                     "algorithmic_bytes_per_launch": survey_b,
                     "count": "per update 2 m n p + m^2 p + 80 (m + n) bytes (p = 4 FP32 / 8 FP64 data), "
                              "summed over every update of the launch",
                     "hbm_bytes_this_design": hbm_b,
                     "frac_hbm_bytes_this_design": hbm_b / ks / 1e9 / HBM_PEAK_GBS,
                     "passes": passes,
                     "note": "most updates of the batch read A (and G^-1) from LDS; the launch lasts as long "
                             "as its slowest LP (makespan_lps), which runs alone on one CU, so the kernel is "
                             "bound by that LP's per-update latency, not by HBM"},
    }

    r64 = None
    if not args.no_compare:
        s64 = abip.abip_default_settings(precision=abip.ABIP_PREC_FP64, bb=args.bb)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs64, ys64, ss64, infos64 = run_batch(abip, As, bs, cs, s64)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t1
        r64 = (_host(xs64), _host(ys64), _host(ss64), infos64)
        log(f"fp64 batched: {e64:.2f} s")
        ok64, worst64, _ = verify(lps, *r64)
        it64 = np.array([i["admm_iters"] for i in infos64])
        line["fp64_batched"] = {"solves_per_s": ok64 / e64, "ms": e64 * 1e3, "correct": ok64,
                                "admm_iters_per_s": float(it64.sum()) / (infos64[0]["kernel_ms"] / 1e3),
                                "admm_iters_total": int(it64.sum()), "worst_kkt": worst64}
        line["speedup_vs_fp64_batched"] = solves_per_s / max(1e-12, ok64 / e64)
        line["fp32_error"] = error_report(lps, r32, r64)
        # the plain FP64 path: one LP per setup/solve call, sequentially; with
        # --plain-sample N, N LPs stratified by m n plus the two with the most FP64
        # iterations, each timed alone, and the batch's sequential time estimated
        # as the slow two plus the rest scaled to the other LPs
        idx = list(range(len(lps)))
        slow = set()
        if args.plain_sample and args.plain_sample < len(lps):
            order = np.argsort([lp["m"] * lp["n"] for lp in lps])
            slow = {int(k) for k in np.argsort(it64)[-2:]}
            strat = {int(order[i]) for i in np.linspace(0, len(lps) - 1, args.plain_sample).round().astype(int)}
            idx = sorted(slow | strat)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        okp = 0
        t_slow = t_rest = 0.0
        for q, k in enumerate(idx):
            tk = time.perf_counter()
            w = abip.abip_setup(As[k], bs[k], cs[k], s64)
            x, y, s_, info = abip.abip_solve(w)
            w.free()
            okp += verify([lps[k]], [x.cpu().numpy()], [y.cpu().numpy()], [s_.cpu().numpy()], [info])[0]
            tk = time.perf_counter() - tk
            if k in slow:
                t_slow += tk
            else:
                t_rest += tk
            if (q + 1) % 32 == 0:
                log(f"fp64 plain: {q + 1}/{len(idx)} LPs, {time.perf_counter() - t2:.1f} s")
        torch.cuda.synchronize()
        ep = time.perf_counter() - t2
        if len(idx) == len(lps):
            est, rate = ep, okp / ep
        else:
            est = t_slow + t_rest * (len(lps) - len(slow)) / max(1, len(idx) - len(slow))
            rate = len(lps) * (okp / len(idx)) / est
        line["fp64_plain_sequential"] = {
            "solves_per_s": rate, "lps": len(idx), "correct": okp, "ms": ep * 1e3,
            "batch_seconds": est,
            "sample": None if len(idx) == len(lps) else
            f"{len(idx)} LPs (indices {idx}): {args.plain_sample} stratified by m n plus the two with the most "
            f"FP64 iterations ({sorted(slow)}); the batch's sequential time is those two plus the others "
            f"scaled by {len(lps) - len(slow)}/{len(idx) - len(slow)}"}
        line["speedup_vs_fp64_plain"] = solves_per_s / max(1e-12, rate)
        iters64 = it64
    else:
        iters64 = iters

    if args.per_lp_out:
        rows = per_lp_rows(lps, infos, r64[3] if r64 else [None] * len(lps), kkt32)
        with open(args.per_lp_out, "w") as fh:
            fh.write("# per-LP counters of the timed FP32-bulk batched solve (bench.py --per-lp-out)\n")
            fh.write("\t".join(PER_LP_HEADER) + "\n")
            for r in rows:
                fh.write("\t".join(f"{v:.6g}" if isinstance(v, float) else str(v) for v in r) + "\n")
        line["per_lp_table"] = args.per_lp_out

    if not args.no_extra:
        for key, fn in extras.items():
            t0 = time.perf_counter()
            line[key] = fn(abip, torch, cpu=not args.no_cpu)
            log(f"{key}: {time.perf_counter() - t0:.1f} s")

    if not args.no_cpu:
        t0 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(lps, iters64, ok, bb=bool(args.bb))
        log(f"cpu_baseline: {time.perf_counter() - t0:.1f} s")

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
