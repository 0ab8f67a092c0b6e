#!/usr/bin/env python3
"""ABIP throughput on one MI355X: many uneven dense LPs solved to 1e-6 relative KKT.

Workload (one "step"): 256 dense random LPs, m ~ U{20..400}, n ~ U{2m..3m},
planted strictly complementary optima, 10% made primal infeasible by a planted
Farkas vector (seed 3).  A step is the whole hot path for the batch: setup
(HSD constants, FP64 SYRK + Cholesky + inverse of I + A A^T, Schur border) and
the batched ABIP solve (FP32-streamed bulk with FP64 checks and FP64 polish) in
one persistent launch, inputs already resident in HBM.

Printed: one JSON line.  value = LP solves/s (LPs ending with the right status,
solved ones re-checked in FP64 on the host at <= 1e-6 relative KKT) over the
end-to-end wall time of the timed steps.
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
    "20c6498551e51a87": {"fetch_kib": 1011746727.5, "write_kib": 19438547.3,
                         "fetch_scale": 1048576.0 / 524315.1, "write_scale": 1.0},
}
KERNEL_SOURCES = ["paper_1805_12344_amd/csrc/abip_solve_wg.hip", "paper_1805_12344_amd/csrc/abip_small.h",
                  "paper_1805_12344_amd/csrc/abip_internal.h"]


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


def verify(lps, xs, ys, ss, infos, eps=1e-6):
    """Host FP64 re-check: status right, and KKT <= eps for solved LPs."""
    ok = 0
    worst = 0.0
    for lp, x, y, s, info in zip(lps, xs, ys, ss, infos):
        if lp["status"] == "solved":
            if info["status"] != 1:
                continue
            A, b, c = lp["A"], lp["b"], lp["c"]
            x, y, s = x.cpu().numpy(), y.cpu().numpy(), s.cpu().numpy()
            pres = np.linalg.norm(A @ x - b) / (1 + np.linalg.norm(b))
            dres = np.linalg.norm(A.T @ y + s - c) / (1 + np.linalg.norm(c))
            pobj, dobj = c @ x, b @ y
            gap = abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj))
            kkt = max(pres, dres, gap)
            worst = max(worst, kkt)
            if kkt <= eps * (1 + 1e-9):
                ok += 1
        else:
            if info["status"] == 2:
                ok += 1
    return ok, worst


def algorithmic_bytes(lps, infos, fp32_stream=True):
    """Bytes the persistent solve launch must move, from its own pass counts.

    Per column pass over A: m*n matrix entries plus 8 doubles per column (x, s
    read and written, c, cbar, Z_x read); per inner update one pass over the
    m x m G^{-1}.  FP32-streamed passes count 4 bytes per matrix entry, FP64
    passes 8.
    """
    tot = 0.0
    for lp, info in zip(lps, infos):
        m, n = lp["m"], lp["n"]
        it64 = info["admm_iters_fp64"]
        it32 = info["admm_iters"] - it64
        tot += info["colpass_fp32"] * (4.0 * m * n + 64.0 * n)
        tot += info["colpass_fp64"] * (8.0 * m * n + 64.0 * n)
        tot += it32 * 4.0 * m * m + it64 * 8.0 * m * m
    return tot


def traffic_bytes():
    t = PMC_TRAFFIC.get(kernel_hash())
    if t is None:
        return None
    return t["fetch_kib"] * 1024.0 * t["fetch_scale"] + t["write_kib"] * 1024.0 * t["write_scale"]


def run_batch(abip, As, bs, cs, settings):
    w = abip.abip_setup_batch(As, bs, cs, settings)
    xs, ys, ss, infos = abip.abip_solve_batch(w)
    w.free()
    return xs, ys, ss, infos


def cpu_baseline(lps, gpu_iters, sample_idx, iters_each=12000):
    """Time the FP64 oracle (as it is) on a bounded sample of the same LPs.

    Each sampled LP runs `iters_each` oracle iterations; its per-iteration time
    times the LP's full iteration count (the same algorithm in FP64 stops at
    the same iteration as the FP64 GPU path) gives its solve time.
    """
    from threadpoolctl import threadpool_limits
    import oracle
    per_lp = []
    t_all = time.perf_counter()
    with threadpool_limits(limits=1):
        for k in sample_idx:
            lp = lps[k]
            s = oracle.Settings(max_admm_iters=iters_each)
            t0 = time.perf_counter()
            out = oracle.solve(lp["A"], lp["b"], lp["c"], s)
            dt = time.perf_counter() - t0
            done = max(1, out["admm_iters"])
            per_lp.append(dt / done * gpu_iters[k])
    wall = time.perf_counter() - t_all
    sec_per_solve = float(np.mean(per_lp))
    return {"value": 1.0 / sec_per_solve, "unit": "LP solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample_idx)} LPs of the batch (indices {list(sample_idx)}), {iters_each} "
                      f"oracle iterations each, per-iteration time x the LP's FP64 iteration count; "
                      f"{wall:.1f} s of CPU work"}


def extra_basis_pursuit(abip, torch):
    """Basis pursuit LP, A = [A0, -A0] with A0 2000 x 8000 Gaussian/sqrt(2000), 5% sparse x_true,
    seed 2: one LP on the whole GPU (grid engine), FP32 bulk + FP64 polish."""
    import lpgen
    lp = lpgen.basis_pursuit(2000, 8000, 400, 2)
    A = torch.tensor(lp["A"], device="cuda")
    b = torch.tensor(lp["b"], device="cuda")
    c = torch.tensor(lp["c"], device="cuda")
    torch.cuda.synchronize()
    s = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
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
    xh, yh, sh = x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy()
    pres = np.linalg.norm(lp["A"] @ xh - lp["b"]) / (1 + np.linalg.norm(lp["b"]))
    dres = np.linalg.norm(lp["A"].T @ yh + sh - lp["c"]) / (1 + np.linalg.norm(lp["c"]))
    po, do = float(lp["c"] @ xh), float(lp["b"] @ yh)
    gap = abs(po - do) / (1 + abs(po) + abs(do))
    m, n = 2000, 16000
    it32 = info["admm_iters"] - info["admm_iters_fp64"]
    it64 = info["admm_iters_fp64"]
    # per update: A once (m n) and G^{-1} once (m^2), plus 8 doubles per column
    byts = info["colpass_fp32"] * (4.0 * m * n + 64.0 * n) + info["colpass_fp64"] * (8.0 * m * n + 64.0 * n) \
        + it32 * 4.0 * m * m + it64 * 8.0 * m * m
    ach = byts / (info["kernel_ms"] / 1e3) / 1e9
    w.free()
    return {"workload": "basis pursuit LP 2000 x 16000 (A = [A0, -A0]), seed 2, eps 1e-6, fp32 bulk + fp64 polish",
            "status": info["status_name"], "admm_iters": info["admm_iters"], "admm_iters_fp64": it64,
            "setup_ms": setup_ms, "solve_s": solve_s, "admm_iters_per_s": info["admm_iters"] / solve_s,
            "us_per_iter": info["kernel_ms"] * 1e3 / max(1, info["admm_iters"]),
            "host_kkt": [pres, dres, gap], "pobj": po, "pstar": lp["pstar"],
            "autotune": tune, "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                           "frac": ach / HBM_PEAK_GBS, "kernel": "grid engine (col + G^-1 + reductions)"}}


def extra_sparse(abip, torch):
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
    xh, yh, sh = x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy()
    pres = np.linalg.norm(As @ xh - lp["b"]) / (1 + np.linalg.norm(lp["b"]))
    dres = np.linalg.norm(As.T @ yh + sh - lp["c"]) / (1 + np.linalg.norm(lp["c"]))
    po, do = float(lp["c"] @ xh), float(lp["b"] @ yh)
    gap = abs(po - do) / (1 + abs(po) + abs(do))
    it = max(1, info["admm_iters"])
    w.free()
    # algorithmic bytes of one CG iteration (the dominant work): CSR(A^T) and CSR(A) once each
    # (8-byte value + 4-byte index per entry, 4-byte row pointers), the 32-byte CG record of
    # every row read by the column pass, q1 written and read (8 bytes per column), and the
    # row update's reads and writes of r, G u, G p (record) and p, a, u (56 + 32 bytes per row)
    m, n, nnz = 10000, 30000, lp["nnz"]
    cg_bytes = 24.0 * nnz + 4.0 * (m + n + 2) + 32.0 * m + 16.0 * n + 88.0 * m
    us_cg = info["kernel_ms"] * 1e3 / max(1, info["cg_iters"])
    achieved = cg_bytes / (us_cg * 1e-6) / 1e9
    return {"workload": "sparse planted LP 10000 x 30000, nnz %d, seed 1, eps 1e-6, CG on I + A A^T, fp64" % lp["nnz"],
            "status": info["status_name"], "admm_iters": info["admm_iters"], "cg_iters": info["cg_iters"],
            "setup_ms": setup_ms, "solve_s": solve_s, "admm_iters_per_s": info["admm_iters"] / solve_s,
            "us_per_iter": info["kernel_ms"] * 1e3 / it, "us_per_cg_iter": info["kernel_ms"] * 1e3 / max(1, info["cg_iters"]),
            "host_kkt": [pres, dres, gap], "pobj": po, "pstar": lp["pstar"],
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "kernel": "k_sp_solve (per CG iteration)",
                         "algorithmic_bytes_per_cg_iteration": cg_bytes,
                         "note": "bound in practice by two grid barriers per CG iteration, not by HBM"}}


def extra_differentiable(abip, torch):
    """64 LPs 200 x 500, seed 4, FP32 forward; adjoint backward of L = w^T x* per LP."""
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
    finite = sum(1 for dc, db in zip(dcs, dbs) if bool(torch.isfinite(dc).all()) and bool(torch.isfinite(db).all()))
    w.free()
    return {"workload": "64 LPs 200 x 500, seed 4, L = w^T x*, fp32 bulk + fp64 polish forward, adjoint backward",
            "solved": ok, "finite_gradients": finite, "forward_s": fwd, "backward_s": bwd,
            "backward_over_forward": bwd / fwd}


def extra_paper_random(abip, torch):
    """The paper's random-LP recipe (lpgen.paper_random, seed 1) at three of its
    Table 1 sizes and its tolerance 1e-3: one LP on the whole GPU (grid engine),
    FP32 bulk + FP64 polish.  The paper's own ABIP times (a laptop CPU, other
    instances drawn from the same recipe) are context, not a target."""
    import lpgen
    paper_s = {(500, 5000): 10.6, (1000, 10000): 56.0, (2000, 10000): 889.0}
    out = []
    for (m, n), ps in paper_s.items():
        lp = lpgen.paper_random(m, n, 1)
        A = torch.tensor(lp["A"], device="cuda")
        b = torch.tensor(lp["b"], device="cuda")
        c = torch.tensor(lp["c"], device="cuda")
        torch.cuda.synchronize()
        s = abip.abip_default_settings(eps=1e-3, engine=abip.ABIP_ENGINE_GRID, precision=abip.ABIP_PREC_FP32_POLISH)
        t0 = time.perf_counter()
        w = abip.abip_setup(A, b, c, s)
        x, y, sv, info = abip.abip_solve(w)
        torch.cuda.synchronize()
        total_s = time.perf_counter() - t0
        xh, yh, sh = x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy()
        pres = np.linalg.norm(lp["A"] @ xh - lp["b"]) / (1 + np.linalg.norm(lp["b"]))
        dres = np.linalg.norm(lp["A"].T @ yh + sh - lp["c"]) / (1 + np.linalg.norm(lp["c"]))
        po, do = float(lp["c"] @ xh), float(lp["b"] @ yh)
        gap = abs(po - do) / (1 + abs(po) + abs(do))
        w.free()
        out.append({"m": m, "n": n, "status": info["status_name"], "admm_iters": info["admm_iters"],
                    "setup_plus_solve_s": total_s, "solve_kernel_s": info["kernel_ms"] / 1e3,
                    "host_kkt": [pres, dres, gap], "pobj": po, "pstar": lp["pstar"],
                    "paper_abip_s_laptop_cpu": ps})
    return {"workload": "paper's random-LP recipe, seed 1, eps 1e-3, fp32 bulk + fp64 polish, grid engine",
            "instances": out}


def extra_sice(abip, torch, d=64, N=1000):
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
            "max_constraint_over_lambda": viol, "l1_norm_of_omega": float(np.abs(B).sum())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra measurements (basis pursuit, sparse CG, differentiable batch, "
                         "the paper's random LPs, SICE)")
    ap.add_argument("--extra-only", default=None,
                    choices=["basis_pursuit", "sparse_cg", "differentiable", "paper_random", "sice"],
                    help="run one extra measurement alone, print its JSON object and exit (for profiling)")
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
    extras = {"basis_pursuit": extra_basis_pursuit, "sparse_cg": extra_sparse,
              "differentiable": extra_differentiable, "paper_random": extra_paper_random, "sice": extra_sice}
    if args.extra_only:
        print(json.dumps({args.extra_only: extras[args.extra_only](abip, torch)}), flush=True)
        return
    lps = make_workload(args.batch, args.seed)
    As, bs, cs = to_device(lps)
    s32 = abip.abip_default_settings(precision=abip.ABIP_PREC_FP32_POLISH)
    log(f"workload: {len(lps)} LPs, sum m*n = {sum(lp['m'] * lp['n'] for lp in lps):.3e}")

    for i in range(args.warmup):
        t0 = time.perf_counter()
        run_batch(abip, As, bs, cs, s32)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.2f} s")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(run_batch(abip, As, bs, cs, s32))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} step(s): {elapsed:.2f} s")

    xs, ys, ss, infos = results[-1]
    ok, worst = verify(lps, xs, ys, ss, infos)
    solves_per_s = ok * args.steps / elapsed
    iters = np.array([i["admm_iters"] for i in infos])
    kernel_ms = infos[0]["kernel_ms"]
    admm_per_s = float(iters.sum()) / (kernel_ms / 1e3)
    bytes_launch = algorithmic_bytes(lps, infos)
    achieved = bytes_launch / (kernel_ms / 1e3) / 1e9
    statuses = np.bincount([i["status"] for i in infos], minlength=5).tolist()
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
        "dtype": "f64 arithmetic on f32-streamed A and G^-1, f64 polish",
        "data": "synthetic",
        "config": {"workload": f"batched dense LPs: {len(lps)} LPs, m~U[20,400], n~U[2m,3m], 10% "
                               f"primal infeasible, seed {args.seed}; eps 1e-6",
                   "global_batch": len(lps), "precision": "fp32 bulk + fp64 polish",
                   "engine": "one workgroup per LP, persistent, largest first"},
        "admm_iters_per_s": admm_per_s,
        "admm_iters_total": int(iters.sum()),
        "admm_iters_fp64_total": int(sum(i["admm_iters_fp64"] for i in infos)),
        "correct": ok,
        "statuses": statuses,
        "worst_kkt": worst,
        "solve_kernel_ms": kernel_ms,
        "setup_plus_solve_ms": elapsed / args.steps * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(),
                     "kernel": "k_solve_wg (persistent batched solve)", "kernel_src": kernel_hash(),
                     "algorithmic_bytes_per_launch": bytes_launch},
    }

    if not args.no_compare:
        s64 = abip.abip_default_settings(precision=abip.ABIP_PREC_FP64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs64, ys64, ss64, infos64 = run_batch(abip, As, bs, cs, s64)
        torch.cuda.synchronize()
        e64 = time.perf_counter() - t1
        ok64, worst64 = verify(lps, xs64, ys64, ss64, infos64)
        it64 = np.array([i["admm_iters"] for i in infos64])
        line["fp64_batched"] = {"solves_per_s": ok64 / e64, "ms": e64 * 1e3, "correct": ok64,
                                "admm_iters_per_s": float(it64.sum()) / (infos64[0]["kernel_ms"] / 1e3),
                                "worst_kkt": worst64}
        # the plain FP64 path: one LP per setup/solve call, sequentially, on a sample
        rng = np.random.default_rng(0)
        sample = sorted(rng.choice(len(lps), size=8, replace=False).tolist())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        okp = 0
        for k in sample:
            w = abip.abip_setup(As[k], bs[k], cs[k], s64)
            x, y, s_, info = abip.abip_solve(w)
            w.free()
            okp += verify([lps[k]], [x], [y], [s_], [info])[0]
        torch.cuda.synchronize()
        ep = time.perf_counter() - t2
        line["fp64_plain_sequential"] = {"solves_per_s": okp / ep, "sample": sample, "correct": okp,
                                         "ms": ep * 1e3}
        line["speedup_vs_fp64_plain"] = solves_per_s / max(1e-12, okp / ep)
        gpu_iters64 = it64
    else:
        gpu_iters64 = iters

    if not args.no_extra:
        for key, fn in extras.items():
            t0 = time.perf_counter()
            line[key] = fn(abip, torch)
            log(f"{key}: {time.perf_counter() - t0:.1f} s")

    if not args.no_cpu:
        rng = np.random.default_rng(1)
        sample = sorted(rng.choice(len(lps), size=8, replace=False).tolist())
        line["cpu_baseline"] = cpu_baseline(lps, gpu_iters64, sample)

    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
