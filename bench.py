#!/usr/bin/env python3
"""Benchmark of the DLMPC-ADMM hot path on one MI355X.

A step is one MPC solve to eps (Algorithm 1 loop body: per-step precompute from x0, ADMM
iterations of Algorithm 2 until the convergence check passes, u(0) read from Phi) on the
1024-subsystem irregular mesh (32x32 grid, 30% of edges dropped, 51 chords; d = 3, T = 15,
|theta| <= 0.8, |u| <= 2), each step with its own seeded x0 already resident in HBM.

Prints one JSON line: value = ADMM iterations per second over the timed steps (whole job),
time-to-eps per solve, the same for the plain FP64 cold-start GPU solve, the roofline of the
dominant kernel, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2103_14990_amd", "csrc", "admm_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes(info: dict, rs: int, n_sub: int, elem: int) -> dict:
    """Bytes each kernel must move per launch (see the design notes), s = element size.

    Null bases are counted once per kernel that applies them (sum_j D_col(j) k_j entries).
    phi_kernel: Psi, Lambda read, Phi written (3 nnz), w/lb/ub read and y written (4 R).
    psi_pass1_kernel: N_j once, Phi and Lambda read (2 nnz).
    psi_pass2_kernel: N_j once, o_c, Phi, Lambda, Psi read, Psi and Lambda written (6 nnz).
    iteration: the minimum for one ADMM iteration, N_j read once (sum_dcol_k + 9 nnz + 4 R).
    """
    nnz, R, dk = info["nnz"], n_sub * rs, info["sum_dcol_k"]
    return {"phi_kernel": elem * (3 * nnz + 4 * R),
            "psi_pass1_kernel": elem * (dk + 2 * nnz),
            "psi_pass2_kernel": elem * (dk + 6 * nnz),
            "conv_kernel": 0,
            "iteration": elem * (dk + 9 * nnz + 4 * R)}


def cpu_baseline(wl, iters_gpu_mean: float, sample_blocks: int = 16) -> dict:
    """The FP64 oracle as it stands, timed on a bounded sample: Phi-comp, Lambda-comp and the
    convergence norms on the full problem, Psi-comp on `sample_blocks` seeded column blocks
    scaled to all N, one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dlmpc_oracle as O

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pb = O.setup_from_network(wl.net, wl.d, wl.T, wl.cost, blocks=False)
        Z = O.build_zab(pb.A, pb.B, pb.lay.T)
        rng = np.random.default_rng(0)
        js = sorted(rng.choice(wl.net.n_sub, sample_blocks, replace=False).tolist())
        t1 = time.perf_counter()
        pb.blocks = [O.column_block(Z, pb.mask, pb.lay, j) for j in js]
        t_fac = time.perf_counter() - t1
        x0 = wl.x0(1000)
        Psi = np.zeros(pb.mask.shape)
        Lam = np.zeros_like(Psi)
        t2 = time.perf_counter()
        Phi, _ = O.phi_comp(pb, Psi, Lam, x0, wl.rho)
        t3 = time.perf_counter()
        Psi_new = O.psi_comp(pb, Phi, Lam)
        t4 = time.perf_counter()
        Lam = O.lambda_comp(Lam, Phi, Psi_new)
        O.conv_residuals(Phi, Psi_new, Psi)
        t5 = time.perf_counter()
    n = wl.net.n_sub
    s_iter = (t3 - t2) + (t4 - t3) * n / sample_blocks + (t5 - t4)
    return {"value": 1.0 / s_iter, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"one ADMM iteration of the FP64 oracle: Phi-comp, Lambda-comp and "
                       f"Conv on all {n} subsystems, Psi-comp on {sample_blocks} seeded column "
                       f"blocks scaled x{n / sample_blocks:.0f}; setup factorisation of those "
                       f"blocks {t_fac:.1f} s (~{t_fac * n / sample_blocks:.0f} s for all)"),
            "time_to_eps_ms_est": 1e3 * s_iter * iters_gpu_mean,
            "wall_s": time.perf_counter() - t0}


def traffic_record(workload: str, kernel: str, launches_bytes: float):
    """HBM traffic of the dominant kernel from committed rocprofv3 counter runs, or None when
    the kernel source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def calibrate_copy(nbytes: int = 1 << 30) -> None:
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="irregular1024_box")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "graph", "persistent"])
    ap.add_argument("--ref-steps", type=int, default=5, help="steps of the plain FP64 solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        return 2
    if args.calibrate_copy:
        calibrate_copy()
        return 0

    import numpy as np
    import torch

    from paper_2103_14990_amd import dlmpc
    from paper_2103_14990_amd import workloads as W

    dev = torch.device("cuda:0")
    wl = W.workload(args.workload)
    net = wl.net
    n_x, n_u = net.n_sub * net.nx, net.n_sub * net.nu
    rs = net.nx * wl.T + net.nu * (wl.T - 1)
    stream = torch.cuda.current_stream(dev)

    def make(precision, schedule):
        t = time.perf_counter()
        p = dlmpc.Problem.from_network(net, wl.d, wl.T, wl.cost, rho=wl.rho, eps=wl.eps,
                                       max_iter=wl.max_iter, precision=precision, device=0,
                                       stream=stream.cuda_stream, schedule=schedule)
        log(f"setup {precision}/{schedule}: {time.perf_counter() - t:.1f} s, info {p.info}")
        return p

    n_steps = args.warmup + args.steps
    seeds = [1000 + i for i in range(n_steps)]
    x0 = torch.tensor(np.stack([wl.x0(s) for s in seeds]), dtype=torch.float64, device=dev)
    u0 = torch.zeros((n_steps, n_u), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()  # the library runs on its own stream

    def run(pr, idx):
        stats = []
        for i in idx:
            st, s = pr.solve_device(x0[i].data_ptr(), u0[i].data_ptr())
            s["status"] = st
            stats.append(s)
        return stats

    pr = make(args.precision, args.schedule)
    run(pr, range(args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = run(pr, range(args.warmup, n_steps))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = [s["iters"] for s in st]
    solve_ms = sorted(s["t_solve_ms"] for s in st)
    conv = sum(1 for s in st if s["status"] == dlmpc.OK)
    u0_main = u0[args.warmup:].cpu().numpy().copy()
    log(f"timed {args.steps} solves in {elapsed:.3f} s; iters {iters}; converged {conv}/{args.steps}; "
        f"host checks {[s['graph_launches'] for s in st]}")

    # Dominant kernel: the persistent kernel (one launch per solve), or the longest kernel of
    # the graph schedule's iteration, timed launch by launch with HIP events on the problem's
    # stream (every launch does work there; no early stop).
    elem = 4 if args.precision == "fp32" else 8
    ab = algorithmic_bytes(pr.info, rs, net.n_sub, elem)
    ku = pr.time_kernels(x0[args.warmup].data_ptr(), 50)
    if pr.info["schedule"] == 1:
        kname = "persistent_kernel"
        dur_s = sum(s["t_iter_ms"] for s in st) / 1e3
        bytes_total = sum(ab["iteration"] * s["iters"] for s in st)
        launch_bytes = bytes_total / len(st)
        avg_launch_us = 1e6 * dur_s / len(st)
    else:
        kname = max(ku, key=ku.get)
        launch_bytes = ab[kname]
        avg_launch_us = ku[kname]
        dur_s = avg_launch_us * 1e-6
        bytes_total = launch_bytes
    achieved = bytes_total / dur_s / 1e9
    per_kernel = {k: {"us": round(v, 2), "GB/s": round(ab[k] / (v * 1e-6) / 1e9, 1) if ab[k] else None}
                  for k, v in ku.items()}
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "avg_launch_us": round(avg_launch_us, 2),
                "algorithmic_bytes_per_launch": int(launch_bytes),
                "iteration_us": round(sum(ku.values()), 2),
                "iteration_algorithmic_bytes": int(ab["iteration"]),
                "per_kernel": per_kernel,
                "traffic": traffic_record(args.workload, kname, launch_bytes)}

    # Plain FP64 cold-start GPU solve on the same x0 (the reference the FP32 path is quoted against).
    ref = {}
    if args.ref_steps > 0 and args.precision != "fp64":
        prf = make("fp64", args.schedule)
        k = min(args.ref_steps, args.steps)
        run(prf, range(args.warmup, args.warmup + 1))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stf = run(prf, range(args.warmup, args.warmup + k))
        torch.cuda.synchronize()
        ef = time.perf_counter() - t1
        u0f = u0[args.warmup:args.warmup + k].cpu().numpy()
        rel = [float(np.abs(u0_main[i] - u0f[i]).max() / np.abs(u0f[i]).max()) for i in range(k)]
        ref = {"fp64_time_to_eps_ms_median": statistics.median(s["t_solve_ms"] for s in stf),
               "fp64_iter_per_s": sum(s["iters"] for s in stf) / ef,
               "fp64_iters": [s["iters"] for s in stf],
               "u0_rel_diff_vs_fp64_gpu_max": max(rel)}
        prf.close()

    out = {
        "metric": "time-to-ε (ms) per MPC solve + ADMM iter/s, 1024-node grid; warm/FP32 vs plain",
        "value": round(sum(iters) / elapsed, 1),
        "unit": "iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_sub": net.n_sub, "d": wl.d, "T": wl.T,
                   "rho": wl.rho, "eps": wl.eps, "max_iter": wl.max_iter, "x0_sigma": wl.sigma,
                   "x0_seeds": [seeds[args.warmup], seeds[-1]], "precision": args.precision,
                   "schedule": ["graph", "persistent"][pr.info["schedule"]],
                   "warm_start": "cold"},
        "time_to_eps_ms": {"median": round(statistics.median(solve_ms), 3),
                           "mean": round(statistics.mean(solve_ms), 3),
                           "std": round(statistics.pstdev(solve_ms), 3),
                           "p95": round(solve_ms[min(len(solve_ms) - 1, int(0.95 * len(solve_ms)))], 3)},
        "iters_mean": statistics.mean(iters), "converged": f"{conv}/{args.steps}",
        "setup_ms": round(pr.info["setup_ms"], 1),
        "tune_us_per_iter": {"graph": round(pr.info["tune_graph_us"], 2),
                             "persistent": round(pr.info["tune_persistent_us"], 2)},
        "plain_fp64_cold": ref,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        out["cpu_baseline"] = cpu_baseline(wl, statistics.mean(iters))
    pr.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
