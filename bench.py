#!/usr/bin/env python3
"""Benchmark: RK4 Bloch steps/s and HBM roofline fraction on one MI355X.

Workload: the driven, dissipatively coupled Bose dimer with N = 1001 levels
(1000 bosons), Bloch dimension M = N^2 - 1 = 1,002,000, FP64; H(t) = H0 +
eps(t) H1 with eps = E + A cos(omega t), one dissipator L at rate 0.1/N.
A step is one classical RK4 step of dv/dt = (Q_H0 + eps(t) Q_H1 + gamma R) v +
gamma K, i.e. four fused SpMV + stage-update launches.  The Lindbladian
assembly (structure constants, Q, R, K) runs once and is timed separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Inputs are synthetic (seeded, no data files).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RK4 Bloch steps/s + HBM roofline % at N=1001; batched/adjoint vs plain, FP64"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--N", type=int, default=1001)
    ap.add_argument("--profile-steps", type=int, default=400,
                    help="steps of the per-launch event-timed pass (roofline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--block-nnz", type=int, default=0)
    ap.add_argument("--threads", type=int, default=256)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def union_nnz(lind, torch):
    """nnz of the union of the sparsity patterns of Q_H0, Q_H1 and R."""
    keys = []
    M = lind.basis.M
    for kind, idx in (("H", 0), ("H", 1), ("L", 0)):
        ex = lind.export(kind, idx)
        rowptr, col = ex[0].long(), ex[1].long()
        rows = torch.repeat_interleave(torch.arange(M, device="cuda"), rowptr[1:] - rowptr[:-1])
        keys.append(rows * M + col)
    return int(torch.unique(torch.cat(keys)).numel())


def cpu_baseline(p, ops, budget_s=12.0):
    """The oracle's density-matrix RK4 (eq. 1 integrated directly), timed on
    the host on a bounded number of steps of the same workload."""
    from oracle import propagate as pr
    N = p.N
    rho = np.zeros((N, N), complex)
    rho[0, 0] = 1.0
    steps_done = 0
    t_start = time.perf_counter()
    chunk = 2
    from workloads import dimer
    while time.perf_counter() - t_start < budget_s and steps_done < 400:
        eps = dimer.drive_table(p, steps=chunk, t0=steps_done * p.dt)
        rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho, eps[:, None], p.dt, chunk)
        steps_done += chunk
    el = time.perf_counter() - t_start
    return {"value": steps_done / el, "unit": "RK4 steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps_done} RK4 steps of the N={N} dimer by the oracle's density-matrix RK4 "
                      f"(scipy sparse x dense, single thread), {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path has no multi-GPU form "
              "in this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1812_11626_amd as sb
    from workloads import dimer

    sb.require_gpu()
    N = args.N
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    M = N * N - 1
    total_steps = args.warmup + args.steps
    log(f"N={N} M={M} steps={args.steps} warmup={args.warmup}")

    # ---- assembly (rows a1-a7), timed once --------------------------------
    dev_ops = {k: sb.DeviceOperator.from_csr(v) for k, v in ops.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    basis = sb.build_basis(N)
    t1 = time.perf_counter()
    lind, prop = sb.expand_lindbladian(basis, dev_ops["H0"], dev_ops["H1"], [(dev_ops["L"], p.gamma_eff)])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if args.block_nnz:
        prop.tune(args.block_nnz, args.threads, False)
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1.0
    v0, _ = basis.expand(sb.DeviceOperator.from_csr(
        dimer.ZCSR.from_diagonals(N, {0: np.eye(N)[0]})))
    v0 = v0.real.contiguous()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    info = prop.info()
    log(f"assembly: basis {1e3*(t1-t0):.1f} ms, expand {1e3*(t2-t1):.1f} ms, fused nnz {info['nnz_fused']}")

    eps = torch.as_tensor(dimer.drive_table(p, steps=total_steps)).cuda().contiguous()
    v = v0.clone()
    # ---- warmup ------------------------------------------------------------
    prop.propagate(v, eps, p.dt, args.warmup)
    torch.cuda.synchronize()
    # ---- timed region -----------------------------------------------------
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    prop.propagate(v, eps[2 * args.warmup:], p.dt, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    steps_per_s = args.steps / (ms / 1e3)
    finite = bool(torch.isfinite(v).all().item())
    log(f"timed: {ms:.1f} ms for {args.steps} steps -> {steps_per_s:.1f} steps/s (finite={finite})")

    # ---- per-launch event timing of the stage kernel (roofline) ------------
    vp = v0.clone()
    ps = min(args.profile_steps, total_steps)
    stage_ms, launches = prop.profile(vp, eps, p.dt, ps)
    avg_launch_s = sum(stage_ms) / launches / 1e3
    nnz_u = union_nnz(lind, torch)
    bytes_per_launch = 12 * nnz_u + 4 * (M + 1) + 20 * M
    achieved = bytes_per_launch / avg_launch_s / 1e9
    layout_bytes = 12 * info["nnz_fused"] + 4 * (M + 1) + 4 * M + 48 * M
    log(f"stage avg {avg_launch_s*1e6:.2f} us, union nnz {nnz_u}, achieved {achieved:.0f} GB/s")

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "RK4 steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dimer-plain-N{N}", "N": N, "M": M, "nnz_union": nnz_u,
                   "nnz_fused": info["nnz_fused"], "steps_per_period": p.steps_per_period,
                   "dt": p.dt, "U_eff": p.U_eff, "gamma_eff": p.gamma_eff, "A": p.A, "E": p.E,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rk4_stage", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": launches,
                     "layout_bytes_per_launch": layout_bytes},
        "assembly_ms": {"build_basis": 1e3 * (t1 - t0), "expand_lindbladian_and_layout": 1e3 * (t2 - t1),
                        "v0": 1e3 * (t3 - t2)},
        "state_finite": finite,
    }

    # ---- batched and adjoint forms, reported against plain -----------------
    out["batched"] = None
    out["adjoint"] = None

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(p, ops)
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['value']:.3f} steps/s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
