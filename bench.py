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
FP64_MFMA_PEAK_TFLOPS = 78.6      # MI355X dense FP64 matrix peak


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
    ap.add_argument("--only", choices=("plain", "batched", "adjoint", "dense", "stationary"), default=None,
                    help="run one leg only (for profiling); prints that leg's report")
    ap.add_argument("--scan", action="store_true",
                    help="assembly time and RK4 steps/s of the plain workload over a range of N (one JSON line)")
    ap.add_argument("--pmc-target", choices=("plain", "batched", "batched-paths", "adjoint", "gemm"),
                    default="plain",
                    help="workload of --pmc-mode")
    ap.add_argument("--pmc-mode", action="store_true",
                    help="short run for rocprofv3 --pmc (stage kernel + calibration copy)")
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


STAGE_SOURCE = "paper_1812_11626_amd/csrc/propagate.hip"
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "k_rk4_sell_dimer-plain-N1001_counters.md")
BATCHED_COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "k_batch_pipe_dimer-batched-512_counters.md")


def stage_source_hash() -> str:
    """SHA-256 of the stage kernel's source: the text between the
    "[stage-kernel source: begin]" / "end" markers of propagate.hip."""
    import hashlib
    import re
    with open(os.path.join(ROOT, STAGE_SOURCE)) as fh:
        text = fh.read()
    parts = re.findall(r"// \[stage-kernel source: begin\]\n(.*?)// \[stage-kernel source: end\]", text, re.S)
    h = hashlib.sha256()
    for part in parts:
        h.update(part.encode())
    return h.hexdigest()


def _summary_fields(path):
    """The `- key: `value`` lines of a committed profile summary."""
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    return fields


def batched_profiled_traffic():
    """(bytes beyond L2 per batched stage launch, the tiling it was taken
    with) from the committed counter summary, or (None, None)."""
    try:
        fields = _summary_fields(BATCHED_COUNTER_SUMMARY)
        return float(fields["bytes_beyond_l2_per_launch"]), fields["tiling"]
    except (OSError, KeyError, ValueError):
        return None, None


def measured_traffic():
    """HBM bytes per stage launch from the committed counter summary, if it
    was taken on the current stage-kernel source (else None)."""
    try:
        fields = _summary_fields(COUNTER_SUMMARY)
        if fields.get("source_sha256") != stage_source_hash():
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _host_info():
    """Host cores this process may use and the CPU model (lscpu)."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    model = ""
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return ncpu, model


def cpu_baseline(p, ops):
    """The oracle's C/OpenMP tier timed on the host: assembly of Q_H0, Q_H1,
    R and K by explicit traces, then its CSR RK4 on the same N = 1001 workload
    on every host core (2000 steps after one warm-up step) and on one thread
    (200 steps); the N = 51 workload over its full 100,000 steps on every core
    (and 10,000 steps on one thread); and the dense tier at N = 4 over its
    full 2,000 steps on one core."""
    from oracle import o2
    from workloads import dimer
    ncpu, model = _host_info()
    threads = int(os.environ.get("OMP_NUM_THREADS") or ncpu)
    threads = max(1, min(threads, ncpu))

    def assemble(q, qops, nth):
        t0 = time.perf_counter()
        Q0 = o2.q_full("H", qops["H0"], threads=nth)
        Q1 = o2.q_full("H", qops["H1"], threads=nth)
        R = o2.q_full("L", qops["L"], threads=nth)
        K = o2.k_vector(qops["L"])
        t = time.perf_counter() - t0
        return [((Q0 + q.gamma_eff * R).tocsr(), q.gamma_eff * K), (Q1, None)], t

    def fock(N):
        v = np.zeros(N * N - 1)
        P = N * (N - 1) // 2
        l = np.arange(1, N)
        v[2 * P:] = 1.0 / np.sqrt(l * (l + 1.0))       # Bloch vector of |0><0|
        return v

    def rate(terms, q, N, steps, nth):
        eps = dimer.drive_table(q, steps=steps + 1)
        coef = np.stack([np.ones_like(eps), eps], axis=1)
        v = o2.rk4(terms, coef[:3], fock(N), q.dt, 1, threads=nth)        # warm-up step
        t0 = time.perf_counter()
        v = o2.rk4(terms, coef[2:], v, q.dt, steps, threads=nth)
        el = time.perf_counter() - t0
        assert np.all(np.isfinite(v))
        return steps / el, el

    terms, t_asm = assemble(p, ops, threads)
    r_mc, el_mc = rate(terms, p, p.N, 2000, threads)
    r_1, el_1 = rate(terms, p, p.N, 200, 1)
    q51 = dimer.plain_config(51)
    ops51 = dimer.dimer_operators(q51)
    terms51, t_asm51 = assemble(q51, ops51, threads)
    r51_mc, el51_mc = rate(terms51, q51, 51, q51.steps, threads)
    r51_1, el51_1 = rate(terms51, q51, 51, 10000, 1)
    # the dense tier at N = 4 (numpy on one core): the terms by explicit
    # traces of dense generators, then the full 10-period horizon
    from oracle import basis as ob, lindblad as lb, propagate as pr
    q4 = dimer.plain_config(4)
    ops4 = dimer.dimer_operators(q4)
    t0 = time.perf_counter()
    F4 = ob.generators(4)
    G0 = lb.q_hamiltonian(F4, ops4["H0"].to_dense()) + q4.gamma_eff * lb.q_dissipator(F4, ops4["L"].to_dense())
    G1 = lb.q_hamiltonian(F4, ops4["H1"].to_dense())
    K4 = q4.gamma_eff * lb.k_dissipator(F4, ops4["L"].to_dense())
    t_asm4 = time.perf_counter() - t0
    eps4 = dimer.drive_table(q4, steps=q4.steps)
    t0 = time.perf_counter()
    v4 = pr.rk4_bloch(G0, [G1], K4, fock(4), eps4[:, None], q4.dt, q4.steps)
    el4 = time.perf_counter() - t0
    assert np.all(np.isfinite(v4))
    return {"value": r_mc, "unit": "RK4 steps/s", "cores": threads, "kind": "oracle",
            "sample": f"2000 RK4 steps ({el_mc:.1f} s) of the N={p.N} dimer by the oracle's C/OpenMP CSR RK4 on "
                      f"{threads} threads after one warm-up step, on Q_H0 + gamma R, Q_H1 and K assembled by the "
                      f"oracle's explicit traces ({t_asm:.1f} s on {threads} threads)",
            "single_thread_steps_per_s": r_1, "single_thread_sample": f"200 steps, {el_1:.1f} s",
            "assembly_s": t_asm, "host_cpus": ncpu, "host_model": model,
            "N51": {"steps_per_s": r51_mc, "cores": threads, "full_100_periods_s": el51_mc,
                    "single_thread_steps_per_s": r51_1, "assembly_s": t_asm51},
            "N4_dense": {"steps_per_s": q4.steps / el4, "cores": 1, "steps": q4.steps, "assembly_s": t_asm4,
                         "sample": "the dense tier (numpy): explicit-trace terms, full 10 periods"}}


def _fock_v0(sb, basis, N, i=0):
    from workloads import dimer
    e = np.zeros(N)
    e[i] = 1.0
    return basis.expand(dimer.ZCSR.from_diagonals(N, {0: e}))[0].real.contiguous()


def small_configs_report(sb, torch, steps=2000):
    """The plain workloads at N = 4 and N = 51 (parity configurations; both
    are latency bound, four stage launches per step): nnz per term, assembly
    time and RK4 steps/s."""
    from workloads import dimer
    res = {}
    for N in (4, 51):
        p = dimer.plain_config(N)
        ops = dimer.dimer_operators(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        basis = sb.build_basis(N)
        lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        torch.cuda.synchronize()
        t_asm = time.perf_counter() - t0
        v = _fock_v0(sb, basis, N)
        # warm-up of 128 steps: builds the layouts and, where used, captures
        # the 64-step graph, so that the timed call only replays
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps + 128)).cuda().contiguous()
        prop.propagate(v, eps, p.dt, 128)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        prop.propagate(v, eps[256:], p.dt, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[str(N)] = {"M": N * N - 1, "nnz_QH0": lind.nnz("H", 0), "nnz_QH1": lind.nnz("H", 1),
                       "nnz_R": lind.nnz("L", 0), "nnz_union": union_nnz(lind, torch),
                       "assembly_ms": 1e3 * t_asm, "steps_per_s": steps / (ms / 1e3),
                       "steps_per_period": p.steps_per_period}
        log(f"plain N={N}: {res[str(N)]['steps_per_s']:.0f} steps/s, assembly {1e3 * t_asm:.1f} ms")
    return res


def general_drive_report(sb, torch, steps=400):
    """General time dependence at N = 1001: square-wave drive on H1 and a
    second dissipation channel L2 = b1^+ b2 whose rate varies in time, i.e.
    two time-dependent terms; the segmented sliced layout (default) against
    the CSR stream layout, RK4 steps/s."""
    from workloads import dimer
    N = 1001
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    s2 = np.sqrt((np.arange(N - 1) + 1.0) * (N - 1.0 - np.arange(N - 1)))
    L2 = dimer.ZCSR.from_diagonals(N, {-1: s2})
    basis = sb.build_basis(N)
    lind = sb.Lindbladian(basis, [ops["H0"], ops["H1"]], [ops["L"], L2])
    prop = lind.propagator([1.0, 0.0, p.gamma_eff, 0.0], [1, 3])
    t = np.arange(2 * (steps + 50) + 1) * 0.5 * p.dt
    table = np.stack([dimer.drive_table_square(p, steps=steps + 50), 0.3 * p.gamma_eff * (1 + 0.5 * np.sin(2 * t))],
                     axis=1)
    coef = torch.as_tensor(table).cuda().contiguous()
    res = {"workload": "dimer-plain-N1001, square-wave drive, second channel b1^+b2 with a time-dependent rate",
           "nnz_fused": prop.info()["nnz_fused"]}
    for name in ("sliced-segmented", "stream"):
        if name == "stream":
            prop.tune(1024, 256, True)
        assert prop.layout()["layout"] == name
        v = _fock_v0(sb, basis, N)
        prop.propagate(v, coef, p.dt, 20)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        prop.propagate(v, coef[100:], p.dt, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[name] = {"steps_per_s": steps / (ms / 1e3), "stage_mean_us": 1e3 * ms / (4 * steps),
                     "finite": bool(torch.isfinite(v).all())}
        log(f"general drive N=1001 ({name}): {res[name]['steps_per_s']:.0f} steps/s")
    return res


def bifurcation_report(sb, torch, N=101, count=128):
    """Stroboscopic population diagram: count values of U at N, ten drive
    periods from |0, N-1><0, N-1| in one batched group over [H_J, H_U, H1, L]
    (autotuned), then P(n1) = rho_ii at t = 10T for every U from the GPU
    readout.  Reports instance-steps/s of the propagation and the wall time
    of the whole diagram."""
    from workloads import dimer
    inst = dimer.bifurcation_instances(N, count=count)
    p0 = inst[0]
    ops = dimer.dimer_operators(p0)
    basis = sb.build_basis(N)
    lind = sb.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"]], [ops["L"]])
    w = np.array([[-q.J, q.U_eff, q.E, q.gamma_eff] for q in inst])
    u = np.array([[0.0, 0.0, q.A, 0.0] for q in inst])
    bp = sb.BatchedPropagator([dict(lind=lind, w=w, u=u, wave=dimer.drive_table_dA(p0, steps=p0.steps), dt=p0.dt,
                                    steps=p0.steps)])
    v0 = _fock_v0(sb, basis, N)
    start = v0.unsqueeze(0).repeat(count, 1)
    bp.set_state(0, start)
    tuned = sb.autotune_batched(bp, probe_steps=8, log=log)
    bp.set_state(0, start)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bp.run(p0.steps)
    V = bp.get_state(0)
    P = torch.stack([basis.density(V[j].contiguous()).diagonal().real for j in range(count)])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    Pc = P.cpu().numpy()
    mean_n1 = (Pc * np.arange(N)).sum(axis=1)
    res = {"workload": f"dimer U scan N={N}, {count} values of U in [0.05, 2] (U_eff = U/(N-1)), "
                       f"{p0.periods} periods x {p0.steps_per_period} steps",
           "instance_steps_per_s": count * p0.steps / el, "diagram_wall_s": el,
           "tile": tuned[0]["tile"], "rows_per_item": tuned[0]["rows_per_item"], "path": tuned[0]["path"],
           "population_sum_max_dev": float(np.abs(Pc.sum(axis=1) - 1.0).max()),
           "mean_n1_at_10T": {f"{q.U:.3f}": float(m) for q, m in list(zip(inst, mean_n1))[::16]}}
    log(f"bifurcation N={N}: {count} U values x {p0.steps} steps in {el:.2f} s "
        f"({res['instance_steps_per_s']:.0f} instance-steps/s)")
    return res


def batched_report(sb, torch):
    """Batched form: the 512-instance dimer workload (N in {51,...,301},
    A ~ U[0.5,3], gamma ~ logU[0.01,0.5]), one launch per RK4 stage for all
    instances, autotuned tiles, timed over its full horizon of 20 drive
    periods (every group through all of its steps); against sequential plain
    solves of the same instances."""
    from workloads import dimer
    inst = dimer.batched_instances()
    byN = {}
    for i, p in enumerate(inst):
        byN.setdefault(p.N, []).append(i)
    specs, meta = [], []
    t0 = time.perf_counter()
    for N in sorted(byN):
        idx = byN[N]
        p0 = inst[idx[0]]
        ops = dimer.dimer_operators(p0)
        basis = sb.build_basis(N)
        lind = sb.Lindbladian(basis, [ops["H0"], ops["H1"]], [ops["L"]])
        w = np.array([[1.0, inst[i].E, inst[i].gamma_eff] for i in idx])
        u = np.array([[0.0, inst[i].A, 0.0] for i in idx])
        specs.append(dict(lind=lind, w=w, u=u, wave=dimer.drive_table_dA(p0), dt=p0.dt, steps=p0.steps))
        meta.append((N, idx, basis, lind, p0))
    bp = sb.BatchedPropagator(specs)
    starts = []
    for g, (N, idx, basis, lind, p0) in enumerate(meta):
        v0 = _fock_v0(sb, basis, N)
        starts.append(v0.unsqueeze(0).repeat(len(idx), 1))
        bp.set_state(g, starts[-1])
    setup_s = time.perf_counter() - t0
    tuned = sb.autotune_batched(bp, probe_steps=8, log=log)
    for g in range(len(meta)):
        bp.set_state(g, starts[g])          # from t = 0 after the tuning probes
    total = sum(len(idx) * p0.steps for (_, idx, _, _, p0) in meta)
    most = max(p0.steps for (_, _, _, _, p0) in meta)
    log(f"batched: {len(inst)} instances, full 20 periods ({total} instance-steps, {most} steps in the longest group)")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bp.run(most)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    finite = all(bool(torch.isfinite(bp.get_state(g)).all()) for g in range(len(meta)))
    batched_rate = total / el
    # algorithmic bytes of the whole run (the batched byte model): per group
    # and stage the fused CSR once (12 per stored entry + 4 per row pointer)
    # plus 20 bytes per state row and instance (gather, base, accumulator and
    # output streams: 80 M per instance-step)
    alg_bytes = 0
    stage_bytes = 0
    launch_bytes = 0          # one stage launch with every group active
    for g, (N, idx, basis, lind, p0) in enumerate(meta):
        info = bp.info(g)
        M = info["M"]
        alg_bytes += p0.steps * 4 * (12 * info["nnz"] + 4 * (M + 1)) + p0.steps * len(idx) * 80 * M
        launch_bytes += 12 * info["nnz"] + 4 * (M + 1) + 20 * M * len(idx)
        # the state streams a four-launch classical RK4 step cannot avoid (the
        # gathered input counted once): 24 + 40 + 40 + 32 = 136 B per state row
        # and instance per step
        stage_bytes += p0.steps * 4 * (12 * info["nnz"] + 4 * (M + 1)) + p0.steps * len(idx) * 136 * M
    tiling = ",".join(f"{tuned[g]['tile']}/{tuned[g]['rows_per_item']}/{tuned[g]['path']}" for g in range(len(meta)))
    prof_bytes, prof_tiling = batched_profiled_traffic()
    traffic = prof_bytes if prof_tiling == tiling else None
    # sequential plain solves: per-step time of one plain instance per N
    seq_time = 0.0
    per_N = {}
    for g, (N, idx, basis, lind, p0) in enumerate(meta):
        p = inst[idx[0]]
        prop = lind.propagator([1.0, 0.0, p.gamma_eff], [1])
        v = _fock_v0(sb, basis, N)
        nst = 200
        eps = torch.as_tensor(dimer.drive_table(p, steps=nst)).cuda().contiguous()
        prop.propagate(v, eps, p.dt, 128)            # warm-up, including the graph capture where used
        torch.cuda.synchronize()
        ta = time.perf_counter()
        prop.propagate(v, eps, p.dt, nst)
        torch.cuda.synchronize()
        tstep = (time.perf_counter() - ta) / nst
        per_N[N] = {"instances": len(idx), "steps_per_period": p0.steps_per_period, "plain_us_per_step": 1e6 * tstep,
                    "tile": tuned[g]["tile"], "rows_per_item": tuned[g]["rows_per_item"],
                    "path": tuned[g]["path"]}
        seq_time += len(idx) * p0.steps * tstep
    seq_rate = total / seq_time
    log(f"batched: 20 periods in {el:.1f} s, {batched_rate:.0f} instance-steps/s vs sequential plain {seq_rate:.0f}; "
        f"algorithmic {alg_bytes / el / 1e9:.0f} GB/s")
    return {"workload": "dimer-batched-512 (N in {51,101,151,201,301}, A~U[0.5,3], gamma~logU[0.01,0.5]/N), "
                        "20 periods",
            "instances": len(inst), "instance_steps": total, "full_20_periods_s": el,
            "instance_steps_per_s": batched_rate, "state_finite": finite,
            "sequential_plain_instance_steps_per_s": seq_rate, "sequential_plain_20_periods_s_est": seq_time,
            "speedup_vs_sequential_plain": batched_rate / seq_rate,
            "roofline": {"bound": "hbm", "algorithmic_bytes": alg_bytes, "achieved": alg_bytes / el / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg_bytes / el / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_launch": launch_bytes, "tiling": tiling,
                         "rk4_stream_bytes": stage_bytes,
                         "rk4_stream_frac": stage_bytes / el / 1e9 / HBM_PEAK_GBS,
                         "traffic": traffic,
                         "profiled_traffic": {"bytes_beyond_l2_per_launch": prof_bytes, "tiling": prof_tiling},
                         "traffic_note": "bytes beyond L2 per stage launch with every group active, from the "
                                         "committed counter summary; null when this run's autotuned tiling "
                                         "differs from the profiled one (profiled_traffic gives it anyway)"},
            "groups": per_N, "setup_s": setup_s}


def _adjoint_problem(sb, N, steps, S, ckpt):
    """AdjointProblem of the dimer (terms H_J, H_U, H1, L; theta = (A, gamma,
    U)) at N (301: the adjoint workload, otherwise the plain one)."""
    import copy
    from workloads import dimer
    p = dimer.adjoint_config(N) if N == 301 else dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    basis = sb.build_basis(p.N)
    lind = sb.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"]], [ops["L"]])
    v0 = _fock_v0(sb, basis, p.N)
    cobs = basis.expand(ops["H1"])[0].real.contiguous()

    def pmap(theta):
        A, g, U = (float(x) for x in theta)
        q = copy.copy(p)
        q.A = A
        dcoef = np.zeros((2 * steps + 1, 1, 3))
        dcoef[:, 0, 0] = dimer.drive_table_dA(q, steps=steps)
        dstatic = np.zeros((4, 3))
        dstatic[1, 2] = p.U_scale
        dstatic[3, 1] = p.gamma_scale
        return dict(static_w=[-p.J, U * p.U_scale, 0.0, g * p.gamma_scale], dyn=[2],
                    coef=dimer.drive_table(q, steps=steps)[:, None], dstatic=dstatic, dcoef=dcoef)

    prob = sb.AdjointProblem(lind, pmap, v0, cobs, p.dt, steps, S, ckpt_every=ckpt)
    return prob, p


def adjoint_report(sb, torch, periods=100, N=301, ckpt=None):
    """Adjoint form at N (301: the adjoint workload over its full horizon of
    100 periods with a checkpoint every period; 1001: the plain workload):
    d<n1-n2>_(last period)/d(A, gamma, U) by the discrete adjoint on a
    PyTorch workspace; time of the gradient over the time of the forward
    objective (both warmed: layouts built, workspace allocated)."""
    from workloads import dimer
    p0 = dimer.adjoint_config(N) if N == 301 else dimer.plain_config(N)
    steps = periods * p0.steps_per_period
    S = p0.steps_per_period
    ckpt = S if ckpt is None else ckpt
    prob, p = _adjoint_problem(sb, N, steps, S, ckpt)
    theta = np.array([p.A, p.gamma, p.U])
    adj, coef, dstatic, dcoef = prob._setup(theta)
    full, low = adj.plan(dstatic, steps, ckpt)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    # warm: the forward objective and a short gradient (builds the reverse layout)
    adj.objective(prob.v0, coef, prob.cobs, p.dt, 16, 8)
    adj.run(prob.v0, coef, dstatic, dcoef, prob.cobs, p.dt, 16, 8, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J_f = adj.objective(prob.v0, coef, prob.cobs, p.dt, steps, S)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    J, g = adj.run(prob.v0, coef, dstatic, dcoef, prob.cobs, p.dt, steps, S, ckpt, workspace=ws)
    t_grad = time.perf_counter() - t0
    log(f"adjoint N={N}: {periods} periods, forward {t_fwd:.2f} s, gradient {t_grad:.2f} s, "
        f"ratio {t_grad/t_fwd:.2f}")
    return {"workload": f"dimer-adjoint-N{N} ({periods} periods x {p.steps_per_period} steps, checkpoint every "
                        f"{ckpt} steps, loss = <n1-n2> averaged over the last period, theta = (A, gamma, U))",
            "steps": steps, "J": J, "J_forward_only": J_f, "grad": {"A": g[0], "gamma": g[1], "U": g[2]},
            "forward_s": t_fwd, "gradient_s": t_grad, "gradient_over_forward": t_grad / t_fwd,
            "forward_steps_per_s": steps / t_fwd, "workspace_bytes": full, "min_workspace_bytes": low}


def dense_report(sb, torch, N=100):
    """Random dense Lindbladian at N = 100 (the size of the paper's random
    ensembles): dense assembly of a random Hermitian H and a random complex L
    (dense sections + one matrix-core product for R), the product alone at
    its shape (M x 2M by 2M x M) against the FP64 matrix peak, and the
    stationary state of that generator."""
    from workloads import random_ops
    M = N * N - 1
    H = random_ops.random_hermitian_csr(N, 1.0, seed=9001)
    L = random_ops.random_complex_csr(N, 1.0, seed=9002)
    basis = sb.build_basis(N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lind = sb.Lindbladian(basis, [H], [L], dense=True)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    g = torch.Generator(device="cuda").manual_seed(7)
    X = torch.randn((M, 2 * M), dtype=torch.float64, device="cuda", generator=g)
    Y = torch.randn((2 * M, M), dtype=torch.float64, device="cuda", generator=g)
    C = torch.empty((M, M), dtype=torch.float64, device="cuda")
    sb.gemm_f64(X, Y, C, -0.5, 0.0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        sb.gemm_f64(X, Y, C, -0.5, 0.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 2.0 * M * M * (2 * M)
    tflops = flops / (ms / 1e3) / 1e12
    del X, Y, C
    torch.cuda.empty_cache()
    prop = lind.propagator([1.0, 0.1], [])
    t0 = time.perf_counter()
    v, iters, relres = prop.stationary([], tau=1.0)
    t_st = time.perf_counter() - t0
    rho = basis.density(v)
    ev = torch.linalg.eigvalsh(rho.cpu())
    log(f"dense N={N}: assembly {t_asm:.2f} s, product {ms:.1f} ms = {tflops:.1f} TFLOP/s "
        f"({100 * tflops / FP64_MFMA_PEAK_TFLOPS:.0f}% of FP64 peak); stationary {iters} it, {t_st:.2f} s")
    return {"workload": f"random dense H and L at N={N} (M={M}), rate 0.1",
            "assembly_s": t_asm, "nnz_R": lind.nnz("L", 0), "nnz_QH": lind.nnz("H", 0),
            "roofline": {"bound": "mfma", "kernel": "k_gemm_f64", "shape": [M, M, 2 * M], "flops": flops,
                         "ms": ms, "achieved": tflops, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP64_MFMA_PEAK_TFLOPS},
            "stationary": {"iterations": iters, "relres": relres, "seconds": t_st,
                           "rho_min_eigenvalue": float(ev.min()), "rho_trace": float(rho.diagonal().real.sum())}}


def stationary_report(sb, torch, Ns=(301, 1001)):
    """Stationary state of the dimer generator at the static drive eps = E:
    GMRES on the RK4 time-tau map (tau = 1) with the step 2.5 / |lambda|max of
    that generator (power iteration, inside the timed region; the fixed point
    of the map does not depend on the step), iterations, time and residual."""
    from workloads import dimer
    res = {}
    for N in Ns:
        p = dimer.plain_config(N)
        ops = dimer.dimer_operators(p)
        basis = sb.build_basis(N)
        lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho = prop.spectral_radius([p.E])
        dt = 2.5 / rho
        v, iters, relres = prop.stationary([p.E], dt=dt, tau=1.0)
        el = time.perf_counter() - t0
        res[str(N)] = {"iterations": iters, "relres": relres, "seconds": el, "dt": dt, "spectral_radius": rho,
                       "steps_per_map": max(1, int(round(1.0 / dt)))}
        log(f"stationary N={N}: {iters} iterations, relres {relres:.1e}, {el:.2f} s")
    return res


def _calibration_copy(torch):
    """Three plain 512 MiB device copies (known bytes) that calibrate the
    byte counters of a profiled run."""
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return a.numel() * 8


def pmc_mode(sb, torch, steps, N=1001, target="plain"):
    """Short runs for profiling, each followed by the calibration copy:
      plain   -- the stage kernel on the plain workload (N = 1001 unless --N
                 says otherwise), `steps` RK4 steps;
      batched -- the 512-instance workload with its autotuned tiling (from the
                 autotuner's cache when a previous run filled it; then no
                 probe launches run), 3 RK4 steps of every group;
      batched-paths -- the N = 301 group of the 512-instance workload alone,
                 3 RK4 steps on path 0 (128-instance tile, 64-row blocks),
                 then 3 on path 5 (128-instance tile);
      adjoint -- the adjoint workload N = 301, 8 steps with a checkpoint every
                 4 (forward and fused reverse stages);
      gemm    -- the dense path's product at N = 100 (9,999 x 19,998 by
                 19,998 x 9,999), once."""
    from workloads import dimer
    info = {"pmc_mode": True, "target": target}
    if target == "plain":
        p = dimer.plain_config(N)
        p.steps_per_period = max(p.steps_per_period, dimer.stable_steps_per_period(N, p.E + p.A))
        ops = dimer.dimer_operators(p)
        basis = sb.build_basis(N)
        lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        v = _fock_v0(sb, basis, N)
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
        prop.propagate(v, eps, p.dt, steps)
        info.update(steps=steps, layout=prop.layout())
    elif target in ("batched", "batched-paths"):
        inst = dimer.batched_instances()
        byN = {}
        for i, q in enumerate(inst):
            byN.setdefault(q.N, []).append(i)
        specs, starts = [], []
        for Ng in sorted(byN):
            idx = byN[Ng]
            p0 = inst[idx[0]]
            ops = dimer.dimer_operators(p0)
            basis = sb.build_basis(Ng)
            lind = sb.Lindbladian(basis, [ops["H0"], ops["H1"]], [ops["L"]])
            specs.append(dict(lind=lind, w=np.array([[1.0, inst[i].E, inst[i].gamma_eff] for i in idx]),
                              u=np.array([[0.0, inst[i].A, 0.0] for i in idx]), wave=dimer.drive_table_dA(p0),
                              dt=p0.dt, steps=p0.steps))
            starts.append(_fock_v0(sb, basis, Ng).unsqueeze(0).repeat(len(idx), 1))
        bp = sb.BatchedPropagator(specs)
        for g, st in enumerate(starts):
            bp.set_state(g, st)
        if target == "batched-paths":
            g = len(specs) - 1                      # the N = 301 group
            ms = {}
            for path in (0, 5):
                bp.tune(g, 128, 64, path)
                bp.set_state(g, starts[g])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                bp.run(3, only_group=g)
                torch.cuda.synchronize()
                ms[f"path{path}"] = (time.perf_counter() - t0) / 3 * 1e3
            info.update(steps=3, N=bp.groups[g]["N"], B=bp.groups[g]["B"], ms_per_step_with_sync=ms)
            info["copy_bytes"] = _calibration_copy(torch)
            print(json.dumps(info), flush=True)
            return
        tuned = sb.autotune_batched(bp, probe_steps=8)
        for g, st in enumerate(starts):
            bp.set_state(g, st)
        bp.run(3)
        info.update(steps=3, tuning=tuned, groups=[{"N": G["N"], "B": G["B"], **bp.info(g)}
                                                    for g, G in enumerate(bp.groups)])
    elif target == "adjoint":
        prob, p = _adjoint_problem(sb, 301, 8, 4, 4)
        J, g = prob.value_and_grad(np.array([p.A, p.gamma, p.U]))
        info.update(steps=8, J=J, grad=list(g))
    elif target == "gemm":
        M = 9999
        g = torch.Generator(device="cuda").manual_seed(7)
        X = torch.randn((M, 2 * M), dtype=torch.float64, device="cuda", generator=g)
        Y = torch.randn((2 * M, M), dtype=torch.float64, device="cuda", generator=g)
        C = torch.empty((M, M), dtype=torch.float64, device="cuda")
        sb.gemm_f64(X, Y, C, -0.5, 0.0)
        torch.cuda.synchronize()
        info.update(shape=[M, M, 2 * M])
    info["copy_bytes"] = _calibration_copy(torch)
    print(json.dumps(info), flush=True)


def scan_report(sb, torch, Ns=(51, 101, 201, 301, 501, 701, 1001, 1501, 2001), steps=200):
    """The plain dimer workload over a range of N (stable step counts from the
    dimer estimate): assembly time, fused nonzeros, layout, RK4 steps/s and
    the stage launch's algorithmic bandwidth, with the union nonzeros from
    the closed form (37N^2 - 93N + 52)/2 (exact for N >= 11)."""
    from workloads import dimer
    rows = []
    for N in Ns:
        p = dimer.plain_config(N)
        p.steps_per_period = dimer.stable_steps_per_period(N, p.E + p.A)
        ops = dimer.dimer_operators(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        basis = sb.build_basis(N)
        lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        torch.cuda.synchronize()
        t_asm = time.perf_counter() - t0
        M = N * N - 1
        v = _fock_v0(sb, basis, N)
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps + 128)).cuda().contiguous()
        prop.propagate(v, eps, p.dt, 128)            # warm-up, including the graph capture where used
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        prop.propagate(v, eps[256:], p.dt, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nnz_union = (37 * N * N - 93 * N + 52) // 2
        b = 12 * nnz_union + 4 * (M + 1) + 20 * M
        stage_us = 1e3 * ms / (4 * steps)
        row = {"N": N, "M": M, "nnz_fused": prop.info()["nnz_fused"], "layout": prop.layout()["layout"],
               "assembly_ms": 1e3 * t_asm, "steps_per_s": steps / (ms / 1e3), "stage_us": stage_us,
               "algorithmic_bytes_per_launch": b, "achieved_GBs": b / stage_us / 1e3,
               "frac_of_8TBs": b / stage_us / 1e3 / HBM_PEAK_GBS, "finite": bool(torch.isfinite(v).all())}
        rows.append(row)
        log(f"scan N={N}: assembly {row['assembly_ms']:.1f} ms, {row['steps_per_s']:.0f} steps/s, "
            f"{row['achieved_GBs']:.0f} GB/s ({row['layout']})")
        del lind, prop, basis, v, eps
        torch.cuda.empty_cache()
    return {"scan": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU "
              "form (the design notes describe how it would shard)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1812_11626_amd as sb
    from workloads import dimer

    sb.require_gpu()
    if args.pmc_mode:
        pmc_mode(sb, torch, min(args.steps, 20), args.N, args.pmc_target)
        return
    if args.scan:
        print(json.dumps(scan_report(sb, torch)), flush=True)
        return
    if args.only == "batched":
        print(json.dumps(batched_report(sb, torch)), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(adjoint_report(sb, torch)), flush=True)
        return
    if args.only == "dense":
        print(json.dumps(dense_report(sb, torch)), flush=True)
        return
    if args.only == "stationary":
        print(json.dumps(stationary_report(sb, torch)), flush=True)
        return
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
    layout = prop.layout()
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

    # ---- roofline of the stage kernel --------------------------------------
    # The timed region above contains only stage-kernel launches (4 per step,
    # back to back on one stream) plus two 8 MB device copies, so its HIP-event
    # time divided by the launch count is the kernel's mean launch duration.
    launches = 4 * args.steps
    avg_launch_s = (ms / 1e3) / launches
    # secondary: HIP event pairs around each launch (serialises dispatch, so
    # it reads a few microseconds above the back-to-back figure)
    vp = v0.clone()
    ps = min(args.profile_steps, total_steps)
    stage_ms, plaunch = prop.profile(vp, eps, p.dt, ps)
    pair_avg_s = sum(stage_ms) / plaunch / 1e3
    nnz_u = union_nnz(lind, torch)
    bytes_per_launch = 12 * nnz_u + 4 * (M + 1) + 20 * M
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # bytes the layout really streams per launch: matrix + per-row metadata
    # (+ the long rows' CSR entries) and the row-wise vectors
    layout_bytes = layout["matrix_bytes_per_launch"] + 12 * (info["nnz_fused"] - layout["stored_entries"]) \
        if layout["layout"] == "sliced" else layout["matrix_bytes_per_launch"]
    layout_bytes += 48 * M
    log(f"stage mean {avg_launch_s*1e6:.2f} us (event pairs {pair_avg_s*1e6:.2f} us), union nnz {nnz_u}, "
        f"achieved {achieved:.0f} GB/s")

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_rk4_sell", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches_timed": launches,
                     "event_pair_avg_launch_us": pair_avg_s * 1e6,
                     "layout_bytes_per_launch_est": layout_bytes, "layout": layout},
        "assembly_ms": {"build_basis": 1e3 * (t1 - t0), "expand_lindbladian_and_layout": 1e3 * (t2 - t1),
                        "v0": 1e3 * (t3 - t2)},
        "state_finite": finite,
    }

    # ---- the same stage kernel with the matrix streamed from HBM -----------
    # (non-temporal loads keep it out of the memory-side cache between launches)
    prop.tune_sliced(nontemporal=True)
    vn = v0.clone()
    prop.propagate(vn, eps, p.dt, 20)
    torch.cuda.synchronize()
    e0.record(stream)
    prop.propagate(vn, eps[2 * args.warmup:], p.dt, min(args.steps, 1000))
    e1.record(stream)
    torch.cuda.synchronize()
    nt_us = 1e3 * e0.elapsed_time(e1) / (4 * min(args.steps, 1000))
    prop.tune_sliced()
    out["roofline"]["hbm_sourced"] = {"avg_launch_us": nt_us, "achieved": bytes_per_launch / nt_us / 1e3,
                                      "frac": bytes_per_launch / nt_us / 1e3 / HBM_PEAK_GBS,
                                      "note": "same kernel with non-temporal matrix loads (stream from HBM)"}
    log(f"stage kernel with the matrix from HBM: {nt_us:.2f} us ({bytes_per_launch / nt_us / 1e3:.0f} GB/s)")

    # ---- further forms, reported against plain ------------------------------
    out["plain_other_configs"] = small_configs_report(sb, torch)
    out["general_drive"] = general_drive_report(sb, torch)
    out["batched"] = None if args.no_batched else batched_report(sb, torch)
    out["bifurcation"] = None if args.no_batched else bifurcation_report(sb, torch)
    out["adjoint"] = None if args.no_adjoint else adjoint_report(sb, torch)
    out["adjoint_N1001"] = None if args.no_adjoint else adjoint_report(sb, torch, periods=1, N=1001, ckpt=2048)
    out["stationary"] = stationary_report(sb, torch)
    out["dense"] = dense_report(sb, torch)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(p, ops)
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['value']:.2f} steps/s on {cb['cores']} threads, "
            f"{cb['single_thread_steps_per_s']:.2f} on one; N=51: {cb['N51']['steps_per_s']:.0f} steps/s")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
