"""Batched form: many (A, gamma, N) instances in one launch per RK4 stage.

Every instance must match, to 1e-12 relative, the oracle's RK4 on its own
generator (dense tier, small N) or the plain GPU propagation of that
instance (the 512-instance workload, sampled), and the result must not
depend on the tiling.
"""

import numpy as np
import pytest
import torch

from helpers import dimer_batch, flush, fock_bloch, rel_vec_err
from oracle import basis as ob, lindblad as lb, propagate as pr
from workloads import dimer

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _small_instances():
    out = []
    rng = np.random.default_rng(77)
    for N, cnt in ((4, 3), (5, 2)):
        for _ in range(cnt):
            p = dimer.plain_config(N)
            p.A = float(rng.uniform(0.5, 3.0))
            p.gamma = float(rng.uniform(0.05, 0.5))
            p.steps_per_period = 200 if N == 4 else 300
            out.append(p)
    return out


def _oracle_instance(p, steps, v0):
    ops = dimer.dimer_operators(p)
    F = ob.generators(p.N)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    K = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    eps = dimer.drive_table(p, steps=steps)
    return pr.rk4_bloch(G0, [G1], K, v0, eps[:, None], p.dt, steps)


def test_small_groups_against_dense_oracle(lib):
    flush("[batched] small groups vs oracle")
    inst = _small_instances()
    steps = {4: 60, 5: 40}
    bp, groups = dimer_batch(lib, inst, steps)
    for g, (N, idx, _, _, _) in enumerate(groups):
        V = np.stack([fock_bloch(N, i % N) for i in range(len(idx))])
        bp.set_state(g, torch.as_tensor(V))
    bp.run(1000)        # every group stops at its own step count
    for g, (N, idx, _, _, st) in enumerate(groups):
        got = bp.get_state(g).cpu().numpy()
        for j, i in enumerate(idx):
            want = _oracle_instance(inst[i], st, fock_bloch(N, j % N))
            assert rel_vec_err(got[j], want) <= TOL, (N, j)


def test_tiling_does_not_change_results(lib):
    flush("[batched] tiling invariance")
    inst = _small_instances()
    bp, groups = dimer_batch(lib, inst, {4: 30, 5: 30})
    starts = [torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx))) for (N, idx, _, _, _) in groups]
    results = []
    for tile, rows, path in ((64, 64, 0), (8, 1, 0), (16, 7, 1), (32, 512, 1), (64, 3, 1), (16, 128, 0),
                             (128, 32, 0), (128, 5, 1), (16, 64, 2), (32, 9, 2), (64, 128, 2), (8, 16, 2),
                             (8, 4, 3), (16, 64, 3), (32, 128, 3), (128, 64, 5), (64, 1, 5), (64, 32, 7),
                             (64, 1, 7), (64, 7, 7)):
        for g in range(len(groups)):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(30)
        results.append([bp.get_state(g).cpu().numpy() for g in range(len(groups))])
    for r in results[1:]:
        for a, b in zip(r, results[0]):
            assert np.array_equal(a, b)


def test_lds_and_global_paths_agree_bitwise(lib):
    """N = 51 and 101 groups (rows span many LDS blocks of <= 1024 entries):
    the LDS-staged path and the per-wavefront path give the same bits."""
    flush("[batched] LDS vs global path")
    rng = np.random.default_rng(5)
    inst = []
    for N in (51, 101):
        for _ in range(70):
            p = dimer.plain_config(N)
            p.A = float(rng.uniform(0.5, 3.0))
            p.gamma = float(rng.uniform(0.01, 0.5))
            inst.append(p)
    bp, groups = dimer_batch(lib, inst, 12)
    starts = [torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx))) for (N, idx, _, _, _) in groups]
    out = []
    for tile, rows, path in ((64, 64, 0), (16, 128, 0), (32, 16, 1), (64, 8, 1), (128, 64, 0), (128, 8, 0),
                             (16, 64, 2), (32, 32, 2), (64, 128, 2), (8, 128, 3), (16, 32, 3), (32, 128, 3),
                             (128, 64, 5), (64, 64, 5), (64, 32, 7), (64, 16, 7)):
        for g in range(len(groups)):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(12)
        out.append([bp.get_state(g).cpu().numpy() for g in range(len(groups))])
    for r in out[1:]:
        for a, b in zip(r, out[0]):
            assert np.array_equal(a, b)


def test_row_wavefront_path_multi_tile_bitwise(lib):
    """Path 5 (one wavefront per row and tile, matrix through the scalar
    cache) and path 7 (pipelined staging, tiles of 64) on groups of 300 and
    130 instances, i.e. 3 and 2 tiles of 128 and 5 and 3 tiles of 64 with
    ragged last tiles, against path 0: bitwise equal after 16 steps, and the
    first instances against the dense oracle."""
    flush("[batched] path 5, several tiles per group, vs path 0")
    rng = np.random.default_rng(11)
    inst = []
    for N, cnt in ((4, 300), (5, 130)):
        for _ in range(cnt):
            p = dimer.plain_config(N)
            p.A = float(rng.uniform(0.5, 3.0))
            p.gamma = float(rng.uniform(0.05, 0.5))
            p.steps_per_period = 200 if N == 4 else 300
            inst.append(p)
    steps = 16
    bp, groups = dimer_batch(lib, inst, steps)
    starts = [torch.as_tensor(np.stack([fock_bloch(N, j % N) for j in range(len(idx))])) for (N, idx, _, _, _) in groups]
    out = []
    for tile, rows, path in ((64, 64, 0), (128, 64, 5), (64, 64, 5), (64, 32, 7)):
        for g in range(len(groups)):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(steps)
        out.append([bp.get_state(g).cpu().numpy() for g in range(len(groups))])
    for r in out[1:]:
        for a, b in zip(r, out[0]):
            assert np.array_equal(a, b)
    for g, (N, idx, _, _, st) in enumerate(groups):
        for j in (0, len(idx) - 1):
            want = _oracle_instance(inst[idx[j]], st, fock_bloch(N, j % N))
            assert rel_vec_err(out[1][g][j], want) <= TOL, (N, j)


def test_pipelined_path_large_groups_bitwise(lib):
    """Path 7 (persistent pipelined staging) on the N = 151, 201 and 301
    groups of the 512-instance workload -- two tiles of 64 instances, the
    last one ragged; at N >= 201 some rows have more distinct columns than a
    block's 128 slots and take the long-row walk -- alone and mixed with
    path 0 in the same launches: bitwise equal to path 0 after 8 steps, and
    the last instance of each group against plain single-instance GPU
    propagation (1e-12)."""
    flush("[batched] path 7 on the large groups vs path 0")
    inst = [p for p in dimer.batched_instances() if p.N in (151, 201, 301)]
    steps = 8
    bp, groups = dimer_batch(lib, inst, steps)
    starts = [torch.as_tensor(np.stack([fock_bloch(N, j % 3) for j in range(len(idx))]))
              for (N, idx, _, _, _) in groups]
    out = []
    for cfg in ([(64, 64, 0)] * 3, [(64, 32, 7)] * 3, [(64, 32, 7), (128, 64, 0), (64, 16, 7)]):
        for g, (tile, rows, path) in enumerate(cfg):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(steps)
        out.append([bp.get_state(g).cpu().numpy() for g in range(len(groups))])
    for r in out[1:]:
        for a, b in zip(r, out[0]):
            assert np.array_equal(a, b)
    for g, (N, idx, lind, dt, st) in enumerate(groups):
        j = len(idx) - 1
        p = inst[idx[j]]
        prop = lind.propagator([1.0, 0.0, p.gamma_eff], [1])
        v = torch.as_tensor(fock_bloch(N, j % 3)).cuda()
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
        prop.propagate(v, eps, dt, steps)
        assert rel_vec_err(out[1][g][j], v.cpu().numpy()) <= TOL, (N, j)


def test_pipelined_path_dense_generator_long_rows(lib):
    """Path 7 on a group where most rows have more distinct columns than a
    block's 127 slots (random dense H0, H1 and L at N = 12, M = 143), with
    70 instances (two tiles of 64, the second ragged): bitwise equal to
    path 0 after 6 steps, and two instances against the dense oracle's RK4
    on their own generators (1e-12)."""
    flush("[batched] path 7, dense random generator (long rows)")
    from workloads import random_ops
    N, B, steps, dt = 12, 70, 6, 0.01
    H0 = random_ops.random_hermitian_csr(N, 1.0, seed=901)
    H1 = random_ops.random_hermitian_csr(N, 0.5, seed=902)
    L = random_ops.random_complex_csr(N, 1.0, seed=903)
    basis = lib.build_basis(N)
    lind = lib.Lindbladian(basis, [H0, H1], [L])
    rng = np.random.default_rng(9)
    A = rng.uniform(0.5, 1.5, B)
    g = rng.uniform(0.05, 0.3, B)
    wave = np.cos(0.5 * dt * np.arange(2 * steps + 1))
    w = np.stack([np.ones(B), np.full(B, 0.3), g], axis=1)
    u = np.stack([np.zeros(B), A, np.zeros(B)], axis=1)
    bp = lib.BatchedPropagator([dict(lind=lind, w=w, u=u, wave=wave, dt=dt, steps=steps)])
    start = torch.as_tensor(np.stack([fock_bloch(N, j % N) for j in range(B)]))
    out = []
    for tile, rows, path in ((64, 64, 0), (64, 32, 7), (64, 8, 7)):
        bp.tune(0, tile, rows, path)
        bp.set_state(0, start)
        bp.run(steps)
        out.append(bp.get_state(0).cpu().numpy())
    assert np.array_equal(out[1], out[0]) and np.array_equal(out[2], out[0])
    F = ob.generators(N)
    QH0 = lb.q_hamiltonian(F, H0.to_dense())
    QH1 = lb.q_hamiltonian(F, H1.to_dense())
    RL = lb.q_dissipator(F, L.to_dense())
    KL = lb.k_dissipator(F, L.to_dense())
    for j in (0, B - 1):
        want = pr.rk4_bloch(QH0 + g[j] * RL, [QH1], g[j] * KL, fock_bloch(N, j % N),
                            (0.3 + A[j] * wave)[:, None], dt, steps)
        assert rel_vec_err(out[1][j], want) <= TOL, j


def test_pipelined_path_many_terms(lib):
    """Path 7 with six terms whose coefficients all differ between
    instances (H_J, H_U, H1 and two dissipators, one a random banded
    operator): the coefficient table of the tile spans more terms than half
    the workgroup's wavefronts; 90 instances at N = 21 and 61, bitwise equal
    to path 0 after 10 steps, and one instance per group against the dense
    oracle (N = 21) or plain single-instance propagation (N = 61) to
    1e-12."""
    flush("[batched] path 7 with six instance-dependent terms")
    from workloads import random_ops
    rng = np.random.default_rng(21)
    steps, dt = 10, 0.002
    specs, meta = [], []
    for N in (21, 61):
        ops = dimer.dimer_operators(dimer.DimerParams(N=N))
        L2 = random_ops.random_complex_csr(N, 3.0 / N, seed=70 + N)
        basis = lib.build_basis(N)
        lind = lib.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"], ops["H1"]], [ops["L"], L2])
        B = 90
        w = rng.uniform(0.5, 1.5, (B, 6)) * np.array([-1.0, 0.02, 1.0, 0.3, 0.01, 0.005])
        u = np.zeros((B, 6))
        u[:, 2] = rng.uniform(0.5, 3.0, B)
        wave = np.cos(0.5 * dt * np.arange(2 * steps + 1))
        specs.append(dict(lind=lind, w=w, u=u, wave=wave, dt=dt, steps=steps))
        meta.append((N, ops, L2, lind, w, u, wave))
    bp = lib.BatchedPropagator(specs)
    starts = [torch.as_tensor(np.stack([fock_bloch(N, j % N) for j in range(90)])) for (N, *_r) in meta]
    out = []
    for tile, rows, path in ((64, 64, 0), (64, 32, 7)):
        for g in range(2):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(steps)
        out.append([bp.get_state(g).cpu().numpy() for g in range(2)])
    for a, b in zip(out[1], out[0]):
        assert np.array_equal(a, b)
    # group 0 (N = 21): the last instance against the dense oracle
    N, ops, L2, lind, w, u, wave = meta[0]
    j = 89
    F = ob.generators(N)
    c = w[j][None, :] + u[j][None, :] * wave[:, None]          # [2 steps + 1][6]
    QJ, QU, Q1 = (lb.q_hamiltonian(F, ops[k].to_dense()) for k in ("HJ", "HU", "H1"))
    RL, R2 = lb.q_dissipator(F, ops["L"].to_dense()), lb.q_dissipator(F, L2.to_dense())
    KL, K2 = lb.k_dissipator(F, ops["L"].to_dense()), lb.k_dissipator(F, L2.to_dense())
    G0 = w[j, 0] * QJ + w[j, 1] * QU + w[j, 3] * Q1 + w[j, 4] * RL + w[j, 5] * R2
    want = pr.rk4_bloch(G0, [Q1], w[j, 4] * KL + w[j, 5] * K2, fock_bloch(N, j % N), c[:, 2:3], dt, steps)
    assert rel_vec_err(out[1][0][j], want) <= TOL
    # group 1 (N = 61): the first instance against plain propagation
    N, ops, L2, lind, w, u, wave = meta[1]
    prop = lind.propagator([w[0, 0], w[0, 1], 0.0, w[0, 3], w[0, 4], w[0, 5]], [2])
    v = torch.as_tensor(fock_bloch(N, 0)).cuda()
    eps = torch.as_tensor(w[0, 2] + u[0, 2] * wave).cuda().contiguous()
    prop.propagate(v, eps, dt, steps)
    assert rel_vec_err(out[1][1][0], v.cpu().numpy()) <= TOL


def test_full_workload_sampled_against_plain(lib):
    """The 512-instance workload (N in {51,...,301}), 24 steps, in the
    launch configuration the benchmark times (autotuned tiles): 3 sampled
    instances per group against plain single-instance GPU propagation, and
    the middle one against the oracle's density-matrix RK4 (eq. 1)."""
    flush("[batched] 512 instances vs plain (sampled)")
    inst = dimer.batched_instances()
    assert len(inst) == 512
    steps = 24
    bp, groups = dimer_batch(lib, inst, steps)
    lib.autotune_batched(bp, probe_steps=2, use_cache=False)
    for g, (N, idx, _, _, _) in enumerate(groups):
        bp.set_state(g, torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx))))
    bp.run(steps)
    for g, (N, idx, lind, dt, st) in enumerate(groups):
        got = bp.get_state(g).cpu().numpy()
        for j in (0, len(idx) // 2, len(idx) - 1):
            p = inst[idx[j]]
            prop = lind.propagator([1.0, 0.0, p.gamma_eff], [1])
            v = torch.as_tensor(fock_bloch(N, 0)).cuda()
            eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
            prop.propagate(v, eps, dt, steps)
            assert rel_vec_err(got[j], v.cpu().numpy()) <= TOL, (N, j)
        p = inst[idx[len(idx) // 2]]
        ops = dimer.dimer_operators(p)
        rho0 = np.zeros((N, N), complex)
        rho0[0, 0] = 1.0
        rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho0,
                         dimer.drive_table(p, steps=steps)[:, None], dt, steps)
        assert rel_vec_err(got[len(idx) // 2], lb.bloch_vector_sparse(rho)) <= TOL, N


def test_N51_group_full_horizon_against_plain(lib):
    """The N = 51 group of the 512-instance workload (104 instances) over its
    full horizon of 20 periods (25,600 steps) on path 7, the autotuner's
    choice for it, and on path 2 (bitwise equal): the first, middle and last
    instances against plain single-instance GPU propagation of the same
    drive, 1e-12 relative at the end."""
    flush("[batched] N=51 group, 20 periods vs plain")
    inst = [p for p in dimer.batched_instances() if p.N == 51]
    steps = inst[0].steps
    assert steps == 20 * inst[0].steps_per_period
    bp, groups = dimer_batch(lib, inst, steps)
    N, idx, lind, dt, st = groups[0]
    start = torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx)))
    bp.tune(0, 32, 32, 2)
    bp.set_state(0, start)
    bp.run(steps)
    got2 = bp.get_state(0).cpu().numpy()
    bp.tune(0, 64, 32, 7)
    bp.set_state(0, start)
    bp.run(steps)
    got = bp.get_state(0).cpu().numpy()
    assert np.array_equal(got, got2)
    for j in (0, len(idx) // 2, len(idx) - 1):
        p = inst[idx[j]]
        prop = lind.propagator([1.0, 0.0, p.gamma_eff], [1])
        v = torch.as_tensor(fock_bloch(N, 0)).cuda()
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
        prop.propagate(v, eps, dt, steps)
        assert rel_vec_err(got[j], v.cpu().numpy()) <= TOL, j


def test_N301_group_one_period_on_pipelined_path_against_plain(lib):
    """The N = 301 group of the 512-instance workload (109 instances: two
    tiles of 64, the second ragged; 186 rows on the long-row walk) over one
    full drive period (6,400 steps) on path 7: the first, middle and last
    instances against plain single-instance GPU propagation of the same
    drive, 1e-12 relative at the end."""
    flush("[batched] N=301 group, one period on path 7 vs plain")
    inst = [p for p in dimer.batched_instances() if p.N == 301]
    steps = inst[0].steps_per_period
    bp, groups = dimer_batch(lib, inst, steps)
    N, idx, lind, dt, st = groups[0]
    bp.tune(0, 64, 32, 7)
    bp.set_state(0, torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx))))
    bp.run(steps)
    got = bp.get_state(0).cpu().numpy()
    for j in (0, len(idx) // 2, len(idx) - 1):
        p = inst[idx[j]]
        prop = lind.propagator([1.0, 0.0, p.gamma_eff], [1])
        v = torch.as_tensor(fock_bloch(N, 0)).cuda()
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
        prop.propagate(v, eps, dt, steps)
        assert rel_vec_err(got[j], v.cpu().numpy()) <= TOL, j


def test_autotuner_picks_valid_tiling(lib, tmp_path, monkeypatch):
    monkeypatch.setenv("SUN_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    inst = _small_instances()
    bp, groups = dimer_batch(lib, inst, {4: 20, 5: 20})
    chosen = lib.autotune_batched(bp, probe_steps=2)
    for g in range(len(groups)):
        info = bp.info(g)
        assert info["tile"] == chosen[g]["tile"] and info["rows_per_item"] == chosen[g]["rows_per_item"]
        assert chosen[g]["path"] in (0, 2, 3, 4, 5, 7)
    again = lib.autotune_batched(bp)
    assert all(c["cached"] for c in again.values())


def test_bifurcation_scan_against_plain_and_oracle(lib):
    """The U scan behind the stroboscopic population diagram (16 values of
    U at N = 51, ten drive periods, one batched group over [H_J, H_U, H1, L]
    with per-instance U): sampled instances against plain propagation; the
    populations P(n1) = rho_ii at t = 10T from the GPU readout sum to 1, are
    >= 0, depend on U, and for one instance equal the oracle's density-matrix
    RK4 populations."""
    from helpers import bifurcation_batch
    N = 51
    flush(f"[batched] bifurcation scan N={N}")
    inst = dimer.bifurcation_instances(N, count=16)
    steps = inst[0].steps
    bp, lind, basis = bifurcation_batch(lib, inst)
    bp.set_state(0, torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(inst))))
    bp.run(steps)
    V = bp.get_state(0)
    for j in (0, 7, 15):
        q = inst[j]
        prop = lind.propagator([-q.J, q.U_eff, 0.0, q.gamma_eff], [2])
        v = torch.as_tensor(fock_bloch(N, 0)).cuda()
        eps = torch.as_tensor(dimer.drive_table(q, steps=steps)).cuda().contiguous()
        prop.propagate(v, eps, q.dt, steps)
        assert rel_vec_err(V[j].cpu().numpy(), v.cpu().numpy()) <= TOL, j
    P = [basis.density(V[j].contiguous()).diagonal().real.cpu().numpy() for j in range(len(inst))]
    for x in P:
        assert abs(x.sum() - 1.0) <= 1e-12 and x.min() >= -1e-10
    assert np.max(np.abs(P[0] - P[-1])) > 1e-3
    q = inst[7]
    ops = dimer.dimer_operators(q)
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1.0
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [q.gamma_eff], rho0,
                     dimer.drive_table(q, steps=steps)[:, None], q.dt, steps)
    assert rel_vec_err(P[7], np.real(np.diag(rho))) <= TOL


def test_instance_major_path_against_oracle_and_other_paths(lib):
    """Path 4 (instance-major state on a segmented sliced layout: H0 merged,
    the drive and the per-instance rate as segments): every instance of the
    small groups against the dense oracle (1e-12), the other paths (1e-12;
    the row sums are grouped differently, so not bitwise), and path 4 with 2,
    4 and 8 instances per wavefront bitwise equal to each other."""
    flush("[batched] path 4 vs oracle and the row-major paths")
    inst = _small_instances()
    steps = {4: 60, 5: 40}
    bp, groups = dimer_batch(lib, inst, steps)
    starts = [torch.as_tensor(np.stack([fock_bloch(N, j % N) for j in range(len(idx))]))
              for (N, idx, _, _, _) in groups]
    res = {}
    for key, (tile, rows, path) in {"p0": (64, 64, 0), "p4k2": (2, 64, 4), "p4k4": (4, 64, 4),
                                    "p4k8": (8, 64, 4)}.items():
        for g in range(len(groups)):
            bp.tune(g, tile, rows, path)
            bp.set_state(g, starts[g])
        bp.run(1000)
        res[key] = [bp.get_state(g).cpu().numpy() for g in range(len(groups))]
    for g, (N, idx, _, _, st) in enumerate(groups):
        for j, i in enumerate(idx):
            want = _oracle_instance(inst[i], st, fock_bloch(N, j % N))
            assert rel_vec_err(res["p4k4"][g][j], want) <= TOL, (N, j)
            assert rel_vec_err(res["p4k4"][g][j], res["p0"][g][j]) <= TOL
    for key in ("p4k2", "p4k8"):
        for a, b in zip(res[key], res["p4k4"]):
            assert np.array_equal(a, b)


def test_instance_major_path_switch_keeps_state(lib):
    """Switching a group between the row-major paths and path 4 in the middle
    of a run moves its state with it: 20 steps on path 0, 20 on path 4, 20 on
    path 2 equal 60 steps on path 0 (1e-12)."""
    inst = dimer.batched_instances(count=12, sizes=(21,), periods=1)
    bp, groups = dimer_batch(lib, inst, steps={21: 60})
    start = torch.as_tensor(np.stack([fock_bloch(21, 0)] * len(groups[0][1])))
    bp.tune(0, 64, 64, 0)
    bp.set_state(0, start)
    bp.run(60)
    ref = bp.get_state(0).cpu().numpy()
    bp.set_state(0, start)
    bp.run(20)
    bp.tune(0, 8, 64, 4)
    bp.run(20)
    bp.tune(0, 16, 64, 2)
    bp.run(20)
    got = bp.get_state(0).cpu().numpy()
    assert rel_vec_err(got, ref) <= TOL
