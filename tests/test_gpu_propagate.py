"""GPU RK4 propagation against the oracle.

Bar: ||v_gpu - v_oracle||_inf <= 1e-12 ||v_oracle||_inf at every compared
step.  The oracle is classical RK4 on matrices from explicit traces (dense
tier at N = 4, column tier at N = 51) and RK4 on the density matrix itself
(N = 51, 1001), which shares nothing with the Bloch form but the drive table.
"""

import os

import numpy as np
import pytest
import torch

from helpers import flush, rel_vec_err
from oracle import basis as ob, lindblad as lb, propagate as pr
from workloads import dimer, random_ops

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu_system(lib, p, ops):
    b = lib.build_basis(p.N)
    lind, prop = lib.expand_lindbladian(b, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    return b, lind, prop


def _fock_v0(N, i=0):
    rho = np.zeros((N, N), complex)
    rho[i, i] = 1
    return lb.bloch_vector_sparse(rho)


def _run_chunks(prop, v0, eps, dt, chunk, nchunks):
    """GPU propagation in chunks, returning the state after every chunk."""
    v = torch.as_tensor(v0).cuda().clone()
    coef = torch.as_tensor(eps).cuda().contiguous()
    out = []
    for c in range(nchunks):
        prop.propagate(v, coef[2 * c * chunk:], dt, chunk)
        out.append(v.cpu().numpy().copy())
    return out


def test_plain_N4_full_horizon_dense_oracle(lib):
    flush("[propagate] N=4 10 periods")
    p = dimer.plain_config(4)
    ops = dimer.dimer_operators(p)
    F = ob.generators(4)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    K = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    eps = dimer.drive_table(p)
    v0 = _fock_v0(4)
    _, rec = pr.rk4_bloch(G0, [G1], K, v0, eps[:, None], p.dt, p.steps, record_every=p.steps_per_period)
    _, _, prop = _gpu_system(lib, p, ops)
    got = _run_chunks(prop, v0, eps, p.dt, p.steps_per_period, p.periods)
    for t, (a, b) in enumerate(zip(got, rec)):
        assert rel_vec_err(a, b) <= TOL, (t, rel_vec_err(a, b))


def test_plain_N51_against_both_oracle_forms(lib):
    flush("[propagate] N=51 two periods")
    p = dimer.plain_config(51)
    ops = dimer.dimer_operators(p)
    G0 = lb.q_full("H", ops["H0"]) + p.gamma_eff * lb.q_full("L", ops["L"])
    G1 = lb.q_full("H", ops["H1"])
    K = p.gamma_eff * lb.k_vector(ops["L"])
    steps = 2 * p.steps_per_period
    eps = dimer.drive_table(p, steps=steps)
    v0 = _fock_v0(51)
    _, rec = pr.rk4_bloch(G0, [G1], K, v0, eps[:, None], p.dt, steps, record_every=250)
    _, _, prop = _gpu_system(lib, p, ops)
    got = _run_chunks(prop, v0, eps, p.dt, 250, steps // 250)
    for t, (a, b) in enumerate(zip(got, rec)):
        assert rel_vec_err(a, b) <= TOL, (t, rel_vec_err(a, b))
    # density-matrix form, first 250 steps
    rho0 = np.zeros((51, 51), complex)
    rho0[0, 0] = 1
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho0, eps[: 2 * 250 + 1, None], p.dt, 250)
    assert rel_vec_err(got[0], lb.bloch_vector_sparse(rho)) <= TOL


def test_plain_N1001_few_steps_rho_form(lib):
    N = 1001
    flush(f"[propagate] N={N} 3 steps")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    steps = 3
    # a random state near the Fock state (Hermitian, unit trace)
    rng = np.random.default_rng(5)
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    rho0 = rho0 + 1e-3 * (X + X.conj().T)
    rho0 /= np.trace(rho0)
    v0 = lb.bloch_vector_sparse(rho0)
    eps = dimer.drive_table(p, steps=steps)
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho0, eps[:, None], p.dt, steps)
    want = lb.bloch_vector_sparse(rho)
    _, _, prop = _gpu_system(lib, p, ops)
    got = _run_chunks(prop, v0, eps, p.dt, steps, 1)[0]
    assert rel_vec_err(got, want) <= TOL


def test_static_only_and_zero_steps(lib):
    """No time-dependent term (drive folded in with a constant weight), and
    steps = 0 leaves v unchanged."""
    N = 5
    flush("[propagate] static-only N=5")
    H = random_ops.random_hermitian_csr(N, 0.8, seed=3)
    L1 = random_ops.random_complex_csr(N, 0.5, seed=4)
    L2 = random_ops.random_complex_csr(N, 0.5, seed=5)
    F = ob.generators(N)
    G = lb.q_hamiltonian(F, H.to_dense()) + 0.3 * lb.q_dissipator(F, L1.to_dense()) \
        + 0.7 * lb.q_dissipator(F, L2.to_dense())
    K = 0.3 * lb.k_dissipator(F, L1.to_dense()) + 0.7 * lb.k_dissipator(F, L2.to_dense())
    v0 = random_ops.random_vector(N * N - 1, seed=6, scale=0.1)
    steps, dt = 300, 0.01
    want = pr.rk4_bloch(G, [], K, v0, np.zeros((2 * steps + 1, 0)), dt, steps)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [H], [L1, L2])
    prop = lind.propagator([1.0, 0.3, 0.7], [])
    v = torch.as_tensor(v0).cuda().clone()
    prop.propagate(v, None, dt, 0)
    assert np.array_equal(v.cpu().numpy(), v0)
    prop.propagate(v, None, dt, steps)
    assert rel_vec_err(v.cpu().numpy(), want) <= TOL


def test_two_dynamic_terms_time_dependent_rate(lib):
    """Drive on H1 and a time-dependent dissipation rate (dynamic L term)."""
    N = 4
    flush("[propagate] two dynamic terms N=4")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    F = ob.generators(N)
    Q0 = lb.q_hamiltonian(F, ops["H0"].to_dense())
    Q1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    R = lb.q_dissipator(F, ops["L"].to_dense())
    KL = lb.k_dissipator(F, ops["L"].to_dense())
    steps = 400
    t = np.arange(2 * steps + 1) * 0.5 * p.dt
    coef = np.stack([p.E + p.A * np.cos(t), 0.1 * (1 + 0.5 * np.sin(2 * t))], axis=1)
    v0 = _fock_v0(N)
    # oracle with K carried by a term: split as G0 = Q0, terms (Q1, R), K via rate
    v = np.array(v0)
    for n in range(steps):
        def rhs(x, c):
            return Q0 @ x + c[0] * (Q1 @ x) + c[1] * (R @ x + KL)
        c0, ch, c1 = coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]
        k1 = rhs(v, c0)
        k2 = rhs(v + 0.5 * p.dt * k1, ch)
        k3 = rhs(v + 0.5 * p.dt * k2, ch)
        k4 = rhs(v + p.dt * k3, c1)
        v = v + (p.dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
    prop = lind.propagator([1.0, 0.0, 0.0], [1, 2])
    g = torch.as_tensor(v0).cuda().clone()
    prop.propagate(g, torch.as_tensor(coef).cuda().contiguous(), p.dt, steps)
    assert rel_vec_err(g.cpu().numpy(), v) <= TOL


def test_deterministic_and_block_size_invariant(lib):
    """Two runs are bitwise equal; another row-block size gives the same
    numbers (each row is summed by one lane in nonzero order)."""
    p = dimer.plain_config(51)
    ops = dimer.dimer_operators(p)
    _, _, prop = _gpu_system(lib, p, ops)
    eps = torch.as_tensor(dimer.drive_table(p, steps=200)).cuda().contiguous()
    v0 = torch.as_tensor(_fock_v0(51)).cuda()
    outs = []
    for bn, nt, remap in ((1024, 256, False), (1024, 256, False), (512, 64, False), (256, 64, True),
                          (8192, 256, True), (2048, 128, False)):
        prop.tune(bn, nt, remap)
        v = v0.clone()
        prop.propagate(v, eps, p.dt, 200)
        outs.append(v.cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_sliced_layout_matches_stream_layout(lib):
    """The sliced-ELL layout (the default) and the CSR stream layout agree to
    rounding, and the sliced layout is deterministic, for several window
    sizes and long-row thresholds (N = 51 has rows from 5 to 62 nonzeros)."""
    p = dimer.plain_config(51)
    ops = dimer.dimer_operators(p)
    _, _, prop = _gpu_system(lib, p, ops)
    assert prop.layout()["layout"] == "sliced"
    eps = torch.as_tensor(dimer.drive_table(p, steps=300)).cuda().contiguous()
    v0 = torch.as_tensor(_fock_v0(51)).cuda()
    prop.tune(1024, 256, False)
    ref = v0.clone()
    prop.propagate(ref, eps, p.dt, 300)
    ref = ref.cpu().numpy()
    for sigma, long_len, cb, rm in ((1024, 64, 1, 1), (1024, 64, 4, 0), (64, 8, 2, 1), (4096, 1, 1, 0),
                                    (256, 4096, 1, 1)):
        prop.tune_sliced(sigma, long_len, cb, rm)
        v = v0.clone()
        prop.propagate(v, eps, p.dt, 300)
        assert rel_vec_err(v.cpu().numpy(), ref) <= 1e-14, (sigma, long_len, cb)
    a = v0.clone()
    b = v0.clone()
    prop.tune_sliced(1024, 64, 1, 1)
    prop.propagate(a, eps, p.dt, 300)
    prop.propagate(b, eps, p.dt, 300)
    assert torch.equal(a, b)


@pytest.mark.parametrize("split", [1, 2, 4])
def test_sliced_kernel_variants_are_bitwise_identical(lib, split):
    """XCD remapping, load hints, entries per load round and (with one
    wavefront per slice) the row sequence the slices are cut from change only
    which wavefront handles a row and how its loads are issued, never the
    order of a row's sum: results are bitwise equal for a given number of
    wavefronts per slice.  2 or 4 wavefronts per slice sum each row in parts
    and agree with one to rounding."""
    N = 101
    flush(f"[propagate] sliced variants N={N} split={split}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    _, _, prop = _gpu_system(lib, p, ops)
    steps = 40
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    v0 = torch.as_tensor(_fock_v0(N)).cuda()
    prop.tune_sliced(split=split)
    ref = v0.clone()
    prop.propagate(ref, eps, p.dt, steps)
    if split == 1:
        variants = (dict(xcd_remap=False), dict(nontemporal=True), dict(unroll=4), dict(unroll=12),
                    dict(unroll=16, nontemporal=True), dict(unroll=4, xcd_remap=False), dict(pairs=True),
                    dict(pairs=True, xcd_remap=False, unroll=6))
    else:
        variants = (dict(xcd_remap=False), dict(nontemporal=True), dict(unroll=4), dict(unroll=8),
                    dict(unroll=4, xcd_remap=False, nontemporal=True))
    for kw in variants:
        prop.tune_sliced(split=split, **kw)
        v = v0.clone()
        prop.propagate(v, eps, p.dt, steps)
        assert torch.equal(v, ref), kw
    prop.tune_sliced(split=1)
    one = v0.clone()
    prop.propagate(one, eps, p.dt, steps)
    assert rel_vec_err(ref.cpu().numpy(), one.cpu().numpy()) <= 1e-14



@pytest.mark.parametrize("N", [11, 31])
def test_spectral_radius_matches_dense_eigenvalues(lib, N):
    """Power iteration on the GPU against the largest |eigenvalue| of the
    oracle's dense generator, at both ends of the drive range."""
    flush(f"[propagate] spectral radius N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    _, _, prop = _gpu_system(lib, p, ops)
    G0 = (lb.q_full("H", ops["H0"]) + p.gamma_eff * lb.q_full("L", ops["L"])).toarray()
    G1 = lb.q_full("H", ops["H1"]).toarray()
    for eps in (p.E - p.A, p.E + p.A):
        want = np.abs(np.linalg.eigvals(G0 + eps * G1)).max()
        got = prop.spectral_radius([eps], iters=300)
        assert abs(got - want) <= 1e-3 * want, (eps, got, want)


def test_configured_step_counts_are_rk4_stable(lib):
    """The step counts per period of the workloads keep |lambda|max dt <= 2.5
    (inside RK4's stability interval on the imaginary axis, 2*sqrt(2)) over the
    whole drive range: plain N = 51, 101, 301, 1001 and every batched group."""
    for N in (51, 101, 301, 1001):
        flush(f"[propagate] stability N={N}")
        p = dimer.plain_config(N)
        ops = dimer.dimer_operators(p)
        _, _, prop = _gpu_system(lib, p, ops)
        for eps in (p.E - p.A, p.E + p.A):
            lam = prop.spectral_radius([eps], iters=200)
            assert lam * p.dt <= 2.5 * (1 + 1e-3), (N, eps, lam * p.dt)
    inst = dimer.batched_instances()
    for N in sorted({q.N for q in inst}):
        group = [q for q in inst if q.N == N]
        q = max(group, key=lambda x: x.A)
        ops = dimer.dimer_operators(q)
        b = lib.build_basis(N)
        lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
        gmax = max(x.gamma_eff for x in group)
        prop = lind.propagator([1.0, 0.0, gmax], [1])
        lam = prop.spectral_radius([q.E + q.A], iters=200)
        assert lam * q.dt <= 2.5 * (1 + 1e-3), (N, lam * q.dt)


def test_plain_N51_full_horizon(lib):
    """The N = 51 workload over its full horizon, 100 periods (100,000 RK4
    steps), against the oracle's Bloch RK4 at every period end."""
    flush("[propagate] N=51 100 periods")
    p = dimer.plain_config(51)
    ops = dimer.dimer_operators(p)
    G0 = lb.q_full("H", ops["H0"]) + p.gamma_eff * lb.q_full("L", ops["L"])
    G1 = lb.q_full("H", ops["H1"])
    K = p.gamma_eff * lb.k_vector(ops["L"])
    eps = dimer.drive_table(p)
    v0 = _fock_v0(51)
    _, rec = pr.rk4_bloch(G0, [G1], K, v0, eps[:, None], p.dt, p.steps, record_every=p.steps_per_period)
    _, _, prop = _gpu_system(lib, p, ops)
    v = torch.as_tensor(v0).cuda().clone()
    states, _ = prop.record(v, torch.as_tensor(eps).cuda().contiguous(), p.dt, p.steps, p.steps_per_period)
    got = states.cpu().numpy()
    worst = max(rel_vec_err(a, b) for a, b in zip(got, rec))
    flush(f"[propagate] N=51 100 periods: worst relative error {worst:.2e}")
    assert worst <= TOL


def _golden_n1001():
    """Oracle values of tests/golden/dimer_n1001_period.txt (written by
    make_dimer_n1001_period.py from the density-matrix RK4 oracle)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dimer_n1001_period.txt")
    if not os.path.exists(path):
        pytest.skip("tests/golden/dimer_n1001_period.txt not written (make_dimer_n1001_period.py)")
    obs, idx, val = {}, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, k, x = line.split()
            if kind == "obs":
                obs[int(k)] = float(x)
            else:
                idx.append(int(k))
                val.append(float(x))
    return obs, np.asarray(idx), np.asarray(val)


def test_plain_N1001_first_period(lib):
    """The N = 1001 workload over its first period (16,384 steps), in the
    launch configuration the benchmark times: <n1 - n2> every 1024 steps and
    sampled entries of v at the end against the oracle's density-matrix RK4
    (stored values), and what holds for any exact solution and RK4 keeps to
    rounding: purity Tr(rho^2) = 1/N + |v|^2 <= 1, rho positive semidefinite
    (eigenvalues >= -1e-9), <n1 - n2> inside its spectrum."""
    N = 1001
    flush(f"[propagate] N={N} first period")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b, _, prop = _gpu_system(lib, p, ops)
    steps = p.steps_per_period
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    v = torch.as_tensor(_fock_v0(N)).cuda().clone()
    x, x0 = b.observable(ops["H1"])
    _, obs = prop.record(v, eps, p.dt, steps, 1024, states=False, observable=(x, x0))
    assert torch.isfinite(v).all()
    vv = v.cpu().numpy()
    assert vv @ vv <= 1.0 - 1.0 / N + 1e-12
    rho = b.density(v).cpu().numpy()
    assert np.linalg.eigvalsh(rho).min() >= -1e-9
    o = obs.cpu().numpy()
    assert np.all(np.abs(o) <= (N - 1) * (1 + 1e-12))
    g_obs, g_idx, g_val = _golden_n1001()
    want_obs = np.asarray([g_obs[k] for k in range(1, len(o) + 1)])
    e_obs, e_v = rel_vec_err(o, want_obs), rel_vec_err(vv[g_idx], g_val)
    flush(f"[propagate] N={N} first period against stored oracle values: <n1-n2> {e_obs:.2e}, v {e_v:.2e}")
    assert e_obs <= TOL
    assert e_v <= TOL


def test_resident_path_matches_sliced_kernel(lib):
    """The single-workgroup resident path against the sliced stage kernel at
    N = 51: the same row order and roundings, so the same bits (no row of the
    N = 51 generator exceeds 64 entries); also through the recorder, with a
    partial last interval."""
    flush("[propagate] resident vs sliced N=51")
    p = dimer.plain_config(51)
    ops = dimer.dimer_operators(p)
    _, _, prop = _gpu_system(lib, p, ops)
    steps = 250
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    v0 = torch.as_tensor(_fock_v0(51)).cuda()
    prop.tune_resident(True)
    a = v0.clone()
    prop.propagate(a, eps, p.dt, steps)              # one launch for all steps
    ra, _ = prop.record(v0.clone(), eps, p.dt, steps, 60)
    prop.tune_sliced(long_len=64, split=1)           # four launches per step, every row on a lane
    b = v0.clone()
    prop.propagate(b, eps, p.dt, steps)
    rb, _ = prop.record(v0.clone(), eps, p.dt, steps, 60)
    assert torch.equal(a, b)
    assert torch.equal(ra, rb)
    prop.tune_resident(True)
    c = v0.clone()
    prop.propagate(c, eps, p.dt, steps)
    assert torch.equal(a, c)
    big = dimer.plain_config(101)
    _, _, prop101 = _gpu_system(lib, big, dimer.dimer_operators(big))
    with pytest.raises(lib.SunError):
        prop101.tune_resident(True)                  # 4 (M + 1) doubles exceed the LDS



def test_periodic_steady_state_N4(lib):
    """300 drive periods (60,000 steps) of the N = 4 workload on the GPU from
    the Fock state land on the fixed point of the oracle's one-period RK4
    map, v* = (1 - Phi)^-1 phi (computed by linear algebra, not by stepping)."""
    flush("[propagate] periodic steady state N=4")
    p = dimer.plain_config(4)
    ops = dimer.dimer_operators(p)
    F = ob.generators(4)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    K = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    S = p.steps_per_period
    eps1 = dimer.drive_table(p, steps=S)[:, None]
    Phi = np.stack([pr.rk4_bloch(G0, [G1], None, np.eye(15)[j], eps1, p.dt, S) for j in range(15)], axis=1)
    phi = pr.rk4_bloch(G0, [G1], K, np.zeros(15), eps1, p.dt, S)
    vstar = np.linalg.solve(np.eye(15) - Phi, phi)
    _, _, prop = _gpu_system(lib, p, ops)
    periods = 300
    eps = torch.as_tensor(dimer.drive_table(p, steps=periods * S)).cuda().contiguous()
    v = torch.as_tensor(_fock_v0(4)).cuda().clone()
    prop.propagate(v, eps, p.dt, periods * S)
    assert rel_vec_err(v.cpu().numpy(), vstar) <= TOL


@pytest.mark.parametrize("N", [4, 51])
def test_square_wave_two_channels_time_dependent_rate(lib, N):
    """Square-wave drive eps = E + A theta(t) (paper Sec. III), a second
    dissipation channel L2 = b1^+ b2 whose rate varies in time (a
    time-dependent dissipator term: its eq. 10 matrix and eq. 11 vector scale
    together), against the oracle's density-matrix RK4 with a rate table."""
    flush(f"[propagate] square wave, two channels, time-dependent rate N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    s = np.sqrt((np.arange(N - 1) + 1.0) * (N - 1.0 - np.arange(N - 1)))
    L2 = dimer.ZCSR.from_diagonals(N, {-1: s})
    steps = 2 * p.steps_per_period if N <= 6 else 400
    eps = dimer.drive_table_square(p, steps=steps)
    t = np.arange(2 * steps + 1) * 0.5 * p.dt
    g2 = 0.3 * p.gamma_eff * (1.0 + 0.5 * np.sin(2.0 * t))
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1.0
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"], L2], [p.gamma_eff, 0.0], rho0, eps[:, None], p.dt, steps,
                     rates=np.stack([np.full_like(t, p.gamma_eff), g2], axis=1))
    want = lb.bloch_vector_sparse(rho)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"], L2])
    prop = lind.propagator([1.0, 0.0, p.gamma_eff, 0.0], [1, 3])
    v = torch.as_tensor(_fock_v0(N)).cuda().clone()
    prop.propagate(v, torch.as_tensor(np.stack([eps, g2], axis=1)).cuda().contiguous(), p.dt, steps)
    assert rel_vec_err(v.cpu().numpy(), want) <= TOL


def test_segmented_layout_two_and_three_dynamic_terms(lib):
    """N = 101 with 2 and 3 time-dependent terms (square-wave drive, a second
    channel with a time-dependent rate, a modulated interaction): the
    segmented sliced layout, default at this size, against the CSR stream
    layout (1e-14) and, for two terms, against the oracle's density-matrix
    RK4 with a rate table."""
    N = 101
    flush(f"[propagate] segmented layout N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    s = np.sqrt((np.arange(N - 1) + 1.0) * (N - 1.0 - np.arange(N - 1)))
    L2 = dimer.ZCSR.from_diagonals(N, {-1: s})
    steps = 150
    eps = dimer.drive_table_square(p, steps=steps)
    t = np.arange(2 * steps + 1) * 0.5 * p.dt
    g2 = 0.3 * p.gamma_eff * (1.0 + 0.5 * np.sin(2.0 * t))
    u = p.U_eff * (1.0 + 0.2 * np.cos(3.0 * t))
    b = lib.build_basis(N)
    HJ = ops["HJ"].scaled(-p.J)
    lind = lib.Lindbladian(b, [HJ, ops["HU"], ops["H1"]], [ops["L"], L2])
    v0 = torch.as_tensor(_fock_v0(N)).cuda()
    for dyn, table, w in (([2, 4], np.stack([eps, g2], axis=1), [1.0, p.U_eff, 0.0, p.gamma_eff, 0.0]),
                          ([2, 4, 1], np.stack([eps, g2, u], axis=1), [1.0, 0.0, 0.0, p.gamma_eff, 0.0])):
        prop = lind.propagator(w, dyn)
        assert prop.layout()["layout"] == "sliced-segmented"
        coef = torch.as_tensor(table).cuda().contiguous()
        a = v0.clone()
        prop.propagate(a, coef, p.dt, steps)
        prop.tune(1024, 256, True)
        assert prop.layout()["layout"] == "stream"
        c = v0.clone()
        prop.propagate(c, coef, p.dt, steps)
        assert rel_vec_err(a.cpu().numpy(), c.cpu().numpy()) <= 1e-14, dyn
        if len(dyn) == 2:
            rho0 = np.zeros((N, N), complex)
            rho0[0, 0] = 1.0
            rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"], L2], [p.gamma_eff, 0.0], rho0, eps[:, None], p.dt, steps,
                             rates=np.stack([np.full_like(t, p.gamma_eff), g2], axis=1))
            assert rel_vec_err(a.cpu().numpy(), lb.bloch_vector_sparse(rho)) <= TOL


def _graph_cases(lib):
    """(name, propagator, coefficient table (2*steps+1 rows), dt, steps) for
    the stream layout (N = 51), the sliced layout (N = 101) and the segmented
    layout (N = 101, two time-dependent terms)."""
    out = []
    steps = 200                      # three 64-step chunks and 8 direct steps
    for N in (51, 101):
        p = dimer.plain_config(N)
        ops = dimer.dimer_operators(p)
        b = lib.build_basis(N)
        lind, prop = lib.expand_lindbladian(b, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        if N == 51:
            prop.tune(1024, 256, True)
        eps = torch.as_tensor(dimer.drive_table(p, steps=3 * steps)).cuda().contiguous()
        out.append((f"N{N}-{prop.layout()['layout']}", prop, eps, p.dt, steps, N))
    N = 101
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    s = np.sqrt((np.arange(N - 1) + 1.0) * (N - 1.0 - np.arange(N - 1)))
    L2 = dimer.ZCSR.from_diagonals(N, {-1: s})
    t = np.arange(2 * 3 * steps + 1) * 0.5 * p.dt
    table = np.stack([dimer.drive_table_square(p, steps=3 * steps), 0.3 * p.gamma_eff * (1.0 + 0.5 * np.sin(2.0 * t))],
                     axis=1)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["HJ"].scaled(-p.J), ops["HU"], ops["H1"]], [ops["L"], L2])
    prop = lind.propagator([1.0, p.U_eff, 0.0, p.gamma_eff, 0.0], [2, 4])
    out.append(("N101-segmented", prop, torch.as_tensor(table).cuda().contiguous(), p.dt, steps, N))
    return out


def test_graph_replay_equals_direct_launches(lib):
    """sun_propagate with HIP-graph replay of 64-step chunks (the default at
    these sizes) against direct launches, bitwise, on three layouts: three
    consecutive calls over successive parts of the coefficient table (every
    replay refreshes the chunk's coefficient rows), with eager PyTorch work
    and synchronisations between the calls; then a different dt (recapture)
    and a re-layout (recapture)."""
    for name, prop, coef, dt, steps, N in _graph_cases(lib):
        flush(f"[propagate] graph replay {name}")
        nd = coef.shape[1] if coef.dim() == 2 else 1
        v0 = torch.as_tensor(_fock_v0(N)).cuda()
        ref, got = [], []
        for mode, out in ((0, ref), (1, got)):
            prop.use_graphs(mode)
            v = v0.clone()
            for k in range(3):
                part = coef[2 * k * steps: 2 * (k + 1) * steps + 1].contiguous()
                prop.propagate(v, part, dt, steps)
                out.append(v.clone())
                junk = torch.randn(4096, device="cuda").sum()        # eager work between replays
                torch.cuda.synchronize()
                assert torch.isfinite(junk)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), name
        part = coef[: 2 * steps + 1].contiguous()
        outs = []
        for mode in (0, 1):
            prop.use_graphs(mode)
            v = v0.clone()
            prop.propagate(v, part, 0.5 * dt, steps)               # new step size: recaptured
            outs.append(v)
        assert torch.equal(outs[0], outs[1]), name
        prop.use_graphs(1)
        if name.startswith("N101-sliced"):
            prop.tune_sliced(sigma=2048)                            # re-layout: recaptured
            outs = []
            for mode in (1, 0):
                prop.use_graphs(mode)
                v = v0.clone()
                prop.propagate(v, part, dt, steps)
                outs.append(v)
            assert torch.equal(outs[0], outs[1]), name
            assert rel_vec_err(outs[0].cpu().numpy(), ref[0].cpu().numpy()) <= 1e-14
