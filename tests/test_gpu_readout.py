"""GPU readout (eq. 5 and expectation values) and recorded propagation
against the oracle.

Bars: rho and Tr(rho X) within 1e-12 of the largest entry (the diagonal of
rho sums up to N-1 terms, in another order than the oracle); recorded states
bitwise equal to chunked propagation (same kernels, same order); recorded
observables within 1e-12 relative of the oracle's RK4 trajectory.
"""

import numpy as np
import pytest
import torch

from helpers import fock_bloch, flush, rel_vec_err
from oracle import basis as ob, lindblad as lb, propagate as pr
from workloads import dimer, random_ops

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [2, 4, 51, 1001])
def test_density_matches_oracle(lib, N):
    flush(f"[readout] density N={N}")
    M = N * N - 1
    v = random_ops.random_vector(M, seed=100 + N, scale=0.1)
    b = lib.build_basis(N)
    got = b.density(torch.as_tensor(v).cuda()).cpu().numpy()
    want = lb.density_from_bloch_dense(v, N)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # exactly Hermitian by construction; unit trace up to rounding
    np.testing.assert_array_equal(got, got.conj().T)
    assert abs(np.trace(got) - 1.0) <= 1e-12


def test_density_of_fock_state_is_projector(lib):
    N = 301
    b = lib.build_basis(N)
    for i in (0, 7, N - 1):
        rho = b.density(torch.as_tensor(fock_bloch(N, i)).cuda()).cpu().numpy()
        want = np.zeros((N, N), complex)
        want[i, i] = 1.0
        assert np.max(np.abs(rho - want)) <= 1e-14


def test_expect_strided_stack_matches_oracle(lib):
    """Tr(rho_i X) for a non-Hermitian X with a trace, over a strided stack
    of Bloch vectors."""
    N = 5
    M = N * N - 1
    flush("[readout] expect N=5")
    F = ob.generators(N)
    X = random_ops.random_complex_csr(N, 0.7, seed=11, traceless=False)
    Xd = X.to_dense()
    V = np.stack([random_ops.random_vector(M, seed=200 + i, scale=0.2) for i in range(6)])
    buf = torch.zeros((6, M + 3), dtype=torch.float64, device="cuda")
    buf[:, :M] = torch.as_tensor(V).cuda()
    b = lib.build_basis(N)
    got = b.expect(buf[:, :M], X).cpu().numpy()
    want = np.array([np.trace(lb.density_from_bloch(F, v) @ Xd) for v in V])
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    one = b.expect(torch.as_tensor(V[2]).cuda(), X).item()
    assert abs(one - want[2]) <= 1e-12 * np.max(np.abs(want))


def test_population_imbalance_of_initial_dimer_state(lib):
    """<n1 - n2> of rho0 = |0, N-1><0, N-1| is -(N-1) (initial state of the
    dimer workload); read out at N = 1001 through the expansion of H1."""
    N = 1001
    flush(f"[readout] <n1-n2>(0) N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    e0 = np.zeros(N)
    e0[0] = 1.0
    v0 = b.expand(dimer.ZCSR.from_diagonals(N, {0: e0}))[0].real.contiguous()
    val = b.expect(v0, ops["H1"]).item()
    assert abs(val.real + (N - 1)) <= 1e-12 * (N - 1) and val.imag == 0.0


def _dimer_system(lib, N):
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    lind, prop = lib.expand_lindbladian(b, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    return p, ops, b, prop


def test_record_matches_chunked_propagation_and_oracle(lib):
    N = 51
    flush(f"[readout] record N={N}")
    p, ops, b, prop = _dimer_system(lib, N)
    steps, every = 130, 20          # 6 records, 10 trailing steps
    eps = dimer.drive_table(p, steps=steps)
    coef = torch.as_tensor(eps).cuda().contiguous()
    v0 = fock_bloch(N, 0)
    x, x0 = b.observable(ops["H1"])
    v = torch.as_tensor(v0).cuda().clone()
    states, obs = prop.record(v, coef, p.dt, steps, every, states=True, observable=(x, x0))
    assert states.shape == (6, N * N - 1) and obs.shape == (6,)
    # same kernels in the same order as chunked calls: bitwise equal
    w = torch.as_tensor(v0).cuda().clone()
    for r in range(6):
        prop.propagate(w, coef[2 * r * every:], p.dt, every)
        assert torch.equal(states[r], w), r
    prop.propagate(w, coef[2 * 6 * every:], p.dt, steps - 6 * every)
    assert torch.equal(v, w)
    # observable against the oracle's trajectory
    G0 = lb.q_full("H", ops["H0"]) + p.gamma_eff * lb.q_full("L", ops["L"])
    G1 = lb.q_full("H", ops["H1"])
    K = p.gamma_eff * lb.k_vector(ops["L"])
    _, rec = pr.rk4_bloch(G0, [G1], K, v0, eps[: 2 * 6 * every + 1, None], p.dt, 6 * every, record_every=every)
    c = lb.bloch_coords(ops["H1"].to_dense()).real
    want = np.array([c @ r for r in rec])
    assert rel_vec_err(obs.cpu().numpy(), want) <= 1e-12
    # the readout entry point gives the same values from the recorded states
    again = b.expect(states, ops["H1"]).real.cpu().numpy()
    assert rel_vec_err(again, want) <= 1e-12


def test_record_observable_only_at_N1001(lib):
    """Large-M path of the recorder (two-level reduction), observable only,
    against per-step readouts of chunked propagation."""
    N = 1001
    flush(f"[readout] record N={N}")
    p, ops, b, prop = _dimer_system(lib, N)
    steps, every = 12, 4
    coef = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    x, x0 = b.observable(ops["H1"])
    v = torch.as_tensor(fock_bloch(N, 0)).cuda()
    w = v.clone()
    st, obs = prop.record(v, coef, p.dt, steps, every, states=False, observable=(x, x0))
    assert st is None
    for r in range(3):
        prop.propagate(w, coef[2 * r * every:], p.dt, every)
        ref = b.expect(w, ops["H1"]).real.item()
        assert abs(obs[r].item() - ref) <= 1e-12 * abs(ref), r
    assert torch.equal(v, w)
