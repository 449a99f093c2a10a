"""Pins of the oracle's time propagation.

* One classical RK4 step of a time-independent affine ODE equals the degree-4
  Taylor polynomial of the augmented generator (textbook property of RK4).
* RK4 converges to the matrix exponential with order four.
* RK4 on the density matrix (eq. 1) and on the Bloch vector (eq. 9) give the
  same trajectory (the map rho <-> v of eq. 5 is affine and fixed).
"""

import math

import numpy as np
import pytest

from oracle import basis, lindblad as lb, propagate as pr
from workloads import dimer, random_ops


def _dimer_system(N):
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    F = basis.generators(N)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    K = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    return p, ops, F, G0, G1, K


def test_rk4_step_is_taylor_polynomial():
    p, ops, F, G0, G1, K = _dimer_system(4)
    G = G0 + 1.3 * G1
    A = pr.augmented(G, K)
    dt = 0.05
    z = dt * A
    P4 = np.eye(A.shape[0])
    term = np.eye(A.shape[0])
    for k in range(1, 5):
        term = term @ z / k
        P4 = P4 + term
    v0 = np.random.default_rng(1).standard_normal(G.shape[0]) * 0.1
    coef = np.full((3, 1), 1.3)
    v1 = pr.rk4_bloch(G0, [G1], K, v0, coef, dt, 1)
    np.testing.assert_allclose(v1, (P4 @ np.concatenate([v0, [1.0]]))[:-1], atol=1e-14)


def test_rk4_fourth_order_convergence():
    p, ops, F, G0, G1, K = _dimer_system(4)
    G = G0 + 0.7 * G1
    v0 = np.random.default_rng(2).standard_normal(G.shape[0]) * 0.1
    t = 1.0
    exact = pr.expm_affine(G, K, v0, t)
    errs = []
    for steps in (20, 40, 80):
        coef = np.full((2 * steps + 1, 1), 0.7)
        v = pr.rk4_bloch(G0, [G1], K, v0, coef, t / steps, steps)
        errs.append(np.max(np.abs(v - exact)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.0 < r1 < 18.0 and 14.0 < r2 < 18.0, (errs, r1, r2)


@pytest.mark.parametrize("N", [4, 5])
def test_rho_form_equals_bloch_form(N):
    p, ops, F, G0, G1, K = _dimer_system(N)
    steps = 60
    coef = dimer.drive_table(p, steps=steps)[:, None]
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    v0 = lb.bloch_vector(F, rho0)
    v = pr.rk4_bloch(G0, [G1], K, v0, coef, p.dt, steps)
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho0, coef, p.dt, steps)
    np.testing.assert_allclose(lb.bloch_vector(F, rho), v, atol=1e-13)
    assert abs(np.trace(rho) - 1) < 1e-13


def test_bloch_rk4_sparse_equals_dense():
    import scipy.sparse as sp
    p, ops, F, G0, G1, K = _dimer_system(4)
    steps = 30
    coef = dimer.drive_table(p, steps=steps)[:, None]
    v0 = random_ops.random_vector(15, seed=4, scale=0.2)
    a = pr.rk4_bloch(G0, [G1], K, v0, coef, p.dt, steps)
    b = pr.rk4_bloch(sp.csr_matrix(G0), [sp.csr_matrix(G1)], K, v0, coef, p.dt, steps)
    np.testing.assert_allclose(a, b, atol=1e-14)


def _one_period_map(p):
    """The one-period RK4 map of the driven N = 4 dimer as v -> Phi v + phi
    (RK4 on an affine ODE is affine in the state), from the dense generators."""
    ops = dimer.dimer_operators(p)
    F = basis.generators(p.N)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    K = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    S = p.steps_per_period
    eps = dimer.drive_table(p, steps=S)[:, None]
    M = p.N * p.N - 1
    Phi = np.stack([pr.rk4_bloch(G0, [G1], None, np.eye(M)[j], eps, p.dt, S) for j in range(M)], axis=1)
    phi = pr.rk4_bloch(G0, [G1], K, np.zeros(M), eps, p.dt, S)
    return F, G0, G1, K, eps, Phi, phi


def test_driven_dimer_periodic_steady_state():
    """With A != 0 the one-period RK4 map has one attracting fixed point v*
    (spectral radius of Phi below 1): it is a valid state (rho* >= 0, trace
    1), the trajectory from the Fock state reaches it after many periods, and
    over one period from v* the population imbalance oscillates with the
    drive and comes back (the asymptotic state is T-periodic, Sec. III)."""
    p = dimer.plain_config(4)
    F, G0, G1, K, eps, Phi, phi = _one_period_map(p)
    M = Phi.shape[0]
    assert np.abs(np.linalg.eigvals(Phi)).max() < 0.99
    vstar = np.linalg.solve(np.eye(M) - Phi, phi)
    rho = lb.density_from_bloch(F, vstar)
    np.testing.assert_allclose(np.trace(rho), 1.0, atol=1e-13)
    assert np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min() > -1e-12
    v0 = lb.bloch_vector(F, np.diag([1.0, 0.0, 0.0, 0.0]).astype(complex))
    v = v0
    for _ in range(300):
        v = Phi @ v + phi
    assert np.max(np.abs(v - vstar)) < 1e-12
    # the same through the time stepper itself, from the Fock state
    S = p.steps_per_period
    eps_long = dimer.drive_table(p, steps=150 * S)[:, None]
    vt = pr.rk4_bloch(G0, [G1], K, v0, eps_long, p.dt, 150 * S)
    assert np.max(np.abs(vt - vstar)) < 1e-10
    _, rec = pr.rk4_bloch(G0, [G1], K, vstar, eps, p.dt, S, record_every=S // 8)
    # <n1 - n2> = Tr(X)/N + v . x with X = diag(-3, -1, 1, 3), Tr X = 0
    n12 = np.real(lb.trace_against(F, np.diag([-3.0, -1.0, 1.0, 3.0]).astype(complex)))
    obs = np.array([x @ n12 for x in rec])
    assert np.max(np.abs(rec[-1] - vstar)) < 1e-12
    assert obs.max() - obs.min() > 1e-3


def test_time_dependent_rates_rho_form_equals_bloch_form():
    """Two dissipation channels, the second with a time-dependent rate, and a
    square-wave drive: the density-matrix RK4 with a rate table and the
    Bloch RK4 with the channel's eq. 10 matrix and eq. 11 vector as one
    time-dependent term give the same trajectory (RK4 commutes with the
    affine map rho <-> v), and both differ from the constant-rate run."""
    N = 4
    p = dimer.plain_config(N)
    p.steps_per_period = 40
    ops = dimer.dimer_operators(p)
    L2 = random_ops.random_complex_csr(N, 0.5, seed=77)
    F = basis.generators(N)
    steps = 100
    eps = dimer.drive_table_square(p, steps=steps)
    assert eps[0] == p.E + p.A and eps[2 * p.steps_per_period - 1] == p.E - p.A
    assert eps[p.steps_per_period] == p.E - p.A and eps[2 * p.steps_per_period] == p.E + p.A
    t = np.arange(2 * steps + 1) * 0.5 * p.dt
    g2 = 0.05 * (1.0 + 0.5 * np.sin(2.0 * t))
    rho0 = np.zeros((N, N), complex)
    rho0[1, 1] = 1.0
    rates = np.stack([np.full_like(t, p.gamma_eff), g2], axis=1)
    rho = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"], L2], [p.gamma_eff, 0.05], rho0, eps[:, None], p.dt, steps,
                     rates=rates)
    G0 = lb.q_hamiltonian(F, ops["H0"].to_dense()) + p.gamma_eff * lb.q_dissipator(F, ops["L"].to_dense())
    K0 = p.gamma_eff * lb.k_dissipator(F, ops["L"].to_dense())
    G1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    R2 = lb.q_dissipator(F, L2.to_dense())
    K2 = lb.k_dissipator(F, L2.to_dense())
    v = pr.rk4_bloch(G0, [G1, R2], K0, lb.bloch_vector(F, rho0), np.stack([eps, g2], axis=1), p.dt, steps,
                     Ks=[None, K2])
    np.testing.assert_allclose(lb.bloch_vector(F, rho), v, atol=1e-13)
    rho_c = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"], L2], [p.gamma_eff, 0.05], rho0, eps[:, None], p.dt, steps)
    assert np.max(np.abs(rho_c - rho)) > 1e-4
