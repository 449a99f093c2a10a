"""Pins of the oracle's gradient of the time-averaged observable.

The discrete adjoint is checked against central finite differences of the
objective (h = 1e-6) and against forward-mode (tangent-linear) sensitivities,
which follow a different route through the same RK4 map.
"""

import numpy as np
import pytest

from oracle import adjoint as adj, basis, lindblad as lb
from workloads import dimer


def _terms(N, A=1.5, gamma=0.1, U=0.5, steps=40):
    p = dimer.adjoint_config(N)
    p.A, p.gamma, p.U = A, gamma, U
    ops = dimer.dimer_operators(p)
    F = basis.generators(N)
    QJ = lb.q_hamiltonian(F, ops["HJ"].to_dense())
    QU = lb.q_hamiltonian(F, ops["HU"].to_dense())
    Q1 = lb.q_hamiltonian(F, ops["H1"].to_dense())
    R = lb.q_dissipator(F, ops["L"].to_dense())
    KL = lb.k_dissipator(F, ops["L"].to_dense())
    Gs = [QJ, QU, Q1, R]
    Ks = [None, None, None, KL]
    eps = dimer.drive_table(p, steps=steps)
    deps = dimer.drive_table_dA(p, steps=steps)
    coef = np.zeros((2 * steps + 1, 4))
    coef[:, 0] = -p.J
    coef[:, 1] = p.U_eff
    coef[:, 2] = eps
    coef[:, 3] = p.gamma_eff
    dcoef = np.zeros((2 * steps + 1, 4, 3))        # theta = (A, gamma, U)
    dcoef[:, 2, 0] = deps
    dcoef[:, 3, 1] = p.gamma_scale
    dcoef[:, 1, 2] = p.U_scale
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    v0 = lb.bloch_vector(F, rho0)
    X = np.diag(2.0 * np.arange(N) - (N - 1)).astype(complex)
    c = lb.bloch_vector(F, X)           # Tr(F_j (n1 - n2))
    return p, Gs, Ks, coef, dcoef, v0, c


@pytest.mark.parametrize("N", [4, 6])
def test_adjoint_equals_tangent_linear(N):
    steps, S = 40, 10
    p, Gs, Ks, coef, dcoef, v0, c = _terms(N, steps=steps)
    J1, g1 = adj.adjoint_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    J2, g2 = adj.tangent_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    assert abs(J1 - J2) <= 1e-13 * abs(J1)
    np.testing.assert_allclose(g1, g2, rtol=1e-11)


def test_adjoint_matches_central_differences():
    N, steps, S = 4, 40, 10
    h = 1e-6
    base = dict(A=1.5, gamma=0.1, U=0.5)
    p, Gs, Ks, coef, dcoef, v0, c = _terms(N, steps=steps, **base)
    _, g = adj.adjoint_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    for i, name in enumerate(("A", "gamma", "U")):
        vals = []
        for sgn in (+1, -1):
            kw = dict(base)
            kw[name] += sgn * h
            q, Gs2, Ks2, coef2, _, v02, c2 = _terms(N, steps=steps, **kw)
            vals.append(adj.objective(Gs2, Ks2, coef2, v02, c2, q.dt, steps, S))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-12, (name, fd, g[i])


def test_planted_sign_error_is_caught():
    """A sign slip in one adjoint term must break the tangent-linear match."""
    N, steps, S = 4, 20, 5
    p, Gs, Ks, coef, dcoef, v0, c = _terms(N, steps=steps)
    bad = [G.copy() for G in Gs]
    bad[3] = -bad[3].T.T            # flip the dissipator only in the adjoint run
    _, g1 = adj.adjoint_gradient(bad, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    _, g2 = adj.tangent_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    assert not np.allclose(g1, g2, rtol=1e-6)


def _rho_route(N, steps, S, A=1.5, gamma=0.1, U=0.5):
    """The same problem for the density-matrix route: terms H_J, H_U, H1 and L
    with their coefficient tables, rho0 = |0><0| and X = n1 - n2."""
    p = dimer.adjoint_config(N)
    p.A, p.gamma, p.U = A, gamma, U
    ops = dimer.dimer_operators(p)
    terms = [("H", ops["HJ"]), ("H", ops["HU"]), ("H", ops["H1"]), ("L", ops["L"])]
    coef = np.zeros((2 * steps + 1, 4))
    coef[:, 0] = -p.J
    coef[:, 1] = p.U_eff
    coef[:, 2] = dimer.drive_table(p, steps=steps)
    coef[:, 3] = p.gamma_eff
    dcoef = np.zeros((2 * steps + 1, 4, 3))
    dcoef[:, 2, 0] = dimer.drive_table_dA(p, steps=steps)
    dcoef[:, 3, 1] = p.gamma_scale
    dcoef[:, 1, 2] = p.U_scale
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    X = np.diag(2.0 * np.arange(N) - (N - 1)).astype(complex)
    return p, terms, coef, dcoef, rho0, X


@pytest.mark.parametrize("N", [4, 5])
def test_density_matrix_tangent_equals_bloch_adjoint(N):
    """The density-matrix route (eq. 1, no SU(N) basis) against the Bloch-form
    discrete adjoint built from explicit traces: same J and gradient, since
    RK4 commutes with the affine map of eq. 5 (X = n1 - n2 is traceless)."""
    steps, S = 40, 10
    p, Gs, Ks, coef, dcoef, v0, c = _terms(N, steps=steps)
    J1, g1 = adj.adjoint_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)
    _, terms, coef2, dcoef2, rho0, X = _rho_route(N, steps, S)
    J2, g2 = adj.tangent_gradient_rho(terms, coef2, dcoef2, rho0, X, p.dt, steps, S)
    assert abs(J1 - J2) <= 1e-12 * abs(J1)
    np.testing.assert_allclose(g2, g1, rtol=1e-10)


def test_density_matrix_tangent_matches_central_differences():
    """Central differences of the density-matrix objective itself (h = 1e-6)."""
    N, steps, S = 4, 40, 10
    h = 1e-6
    base = dict(A=1.5, gamma=0.1, U=0.5)
    p, terms, coef, dcoef, rho0, X = _rho_route(N, steps, S, **base)
    _, g = adj.tangent_gradient_rho(terms, coef, dcoef, rho0, X, p.dt, steps, S)
    zero = np.zeros((2 * steps + 1, 4, 3))
    for i, name in enumerate(("A", "gamma", "U")):
        vals = []
        for sgn in (+1, -1):
            kw = dict(base)
            kw[name] += sgn * h
            q, terms2, coef2, _, rho02, X2 = _rho_route(N, steps, S, **kw)
            vals.append(adj.tangent_gradient_rho(terms2, coef2, zero, rho02, X2, q.dt, steps, S)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-12, (name, fd, g[i])
