"""Pins of the oracle's Bloch-form generator (Q, R, K by traces).

Fixed points used: the textbook qubit Bloch equations (Larmor precession and
amplitude damping), skew-symmetry of the unitary part (Sec. II), the closed
form of a diagonal Hamiltonian, the kernel of the dense N^2 x N^2 Liouvillian
built by Kronecker products (no basis involved), and the Bloch vector of a
pure Fock state.
"""

import math

import numpy as np
import pytest

from oracle import basis, lindblad as lb
from workloads import dimer, random_ops


def test_larmor_precession_qubit():
    F = basis.generators(2)
    w0 = 1.7
    H = 0.5 * w0 * np.diag([1.0, -1.0]).astype(complex)
    Q = lb.q_hamiltonian(F, H)
    np.testing.assert_allclose(Q, [[0, -w0, 0], [w0, 0, 0], [0, 0, 0]], atol=1e-14)


def test_amplitude_damping_qubit_closed_form():
    F = basis.generators(2)
    w0, g = 1.3, 0.7
    H = 0.5 * w0 * np.diag([1.0, -1.0]).astype(complex)
    L = np.zeros((2, 2), complex)
    L[1, 0] = 1.0                          # |2><1|: decay from level 1 to 2
    G = lb.q_hamiltonian(F, H) + g * lb.q_dissipator(F, L)
    K = g * lb.k_dissipator(F, L)
    np.testing.assert_allclose(G, [[-g / 2, -w0, 0], [w0, -g / 2, 0], [0, 0, -g]], atol=1e-14)
    np.testing.assert_allclose(K, [0, 0, -g / math.sqrt(2)], atol=1e-14)
    # steady state: <sigma_z> = sqrt(2) v_z = -1 (all population in level 2)
    v_inf = np.linalg.solve(G, -K)
    assert abs(math.sqrt(2) * v_inf[2] + 1.0) < 1e-14


@pytest.mark.parametrize("N", [3, 4, 5])
def test_unitary_part_skew_symmetric(N):
    F = basis.generators(N)
    H = random_ops.random_hermitian_csr(N, 0.7, seed=N).to_dense()
    Q = lb.q_hamiltonian(F, H)
    np.testing.assert_allclose(Q.T, -Q, atol=1e-13)


@pytest.mark.parametrize("N", [3, 5])
def test_diagonal_hamiltonian_closed_form(N):
    F = basis.generators(N)
    x = np.random.default_rng(7).standard_normal(N)
    Q = lb.q_hamiltonian(F, np.diag(x).astype(complex))
    P = N * (N - 1) // 2
    expect = np.zeros_like(Q)
    p = 0
    for j in range(N):
        for k in range(j + 1, N):
            expect[P + p, p] = x[j] - x[k]     # q(J_jk, S_jk)
            expect[p, P + p] = -(x[j] - x[k])  # q(S_jk, J_jk)
            p += 1
    np.testing.assert_allclose(Q, expect, atol=1e-13)


@pytest.mark.parametrize("N", [3, 4])
def test_bloch_generator_matches_dense_liouvillian(N):
    """(Q + R) v + K is the Bloch vector of L(rho(v)), L from Kronecker products."""
    F = basis.generators(N)
    H = random_ops.random_hermitian_csr(N, 0.8, seed=11).to_dense()
    L = random_ops.random_complex_csr(N, 0.8, seed=12).to_dense()
    g = 0.37
    G = lb.q_hamiltonian(F, H) + g * lb.q_dissipator(F, L)
    K = g * lb.k_dissipator(F, L)
    v = np.random.default_rng(3).standard_normal(N * N - 1) * 0.1
    rho = lb.density_from_bloch(F, v)
    Lv = lb.liouvillian(H, [L], [g])
    drho = lb.unvec(Lv @ lb.vec(rho), N)
    np.testing.assert_allclose(G @ v + K, lb.bloch_vector(F, drho), atol=1e-12)


def test_unital_dissipator_has_zero_free_vector():
    N = 4
    F = basis.generators(N)
    Lh = random_ops.random_hermitian_csr(N, 0.8, seed=5, traceless=True).to_dense()
    np.testing.assert_allclose(lb.k_dissipator(F, Lh), 0, atol=1e-13)
    Ln = random_ops.random_complex_csr(N, 0.8, seed=6).to_dense()
    assert np.max(np.abs(lb.k_dissipator(F, Ln))) > 1e-3


def test_dimer_asymptotic_state_is_liouvillian_kernel():
    """Static drive (A = 0): v_inf = -(G)^-1 K equals the Bloch vector of the
    normalised kernel of the dense Liouvillian; it is a valid state and not
    the maximally mixed one (Sec. III: L is non-Hermitian)."""
    p = dimer.plain_config(4)
    ops = dimer.dimer_operators(p)
    N = p.N
    F = basis.generators(N)
    H = ops["H0"].to_dense() + p.E * ops["H1"].to_dense()
    L = ops["L"].to_dense()
    G = lb.q_hamiltonian(F, H) + p.gamma_eff * lb.q_dissipator(F, L)
    K = p.gamma_eff * lb.k_dissipator(F, L)
    v_inf = np.linalg.solve(G, -K)
    Lv = lb.liouvillian(H, [L], [p.gamma_eff])
    w, V = np.linalg.eig(Lv)
    k = np.argmin(np.abs(w))
    assert abs(w[k]) < 1e-10
    rho = lb.unvec(V[:, k], N)
    rho = rho / np.trace(rho)
    np.testing.assert_allclose(lb.bloch_vector(F, rho), v_inf, atol=1e-10)
    ev = np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))
    assert ev.min() > -1e-10
    assert np.max(np.abs(rho - np.eye(N) / N)) > 1e-3


@pytest.mark.parametrize("N", [3, 4, 5])
def test_sparse_tier_matches_dense_tier(N):
    F = basis.generators(N)
    H = random_ops.random_hermitian_csr(N, 0.6, seed=21 + N)
    L = random_ops.random_complex_csr(N, 0.6, seed=31 + N)
    Qd = lb.q_hamiltonian(F, H.to_dense())
    Rd = lb.q_dissipator(F, L.to_dense())
    Kd = lb.k_dissipator(F, L.to_dense())
    np.testing.assert_allclose(lb.q_full("H", H).toarray(), Qd, atol=1e-13)
    np.testing.assert_allclose(lb.q_full("L", L).toarray(), Rd, atol=1e-12)
    np.testing.assert_allclose(lb.k_vector(L), Kd, atol=1e-13)
    cols = [0, N * N - 2, N]
    np.testing.assert_allclose(lb.q_columns("L", L, cols), Rd[:, cols], atol=1e-12)
    # a dissipator with a trace, taken by both tiers from the definition
    Lt = random_ops.random_complex_csr(N, 0.6, seed=41 + N, traceless=False)
    assert abs(np.trace(Lt.to_dense())) > 1e-3
    np.testing.assert_allclose(lb.q_full("L", Lt).toarray(), lb.q_dissipator(F, Lt.to_dense()), atol=1e-12)
    np.testing.assert_allclose(lb.k_vector(Lt), lb.k_dissipator(F, Lt.to_dense()), atol=1e-13)


@pytest.mark.parametrize("N", [4, 11])
def test_fock_state_bloch_vector(N):
    """rho0 = |0><0|: |v|^2 = 1 - 1/N (pure state) and <n1 - n2> = -(N-1)."""
    rho = np.zeros((N, N), complex)
    rho[0, 0] = 1
    v = lb.bloch_vector_sparse(rho)
    assert abs(v @ v - (1 - 1 / N)) < 1e-13
    X = np.diag(2.0 * np.arange(N) - (N - 1)).astype(complex)   # n1 - n2
    c = lb.bloch_coords(X).real
    assert abs(c @ v - (-(N - 1))) < 1e-12
    np.testing.assert_allclose(lb.density_from_bloch_dense(v, N), rho, atol=1e-14)


def test_dimer_operators_structure():
    p = dimer.plain_config(6)
    ops = dimer.dimer_operators(p)
    for name in ("H0", "H1", "HJ", "HU"):
        X = ops[name].to_dense()
        np.testing.assert_allclose(X, X.conj().T, atol=0)
    L = ops["L"].to_dense()
    assert abs(np.trace(L)) < 1e-12 and abs(np.trace(ops["H1"].to_dense())) < 1e-12
    off = L - np.diag(np.diag(L))
    np.testing.assert_allclose(off, -off.T, atol=0)      # antisymmetric off-diagonal
    # two-mode Fock space with 0..N-1 bosons per mode, projected onto the
    # subspace of N-1 bosons in total; state i = |n1 = i, n2 = N-1-i>
    N = p.N
    a = np.diag(np.sqrt(np.arange(1, N)), 1)              # single-mode annihilator
    I = np.eye(N)
    b1 = np.kron(a, I)
    b2 = np.kron(I, a)
    proj = np.zeros((N * N, N))
    for i in range(N):
        proj[i * N + (N - 1 - i), i] = 1.0
    sub = lambda X: proj.T @ X @ proj
    np.testing.assert_allclose(L, sub((b1.T + b2.T) @ (b1 - b2)), atol=1e-12)
    np.testing.assert_allclose(ops["HJ"].to_dense(), sub(b1.T @ b2 + b2.T @ b1), atol=1e-12)
    n1, n2 = b1.T @ b1, b2.T @ b2
    np.testing.assert_allclose(ops["H1"].to_dense(), sub(n1 - n2), atol=1e-12)
    np.testing.assert_allclose(ops["HU"].to_dense(),
                               sub(0.5 * (n1 @ (n1 - np.eye(N * N)) + n2 @ (n2 - np.eye(N * N)))),
                               atol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_entrywise_density_matches_generator_sum(N):
    """The entry-by-entry reconstruction of rho from v equals eq. 5 summed
    over the explicit generators, for a random (not necessarily positive) v;
    the result has unit trace and is Hermitian."""
    F = basis.generators(N)
    v = random_ops.random_vector(N * N - 1, seed=40 + N)
    rho = lb.density_from_bloch_dense(v, N)
    np.testing.assert_allclose(rho, lb.density_from_bloch(F, v), atol=1e-15)
    assert abs(np.trace(rho) - 1) < 1e-14
    np.testing.assert_array_equal(rho, rho.conj().T)
    np.testing.assert_allclose(lb.bloch_vector(F, rho), v, atol=1e-14)


def test_gauge_identity_for_dissipator_with_trace():
    """For L = c 1 + L' (c = Tr L / N): D_L(X) = D_L'(X) - i[H_c, X] with
    H_c = (i/2)(conj(c) L' - c L'^+) Hermitian, for a random X; hence the
    Bloch matrices satisfy R(L) = R(L') + Q(H_c) and K(L) = K(L')."""
    N = 4
    rng = np.random.default_rng(12)
    L = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    c = np.trace(L) / N
    Lp = L - c * np.eye(N)
    Hc = 0.5j * (np.conj(c) * Lp - c * Lp.conj().T)
    np.testing.assert_allclose(Hc, Hc.conj().T, atol=1e-15)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    np.testing.assert_allclose(lb.dissipator(L, X), lb.dissipator(Lp, X) - 1j * (Hc @ X - X @ Hc), atol=1e-13)
    F = basis.generators(N)
    np.testing.assert_allclose(lb.q_dissipator(F, L), lb.q_dissipator(F, Lp) + lb.q_hamiltonian(F, Hc), atol=1e-13)
    np.testing.assert_allclose(lb.k_dissipator(F, L), lb.k_dissipator(F, Lp), atol=1e-14)
    # the coefficients of H_c follow from those of L: h_j = -Im(conj(c) l_j)
    l = lb.expand(F, L)
    np.testing.assert_allclose(lb.expand(F, Hc).real, -np.imag(np.conj(c) * l), atol=1e-14)



@pytest.mark.parametrize("N", [4, 5])
def test_stationary_bloch_is_liouvillian_kernel(N):
    """lindblad.stationary_bloch (sparse solve of G v = -K) equals the Bloch
    vector of the normalised kernel of the dense Liouvillian (Kronecker
    products, no basis)."""
    import scipy.sparse as sps
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    F = basis.generators(N)
    H = ops["H0"].to_dense() + p.E * ops["H1"].to_dense()
    L = ops["L"].to_dense()
    G = lb.q_hamiltonian(F, H) + p.gamma_eff * lb.q_dissipator(F, L)
    K = p.gamma_eff * lb.k_dissipator(F, L)
    v = lb.stationary_bloch(sps.csr_matrix(G), K)
    w, V = np.linalg.eig(lb.liouvillian(H, [L], [p.gamma_eff]))
    k = np.argmin(np.abs(w))
    rho = lb.unvec(V[:, k], N)
    rho = rho / np.trace(rho)
    np.testing.assert_allclose(v, lb.bloch_vector(F, rho), atol=1e-10)


def test_stationary_bloch_is_long_time_limit():
    """At N = 21 the stationary state is where RK4 with the static drive
    ends up after t = 200 (every mode decays at a rate >= 0.15)."""
    from oracle import propagate as pr
    N = 21
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    G = lb.q_full("H", ops["H0"]) + p.E * lb.q_full("H", ops["H1"]) + p.gamma_eff * lb.q_full("L", ops["L"])
    K = p.gamma_eff * lb.k_vector(ops["L"])
    v = lb.stationary_bloch(G, K)
    steps = 20000
    dt = 200.0 / steps
    v0 = np.zeros(N * N - 1)
    vt = pr.rk4_bloch(G, [], K, v0, np.zeros((2 * steps + 1, 0)), dt, steps)
    assert np.max(np.abs(vt - v)) <= 1e-9 * np.max(np.abs(v))
