"""GPU assembly of Q_H, R and K against the oracle's explicit traces.

Bar: max |dQ| <= 1e-12 max|Q| over the union of both patterns, same for R
and K (relative to max|K|).  Cases: random dense-ish complex operators
(non-Hermitian, non-normal L) for N = 3..6 against the dense tier, the dimer
at N = 4, 6, 21, 51 against the column-by-column tier (full matrices), and
the dimer at N = 1001 on sampled columns.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from helpers import flush, rel_matrix_err, rel_vec_err, to_scipy
from oracle import basis as ob, lindblad as lb, o2
from workloads import dimer, random_ops

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_random_operators_dense_oracle(lib, N):
    flush(f"[assembly random] N={N}")
    H = random_ops.random_hermitian_csr(N, 0.7, seed=100 + N)
    L = random_ops.random_complex_csr(N, 0.7, seed=200 + N)
    F = ob.generators(N)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [H], [L])
    M = N * N - 1
    Q = to_scipy(*lind.export("H", 0), M)
    rp, c, v, K = lind.export("L", 0)
    R = to_scipy(rp, c, v, M)
    assert rel_matrix_err(Q, lb.q_hamiltonian(F, H.to_dense())) <= TOL
    assert rel_matrix_err(R, lb.q_dissipator(F, L.to_dense())) <= TOL
    assert rel_vec_err(K.cpu().numpy(), lb.k_dissipator(F, L.to_dense())) <= TOL
    # skew-symmetry of the unitary part on the GPU result itself
    assert rel_matrix_err(Q.T, -Q) <= TOL


def test_amplitude_damping_qubit(lib):
    """N = 2, L = |2><1|: R = diag(-1/2, -1/2, -1), K = (0, 0, -1/sqrt2)."""
    L = np.zeros((2, 2), complex)
    L[1, 0] = 1
    H = 0.5 * np.diag([1.0, -1.0]).astype(complex)
    b = lib.build_basis(2)
    lind = lib.Lindbladian(b, [sp.csr_matrix(H)], [sp.csr_matrix(L)])
    Q = to_scipy(*lind.export("H", 0), 3).toarray()
    rp, c, v, K = lind.export("L", 0)
    R = to_scipy(rp, c, v, 3).toarray()
    np.testing.assert_allclose(Q, [[0, -1, 0], [1, 0, 0], [0, 0, 0]], atol=1e-15)
    np.testing.assert_allclose(R, np.diag([-0.5, -0.5, -1.0]), atol=1e-15)
    np.testing.assert_allclose(K.cpu().numpy(), [0, 0, -1 / np.sqrt(2)], atol=1e-15)


@pytest.mark.parametrize("N", [4, 6, 21, 51])
def test_dimer_full_matrices(lib, N):
    flush(f"[assembly dimer] N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
    M = N * N - 1
    for a, name in enumerate(("H0", "H1")):
        G = to_scipy(*lind.export("H", a), M)
        O = lb.q_full("H", ops[name])
        assert rel_matrix_err(G, O) <= TOL, name
    rp, c, v, K = lind.export("L", 0)
    R = to_scipy(rp, c, v, M)
    assert rel_matrix_err(R, lb.q_full("L", ops["L"])) <= TOL
    assert rel_vec_err(K.cpu().numpy(), lb.k_vector(ops["L"])) <= TOL
    if N >= 11:
        # exact nonzero counts of the dimer matrices (closed forms in N)
        assert lind.nnz("H", 0) == 5 * N * N - 10 * N + 3
        assert lind.nnz("H", 1) == N * (N - 1)
        assert lind.nnz("L", 0) == (27 * N * N - 75 * N + 48) // 2


def test_dimer_1001_sampled_columns(lib):
    N = 1001
    flush(f"[assembly dimer sampled] N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
    M = N * N - 1
    P = N * (N - 1) // 2
    rng = np.random.default_rng(1001)
    cols = sorted(set(rng.integers(0, M, 24).tolist() + [0, P - 1, P, 2 * P - 1, 2 * P, M - 1, 1000, P + 1000]))
    assert lind.nnz("H", 0) == 5 * N * N - 10 * N + 3
    assert lind.nnz("L", 0) == (27 * N * N - 75 * N + 48) // 2
    for kind, idx, name in (("H", 0, "H0"), ("H", 1, "H1"), ("L", 0, "L")):
        ex = lind.export(kind, idx)
        G = to_scipy(ex[0], ex[1], ex[2], M).tocsc()
        O = lb.q_columns("H" if kind == "H" else "L", ops[name], cols)
        Gc = G[:, cols].toarray()
        scale = np.max(np.abs(G.data))
        assert np.max(np.abs(Gc - O)) <= TOL * scale, name
    K = lind.export("L", 0)[3].cpu().numpy()
    assert rel_vec_err(K, lb.k_vector(ops["L"])) <= TOL


@pytest.mark.parametrize("N", [301, 1001])
def test_dimer_full_matrices_c_oracle(lib, N):
    """Every entry of Q_H0, Q_H1, R and K at the adjoint size (N = 301,
    M = 90,600) and the headline size (N = 1001, M = 1,002,000) against the
    C/OpenMP oracle's explicit traces (Tr(F_s L(F_m)) column by column)."""
    flush(f"[assembly dimer full, C oracle] N={N}")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
    M = N * N - 1
    for kind, idx, name in (("H", 0, "H0"), ("H", 1, "H1"), ("L", 0, "L")):
        ex = lind.export(kind, idx)
        G = to_scipy(ex[0], ex[1], ex[2], M)
        O = o2.q_full(kind, ops[name])
        assert G.nnz == O.nnz, name
        assert rel_matrix_err(G, O) <= TOL, name
    K = lind.export("L", 0)[3].cpu().numpy()
    assert rel_vec_err(K, o2.k_vector(ops["L"])) <= TOL
