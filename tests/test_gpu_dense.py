"""Dense-operator path: the FP64 matrix-core product (sun_gemm_f64) and the
assembly of Q_H, R, K for dense or random operators
(sun_expand_lindbladian_dense: dense sections, R = -(1/2) Re(B^T A) as one
product), against the oracle.

GEMM bar: |C - C_ref| <= 2 (K + 2) u (|alpha| |A||B| + |beta| |C0|) entry by
entry (u = 2^-53; the standard bound of a K-term dot product), with C_ref
from numpy's float64 product of the same inputs.  Assembly bar: as the sparse
path, max|dQ| <= 1e-12 max|Q| per matrix (the dense path sums each row of a
section in the same order as the sparse path; R's K = 2M contraction adds
O(M u) relative rounding, ~1e-12 at M ~ 1e4).
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from helpers import flush, rel_matrix_err, rel_vec_err, to_scipy
from oracle import basis as ob, lindblad as lb, o2
from workloads import dimer, random_ops

pytestmark = pytest.mark.gpu

TOL = 1e-12
U = 2.0 ** -53


@pytest.mark.parametrize("shape", [(1, 1, 1), (16, 16, 4), (17, 33, 5), (128, 128, 16), (129, 130, 17),
                                   (300, 257, 515), (1000, 999, 2001)])
@pytest.mark.parametrize("beta", [0.0, -1.3])
def test_gemm_against_float64_product(lib, shape, beta):
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    alpha = 0.7
    C = lib.gemm_f64(torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda(), torch.as_tensor(C0).cuda(), alpha,
                     beta).cpu().numpy()
    ref = alpha * (A @ B) + beta * C0
    bound = 2 * (K + 2) * U * (abs(alpha) * (np.abs(A) @ np.abs(B)) + abs(beta) * np.abs(C0)) + 1e-300
    assert np.all(np.abs(C - ref) <= bound)


def test_gemm_integer_entries_exact(lib):
    """Small integers: every product and partial sum is exact, so any
    misplaced operand of the matrix instruction shows as a wrong integer."""
    rng = np.random.default_rng(5)
    for M, N, K in ((16, 16, 4), (64, 48, 36), (130, 70, 33)):
        A = rng.integers(-3, 4, (M, K)).astype(np.float64)
        B = rng.integers(-3, 4, (K, N)).astype(np.float64)
        C = lib.gemm_f64(torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda()).cpu().numpy()
        assert np.array_equal(C, A @ B)


def _export(lind, M):
    QH = [to_scipy(*lind.export("H", a), M) for a in range(lind.nH)]
    R, K = [], []
    for p in range(lind.P):
        rp, c, v, k = lind.export("L", p)
        R.append(to_scipy(rp, c, v, M))
        K.append(k.cpu().numpy())
    return QH, R, K


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_dense_random_operators_against_dense_oracle(lib, N):
    flush(f"[dense] random dense operators N={N}")
    H = random_ops.random_hermitian_csr(N, 1.0, seed=300 + N)
    L = random_ops.random_complex_csr(N, 1.0, seed=400 + N)
    Lt = random_ops.random_complex_csr(N, 1.0, seed=500 + N, traceless=False)
    F = ob.generators(N)
    M = N * N - 1
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [H], [L, Lt], dense=True)
    QH, R, K = _export(lind, M)
    assert rel_matrix_err(QH[0], lb.q_hamiltonian(F, H.to_dense())) <= TOL
    for Lx, Rx, Kx in ((L, R[0], K[0]), (Lt, R[1], K[1])):
        assert rel_matrix_err(Rx, lb.q_dissipator(F, Lx.to_dense())) <= TOL
        assert rel_vec_err(Kx, lb.k_dissipator(F, Lx.to_dense())) <= TOL


@pytest.mark.parametrize("N", [21, 51])
def test_dense_path_equals_sparse_path_for_dimer(lib, N):
    flush(f"[dense] dimer N={N}: dense path vs sparse path")
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(N)
    M = N * N - 1
    sparse = _export(lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]]), M)
    dense = _export(lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]], dense=True), M)
    for a in range(2):
        assert dense[0][a].nnz == sparse[0][a].nnz
        assert rel_matrix_err(dense[0][a], sparse[0][a]) <= TOL
    assert dense[1][0].nnz == sparse[1][0].nnz
    assert rel_matrix_err(dense[1][0], sparse[1][0]) <= TOL
    assert rel_vec_err(dense[2][0], sparse[2][0]) <= TOL


def test_dense_random_L_N30_against_c_oracle(lib):
    N = 30
    flush(f"[dense] random dense L N={N} vs C oracle")
    L = random_ops.random_complex_csr(N, 1.0, seed=30)
    M = N * N - 1
    b = lib.build_basis(N)
    QH, R, K = _export(lib.Lindbladian(b, [], [L], dense=True), M)
    assert rel_matrix_err(R[0], o2.q_full("L", L)) <= TOL
    assert rel_vec_err(K[0], o2.k_vector(L)) <= TOL


def test_sparse_path_falls_back_to_dense(lib):
    """A dense L at N = 70 exceeds the sparse path's per-row limit; the
    default assembly then takes the dense path (bitwise the same result)."""
    N = 70
    flush(f"[dense] fallback N={N}")
    L = random_ops.random_complex_csr(N, 1.0, seed=70)
    b = lib.build_basis(N)
    M = N * N - 1
    _, R1, K1 = _export(lib.Lindbladian(b, [], [L]), M)
    _, R2, K2 = _export(lib.Lindbladian(b, [], [L], dense=True), M)
    assert (R1[0] != R2[0]).nnz == 0 and np.array_equal(K1[0], K2[0])


def test_random_dense_L_N100_sampled_columns(lib):
    """N = 100 (M = 9,999), a random dense L, the size of the paper's random
    Lindbladian ensembles: 40 sampled columns of R against the oracle's
    explicit traces, K in full."""
    N = 100
    flush(f"[dense] random dense L N={N}")
    L = random_ops.random_complex_csr(N, 1.0, seed=100)
    b = lib.build_basis(N)
    M = N * N - 1
    _, R, K = _export(lib.Lindbladian(b, [], [L], dense=True), M)
    P = N * (N - 1) // 2
    rng = np.random.default_rng(100)
    cols = sorted(set(rng.integers(0, M, 32).tolist() + [0, P - 1, P, 2 * P - 1, 2 * P, 2 * P + 50, M - 2, M - 1]))
    O = lb.q_columns("L", L, cols)
    G = R[0].tocsc()[:, cols].toarray()
    assert np.max(np.abs(G - O)) <= TOL * np.max(np.abs(R[0].data))
    assert rel_vec_err(K[0], lb.k_vector(L)) <= TOL
