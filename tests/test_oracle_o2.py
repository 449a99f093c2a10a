"""Pins of the C/OpenMP oracle tier (oracle/o2.c): Q, R, K by explicit traces
column by column, and its CSR RK4.

Fixed points: the dense trace tier (pinned by the qubit closed forms, the
Liouvillian kernel and skew-symmetry in test_oracle_lindblad.py) for random
Hermitian H and random non-Hermitian L (also with a trace), the qubit
amplitude-damping Bloch equations, the Python column tier for the dimer, the
dimer's nonzero counts (closed forms of the union pattern), and the Python
RK4 (itself pinned by the Taylor polynomial of the augmented generator).
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import basis, lindblad as lb, o2, propagate as pr
from workloads import dimer, random_ops


def test_amplitude_damping_qubit_closed_form():
    w0, g = 1.3, 0.7
    H = 0.5 * w0 * np.diag([1.0, -1.0]).astype(complex)
    L = np.zeros((2, 2), complex)
    L[1, 0] = 1.0
    G = (o2.q_full("H", H) + g * o2.q_full("L", L)).toarray()
    K = g * o2.k_vector(L)
    np.testing.assert_allclose(G, [[-g / 2, -w0, 0], [w0, -g / 2, 0], [0, 0, -g]], atol=1e-14)
    np.testing.assert_allclose(K, [0, 0, -g / math.sqrt(2)], atol=1e-14)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_random_operators_equal_dense_tier(N):
    F = basis.generators(N)
    H = random_ops.random_hermitian_csr(N, 0.6, seed=10 + N)
    Lt = random_ops.random_complex_csr(N, 0.5, seed=20 + N, traceless=False)   # with a trace
    QH = o2.q_full("H", H).toarray()
    R = o2.q_full("L", Lt).toarray()
    K = o2.k_vector(Lt)
    QHd = lb.q_hamiltonian(F, H.to_dense())
    Rd = lb.q_dissipator(F, Lt.to_dense())
    Kd = lb.k_dissipator(F, Lt.to_dense())
    scale = max(np.max(np.abs(QHd)), 1.0)
    assert np.max(np.abs(QH - QHd)) <= 1e-13 * scale
    assert np.max(np.abs(R - Rd)) <= 1e-13 * max(np.max(np.abs(Rd)), 1.0)
    assert np.max(np.abs(K - Kd)) <= 1e-13 * max(np.max(np.abs(Kd)), 1.0)


@pytest.mark.parametrize("N", [11, 21])
def test_dimer_equals_python_column_tier(N):
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    for kind, key in (("H", "H0"), ("H", "H1"), ("L", "L")):
        A = o2.q_full(kind, ops[key])
        B = lb.q_full(kind, ops[key])
        assert A.nnz == B.nnz
        d = (A - B).tocsr()
        assert (np.max(np.abs(d.data)) if d.nnz else 0.0) <= 1e-13 * np.max(np.abs(B.data))
    np.testing.assert_allclose(o2.k_vector(ops["L"]), lb.k_vector(ops["L"]), atol=1e-14)


@pytest.mark.parametrize("N", [11, 51])
def test_dimer_nonzero_counts(N):
    """nnz of Q_H0 = 5N^2 - 10N + 3, Q_H1 = N(N-1), R = 13.5N^2 - 37.5N + 24 and
    of their union (37N^2 - 93N + 52)/2, for N >= 11."""
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    Q0 = o2.q_full("H", ops["H0"])
    Q1 = o2.q_full("H", ops["H1"])
    R = o2.q_full("L", ops["L"])
    assert Q0.nnz == 5 * N * N - 10 * N + 3
    assert Q1.nnz == N * (N - 1)
    assert 2 * R.nnz == 27 * N * N - 75 * N + 48
    U = (abs(Q0) + abs(Q1) + abs(R)).tocsr()
    assert 2 * U.nnz == 37 * N * N - 93 * N + 52
    # skew-symmetry of the unitary parts
    assert abs(Q0 + Q0.T).max() <= 1e-13 * abs(Q0).max()


def test_rk4_equals_python_rk4():
    N, steps = 21, 50
    p = dimer.plain_config(N)
    p.steps_per_period = 1000
    ops = dimer.dimer_operators(p)
    G0 = o2.q_full("H", ops["H0"]) + p.gamma_eff * o2.q_full("L", ops["L"])
    G1 = o2.q_full("H", ops["H1"])
    K = p.gamma_eff * o2.k_vector(ops["L"])
    eps = dimer.drive_table(p, steps=steps)
    v0 = random_ops.random_vector(N * N - 1, seed=3, scale=0.05)
    want = pr.rk4_bloch(G0, [G1], K, v0, eps[:, None], p.dt, steps)
    coef = np.stack([np.ones_like(eps), eps], axis=1)
    for threads in (1, 3):
        got = o2.rk4([(G0, K), (G1, None)], coef, v0, p.dt, steps, threads=threads)
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
