"""Seeded random operators and vectors for parity tests.

Only random-number draws and matrix bookkeeping live here (no method
arithmetic).  Every generator takes an explicit seed.
"""

from __future__ import annotations

import numpy as np

from .dimer import ZCSR


def _csr_from_dense(a: np.ndarray) -> ZCSR:
    return ZCSR.from_dense(a, tol=0.0)


def random_hermitian_csr(N: int, density: float, seed: int,
                         traceless: bool = False, real: bool = False) -> ZCSR:
    """Random Hermitian N x N operator with about ``density`` of its
    off-diagonal entries filled and a random diagonal."""
    rng = np.random.default_rng(seed)
    a = np.zeros((N, N), dtype=np.complex128)
    for j in range(N):
        a[j, j] = rng.standard_normal()
        for k in range(j + 1, N):
            if rng.random() < density:
                z = rng.standard_normal() + (0.0 if real else 1j * rng.standard_normal())
                a[j, k] = z
                a[k, j] = np.conj(z)
    if traceless:
        a -= np.trace(a) / N * np.eye(N)
    return _csr_from_dense(a)


def random_complex_csr(N: int, density: float, seed: int,
                       traceless: bool = True) -> ZCSR:
    """Random general (non-Hermitian, non-normal) complex operator."""
    rng = np.random.default_rng(seed)
    mask = rng.random((N, N)) < density
    a = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) * mask
    for j in range(N):
        a[j, j] = rng.standard_normal() + 1j * rng.standard_normal()
    if traceless:
        a -= np.trace(a) / N * np.eye(N)
    return _csr_from_dense(a)


def random_tridiagonal_hermitian(N: int, seed: int) -> ZCSR:
    """Random Hermitian tridiagonal operator (dimer-like band structure)."""
    rng = np.random.default_rng(seed)
    off = rng.standard_normal(N - 1) + 1j * rng.standard_normal(N - 1)
    dia = rng.standard_normal(N)
    return ZCSR.from_diagonals(N, {-1: np.conj(off), 0: dia, 1: off})


def random_vector(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Random float64 vector of length n (e.g. a Bloch vector for parity
    tests; it need not describe a positive density matrix)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(n)
