"""SU(N) generator basis and structure constants, by brute force (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Basis (paper Sec. II, list of generators): for 0 <= j < k < N

    S^(j,k) = (G_jk + G_kj)/sqrt(2)
    J^(j,k) = -i (G_jk - G_kj)/sqrt(2)
    D^l     = (sum_{i<l} G_ii - l G_ll)/sqrt(l(l+1)),   l = 1..N-1

with G_jk = |j><k| (0-based here).  Two readings of the printed text are
taken (both listed in the design notes):

* the diagonal generators are printed with a leading factor i, which would
  make them anti-Hermitian and contradict Tr(F_i F_k) = delta_ik; the factor
  is dropped;
* the paper does not fix the order of the M = N^2 - 1 generators; the order
  used throughout is "grouped": all S^(j,k) with (j,k) row-major over j<k
  (index p), then all J^(j,k) in the same order (index P + p, P = N(N-1)/2),
  then D^1..D^{N-1} (index 2P + l - 1).

Structure constants (Sec. II, eqs. 2-4) by their trace definitions:

    f_mns = -i Tr(F_s [F_m, F_n]),   d_mns = Tr(F_s {F_m, F_n}).

Parity: pinned (Gram matrix, SU(2)/SU(3) textbook tables, the paper's nonzero
counts, Casimir and Jacobi identities -- see tests/test_oracle_basis.py).
"""

from __future__ import annotations

import math

import numpy as np


def num_generators(N: int) -> int:
    return N * N - 1


def labels(N: int) -> list:
    """Grouped-order labels: ('S', j, k), ('J', j, k) or ('D', l, l)."""
    pairs = [(j, k) for j in range(N) for k in range(j + 1, N)]
    out = [("S", j, k) for (j, k) in pairs]
    out += [("J", j, k) for (j, k) in pairs]
    out += [("D", l, l) for l in range(1, N)]
    return out


def generators(N: int) -> np.ndarray:
    """Dense generators, shape (M, N, N), complex128, grouped order."""
    M = num_generators(N)
    F = np.zeros((M, N, N), dtype=np.complex128)
    r2 = math.sqrt(2.0)
    for idx, (kind, a, b) in enumerate(labels(N)):
        if kind == "S":
            F[idx, a, b] = 1.0 / r2
            F[idx, b, a] = 1.0 / r2
        elif kind == "J":
            F[idx, a, b] = -1j / r2
            F[idx, b, a] = 1j / r2
        else:
            l = a
            c = 1.0 / math.sqrt(l * (l + 1))
            for i in range(l):
                F[idx, i, i] = c
            F[idx, l, l] = -l * c
    return F


def structure_constants(N: int):
    """(f, d) as dense (M, M, M) float64 arrays from eq. (4).

    Computed literally: commutators and anticommutators of every pair of
    generators, then the trace against every generator.
    """
    F = generators(N)
    prod = np.einsum("mab,nbc->mnac", F, F)          # F_m F_n
    comm = prod - prod.transpose(1, 0, 2, 3)          # [F_m, F_n]
    acom = prod + prod.transpose(1, 0, 2, 3)          # {F_m, F_n}
    # Tr(F_s X) = sum_ab F_s[a,b] X[b,a]
    f = -1j * np.einsum("sab,mnba->mns", F, comm)
    d = np.einsum("sab,mnba->mns", F, acom)
    assert np.max(np.abs(f.imag)) < 1e-12, "f must be real"
    assert np.max(np.abs(d.imag)) < 1e-12, "d must be real"
    return f.real.copy(), d.real.copy()


def nonzero_triples(t: np.ndarray, tol: float = 1e-12):
    """Nonzero entries of a dense 3-tensor: (idx (nnz,3) int64, vals).

    Entries with |t| > tol count as nonzero (the smallest true nonzero of f or
    d for N <= 8 is above 0.1, rounding residues are below 1e-15).  Triples
    are listed in lexicographic order of (m, n, s), all index orders included.
    """
    idx = np.argwhere(np.abs(t) > tol)            # argwhere is lexicographic
    vals = t[idx[:, 0], idx[:, 1], idx[:, 2]]
    return idx.astype(np.int64), vals


def gram(F: np.ndarray) -> np.ndarray:
    """Tr(F_i F_j) for all i, j."""
    return np.einsum("iab,jba->ij", F, F)
