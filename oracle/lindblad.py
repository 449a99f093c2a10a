"""Bloch-vector form of a GKSL generator by explicit traces (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The GKSL generator (paper Sec. I, eq. 1) is

    L(rho) = -i[H, rho] + sum_p gamma_p D_p(rho),
    D_p(rho) = L_p rho L_p^+ - (1/2){L_p^+ L_p, rho}

(the paper writes D_p with two commutators; expanded, they give exactly this).
Writing rho = 1/N + sum_m v_m F_m (eq. 5), the Bloch vector obeys the real
ODE dv/dt = (Q + R) v + K (eq. 9) with

    Q_sm = Tr(F_s (-i[H, F_m]))          (unitary part, eq. 6)
    R_sm = Tr(F_s D(F_m))                (dissipative part, eq. 10)
    K_s  = Tr(F_s D(1)) / N              (free vector, eq. 11)

because Tr(F_s F_m) = delta_sm.  This module evaluates these traces with no
use of structure constants, which is what makes it an independent check of
the contraction formulas (eqs. 6, 10, 11) that the GPU path uses.

Two tiers:

* dense (``q_hamiltonian``, ``q_dissipator``, ``k_dissipator``,
  ``liouvillian``): every generator as a dense N x N matrix; N <= 8.
* column-by-column with sparse operators (``q_columns``, ``q_full``,
  ``k_vector``): column m of Q or R is the Bloch coordinate vector of
  L(F_m), with F_m sparse and H, L as scipy sparse matrices; any N.

``stationary_bloch`` solves G v = -K for a time-independent generator.

Parity: pinned -- qubit amplitude damping closed form, Larmor precession,
skew-symmetry of the unitary part, dense-Liouvillian kernel, agreement of the
two tiers, the stationary state against the Liouvillian's kernel and against
long-time RK4 (tests/test_oracle_lindblad.py).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Dense tier
# ---------------------------------------------------------------------------

def trace_against(F: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Tr(F_s X) for every generator s (complex)."""
    return np.einsum("sab,ba->s", F, X)


def bloch_vector(F: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """v_j = Tr(F_j rho) (eq. 5 inverted with Tr(F_i F_j) = delta_ij)."""
    v = trace_against(F, rho)
    assert np.max(np.abs(v.imag)) < 1e-12 * max(1.0, np.max(np.abs(v.real)))
    return v.real.copy()


def density_from_bloch(F: np.ndarray, v: np.ndarray) -> np.ndarray:
    """rho = 1/N + sum_j v_j F_j (eq. 5)."""
    N = F.shape[1]
    return np.eye(N, dtype=np.complex128) / N + np.einsum("j,jab->ab", v, F)


def expand(F: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Expansion coefficients x_m = Tr(F_m X) (complex for non-Hermitian X)."""
    return trace_against(F, X)


def dissipator(L: np.ndarray, X: np.ndarray) -> np.ndarray:
    """D_L(X) = L X L^+ - (1/2){L^+ L, X} (eq. 1)."""
    Ld = L.conj().T
    LdL = Ld @ L
    return L @ X @ Ld - 0.5 * (LdL @ X + X @ LdL)


def q_hamiltonian(F: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Q_sm = Tr(F_s (-i[H, F_m])), dense (M, M) float64."""
    M = F.shape[0]
    Q = np.zeros((M, M), dtype=np.complex128)
    for m in range(M):
        Y = -1j * (H @ F[m] - F[m] @ H)
        Q[:, m] = trace_against(F, Y)
    assert np.max(np.abs(Q.imag)) < 1e-12 * max(1.0, np.max(np.abs(Q.real)))
    return Q.real.copy()


def q_dissipator(F: np.ndarray, L: np.ndarray) -> np.ndarray:
    """R_sm = Tr(F_s D_L(F_m)) at unit rate, dense (M, M) float64."""
    M = F.shape[0]
    R = np.zeros((M, M), dtype=np.complex128)
    for m in range(M):
        R[:, m] = trace_against(F, dissipator(L, F[m]))
    assert np.max(np.abs(R.imag)) < 1e-12 * max(1.0, np.max(np.abs(R.real)))
    return R.real.copy()


def k_dissipator(F: np.ndarray, L: np.ndarray) -> np.ndarray:
    """K_s = Tr(F_s D_L(1)) / N at unit rate, float64 (M,)."""
    N = F.shape[1]
    k = trace_against(F, dissipator(L, np.eye(N, dtype=np.complex128))) / N
    assert np.max(np.abs(k.imag)) < 1e-12 * max(1.0, np.max(np.abs(k.real)))
    return k.real.copy()


def liouvillian(H: np.ndarray, Ls, gammas) -> np.ndarray:
    """Dense N^2 x N^2 matrix of eq. (1) on column-stacked vec(rho).

    Uses vec(A X B) = (B^T kron A) vec(X); independent of any basis.
    """
    N = H.shape[0]
    I = np.eye(N, dtype=np.complex128)
    Lv = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for L, g in zip(Ls, gammas):
        Ld = L.conj().T
        LdL = Ld @ L
        Lv = Lv + g * (np.kron(L.conj(), L)
                       - 0.5 * np.kron(I, LdL) - 0.5 * np.kron(LdL.T, I))
    return Lv


def vec(X: np.ndarray) -> np.ndarray:
    return X.reshape(-1, order="F")


def unvec(x: np.ndarray, N: int) -> np.ndarray:
    return x.reshape((N, N), order="F")


# ---------------------------------------------------------------------------
# Sparse, column-by-column tier (any N)
# ---------------------------------------------------------------------------

def _pair_index(N: int, j: int, k: int) -> int:
    return j * (2 * N - j - 1) // 2 + (k - j - 1)


def generator_sparse(N: int, m: int) -> sp.csr_matrix:
    """F_m (grouped order) as a scipy CSR matrix."""
    P = N * (N - 1) // 2
    r2 = math.sqrt(2.0)
    if m < 2 * P:
        q = m if m < P else m - P
        # invert the row-major pair index
        j = 0
        while q >= N - 1 - j:
            q -= N - 1 - j
            j += 1
        k = j + 1 + q
        if m < P:
            rows, cols, vals = [j, k], [k, j], [1 / r2, 1 / r2]
        else:
            rows, cols, vals = [j, k], [k, j], [-1j / r2, 1j / r2]
    else:
        l = m - 2 * P + 1
        c = 1.0 / math.sqrt(l * (l + 1))
        rows = list(range(l + 1))
        cols = list(range(l + 1))
        vals = [c] * l + [-l * c]
    return sp.csr_matrix((np.asarray(vals, np.complex128), (rows, cols)),
                         shape=(N, N))


def bloch_coords(Y) -> np.ndarray:
    """Tr(F_s Y) for all s by index arithmetic on the entries of Y.

    Tr(S^(j,k) Y) = (Y_jk + Y_kj)/sqrt2, Tr(J^(j,k) Y) = i(Y_jk - Y_kj)/sqrt2,
    Tr(D^l Y) = (sum_{i<l} Y_ii - l Y_ll)/sqrt(l(l+1)).  Returns complex (M,).
    Y may be dense or scipy sparse.
    """
    Y = sp.coo_matrix(Y)
    N = Y.shape[0]
    P = N * (N - 1) // 2
    M = N * N - 1
    out = np.zeros(M, dtype=np.complex128)
    r2 = math.sqrt(2.0)
    a = Y.row.astype(np.int64)
    b = Y.col.astype(np.int64)
    y = Y.data.astype(np.complex128)
    dmask = a == b
    diag = np.zeros(N, dtype=np.complex128)
    np.add.at(diag, a[dmask], y[dmask])
    o = ~dmask
    a, b, y = a[o], b[o], y[o]
    j = np.minimum(a, b)
    k = np.maximum(a, b)
    p = j * (2 * N - j - 1) // 2 + (k - j - 1)
    np.add.at(out, p, y / r2)
    sign = np.where(a < b, 1j, -1j)         # Y_jk (a<b) or Y_kj (a>b)
    np.add.at(out, P + p, sign * y / r2)
    prefix = np.concatenate([[0.0], np.cumsum(diag)])
    l = np.arange(1, N)
    out[2 * P:] = (prefix[l] - l * diag[l]) / np.sqrt(l * (l + 1.0))
    return out


def _as_sparse(op) -> sp.csr_matrix:
    if sp.issparse(op):
        return op.tocsr().astype(np.complex128)
    if hasattr(op, "indptr") and hasattr(op, "re"):      # workloads.ZCSR
        return sp.csr_matrix((op.re + 1j * op.im, op.indices, op.indptr),
                             shape=(op.n, op.n))
    return sp.csr_matrix(np.asarray(op, dtype=np.complex128))


def _apply(kind: str, op: sp.csr_matrix, X: sp.csr_matrix) -> sp.csr_matrix:
    if kind == "H":
        return -1j * (op @ X - X @ op)
    if kind == "L":
        Ld = op.conj().T.tocsr()
        LdL = Ld @ op
        return op @ X @ Ld - 0.5 * (LdL @ X + X @ LdL)
    raise ValueError(kind)


def q_columns(kind: str, op, cols) -> np.ndarray:
    """Columns ``cols`` of Q (kind 'H', op = H) or R (kind 'L', op = L, unit
    rate), by traces.  Returns float64 (M, len(cols))."""
    A = _as_sparse(op)
    N = A.shape[0]
    M = N * N - 1
    out = np.zeros((M, len(cols)), dtype=np.float64)
    for t, m in enumerate(cols):
        y = bloch_coords(_apply(kind, A, generator_sparse(N, int(m))))
        scale = max(1.0, np.max(np.abs(y.real))) if y.size else 1.0
        assert np.max(np.abs(y.imag)) < 1e-11 * scale
        out[:, t] = y.real
    return out


def q_full(kind: str, op, rel_drop: float = 1e-12) -> sp.csr_matrix:
    """All columns of Q or R as a scipy CSR matrix.

    Entries with |q| <= rel_drop * max|q| are exact cancellations in exact
    arithmetic and are removed (the paper computes only nonzero entries).
    """
    A = _as_sparse(op)
    N = A.shape[0]
    M = N * N - 1
    rows, cols, vals = [], [], []
    for m in range(M):
        y = bloch_coords(_apply(kind, A, generator_sparse(N, m))).real
        nz = np.nonzero(y)[0]
        rows.append(nz)
        cols.append(np.full(nz.size, m))
        vals.append(y[nz])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Q = sp.csr_matrix((vals, (rows, cols)), shape=(M, M))
    if Q.nnz:
        thr = rel_drop * np.max(np.abs(Q.data))
        Q.data[np.abs(Q.data) <= thr] = 0.0
        Q.eliminate_zeros()
    Q.sort_indices()
    return Q


def k_vector(L) -> np.ndarray:
    """K_s = Tr(F_s D_L(1))/N at unit rate, any N."""
    A = _as_sparse(L)
    N = A.shape[0]
    I = sp.identity(N, dtype=np.complex128, format="csr")
    y = bloch_coords(_apply("L", A, I)) / N
    assert np.max(np.abs(y.imag)) < 1e-11 * max(1.0, np.max(np.abs(y.real)))
    return y.real.copy()


def bloch_vector_sparse(rho) -> np.ndarray:
    """v_j = Tr(F_j rho) for a (possibly large) density matrix."""
    y = bloch_coords(rho)
    return y.real.copy()


def density_from_bloch_dense(v: np.ndarray, N: int) -> np.ndarray:
    """rho = 1/N + sum v_j F_j assembled entry by entry (any N)."""
    P = N * (N - 1) // 2
    r2 = math.sqrt(2.0)
    rho = np.zeros((N, N), dtype=np.complex128)
    jj, kk = np.triu_indices(N, 1)          # row-major pair order
    vs = v[:P]
    vj = v[P:2 * P]
    rho[jj, kk] = (vs - 1j * vj) / r2
    rho[kk, jj] = (vs + 1j * vj) / r2
    d = np.full(N, 1.0 / N, dtype=np.complex128)
    for l in range(1, N):
        c = 1.0 / math.sqrt(l * (l + 1))
        d[:l] += v[2 * P + l - 1] * c
        d[l] += v[2 * P + l - 1] * (-l * c)
    rho[np.arange(N), np.arange(N)] = d
    return rho


def stationary_bloch(G, K) -> np.ndarray:
    """Stationary Bloch vector of a time-independent generator: the solution
    of G v = -K (eq. 9 with dv/dt = 0; the asymptotic state of Sec. I in Bloch
    form), by a sparse direct solve (scipy's LU as the library primitive).
    G: dense or scipy sparse (M, M); K: (M,)."""
    import scipy.sparse.linalg as spla
    if sp.issparse(G):
        return spla.spsolve(sp.csc_matrix(G), -np.asarray(K, dtype=np.float64))
    return np.linalg.solve(np.asarray(G, dtype=np.float64), -np.asarray(K, dtype=np.float64))
