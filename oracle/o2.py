"""Oracle tier O2: explicit traces column by column and a multi-core CSR RK4,
in plain C + OpenMP (``oracle/o2.c``, built into ``oracle/libo2.so``).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* ``q_full``      -- Q_H (kind 'H', eq. 6) or R_L (kind 'L', eq. 10, unit rate)
                     as a scipy CSR matrix, column m = Bloch coordinates of
                     the generator applied to F_m (Sec. II); any N, O(nnz)
                     work for banded operators; exact cancellations dropped by
                     the same rule as ``lindblad.q_full``.
* ``k_vector``    -- K_L = Tr(F_s D_L(1))/N (eq. 11, unit rate).
* ``rk4``         -- classical RK4 (Sec. IV step 3.1) on a list of CSR terms
                     with a half-step coefficient table, OpenMP over rows.

Parity: pinned -- equal to the dense trace tier (itself pinned by the qubit
closed forms, the Liouvillian kernel and skew-symmetry) for random operators,
equal to ``lindblad.q_full`` for the dimer, the qubit amplitude-damping closed
form, the dimer's nonzero counts (37N^2 - 93N + 52)/2 of the union, and
``rk4`` equal to ``propagate.rk4_bloch`` (tests/test_oracle_o2.py).
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libo2.so")
SOURCE = os.path.join(HERE, "o2.c")


class _Op(C.Structure):
    _fields_ = [("n", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p), ("re", C.c_void_p),
                ("im", C.c_void_p)]


_lib = None


def build(path: str = LIB_PATH) -> str:
    """Compile o2.c with gcc -fopenmp into ``path``."""
    import subprocess
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", SOURCE, "-o", path, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the O2 oracle failed:\n{r.stderr}")
    return path


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SOURCE):
        build()
    lib = C.CDLL(LIB_PATH)
    lib.o2_columns.restype = C.c_int
    lib.o2_columns.argtypes = [C.c_int, C.POINTER(_Op), C.c_int, C.c_void_p, C.POINTER(C.c_void_p),
                               C.POINTER(C.c_void_p), C.POINTER(C.c_double)]
    lib.o2_k_vector.restype = C.c_int
    lib.o2_k_vector.argtypes = [C.POINTER(_Op), C.c_void_p, C.POINTER(C.c_double)]
    lib.o2_free.restype = None
    lib.o2_free.argtypes = [C.c_void_p]
    lib.o2_rk4.restype = C.c_int
    lib.o2_rk4.argtypes = [C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_double, C.c_int64, C.c_void_p, C.c_int]
    lib.o2_max_threads.restype = C.c_int
    _lib = lib
    return lib


def _csr(op):
    """(indptr, indices, re, im) arrays of an operator (scipy sparse, dense or
    an object with n/indptr/indices/re/im)."""
    if hasattr(op, "indptr") and hasattr(op, "re"):
        m = sp.csr_matrix((np.asarray(op.re) + 1j * np.asarray(op.im), op.indices, op.indptr), shape=(op.n, op.n))
    else:
        m = sp.csr_matrix(op, dtype=np.complex128)
    m.sum_duplicates()
    m.sort_indices()
    n = m.shape[0]
    keep = (np.ascontiguousarray(m.indptr, dtype=np.int32), np.ascontiguousarray(m.indices, dtype=np.int32),
            np.ascontiguousarray(m.data.real, dtype=np.float64), np.ascontiguousarray(m.data.imag, dtype=np.float64))
    s = _Op(n, keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data, keep[3].ctypes.data)
    return s, keep, n


def max_threads() -> int:
    return int(load().o2_max_threads())


def q_full(kind: str, op, rel_drop: float = 1e-12, threads: int = 0) -> sp.csr_matrix:
    """All columns of Q (kind 'H') or R (kind 'L', unit rate) as scipy CSR;
    entries with |q| <= rel_drop max|q| are exact cancellations and dropped."""
    lib = load()
    s, keep, n = _csr(op)
    M = n * n - 1
    colptr = np.zeros(M + 1, dtype=np.int64)
    rows, vals = C.c_void_p(), C.c_void_p()
    mi = C.c_double()
    st = lib.o2_columns(0 if kind == "H" else 1, C.byref(s), int(threads), colptr.ctypes.data, C.byref(rows),
                        C.byref(vals), C.byref(mi))
    if st != 0:
        raise MemoryError("o2_columns: out of host memory")
    try:
        nnz = int(colptr[-1])
        r = np.ctypeslib.as_array(C.cast(rows, C.POINTER(C.c_int32)), shape=(max(nnz, 1),))[:nnz].copy()
        v = np.ctypeslib.as_array(C.cast(vals, C.POINTER(C.c_double)), shape=(max(nnz, 1),))[:nnz].copy()
    finally:
        lib.o2_free(rows)
        lib.o2_free(vals)
    Q = sp.csc_matrix((v, r, colptr), shape=(M, M)).tocsr()
    scale = np.max(np.abs(Q.data)) if Q.nnz else 1.0
    assert mi.value <= 1e-11 * max(1.0, scale), mi.value
    if Q.nnz:
        Q.data[np.abs(Q.data) <= rel_drop * scale] = 0.0
        Q.eliminate_zeros()
    Q.sort_indices()
    return Q


def k_vector(L) -> np.ndarray:
    lib = load()
    s, keep, n = _csr(L)
    k = np.zeros(n * n - 1)
    mi = C.c_double()
    if lib.o2_k_vector(C.byref(s), k.ctypes.data, C.byref(mi)) != 0:
        raise MemoryError("o2_k_vector: out of host memory")
    assert mi.value <= 1e-11 * max(1.0, np.max(np.abs(k)) if k.size else 1.0)
    return k


def rk4(terms, coef, v0, dt: float, steps: int, threads: int = 0) -> np.ndarray:
    """Classical RK4 for dv/dt = sum_a c_a(t) (G_a v + K_a).

    terms: list of (G_a scipy sparse (M, M), K_a (M,) or None); coef:
    (2*steps+1, nterm) half-step table.  Returns v after ``steps`` steps."""
    lib = load()
    mats = [sp.csr_matrix(G) for G, _ in terms]
    for m in mats:
        m.sort_indices()
    M = mats[0].shape[0]
    rp = [np.ascontiguousarray(m.indptr, dtype=np.int32) for m in mats]
    cl = [np.ascontiguousarray(m.indices, dtype=np.int32) for m in mats]
    vl = [np.ascontiguousarray(m.data, dtype=np.float64) for m in mats]
    ks = [None if K is None else np.ascontiguousarray(K, dtype=np.float64) for _, K in terms]
    n = len(terms)
    prp = (C.c_void_p * n)(*[a.ctypes.data for a in rp])
    pcl = (C.c_void_p * n)(*[a.ctypes.data for a in cl])
    pvl = (C.c_void_p * n)(*[a.ctypes.data for a in vl])
    pk = (C.c_void_p * n)(*[0 if a is None else a.ctypes.data for a in ks])
    tab = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(2 * steps + 1, n))
    v = np.array(v0, dtype=np.float64, copy=True)
    if lib.o2_rk4(M, n, prp, pcl, pvl, pk, tab.ctypes.data, float(dt), int(steps), v.ctypes.data,
                  int(threads)) != 0:
        raise MemoryError("o2_rk4: out of host memory")
    return v
