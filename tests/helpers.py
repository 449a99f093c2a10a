"""Shared helpers for the parity tests (host-side comparisons only)."""

import numpy as np
import scipy.sparse as sp


def to_scipy(rowptr, col, val, M):
    """Device CSR tensors -> scipy CSR on the host."""
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rowptr.cpu().numpy()), shape=(M, M))


def rel_matrix_err(A, B):
    """max |A - B| over the union of patterns, relative to max |B|."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    d = (A - B).tocsr()
    scale = np.max(np.abs(B.data)) if B.nnz else 1.0
    return (np.max(np.abs(d.data)) if d.nnz else 0.0) / scale


def rel_vec_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def flush(msg):
    print(msg, flush=True)
