"""Edge cases and error paths of the C ABI on the GPU.

Every error here is detected by a host-side check or by a kernel that only
raises a flag; none of them can touch memory out of bounds.
"""

import ctypes

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from helpers import flush, rel_matrix_err, rel_vec_err, to_scipy
from oracle import basis as ob, lindblad as lb, o2
from workloads import dimer, random_ops

pytestmark = pytest.mark.gpu


def test_non_hermitian_hamiltonian_rejected(lib):
    flush("[edge] non-Hermitian H")
    b = lib.build_basis(4)
    H = random_ops.random_complex_csr(4, 0.8, seed=1)
    with pytest.raises(lib.SunError) as e:
        lib.Lindbladian(b, [H], [])
    assert "Hermitian" in str(e.value) and e.value.code == -1


def test_dissipator_with_trace_matches_definition(lib):
    """A dissipator with a trace (taken through the gauge identity on the GPU)
    against the oracle's R and K from explicit traces of D_L itself: a dense
    random L at N = 5 and a banded one at N = 31."""
    N = 5
    b = lib.build_basis(N)
    L = random_ops.random_complex_csr(N, 0.8, seed=2, traceless=False)
    assert abs(np.trace(L.to_dense())) > 0.1
    lind = lib.Lindbladian(b, [], [L])
    rp, c, v, K = lind.export("L", 0)
    F = ob.generators(N)
    assert rel_matrix_err(to_scipy(rp, c, v, N * N - 1), lb.q_dissipator(F, L.to_dense())) <= 1e-12
    assert rel_vec_err(K.cpu().numpy(), lb.k_dissipator(F, L.to_dense())) <= 1e-12
    N = 31
    rng = np.random.default_rng(8)
    diags = {k: rng.standard_normal(N - abs(k)) + 1j * rng.standard_normal(N - abs(k)) for k in (-1, 0, 1)}
    diags[0] = diags[0] + (2.0 - 0.5j)                 # a sizeable trace
    Lb = dimer.ZCSR.from_diagonals(N, diags)
    lind = lib.Lindbladian(lib.build_basis(N), [], [Lb])
    rp, c, v, K = lind.export("L", 0)
    M = N * N - 1
    assert rel_matrix_err(to_scipy(rp, c, v, M), lb.q_full("L", Lb)) <= 1e-12
    assert rel_vec_err(K.cpu().numpy(), lb.k_vector(Lb)) <= 1e-12


def test_negative_rate_rejected(lib):
    p = dimer.plain_config(4)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(4)
    lind = lib.Lindbladian(b, [ops["H0"], ops["H1"]], [ops["L"]])
    with pytest.raises(lib.SunError) as e:
        lind.propagator([1.0, 0.0, -0.1], [1])
    assert e.value.code == -1


def test_malformed_csr_rejected(lib):
    b = lib.build_basis(3)
    bad = sp.csr_matrix(np.eye(3, dtype=complex))
    op = lib.DeviceOperator.from_csr(bad)
    op.col[0] = 7                                    # column out of range
    with pytest.raises(lib.SunError) as e:
        lib.Lindbladian(b, [op], [])
    assert e.value.code == -1
    op2 = lib.DeviceOperator.from_csr(sp.csr_matrix(np.ones((3, 3), dtype=complex)))
    op2.col[1] = 0                                   # not strictly increasing
    with pytest.raises(lib.SunError):
        lib.Lindbladian(b, [op2], [])
    with pytest.raises(lib.SunError):               # wrong dimension
        lib.Lindbladian(b, [sp.csr_matrix(np.eye(4, dtype=complex))], [])


def test_zero_operator_and_smallest_system(lib):
    """N = 2 (M = 3) with a zero Hamiltonian term and a real Hermitian L (K=0)."""
    b = lib.build_basis(2)
    Z = sp.csr_matrix((2, 2), dtype=complex)
    Lh = sp.csr_matrix(np.array([[1.0, 0.5], [0.5, -1.0]], dtype=complex))
    lind = lib.Lindbladian(b, [Z], [Lh])
    assert lind.nnz("H", 0) == 0
    rp, c, v, K = lind.export("L", 0)
    F = ob.generators(2)
    assert rel_matrix_err(to_scipy(rp, c, v, 3), lb.q_dissipator(F, Lh.toarray())) <= 1e-12
    assert np.max(np.abs(K.cpu().numpy())) == 0.0
    prop = lind.propagator([1.0, 0.7], [])
    v0 = torch.tensor([0.1, -0.2, 0.3], dtype=torch.float64, device="cuda")
    prop.propagate(v0, None, 0.01, 10)
    assert torch.isfinite(v0).all()


def test_expand_operator_matches_traces(lib):
    """Bloch coordinates of a random non-Hermitian operator and its trace."""
    N = 5
    b = lib.build_basis(N)
    X = random_ops.random_complex_csr(N, 0.6, seed=9, traceless=False)
    x, tr = b.expand(X)
    F = ob.generators(N)
    want = lb.expand(F, X.to_dense())
    np.testing.assert_allclose(x.cpu().numpy(), want, atol=1e-14)
    assert abs(tr - np.trace(X.to_dense())) < 1e-13


def test_banded_random_operators_larger_N(lib):
    """Random tridiagonal Hermitian H and a random tridiagonal complex L at
    N = 31 (pattern like the dimer, random values) against the column tier."""
    N = 31
    flush(f"[edge] random banded N={N}")
    H = random_ops.random_tridiagonal_hermitian(N, seed=4)
    rng = np.random.default_rng(5)
    off1 = rng.standard_normal(N - 1) + 1j * rng.standard_normal(N - 1)
    off2 = rng.standard_normal(N - 1) + 1j * rng.standard_normal(N - 1)
    dia = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    dia -= dia.mean()
    L = dimer.ZCSR.from_diagonals(N, {-1: off1, 0: dia, 1: off2})
    b = lib.build_basis(N)
    lind = lib.Lindbladian(b, [H], [L])
    M = N * N - 1
    assert rel_matrix_err(to_scipy(*lind.export("H", 0), M), lb.q_full("H", H)) <= 1e-12
    rp, c, v, K = lind.export("L", 0)
    assert rel_matrix_err(to_scipy(rp, c, v, M), lb.q_full("L", L)) <= 1e-12
    assert rel_vec_err(K.cpu().numpy(), lb.k_vector(L)) <= 1e-12


def test_dense_operator_beyond_row_capacity_takes_dense_path(lib):
    """A dense complex L at N = 40 gives product rows beyond the sparse
    assembly's LDS sort capacity (detected from the per-row counts before
    anything is filled); the default assembly then takes the dense path, and
    R and K equal the C oracle's explicit traces to 1e-12."""
    N = 40
    flush(f"[edge] dense L beyond the sparse row capacity N={N}")
    M = N * N - 1
    b = lib.build_basis(N)
    L = random_ops.random_complex_csr(N, 1.0, seed=3)
    lind = lib.Lindbladian(b, [], [L])
    rp, c, v, k = lind.export("L", 0)
    assert rel_matrix_err(to_scipy(rp, c, v, M), o2.q_full("L", L)) <= 1e-12
    assert rel_vec_err(k.cpu().numpy(), o2.k_vector(L)) <= 1e-12


def test_dense_path_size_limit_is_refused(lib):
    """Past the dense path's index limit (M^2 >= 2^33, N = 305) a dense L is
    refused with SUN_ENOTSUP before any dense array is allocated."""
    N = 305
    flush(f"[edge] dense path limit N={N}")
    b = lib.build_basis(N)
    L = random_ops.random_complex_csr(N, 1.0, seed=5)
    with pytest.raises(lib.SunError) as e:
        lib.Lindbladian(b, [], [L], dense=True)
    assert e.value.code == -4
    assert "dense path" in str(e.value)


def test_propagate_argument_checks(lib):
    p = dimer.plain_config(4)
    ops = dimer.dimer_operators(p)
    b = lib.build_basis(4)
    lind, prop = lib.expand_lindbladian(b, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    from paper_1812_11626_amd import _lib
    L = _lib.load()
    v = torch.zeros(15, dtype=torch.float64, device="cuda")
    assert L.sun_propagate(prop.handle, ctypes.c_void_p(v.data_ptr()), None, ctypes.c_double(0.1),
                           ctypes.c_int64(5), None) == _lib.SUN_EINVAL          # coef missing
    assert L.sun_propagate(prop.handle, ctypes.c_void_p(v.data_ptr()), None, ctypes.c_double(0.1),
                           ctypes.c_int64(-1), None) == _lib.SUN_EINVAL         # negative steps
    with pytest.raises(lib.SunError):
        prop.tune(100, 256, False)                                              # not a power of two
    with pytest.raises(lib.SunError):
        prop.tune_sliced(4096, 64, 3)                                           # bad byte width
    with pytest.raises(lib.SunError):
        prop.tune_sliced(unroll=5)                                              # unsupported unroll
    with pytest.raises(lib.SunError):
        prop.tune_sliced(split=3)                                               # 1, 2 or 4 wavefronts per slice
    with pytest.raises(lib.SunError):
        prop.tune_sliced(split=2, unroll=12)                                    # split slices take 4 or 8 per round
    with pytest.raises(lib.SunError):
        lind.propagator([1.0, 0.0, 0.1], [0, 1, 2, 0, 1])                       # > 4 dynamic terms


def test_batch_tune_argument_checks(lib):
    from helpers import dimer_batch
    inst = [dimer.plain_config(4) for _ in range(3)]
    bp, _ = dimer_batch(lib, inst, 4)
    for tile, rows, path in ((12, 64, 0),        # tile not a power of two in range
                             (64, 0, 0),         # no rows per item
                             (16, 64, 4),        # unknown path
                             (64, 64, 3),        # path 3 takes tiles 8, 16, 32
                             (128, 64, 3)):
        with pytest.raises(lib.SunError):
            bp.tune(0, tile, rows, path)
    bp.tune(0, 16, 64, 3)                        # valid after the rejected calls
    bp.run(4)
