"""Python binding of the sunbloch C ABI (argument marshalling only).

Device memory and streams come from PyTorch (ROCm); every computation runs in
the HIP library.  There is no CPU fallback: without a GPU or without
libsunbloch.so every call raises.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import SUN_TERM_H, SUN_TERM_L, ZCSR, check


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("sunbloch needs a HIP GPU (torch.cuda.is_available() is False)")
    _lib.load()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


@dataclass
class DeviceOperator:
    """An N x N operator in CSR form on the GPU (keeps the tensors alive)."""

    n: int
    rowptr: torch.Tensor
    col: torch.Tensor
    re: torch.Tensor
    im: torch.Tensor | None

    @staticmethod
    def from_csr(op, device="cuda") -> "DeviceOperator":
        """From an object with n, indptr, indices, re, im (e.g. workloads.ZCSR)
        or a scipy sparse matrix."""
        if hasattr(op, "indptr") and hasattr(op, "re"):
            n, indptr, indices, re, im = op.n, op.indptr, op.indices, op.re, op.im
        else:
            import scipy.sparse as sp
            m = sp.csr_matrix(op)
            m.sort_indices()
            n = m.shape[0]
            indptr, indices = m.indptr, m.indices
            re, im = np.real(m.data), np.imag(m.data)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        return DeviceOperator(int(n), t(indptr, torch.int32), t(indices, torch.int32),
                              t(re, torch.float64), t(im, torch.float64))

    def as_struct(self) -> ZCSR:
        return ZCSR(self.n, int(self.col.numel()), self.rowptr.data_ptr(), self.col.data_ptr(),
                    self.re.data_ptr(), 0 if self.im is None else self.im.data_ptr())


def _dev_op(op) -> DeviceOperator:
    return op if isinstance(op, DeviceOperator) else DeviceOperator.from_csr(op)


class Basis:
    """SU(N) basis metadata on the GPU (sun_build_basis)."""

    def __init__(self, N: int):
        require_gpu()
        self._lib = _lib.load()
        h = C.c_void_p()
        check(self._lib.sun_build_basis(int(N), _stream(), C.byref(h)))
        self.handle = h
        self.N = int(N)
        self.M = self.N * self.N - 1
        self.P = self.N * (self.N - 1) // 2

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.sun_basis_free(self.handle)
            self.handle = None

    def counts(self):
        """(nnz_f, nnz_d) of the full structure-constant tensors."""
        nf, nd = C.c_int64(), C.c_int64()
        check(self._lib.sun_basis_counts(self.handle, _stream(), C.byref(nf), C.byref(nd)))
        return nf.value, nd.value

    def export(self, which: str, canonical: bool = False):
        """Nonzero entries of f ('f') or d ('d'): (idx int32 (nnz,3), val
        float64), all index orders, or with canonical=True only m<n<s (f) /
        m<=n<=s (d)."""
        w = {"f": 0, "d": 1}[which]
        c = int(bool(canonical))
        n = C.c_int64()
        st = self._lib.sun_basis_export(self.handle, w, c, None, None, 0, C.byref(n), _stream())
        if st not in (_lib.SUN_OK, _lib.SUN_ERANGE):
            check(st)
        idx = torch.empty((max(n.value, 1), 3), dtype=torch.int32, device="cuda")
        val = torch.empty(max(n.value, 1), dtype=torch.float64, device="cuda")
        check(self._lib.sun_basis_export(self.handle, w, c, _ptr(idx), _ptr(val), n.value, C.byref(n), _stream()))
        return idx[: n.value], val[: n.value]

    def expand(self, op):
        """Coefficients x_m = Tr(F_m X) (complex128 tensor) and Tr(X)."""
        d = _dev_op(op)
        re = torch.empty(self.M, dtype=torch.float64, device="cuda")
        im = torch.empty(self.M, dtype=torch.float64, device="cuda")
        tr = (C.c_double * 2)()
        s = d.as_struct()
        check(self._lib.sun_expand_operator(self.handle, C.byref(s), _ptr(re), _ptr(im), tr, _stream()))
        return torch.complex(re, im), complex(tr[0], tr[1])

    def density(self, v: torch.Tensor) -> torch.Tensor:
        """rho = 1/N + sum_j v_j F_j (eq. 5) as a complex128 (N, N) tensor."""
        assert v.dtype == torch.float64 and v.is_cuda and v.is_contiguous() and v.numel() == self.M
        re = torch.empty((self.N, self.N), dtype=torch.float64, device="cuda")
        im = torch.empty((self.N, self.N), dtype=torch.float64, device="cuda")
        check(self._lib.sun_bloch_density(self.handle, _ptr(v), _ptr(re), _ptr(im), _stream()))
        return torch.complex(re, im)

    def observable(self, op):
        """(x, x0): real coefficients x_j = Re Tr(F_j X) (float64 (M,) tensor)
        and Re Tr(X)/N of a Hermitian X, as taken by Propagator.record."""
        x, tr = self.expand(op)
        return x.real.contiguous(), tr.real / self.N

    def expect(self, v: torch.Tensor, op) -> torch.Tensor:
        """Tr(rho X) for one Bloch vector (shape (M,)) or a stack (shape (n, M)
        or any 2-D view with unit column stride); complex128 result."""
        assert v.dtype == torch.float64 and v.is_cuda and v.shape[-1] == self.M and v.stride(-1) == 1
        vv = v if v.dim() == 2 else v.reshape(1, self.M)
        n = vv.shape[0]
        x, tr = self.expand(op)
        xr, xi = x.real.contiguous(), x.imag.contiguous()
        t = (C.c_double * 2)(tr.real, tr.imag)
        out_re = torch.empty(n, dtype=torch.float64, device="cuda")
        out_im = torch.empty(n, dtype=torch.float64, device="cuda")
        ld = vv.stride(0) if n > 1 else self.M
        check(self._lib.sun_bloch_expect(self.handle, _ptr(vv), n, ld, _ptr(xr), _ptr(xi), t, _ptr(out_re),
                                         _ptr(out_im), _stream()))
        out = torch.complex(out_re, out_im)
        return out if v.dim() == 2 else out[0]


_ALLOCATOR = None   # the installed ctypes callbacks (kept alive while installed)


def use_torch_allocator():
    """Route every device allocation of the library (object layouts, assembly
    temporaries, work buffers) through PyTorch's caching allocator, on the
    stream of the library call that allocates, so that PyTorch accounts for
    the memory (torch.cuda.memory_allocated) and can reuse it.  Buffers
    allocated before the switch are still released by hipFree."""
    global _ALLOCATOR

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:                           # out of memory: the library returns SUN_ENOMEM
            return None

    def _release(ptr, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    cbs = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
    check(_lib.load().sun_set_allocator(cbs[0], cbs[1], None))
    _ALLOCATOR = cbs


def use_default_allocator():
    """Back to hipMalloc/hipFree for new allocations (buffers allocated
    through PyTorch are still released through it)."""
    global _ALLOCATOR
    check(_lib.load().sun_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None))
    # the old callbacks must outlive every buffer they allocated: keep them
    if _ALLOCATOR is not None:
        _RETIRED_ALLOCATORS.append(_ALLOCATOR)
    _ALLOCATOR = None


_RETIRED_ALLOCATORS = []


def gemm_f64(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None, alpha: float = 1.0,
             beta: float = 0.0) -> torch.Tensor:
    """C = alpha A B + beta C on the matrix cores (sun_gemm_f64); float64
    CUDA tensors, row-major with unit column stride."""
    assert A.dtype == B.dtype == torch.float64 and A.is_cuda and B.is_cuda
    assert A.dim() == B.dim() == 2 and A.shape[1] == B.shape[0] and A.stride(1) == 1 and B.stride(1) == 1
    M, K = A.shape
    N = B.shape[1]
    if C is None:
        C = torch.empty((M, N), dtype=torch.float64, device="cuda")
        beta = 0.0
    assert C.shape == (M, N) and C.stride(1) == 1
    check(_lib.load().sun_gemm_f64(M, N, K, float(alpha), _ptr(A), A.stride(0), _ptr(B), B.stride(0), float(beta),
                                   _ptr(C), C.stride(0), _stream()))
    return C


def build_basis(N: int) -> Basis:
    return Basis(N)


class Lindbladian:
    """Assembled Bloch-form generator: Q_a per Hamiltonian term, R_p and K_p
    per dissipator (unit rates), kept on the GPU (sun_expand_lindbladian)."""

    def __init__(self, basis: Basis, H: list, L: list, dense: bool = False):
        """dense=True assembles every term by the dense path (dense sections,
        R by a matrix-core product); otherwise the sparse row path, which
        switches to the dense one for terms beyond its per-row limit."""
        self.basis = basis
        self._lib = basis._lib
        hs = [_dev_op(h) for h in H]
        ls = [_dev_op(l) for l in L]
        Harr = (ZCSR * max(1, len(hs)))(*[h.as_struct() for h in hs])
        Larr = (ZCSR * max(1, len(ls)))(*[l.as_struct() for l in ls])
        h = C.c_void_p()
        fn = self._lib.sun_expand_lindbladian_dense if dense else self._lib.sun_expand_lindbladian
        check(fn(basis.handle, Harr, len(hs), Larr, len(ls), _stream(), C.byref(h)))
        self.handle = h
        self.nH = len(hs)
        self.P = len(ls)

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.sun_lind_free(self.handle)
            self.handle = None

    def device_bytes(self) -> int:
        """Device memory the assembled terms hold."""
        b = C.c_size_t()
        check(self._lib.sun_lind_device_bytes(self.handle, C.byref(b)))
        return int(b.value)

    def nnz(self, which: str, index: int) -> int:
        w = SUN_TERM_H if which == "H" else SUN_TERM_L
        n = C.c_int64()
        check(self._lib.sun_lind_nnz(self.handle, w, int(index), C.byref(n)))
        return n.value

    def export(self, which: str, index: int):
        """(rowptr, col, val[, K]) device tensors of Q_index ('H') or R_index ('L')."""
        w = SUN_TERM_H if which == "H" else SUN_TERM_L
        n = self.nnz(which, index)
        M = self.basis.M
        rowptr = torch.empty(M + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        K = torch.empty(M, dtype=torch.float64, device="cuda") if w == SUN_TERM_L else None
        check(self._lib.sun_lind_export(self.handle, w, int(index), _ptr(rowptr), _ptr(col), _ptr(val),
                                        _ptr(K), _stream()))
        if K is None:
            return rowptr, col[:n], val[:n]
        return rowptr, col[:n], val[:n], K

    def propagator(self, static_w, dyn=()) -> "Propagator":
        return Propagator(self, static_w, dyn)


def expand_lindbladian(basis: Basis, H0, H1=None, dissipators=()):
    """H0 (constant), H1 (multiplied by eps(t)) and [(L_p, gamma_p)]:
    returns (Lindbladian, Propagator) with G(t) = Q_H0 + eps(t) Q_H1 +
    sum_p gamma_p R_p and K = sum_p gamma_p K_p."""
    Hs = [H0] + ([H1] if H1 is not None else [])
    Ls = [l for l, _ in dissipators]
    lind = Lindbladian(basis, Hs, Ls)
    w = [1.0] + ([0.0] if H1 is not None else []) + [float(g) for _, g in dissipators]
    dyn = [1] if H1 is not None else []
    return lind, lind.propagator(w, dyn)


class Propagator:
    """RK4 propagator over a fused static + dynamic layout (sun_prop_create)."""

    def __init__(self, lind: Lindbladian, static_w, dyn=()):
        self.lind = lind
        self._lib = lind._lib
        w = (C.c_double * len(static_w))(*[float(x) for x in static_w])
        dyn = list(dyn)
        d = (C.c_int32 * max(1, len(dyn)))(*dyn)
        h = C.c_void_p()
        check(self._lib.sun_prop_create(lind.handle, w, d, len(dyn), _stream(), C.byref(h)))
        self.handle = h
        self.ndyn = len(dyn)
        self.M = lind.basis.M

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.sun_prop_free(self.handle)
            self.handle = None

    def info(self):
        nnz, nb, M = C.c_int64(), C.c_int64(), C.c_int64()
        check(self._lib.sun_prop_info(self.handle, C.byref(nnz), C.byref(nb), C.byref(M)))
        return {"nnz_fused": nnz.value, "nblocks": nb.value, "M": M.value}

    def tune(self, block_nnz: int = 1024, threads: int = 256, xcd_remap: bool = False):
        """Select the CSR-stream layout with these knobs."""
        check(self._lib.sun_prop_tune(self.handle, int(block_nnz), int(threads), int(bool(xcd_remap)),
                                      _stream()))

    def tune_sliced(self, sigma: int = 4096, long_len: int = 32, min_col_bytes: int = 1, xcd_remap: bool = True,
                    nontemporal: bool = False, unroll: int = 0, pairs: bool = False, split: int = 0):
        """Select the sliced-ELL layout with these knobs (unroll: entries a
        lane loads per round; split: wavefronts per slice, 1, 2 or 4; 0 for
        either = the size-based choice)."""
        flags = int(bool(xcd_remap)) | (int(bool(nontemporal)) << 1) | (int(bool(pairs)) << 2) | \
            ((int(unroll) & 0xFF) << 16) | ((int(split) & 7) << 24)
        check(self._lib.sun_prop_tune_sliced(self.handle, int(sigma), int(long_len), int(min_col_bytes), flags,
                                             _stream()))

    def device_bytes(self) -> int:
        """Device memory this propagator holds."""
        b = C.c_size_t()
        check(self._lib.sun_prop_device_bytes(self.handle, C.byref(b)))
        return int(b.value)

    def use_graphs(self, mode: int = 1):
        """HIP-graph replay of 64-step chunks in propagate: 0 never, 1 where
        M <= 160,000 (default), 2 always."""
        check(self._lib.sun_prop_use_graphs(self.handle, int(mode)))

    def tune_resident(self, on: bool = True):
        """Run all steps of a call in one single-workgroup launch (small systems)."""
        check(self._lib.sun_prop_tune_resident(self.handle, int(bool(on))))

    def layout(self):
        lay, stored, nlong, nb = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        check(self._lib.sun_prop_layout(self.handle, C.byref(lay), C.byref(stored), C.byref(nlong), C.byref(nb)))
        name = {0: "stream", 1: "sliced", 2: "sliced-segmented"}.get(lay.value, "stream")
        return {"layout": name, "stored_entries": stored.value,
                "long_rows": nlong.value, "matrix_bytes_per_launch": nb.value}

    def propagate(self, v: torch.Tensor, coef: torch.Tensor | None, dt: float, steps: int) -> torch.Tensor:
        """In-place RK4 on v (float64 cuda tensor of length M); coef is the
        (2*steps+1, ndyn) half-step coefficient table on the GPU."""
        assert v.dtype == torch.float64 and v.is_cuda and v.is_contiguous() and v.numel() == self.M
        if self.ndyn:
            assert coef is not None and coef.dtype == torch.float64 and coef.is_cuda and coef.is_contiguous()
            assert coef.numel() >= (2 * steps + 1) * self.ndyn
        check(self._lib.sun_propagate(self.handle, _ptr(v), _ptr(coef), float(dt), int(steps), _stream()))
        return v

    def guard_stability(self, coef_lo=(), coef_hi=(), iters: int = 200, limit: float = 0.0) -> float:
        """Estimate |lambda|max at the corners of the coefficient box and
        refuse later steps with |dt| |lambda|max > limit (0: 2.6, inside RK4's
        stability region everywhere in the left half-plane; < 0: guard off).
        Returns the estimate."""
        lo, hi = list(coef_lo), list(coef_hi)
        assert len(lo) == len(hi) == self.ndyn
        blo = (C.c_double * max(1, len(lo)))(*[float(x) for x in lo])
        bhi = (C.c_double * max(1, len(hi)))(*[float(x) for x in hi])
        rho = C.c_double()
        check(self._lib.sun_prop_guard_stability(self.handle, blo, bhi, int(iters), float(limit), C.byref(rho),
                                                 _stream()))
        self._guard = (lo, hi) if limit >= 0 else None
        return rho.value

    def stationary(self, coef=(), dt: float = 0.0, tau: float = 1.0, restart: int = 80, max_iter: int = 800,
                   tol: float = 1e-10, v0: torch.Tensor | None = None):
        """Stationary state of the generator with the time-dependent
        coefficients frozen at ``coef``: G v = -K by GMRES on the RK4
        time-tau map (sun_stationary).  dt: a stable RK4 step (default: 2.5 /
        |lambda|max from the power iteration).  Returns (v, iterations,
        ||G v + K|| / ||K||)."""
        c = list(coef)
        assert len(c) == self.ndyn
        buf = (C.c_double * max(1, len(c)))(*[float(x) for x in c])
        if not dt:
            dt = 2.5 / self.spectral_radius(c)
        n = max(1, int(round(tau / dt)))
        v = torch.zeros(self.M, dtype=torch.float64, device="cuda") if v0 is None \
            else v0.detach().to("cuda", torch.float64).clone().contiguous()
        it, rr = C.c_int32(), C.c_double()
        check(self._lib.sun_stationary(self.handle, buf, float(dt), n, int(restart), int(max_iter), float(tol),
                                       _ptr(v), C.byref(it), C.byref(rr), _stream()))
        return v, it.value, rr.value

    def check_finite(self, on: bool = True):
        """Finite check of the state at the end of every propagation call
        (on by default; SUN_EDIVERGED when it fails)."""
        check(self._lib.sun_prop_check_finite(self.handle, int(bool(on))))

    def spectral_radius(self, coef=(), iters: int = 200) -> float:
        """|lambda|max of the generator's linear part with the time-dependent
        coefficients frozen at `coef` (power iteration on the GPU)."""
        c = list(coef)
        assert len(c) == self.ndyn
        buf = (C.c_double * max(1, len(c)))(*[float(x) for x in c])
        rho = C.c_double()
        check(self._lib.sun_prop_spectral_radius(self.handle, buf, int(iters), C.byref(rho), _stream()))
        return rho.value

    def record(self, v: torch.Tensor, coef: torch.Tensor | None, dt: float, steps: int, every: int,
               states: bool = True, observable=None, noalloc: bool = False):
        """RK4 like ``propagate`` (in place on v), recording after every
        ``every`` steps.  Returns (states (nrec, M) or None, obs (nrec,) or
        None); observable = (x, x0) gives obs = x0 + x . v (e.g. from
        Basis.observable).  noalloc=True calls sun_propagate_record_noalloc
        (the library allocates nothing during the call)."""
        assert v.dtype == torch.float64 and v.is_cuda and v.is_contiguous() and v.numel() == self.M
        if self.ndyn:
            assert coef is not None and coef.dtype == torch.float64 and coef.is_cuda and coef.is_contiguous()
            assert coef.numel() >= (2 * steps + 1) * self.ndyn
        nrec = int(steps) // int(every)
        st = torch.empty((nrec, self.M), dtype=torch.float64, device="cuda") if states else None
        x, x0, obs = None, 0.0, None
        if observable is not None:
            x, x0 = observable
            assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == self.M
            obs = torch.empty(nrec, dtype=torch.float64, device="cuda")
        fn = self._lib.sun_propagate_record_noalloc if noalloc else self._lib.sun_propagate_record
        check(fn(self.handle, _ptr(v), _ptr(coef), float(dt), int(steps), int(every), _ptr(st), self.M, _ptr(x),
                 float(x0), _ptr(obs), _stream()))
        return st, obs


def _profile(self, v, coef, dt, steps):
    """Propagate like ``propagate`` while timing every stage launch with HIP
    events on the launch stream.  Returns per-stage summed ms (list of 4) and
    the launch count."""
    ms = (C.c_double * 4)()
    n = C.c_int64()
    check(self._lib.sun_propagate_profile(self.handle, _ptr(v), _ptr(coef), float(dt), int(steps), _stream(),
                                          ms, C.byref(n)))
    return list(ms), n.value


Propagator.profile = _profile


def propagate(prop: Propagator, v0, eps, dt: float, steps: int) -> torch.Tensor:
    """propagate(v0, eps(t), dt, steps): eps is a (2*steps+1,) table (numpy)
    or a callable sampled on the half-step grid t = k dt/2.  Sets the
    propagator's stability guard over the table's range first (a step beyond
    RK4's stability bound raises SUN_EUNSTABLE) and returns the new state (the
    finite check raises SUN_EDIVERGED for a non-finite one)."""
    if callable(eps):
        t = np.arange(2 * steps + 1) * (0.5 * dt)
        eps = np.asarray([eps(x) for x in t], dtype=np.float64)
    table = np.asarray(eps, dtype=np.float64).reshape(2 * steps + 1, -1) if prop.ndyn else None
    if table is not None and steps > 0:
        # stability guard over the drive range of this table (estimated once
        # per propagator and range; SUN_EUNSTABLE for a step that is too large)
        lo, hi = list(np.nanmin(table, axis=0)), list(np.nanmax(table, axis=0))   # NaNs: the finite check
        g = getattr(prop, "_guard", None)
        if g is None or any(a < b for a, b in zip(lo, g[0])) or any(a > b for a, b in zip(hi, g[1])):
            prop.guard_stability(lo, hi)
    elif getattr(prop, "_guard", None) is None and steps > 0:
        prop.guard_stability()
    coef = torch.as_tensor(table).cuda().contiguous() if table is not None else None
    v = torch.as_tensor(np.asarray(v0, dtype=np.float64)).cuda().clone() if not torch.is_tensor(v0) \
        else v0.detach().to("cuda", torch.float64).clone()
    return prop.propagate(v, coef, dt, steps)


class BatchedPropagator:
    """Many parameter instances advanced together (sun_batch_*).

    groups: list of dicts with keys
      lind  -- Lindbladian shared by the group's instances
      w, u  -- (B, nt) coefficient arrays: c_{b,a}(t_k) = w[b,a] + u[b,a] wave[k]
      wave  -- (2*steps+1,) waveform on the half-step grid
      dt, steps
    """

    def __init__(self, groups):
        require_gpu()
        self._lib = _lib.load()
        self.groups = []
        keep = []
        for g in groups:
            lind = g["lind"]
            nt = lind.nH + lind.P
            w = torch.as_tensor(np.asarray(g["w"], dtype=np.float64).reshape(-1, nt)).cuda().contiguous()
            u = torch.as_tensor(np.asarray(g["u"], dtype=np.float64).reshape(-1, nt)).cuda().contiguous()
            wave = torch.as_tensor(np.asarray(g["wave"], dtype=np.float64)).cuda().contiguous()
            assert wave.numel() >= 2 * int(g["steps"]) + 1
            self.groups.append(dict(lind=lind, w=w, u=u, wave=wave, dt=float(g["dt"]), steps=int(g["steps"]),
                                    B=w.shape[0], M=lind.basis.M, N=lind.basis.N, nt=nt))
            keep.append(lind)
        n = len(self.groups)
        linds = (C.c_void_p * n)(*[g["lind"].handle.value for g in self.groups])
        B = (C.c_int32 * n)(*[g["B"] for g in self.groups])
        wp = (C.c_void_p * n)(*[g["w"].data_ptr() for g in self.groups])
        up = (C.c_void_p * n)(*[g["u"].data_ptr() for g in self.groups])
        vp = (C.c_void_p * n)(*[g["wave"].data_ptr() for g in self.groups])
        dt = (C.c_double * n)(*[g["dt"] for g in self.groups])
        st = (C.c_int64 * n)(*[g["steps"] for g in self.groups])
        h = C.c_void_p()
        check(self._lib.sun_batch_create(linds, n, B, wp, up, vp, dt, st, _stream(), C.byref(h)))
        self.handle = h
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.sun_batch_free(self.handle)
            self.handle = None

    def set_state(self, g: int, V: torch.Tensor):
        G = self.groups[g]
        V = V.to("cuda", torch.float64).contiguous()
        assert V.shape == (G["B"], G["M"])
        check(self._lib.sun_batch_set_state(self.handle, int(g), _ptr(V), _stream()))
        torch.cuda.current_stream().synchronize()

    def get_state(self, g: int) -> torch.Tensor:
        G = self.groups[g]
        V = torch.empty((G["B"], G["M"]), dtype=torch.float64, device="cuda")
        check(self._lib.sun_batch_get_state(self.handle, int(g), _ptr(V), _stream()))
        return V

    def run(self, nsteps: int, only_group: int = -1):
        check(self._lib.sun_batch_run(self.handle, int(nsteps), int(only_group), _stream()))

    def tune(self, g: int, tile: int, rows_per_item: int, path: int = 0):
        """Tiling of group g; path 0 = LDS-staged row blocks (when every row
        fits), 1 = one wavefront per (rows, tile) reading the matrix from
        global memory, 2 = path 0 with two instances per lane for every tile
        width, 3 = path 2 with the gathered state rows staged in LDS as well
        (tiles 8, 16, 32). 4 = instance-major state on a
        segmented sliced layout (tile = 2, 4 or 8 instances per wavefront;
        needs 1 to 3 terms whose coefficients differ between instances),
        5 = one wavefront per (row, tile of 64 or 128), 7 = persistent
        workgroups with each block's gathered state rows staged in LDS
        while the previous block is summed (tile 64, rows_per_item <= 32)"""
        check(self._lib.sun_batch_tune(self.handle, int(g), int(tile), int(rows_per_item), int(path), _stream()))

    def device_bytes(self) -> int:
        """Device memory the batch holds (every group's layout and states)."""
        b = C.c_size_t()
        check(self._lib.sun_batch_device_bytes(self.handle, C.byref(b)))
        return int(b.value)

    def info(self, g: int):
        M, nnz, tile, rows = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        check(self._lib.sun_batch_info(self.handle, int(g), C.byref(M), C.byref(nnz), C.byref(tile),
                                       C.byref(rows)))
        return {"M": M.value, "nnz": nnz.value, "tile": tile.value, "rows_per_item": rows.value}


class Adjoint:
    """Forward + transposed propagators for the discrete adjoint (sun_adjoint_*)."""

    def __init__(self, lind: Lindbladian, static_w, dyn=()):
        self.lind = lind
        self._lib = lind._lib
        self.nt = lind.nH + lind.P
        w = (C.c_double * self.nt)(*[float(x) for x in static_w])
        dyn = list(dyn)
        d = (C.c_int32 * max(1, len(dyn)))(*dyn)
        h = C.c_void_p()
        check(self._lib.sun_adjoint_create(lind.handle, w, d, len(dyn), _stream(), C.byref(h)))
        self.handle = h
        self.ndyn = len(dyn)
        self.M = lind.basis.M

    def __del__(self):
        if getattr(self, "handle", None):
            self._lib.sun_adjoint_free(self.handle)
            self.handle = None

    def set_weights(self, static_w):
        """New static weights for the same terms (only the forward propagator is rebuilt)."""
        w = (C.c_double * self.nt)(*[float(x) for x in static_w])
        check(self._lib.sun_adjoint_set_weights(self.handle, w, _stream()))

    def plan(self, dstatic, steps, ckpt_every):
        """(workspace bytes that keep the stage inputs, minimum workspace bytes)."""
        dstatic = np.ascontiguousarray(np.asarray(dstatic, dtype=np.float64).reshape(self.nt, -1))
        full, low = C.c_size_t(), C.c_size_t()
        check(self._lib.sun_adjoint_plan(self.handle, dstatic.ctypes.data_as(C.POINTER(C.c_double)),
                                         dstatic.shape[1], int(steps), int(ckpt_every), _stream(), C.byref(full),
                                         C.byref(low)))
        return full.value, low.value

    def run(self, v0, coef, dstatic, dcoef, cobs, dt, steps, S_avg, ckpt_every, workspace=None):
        """(J, dJ/dtheta).  dstatic: host (nt, ntheta); dcoef: device
        (2*steps+1, ndyn, ntheta) tensor or None.  The workspace is a uint8
        CUDA tensor from PyTorch's allocator (sized by ``plan`` when not
        given), so the run's device memory is PyTorch's."""
        dstatic = np.ascontiguousarray(np.asarray(dstatic, dtype=np.float64).reshape(self.nt, -1))
        ntheta = dstatic.shape[1]
        ds = dstatic.ctypes.data_as(C.POINTER(C.c_double))
        if workspace is None:
            full, _ = self.plan(dstatic, steps, ckpt_every)
            workspace = torch.empty(full, dtype=torch.uint8, device="cuda")
        J = C.c_double()
        g = (C.c_double * max(1, ntheta))()
        check(self._lib.sun_adjoint_execute(self.handle, _ptr(v0), _ptr(coef), ds, _ptr(dcoef), ntheta, _ptr(cobs),
                                            float(dt), int(steps), int(S_avg), int(ckpt_every), _ptr(workspace),
                                            workspace.numel(), C.byref(J), g, _stream()))
        return J.value, np.array(g[:ntheta])

    def objective(self, v0, coef, cobs, dt, steps, S_avg):
        J = C.c_double()
        check(self._lib.sun_adjoint_objective(self.handle, _ptr(v0), _ptr(coef), _ptr(cobs), float(dt), int(steps),
                                              int(S_avg), C.byref(J), _stream()))
        return J.value


class AdjointProblem:
    """A parametrised propagation problem for the adjoint form.

    lind       -- assembled terms T_a (fixed)
    param_map  -- callable theta -> dict(static_w (nt,), dyn (list), coef
                  (2*steps+1, ndyn) array, dstatic (nt, ntheta), dcoef
                  (2*steps+1, ndyn, ntheta) array)
    v0, cobs   -- device tensors (length M): initial Bloch vector and the
                  observable's coefficients
    """

    def __init__(self, lind, param_map, v0, cobs, dt, steps, S_avg, ckpt_every):
        self.lind = lind
        self.param_map = param_map
        self.v0 = v0.to("cuda", torch.float64).contiguous()
        self.cobs = cobs.to("cuda", torch.float64).contiguous()
        self.dt, self.steps, self.S_avg, self.ckpt_every = float(dt), int(steps), int(S_avg), int(ckpt_every)

    def _setup(self, theta):
        """The Adjoint object (kept across calls: its transposed terms and
        reverse layouts do not depend on theta; new static weights only
        rebuild the forward propagator) and the tables for theta."""
        p = self.param_map(np.asarray(theta, dtype=np.float64))
        dyn = list(p["dyn"])
        adj = getattr(self, "_adj", None)
        if adj is None or self._adj_dyn != dyn:
            adj = Adjoint(self.lind, p["static_w"], dyn)
            self._adj, self._adj_dyn = adj, dyn
        else:
            adj.set_weights(p["static_w"])
        coef = torch.as_tensor(np.ascontiguousarray(p["coef"], dtype=np.float64)).cuda() if len(dyn) else None
        dcoef = torch.as_tensor(np.ascontiguousarray(p["dcoef"], dtype=np.float64)).cuda() \
            if len(dyn) and p.get("dcoef") is not None else None
        return adj, coef, p["dstatic"], dcoef

    def value_and_grad(self, theta):
        adj, coef, dstatic, dcoef = self._setup(theta)
        return adj.run(self.v0, coef, dstatic, dcoef, self.cobs, self.dt, self.steps, self.S_avg, self.ckpt_every)

    def value(self, theta):
        adj, coef, _, _ = self._setup(theta)
        return adj.objective(self.v0, coef, self.cobs, self.dt, self.steps, self.S_avg)


class SunBlochLoss(torch.autograd.Function):
    """J(theta) of an AdjointProblem with the adjoint gradient as backward.

        J = SunBlochLoss.apply(theta, problem);  J.backward()
    """

    @classmethod
    def apply(cls, theta, problem):
        # no gradient wanted (theta does not require it, or grad mode is off):
        # the forward objective alone, 2-3x cheaper than the adjoint run
        if not (torch.is_grad_enabled() and theta.requires_grad):
            J = problem.value(theta.detach().cpu().numpy())
            return torch.tensor(J, dtype=theta.dtype, device=theta.device)
        return super().apply(theta, problem)

    @staticmethod
    def forward(ctx, theta, problem):
        th = theta.detach().cpu().numpy()
        J, g = problem.value_and_grad(th)
        ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
        return torch.tensor(J, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout * g, None
