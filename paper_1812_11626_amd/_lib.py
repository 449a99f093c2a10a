"""ctypes declarations of libsunbloch.so (the C ABI in include/sunbloch.h)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsunbloch.so")

SUN_OK = 0
SUN_EINVAL = -1
SUN_ENOMEM = -2
SUN_EDEVICE = -3
SUN_ENOTSUP = -4
SUN_ERANGE = -5
SUN_EDIVERGED = -6
SUN_EUNSTABLE = -7
SUN_ENOTCONVERGED = -8
SUN_TERM_H = 0
SUN_TERM_L = 1

_STATUS_NAMES = {SUN_EINVAL: "SUN_EINVAL", SUN_ENOMEM: "SUN_ENOMEM", SUN_EDEVICE: "SUN_EDEVICE",
                 SUN_ENOTSUP: "SUN_ENOTSUP", SUN_ERANGE: "SUN_ERANGE", SUN_EDIVERGED: "SUN_EDIVERGED",
                 SUN_EUNSTABLE: "SUN_EUNSTABLE", SUN_ENOTCONVERGED: "SUN_ENOTCONVERGED"}


class SunError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class ZCSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("re", C.c_void_p), ("im", C.c_void_p)]


vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
f64 = C.c_double
P = C.POINTER

# caller allocator (sun_set_allocator): alloc(bytes, stream, ctx) -> ptr, release(ptr, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# name: (restype, argtypes)
PROTOS = {
    "sun_last_error": (C.c_char_p, []),
    "sun_version": (C.c_int, []),
    "sun_set_allocator": (C.c_int, [ALLOC_FN, RELEASE_FN, vp]),
    "sun_build_basis": (C.c_int, [i32, vp, P(vp)]),
    "sun_basis_dims": (C.c_int, [vp, P(i32), P(i64)]),
    "sun_basis_counts": (C.c_int, [vp, vp, P(i64), P(i64)]),
    "sun_basis_export": (C.c_int, [vp, i32, i32, vp, vp, i64, P(i64), vp]),
    "sun_basis_free": (None, [vp]),
    "sun_expand_operator": (C.c_int, [vp, P(ZCSR), vp, vp, P(f64), vp]),
    "sun_expand_lindbladian": (C.c_int, [vp, P(ZCSR), i32, P(ZCSR), i32, vp, P(vp)]),
    "sun_expand_lindbladian_dense": (C.c_int, [vp, P(ZCSR), i32, P(ZCSR), i32, vp, P(vp)]),
    "sun_gemm_f64": (C.c_int, [i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64, vp]),
    "sun_lind_nnz": (C.c_int, [vp, i32, i32, P(i64)]),
    "sun_lind_export": (C.c_int, [vp, i32, i32, vp, vp, vp, vp, vp]),
    "sun_lind_free": (None, [vp]),
    "sun_bloch_density": (C.c_int, [vp, vp, vp, vp, vp]),
    "sun_bloch_expect": (C.c_int, [vp, vp, i64, i64, vp, vp, P(f64), vp, vp, vp]),
    "sun_prop_create": (C.c_int, [vp, P(f64), P(i32), i32, vp, P(vp)]),
    "sun_propagate": (C.c_int, [vp, vp, vp, f64, i64, vp]),
    "sun_propagate_profile": (C.c_int, [vp, vp, vp, f64, i64, vp, P(f64), P(i64)]),
    "sun_propagate_record": (C.c_int, [vp, vp, vp, f64, i64, i64, vp, i64, vp, f64, vp, vp]),
    "sun_propagate_record_noalloc": (C.c_int, [vp, vp, vp, f64, i64, i64, vp, i64, vp, f64, vp, vp]),
    "sun_prop_info": (C.c_int, [vp, P(i64), P(i64), P(i64)]),
    "sun_prop_spectral_radius": (C.c_int, [vp, P(f64), i32, P(f64), vp]),
    "sun_prop_guard_stability": (C.c_int, [vp, P(f64), P(f64), i32, f64, P(f64), vp]),
    "sun_prop_check_finite": (C.c_int, [vp, i32]),
    "sun_stationary": (C.c_int, [vp, P(f64), f64, i64, i32, i32, f64, vp, P(i32), P(f64), vp]),
    "sun_debug_inject_failure": (C.c_int, [i32]),
    "sun_prop_tune": (C.c_int, [vp, i32, i32, i32, vp]),
    "sun_prop_tune_sliced": (C.c_int, [vp, i32, i32, i32, i32, vp]),
    "sun_prop_use_graphs": (C.c_int, [vp, i32]),
    "sun_prop_device_bytes": (C.c_int, [vp, P(C.c_size_t)]),
    "sun_lind_device_bytes": (C.c_int, [vp, P(C.c_size_t)]),
    "sun_batch_device_bytes": (C.c_int, [vp, P(C.c_size_t)]),
    "sun_prop_tune_resident": (C.c_int, [vp, i32]),
    "sun_prop_layout": (C.c_int, [vp, P(i32), P(i64), P(i64), P(i64)]),
    "sun_prop_free": (None, [vp]),
    "sun_batch_create": (C.c_int, [P(vp), i32, P(i32), P(vp), P(vp), P(vp), P(f64), P(i64), vp, P(vp)]),
    "sun_batch_set_state": (C.c_int, [vp, i32, vp, vp]),
    "sun_batch_get_state": (C.c_int, [vp, i32, vp, vp]),
    "sun_batch_run": (C.c_int, [vp, i64, i32, vp]),
    "sun_batch_info": (C.c_int, [vp, i32, P(i64), P(i64), P(i32), P(i32)]),
    "sun_batch_tune": (C.c_int, [vp, i32, i32, i32, i32, vp]),
    "sun_batch_free": (None, [vp]),
    "sun_propagate_batched": (C.c_int, [P(vp), i32, P(i32), P(vp), P(vp), P(vp), P(f64), P(i64), P(vp), vp]),
    "sun_adjoint_create": (C.c_int, [vp, P(f64), P(i32), i32, vp, P(vp)]),
    "sun_adjoint_run": (C.c_int, [vp, vp, vp, P(f64), vp, i32, vp, f64, i64, i64, i64, P(f64), P(f64), vp]),
    "sun_adjoint_objective": (C.c_int, [vp, vp, vp, vp, f64, i64, i64, P(f64), vp]),
    "sun_adjoint_plan": (C.c_int, [vp, P(f64), i32, i64, i64, vp, P(C.c_size_t), P(C.c_size_t)]),
    "sun_adjoint_execute": (C.c_int, [vp, vp, vp, P(f64), vp, i32, vp, f64, i64, i64, i64, vp, C.c_size_t, P(f64),
                                      P(f64), vp]),
    "sun_adjoint_set_weights": (C.c_int, [vp, P(f64), vp]),
    "sun_adjoint_free": (None, [vp]),
}

_lib = None


def load():
    """Load libsunbloch.so from the package directory; raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1812_11626_amd.build` "
                          "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list:
    lib = load()
    return [n for n in PROTOS if getattr(lib, n, None) is not None]


def check(status: int):
    if status != SUN_OK:
        msg = load().sun_last_error()
        raise SunError(status, msg.decode() if msg else "")
