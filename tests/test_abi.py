"""The C-ABI library loads and exports every entry point the header declares
(no compute calls: runs without a GPU)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sunbloch.h")
LIB = os.path.join(ROOT, "paper_1812_11626_amd", "libsunbloch.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sun_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    syms = declared_symbols()
    for name in ("sun_build_basis", "sun_expand_lindbladian", "sun_propagate"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_version_and_error_calls_need_no_gpu():
    lib = ctypes.CDLL(LIB)
    lib.sun_version.restype = ctypes.c_int
    assert lib.sun_version() >= 100
    lib.sun_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.sun_last_error(), bytes)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_checks():
    """Invalid arguments are rejected on the host before any device work."""
    from paper_1812_11626_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.sun_build_basis(1, None, ctypes.byref(h)) == _lib.SUN_EINVAL
    assert b"N must be" in lib.sun_last_error()
    assert lib.sun_build_basis(50000, None, ctypes.byref(h)) == _lib.SUN_EINVAL
    assert lib.sun_build_basis(4, None, None) == _lib.SUN_EINVAL
    assert lib.sun_propagate(None, None, None, 0.1, 1, None) == _lib.SUN_EINVAL
    assert lib.sun_prop_tune(None, 2048, 256, 1, None) == _lib.SUN_EINVAL
    assert lib.sun_propagate_record(None, None, None, 0.1, 1, 1, None, 0, None, 0.0, None, None) == _lib.SUN_EINVAL
    assert lib.sun_bloch_density(None, None, None, None, None) == _lib.SUN_EINVAL
    r = ctypes.c_double()
    assert lib.sun_prop_spectral_radius(None, None, 100, ctypes.byref(r), None) == _lib.SUN_EINVAL
    assert lib.sun_bloch_expect(None, None, 1, 0, None, None, None, None, None, None) == _lib.SUN_EINVAL
    n = ctypes.c_int64()
    assert lib.sun_lind_nnz(None, 0, 0, ctypes.byref(n)) == _lib.SUN_EINVAL
    assert lib.sun_propagate_record_noalloc(None, None, None, 0.1, 1, 1, None, 0, None, 0.0, None,
                                            None) == _lib.SUN_EINVAL
    assert lib.sun_prop_guard_stability(None, None, None, 100, 0.0, None, None) == _lib.SUN_EINVAL
    assert lib.sun_prop_check_finite(None, 1) == _lib.SUN_EINVAL
    assert lib.sun_debug_inject_failure(7) == _lib.SUN_EINVAL
    assert lib.sun_debug_inject_failure(0) == _lib.SUN_OK
    sz = ctypes.c_size_t()
    assert lib.sun_adjoint_plan(None, None, 0, 10, 5, None, ctypes.byref(sz), None) == _lib.SUN_EINVAL
    J = ctypes.c_double()
    assert lib.sun_adjoint_execute(None, None, None, None, None, 0, None, 0.1, 10, 5, 5, None, 0, ctypes.byref(J),
                                   None, None) == _lib.SUN_EINVAL
    assert lib.sun_adjoint_set_weights(None, None, None) == _lib.SUN_EINVAL
    assert lib.sun_propagate_batched(None, 1, None, None, None, None, None, None, None, None) == _lib.SUN_EINVAL
    it, rr = ctypes.c_int32(), ctypes.c_double()
    assert lib.sun_stationary(None, None, 0.1, 10, 30, 100, 1e-10, None, ctypes.byref(it), ctypes.byref(rr),
                              None) == _lib.SUN_EINVAL


def test_status_codes_match_header():
    """The binding's status constants are the header's."""
    from paper_1812_11626_amd import _lib
    text = open(HEADER).read()
    for name in ("SUN_EINVAL", "SUN_ENOMEM", "SUN_EDEVICE", "SUN_ENOTSUP", "SUN_ERANGE", "SUN_EDIVERGED",
                 "SUN_EUNSTABLE", "SUN_ENOTCONVERGED"):
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert m is not None, name
        assert int(m.group(1)) == getattr(_lib, name), name


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_plain_c99(tmp_path):
    """The boundary header compiles as strict C99 (no C++ or HIP types)."""
    src = tmp_path / "use.c"
    src.write_text('#include "sunbloch.h"\nint main(void) { return sun_last_error() == 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_allocator_hook_arguments_need_no_gpu():
    """sun_set_allocator checks its arguments on the host: one function of
    the pair alone is SUN_EINVAL; both NULL (hipMalloc/hipFree) is accepted."""
    from paper_1812_11626_amd import _lib
    L = _lib.load()
    alloc = _lib.ALLOC_FN(lambda n, s, c: None)
    release = _lib.RELEASE_FN(lambda p, c: None)
    assert L.sun_set_allocator(alloc, _lib.RELEASE_FN(), None) == _lib.SUN_EINVAL
    assert L.sun_set_allocator(_lib.ALLOC_FN(), release, None) == _lib.SUN_EINVAL
    assert L.sun_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == _lib.SUN_OK
