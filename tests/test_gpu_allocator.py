"""Caller allocator (sun_set_allocator): every device allocation of the
library routed through PyTorch's caching allocator gives the same results,
bitwise, as hipMalloc, and PyTorch accounts for the memory while the objects
live and gets it back when they are freed.  Exercised on the plain
propagator (sliced layout, assembly temporaries), the batched form and the
adjoint (whose run allocates its own workspace here)."""

import gc

import numpy as np
import pytest
import torch

from helpers import dimer_adjoint_problem, dimer_batch, flush, fock_bloch
from workloads import dimer

pytestmark = pytest.mark.gpu


def _run_all(lib):
    out = {}
    p = dimer.plain_config(101)
    ops = dimer.dimer_operators(p)
    basis = lib.build_basis(p.N)
    lind, prop = lib.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    v = torch.as_tensor(fock_bloch(p.N, 0)).cuda()
    eps = torch.as_tensor(dimer.drive_table(p, steps=50)).cuda().contiguous()
    prop.propagate(v, eps, p.dt, 50)
    out["plain"] = v.cpu().numpy()
    rng = np.random.default_rng(3)
    inst = []
    for N in (4, 51):
        for _ in range(20):
            q = dimer.plain_config(N)
            q.A = float(rng.uniform(0.5, 3.0))
            inst.append(q)
    bp, groups = dimer_batch(lib, inst, 12)
    for g, (N, idx, _, _, _) in enumerate(groups):
        bp.set_state(g, torch.as_tensor(np.stack([fock_bloch(N, 0)] * len(idx))))
    bp.run(12)
    out["batched"] = [bp.get_state(g).cpu().numpy() for g in range(len(groups))]
    q = dimer.plain_config(51)
    prob, _, _ = dimer_adjoint_problem(lib, q, 120, 40, ckpt_every=32)
    J, grad = prob.value_and_grad(np.array([1.5, 0.1, 0.5]))
    out["adjoint"] = (J, np.asarray(grad))
    torch.cuda.synchronize()
    return out


def _requested() -> int:
    """Bytes requested from PyTorch's caching allocator and not yet freed,
    before its rounding (memory_allocated() counts whole blocks, which
    depend on what the cache already holds)."""
    return torch.cuda.memory_stats()["requested_bytes.all.current"]


def test_torch_allocator_matches_hipmalloc(lib):
    flush("[allocator] hipMalloc run")
    ref = _run_all(lib)
    gc.collect()
    torch.cuda.synchronize()
    base = _requested()
    lib.use_torch_allocator()
    try:
        flush("[allocator] PyTorch caching allocator run")
        p = dimer.plain_config(301)
        ops = dimer.dimer_operators(p)
        basis = lib.build_basis(p.N)
        lind, prop = lib.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
        torch.cuda.synchronize()
        held = _requested() - base
        # the N = 301 terms and propagator layouts (> 40 MB) are now PyTorch's;
        # the objects' own memory queries account for every byte of it but
        # the basis tables (pair indices j and k, P ints each, and N doubles)
        assert held > 40e6, held
        own = lind.device_bytes() + prop.device_bytes()
        assert held == own + 2 * basis.P * 4 + basis.N * 8, (own, held)
        del lind, prop, basis
        gc.collect()
        torch.cuda.synchronize()
        assert _requested() == base
        got = _run_all(lib)
    finally:
        lib.use_default_allocator()
    assert np.array_equal(got["plain"], ref["plain"])
    for a, b in zip(got["batched"], ref["batched"]):
        assert np.array_equal(a, b)
    assert got["adjoint"][0] == ref["adjoint"][0]
    assert np.array_equal(got["adjoint"][1], ref["adjoint"][1])


def test_allocator_arguments_checked(lib):
    from paper_1812_11626_amd import _lib
    L = _lib.load()
    alloc = _lib.ALLOC_FN(lambda n, s, c: None)
    release = _lib.RELEASE_FN(lambda p, c: None)
    assert L.sun_set_allocator(alloc, _lib.RELEASE_FN(), None) == _lib.SUN_EINVAL
    # an allocator that fails: the library reports SUN_ENOMEM, then recovers
    assert L.sun_set_allocator(alloc, release, None) == _lib.SUN_OK
    try:
        with pytest.raises(lib.SunError) as e:
            lib.build_basis(8)
        assert e.value.code == _lib.SUN_ENOMEM
    finally:
        assert L.sun_set_allocator(_lib.ALLOC_FN(), _lib.RELEASE_FN(), None) == _lib.SUN_OK
    assert lib.build_basis(8).M == 63
