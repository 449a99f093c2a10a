"""The allocation-free recording entry point (sun_propagate_record_noalloc)
against sun_propagate_record, through the C ABI: same states and observable
values on two calls in a row, the second on a smaller system, with the
partial-sum array shared between the calls."""

import ctypes as C

import numpy as np
import pytest
import torch

from helpers import flush
from workloads import dimer

pytestmark = pytest.mark.gpu


def _system(sb, N):
    p = dimer.plain_config(N)
    p.steps_per_period = max(p.steps_per_period, dimer.stable_steps_per_period(N, p.E + p.A))
    ops = dimer.dimer_operators(p)
    basis = sb.build_basis(N)
    lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    e0 = np.zeros(N)
    e0[0] = 1.0
    v0 = basis.expand(dimer.ZCSR.from_diagonals(N, {0: e0}))[0].real.contiguous()
    x, x0 = basis.observable(ops["H1"])
    return p, basis, lind, prop, v0, x, x0


def _record(lib, fn, prop, v0, eps, dt, steps, every, x, x0):
    v = v0.clone()
    nrec = steps // every
    st = torch.empty((nrec, prop.M), dtype=torch.float64, device="cuda")
    obs = torch.empty(nrec, dtype=torch.float64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib._lib.check(fn(prop.handle, C.c_void_p(v.data_ptr()), C.c_void_p(eps.data_ptr()), float(dt), int(steps),
                      int(every), C.c_void_p(st.data_ptr()), prop.M, C.c_void_p(x.data_ptr()), float(x0),
                      C.c_void_p(obs.data_ptr()), stream))
    torch.cuda.synchronize()
    return v.cpu().numpy(), st.cpu().numpy(), obs.cpu().numpy()


@pytest.mark.parametrize("sizes", [(1001, 101)])
def test_noalloc_record_matches_record(lib, sizes):
    L = lib._lib.load()
    # the second call is on the smaller system: the array keeps the first
    # call's partials, which must not leak into the second's results
    for N, steps, every in ((sizes[0], 24, 8), (sizes[1], 30, 5)):
        flush(f"[noalloc] N={N} steps={steps} every={every}")
        p, basis, lind, prop, v0, x, x0 = _system(lib, N)
        eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
        ref = _record(lib, L.sun_propagate_record, prop, v0, eps, p.dt, steps, every, x, x0)
        got = _record(lib, L.sun_propagate_record_noalloc, prop, v0, eps, p.dt, steps, every, x, x0)
        for a, b in zip(got, ref):
            assert np.all(np.isfinite(b))
            # same kernels, same fixed-order reductions: bitwise equal (the
            # 1e-12 bar of the propagated states holds a fortiori)
            assert np.array_equal(a, b)
        # both sizes reduce the observable over more than one block, i.e.
        # through the partial-sum array (blocks = ceil(M / 4096))
        assert (N * N - 1 + 4095) // 4096 > 1
