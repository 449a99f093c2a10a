"""Boundary behaviour through the C ABI: the run-time checks (SUN_EDIVERGED
for a non-finite state, SUN_EUNSTABLE for a step beyond RK4's stability
bound), a re-layout that fails part-way (the propagator refuses to launch
until a layout is selected again), the adjoint's plan -> caller workspace ->
execute form, cached adjoint objects across parameter values, and the
single-call batched form.  Every failure is forced from the host (NaN inputs,
an oversized dt, an injected allocation failure); the kernels run normally."""

import ctypes as C

import numpy as np
import pytest
import torch

from helpers import dimer_adjoint_problem, dimer_batch, flush
from workloads import dimer

pytestmark = pytest.mark.gpu


def _plain(sb, N):
    p = dimer.plain_config(N)
    p.steps_per_period = max(p.steps_per_period, dimer.stable_steps_per_period(N, p.E + p.A))
    ops = dimer.dimer_operators(p)
    basis = sb.build_basis(N)
    lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    e0 = np.zeros(N)
    e0[0] = 1.0
    v0 = basis.expand(dimer.ZCSR.from_diagonals(N, {0: e0}))[0].real.contiguous()
    return p, basis, lind, prop, v0


def _code(exc):
    return exc.value.code


@pytest.mark.parametrize("N", [4, 51, 101])
def test_nan_state_is_reported(lib, N):
    """NaN in v0 (resident path at N = 4, sliced at 51 and 101):
    SUN_EDIVERGED, from sun_propagate and from sun_propagate_record."""
    flush(f"[boundary] NaN state N={N}")
    p, basis, lind, prop, v0 = _plain(lib, N)
    steps = 20
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    v = v0.clone()
    prop.propagate(v, eps, p.dt, steps)                      # finite: fine
    bad = v0.clone()
    bad[N // 2] = float("nan")
    with pytest.raises(lib.SunError) as e:
        prop.propagate(bad, eps, p.dt, steps)
    assert _code(e) == lib._lib.SUN_EDIVERGED
    with pytest.raises(lib.SunError) as e:
        prop.record(v0.clone().fill_(float("inf")), eps, p.dt, steps, 5)
    assert _code(e) == lib._lib.SUN_EDIVERGED
    # the flag is reset: the next finite run succeeds
    v = v0.clone()
    prop.propagate(v, eps, p.dt, steps)
    assert torch.isfinite(v).all()
    # with the check off the call returns the non-finite state without error
    prop.check_finite(False)
    bad = v0.clone()
    bad[0] = float("nan")
    prop.propagate(bad, eps, p.dt, steps)
    torch.cuda.synchronize()
    assert not torch.isfinite(bad).all()


def test_nan_in_drive_table_is_reported(lib):
    flush("[boundary] NaN drive table N=101")
    p, basis, lind, prop, v0 = _plain(lib, 101)
    steps = 10
    eps = dimer.drive_table(p, steps=steps)
    eps[7] = np.nan
    with pytest.raises(lib.SunError) as e:
        lib.propagate(prop, v0, eps, p.dt, steps)
    assert _code(e) == lib._lib.SUN_EDIVERGED


@pytest.mark.parametrize("N", [51, 301])
def test_stability_guard(lib, N):
    """The configured step passes the guard; a step 1.5x beyond the bound
    is refused before any launch (the state is left untouched)."""
    flush(f"[boundary] stability guard N={N}")
    p, basis, lind, prop, v0 = _plain(lib, N)
    rho = prop.guard_stability([p.E - p.A], [p.E + p.A])
    assert rho * p.dt <= 2.6
    steps = 4
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    v = v0.clone()
    prop.propagate(v, eps, p.dt, steps)
    dt_bad = 1.5 * 2.6 / rho
    v = v0.clone()
    with pytest.raises(lib.SunError) as e:
        prop.propagate(v, eps, dt_bad, steps)
    assert _code(e) == lib._lib.SUN_EUNSTABLE
    assert torch.equal(v, v0)
    with pytest.raises(lib.SunError) as e:
        prop.record(v, eps, dt_bad, steps, 2)
    assert _code(e) == lib._lib.SUN_EUNSTABLE
    # the top-level helper guards by itself
    with pytest.raises(lib.SunError) as e:
        lib.propagate(prop, v0, dimer.drive_table(p, steps=steps), dt_bad, steps)
    assert _code(e) == lib._lib.SUN_EUNSTABLE
    prop.guard_stability([p.E - p.A], [p.E + p.A], limit=-1.0)    # off
    v = v0.clone()
    prop.propagate(v, eps, p.dt, steps)


def test_failed_relayout_leaves_propagator_refusing(lib):
    """An allocation failure injected in the middle of a re-layout: the call
    reports it, every launching call then refuses (no kernel reads the
    half-built layout), and selecting a layout again restores bitwise the
    same results."""
    flush("[boundary] injected re-layout failure N=101")
    L = lib._lib.load()
    p, basis, lind, prop, v0 = _plain(lib, 101)
    steps = 8
    eps = torch.as_tensor(dimer.drive_table(p, steps=steps)).cuda().contiguous()
    ref = v0.clone()
    prop.propagate(ref, eps, p.dt, steps)
    for retune in (lambda: prop.tune_sliced(), lambda: prop.tune(block_nnz=1024)):
        lib._lib.check(L.sun_debug_inject_failure(1))
        with pytest.raises(lib.SunError) as e:
            retune()
        assert _code(e) == lib._lib.SUN_ENOMEM
        v = v0.clone()
        with pytest.raises(lib.SunError) as e:
            prop.propagate(v, eps, p.dt, steps)
        assert _code(e) == lib._lib.SUN_EINVAL
        with pytest.raises(lib.SunError):
            prop.record(v, eps, p.dt, steps, 4)
        with pytest.raises(lib.SunError):
            prop.spectral_radius([p.E], iters=10)
        assert torch.equal(v, v0)
    prop.tune_sliced()
    v = v0.clone()
    prop.propagate(v, eps, p.dt, steps)
    assert torch.equal(v, ref)
    lib._lib.check(L.sun_debug_inject_failure(0))


def test_failed_batch_retiling_refuses_group(lib):
    """An allocation failure injected in the middle of a batch group's
    re-tiling (to path 7): the call reports it, sun_batch_run then refuses
    to advance the group (no kernel reads its half-built layout), and tuning
    it again restores bitwise the same results."""
    flush("[boundary] injected batch re-tiling failure N=51")
    from helpers import dimer_batch, fock_bloch
    L = lib._lib.load()
    inst = [p for p in dimer.batched_instances() if p.N == 51][:10]
    steps = 8
    bp, groups = dimer_batch(lib, inst, steps)
    start = torch.as_tensor(np.stack([fock_bloch(51, 0)] * len(inst)))
    bp.tune(0, 64, 32, 7)
    bp.set_state(0, start)
    bp.run(steps)
    ref = bp.get_state(0)
    lib._lib.check(L.sun_debug_inject_failure(1))
    with pytest.raises(lib.SunError) as e:
        bp.tune(0, 64, 16, 7)
    assert _code(e) == lib._lib.SUN_ENOMEM
    bp.set_state(0, start)
    with pytest.raises(lib.SunError) as e:
        bp.run(steps)
    assert _code(e) == lib._lib.SUN_EINVAL
    assert torch.equal(bp.get_state(0), start.cuda())
    bp.tune(0, 64, 32, 7)
    bp.set_state(0, start)
    bp.run(steps)
    assert torch.equal(bp.get_state(0), ref)
    lib._lib.check(L.sun_debug_inject_failure(0))


def test_adjoint_plan_execute_workspace(lib):
    """sun_adjoint_execute on a PyTorch workspace sized by sun_adjoint_plan
    equals sun_adjoint_run bitwise, with the stage inputs kept (full
    workspace) and recomputed (minimum workspace); a smaller workspace is
    refused with SUN_ERANGE."""
    flush("[boundary] adjoint plan/execute N=51")
    p = dimer.plain_config(51)
    steps, S = 300, 100
    prob, lind, basis = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=64)
    theta = np.array([1.5, 0.1, 0.5])
    adj, coef, dstatic, dcoef = prob._setup(theta)
    L = lib._lib.load()
    ds = np.ascontiguousarray(np.asarray(dstatic, dtype=np.float64))
    J = C.c_double()
    g = (C.c_double * 3)()
    lib._lib.check(L.sun_adjoint_run(adj.handle, C.c_void_p(prob.v0.data_ptr()), C.c_void_p(coef.data_ptr()),
                                     ds.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(dcoef.data_ptr()), 3,
                                     C.c_void_p(prob.cobs.data_ptr()), p.dt, steps, S, 64, C.byref(J), g,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    ref = (J.value, np.array(g[:3]))
    full, low = adj.plan(ds, steps, 64)
    assert low < full
    for size in (full, low):
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        got = adj.run(prob.v0, coef, ds, dcoef, prob.cobs, p.dt, steps, S, 64, workspace=ws)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1])
    ws = torch.empty(low - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.SunError) as e:
        adj.run(prob.v0, coef, ds, dcoef, prob.cobs, p.dt, steps, S, 64, workspace=ws)
    assert _code(e) == lib._lib.SUN_ERANGE


def test_adjoint_problem_reuses_object_across_theta(lib):
    """AdjointProblem keeps one adjoint object and only refreshes its static
    weights: results equal those of a fresh problem bitwise, for a sequence
    of parameter values."""
    flush("[boundary] adjoint object reuse N=21")
    p = dimer.plain_config(21)
    steps, S = 200, 50
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=50)
    for theta in ([1.5, 0.1, 0.5], [1.2, 0.3, 0.9], [1.5, 0.1, 0.5]):
        got = prob.value_and_grad(np.array(theta))
        fresh, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=50)
        want = fresh.value_and_grad(np.array(theta))
        assert got[0] == want[0]
        assert np.array_equal(got[1], want[1])
        assert prob.value(np.array(theta)) == fresh.value(np.array(theta))
    # no gradient wanted: the objective alone
    th = torch.tensor([1.5, 0.1, 0.5], dtype=torch.float64)
    assert float(lib.SunBlochLoss.apply(th, prob)) == prob.value(th.numpy())


def test_single_call_batched_matches_object(lib):
    """sun_propagate_batched (create, load, run, read back, free in one call)
    equals the batched object's run bitwise."""
    flush("[boundary] single-call batched")
    inst = dimer.batched_instances(count=24, sizes=(21, 31), periods=1)
    steps = {21: 60, 31: 40}
    bp, groups = dimer_batch(lib, inst, steps=steps)
    V0 = []
    for gi, (N, idx, lind, dt, st) in enumerate(groups):
        e0 = np.zeros(N)
        e0[0] = 1.0
        v0 = bp.groups[gi]["lind"].basis.expand(dimer.ZCSR.from_diagonals(N, {0: e0}))[0].real
        V = v0.repeat(len(idx), 1).contiguous()
        V0.append(V)
        bp.set_state(gi, V)
    bp.run(max(steps.values()))
    want = [bp.get_state(g).cpu().numpy() for g in range(len(groups))]
    L = lib._lib.load()
    n = len(bp.groups)
    Vs = [v.clone() for v in V0]
    linds = (C.c_void_p * n)(*[g["lind"].handle.value for g in bp.groups])
    B = (C.c_int32 * n)(*[g["B"] for g in bp.groups])
    wp = (C.c_void_p * n)(*[g["w"].data_ptr() for g in bp.groups])
    up = (C.c_void_p * n)(*[g["u"].data_ptr() for g in bp.groups])
    wv = (C.c_void_p * n)(*[g["wave"].data_ptr() for g in bp.groups])
    dt = (C.c_double * n)(*[g["dt"] for g in bp.groups])
    st = (C.c_int64 * n)(*[g["steps"] for g in bp.groups])
    vp = (C.c_void_p * n)(*[v.data_ptr() for v in Vs])
    lib._lib.check(L.sun_propagate_batched(linds, n, B, wp, up, wv, dt, st, vp,
                                           C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    for g in range(n):
        assert np.array_equal(Vs[g].cpu().numpy(), want[g])
    # a NaN state: SUN_EDIVERGED from the batched run
    Vs[0][0, 0] = float("nan")
    vp = (C.c_void_p * n)(*[v.data_ptr() for v in Vs])
    st_code = L.sun_propagate_batched(linds, n, B, wp, up, wv, dt, st, vp,
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st_code == lib._lib.SUN_EDIVERGED
