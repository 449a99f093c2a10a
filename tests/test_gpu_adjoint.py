"""Adjoint form: gradient of the period-averaged <n1 - n2> with respect to
(A, gamma, U) by the hand-written adjoint RK4 kernels.

Checks: against the oracle's dense discrete adjoint at N = 6 (J to 1e-12,
gradient to 1e-7 relative), against central finite differences (h = 1e-6)
of the GPU objective at N = 6 and N = 51, at the benchmark's sizes N = 301
and N = 1001 against stored oracle values (J and the gradient, from the
density-matrix tangent route), invariance under the checkpoint interval,
and the torch.autograd.Function wrapper.
"""

import numpy as np
import pytest
import torch

from helpers import dimer_adjoint_problem, flush
from oracle import adjoint as oadj, basis as ob, lindblad as lb
from workloads import dimer

pytestmark = pytest.mark.gpu

THETA = np.array([1.5, 0.1, 0.5])


def _oracle(p, steps, S):
    ops = dimer.dimer_operators(p)
    F = ob.generators(p.N)
    Gs = [lb.q_hamiltonian(F, ops[k].to_dense()) for k in ("HJ", "HU", "H1")]
    Gs.append(lb.q_dissipator(F, ops["L"].to_dense()))
    Ks = [None, None, None, lb.k_dissipator(F, ops["L"].to_dense())]
    coef = np.zeros((2 * steps + 1, 4))
    coef[:, 0] = -p.J
    coef[:, 1] = p.U_eff
    coef[:, 2] = dimer.drive_table(p, steps=steps)
    coef[:, 3] = p.gamma_eff
    dcoef = np.zeros((2 * steps + 1, 4, 3))
    dcoef[:, 2, 0] = dimer.drive_table_dA(p, steps=steps)
    dcoef[:, 3, 1] = p.gamma_scale
    dcoef[:, 1, 2] = p.U_scale
    rho0 = np.zeros((p.N, p.N), complex)
    rho0[0, 0] = 1
    v0 = lb.bloch_vector(F, rho0)
    c = lb.bloch_vector(F, ops["H1"].to_dense())
    return oadj.adjoint_gradient(Gs, Ks, coef, dcoef, v0, c, p.dt, steps, S)


def test_dense_adjoint_N6(lib):
    flush("[adjoint] N=6 vs dense oracle adjoint")
    p = dimer.adjoint_config(6)
    steps, S = 2 * p.steps_per_period, p.steps_per_period
    J_o, g_o = _oracle(p, steps, S)
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=p.steps_per_period)
    J, g = prob.value_and_grad(THETA)
    assert abs(J - J_o) <= 1e-12 * abs(J_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-7)
    assert abs(prob.value(THETA) - J_o) <= 1e-12 * abs(J_o)


@pytest.mark.parametrize("N", [6, 51])
def test_central_differences(lib, N):
    flush(f"[adjoint] N={N} vs central differences")
    p = dimer.adjoint_config(N) if N <= 6 else dimer.plain_config(N)
    steps = 2 * p.steps_per_period if N <= 6 else p.steps_per_period
    S = p.steps_per_period if N <= 6 else p.steps_per_period // 2
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=max(1, steps // 4))
    theta = THETA.copy()
    J, g = prob.value_and_grad(theta)
    h = 1e-6
    for i in range(3):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (prob.value(tp) - prob.value(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-11, (i, fd, g[i])


def _golden(name):
    """(N, steps, S, J, grad) stored by tests/golden/make_adjoint_goldens.py
    (oracle density-matrix tangent route)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_goldens.txt")
    for line in open(path):
        f = line.split()
        if f and f[0] == name:
            return int(f[1]), int(f[2]), int(f[3]), float(f[4]), np.array([float(x) for x in f[5:8]])
    raise KeyError(name)


def test_N301_benchmark_configuration(lib):
    """N = 301 (M = 90,600) with a checkpoint every S steps as the benchmark
    runs it, over 256 steps: J (1e-12) and dJ/d(A, gamma, U) (1e-7) against
    the stored oracle values (density-matrix tangent route, no SU(N) basis),
    and the gradient against central differences of the GPU objective."""
    N, steps, S, J_o, g_o = _golden("adjoint-N301")
    flush(f"[adjoint] N={N} benchmark configuration")
    p = dimer.adjoint_config(N)
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=S)
    J, g = prob.value_and_grad(THETA.copy())
    assert abs(J - J_o) <= 1e-12 * abs(J_o), (J, J_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-7)
    h = 1e-6
    for i in range(3):
        tp, tm = THETA.copy(), THETA.copy()
        tp[i] += h
        tm[i] -= h
        fd = (prob.value(tp) - prob.value(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-11, (i, fd, g[i])


def test_N301_ten_periods_central_differences(lib):
    """The adjoint workload at N = 301 over 10 of its 100 periods (40,960
    steps, a checkpoint every period as the benchmark runs it, so the
    backward sweep recomputes 9 intervals from their checkpoints), J over the
    last period: dJ/d(A, gamma, U) against central differences of the GPU's
    own forward objective to 1e-7 (a property of the exact discrete gradient
    at any horizon; the oracle's gradient is pinned at 256 steps above)."""
    flush("[adjoint] N=301 ten periods vs central differences")
    p = dimer.adjoint_config(301)
    S = p.steps_per_period
    steps = 10 * S
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=S)
    J, g = prob.value_and_grad(THETA.copy())
    assert np.isfinite(J) and np.all(np.isfinite(g))
    assert abs(J - prob.value(THETA.copy())) <= 1e-12 * abs(J)
    h = 1e-6
    for i in range(3):
        tp, tm = THETA.copy(), THETA.copy()
        tp[i] += h
        tm[i] -= h
        fd = (prob.value(tp) - prob.value(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * abs(g[i]) + 1e-11, (i, fd, g[i])


def test_N1001_plain_workload_gradient(lib):
    """The plain N = 1001 workload (M = 1,002,000) on the adjoint path the
    benchmark times there (fused reverse stages, several checkpoint intervals
    recomputed, stage inputs kept): from the Fock state, J over the last half
    of the stored run, four checkpoint intervals; J (1e-12) and the gradient
    (1e-7) against the stored oracle values."""
    N, steps, S, J_o, g_o = _golden("plain-N1001")
    flush(f"[adjoint] N={N} plain workload, {steps} steps")
    p = dimer.plain_config(N)
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=steps // 4)
    J, g = prob.value_and_grad(THETA.copy())
    assert abs(J - J_o) <= 1e-12 * abs(J_o), (J, J_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-7)


def test_checkpoint_interval_invariance(lib):
    p = dimer.adjoint_config(6)
    steps, S = 150, 40
    res = []
    for ck in (1, 7, 64, 150):
        prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=ck)
        res.append(prob.value_and_grad(THETA))
    for J, g in res[1:]:
        assert J == res[0][0]
        assert np.array_equal(g, res[0][1])


def test_autograd_function(lib):
    p = dimer.adjoint_config(6)
    steps, S = 100, 50
    prob, _, _ = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=25)
    theta = torch.tensor(THETA, dtype=torch.float64, requires_grad=True)
    J = lib.SunBlochLoss.apply(theta, prob)
    (2.0 * J).backward()
    J2, g = prob.value_and_grad(THETA)
    assert float(J.detach()) == J2
    np.testing.assert_array_equal(theta.grad.numpy(), 2.0 * g)


def test_four_dependent_terms_against_dense_adjoint(lib):
    """theta = (A, gamma, U, J): all four terms depend on a parameter, more
    than the fused reverse stages take, so the per-term dot-product path
    runs.  Against the oracle's dense adjoint at N = 6, and its (A, gamma, U)
    components against the fused path of the three-parameter problem."""
    import copy
    flush("[adjoint] N=6 four parameter-dependent terms")
    p = dimer.adjoint_config(6)
    steps, S = 2 * p.steps_per_period, p.steps_per_period
    prob3, lind, basis = dimer_adjoint_problem(lib, p, steps, S, ckpt_every=p.steps_per_period)

    def pmap4(theta):
        A, g, U, Jh = (float(x) for x in theta)
        q = copy.copy(p)
        q.A = A
        coef = dimer.drive_table(q, steps=steps)[:, None]
        dcoef = np.zeros((2 * steps + 1, 1, 4))
        dcoef[:, 0, 0] = dimer.drive_table_dA(q, steps=steps)
        static_w = [-Jh, U * p.U_scale, 0.0, g * p.gamma_scale]
        dstatic = np.zeros((4, 4))
        dstatic[0, 3] = -1.0
        dstatic[1, 2] = p.U_scale
        dstatic[3, 1] = p.gamma_scale
        return dict(static_w=static_w, dyn=[2], coef=coef, dstatic=dstatic, dcoef=dcoef)

    prob4 = lib.AdjointProblem(lind, pmap4, prob3.v0, prob3.cobs, p.dt, steps, S, p.steps_per_period)
    theta4 = np.array([1.5, 0.1, 0.5, p.J])
    J4, g4 = prob4.value_and_grad(theta4)
    J3, g3 = prob3.value_and_grad(THETA)
    # oracle: the dense adjoint with the J derivative added
    ops = dimer.dimer_operators(p)
    F = ob.generators(p.N)
    Gs = [lb.q_hamiltonian(F, ops[k].to_dense()) for k in ("HJ", "HU", "H1")]
    Gs.append(lb.q_dissipator(F, ops["L"].to_dense()))
    Ks = [None, None, None, lb.k_dissipator(F, ops["L"].to_dense())]
    coef = np.zeros((2 * steps + 1, 4))
    coef[:, 0] = -p.J
    coef[:, 1] = p.U_eff
    coef[:, 2] = dimer.drive_table(p, steps=steps)
    coef[:, 3] = p.gamma_eff
    dcoef = np.zeros((2 * steps + 1, 4, 4))
    dcoef[:, 2, 0] = dimer.drive_table_dA(p, steps=steps)
    dcoef[:, 3, 1] = p.gamma_scale
    dcoef[:, 1, 2] = p.U_scale
    dcoef[:, 0, 3] = -1.0
    rho0 = np.zeros((p.N, p.N), complex)
    rho0[0, 0] = 1
    J_o, g_o = oadj.adjoint_gradient(Gs, Ks, coef, dcoef, lb.bloch_vector(F, rho0),
                                     lb.bloch_vector(F, ops["H1"].to_dense()), p.dt, steps, S)
    assert abs(J4 - J_o) <= 1e-12 * abs(J_o)
    np.testing.assert_allclose(g4, g_o, rtol=1e-7)
    assert J4 == J3
    np.testing.assert_allclose(g4[:3], g3, rtol=1e-11)


@pytest.mark.parametrize("params", ["gamma,U", "gamma"])
def test_static_generator_adjoint_against_dense(lib, params):
    """No time-dependent term (the drive frozen at eps = E + A, folded into a
    static weight): theta = (gamma, U) or (gamma) alone, i.e. two or one
    segments on the fused reverse stages, against the oracle's dense adjoint
    at N = 5 over three checkpoint intervals."""
    flush(f"[adjoint] N=5 static generator, theta = ({params})")
    p = dimer.adjoint_config(5)
    steps, S = 120, 40
    ops = dimer.dimer_operators(p)
    basis = lib.build_basis(p.N)
    lind = lib.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"]], [ops["L"]])
    e0 = np.zeros(p.N)
    e0[0] = 1.0
    v0 = basis.expand(dimer.ZCSR.from_diagonals(p.N, {0: e0}))[0].real.contiguous()
    cobs = basis.expand(ops["H1"])[0].real.contiguous()
    eps0 = p.E + p.A
    with_u = params == "gamma,U"
    nth = 2 if with_u else 1

    def pmap(theta):
        g = float(theta[0])
        U = float(theta[1]) if with_u else p.U
        dstatic = np.zeros((4, nth))
        dstatic[3, 0] = p.gamma_scale
        if with_u:
            dstatic[1, 1] = p.U_scale
        return dict(static_w=[-p.J, U * p.U_scale, eps0, g * p.gamma_scale], dyn=[], coef=None,
                    dstatic=dstatic, dcoef=None)

    prob = lib.AdjointProblem(lind, pmap, v0, cobs, p.dt, steps, S, 50)
    J, g = prob.value_and_grad(np.array([p.gamma, p.U][:nth]))
    F = ob.generators(p.N)
    Gs = [lb.q_hamiltonian(F, ops[k].to_dense()) for k in ("HJ", "HU", "H1")]
    Gs.append(lb.q_dissipator(F, ops["L"].to_dense()))
    Ks = [None, None, None, lb.k_dissipator(F, ops["L"].to_dense())]
    coef = np.tile(np.array([-p.J, p.U_eff, eps0, p.gamma_eff]), (2 * steps + 1, 1))
    dcoef = np.zeros((2 * steps + 1, 4, nth))
    dcoef[:, 3, 0] = p.gamma_scale
    if with_u:
        dcoef[:, 1, 1] = p.U_scale
    rho0 = np.zeros((p.N, p.N), complex)
    rho0[0, 0] = 1
    J_o, g_o = oadj.adjoint_gradient(Gs, Ks, coef, dcoef, lb.bloch_vector(F, rho0),
                                     lb.bloch_vector(F, ops["H1"].to_dense()), p.dt, steps, S)
    assert abs(J - J_o) <= 1e-12 * abs(J_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-7)
