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


def dimer_batch(sb, instances, steps=None):
    """Group dimer instances by N and build a BatchedPropagator over the terms
    [H0, H1, L] with c = (1, E + A_b cos(omega t), gamma_b).  Returns
    (bp, groups) with groups = [(N, [instance indices], lind, dt, steps)]."""
    import numpy as np
    from workloads import dimer
    byN = {}
    for i, p in enumerate(instances):
        byN.setdefault(p.N, []).append(i)
    specs, groups = [], []
    for N in sorted(byN):
        idx = byN[N]
        p0 = instances[idx[0]]
        ops = dimer.dimer_operators(p0)
        basis = sb.build_basis(N)
        lind = sb.Lindbladian(basis, [ops["H0"], ops["H1"]], [ops["L"]])
        st = p0.steps if steps is None else (steps[N] if isinstance(steps, dict) else steps)
        w = np.array([[1.0, instances[i].E, instances[i].gamma_eff] for i in idx])
        u = np.array([[0.0, instances[i].A, 0.0] for i in idx])
        wave = dimer.drive_table_dA(p0, steps=st)
        specs.append(dict(lind=lind, w=w, u=u, wave=wave, dt=p0.dt, steps=st))
        groups.append((N, idx, lind, p0.dt, st))
    return sb.BatchedPropagator(specs), groups


def fock_bloch(N, i=0):
    """Bloch vector of |i><i| (oracle-side construction, tests only)."""
    import numpy as np
    from oracle import lindblad as lb
    rho = np.zeros((N, N), complex)
    rho[i, i] = 1
    return lb.bloch_vector_sparse(rho)


def dimer_adjoint_problem(sb, p, steps, S_avg, ckpt_every):
    """AdjointProblem for the dimer with theta = (A, gamma, U): terms
    [H_J, H_U, H1] and [L], coefficients (-J, U U_scale, E + A cos(omega t),
    gamma gamma_scale).  Returns (problem, lind, basis)."""
    import copy
    import numpy as np
    import torch
    from workloads import dimer
    ops = dimer.dimer_operators(p)
    N = p.N
    basis = sb.build_basis(N)
    lind = sb.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"]], [ops["L"]])
    e0 = np.zeros(N)
    e0[p.rho0_index] = 1.0
    v0 = basis.expand(dimer.ZCSR.from_diagonals(N, {0: e0}))[0].real.contiguous()
    cobs = basis.expand(ops["H1"])[0].real.contiguous()

    def pmap(theta):
        A, g, U = (float(x) for x in theta)
        q = copy.copy(p)
        q.A = A
        coef = dimer.drive_table(q, steps=steps)[:, None]
        dcoef = np.zeros((2 * steps + 1, 1, 3))
        dcoef[:, 0, 0] = dimer.drive_table_dA(q, steps=steps)
        static_w = [-p.J, U * p.U_scale, 0.0, g * p.gamma_scale]
        dstatic = np.zeros((4, 3))
        dstatic[1, 2] = p.U_scale
        dstatic[3, 1] = p.gamma_scale
        return dict(static_w=static_w, dyn=[2], coef=coef, dstatic=dstatic, dcoef=dcoef)

    prob = sb.AdjointProblem(lind, pmap, v0, cobs, p.dt, steps, S_avg, ckpt_every)
    return prob, lind, basis


def bifurcation_batch(sb, instances):
    """One batched group over the terms [H_J, H_U, H1, L] with per-instance
    coefficients (-J, U_eff, E + A cos(omega t), gamma_eff): the U scan of
    workloads.dimer.bifurcation_instances.  Returns (bp, lind, basis)."""
    import numpy as np
    from workloads import dimer
    p0 = instances[0]
    ops = dimer.dimer_operators(p0)
    basis = sb.build_basis(p0.N)
    lind = sb.Lindbladian(basis, [ops["HJ"], ops["HU"], ops["H1"]], [ops["L"]])
    w = np.array([[-q.J, q.U_eff, q.E, q.gamma_eff] for q in instances])
    u = np.array([[0.0, 0.0, q.A, 0.0] for q in instances])
    wave = dimer.drive_table_dA(p0, steps=p0.steps)
    bp = sb.BatchedPropagator([dict(lind=lind, w=w, u=u, wave=wave, dt=p0.dt, steps=p0.steps)])
    return bp, lind, basis
