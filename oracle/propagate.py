"""Time propagation of the Bloch ODE and of the density matrix (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The paper integrates eq. (9), dv/dt = (Q(t) + R) v + K, with the classical
fourth-order Runge-Kutta method (Sec. IV, step 3.1).  Reading taken for the
time dependence: the generator is

    G(t) = G0 + sum_a c_a(t) G_a

and the coefficients c_a are sampled on the half-step grid t0 + k dt/2
(k = 0..2*steps) into a table ``coef`` of shape (2*steps+1, nterms) that the
caller provides; stage times of step n are t_n, t_n + dt/2, t_n + dt/2,
t_n + dt, i.e. rows 2n, 2n+1, 2n+1, 2n+2.

* ``rk4_bloch``  -- classical RK4 on eq. (9) with dense or scipy-sparse
                    matrices.
* ``rk4_rho``    -- the same RK4 applied to eq. (1) on the N x N density
                    matrix.  RK4 commutes with the affine map rho <-> v
                    (eq. 5), so in exact arithmetic both give the same
                    trajectory; this form never touches the SU(N) basis.
* ``expm_affine``-- exact propagator of a time-independent affine ODE by the
                    matrix exponential of the augmented generator.

Parity: pinned -- one RK4 step equals the degree-4 Taylor polynomial of the
augmented generator, fourth-order convergence to ``expm_affine``, and
``rk4_rho`` == ``rk4_bloch`` (tests/test_oracle_propagate.py).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _coef_rows(coef: np.ndarray, n: int):
    return coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]


def rk4_bloch(G0, Gs, K, v0, coef, dt: float, steps: int,
              record_every: int = 0, Ks=None):
    """Classical RK4 for dv/dt = (G0 + sum_a c_a(t) G_a) v + K(t), with
    K(t) = K + sum_a c_a(t) Ks[a].

    G0, Gs[a]: dense arrays or scipy sparse matrices (M, M); K (M,) or None;
    coef: (2*steps+1, len(Gs)); Ks: None, or one free vector (M,) or None per
    time-dependent term (a dissipation channel whose rate varies carries its
    eq. 11 vector with its eq. 10 matrix).  Returns v at the end, and if
    record_every > 0 also the list of states after every record_every steps.
    """
    coef = np.asarray(coef, dtype=np.float64).reshape(2 * steps + 1, -1) \
        if len(Gs) else np.zeros((2 * steps + 1, 0))
    v = np.array(v0, dtype=np.float64, copy=True)
    Kv = np.zeros_like(v) if K is None else np.asarray(K, dtype=np.float64)
    Ka = [None] * len(Gs) if Ks is None else [None if k is None else np.asarray(k, dtype=np.float64) for k in Ks]
    rec = []

    def rhs(x, c):
        y = G0 @ x + Kv
        for a, Ga in enumerate(Gs):
            y = y + c[a] * (Ga @ x)
            if Ka[a] is not None:
                y = y + c[a] * Ka[a]
        return y

    for n in range(steps):
        c0, ch, c1 = _coef_rows(coef, n)
        k1 = rhs(v, c0)
        k2 = rhs(v + 0.5 * dt * k1, ch)
        k3 = rhs(v + 0.5 * dt * k2, ch)
        k4 = rhs(v + dt * k3, c1)
        v = v + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if record_every and (n + 1) % record_every == 0:
            rec.append(v.copy())
    if record_every:
        return v, rec
    return v


def _sp(op):
    if sp.issparse(op):
        return op.tocsr().astype(np.complex128)
    if hasattr(op, "indptr") and hasattr(op, "re"):
        return sp.csr_matrix((op.re + 1j * op.im, op.indices, op.indptr),
                             shape=(op.n, op.n))
    return sp.csr_matrix(np.asarray(op, dtype=np.complex128))


def rk4_rho(H0, Hs, Ls, gammas, rho0, coef, dt: float, steps: int,
            record_every: int = 0, rates=None):
    """Classical RK4 on drho/dt = -i[H(t), rho] + sum_p g_p D_p(rho) (eq. 1).

    H(t) = H0 + sum_a c_a(t) Hs[a].  Operators may be dense, scipy sparse or
    workloads.ZCSR; rho is a dense complex N x N array.  rates: None (the
    constant g_p = gammas[p]) or a (2*steps+1, P) table of g_p on the same
    half-step grid as coef.
    """
    H0 = _sp(H0)
    Hs = [_sp(h) for h in Hs]
    Ls = [_sp(L) for L in Ls]
    Lds = [L.conj().T.tocsr() for L in Ls]
    LdLs = [(Ld @ L).tocsr() for L, Ld in zip(Ls, Lds)]
    coef = np.asarray(coef, dtype=np.float64).reshape(2 * steps + 1, -1) \
        if len(Hs) else np.zeros((2 * steps + 1, 0))
    rho = np.array(rho0, dtype=np.complex128, copy=True)
    rtab = np.tile(np.asarray(gammas, dtype=np.float64), (2 * steps + 1, 1)) if rates is None \
        else np.asarray(rates, dtype=np.float64).reshape(2 * steps + 1, len(Ls))
    rec = []

    def rhs(r, c, gs):
        H = H0
        for a, Ha in enumerate(Hs):
            H = H + c[a] * Ha
        out = -1j * (H @ r - (H.T @ r.T).T)          # r @ H
        for g, L, Ld, LdL in zip(gs, Ls, Lds, LdLs):
            rLd = (Ld.T @ r.T).T                       # r @ Ld
            out = out + g * (L @ rLd - 0.5 * (LdL @ r + (LdL.T @ r.T).T))
        return out

    for n in range(steps):
        c0, ch, c1 = _coef_rows(coef, n)
        g0, gh, g1 = _coef_rows(rtab, n)
        k1 = rhs(rho, c0, g0)
        k2 = rhs(rho + 0.5 * dt * k1, ch, gh)
        k3 = rhs(rho + 0.5 * dt * k2, ch, gh)
        k4 = rhs(rho + dt * k3, c1, g1)
        rho = rho + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if record_every and (n + 1) % record_every == 0:
            rec.append(rho.copy())
    if record_every:
        return rho, rec
    return rho


def augmented(G: np.ndarray, K: np.ndarray) -> np.ndarray:
    """[[G, K], [0, 0]]: the affine ODE dv/dt = G v + K as a linear one on
    (v, 1)."""
    M = G.shape[0]
    A = np.zeros((M + 1, M + 1))
    A[:M, :M] = G
    A[:M, M] = K
    return A


def expm_affine(G: np.ndarray, K: np.ndarray, v0: np.ndarray, t: float):
    """v(t) = first M entries of expm(t [[G, K], [0, 0]]) (v0, 1)."""
    A = augmented(np.asarray(G, dtype=np.float64), np.asarray(K, dtype=np.float64))
    x = np.concatenate([v0, [1.0]])
    return (sla.expm(t * A) @ x)[:-1]
