"""Gradient of a time-averaged observable through the RK4 map (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Setting.  The generator is a linear combination of fixed terms,

    G(t) = sum_a c_a(t) G_a,        K(t) = sum_a c_a(t) K_a,

with coefficients tabulated on the half-step grid (``coef`` shape
(2*steps+1, nterms)) and their derivatives with respect to the parameters
theta (``dcoef`` shape (2*steps+1, nterms, ntheta)).  For the driven dimer
the terms are the hopping, interaction and drive Hamiltonians and the
dissipator, and theta = (A, gamma, U).

The states v_0..v_steps come from classical RK4 (Sec. IV, step 3.1, same
stage layout as ``oracle.propagate.rk4_bloch``).  The objective is the mean
of the observable c.v over the last S grid states,

    J = (1/S) sum_{n = steps-S+1}^{steps} c . v_n,

(reading for "averaged over the last period": right-endpoint mean over the
S grid states of that period).  The derivative is that of this discrete J
(differentiate the discretisation, not the ODE).

* ``adjoint_gradient``  -- reverse sweep through every RK4 step with all
                           states stored (dense; small N).
* ``tangent_gradient``  -- forward-mode sensitivities dv/dtheta carried
                           along every step; an independent route to the
                           same numbers.
* ``objective``         -- J alone (used for finite differences).
* ``tangent_gradient_rho`` -- forward-mode sensitivities of classical RK4
                           applied to the density matrix itself (eq. 1),
                           J = mean of Re Tr(X rho_n); never touches the
                           SU(N) basis, so it is a third, independent route,
                           and cheap at large N for banded operators.

Parity: pinned -- central finite differences of ``objective`` and agreement
of the Bloch-form routes with each other and with the density-matrix route
(tests/test_oracle_adjoint.py).
"""

from __future__ import annotations

import numpy as np


def _G(Gs, c):
    out = c[0] * Gs[0]
    for a in range(1, len(Gs)):
        out = out + c[a] * Gs[a]
    return out


def _K(Ks, c, M):
    out = np.zeros(M)
    for a, Ka in enumerate(Ks):
        if Ka is not None:
            out = out + c[a] * Ka
    return out


def forward_states(Gs, Ks, coef, v0, dt, steps):
    """All RK4 grid states v_0..v_steps, shape (steps+1, M)."""
    M = v0.shape[0]
    V = np.zeros((steps + 1, M))
    V[0] = v0
    v = np.array(v0, dtype=np.float64)
    for n in range(steps):
        c0, ch, c1 = coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]
        G0, Gh, G1 = _G(Gs, c0), _G(Gs, ch), _G(Gs, c1)
        K0, Kh, K1 = _K(Ks, c0, M), _K(Ks, ch, M), _K(Ks, c1, M)
        k1 = G0 @ v + K0
        k2 = Gh @ (v + 0.5 * dt * k1) + Kh
        k3 = Gh @ (v + 0.5 * dt * k2) + Kh
        k4 = G1 @ (v + dt * k3) + K1
        v = v + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        V[n + 1] = v
    return V


def objective(Gs, Ks, coef, v0, cvec, dt, steps, S):
    V = forward_states(Gs, Ks, coef, v0, dt, steps)
    return float(np.mean(V[steps - S + 1: steps + 1] @ cvec))


def adjoint_gradient(Gs, Ks, coef, dcoef, v0, cvec, dt, steps, S):
    """Return (J, dJ/dtheta) by the discrete adjoint of the RK4 map."""
    M = v0.shape[0]
    ntheta = dcoef.shape[2]
    V = forward_states(Gs, Ks, coef, v0, dt, steps)
    J = float(np.mean(V[steps - S + 1: steps + 1] @ cvec))
    grad = np.zeros(ntheta)
    lam = np.zeros(M)                       # dJ/dv_{n+1}, accumulated
    for n in range(steps - 1, -1, -1):
        if n + 1 >= steps - S + 1:
            lam = lam + cvec / S            # direct dependence of J on v_{n+1}
        v = V[n]
        c0, ch, c1 = coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]
        d0, dh, d1 = dcoef[2 * n], dcoef[2 * n + 1], dcoef[2 * n + 2]
        G0, Gh, G1 = _G(Gs, c0), _G(Gs, ch), _G(Gs, c1)
        K0, Kh, K1 = _K(Ks, c0, M), _K(Ks, ch, M), _K(Ks, c1, M)
        # recompute the stages of step n
        x1 = v
        k1 = G0 @ x1 + K0
        x2 = v + 0.5 * dt * k1
        k2 = Gh @ x2 + Kh
        x3 = v + 0.5 * dt * k2
        k3 = Gh @ x3 + Kh
        x4 = v + dt * k3
        # v' = v + dt/6 (k1 + 2 k2 + 2 k3 + k4)
        kb1 = (dt / 6.0) * lam
        kb2 = (dt / 3.0) * lam
        kb3 = (dt / 3.0) * lam
        kb4 = (dt / 6.0) * lam
        vb = lam.copy()

        def dtheta(kb, x, dc):
            # kb . (dG/dtheta x + dK/dtheta) for every theta
            out = np.zeros(ntheta)
            for a in range(len(Gs)):
                if np.any(dc[a] != 0.0):
                    s = kb @ (Gs[a] @ x)
                    if Ks[a] is not None:
                        s += kb @ Ks[a]
                    out += dc[a] * s
            return out

        # k4 = G1 x4 + K1
        grad += dtheta(kb4, x4, d1)
        xb4 = G1.T @ kb4
        vb += xb4
        kb3 = kb3 + dt * xb4
        # k3 = Gh x3 + Kh
        grad += dtheta(kb3, x3, dh)
        xb3 = Gh.T @ kb3
        vb += xb3
        kb2 = kb2 + 0.5 * dt * xb3
        # k2 = Gh x2 + Kh
        grad += dtheta(kb2, x2, dh)
        xb2 = Gh.T @ kb2
        vb += xb2
        kb1 = kb1 + 0.5 * dt * xb2
        # k1 = G0 x1 + K0
        grad += dtheta(kb1, x1, d0)
        vb += G0.T @ kb1
        lam = vb
    return J, grad


def tangent_gradient(Gs, Ks, coef, dcoef, v0, cvec, dt, steps, S):
    """Return (J, dJ/dtheta) by forward-mode sensitivities W = dv/dtheta."""
    M = v0.shape[0]
    ntheta = dcoef.shape[2]
    v = np.array(v0, dtype=np.float64)
    W = np.zeros((M, ntheta))
    J = 0.0
    grad = np.zeros(ntheta)

    def stage(c, dc, x, Wx):
        G = _G(Gs, c)
        k = G @ x + _K(Ks, c, M)
        dk = G @ Wx
        for a in range(len(Gs)):
            if np.any(dc[a] != 0.0):
                t = Gs[a] @ x
                if Ks[a] is not None:
                    t = t + Ks[a]
                dk += np.outer(t, dc[a])
        return k, dk

    for n in range(steps):
        c0, ch, c1 = coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]
        d0, dh, d1 = dcoef[2 * n], dcoef[2 * n + 1], dcoef[2 * n + 2]
        k1, W1 = stage(c0, d0, v, W)
        k2, W2 = stage(ch, dh, v + 0.5 * dt * k1, W + 0.5 * dt * W1)
        k3, W3 = stage(ch, dh, v + 0.5 * dt * k2, W + 0.5 * dt * W2)
        k4, W4 = stage(c1, d1, v + dt * k3, W + dt * W3)
        v = v + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        W = W + (dt / 6.0) * (W1 + 2 * W2 + 2 * W3 + W4)
        if n + 1 >= steps - S + 1:
            J += (cvec @ v) / S
            grad += (cvec @ W) / S
    return J, grad


def tangent_gradient_rho(terms, coef, dcoef, rho0, X, dt, steps, S):
    """Return (J, dJ/dtheta) for RK4 on the density matrix (eq. 1).

    terms: list of (kind, op) with kind 'H' (contributes c_a(t) (-i[H_a, rho]))
    or 'L' (contributes c_a(t) D_{L_a}(rho), D_L(r) = L r L^+ - {L^+ L, r}/2);
    op dense, scipy sparse or workloads.ZCSR.  coef (2*steps+1, nterms) and
    dcoef (2*steps+1, nterms, ntheta) on the half-step grid, as for the Bloch
    form.  J = (1/S) sum_{n=steps-S+1}^{steps} Re Tr(X rho_n).

    The map rho -> rhs is linear in rho and in the coefficients, so the
    sensitivity W = d rho/d theta obeys dW/dt = rhs(W, c) + sum_a dc_a/dtheta
    term_a(rho), stepped with the same RK4 stages.  Since RK4 commutes with
    the affine map rho <-> v (eq. 5) and Re Tr(X rho) = Tr(X)/N + c.v with
    c_j = Tr(F_j X) for Hermitian X, this J (minus Tr(X)/N) and its gradient
    equal the Bloch-form ones in exact arithmetic.
    """
    import scipy.sparse as _sp

    def as_sp(op):
        if _sp.issparse(op):
            return op.tocsr().astype(np.complex128)
        if hasattr(op, "indptr") and hasattr(op, "re"):
            return _sp.csr_matrix((op.re + 1j * op.im, op.indices, op.indptr), shape=(op.n, op.n))
        return _sp.csr_matrix(np.asarray(op, dtype=np.complex128))

    ops = []
    for kind, op in terms:
        A = as_sp(op)
        if kind == "H":
            ops.append(("H", A, None, None))
        elif kind == "L":
            Ad = A.conj().T.tocsr()
            ops.append(("L", A, Ad, (Ad @ A).tocsr()))
        else:
            raise ValueError(kind)
    nt = len(ops)
    ntheta = dcoef.shape[2]
    Xd = as_sp(X)

    def right(r, B):                       # r @ B with B sparse
        return (B.T @ r.T).T

    def term(a, r):
        kind, A, Ad, AdA = ops[a]
        if kind == "H":
            return -1j * (A @ r - right(r, A))
        return A @ right(r, Ad) - 0.5 * (AdA @ r + right(r, AdA))

    def rhs(r, c):
        out = np.zeros_like(r)
        for a in range(nt):
            if c[a] != 0.0:
                out += c[a] * term(a, r)
        return out

    def stage(c, dc, x, Wx):
        k = rhs(x, c)
        dk = [rhs(Wx[th], c) for th in range(ntheta)]
        for a in range(nt):
            if np.any(dc[a] != 0.0):
                t = term(a, x)
                for th in range(ntheta):
                    if dc[a, th] != 0.0:
                        dk[th] = dk[th] + dc[a, th] * t
        return k, dk

    def obs(r):
        return float(np.real((Xd.multiply(r.T)).sum()))     # Re Tr(X r)

    rho = np.array(rho0, dtype=np.complex128, copy=True)
    W = [np.zeros_like(rho) for _ in range(ntheta)]
    J = 0.0
    grad = np.zeros(ntheta)
    for n in range(steps):
        c0, ch, c1 = coef[2 * n], coef[2 * n + 1], coef[2 * n + 2]
        d0, dh, d1 = dcoef[2 * n], dcoef[2 * n + 1], dcoef[2 * n + 2]
        k1, W1 = stage(c0, d0, rho, W)
        k2, W2 = stage(ch, dh, rho + 0.5 * dt * k1, [W[t] + 0.5 * dt * W1[t] for t in range(ntheta)])
        k3, W3 = stage(ch, dh, rho + 0.5 * dt * k2, [W[t] + 0.5 * dt * W2[t] for t in range(ntheta)])
        k4, W4 = stage(c1, d1, rho + dt * k3, [W[t] + dt * W3[t] for t in range(ntheta)])
        rho = rho + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        W = [W[t] + (dt / 6.0) * (W1[t] + 2.0 * W2[t] + 2.0 * W3[t] + W4[t]) for t in range(ntheta)]
        if n + 1 >= steps - S + 1:
            J += obs(rho) / S
            grad += np.array([obs(w) for w in W]) / S
    return J, grad
