"""Stationary state of a time-independent generator (G v = -K) by GMRES on
the RK4 time-tau map (sun_stationary), against the oracle.

Bar: ||G v + K||_2 <= 1e-10 ||K||_2 (the solver's own criterion, recomputed
here from the oracle's explicit-trace matrices), and ||v - v_o||_2 <=
1e-9 ||v_o||_2 against the oracle's solution v_o: the error is at most
||G^-1||_2 times the residual, and ||K||_2 / sigma_min(G) is about 1.4 for the
dimer at N = 21 and 51 (so a residual of 1e-10 ||K|| moves v by at most
~1.5e-10 ||v||), plus the oracle's own LU residual (<= 2e-11).
Oracle: the normalised kernel of the dense Liouvillian (N = 4) and a sparse
LU solve on the C oracle's trace matrices (N = 51, 101, 301).
"""

import numpy as np
import pytest
import torch

from helpers import flush
from oracle import basis as ob, lindblad as lb, o2
from workloads import dimer

pytestmark = pytest.mark.gpu


def _system(sb, N):
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    basis = sb.build_basis(N)
    lind, prop = sb.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["L"], p.gamma_eff)])
    return p, ops, basis, lind, prop


def _oracle(p, ops):
    N = p.N
    if N <= 6:
        F = ob.generators(N)
        H = ops["H0"].to_dense() + p.E * ops["H1"].to_dense()
        L = ops["L"].to_dense()
        w, V = np.linalg.eig(lb.liouvillian(H, [L], [p.gamma_eff]))
        rho = lb.unvec(V[:, np.argmin(np.abs(w))], N)
        rho = rho / np.trace(rho)
        G = lb.q_hamiltonian(F, H) + p.gamma_eff * lb.q_dissipator(F, L)
        K = p.gamma_eff * lb.k_dissipator(F, L)
        return lb.bloch_vector(F, rho), G, K
    G = (o2.q_full("H", ops["H0"]) + p.E * o2.q_full("H", ops["H1"]) + p.gamma_eff * o2.q_full("L", ops["L"]))
    K = p.gamma_eff * o2.k_vector(ops["L"])
    return lb.stationary_bloch(G, K), G, K


@pytest.mark.parametrize("N,tau", [(4, 1.0), (51, 1.0), (101, 1.0), (301, 1.0), (51, 5.0)])
def test_stationary_against_oracle(lib, N, tau):
    flush(f"[stationary] N={N} tau={tau}")
    p, ops, basis, lind, prop = _system(lib, N)
    v, iters, relres = prop.stationary([p.E], tau=tau)
    flush(f"[stationary] N={N} tau={tau}: {iters} GMRES iterations, relres {relres:.2e}")
    v = v.cpu().numpy()
    v_o, G, K = _oracle(p, ops)
    assert relres <= 1e-10
    assert np.linalg.norm(G @ v + K) <= 1e-10 * np.linalg.norm(K)
    assert np.linalg.norm(v - v_o) <= 1e-9 * np.linalg.norm(v_o)
    assert iters <= 60


def test_unital_generator_returns_maximally_mixed_state(lib):
    """Pure dephasing (L = n1 - n2, Hermitian): K = 0, and v = 0 (rho = 1/N)
    is returned with zero residual."""
    N = 21
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    basis = lib.build_basis(N)
    lind, prop = lib.expand_lindbladian(basis, ops["H0"], ops["H1"], [(ops["H1"], 0.3)])
    v, iters, relres = prop.stationary([p.E], tau=5.0, v0=torch.ones(N * N - 1, dtype=torch.float64))
    assert relres == 0.0 and iters == 0
    assert torch.count_nonzero(v).item() == 0


def test_iteration_limit_and_nonfinite_guess(lib):
    p, ops, basis, lind, prop = _system(lib, 21)
    with pytest.raises(lib.SunError) as e:
        prop.stationary([p.E], tau=0.5, max_iter=2, tol=1e-14)
    assert e.value.code == lib._lib.SUN_ENOTCONVERGED
    bad = torch.zeros(21 * 21 - 1, dtype=torch.float64)
    bad[5] = float("nan")
    with pytest.raises(lib.SunError) as e:
        prop.stationary([p.E], tau=5.0, v0=bad)
    assert e.value.code == lib._lib.SUN_EDIVERGED
