"""Write dimer_n1001_period.txt: the plain N = 1001 dimer workload (Fock state
|0, N-1><0, N-1| at t = 0, drive eps(t) = E + A cos(omega t)) after one drive
period of 16,384 RK4 steps, integrated by the oracle's density-matrix RK4
(eq. 1; RK4 commutes with the affine map rho <-> v of eq. 5, so the Bloch
form reaches the same state up to rounding).  Records <n1 - n2> every 1024
steps and the Bloch vector v_j = Tr(F_j rho) at seeded sample indices.

Calls only oracle/ and the workload input generators; takes about two hours
on one CPU core."""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lindblad as lb, propagate as pr  # noqa: E402
from workloads import dimer  # noqa: E402

EVERY = 1024
NSAMPLE = 1500


def sample_indices(N: int) -> np.ndarray:
    """Seeded uniform sample over all M generators, every other D_l, and the
    S and J generators of near-diagonal pairs (k = j + 1 for every third j,
    k = j + 2 for every third j), where the coherences are largest."""
    M = N * N - 1
    P = N * (N - 1) // 2
    rng = np.random.default_rng(1001)
    idx = rng.choice(M, size=NSAMPLE, replace=False)

    def pair(j, k):   # grouped order: S_jk at p, J_jk at P + p
        return j * (2 * N - j - 1) // 2 + (k - j - 1)

    near = [pair(j, j + 1) for j in range(0, N - 1, 3)] + [pair(j, j + 2) for j in range(1, N - 2, 3)]
    near = np.asarray(near)
    return np.unique(np.concatenate([idx, np.arange(2 * P, M, 2), near, P + near]))


def main():
    N = 1001
    p = dimer.plain_config(N)
    ops = dimer.dimer_operators(p)
    steps = p.steps_per_period
    eps = dimer.drive_table(p, steps=steps)
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1.0
    t0 = time.time()
    rho, rec = pr.rk4_rho(ops["H0"], [ops["H1"]], [ops["L"]], [p.gamma_eff], rho0, eps[:, None], p.dt, steps,
                          record_every=EVERY)
    n1mn2 = 2.0 * np.arange(N) - (N - 1)
    obs = [float(np.real(np.diag(r)) @ n1mn2) for r in rec]
    v = lb.bloch_vector_sparse(rho)
    idx = sample_indices(N)
    with open(os.path.join(HERE, "dimer_n1001_period.txt"), "w") as fh:
        fh.write("# Plain dimer N=1001 (U_eff=0.5/1000, gamma_eff=0.1/1001, A=1.5, E=1, omega=1), rho0 = |0><0|,\n")
        fh.write(f"# {steps} RK4 steps of dt = T/{steps} (one period), oracle density-matrix RK4 (eq. 1).\n")
        fh.write(f"# Written by make_dimer_n1001_period.py in {time.time() - t0:.0f} s.\n")
        fh.write(f"# obs k <n1-n2> after k*{EVERY} steps; v j v_j after the period (grouped basis order)\n")
        for k, o in enumerate(obs, start=1):
            fh.write(f"obs {k} {o!r}\n")
        for j in idx:
            fh.write(f"v {int(j)} {float(v[j])!r}\n")


if __name__ == "__main__":
    main()
