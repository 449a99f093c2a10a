"""Write adjoint_goldens.txt: J and dJ/d(A, gamma, U) of the period-averaged
<n1 - n2> through the RK4 map for the dimer problems whose gradients the GPU
reports at scale, computed by the oracle's density-matrix route
(``oracle.adjoint.tangent_gradient_rho``: forward-mode sensitivities of RK4
applied to eq. 1 directly, no SU(N) basis; equal to the Bloch-form discrete
adjoint in exact arithmetic, pinned against it at small N).

Problems (terms H_J, H_U, H1, L with coefficients -J, U U_scale,
E + A cos(omega t), gamma gamma_scale; theta = (A, gamma, U); rho0 = |0><0|):

* adjoint-N301: the adjoint workload (U_eff = U/300, gamma_eff = gamma/301,
  4096 steps per period), 256 steps, J averaged over the last 128 states.
* plain-N1001: the plain N = 1001 workload (U_eff = U/1000,
  gamma_eff = gamma/1001, 16384 steps per period), 512 steps, J averaged
  over the last 256 states.

Calls only oracle/ and the workload input generators.  About 25 minutes on
one CPU core."""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint as oadj  # noqa: E402
from workloads import dimer  # noqa: E402

THETA = (1.5, 0.1, 0.5)
PROBLEMS = (("adjoint-N301", 301, 256, 128), ("plain-N1001", 1001, 512, 256))


def problem(name, N):
    p = dimer.adjoint_config(N) if name.startswith("adjoint") else dimer.plain_config(N)
    p.A, p.gamma, p.U = THETA
    return p


def solve(name, N, steps, S):
    p = problem(name, N)
    ops = dimer.dimer_operators(p)
    terms = [("H", ops["HJ"]), ("H", ops["HU"]), ("H", ops["H1"]), ("L", ops["L"])]
    coef = np.zeros((2 * steps + 1, 4))
    coef[:, 0] = -p.J
    coef[:, 1] = p.U_eff
    coef[:, 2] = dimer.drive_table(p, steps=steps)
    coef[:, 3] = p.gamma_eff
    dcoef = np.zeros((2 * steps + 1, 4, 3))
    dcoef[:, 2, 0] = dimer.drive_table_dA(p, steps=steps)
    dcoef[:, 3, 1] = p.gamma_scale
    dcoef[:, 1, 2] = p.U_scale
    rho0 = np.zeros((N, N), complex)
    rho0[p.rho0_index, p.rho0_index] = 1.0
    X = ops["H1"]
    return oadj.tangent_gradient_rho(terms, coef, dcoef, rho0, X, p.dt, steps, S)


def main():
    lines = ["# J and dJ/d(A, gamma, U) of the period-averaged <n1-n2> (oracle density-matrix tangent route).",
             "# name N steps S_avg J dJ/dA dJ/dgamma dJ/dU   (theta = A, gamma, U = %r)" % (THETA,)]
    for name, N, steps, S in PROBLEMS:
        t0 = time.time()
        J, g = solve(name, N, steps, S)
        lines.append(f"{name} {N} {steps} {S} {float(J)!r} {float(g[0])!r} {float(g[1])!r} {float(g[2])!r}")
        print(f"{name}: J={J!r} grad={list(g)} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "adjoint_goldens.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
