"""Driven, dissipatively coupled Bose dimer (paper Sec. III, testbed model).

The workloads used here are a variant of the paper's model, eqs. (12)-(13):

    H(t) = -J (b1^+ b2 + b2^+ b1) + (U_eff/2) sum_j n_j (n_j - 1) + eps(t) (n1 - n2)
    eps(t) = E + A cos(omega t)
    L      = (b1^+ + b2^+)(b1 - b2)        with rate gamma_eff

on N-1 bosons, i.e. an N-dimensional Hilbert space.  The Fock basis is
ordered by the occupation of site 1: state i is |n1 = i, n2 = N-1-i>,
i = 0..N-1, so that <i+1| b1^+ b2 |i> = sqrt((i+1)(N-1-i)).

In this basis H_J = b1^+ b2 + b2^+ b1 is symmetric tridiagonal, the
interaction and drive terms are diagonal, and L is diag(n1 - n2) plus an
antisymmetric nearest-neighbour part (paper Sec. III, last paragraph).

Everything here is *input construction*: operator matrix elements in the Fock
basis and drive values on a time grid.  Nothing in this module knows about the
SU(N) expansion or about time stepping beyond the sampling grid.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Steps per drive period used for each Hilbert-space dimension.  RK4 on the
# Bloch equations is stable only while |lambda_max| * dt stays inside the
# stability region (about 2.83 on the imaginary axis); for the dimer
# |lambda_max| grows like 2 sqrt(eps^2 + J^2) (N - 1), so the step count per
# period grows linearly with N.  Values for N <= 51 are the nominal ones.
STEPS_PER_PERIOD = {4: 200, 6: 200, 51: 1000, 101: 2048, 151: 2048,
                    201: 4096, 301: 4096, 1001: 16384}


@dataclass
class ZCSR:
    """Complex N x N operator in CSR form (0-based, sorted columns).

    ``indptr`` (n+1,) int32, ``indices`` (nnz,) int32, ``re``/``im`` (nnz,)
    float64.  This is the operator format the library boundary takes.
    """

    n: int
    indptr: np.ndarray
    indices: np.ndarray
    re: np.ndarray
    im: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.n), dtype=np.complex128)
        for r in range(self.n):
            for e in range(self.indptr[r], self.indptr[r + 1]):
                out[r, self.indices[e]] += self.re[e] + 1j * self.im[e]
        return out

    @staticmethod
    def from_dense(a: np.ndarray, tol: float = 0.0) -> "ZCSR":
        a = np.asarray(a, dtype=np.complex128)
        n = a.shape[0]
        indptr = [0]
        idx, re, im = [], [], []
        for r in range(n):
            for c in range(n):
                if abs(a[r, c]) > tol:
                    idx.append(c)
                    re.append(a[r, c].real)
                    im.append(a[r, c].imag)
            indptr.append(len(idx))
        return ZCSR(n, np.asarray(indptr, np.int32), np.asarray(idx, np.int32),
                    np.asarray(re, np.float64), np.asarray(im, np.float64))

    @staticmethod
    def from_diagonals(n: int, diags: dict) -> "ZCSR":
        """Build from {offset: values} (offset k: entries (i, i+k))."""
        rows = [[] for _ in range(n)]
        for k, vals in diags.items():
            vals = np.asarray(vals, dtype=np.complex128)
            for t, v in enumerate(vals):
                i = t if k >= 0 else t - k
                j = i + k
                if v != 0:
                    rows[i].append((j, v))
        indptr = [0]
        idx, re, im = [], [], []
        for r in range(n):
            for c, v in sorted(rows[r]):
                idx.append(c)
                re.append(v.real)
                im.append(v.imag)
            indptr.append(len(idx))
        return ZCSR(n, np.asarray(indptr, np.int32), np.asarray(idx, np.int32),
                    np.asarray(re, np.float64), np.asarray(im, np.float64))

    def scaled(self, c: float) -> "ZCSR":
        return ZCSR(self.n, self.indptr.copy(), self.indices.copy(),
                    self.re * c, self.im * c)


@dataclass
class DimerParams:
    """Physical parameters of one dimer instance (effective values)."""

    N: int                 # Hilbert-space dimension (N - 1 bosons)
    J: float = 1.0
    U: float = 0.5         # nominal interaction strength
    U_scale: float = 1.0   # U_eff = U * U_scale
    E: float = 1.0
    A: float = 1.5
    omega: float = 1.0
    gamma: float = 0.1     # nominal dissipation rate
    gamma_scale: float = 1.0  # gamma_eff = gamma * gamma_scale
    steps_per_period: int = 200
    periods: int = 10
    rho0_index: int = 0    # initial pure Fock state |i><i|
    label: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def U_eff(self) -> float:
        return self.U * self.U_scale

    @property
    def gamma_eff(self) -> float:
        return self.gamma * self.gamma_scale

    @property
    def T(self) -> float:
        return 2.0 * math.pi / self.omega

    @property
    def dt(self) -> float:
        return self.T / self.steps_per_period

    @property
    def steps(self) -> int:
        return self.steps_per_period * self.periods


def _hop_amplitudes(N: int) -> np.ndarray:
    i = np.arange(N - 1, dtype=np.float64)
    return np.sqrt((i + 1.0) * (N - 1.0 - i))


def dimer_operators(p: DimerParams) -> dict:
    """Fock-basis CSR operators of the dimer.

    Returns a dict with
      H0  = -J H_J + (U_eff/2) sum_j n_j(n_j-1)   (time independent part)
      H1  = n1 - n2                                (multiplied by eps(t))
      HJ  = H_J = b1^+ b2 + b2^+ b1
      HU  = (1/2) sum_j n_j(n_j-1)                (so dH/dU_eff = HU)
      L   = (b1^+ + b2^+)(b1 - b2)                 (unit rate)
    """
    N = p.N
    s = _hop_amplitudes(N)
    i = np.arange(N, dtype=np.float64)
    n1 = i
    n2 = (N - 1) - i
    inter = 0.5 * (n1 * (n1 - 1) + n2 * (n2 - 1))
    HJ = ZCSR.from_diagonals(N, {-1: s, 1: s})
    H0 = ZCSR.from_diagonals(N, {-1: -p.J * s, 0: p.U_eff * inter, 1: -p.J * s})
    H1 = ZCSR.from_diagonals(N, {0: n1 - n2})
    HU = ZCSR.from_diagonals(N, {0: inter})
    # (b1^+ + b2^+)(b1 - b2) = n1 - n2 - b1^+ b2 + b2^+ b1
    # <i+1| b1^+ b2 |i> = s_i  -> entry (i+1, i) gets -s_i
    # <i| b2^+ b1 |i+1> = s_i  -> entry (i, i+1) gets +s_i
    L = ZCSR.from_diagonals(N, {-1: -s, 0: n1 - n2, 1: s})
    return {"H0": H0, "H1": H1, "HJ": HJ, "HU": HU, "L": L}


def drive_table(p: DimerParams, steps: int | None = None, t0: float = 0.0,
                dt: float | None = None) -> np.ndarray:
    """eps(t_k) on the half-step grid t_k = t0 + k dt/2, k = 0..2*steps.

    Both sides read the drive from this one table, so they see identical
    values.  Shape (2*steps+1,), float64.
    """
    steps = p.steps if steps is None else steps
    dt = p.dt if dt is None else dt
    k = np.arange(2 * steps + 1, dtype=np.float64)
    t = t0 + k * (0.5 * dt)
    return p.E + p.A * np.cos(p.omega * t)


def drive_table_square(p: DimerParams, steps: int | None = None) -> np.ndarray:
    """eps = E + A theta(t) with the square wave theta = +1 on the first half
    of every period and -1 on the second (paper Sec. III), on the half-step
    grid t_k = k dt/2 of a run that starts at t = 0 with steps_per_period
    steps per period.  The half is decided by the integer phase index
    k mod (2 steps_per_period), so the jumps fall exactly on grid points
    (t = T/2 takes -1, t = T takes +1)."""
    steps = p.steps if steps is None else steps
    k = np.arange(2 * steps + 1)
    half = p.steps_per_period
    theta = np.where((k % (2 * half)) < half, 1.0, -1.0)
    return p.E + p.A * theta


def drive_table_dA(p: DimerParams, steps: int | None = None, t0: float = 0.0,
                   dt: float | None = None) -> np.ndarray:
    """d eps / dA on the same half-step grid (= cos(omega t_k))."""
    steps = p.steps if steps is None else steps
    dt = p.dt if dt is None else dt
    k = np.arange(2 * steps + 1, dtype=np.float64)
    t = t0 + k * (0.5 * dt)
    return np.cos(p.omega * t)


def plain_config(N: int) -> DimerParams:
    """The plain-propagation workloads: N = 4, 51 and 1001.

    N = 4 uses the literal parameters (U = 0.5, gamma = 0.1).  For larger N the
    interaction is normalised by the boson number, U_eff = 0.5/(N-1), and the
    rate by the dimension, gamma_eff = 0.1/N.
    """
    if N <= 6:
        return DimerParams(N=N, steps_per_period=STEPS_PER_PERIOD.get(N, 200),
                           periods=10, label=f"dimer-plain-N{N}")
    periods = {51: 100, 1001: 50}.get(N, 10)
    return DimerParams(N=N, U_scale=1.0 / (N - 1), gamma_scale=1.0 / N,
                       steps_per_period=STEPS_PER_PERIOD.get(N, 4096),
                       periods=periods, label=f"dimer-plain-N{N}")


BATCH_SEED = 181211626
BATCH_SIZES = (51, 101, 151, 201, 301)


def stable_steps_per_period(N: int, eps_max: float, J: float = 1.0,
                            omega: float = 1.0, nominal: int = 1000,
                            quantum: int = 256, margin: float = 1.02) -> int:
    """Smallest step count per period (a multiple of ``quantum``, at least
    ``nominal``) with |lambda_max| dt <= 2.5, using the dimer estimate
    |lambda_max| ~= 2 sqrt(eps_max^2 + J^2) (N - 1) times ``margin`` (the
    interaction and dissipation terms raise the true spectral radius by up to
    ~1% at the workloads' parameters)."""
    lam = 2.0 * math.sqrt(eps_max * eps_max + J * J) * (N - 1) * margin
    T = 2.0 * math.pi / omega
    need = math.ceil(T * lam / 2.5)
    need = quantum * math.ceil(need / quantum)
    return max(nominal, need)


def batched_instances(count: int = 512, seed: int = BATCH_SEED,
                      sizes=BATCH_SIZES, periods: int = 20) -> list:
    """Seeded draw of the batched workload.

    N ~ uniform over ``sizes``, A ~ U[0.5, 3.0], gamma ~ logU[0.01, 0.5]
    (gamma_eff = gamma / N), U_eff = 0.5/(N-1); other parameters as in the
    plain workloads.  Draw order: all N, then all A, then all log gamma.
    All instances of one N share a step size: the stable step count of the
    largest drive amplitude drawn for that N.
    """
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sizes), size=count)
    As = rng.uniform(0.5, 3.0, size=count)
    gs = np.exp(rng.uniform(math.log(0.01), math.log(0.5), size=count))
    spp = {}
    for N in sizes:
        sel = As[Ns == N]
        amax = float(sel.max()) if sel.size else 3.0
        spp[int(N)] = stable_steps_per_period(int(N), 1.0 + amax)
    out = []
    for b in range(count):
        N = int(Ns[b])
        out.append(DimerParams(N=N, A=float(As[b]), gamma=float(gs[b]),
                               U_scale=1.0 / (N - 1), gamma_scale=1.0 / N,
                               steps_per_period=spp[N],
                               periods=periods, label=f"batched-{b}"))
    return out


def bifurcation_instances(N: int, count: int = 64, U_min: float = 0.05, U_max: float = 2.0,
                          periods: int = 10) -> list:
    """U scan for the stroboscopic population diagram (paper Sec. III, Fig. 2:
    P(n bosons on site 1) at t = 10T against the interaction): count values
    of U evenly spaced in [U_min, U_max], U_eff = U/(N-1), gamma_eff = 0.1/N,
    A = 1.5, E = 1, J = 1, omega = 1, rho0 = |0, N-1><0, N-1|.  All share the
    stable step count of the drive range E +- A."""
    spp = stable_steps_per_period(N, 1.0 + 1.5)
    out = []
    for i, U in enumerate(np.linspace(U_min, U_max, count)):
        out.append(DimerParams(N=N, U=float(U), U_scale=1.0 / (N - 1), gamma_scale=1.0 / N,
                               steps_per_period=spp, periods=periods, label=f"bifurcation-{i}"))
    return out


def adjoint_config(N: int = 301) -> DimerParams:
    """Adjoint workload: N = 301, 100 periods, loss = <n1 - n2> averaged over
    the last period.  Small-N variants (N <= 6) use literal parameters."""
    if N <= 6:
        return DimerParams(N=N, steps_per_period=200, periods=2,
                           label=f"adjoint-N{N}")
    return DimerParams(N=N, U_scale=1.0 / (N - 1), gamma_scale=1.0 / N,
                       steps_per_period=STEPS_PER_PERIOD.get(N, 4096),
                       periods=100, label=f"adjoint-N{N}")
