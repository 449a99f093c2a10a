"""CPU oracle for the SU(N) Bloch-vector Lindblad path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product path (the
HIP library and its Python binding) never calls it and shares no code with it.

Everything here is plain float64 NumPy/SciPy written from the definitions in
the paper:

* ``basis``       -- the SU(N) generators S, J, D (Sec. II) built densely, and
                     the structure constants f, d by their trace definitions
                     (Sec. II, eq. 4).  Brute force, N <= 8.
* ``lindblad``    -- Q, R (=Q_D) and K by explicit traces of the GKSL
                     generator (eq. 1) against the basis (dense, small N), the
                     same traces column by column with sparse operators at any
                     N, the dense N^2 x N^2 Liouvillian, Bloch vectors (eq. 5).
* ``propagate``   -- classical RK4 on the real ODE (eq. 9), RK4 on the density
                     matrix itself (eq. 1), and matrix-exponential propagation.
* ``adjoint``     -- the discrete adjoint of the RK4 map for a time-averaged
                     observable, plus forward-mode (tangent-linear)
                     sensitivities, dense, and the same sensitivities of RK4
                     on the density matrix itself (no basis).
* ``o2``          -- plain C + OpenMP (``o2.c``, compiled by build() into
                     ``libo2.so``): Q, R, K by the same explicit traces column
                     by column at any N, and a multi-core CSR RK4 (the timed
                     CPU baseline).

Parity status of each function is stated in its own docstring; every function
is pinned by tests against values the paper or the mathematics fixes.
"""

from . import basis, lindblad, propagate, adjoint, o2  # noqa: F401
