"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only *builds inputs*: operator matrices in the Fock basis of the
driven Bose dimer, drive-coefficient tables sampled on the half-step grid,
random operators for parity tests and the seeded draw of the batched
instances.  It contains none of the method's arithmetic (no SU(N) basis, no
structure constants, no expansion, no propagation), so both the oracle and the
HIP path can take their inputs from here without sharing any of the method.
"""

from .dimer import (  # noqa: F401
    ZCSR,
    DimerParams,
    dimer_operators,
    drive_table,
    drive_table_dA,
    plain_config,
    batched_instances,
    adjoint_config,
    STEPS_PER_PERIOD,
    stable_steps_per_period,
)
from .random_ops import (  # noqa: F401
    random_hermitian_csr,
    random_complex_csr,
    random_tridiagonal_hermitian,
    random_vector,
)
