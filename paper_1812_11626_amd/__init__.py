"""sunbloch: SU(N) Bloch-vector Lindblad expansion and RK4 propagation on
AMD Instinct MI355X (gfx950), FP64, as hand-written HIP kernels behind a C ABI
(include/sunbloch.h).

Public entry points mirror the C ABI:

    basis = build_basis(N)
    lind, prop = expand_lindbladian(basis, H0, H1, [(L, gamma)])
    v = propagate(prop, v0, eps, dt, steps)

plus the batched form (``BatchedPropagator``, ``autotune_batched``) and the
adjoint form (``Adjoint``, ``AdjointProblem``, ``SunBlochLoss``).  The package has no CPU fallback.
"""

from ._lib import SunError, load as load_library  # noqa: F401
from .api import (  # noqa: F401
    Adjoint,
    AdjointProblem,
    BatchedPropagator,
    Basis,
    DeviceOperator,
    Lindbladian,
    Propagator,
    build_basis,
    expand_lindbladian,
    gemm_f64,
    propagate,
    require_gpu,
    SunBlochLoss,
    use_default_allocator,
    use_torch_allocator,
)
from .autotune import autotune_batched  # noqa: F401
