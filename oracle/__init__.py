"""Plain, slow, float64 CPU oracle of the bistochastic kernel EVD method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the GPU library never
calls it and shares no code with it.

Each function cites the part of the paper it follows (Vales & Giannakis,
"Accelerated decomposition of bistochastic kernel matrices by low rank
approximation").  Where the paper leaves a detail open, the reading taken is
stated next to the code that implements it.

`oracle.surrogate` holds the float64 reference of the learned surrogate of
the Nystrom extension (multilayer perceptron, its gradients and AdamW).
"""
from .kernel import gaussian_kernel, sq_distances
from .arpc import (
    quantize_rho,
    inverse_cdf_pivot,
    greedy_pivot,
    accept_reject,
    arpc,
    QSCALE,
)
from . import surrogate
from .bistoch import (
    bistoch_degrees,
    bistoch_eig,
    sign_normalize,
    nystrom_extend,
    dense_bistochastic,
    dense_symmetric,
    symmetric_eig,
    symmetric_extend,
)

__all__ = [
    "gaussian_kernel",
    "sq_distances",
    "quantize_rho",
    "inverse_cdf_pivot",
    "greedy_pivot",
    "accept_reject",
    "arpc",
    "QSCALE",
    "bistoch_degrees",
    "bistoch_eig",
    "sign_normalize",
    "nystrom_extend",
    "dense_bistochastic",
    "dense_symmetric",
    "symmetric_eig",
    "symmetric_extend",
    "surrogate",
]
