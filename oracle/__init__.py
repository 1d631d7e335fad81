"""CPU FP64 oracle for piecewise-constant GRAPE, unitary and state-to-state,
open-system (Lindblad) GRAPE in Liouville space (oracle.lindblad) and the
trust-region method on the GRAPE residual (oracle.trm)
(test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its Python
binding) never imports, calls or links anything here.
"""
from . import lindblad, trm
from .grape import (
    slice_hamiltonians,
    expm_herm,
    slice_propagators,
    forward_products,
    backward_products,
    fidelity,
    frechet_dk,
    gradient,
    grape_ref,
    fidelity_ref,
)
from .state import (
    forward_states,
    backward_costates,
    state_overlap,
    state_dg,
    state_gradient,
    state_ref,
)

__all__ = [
    "slice_hamiltonians",
    "expm_herm",
    "slice_propagators",
    "forward_products",
    "backward_products",
    "fidelity",
    "frechet_dk",
    "gradient",
    "grape_ref",
    "fidelity_ref",
    "forward_states",
    "backward_costates",
    "state_overlap",
    "state_dg",
    "state_gradient",
    "state_ref",
]
