"""Seeded synthetic GRAPE workloads (spin-chain Hamiltonians, controls, targets).

This package only builds inputs: Pauli operators, spin-chain drift and
control Hamiltonians, control amplitudes and Haar-random target unitaries.
It contains none of the method's arithmetic (no exponentials, products,
fidelities or gradients), so both the CPU oracle and the HIP path can take
their inputs from it without sharing any computation.
"""
from .spin import (
    Problem,
    StateProblem,
    LindbladProblem,
    make_lindblad,
    haar_state,
    basis_state,
    make_state,
    make_state_batch,
    make_state_random,
    pauli,
    site_op,
    heisenberg_drift,
    ising_drift,
    xy_controls,
    haar_unitary,
    make_config,
    make_batch,
    make_request,
    make_random,
    make_random_monomial,
    random_hermitian,
    random_monomial_hermitian,
    poisson_trace,
    SERVE_DIMS,
    SERVE_WEIGHTS,
)

__all__ = [
    "Problem",
    "StateProblem",
    "LindbladProblem",
    "make_lindblad",
    "haar_state",
    "basis_state",
    "make_state",
    "make_state_batch",
    "make_state_random",
    "pauli",
    "site_op",
    "heisenberg_drift",
    "ising_drift",
    "xy_controls",
    "haar_unitary",
    "make_config",
    "make_batch",
    "make_request",
    "make_random",
    "make_random_monomial",
    "random_hermitian",
    "random_monomial_hermitian",
    "poisson_trace",
    "SERVE_DIMS",
    "SERVE_WEIGHTS",
]
