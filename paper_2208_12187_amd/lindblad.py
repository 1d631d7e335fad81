"""Open-system (Lindblad) GRAPE on libqoc's general-generator path.

The master equation d rho/dt = -i [H_k, rho] + sum_l (L_l rho L_l^dag -
1/2 {L_l^dag L_l, rho}) with H_k = H0 + sum_j u[j, k] H_j is linear in rho; on
the row-major vectorisation vec(rho)[a d + b] = rho[a, b] (vec(A rho B) =
(A (x) B^T) vec(rho)) its generator is

    G_k = G0 + sum_j u[j, k] G_j,
    G0  = -i (H0 (x) I - I (x) H0^T) + sum_l (L_l (x) conj(L_l)
          - 1/2 (L_l^dag L_l (x) I + I (x) (L_l^dag L_l)^T)),
    G_j = -i (H_j (x) I - I (x) H_j^T).

libqoc runs the slices S_k = exp(dt G_k), the products X_N, the fidelity
against the target's superoperator T = V (x) conj(V) (T vec(rho) =
vec(V rho V^dag)), F = |Tr(T^dag X_N)|^2 / d^4, and the exact gradient, with
its general-generator option (qoc_options.generators): the same kernels as
the closed system, with the adjoint built from A_k^dag.  This module only
builds the d^2 x d^2 inputs; for a closed system F = F_unitary^2.
"""
from __future__ import annotations

import numpy as np

from . import qoc


def liouvillian(H0, Hc, Ls):
    """(G0, G[j]) of the master equation, d^2 x d^2 complex128."""
    H0 = np.asarray(H0, dtype=np.complex128)
    d = H0.shape[0]
    I = np.eye(d, dtype=np.complex128)
    comm = lambda H: -1j * (np.kron(H, I) - np.kron(I, H.T))
    G0 = comm(H0)
    for L in Ls:
        L = np.asarray(L, dtype=np.complex128)
        LdL = L.conj().T @ L
        G0 = G0 + np.kron(L, L.conj()) - 0.5 * (np.kron(LdL, I) + np.kron(I, LdL.T))
    Gc = np.stack([comm(np.asarray(H, dtype=np.complex128)) for H in Hc])
    return G0, Gc


def target_superoperator(V):
    V = np.asarray(V, dtype=np.complex128)
    return np.kron(V, V.conj())


def gradient(problem, precision="fp64", hbm_budget=0, chunk=0):
    """(F, grad) of a workloads.LindbladProblem through libqoc."""
    G0, Gc = liouvillian(problem.H0, problem.Hc, problem.Ls)
    return qoc.gradient(G0, Gc, problem.u, problem.dt, target_superoperator(problem.V), precision,
                        hbm_budget=hbm_budget, chunk=chunk, generators=True)


def propagate(problem, precision="fp64"):
    """The Liouville-space X_N (d^2 x d^2) through libqoc."""
    G0, Gc = liouvillian(problem.H0, problem.Hc, problem.Ls)
    return qoc.propagate(G0, Gc, problem.u, problem.dt, precision, generators=True)
