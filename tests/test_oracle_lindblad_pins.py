"""Pins of the open-system (Lindblad) oracle.

* Its generator builder against the textbook Kronecker forms
  -i (H (x) I - I (x) H^T) and L (x) conj(L) - 1/2 (L^dag L (x) I + I (x) (L^dag L)^T).
* A closed system reduces to the (separately pinned) unitary oracle:
  X_N = U_N (x) conj(U_N), F = F_u^2 and dF/du = 2 F_u dF_u/du.
* Pure dephasing and amplitude damping of one qubit in closed form.
* The evolution preserves the trace: vec(I)^T X_N = vec(I)^T.
* Central finite differences of F on every entry.
"""
import numpy as np
import pytest

import oracle
from oracle import lindblad as LB
from workloads import LindbladProblem, make_lindblad, make_random, pauli

SX, SZ = pauli("x"), pauli("z")
LOWER = np.array([[0, 1], [0, 0]], dtype=np.complex128)


def test_generators_match_the_kronecker_forms():
    rng = np.random.default_rng(1)
    d = 3
    H = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H = H + H.conj().T
    L = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    I = np.eye(d)
    assert np.max(np.abs(LB.commutator_generator(H) - (-1j) * (np.kron(H, I) - np.kron(I, H.T)))) < 1e-14
    LdL = L.conj().T @ L
    ref = np.kron(L, L.conj()) - 0.5 * (np.kron(LdL, I) + np.kron(I, LdL.T))
    assert np.max(np.abs(LB.dissipator([L], d) - ref)) < 1e-13


def test_closed_system_reduces_to_the_unitary_oracle():
    p = make_random(5, 3, 2, 8, 0.1)
    F, g, grad, XN = LB.lindblad_gradient(p.H0, p.Hc, [], p.u, p.dt, p.V)
    ref = oracle.grape_ref(p)
    assert np.max(np.abs(XN - np.kron(ref["XN"], ref["XN"].conj()))) < 1e-13
    assert abs(F - ref["F"] ** 2) < 1e-14
    assert np.max(np.abs(grad - 2 * ref["F"] * ref["grad"])) < 1e-13


def test_single_qubit_dephasing_closed_form():
    """H = 0, L = sqrt(g) Z: coherences decay as exp(-2 g T), populations stay."""
    gam, N, dt = 0.3, 20, 0.05
    _, _, _, XN = LB.lindblad_gradient(np.zeros((2, 2)), SX[None], [np.sqrt(gam) * SZ], np.zeros((1, N)), dt,
                                       np.eye(2))
    e = np.exp(-2 * gam * N * dt)
    assert np.max(np.abs(XN - np.diag([1, e, e, 1]))) < 1e-13


def test_single_qubit_amplitude_damping_closed_form():
    """L = sqrt(g) |0><1|: rho_11 -> e^{-gT} rho_11, rho_00 -> rho_00 + (1 - e^{-gT}) rho_11,
    rho_01 -> e^{-gT/2} rho_01."""
    gam, N, dt = 0.4, 25, 0.04
    _, _, _, XN = LB.lindblad_gradient(np.zeros((2, 2)), SX[None], [np.sqrt(gam) * LOWER], np.zeros((1, N)), dt,
                                       np.eye(2))
    T = N * dt
    ref = np.zeros((4, 4))
    ref[0, 0], ref[0, 3], ref[3, 3] = 1.0, 1 - np.exp(-gam * T), np.exp(-gam * T)
    ref[1, 1] = ref[2, 2] = np.exp(-gam * T / 2)
    assert np.max(np.abs(XN - ref)) < 1e-13


@pytest.mark.parametrize("nq,N", [(1, 12), (2, 6)])
def test_trace_is_preserved(nq, N):
    p = make_lindblad(nq, N, dt=0.05, gamma_damp=0.2, gamma_deph=0.1)
    XN = oracle.lindblad.lindblad_ref(p)["XN"]
    vI = np.eye(p.d).reshape(-1)
    assert np.max(np.abs(vI @ XN - vI)) < 1e-13


@pytest.mark.parametrize("nq,N", [(1, 7), (2, 4)])
def test_gradient_matches_central_differences(nq, N):
    p = make_lindblad(nq, N, dt=0.08, gamma_damp=0.15, gamma_deph=0.05, seed=3)
    r = LB.lindblad_ref(p)
    h = 1e-6
    gmax = np.max(np.abs(r["grad"]))
    for j in range(p.m):
        for k in range(p.N):
            up, dn = p.u.copy(), p.u.copy()
            up[j, k] += h
            dn[j, k] -= h
            fd = (LB.lindblad_ref(p.with_u(up))["F"] - LB.lindblad_ref(p.with_u(dn))["F"]) / (2 * h)
            assert abs(fd - r["grad"][j, k]) < 1e-7 * max(gmax, 1e-3), (j, k)
