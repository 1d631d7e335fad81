"""Pins that fix the state-to-state oracle to facts outside itself.

Closed forms of the single-qubit transfer |0> -> |1>, the commuting-field
gradient, the constant-field sum rule, conservation of norm and of the overlap
<lam_k | psi_k> along the chain, the stationary point at chi = psi_N, central
finite differences, and the decomposition of the unitary trace into basis-state
transfers: with psi0 = e_a and chi = V e_a, g_a = (V^dag X_N)_aa, so
sum_a g_a = Tr(V^dag X_N) and sum_a dg_a/du = dg/du of the (separately
pinned) unitary oracle.  A dropped drift, a wrong sign of i, a costate taken
one slice early or late, a missing conjugate or a transposed control fails
at least one of them.
"""
import numpy as np
import pytest

import oracle
from workloads import (Problem, StateProblem, basis_state, make_config, make_random, make_state,
                       make_state_random, pauli)

SX, SY, SZ = pauli("x"), pauli("y"), pauli("z")
E0, E1 = basis_state(2, 0), basis_state(2, 1)


def _qubit(omega, u, N, dt):
    return StateProblem(0.5 * omega * SZ, SX[None], np.full((1, N), float(u)), dt, E0, E1)


@pytest.mark.parametrize("omega,u", [(1.0, 0.7), (1.0, -0.3), (2.5, 1.9)])
def test_closed_form_single_qubit_transfer(omega, u):
    """H = (w/2) Z + u X: psi_N = X_N |0> with X_N = cos(bT) I - i sin(bT)(u X + (w/2) Z)/b,
    so psi_N = (cos bT - i (w/2) sin(bT)/b, -i u sin(bT)/b) and F = u^2 sin^2(bT)/b^2."""
    N, dt = 100, 0.01
    r = oracle.state_ref(_qubit(omega, u, N, dt))
    T, b = N * dt, np.sqrt(u * u + omega * omega / 4)
    psiN = np.array([np.cos(b * T) - 0.5j * omega * np.sin(b * T) / b, -1j * u * np.sin(b * T) / b])
    assert np.max(np.abs(r["psiN"] - psiN)) < 1e-13
    assert abs(r["F"] - u * u * np.sin(b * T) ** 2 / b ** 2) < 1e-13


@pytest.mark.parametrize("omega,u", [(1.0, 0.7), (2.5, -1.1)])
def test_constant_field_sum_rule(omega, u):
    """Sum over slices of dF/du_k = dF/du of the closed form, with s = sin bT, c = cos bT:
    d/du [u^2 s^2 / b^2] = 2u s^2/b^2 + 2u^3 s c T / b^3 - 2u^3 s^2 / b^4."""
    N, dt = 100, 0.01
    r = oracle.state_ref(_qubit(omega, u, N, dt))
    T, b = N * dt, np.sqrt(u * u + omega * omega / 4)
    s, c = np.sin(b * T), np.cos(b * T)
    dF = 2 * u * s * s / b ** 2 + 2 * u ** 3 * s * c * T / b ** 3 - 2 * u ** 3 * s * s / b ** 4
    assert abs(r["grad"].sum() - dF) < 1e-13


def test_commuting_field_gradient_closed_form():
    """H0 = 0, one X control, |0> -> |1>: g = -i sin(Theta) with Theta = dt sum_k u_k,
    F = sin^2 Theta and dF/du_k = dt sin(2 Theta) for every k."""
    p0 = make_config(1)
    p = StateProblem(np.zeros((2, 2), complex), SX[None], p0.u, p0.dt, E0, E1)
    r = oracle.state_ref(p)
    th = p.dt * p.u.sum()
    assert abs(r["g"] - (-1j * np.sin(th))) < 1e-14
    assert abs(r["F"] - np.sin(th) ** 2) < 1e-14
    assert np.max(np.abs(r["grad"] - p.dt * np.sin(2 * th))) < 1e-15


@pytest.mark.parametrize("seed,d,m,N,dt", [(1, 5, 3, 17, 0.05), (2, 16, 4, 30, 0.02)])
def test_norm_and_overlap_are_conserved_along_the_chain(seed, d, m, N, dt):
    """|psi_k| = |lam_k| = 1 and <lam_k | psi_k> = g for every k."""
    p = make_state_random(seed, d, m, N, dt)
    Us, _, _ = oracle.slice_propagators(p.H0, p.Hc, p.u, p.dt)
    psis = oracle.forward_states(Us, p.psi0)
    lams = oracle.backward_costates(Us, p.chi)
    g, _ = oracle.state_overlap(p.chi, psis[-1])
    assert np.max(np.abs(np.linalg.norm(psis, axis=1) - 1)) < 1e-13
    assert np.max(np.abs(np.linalg.norm(lams, axis=1) - 1)) < 1e-13
    ov = np.einsum("ka,ka->k", lams.conj(), psis)
    assert np.max(np.abs(ov - g)) < 1e-13


@pytest.mark.parametrize("d,m,N", [(4, 2, 9), (16, 3, 12)])
def test_basis_state_transfers_sum_to_the_unitary_trace(d, m, N):
    """psi0 = e_a, chi = V e_a: sum_a g_a = Tr(V^dag X_N) and
    (2/d^2) Re(conj(sum_a g_a) sum_a dg_a) = the unitary oracle's dF/du."""
    p = make_random(7, d, m, N, 0.05)
    G, DG = 0.0, 0.0
    for a in range(d):
        g, dg, _ = oracle.state_dg(p.H0, p.Hc, p.u, p.dt, basis_state(d, a), p.V[:, a])
        G, DG = G + g, DG + dg
    ref = oracle.grape_ref(p)
    assert abs(G - ref["g"]) < 1e-12
    grad = 2.0 / d ** 2 * (np.conj(G) * DG).real
    assert np.max(np.abs(grad - ref["grad"])) < 1e-13 * max(1.0, np.max(np.abs(ref["grad"])) * 1e3)


@pytest.mark.parametrize("seed,d,m,N,dt", [(3, 3, 2, 11, 0.1), (4, 8, 3, 14, 0.05), (5, 16, 2, 9, 0.08)])
def test_gradient_matches_central_differences(seed, d, m, N, dt):
    """Central differences of F (h = 1e-6) on every entry."""
    p = make_state_random(seed, d, m, N, dt)
    r = oracle.state_ref(p)
    h = 1e-6
    gmax = np.max(np.abs(r["grad"]))
    for j in range(m):
        for k in range(N):
            up, dn = p.u.copy(), p.u.copy()
            up[j, k] += h
            dn[j, k] -= h
            fd = (oracle.state_ref(p.with_u(up))["F"] - oracle.state_ref(p.with_u(dn))["F"]) / (2 * h)
            assert abs(fd - r["grad"][j, k]) < 1e-7 * max(gmax, 1e-3), (j, k)


def test_stationary_point_at_the_reached_state():
    """chi = psi_N(u): F = 1 and every derivative vanishes (F is at its maximum)."""
    p = make_state_random(6, 12, 3, 25, 0.05)
    psiN = oracle.state_ref(p)["psiN"]
    r = oracle.state_ref(p.with_target(psiN))
    assert abs(r["F"] - 1.0) < 1e-13
    assert np.max(np.abs(r["grad"])) < 1e-13


def test_global_phase_of_the_target_does_not_matter():
    p = make_state(2, N=40)
    r0 = oracle.state_ref(p)
    r1 = oracle.state_ref(p.with_target(np.exp(0.73j) * p.chi))
    assert abs(r0["F"] - r1["F"]) < 1e-15
    assert np.max(np.abs(r0["grad"] - r1["grad"])) < 1e-15
