"""GPU parity of open-system (Lindblad) GRAPE, the general-generator path of
libqoc, against the Lindblad oracle (Liouvillian built column by column,
scipy expm and expm_frechet): open spin chains of 1, 2 and 3 qubits (Liouville
dimension 4, 16 and 64) in FP64 and FP32; random non-normal generators in
every padding class (the adjoint's conjugate transposes at D = 16, 32, 64 and
128); the closed-system limit F = F_unitary^2 against the Hermitian path; and
checkpointed recomputation bit for bit.  Tolerances as for the unitary path."""
import numpy as np
import pytest

import oracle
from oracle import lindblad as LB
from workloads import make_lindblad, make_random

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-10, True), "fp32": (1e-5, 1e-4, False)}


def _check(F, g, ref, prec, label):
    ftol, gtol, rel = TOL[prec]
    assert abs(F - ref["F"]) <= (ftol * ref["F"] if rel else ftol), (label, F, ref["F"])
    gmax = np.max(np.abs(ref["grad"]))
    assert np.max(np.abs(g - ref["grad"])) <= gtol * gmax, (label, np.max(np.abs(g - ref["grad"])) / gmax)


@pytest.mark.parametrize("nq,N", [(1, 60), (2, 200), (3, 40)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_open_spin_chain_matches_oracle(gpu_lib, nq, N, prec):
    from paper_2208_12187_amd import lindblad

    p = make_lindblad(nq, N, dt=0.02, gamma_damp=0.05, gamma_deph=0.02, seed=1)
    print(f"[lindblad] {nq} qubits, N = {N}, {prec}", flush=True)
    ref = LB.lindblad_ref(p)
    F, g = lindblad.gradient(p, prec)
    _check(F, g, ref, prec, (nq, N, prec))
    XN = lindblad.propagate(p, prec)
    assert np.max(np.abs(XN - ref["XN"])) <= (1e-10 if prec == "fp64" else 1e-5)


def _nonnormal(seed, D, m, N, dt):
    rng = np.random.default_rng(seed)
    G = lambda: (rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))) / np.sqrt(D)
    G0 = G()
    Gc = np.stack([G() for _ in range(m)])
    u = rng.normal(0, 0.5, (m, N))
    T = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    return G0, Gc, u, dt, T


@pytest.mark.parametrize("D,prec", [(5, "fp64"), (16, "fp32"), (27, "fp64"), (64, "fp64"), (100, "fp64"),
                                    (120, "fp32"), (48, "fp32")])
def test_nonnormal_generators_match_oracle(gpu_lib, D, prec):
    from paper_2208_12187_amd import qoc

    G0, Gc, u, dt, T = _nonnormal(500 + D, D, 3, 9, 0.08)
    print(f"[lindblad] non-normal generators D = {D}, {prec}", flush=True)
    F_ref, g_ref, grad_ref, XN_ref = LB.generator_gradient(G0, Gc, u, dt, T)
    F, g = qoc.gradient(G0, Gc, u, dt, T, prec, generators=True)
    _check(F, g, {"F": F_ref, "grad": grad_ref}, prec, D)


def test_closed_system_limit_against_the_hermitian_path(gpu_lib):
    from paper_2208_12187_amd import lindblad, qoc

    p = make_lindblad(3, 80, dt=0.02, gamma_damp=0.0, gamma_deph=0.0, seed=2)
    F_u, g_u = qoc.gradient(p.H0, p.Hc, p.u, p.dt, p.V, "fp64")
    F_l, g_l = lindblad.gradient(p, "fp64")
    assert abs(F_l - F_u ** 2) <= 1e-10 * F_l
    assert np.max(np.abs(g_l - 2 * F_u * g_u)) <= 1e-10 * np.max(np.abs(g_l))


def test_checkpointed_generators_are_bitwise_identical(gpu_lib):
    from paper_2208_12187_amd import lindblad, qoc

    p = make_lindblad(3, 120, dt=0.02, seed=3)
    F0, g0 = lindblad.gradient(p, "fp64")
    full = qoc.workspace_size(1, 64, p.m, p.N, "fp64")
    F1, g1 = lindblad.gradient(p, "fp64", hbm_budget=full // 3)
    assert F0 == F1 and np.array_equal(g0, g1)
