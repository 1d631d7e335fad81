"""GPU parity of the state-to-state path (qoc_state_*) against the FP64 state
oracle: seeded random problems of every padding class (dense controls and
controls with one nonzero per row), the single-qubit closed form, slices long
enough to need scaling and squaring (R = 2^s sub-steps), the batched device
entry point at the configuration-3 size (d = 64, m = 12, N = 2000) in both
precisions, and bitwise agreement of a batch member with the same problem run
alone.  Tolerances: FP64 |F - F_ref| <= 1e-10 F_ref and
max|grad - ref| <= 1e-10 max|ref|; FP32 |F - F_ref| <= 1e-5 and
max|grad - ref| <= 1e-4 max|ref|."""
import numpy as np
import pytest

import oracle
from workloads import StateProblem, basis_state, make_state, make_state_batch, make_state_random, pauli

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-10, True), "fp32": (1e-5, 1e-4, False)}


def _check(F, g, ref, prec, label):
    ftol, gtol, rel = TOL[prec]
    assert abs(F - ref["F"]) <= (ftol * ref["F"] if rel else ftol), (label, F, ref["F"])
    gmax = np.max(np.abs(ref["grad"]))
    err = np.max(np.abs(g - ref["grad"]))
    assert err <= gtol * gmax, (label, err / gmax)


def test_single_qubit_closed_form(gpu_lib):
    from paper_2208_12187_amd import qoc

    omega, u, N, dt = 1.0, 0.7, 100, 0.01
    SX, SZ = pauli("x"), pauli("z")
    p = StateProblem(0.5 * omega * SZ, SX[None], np.full((1, N), u), dt, basis_state(2, 0), basis_state(2, 1))
    T, b = N * dt, np.sqrt(u * u + omega * omega / 4)
    psiN = qoc.state_propagate(p.H0, p.Hc, p.u, p.dt, p.psi0, "fp64")
    ref = np.array([np.cos(b * T) - 0.5j * omega * np.sin(b * T) / b, -1j * u * np.sin(b * T) / b])
    assert np.max(np.abs(psiN - ref)) < 1e-13
    F, g = qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, "fp64")
    assert abs(F - u * u * np.sin(b * T) ** 2 / b ** 2) < 1e-13
    _check(F, g, oracle.state_ref(p), "fp64", "closed form")


def _cases():
    out = []
    dims = [2, 3, 7, 16, 17, 29, 32, 40, 64, 65, 100, 128]
    rng = np.random.default_rng(77)
    for i, d in enumerate(dims):
        m = int(rng.integers(1, 6))
        N = int(rng.integers(1, 25 if d > 64 else 40))
        out.append((i, d, m, N, bool(i % 2), "fp64" if i % 3 != 2 else "fp32"))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}_d{c[1]}_m{c[2]}_N{c[3]}_{'mono' if c[4] else 'dense'}_{c[5]}")
def test_random_state_problem_matches_oracle(gpu_lib, case):
    from paper_2208_12187_amd import qoc

    i, d, m, N, mono, prec = case
    p = make_state_random(200 + i, d, m, N, 0.04, monomial=mono)
    print(f"[state] case {i}: d={d} m={m} N={N} {'mono' if mono else 'dense'} {prec}", flush=True)
    ref = oracle.state_ref(p)
    F, g = qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, prec, validate=True)
    _check(F, g, ref, prec, case)
    psiN = qoc.state_propagate(p.H0, p.Hc, p.u, p.dt, p.psi0, prec)
    assert np.max(np.abs(psiN - ref["psiN"])) <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("d,mono", [(5, False), (16, True), (64, True), (100, False)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_slices_take_scaled_substeps(gpu_lib, d, mono, prec):
    """dt large enough that theta_k > 1: the plan scales by 2^s and every slice
    is applied (and differentiated) as 2^s sub-steps."""
    from paper_2208_12187_amd import qoc

    p = make_state_random(300 + d, d, 3, 6, 0.9, monomial=mono)
    plan = qoc.slice_plan(p.H0, p.Hc, p.u, p.dt, prec)
    assert plan[:, 0].max() >= 1
    print(f"[state] long slices d={d} {prec}: s = {sorted(set(plan[:, 0].tolist()))}", flush=True)
    ref = oracle.state_ref(p)
    F, g = qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, prec)
    _check(F, g, ref, prec, (d, prec))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config3_state_transfer_at_full_size(gpu_lib, prec):
    """The state-transfer workload of configuration 3 (d = 64, m = 12,
    N = 2000): a batch of 8 through the device entry point, two members
    against the oracle in full, every member against 0 <= F <= 1 and the bound
    |dF/du_jk| <= 2 sqrt(F) dt ||Hc[j]||_2, and one member alone bit for bit."""
    import torch
    from paper_2208_12187_amd import qoc

    probs = make_state_batch(3, 8)
    p0 = probs[0]
    assert (p0.d, p0.m, p0.N) == (64, 12, 2000)
    print(f"[state] configuration 3, batch 8, {prec}", flush=True)
    r = qoc.StateRunner(8, 64, 12, 2000, prec)
    F, g = r.gradient(qoc.StateBatch.from_problems(probs))
    torch.cuda.synchronize()
    F, g = F.cpu().numpy(), g.cpu().numpy()
    norms = np.array([np.linalg.norm(h, 2) for h in p0.Hc])
    for b in range(8):
        assert 0.0 <= F[b] <= 1.0
        bound = 2 * np.sqrt(F[b]) * p0.dt * norms[:, None]
        assert np.all(np.abs(g[b]) <= bound * (1 + 1e-6) + 1e-14)
    for b in (0, 5):
        _check(F[b], g[b], oracle.state_ref(probs[b]), prec, b)
    one = qoc.StateRunner(1, 64, 12, 2000, prec)
    F1, g1 = one.gradient(qoc.StateBatch.from_problems(probs[5:6]))
    torch.cuda.synchronize()
    assert F1.cpu().numpy()[0] == F[5]
    assert np.array_equal(g1.cpu().numpy()[0], g[5])


def test_dense_and_row_table_paths_agree(gpu_lib):
    """The spin-chain controls (Pauli strings) take the row tables by default;
    forcing the dense kernels gives the same result to rounding."""
    from paper_2208_12187_amd import qoc

    p = make_state(2, N=300)
    F1, g1 = qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, "fp64")
    F2, g2 = qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, "fp64", dense_controls=True)
    assert abs(F1 - F2) <= 1e-12 * F1
    assert np.max(np.abs(g1 - g2)) <= 1e-11 * np.max(np.abs(g1))


def test_state_argument_errors(gpu_lib):
    from paper_2208_12187_amd import qoc

    p = make_state_random(9, 8, 2, 10, 0.05)
    with pytest.raises(qoc.QocError) as e:
        qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, p.psi0, p.chi, "bf16x3")
    assert e.value.code == -6
    with pytest.raises(qoc.QocError) as e:
        qoc.state_gradient(p.H0, p.Hc, p.u, p.dt, 2 * p.psi0, p.chi, "fp64", validate=True)
    assert e.value.code == -7
