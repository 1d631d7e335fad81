"""Parity at the benchmark's full size and in its launch configuration:
configuration 3 (6-qubit Ising chain, d = 64, m = 12, N = 2000, dt = 0.002),
a batch of 32 seeded problems through one Runner, called repeatedly on one
workspace as the benchmark times it.

The oracle takes a few seconds per problem at this size, so three members of
the batch are checked in full (F and all m N gradient entries).  Every member
is checked against properties that hold at any size: 0 <= F <= 1, and
|dF/du_jk| <= 2 sqrt(F) dt ||Hc[j]||_2 (the derivative of Tr(V^dag X_N) in
u_jk is a trace of d x d matrices of 2-norm at most dt ||Hc[j]||_2, since the
Frechet derivative of the exponential of a skew-Hermitian matrix does not
increase the 2-norm).  A member run alone gives the same bits as in the
batch.

Configuration 4 (7-qubit Heisenberg chain, d = 128, m = 14, N = 1000) is
checked the same way at its benchmark batch of 8, with one member against
the oracle.

The gradient gate (1e-4 of max|grad|) is met by every precision on the
sampled members, member 31 among them: its gradient is small (max|grad| =
2.5e-8), so an absolute error in Tr(V^dag X_N) shows there first.  The
default Newton-Schulz step on every chunk product and FP32 forward chains
for the split-BF16 precision keep that error down (measured 7.5e-6 FP32 and
1.6e-5 split BF16 of max|grad| over all 32 members)."""
import numpy as np
import pytest

import oracle
from workloads import make_batch

pytestmark = pytest.mark.gpu

B = 32
SAMPLED = (0, 13, 31)
TOL = {"fp64": (1e-10, 1e-10, True), "fp32": (1e-5, 1e-4, False), "bf16x3": (1e-5, 1e-4, False)}


@pytest.fixture(scope="module")
def problems():
    return make_batch(3, B)


@pytest.fixture(scope="module")
def refs(problems):
    out = {}
    for i in SAMPLED:
        print(f"[fullsize] oracle, problem {i} ...", flush=True)
        out[i] = oracle.grape_ref(problems[i])
    return out


def _run_batch(problems, prec):
    import torch
    from paper_2208_12187_amd import qoc

    p, nb = problems[0], len(problems)
    print(f"[fullsize] d = {p.d}, N = {p.N}, batch {nb}, {prec}", flush=True)
    batch = qoc.Batch.from_problems(problems)
    runner = qoc.Runner(nb, p.d, p.m, p.N, prec)
    F = torch.empty(nb, dtype=torch.float64, device="cuda")
    grad = torch.empty((nb, p.m, p.N), dtype=torch.float64, device="cuda")
    runner.gradient(batch, F, grad)
    F1, g1 = F.clone(), grad.clone()
    runner.gradient(batch, F, grad)  # the same workspace again
    torch.cuda.synchronize()
    assert torch.equal(F, F1) and torch.equal(grad, g1)
    return F.cpu().numpy(), grad.cpu().numpy()


def _properties(problems, Fh, gh):
    assert np.all(np.isfinite(gh))
    for i, q in enumerate(problems):
        assert 0.0 <= Fh[i] <= 1.0
        norms = np.linalg.norm(q.Hc, ord=2, axis=(1, 2))
        bound = 2 * np.sqrt(Fh[i]) * q.dt * norms[:, None] * (1 + 1e-6) + 1e-12
        assert np.all(np.abs(gh[i]) <= bound), i


def _grad_gate(gh, refs, prec):
    gtol = TOL[prec][1]
    for i in refs:
        gmax = np.max(np.abs(refs[i]["grad"]))
        err = np.max(np.abs(gh[i] - refs[i]["grad"]))
        print(f"[fullsize] {prec} problem {i}: grad err {err / gmax:.2e} of max|grad| {gmax:.2e}", flush=True)
        assert err <= gtol * gmax, (i, err / gmax)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_config3_batch_of_32(gpu_lib, problems, refs, prec):
    import torch
    from paper_2208_12187_amd import qoc

    p = problems[0]
    Fh, gh = _run_batch(problems, prec)
    ftol, _, rel = TOL[prec]
    for i in SAMPLED:
        ref = refs[i]
        assert abs(Fh[i] - ref["F"]) <= (ftol * ref["F"] if rel else ftol), (i, Fh[i], ref["F"])
    _grad_gate(gh, refs, prec)

    _properties(problems, Fh, gh)

    i = SAMPLED[1]
    alone = qoc.Runner(1, p.d, p.m, p.N, prec)
    Fa, ga = alone.gradient(qoc.Batch.from_problems([problems[i]]))
    torch.cuda.synchronize()
    assert Fa[0].item() == Fh[i] and np.array_equal(ga[0].cpu().numpy(), gh[i])


B4, SAMPLED4 = 8, 5


@pytest.fixture(scope="module")
def problems4():
    return make_batch(4, B4)


@pytest.fixture(scope="module")
def ref4(problems4):
    print(f"[fullsize] oracle, config 4 problem {SAMPLED4} ...", flush=True)
    return {SAMPLED4: oracle.grape_ref(problems4[SAMPLED4])}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_config4_batch_of_8(gpu_lib, problems4, ref4, prec):
    Fh, gh = _run_batch(problems4, prec)
    ftol, _, rel = TOL[prec]
    ref = ref4[SAMPLED4]
    assert abs(Fh[SAMPLED4] - ref["F"]) <= (ftol * ref["F"] if rel else ftol), (Fh[SAMPLED4], ref["F"])
    _grad_gate(gh, ref4, prec)
    _properties(problems4, Fh, gh)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config2_at_full_size(gpu_lib, prec):
    """Configuration 2 (4-qubit Heisenberg chain, d = 16, m = 8, N = 1000,
    dt = 0.005) at its own size: FP32 rounding accumulates over the whole
    1000-slice chain, so both precisions are gated against the oracle here,
    over a batch of 4 seeded copies through one Runner."""
    import torch
    from paper_2208_12187_amd import qoc

    probs = make_batch(2, 4)
    assert probs[0].N == 1000 and probs[0].d == 16
    print(f"[fullsize] configuration 2, batch 4, {prec}", flush=True)
    batch = qoc.Batch.from_problems(probs)
    runner = qoc.Runner(4, 16, 8, 1000, prec)
    F, grad = runner.gradient(batch)
    torch.cuda.synchronize()
    F, grad = F.cpu().numpy(), grad.cpu().numpy()
    ftol, gtol, rel = TOL[prec]
    for b, p in enumerate(probs):
        ref = oracle.grape_ref(p)
        assert abs(F[b] - ref["F"]) <= (ftol * ref["F"] if rel else ftol), (b, F[b], ref["F"])
        gmax = np.max(np.abs(ref["grad"]))
        err = np.max(np.abs(grad[b] - ref["grad"])) / gmax
        print(f"[fullsize] cfg2 {prec} member {b}: |dF| = {abs(F[b] - ref['F']):.2e}, grad err {err:.2e}",
              flush=True)
        assert err <= gtol, (b, err)
