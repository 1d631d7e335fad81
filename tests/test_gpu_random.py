"""Randomised parity: seeded random problems of every padding class, dense
random Hermitian controls, random chunk lengths and HBM budgets, FP64 and
FP32, each compared element by element with the oracle.  The case list is
drawn once from a fixed seed, so the test is deterministic."""
import numpy as np
import pytest

import oracle
from workloads import make_random

pytestmark = pytest.mark.gpu


def _cases(n=14, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    dims = [2, 3, 7, 16, 17, 29, 32, 40, 53, 64, 65, 90, 128]
    for i in range(n):
        d = int(dims[i % len(dims)]) if i < len(dims) else int(rng.integers(2, 65))
        big = d > 64
        m = int(rng.integers(1, 5))
        N = int(rng.integers(1, 12 if big else 40))
        dt = float(rng.uniform(0.002, 0.06 if big else 0.1))
        prec = "fp64" if i % 2 == 0 else "fp32"
        chunk = int(rng.integers(1, N + 1)) if rng.random() < 0.5 else 0
        out.append((i, d, m, N, dt, prec, chunk))
    return out


def _budget(qoc, d, m, N, prec, chunk):
    # a budget that forces one-chunk segments when the problem has several chunks
    full = qoc.workspace_size(1, d, m, N, prec, chunk)
    return full // 3


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}_d{c[1]}_m{c[2]}_N{c[3]}_{c[5]}_L{c[6]}")
def test_random_problem_matches_oracle(gpu_lib, case):
    from paper_2208_12187_amd import qoc

    i, d, m, N, dt, prec, chunk = case
    p = make_random(100 + i, d, m, N, dt)
    print(f"[random] case {i}: d={d} m={m} N={N} dt={dt:.4f} {prec} chunk={chunk}", flush=True)
    ref = oracle.grape_ref(p)
    budget = _budget(qoc, d, m, N, prec, chunk) if i % 3 == 1 else 0
    F, g = qoc.gradient(p.H0, p.Hc, p.u, p.dt, p.V, prec, chunk=chunk, hbm_budget=budget)
    gmax = max(np.max(np.abs(ref["grad"])), 1e-300)
    if prec == "fp64":
        assert abs(F - ref["F"]) <= 1e-10 * ref["F"]
        assert np.max(np.abs(g - ref["grad"])) <= 1e-10 * gmax
    else:
        assert abs(F - ref["F"]) <= 1e-5
        assert np.max(np.abs(g - ref["grad"])) <= 1e-4 * gmax
    XN = qoc.propagate(p.H0, p.Hc, p.u, p.dt, prec, chunk=chunk)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert np.max(np.abs(XN - ref["XN"])) <= tol
