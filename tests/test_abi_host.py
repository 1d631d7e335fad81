"""CPU tests of the C ABI: the library loads, exports every declared symbol,
rejects bad arguments before touching a device, and its per-slice plan obeys
the Taylor remainder bounds it states.  No GPU work is launched here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2208_12187_amd import qoc
from workloads import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "qoc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qoc_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    L = qoc.lib()
    declared = _declared_functions()
    assert set(declared) == set(qoc.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_version_and_defaults():
    assert "libqoc" in qoc.version()
    o = qoc.options()
    assert o.precision == qoc.FP64 and o.chunk == 0 and o.reunitarise_tol == 0.0 and not o.diagnostics
    assert o.dense_controls == 0 and qoc.options(dense_controls=True).dense_controls == 1


def _err(fn, *a):
    with pytest.raises(qoc.QocError) as e:
        fn(*a)
    return e.value.code


def test_argument_errors_before_any_launch():
    p = make_config(2, N=10)
    assert _err(qoc.gradient, p.H0, p.Hc, p.u, 0.0, p.V) == -1          # dt <= 0
    assert _err(qoc.gradient, p.H0, p.Hc, p.u, -1.0, p.V) == -1
    assert _err(qoc.gradient, p.H0, p.Hc, p.u, float("nan"), p.V) == -1
    big = np.eye(129, dtype=complex)
    assert _err(qoc.gradient, big, big[None], np.zeros((1, 3)), 0.1, big) == -6   # d > 128
    bad = p.Hc.copy()
    bad[3, 0, 1] += 0.5                                                   # not Hermitian
    assert _err(qoc.gradient, p.H0, bad, p.u, p.dt, p.V, "fp64", True) == -2
    u = p.u.copy()
    u[2, 5] = np.inf
    assert _err(qoc.gradient, p.H0, p.Hc, u, p.dt, p.V, "fp64", True) == -3
    assert _err(qoc.gradient, p.H0, p.Hc, p.u, p.dt, p.V, 7) == -6      # unknown precision
    assert _err(qoc.gradient, p.H0, p.Hc, p.u, p.dt, 1.001 * p.V, "fp64", True) == -7   # V not unitary
    Vp = p.V.copy()
    Vp[:, [0, 1]] = Vp[:, [1, 0]]                                        # still unitary: passes the check
    assert _err(qoc.gradient, p.H0, bad, p.u, p.dt, Vp, "fp64", True) == -2
    assert _err(qoc.gradient, p.H0, p.Hc, p.u[:, :0], p.dt, p.V) == -1   # no slices
    assert _err(qoc.gradient, p.H0, p.Hc[:0], p.u[:0], p.dt, p.V) == -1  # no controls
    assert _err(qoc.fidelity, p.H0, p.Hc, p.u[:, :0], p.dt, p.V) == -1
    L = qoc.lib()
    assert L.qoc_workspace_size(0, 16, 1, 1, 0, 0, 0) == 0
    assert L.qoc_workspace_size(1, 16, 0, 1, 0, 0, 0) == 0
    assert L.qoc_workspace_size(1, 16, 1, 1, 5, 0, 0) == 0


def test_default_chunk():
    # ceil(sqrt(N / 2)) for d <= 64, ceil(sqrt(N)) for d = 128
    assert qoc.default_chunk(64, 2000) == 32 and qoc.default_chunk(16, 1000) == 23
    assert qoc.default_chunk(2, 1) == 1 and qoc.default_chunk(5, 3) == 2
    assert qoc.default_chunk(128, 1000) == 32 and qoc.default_chunk(100, 2000) == 45
    L = qoc.lib()
    assert L.qoc_default_chunk(0, 10) == 0 and L.qoc_default_chunk(129, 10) == 0 and L.qoc_default_chunk(8, 0) == 0
    # the serving engine's latency chunk: ceil(sqrt(N / 8)), shorter than the default
    assert qoc.engine_chunk(64, 2000) == 16 and qoc.engine_chunk(128, 1000) == 12 and qoc.engine_chunk(2, 1) == 1
    assert all(qoc.engine_chunk(d, N) <= qoc.default_chunk(d, N) for d in (2, 16, 64, 128) for N in (1, 7, 100, 2000))
    assert L.qoc_engine_chunk(0, 10) == 0 and L.qoc_engine_chunk(129, 10) == 0 and L.qoc_engine_chunk(8, 0) == 0


def test_workspace_size_scales_with_batch_and_precision():
    a = qoc.workspace_size(1, 64, 12, 2000, "fp64")
    b = qoc.workspace_size(4, 64, 12, 2000, "fp64")
    c = qoc.workspace_size(1, 64, 12, 2000, "fp32")
    assert 3.9 * a < b < 4.1 * a
    # four per-slice arrays of N complex D x D matrices dominate; FP32 keeps a
    # fifth, X^2 for the adjoint, at half the element size
    assert 0.55 * a < c < 0.7 * a
    assert a > 4 * 2000 * 64 * 64 * 16 and c > 5 * 2000 * 64 * 64 * 8


def _remainder(r, q):
    return r ** (q + 1) / math.factorial(q + 1) / (1 - r / (q + 2))


def _block_remainder(r, qb):
    return r ** qb / math.factorial(qb) / (1 - r / (qb + 1))


@pytest.mark.parametrize("cfg,prec", [(2, "fp64"), (3, "fp64"), (3, "fp32"), (4, "fp32"), (1, "fp64")])
def test_slice_plan_meets_the_taylor_bounds(cfg, prec):
    p = make_config(cfg, N=50)
    plan = qoc.slice_plan(p.H0, p.Hc, p.u, p.dt, prec, True)
    ur = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    n1 = lambda H: np.abs(H).sum(axis=0).max()
    for k in range(p.N):
        th = p.dt * (n1(p.H0) + sum(abs(p.u[j, k]) * n1(p.Hc[j]) for j in range(p.m)))
        s, q, qb = plan[k]
        r = th / 2 ** s
        assert r <= 1.0 + 1e-15
        assert _remainder(r, q) <= ur * (1 + 1e-12)
        assert q == 1 or _remainder(r, q - 1) > ur
        assert _block_remainder(r, qb) <= ur * (1 + 1e-12)
        assert qb == 2 or _block_remainder(r, qb - 1) > ur


def test_slice_plan_prefers_fewer_products():
    # a large theta forces squaring; the chosen s minimises the product count
    p = make_config(2, N=4)
    plan = qoc.slice_plan(p.H0, p.Hc, 40 * p.u, 20 * p.dt, "fp64", True)
    assert (plan[:, 0] > 0).all()


def test_engine_footprint_tracks_the_stored_propagators():
    """About 4 N D^2 c bytes of per-slice arrays (three stored propagators and
    the slice Hamiltonians kept for the adjoint; 5 N D^2 c in FP32, which
    also keeps X^2) dominate a request at D >= 32, 3 N D^2 c at D = 16."""
    L = qoc.lib()
    for prec, c, n in (("fp32", 8, 5), ("fp64", 16, 4)):
        f = qoc.Engine.footprint(prec, 64, 12, 2000)
        core = n * 2000 * 64 * 64 * c
        assert core < f < 1.2 * core
        assert qoc.Engine.footprint(prec, 64, 12, 1000) < f
        # d = 3 is padded to 16: same stored propagators, smaller inputs
        assert 3 * 100 * 16 * 16 * c < qoc.Engine.footprint(prec, 3, 6, 100) < qoc.Engine.footprint(prec, 16, 6, 100)
        assert qoc.Engine.footprint(prec, 16, 6, 100) < 1.3 * 3 * 100 * 16 * 16 * c + (1 << 20)
        f128 = qoc.Engine.footprint(prec, 128, 14, 1000)
        assert n * 1000 * 128 * 128 * c < f128 < 1.2 * n * 1000 * 128 * 128 * c
    assert L.qoc_engine_footprint(1, 0, 1, 1) == 0
    assert L.qoc_engine_footprint(1, 129, 1, 1) == 0


def test_noalloc_rejects_oversized_call_before_any_launch():
    """The no-allocation entry point refuses a call whose workspace exceeds its
    static scratch, before it looks up the scratch or touches a device."""
    L = qoc.lib()
    need = qoc.workspace_size(1, 64, 12, 2000, "fp32")
    assert need > qoc.NOALLOC_SCRATCH_BYTES
    o = qoc.options("fp32")
    rc = L.qoc_gradient_dev_noalloc(1, 64, 12, 2000, None, None, None, 0.002, None, None, None, ctypes.byref(o))
    assert rc == -1
    assert "static scratch" in L.qoc_last_error().decode()
    assert qoc.workspace_size(2, 16, 8, 1000, "fp64") <= qoc.NOALLOC_SCRATCH_BYTES
