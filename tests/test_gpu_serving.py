"""GPU tests of the continuous-batching engine: every request's result in a
mixed batch equals its result alone and the host entry point's, admission
works under a small pool, oversize requests are rejected, and FP64 results
match the oracle."""
import numpy as np
import pytest

import oracle
from workloads import make_request

pytestmark = pytest.mark.gpu

MIX = [(2, 150), (4, 333), (8, 90), (16, 400), (32, 123), (64, 257), (128, 61), (16, 777), (64, 31), (8, 1)]


def _requests():
    return [make_request(i, d, N, trace_seed=9) for i, (d, N) in enumerate(MIX)]


def _run(eng, probs):
    ids = {eng.submit(p.H0, p.Hc, p.u, p.dt, p.V): i for i, p in enumerate(probs)}
    out = {}
    while len(out) < len(probs):
        eng.step(wait=True)
        for rid, F in eng.poll():
            out[ids[rid]] = (F, eng.fetch(rid))
    return [out[i] for i in range(len(probs))]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_engine_mix_equals_alone_and_api(gpu_lib, prec):
    from paper_2208_12187_amd import qoc

    probs = _requests()
    print(f"[serving] mix of {len(probs)} requests, {prec}", flush=True)
    eng = qoc.Engine(prec, pool_bytes=8 << 30, host_bytes=1 << 30, max_active=64)
    mix = _run(eng, probs)
    eng.close()
    one = qoc.Engine(prec, pool_bytes=8 << 30, host_bytes=1 << 30, max_active=1)
    alone = _run(one, probs)
    one.close()
    for i, p in enumerate(probs):
        F_api, g_api = qoc.gradient(p.H0, p.Hc, p.u, p.dt, p.V, prec, chunk=qoc.engine_chunk(p.d, p.N))
        assert mix[i][0] == alone[i][0] == F_api, (i, mix[i][0], alone[i][0], F_api)
        assert np.array_equal(mix[i][1], alone[i][1])
        assert np.array_equal(mix[i][1], g_api)


def test_split_bf16_engine(gpu_lib):
    """A split-BF16 engine serves 17 <= d <= 64 (other d are refused at
    submit) and gives the host entry point's results bit for bit, within the
    gates of the oracle."""
    from paper_2208_12187_amd import qoc

    probs = [make_request(i, d, N, trace_seed=17) for i, (d, N) in enumerate([(32, 210), (64, 95), (32, 17)])]
    eng = qoc.Engine("bf16x3", pool_bytes=4 << 30, host_bytes=1 << 28, max_active=8)
    small = make_request(9, 16, 30, trace_seed=17)
    with pytest.raises(qoc.QocError) as e:
        eng.submit(small.H0, small.Hc, small.u, small.dt, small.V)
    assert e.value.code == -6
    res = _run(eng, probs)
    eng.close()
    for (F, g), p in zip(res, probs):
        F_api, g_api = qoc.gradient(p.H0, p.Hc, p.u, p.dt, p.V, "bf16x3", chunk=qoc.engine_chunk(p.d, p.N))
        assert F == F_api and np.array_equal(g, g_api)
        ref = oracle.grape_ref(p)
        assert abs(F - ref["F"]) <= 1e-5
        assert np.max(np.abs(g - ref["grad"])) <= 1e-4 * np.max(np.abs(ref["grad"]))


def test_engine_fp64_matches_oracle(gpu_lib):
    from paper_2208_12187_amd import qoc

    probs = [make_request(i, d, N, trace_seed=11) for i, (d, N) in enumerate([(2, 40), (8, 60), (32, 30)])]
    eng = qoc.Engine("fp64", pool_bytes=1 << 30, host_bytes=1 << 28, max_active=8)
    res = _run(eng, probs)
    eng.close()
    for (F, g), p in zip(res, probs):
        ref = oracle.grape_ref(p)
        assert abs(F - ref["F"]) <= 1e-10 * ref["F"]
        assert np.max(np.abs(g - ref["grad"])) <= 1e-10 * np.max(np.abs(ref["grad"]))


def test_engine_admission_with_a_small_pool(gpu_lib):
    """A pool that holds only the largest request admits the rest in FIFO
    order as memory frees up; every request still completes correctly."""
    from paper_2208_12187_amd import qoc

    probs = _requests()
    need = max(qoc.Engine.footprint("fp32", p.d, p.m, p.N) for p in probs)
    eng = qoc.Engine("fp32", pool_bytes=need + (1 << 20), host_bytes=1 << 30, max_active=64)
    res = _run(eng, probs)
    eng.close()
    for (F, g), p in zip(res, probs):
        F_api, g_api = qoc.gradient(p.H0, p.Hc, p.u, p.dt, p.V, "fp32", chunk=qoc.engine_chunk(p.d, p.N))
        assert F == F_api and np.array_equal(g, g_api)


def test_engine_rejects_a_request_larger_than_the_pool(gpu_lib):
    from paper_2208_12187_amd import qoc

    p = make_request(0, 64, 2000, trace_seed=3)
    eng = qoc.Engine("fp32", pool_bytes=64 << 20, host_bytes=1 << 28, max_active=4)
    with pytest.raises(qoc.QocError) as e:
        eng.submit(p.H0, p.Hc, p.u, p.dt, p.V)
    assert e.value.code == -4
    eng.close()


def test_engine_rejects_empty_and_oversized_requests(gpu_lib):
    from paper_2208_12187_amd import qoc

    p = make_request(0, 8, 20, trace_seed=3)
    eng = qoc.Engine("fp32", pool_bytes=64 << 20, host_bytes=1 << 26, max_active=4)
    for args, code in (((p.H0, p.Hc, p.u[:, :0], p.dt, p.V), -1),          # no slices
                       ((p.H0, p.Hc[:0], p.u[:0], p.dt, p.V), -1),         # no controls
                       ((p.H0, p.Hc, p.u, 0.0, p.V), -1),                  # dt <= 0
                       ((np.eye(129, dtype=complex), np.eye(129, dtype=complex)[None], np.zeros((1, 4)), 0.1,
                         np.eye(129, dtype=complex)), -6)):                  # d > 128
        with pytest.raises(qoc.QocError) as e:
            eng.submit(*args)
        assert e.value.code == code
    # the engine still serves a valid request afterwards
    rid = eng.submit(p.H0, p.Hc, p.u, p.dt, p.V)
    got = []
    while not got:
        eng.step(wait=True)
        got = eng.poll()
    assert got[0][0] == rid and 0 <= got[0][1] <= 1
    eng.close()


def test_engine_poisson_replay_reports_latency(gpu_lib):
    from paper_2208_12187_amd import serve

    probs = [make_request(i, d, N, trace_seed=13) for i, (d, N) in enumerate(MIX * 3)]
    arr = serve.poisson_arrivals(len(probs), rate=400.0, seed=13)
    res = serve.replay(probs, arr, "fp32", max_active=32, pool_bytes=8 << 30, host_bytes=1 << 30)
    s = serve.summary(res)
    print(f"[serving] replay: {s}", flush=True)
    assert s["p50_ms"] > 0 and s["p99_ms"] >= s["p50_ms"]
    assert np.all(res["latency"] > 0)
    by_d = serve.per_d(res, probs)
    assert sum(v["requests"] for v in by_d.values()) == len(probs)
    assert sum(v["slice_steps"] for v in by_d.values()) == sum(p.N for p in probs)
