"""The seeded input generators: shapes, Hermiticity, unitarity of targets and
determinism (every consumer must see the same problem)."""
import numpy as np

from workloads import make_config, make_random, make_random_monomial, make_request, poisson_trace


def _check(p):
    d, m, N = p.d, p.m, p.N
    assert p.H0.shape == (d, d) and p.Hc.shape == (m, d, d) and p.u.shape == (m, N) and p.V.shape == (d, d)
    assert np.allclose(p.H0, p.H0.conj().T, atol=0, rtol=0)
    for H in p.Hc:
        assert np.array_equal(H, H.conj().T)
    assert np.max(np.abs(p.V.conj().T @ p.V - np.eye(d))) < 1e-12


def test_generators_are_hermitian_unitary_and_deterministic():
    for p, q in ((make_random(3, 29, 3, 11, 0.02), make_random(3, 29, 3, 11, 0.02)),
                 (make_config(3, copy=2, N=50), make_config(3, copy=2, N=50)),
                 (make_request(7, 16, 40, trace_seed=5), make_request(7, 16, 40, trace_seed=5))):
        _check(p)
        assert np.array_equal(p.H0, q.H0) and np.array_equal(p.Hc, q.Hc)
        assert np.array_equal(p.u, q.u) and np.array_equal(p.V, q.V)
    assert not np.array_equal(make_random(3, 29, 3, 11, 0.02).u, make_random(4, 29, 3, 11, 0.02).u)


def test_monomial_controls_have_one_nonzero_per_row_at_most():
    for d in (1, 2, 5, 16, 33, 64):
        p = make_random_monomial(2, d, 4, 10, 0.05)
        q = make_random_monomial(2, d, 4, 10, 0.05)
        _check(p)
        assert np.array_equal(p.Hc, q.Hc) and np.array_equal(p.u, q.u)
        for H in p.Hc:
            assert np.all(np.count_nonzero(H, axis=1) <= 1)
            assert np.all(np.count_nonzero(H, axis=0) <= 1)
    # every kind of row occurs: paired, diagonal and empty
    H = np.concatenate(list(make_random_monomial(2, 64, 4, 10, 0.05).Hc))
    nz = np.count_nonzero(H, axis=1)
    assert (nz == 0).any() and (nz == 1).any()
    assert any(np.count_nonzero(np.diag(h)) > 0 for h in make_random_monomial(2, 64, 4, 10, 0.05).Hc)


def test_poisson_trace_shapes_do_not_depend_on_the_rate():
    a = poisson_trace(200, rate=100.0, seed=5)
    b = poisson_trace(200, rate=0.0, seed=5)
    assert [(x["d"], x["N"]) for x in a] == [(x["d"], x["N"]) for x in b]
    t = np.array([x["t_arrival"] for x in a])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert all(x["t_arrival"] == 0.0 for x in b)
