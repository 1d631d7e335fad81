"""Pins of the trust-region oracle (the paper's Alg. 1-3 and App. B) and of
the GRAPE least-squares residual and Jacobian it drives.

* App. B: the SVD step equals the direct solve of (J^T J + alpha I) p = -J^T r
  (tall and wide J), and the alpha = 0 step of a full-rank tall J is the
  Gauss-Newton step -lstsq(J, r).
* Alg. 2: the returned alpha puts |p| within sigma Delta of Delta.
* Alg. 1 + 3: a linear residual converges to numpy.linalg.lstsq's solution;
  the Rosenbrock residual (10 (x2 - x1^2), 1 - x1) reaches (1, 1) from
  (-1.2, 1); noise-free exponential-decay data return the true parameters.
* GRAPE: every Jacobian column against central differences of the residual,
  the phi column in closed form, and a TRM run on a one-qubit problem that
  reaches F = 1 with f decreasing on every accepted step.
"""
import numpy as np
import pytest

from oracle import trm as T
from workloads import make_config, make_random


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("v,n", [(30, 7), (8, 20)])
def test_svd_step_solves_the_lm_system(v, n):
    J, r = _rand((v, n), 1), _rand(v, 2)
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    for alpha in (1e-3, 0.7, 12.0):
        p = T.svd_step(s, U.T @ r, Vt, alpha)
        ref = -np.linalg.solve(J.T @ J + alpha * np.eye(n), J.T @ r)
        assert np.max(np.abs(p - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))


def test_zero_alpha_step_is_gauss_newton():
    J, r = _rand((25, 6), 3), _rand(25, 4)
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    p = T.svd_step(s, U.T @ r, Vt, 0.0)
    assert np.max(np.abs(p + np.linalg.lstsq(J, r, rcond=None)[0])) < 1e-12


@pytest.mark.parametrize("v,n,full", [(40, 9, True), (10, 30, False)])
def test_lm_parameter_lands_on_the_trust_radius(v, n, full):
    J, r = _rand((v, n), 5), _rand(v, 6)
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    c = U.T @ r
    pt = np.linalg.norm(T.svd_step(s, c, Vt, 0.0))
    for frac in (0.9, 0.3, 0.02):
        Delta = frac * pt
        alpha = T.lm_parameter(s, c, Delta, 0.1, full)
        assert alpha > 0
        assert abs(np.linalg.norm(T.svd_step(s, c, Vt, alpha)) - Delta) <= 0.1 * Delta


def test_linear_residual_converges_to_lstsq():
    A, b = _rand((50, 8), 7), _rand(50, 8)
    x, info = T.trm(lambda x: A @ x - b, lambda x: A, np.zeros(8), Delta0=0.05, max_iter=100)
    assert np.max(np.abs(x - np.linalg.lstsq(A, b, rcond=None)[0])) < 1e-9
    assert all(f1 <= f0 for f0, f1 in zip(info["f"], info["f"][1:]))


def test_rosenbrock_reaches_its_minimum():
    fun = lambda x: np.array([10 * (x[1] - x[0] ** 2), 1 - x[0]])
    jac = lambda x: np.array([[-20 * x[0], 10.0], [-1.0, 0.0]])
    x, info = T.trm(fun, jac, np.array([-1.2, 1.0]), max_iter=200, gtol=1e-14)
    assert np.max(np.abs(x - 1.0)) < 1e-8, (x, info["reason"])


def test_noise_free_exponential_decay_returns_true_parameters():
    y = np.linspace(0, 4, 60)
    true = np.array([2.5, 1.3, -0.4])
    z = true[0] * np.exp(-true[1] * y) + true[2]
    fun = lambda x: x[0] * np.exp(-x[1] * y) + x[2] - z
    jac = lambda x: np.stack([np.exp(-x[1] * y), -x[0] * y * np.exp(-x[1] * y), np.ones_like(y)], axis=1)
    x, _ = T.trm(fun, jac, np.array([1.0, 0.5, 0.0]), max_iter=200, gtol=1e-13)
    assert np.max(np.abs(x - true)) < 1e-8


@pytest.mark.parametrize("d,m,N", [(3, 2, 4), (4, 2, 3)])
def test_grape_jacobian_matches_central_differences(d, m, N):
    p = make_random(11, d, m, N, 0.2)
    phi = 0.37
    J = T.grape_residual_jacobian(p.H0, p.Hc, p.u, p.dt, p.V, phi)
    h = 1e-6
    x = np.concatenate([p.u.ravel(), [phi]])

    def r(x):
        return T.grape_residual(p.H0, p.Hc, x[:-1].reshape(m, N), p.dt, p.V, x[-1])

    for col in range(m * N + 1):
        e = np.zeros_like(x)
        e[col] = h
        fd = (r(x + e) - r(x - e)) / (2 * h)
        assert np.max(np.abs(fd - J[:, col])) < 1e-8, col
    dphi = (-1j * np.exp(1j * phi) * p.V).ravel()
    assert np.max(np.abs(J[:, -1] - np.concatenate([dphi.real, dphi.imag]))) < 1e-15


def test_grape_residual_is_d_minus_sqrt_fidelity_at_the_best_phase():
    """f = d - Re(e^{-i phi} g), = d (1 - sqrt(F)) at phi = arg g."""
    import oracle

    p = make_random(12, 5, 2, 6, 0.1)
    ref = oracle.fidelity_ref(p)
    phi = float(np.angle(ref["g"]))
    r = T.grape_residual(p.H0, p.Hc, p.u, p.dt, p.V, phi)
    assert abs(0.5 * r @ r - p.d * (1 - np.sqrt(ref["F"]))) < 1e-12


def test_grape_trm_reaches_the_target_on_one_qubit():
    import oracle

    p = make_config(1, N=20)
    u, phi, info = T.grape_trm(p, max_iter=60, gtol=1e-12)
    F = oracle.fidelity_ref(p.with_u(u))["F"]
    assert F > 1 - 1e-10, (F, info["reason"])
    assert all(f1 < f0 for f0, f1 in zip(info["f"], info["f"][1:]))


def test_lm_update_is_exact_for_one_singular_value():
    """With a single singular value 1/|p(alpha)| = (s^2 + alpha)/(s |c|) is
    linear in alpha, and the update of Eq. alphaupdate is Newton's method on
    1/|p| - 1/Delta: one update lands exactly on the trust radius."""
    J, r = _rand((12, 1), 8), _rand(12, 9)
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    c = U.T @ r
    pt = np.linalg.norm(T.svd_step(s, c, Vt, 0.0))
    for frac in (0.8, 0.1):
        Delta = frac * pt
        alpha = T.lm_parameter(s, c, Delta, 1e-13, True, max_iter=2)
        assert abs(np.linalg.norm(T.svd_step(s, c, Vt, alpha)) - Delta) <= 1e-12 * Delta
