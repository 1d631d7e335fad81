"""Spin-chain GRAPE problems with seeded random couplings, controls and targets.

Conventions (fixed here once so every consumer sees the same problem):

* Pauli matrices sigma_x = [[0,1],[1,0]], sigma_y = [[0,-i],[i,0]],
  sigma_z = diag(1,-1).
* Qubit 0 is the leftmost (most significant) tensor factor:
  op_i = I^(x i) (x) sigma (x) I^(x (n_q-1-i)).
* Chains have open boundaries (n_q - 1 bonds).
* Controls are ordered [X_0, Y_0, X_1, Y_1, ...], so control j = 2i + {0: x, 1: y}.
* Amplitudes are an m x N row-major array, u[j, k] = control j in slice k;
  slice 0 acts first.
* N(mu, s) means a normal draw with standard deviation s.
* A problem drawn for configuration i uses numpy's default_rng seeded with
  SeedSequence(i) (or SeedSequence([i, b]) for the b-th copy in a batch) and
  draws in the order couplings J, local fields h, amplitudes u, target V.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_PAULI = {"x": _SX, "y": _SY, "z": _SZ}


@dataclass
class Problem:
    """One GRAPE evaluation: drift H0, controls Hc[j], amplitudes u[j, k], slice
    length dt and target unitary V (all complex128 / float64, row-major)."""

    H0: np.ndarray
    Hc: np.ndarray
    u: np.ndarray
    dt: float
    V: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return int(self.H0.shape[0])

    @property
    def m(self) -> int:
        return int(self.Hc.shape[0])

    @property
    def N(self) -> int:
        return int(self.u.shape[1])

    def with_u(self, u: np.ndarray) -> "Problem":
        return Problem(self.H0, self.Hc, np.ascontiguousarray(u, dtype=np.float64),
                       self.dt, self.V, self.name, dict(self.meta))

    def with_target(self, V: np.ndarray) -> "Problem":
        return Problem(self.H0, self.Hc, self.u, self.dt,
                       np.ascontiguousarray(V, dtype=np.complex128), self.name, dict(self.meta))


@dataclass
class StateProblem:
    """One state-to-state GRAPE evaluation: drift H0, controls Hc[j],
    amplitudes u[j, k], slice length dt, initial state psi0 and target state
    chi (unit vectors of length d; complex128 / float64, row-major)."""

    H0: np.ndarray
    Hc: np.ndarray
    u: np.ndarray
    dt: float
    psi0: np.ndarray
    chi: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return int(self.H0.shape[0])

    @property
    def m(self) -> int:
        return int(self.Hc.shape[0])

    @property
    def N(self) -> int:
        return int(self.u.shape[1])

    def with_u(self, u: np.ndarray) -> "StateProblem":
        return StateProblem(self.H0, self.Hc, np.ascontiguousarray(u, dtype=np.float64), self.dt,
                            self.psi0, self.chi, self.name, dict(self.meta))

    def with_target(self, chi: np.ndarray) -> "StateProblem":
        return StateProblem(self.H0, self.Hc, self.u, self.dt, self.psi0,
                            np.ascontiguousarray(chi, dtype=np.complex128), self.name, dict(self.meta))


@dataclass
class LindbladProblem:
    """One open-system GRAPE evaluation: drift H0, controls Hc[j], collapse
    operators Ls[l] (rates folded in: L = sqrt(gamma) A), amplitudes u[j, k],
    slice length dt and the target unitary V (d x d)."""

    H0: np.ndarray
    Hc: np.ndarray
    Ls: List[np.ndarray]
    u: np.ndarray
    dt: float
    V: np.ndarray
    name: str = ""

    @property
    def d(self) -> int:
        return int(self.H0.shape[0])

    @property
    def m(self) -> int:
        return int(self.Hc.shape[0])

    @property
    def N(self) -> int:
        return int(self.u.shape[1])

    def with_u(self, u: np.ndarray) -> "LindbladProblem":
        return LindbladProblem(self.H0, self.Hc, self.Ls, np.ascontiguousarray(u, dtype=np.float64), self.dt,
                               self.V, self.name)


def pauli(a: str) -> np.ndarray:
    return _PAULI[a].copy()


def site_op(i: int, a: str, nq: int) -> np.ndarray:
    """sigma_a acting on qubit i of an nq-qubit register (qubit 0 leftmost)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(nq):
        out = np.kron(out, _PAULI[a] if q == i else np.eye(2, dtype=np.complex128))
    return out


def heisenberg_drift(J: Sequence[float], h: Sequence[float]) -> np.ndarray:
    """sum_i J_i (XX + YY + ZZ)_{i,i+1} + sum_i h_i Z_i on len(h) qubits."""
    nq = len(h)
    d = 2 ** nq
    H = np.zeros((d, d), dtype=np.complex128)
    for i, Ji in enumerate(J):
        for a in "xyz":
            H += Ji * site_op(i, a, nq) @ site_op(i + 1, a, nq)
    for i, hi in enumerate(h):
        H += hi * site_op(i, "z", nq)
    return H


def ising_drift(J: Sequence[float], gx: float, nq: int) -> np.ndarray:
    """sum_i J_i Z_i Z_{i+1} + gx * sum_i X_i on nq qubits."""
    d = 2 ** nq
    H = np.zeros((d, d), dtype=np.complex128)
    for i, Ji in enumerate(J):
        H += Ji * site_op(i, "z", nq) @ site_op(i + 1, "z", nq)
    for i in range(nq):
        H += gx * site_op(i, "x", nq)
    return H


def xy_controls(nq: int) -> np.ndarray:
    """[X_0, Y_0, X_1, Y_1, ...] stacked as an (2 nq, d, d) array."""
    return np.stack([site_op(i, a, nq) for i in range(nq) for a in "xy"])


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed d x d unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :])


def _heisenberg_problem(nq: int, N: int, dt: float, rng: np.random.Generator,
                        name: str, u_scale: float = 0.5) -> Problem:
    J = rng.uniform(0.5, 1.5, size=nq - 1)
    h = rng.normal(0.0, 0.2, size=nq)
    H0 = heisenberg_drift(J, h)
    Hc = xy_controls(nq)
    u = rng.normal(0.0, u_scale, size=(Hc.shape[0], N))
    V = haar_unitary(2 ** nq, rng)
    return Problem(H0, Hc, u, dt, V, name, {"J": J, "h": h})


def make_config(i: int, copy: Optional[int] = None, N: Optional[int] = None) -> Problem:
    """Workload i (1..4) of the benchmark suite.

    1: single qubit, H0 = sigma_z / 2, one sigma_x control, N=100, dt=0.01,
       u ~ U[-1, 1], target X.
    2: 4-qubit Heisenberg chain (d=16), J ~ U[0.5,1.5], h ~ N(0, 0.2),
       8 controls, N=1000, dt=0.005, u ~ N(0, 0.5), Haar target.
    3: 6-qubit Ising chain (d=64), ZZ couplings J ~ U[0.5,1.5], transverse
       field 0.3 sum X, 12 controls, N=2000, dt=0.002, u ~ N(0, 0.5), Haar target.
    4: 7-qubit Heisenberg chain (d=128) as in 2, 14 controls, N=1000,
       dt=0.005, u ~ N(0, 0.5), Haar target.

    ``copy`` selects an independent draw of the same configuration (seeded
    with SeedSequence([i, copy])); ``N`` overrides the slice count (the draw
    order is unchanged, so u and V then differ from the full-size draw).
    """
    ss = np.random.SeedSequence(i if copy is None else [i, copy])
    rng = np.random.default_rng(ss)
    tag = f"config{i}" + ("" if copy is None else f".{copy}")
    if i == 1:
        n = 100 if N is None else N
        H0 = 0.5 * pauli("z")
        Hc = pauli("x")[None]
        u = rng.uniform(-1.0, 1.0, size=(1, n))
        return Problem(H0, Hc, u, 0.01, pauli("x"), tag)
    if i == 2:
        return _heisenberg_problem(4, 1000 if N is None else N, 0.005, rng, tag)
    if i == 3:
        nq = 6
        J = rng.uniform(0.5, 1.5, size=nq - 1)
        H0 = ising_drift(J, 0.3, nq)
        Hc = xy_controls(nq)
        n = 2000 if N is None else N
        u = rng.normal(0.0, 0.5, size=(Hc.shape[0], n))
        V = haar_unitary(2 ** nq, rng)
        return Problem(H0, Hc, u, 0.002, V, tag, {"J": J, "gx": 0.3})
    if i == 4:
        return _heisenberg_problem(7, 1000 if N is None else N, 0.005, rng, tag)
    raise ValueError(f"unknown configuration {i}")


def haar_state(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unit vector of length d: a complex Gaussian vector
    normalised."""
    z = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    return np.ascontiguousarray(z / np.linalg.norm(z))


def basis_state(d: int, a: int = 0) -> np.ndarray:
    e = np.zeros(d, dtype=np.complex128)
    e[a] = 1.0
    return e


def make_state(i: int, copy: Optional[int] = None, N: Optional[int] = None) -> StateProblem:
    """State-to-state transfer on the drift, controls, amplitudes and dt of
    configuration i (make_config(i, copy, N)), from psi0 = |0...0> (the first
    basis vector).  The target is chi = X|0> = |1> for configuration 1 and a
    Haar-random state otherwise, drawn with SeedSequence([i, copy or 0, 2])."""
    p = make_config(i, copy, N)
    psi0 = basis_state(p.d)
    if i == 1:
        chi = basis_state(2, 1)
    else:
        chi = haar_state(p.d, np.random.default_rng(np.random.SeedSequence([i, 0 if copy is None else copy, 2])))
    return StateProblem(p.H0, p.Hc, p.u, p.dt, psi0, chi, "state-" + p.name, dict(p.meta))


def make_state_batch(i: int, B: int, N: Optional[int] = None) -> List[StateProblem]:
    """B independent state-transfer draws of configuration i (copies 1..B)."""
    return [make_state(i, copy=b + 1, N=N) for b in range(B)]


def make_state_random(seed: int, d: int, m: int, N: int, dt: float, monomial: bool = False,
                      u_scale: float = 0.5) -> StateProblem:
    """State transfer with the drift, controls and amplitudes of
    make_random (or make_random_monomial) and Haar-random psi0 and chi, drawn
    with SeedSequence([seed, d, m, N, 3]) in the order psi0, chi."""
    p = (make_random_monomial if monomial else make_random)(seed, d, m, N, dt, u_scale)
    rng = np.random.default_rng(np.random.SeedSequence([seed, d, m, N, 3]))
    psi0 = haar_state(d, rng)
    chi = haar_state(d, rng)
    return StateProblem(p.H0, p.Hc, p.u, dt, psi0, chi, "state-" + p.name)


def make_lindblad(nq: int, N: int, dt: float = 0.02, gamma_damp: float = 0.05, gamma_deph: float = 0.02,
                  seed: int = 0) -> LindbladProblem:
    """Open Heisenberg chain on nq qubits (J ~ U[0.5, 1.5], h ~ N(0, 0.2) as in
    configuration 2), X/Y controls on every qubit, u ~ N(0, 0.5), a Haar
    target, and on every qubit amplitude damping sqrt(gamma_damp) sigma_- and
    dephasing sqrt(gamma_deph) Z (sigma_- = |0><1|).  Seeded with
    SeedSequence([nq, N, seed, 4]), drawn in the order J, h, u, V."""
    rng = np.random.default_rng(np.random.SeedSequence([nq, N, seed, 4]))
    p = _heisenberg_problem(nq, N, dt, rng, f"lindblad{nq}.{N}.{seed}") if nq > 1 else None
    if p is None:
        H0 = rng.normal(0.0, 0.2) * pauli("z")
        Hc = xy_controls(1)
        u = rng.normal(0.0, 0.5, size=(2, N))
        V = haar_unitary(2, rng)
    else:
        H0, Hc, u, V = p.H0, p.Hc, p.u, p.V
    lower = np.array([[0, 1], [0, 0]], dtype=np.complex128)
    Ls = []
    for i in range(nq):
        op = np.ones((1, 1), dtype=np.complex128)
        for q in range(nq):
            op = np.kron(op, lower if q == i else np.eye(2, dtype=np.complex128))
        if gamma_damp > 0:
            Ls.append(np.sqrt(gamma_damp) * op)
        if gamma_deph > 0:
            Ls.append(np.sqrt(gamma_deph) * site_op(i, "z", nq))
    return LindbladProblem(H0, Hc, Ls, u, dt, V, f"lindblad{nq}.{N}.{seed}")


def make_batch(i: int, B: int, N: Optional[int] = None) -> List[Problem]:
    """B independent draws of configuration i (copies 1..B)."""
    return [make_config(i, copy=b + 1, N=N) for b in range(B)]


def random_hermitian(d: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    """(G + G^dag) / 2 for a complex Ginibre matrix G with unit-variance
    entries, times scale / sqrt(d) (spectral radius of order scale)."""
    g = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return np.ascontiguousarray(scale * (g + g.conj().T) / (2.0 * np.sqrt(d)))


def make_random(seed: int, d: int, m: int, N: int, dt: float, u_scale: float = 0.5) -> Problem:
    """A problem with dense random Hermitian drift and controls of any d (not
    only powers of two), u ~ N(0, u_scale), Haar target; seeded with
    SeedSequence([seed, d, m, N]) and drawn in the order H0, Hc, u, V."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, d, m, N]))
    H0 = random_hermitian(d, rng)
    Hc = np.stack([random_hermitian(d, rng) for _ in range(m)])
    u = rng.normal(0.0, u_scale, size=(m, N))
    V = haar_unitary(d, rng)
    return Problem(H0, Hc, u, dt, V, f"random{seed}.{d}x{m}x{N}")


# Serving workload: request dimensions and their weights.
SERVE_DIMS = (2, 4, 8, 16, 32, 64, 128)
SERVE_WEIGHTS = (0.10, 0.15, 0.20, 0.20, 0.15, 0.12, 0.08)


def random_monomial_hermitian(d: int, rng: np.random.Generator) -> np.ndarray:
    """A Hermitian matrix with at most one nonzero per row (a phased involution,
    as a Pauli string is): rows are paired by a random involution; a pair (a, b)
    gets H[a, b] = z and H[b, a] = conj(z) with z of unit modulus times a
    uniform factor in [0.5, 1.5], a fixed point a a real H[a, a] in
    [-1.5, 1.5], and with probability 0.1 a row is left empty."""
    H = np.zeros((d, d), dtype=np.complex128)
    order = rng.permutation(d)
    i = 0
    while i < d:
        a = int(order[i])
        if rng.random() < 0.1:
            i += 1  # an empty row (and column)
        elif i + 1 < d and rng.random() < 0.7:
            b = int(order[i + 1])
            z = rng.uniform(0.5, 1.5) * np.exp(1j * rng.uniform(0, 2 * np.pi))
            H[a, b] = z
            H[b, a] = np.conj(z)
            i += 2
        else:
            H[a, a] = rng.uniform(-1.5, 1.5)
            i += 1
    return H


def make_random_monomial(seed: int, d: int, m: int, N: int, dt: float, u_scale: float = 0.5) -> Problem:
    """A problem with a dense random Hermitian drift, m controls of
    random_monomial_hermitian, u ~ N(0, u_scale) and a Haar target; seeded with
    SeedSequence([seed, d, m, N, 1]) and drawn in the order H0, Hc, u, V."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, d, m, N, 1]))
    H0 = random_hermitian(d, rng)
    Hc = np.stack([random_monomial_hermitian(d, rng) for _ in range(m)])
    u = rng.normal(0.0, u_scale, size=(m, N))
    V = haar_unitary(d, rng)
    return Problem(H0, Hc, u, dt, V, f"monomial{seed}.{d}x{m}x{N}")


def make_request(index: int, d: int, N: int, trace_seed: int = 5) -> Problem:
    """One serving request: Heisenberg chain on log2(d) qubits (d = 2: the
    drift is h_0 Z_0 alone), 2 log2(d) controls, u ~ N(0, 0.5), dt = 0.005,
    Haar target; seeded with SeedSequence([trace_seed, index])."""
    nq = int(round(np.log2(d)))
    if 2 ** nq != d:
        raise ValueError("d must be a power of two")
    rng = np.random.default_rng(np.random.SeedSequence([trace_seed, index]))
    return _heisenberg_problem(nq, N, 0.005, rng, f"req{index}")


def poisson_trace(n: int, rate: float, seed: int = 5, N_range=(100, 2000)):
    """n requests with exponential inter-arrival times of mean 1/rate seconds.
    Returns a list of dicts {index, t_arrival, d, N}; d is drawn with
    SERVE_WEIGHTS and N uniformly from N_range (inclusive)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    unit = rng.exponential(1.0, size=n)          # drawn for any rate, so shapes never depend on it
    gaps = unit / rate if rate > 0 else np.zeros(n)   # rate <= 0: everything arrives at t = 0
    t = np.cumsum(gaps) - (gaps[0] if n else 0.0)
    ds = rng.choice(np.array(SERVE_DIMS), size=n, p=np.array(SERVE_WEIGHTS))
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=n)
    return [{"index": i, "t_arrival": float(t[i]), "d": int(ds[i]), "N": int(Ns[i])}
            for i in range(n)]
