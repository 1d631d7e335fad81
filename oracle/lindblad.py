"""Plain CPU FP64 oracle for open-system (Lindblad) GRAPE in Liouville space.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline may import this module; the HIP product path shares no code with it.

The dynamics (Gorini-Kossakowski-Sudarshan-Lindblad master equation, hbar = 1)
with piecewise-constant controls:

    d rho / dt = -i [H_k, rho] + sum_l (L_l rho L_l^dag - 1/2 {L_l^dag L_l, rho}),
    H_k = H0 + sum_j u[j, k] H_j.

On the row-major vectorisation vec(rho)[a d + b] = rho[a, b] the right-hand
side is a d^2 x d^2 matrix G_k = G0 + sum_j u[j, k] G_j (G0 holds the drift
and the dissipator, G_j the commutator with H_j).  The oracle builds each
generator column by column from its definition, column (a d + b) being
vec of the map applied to the matrix unit E_ab, so that it shares no
Kronecker-product identity with the product path.

    S_k = exp(dt G_k),  X_N = S_{N-1} ... S_0,
    g = Tr(T^dag X_N) with T = V (x) conj(V) the target unitary's
        superoperator (T vec(rho) = vec(V rho V^dag)),
    F = |g|^2 / d^4,
    dF/du[j, k] = (2 / d^4) Re(conj(g) <W_k, L(dt G_k, dt G_j)>_F),
    W_k = B_{k+1} X_k^dag (B_N = T, B_k = S_k^dag B_{k+1}).

S_k is not unitary and G_k not normal, so the exponentials are
scipy.linalg.expm (Pade scaling and squaring) and the Frechet derivative is
scipy.linalg.expm_frechet (Al-Mohy and Higham 2009), library routines used as
single steps.  For a closed system (no L_l) X_N = U_N (x) conj(U_N) and
F = F_unitary^2.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def superop(fn, d: int) -> np.ndarray:
    """Matrix of the linear map fn on d x d matrices, in the row-major
    vectorisation: column a d + b is vec(fn(E_ab))."""
    S = np.empty((d * d, d * d), dtype=np.complex128)
    for a in range(d):
        for b in range(d):
            E = np.zeros((d, d), dtype=np.complex128)
            E[a, b] = 1.0
            S[:, a * d + b] = np.asarray(fn(E), dtype=np.complex128).reshape(-1)
    return S


def commutator_generator(H: np.ndarray) -> np.ndarray:
    """rho -> -i [H, rho]."""
    H = np.asarray(H, dtype=np.complex128)
    return superop(lambda r: -1j * (H @ r - r @ H), H.shape[0])


def dissipator(Ls, d: int) -> np.ndarray:
    """rho -> sum_l (L rho L^dag - 1/2 {L^dag L, rho})."""
    Ls = [np.asarray(L, dtype=np.complex128) for L in Ls]

    def fn(r):
        out = np.zeros_like(r)
        for L in Ls:
            LdL = L.conj().T @ L
            out += L @ r @ L.conj().T - 0.5 * (LdL @ r + r @ LdL)
        return out

    return superop(fn, d)


def target_superop(V: np.ndarray) -> np.ndarray:
    """rho -> V rho V^dag."""
    V = np.asarray(V, dtype=np.complex128)
    return superop(lambda r: V @ r @ V.conj().T, V.shape[0])


def generators(H0, Hc, Ls):
    """(G0, [G_j]) of the master equation."""
    d = np.asarray(H0).shape[0]
    G0 = commutator_generator(H0) + (dissipator(Ls, d) if len(Ls) else 0.0)
    return G0, np.stack([commutator_generator(H) for H in Hc])


def lindblad_gradient(H0, Hc, Ls, u, dt, V):
    """Returns (F, g, grad (m x N), X_N) of the open-system problem."""
    G0, Gc = generators(H0, Hc, Ls)
    return generator_gradient(G0, Gc, u, dt, target_superop(V))


def generator_gradient(G0, Gc, u, dt, T):
    """The same for any generators G0, Gc[j] (D x D) and target T (D x D):
    S_k = exp(dt (G0 + sum_j u[j, k] Gc[j])), g = Tr(T^dag X_N), F = |g|^2 / D^2.
    Returns (F, g, grad, X_N)."""
    G0 = np.asarray(G0, dtype=np.complex128)
    Gc = np.asarray(Gc, dtype=np.complex128)
    T = np.asarray(T, dtype=np.complex128)
    u = np.asarray(u, dtype=np.float64)
    m, N = u.shape
    D = G0.shape[0]
    As = [dt * (G0 + np.einsum("j,jab->ab", u[:, k], Gc)) for k in range(N)]
    Ss = [sla.expm(A) for A in As]
    Xs = [np.eye(D, dtype=np.complex128)]
    for S in Ss:
        Xs.append(S @ Xs[-1])
    Bs = [None] * (N + 1)
    Bs[N] = T
    for k in range(N - 1, -1, -1):
        Bs[k] = Ss[k].conj().T @ Bs[k + 1]
    g = complex(np.trace(T.conj().T @ Xs[-1]))
    F = abs(g) ** 2 / D ** 2
    grad = np.empty((m, N))
    for k in range(N):
        W = Bs[k + 1] @ Xs[k].conj().T
        for j in range(m):
            L = sla.expm_frechet(As[k], dt * Gc[j], compute_expm=False)
            grad[j, k] = 2.0 / D ** 2 * (np.conj(g) * np.sum(W.conj() * L)).real
    return F, g, grad, Xs[-1]


def lindblad_ref(problem):
    """Oracle result for a workloads.LindbladProblem: F, g, grad, X_N."""
    F, g, grad, XN = lindblad_gradient(problem.H0, problem.Hc, problem.Ls, problem.u, problem.dt, problem.V)
    return {"F": F, "g": g, "grad": grad, "XN": XN}
