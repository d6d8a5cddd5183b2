"""NumPy dense-matrix checker for tiny lattices (TEST INFRASTRUCTURE ONLY).

Writes the Wilson operator D_w out as an explicit (12V x 12V) matrix from its
definition, independently of the C oracle (own gamma matrices, own indexing),
so that the C stencil, the Clenshaw sign and the CG can be pinned against
dense linear algebra: eigendecomposition, spectral functions and direct
solves.  Meant for V <= 256 (4^4 gives 3072 x 3072).

Conventions (the same readings as the C oracle, written again here):
  chiral gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]];
  D_w = (4 + m_w) - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) T_+mu + (1 + gamma_mu) U_mu(x-mu)^dag T_-mu];
  boundary multiplier b in {1, -1, 0} on wrapping hops; U(1) phase exp(i q eta t) on mu = 0;
  component index (site * 4 + spin) * 3 + colour.
"""
from __future__ import annotations

import numpy as np

_PAULI = [np.array([[0, 1], [1, 0]], complex),
          np.array([[0, -1j], [1j, 0]], complex),
          np.array([[1, 0], [0, -1]], complex)]


def gammas():
    """[gamma_1, gamma_2, gamma_3, gamma_4, gamma_5] in the chiral basis."""
    Z, I2 = np.zeros((2, 2)), np.eye(2)
    g = [np.block([[Z, -1j * s], [1j * s, Z]]) for s in _PAULI]
    g.append(np.block([[Z, I2], [I2, Z]]).astype(complex))
    g.append(g[0] @ g[1] @ g[2] @ g[3])
    return g


def _coords(L, i):
    Lx, Ly, Lz, Lt = L
    return [i % Lx, (i // Lx) % Ly, (i // (Lx * Ly)) % Lz, i // (Lx * Ly * Lz)]


def _index(L, c):
    Lx, Ly, Lz, Lt = L
    return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))


def dense_dw(L, bc, mw, U, qeta=0.0):
    """Explicit Wilson matrix D_w, shape (12V, 12V)."""
    L = tuple(int(v) for v in L)
    V = int(np.prod(L))
    g = gammas()
    bcf = {0: 1.0, 1: -1.0, 2: 0.0}
    D = (4.0 + mw) * np.eye(12 * V, dtype=complex)
    for i in range(V):
        c = _coords(L, i)
        for mu in range(4):
            ph = np.exp(1j * qeta * c[3]) if mu == 0 else 1.0
            # forward hop i -> i + mu with link U_mu(i)
            cf = list(c)
            cf[mu] += 1
            b = 1.0
            if cf[mu] == L[mu]:
                cf[mu] = 0
                b = bcf[bc[mu]]
            j = _index(L, cf)
            if b != 0.0:
                blk = -0.5 * b * np.kron(np.eye(4) - g[mu], ph * U[mu, i])
                D[12 * i:12 * i + 12, 12 * j:12 * j + 12] += blk
            # the same link seen from j: backward hop j -> i with U_mu(i)^dag
            if b != 0.0:
                blk = -0.5 * b * np.kron(np.eye(4) + g[mu], np.conj(ph * U[mu, i]).T)
                D[12 * j:12 * j + 12, 12 * i:12 * i + 12] += blk
    return D


def gamma5_full(V):
    return np.kron(np.eye(V), np.kron(gammas()[4], np.eye(3)))


def dense_hw(L, bc, mw, U, qeta=0.0):
    D = dense_dw(L, bc, mw, U, qeta)
    return gamma5_full(D.shape[0] // 12) @ D


def free_field_eigs(L, bc, mw):
    """Closed-form D_w spectrum for unit links: M(p) +/- i |sin p|, each 6-fold.

    M(p) = m_w + sum_mu (1 - cos p_mu); p_mu = 2 pi n / L (periodic) or
    pi (2n + 1) / L (antiperiodic).
    """
    ps = []
    for mu in range(4):
        n = np.arange(L[mu])
        ps.append(2 * np.pi * n / L[mu] if bc[mu] == 0 else np.pi * (2 * n + 1) / L[mu])
    P = np.meshgrid(*ps, indexing="ij")
    M = mw + sum(1 - np.cos(p) for p in P)
    S = np.sqrt(sum(np.sin(p) ** 2 for p in P))
    ev = np.concatenate([np.repeat((M + 1j * S).ravel(), 6), np.repeat((M - 1j * S).ravel(), 6)])
    return ev


def spectral_sign(H, norm, n, eps, c, l):
    """Spectral image of the approximate sign of a dense Hermitian H.

    Exact sgn on the l eigenvalues of smallest |lambda| ("small space"),
    q P(q^2) with q = lambda / norm on the rest, P(y) = sum c_k T_k(t(y))
    evaluated by numpy's Chebyshev series routine.  Returns (S, w, v, small)
    with S the dense matrix, (w, v) the eigenpairs and ``small`` the indices
    of the small space.
    """
    w, v = np.linalg.eigh(H)
    order = np.argsort(np.abs(w), kind="stable")
    small = order[:l]
    q = w / norm
    t = (2 * q * q - 1 - eps) / (1 - eps)
    f = q * np.polynomial.chebyshev.chebval(t, c)
    f[small] = np.where(w[small] >= 0, 1.0, -1.0)
    S = (v * f) @ v.conj().T
    return S, w, v, small


def exact_sign(H):
    w, v = np.linalg.eigh(H)
    return (v * np.where(w >= 0, 1.0, -1.0)) @ v.conj().T


def small_space(H, l):
    """l eigenvectors of smallest |lambda| as (l, V, 4, 3) and their eigenvalues."""
    w, v = np.linalg.eigh(H)
    order = np.argsort(np.abs(w), kind="stable")[:l]
    V = H.shape[0] // 12
    return np.ascontiguousarray(v[:, order].T.reshape(l, V, 4, 3)), w[order]


def dense_dm(S, m):
    """D(m) = (1 - m/2)(1 + gamma5 S) + m for a dense sign matrix S."""
    n = S.shape[0]
    G5 = gamma5_full(n // 12)
    return (1 - m / 2) * (np.eye(n) + G5 @ S) + m * np.eye(n)
