"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only *draws* inputs: random SU(3) gauge links, Gaussian and point
spinor sources, random orthonormal bases and random gauge rotations.  It holds
none of the overlap method's arithmetic (no Dirac operator, no sign function,
no phases, no boundary conditions); both implementations apply those
themselves to the arrays produced here.

Canonical layouts (complex128, C order):

* site index ``i = x + Lx*(y + Ly*(z + Lz*t))`` for ``L = (Lx, Ly, Lz, Lt)``;
* gauge field ``U[mu, i, a, b]`` of shape ``(4, V, 3, 3)``, mu = 0..3 for
  x, y, z, t; ``U[mu, i]`` is the link from site i to site i + mu-hat;
* spinor field ``psi[i, s, c]`` of shape ``(V, 4, 3)``; a batch of fields has a
  leading ``nrhs`` axis.

The links follow the recipe of the synthetic workloads: U = exp(i*alpha*H)
with H = sum_a omega_a lambda_a / 2 over the eight Gell-Mann matrices and
omega_a i.i.d. standard normal (numpy PCG64, seeded).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "site_index", "coords", "gell_mann", "su3_field", "su3_links",
    "gaussian_spinors", "point_source", "point_sources", "random_orthonormal",
    "random_orthonormal_torch", "random_algebra_field",
]


def volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def site_index(L, x, y, z, t) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return x + Lx * (y + Ly * (z + Lz * t))


def coords(L) -> np.ndarray:
    """Integer coordinates (V, 4) in canonical site order."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0] = 1
    g[2][1, 1] = -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def su3_field(n: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """n random SU(3) matrices exp(i*alpha*H), H = sum omega_a lambda_a/2."""
    omega = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", omega, gell_mann()) / 2.0
    w, vec = np.linalg.eigh(H)
    ph = np.exp(1j * alpha * w)
    return np.einsum("nij,nj,nkj->nik", vec, ph, vec.conj())


def su3_links(L, alpha: float, seed: int) -> np.ndarray:
    """Gauge field (4, V, 3, 3) of random SU(3) links; alpha=0 gives unit links."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    U = su3_field(4 * V, alpha, rng)
    return np.ascontiguousarray(U.reshape(4, V, 3, 3))


def random_algebra_field(L, seed: int, shape_prefix=(4,)) -> np.ndarray:
    """Random Hermitian traceless 3x3 matrices X (Gell-Mann, N(0,1) weights).

    Used as finite-difference directions U -> exp(i h X) U.
    """
    V = volume(L)
    n = int(np.prod(shape_prefix)) * V
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((n, 8))
    X = np.einsum("na,aij->nij", omega, gell_mann()) / 2.0
    return np.ascontiguousarray(X.reshape(*shape_prefix, V, 3, 3))


def gaussian_spinors(L, nrhs: int, seed: int) -> np.ndarray:
    """(nrhs, V, 4, 3) complex Gaussian spinors, unit variance per real part."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nrhs, V, 4, 3, 2))
    return np.ascontiguousarray(a[..., 0] + 1j * a[..., 1])


def point_source(L, x0, s: int, c: int) -> np.ndarray:
    V = volume(L)
    psi = np.zeros((V, 4, 3), dtype=np.complex128)
    psi[site_index(L, *x0), s, c] = 1.0
    return psi


def point_sources(L, x0) -> np.ndarray:
    """The 12 spin-colour point sources at site x0, shape (12, V, 4, 3)."""
    return np.stack([point_source(L, x0, s, c) for s in range(4) for c in range(3)])


def random_orthonormal(L, l: int, seed: int) -> np.ndarray:
    """l orthonormal vectors (l, V, 4, 3): QR of a seeded Gaussian block."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((12 * V, l, 2))
    q, _ = np.linalg.qr(a[..., 0] + 1j * a[..., 1])
    return np.ascontiguousarray(q.T.reshape(l, V, 4, 3))


def random_orthonormal_torch(L, l: int, seed: int, device, dtype=None):
    """Large-lattice variant of :func:`random_orthonormal` drawn on a torch device.

    Draws a seeded complex Gaussian block of shape (l, 12V) with torch's
    generator and orthonormalises its rows by CholeskyQR2 (two rounds of Gram
    matrix, Cholesky factor, multiplication by the inverse factor), which
    keeps the work in big matrix products.  The result differs from the numpy variant's numbers and
    is meant for throughput runs where the oracle is not asked for the whole
    field.  Returns a (l, V, 4, 3) complex128 tensor on ``device``.
    """
    import torch

    V = volume(L)
    dtype = dtype or torch.complex128
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    A = torch.randn((l, 12 * V), dtype=dtype, device=device, generator=g)
    for _ in range(2):
        G = A @ A.conj().T                      # (l, l) Gram matrix
        R = torch.linalg.cholesky(G)            # G = R R^H, R lower
        A = torch.linalg.inv(R) @ A             # (l, l) inverse, one large product
    return A.reshape(l, V, 4, 3)
