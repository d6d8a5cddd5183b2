"""Lowest-|lambda| eigenpairs of H_w (TEST INFRASTRUCTURE ONLY).

The small space of the sign function is the set of eigenvectors of H_w with
the smallest |lambda| (Sec. 2, Fig. 1); the paper finds them with Arnoldi and
Chebyshev acceleration (Sec. 3.1).  What is computed has a plain definition,
so the oracle is that definition: the eigenpairs of smallest |lambda| of the
Hermitian operator H_w of the C oracle.

* ``hw_low_modes_dense``: dense eigendecomposition (<= 4^4).
* ``hw_low_modes``: Lanczos (scipy's ARPACK, a library routine) for the
  smallest eigenvalues of H_w^2 with the C oracle's H_w as the operator, then
  Rayleigh-Ritz with H_w itself on the subspace found, which splits the
  pairs +lambda, -lambda that H_w^2 cannot tell apart.

* ``dov_sector_low_modes_dense``: the lowest eigenpairs of D_ov^dag D_ov in
  one chirality sector (the deflation basis, Sec. 2 end and Sec. 3.1), by
  dense eigendecomposition of the sector block.

Never imported by the product path.
"""
from __future__ import annotations

import numpy as np

from . import api, dense


def hw_low_modes_dense(L, bc, mw, U, qeta, l):
    """(lambda[l], V (l, V, 4, 3)) from the dense H_w, ascending |lambda|."""
    H = dense.dense_hw(L, bc, mw, U, qeta)
    w, v = np.linalg.eigh(H)
    order = np.argsort(np.abs(w), kind="stable")[:l]
    V = H.shape[0] // 12
    return w[order], np.ascontiguousarray(v[:, order].T.reshape(l, V, 4, 3))


def hw_low_modes(lat: api.Lattice, l, extra=8, tol=1e-13, seed=0):
    """(lambda[l], V (l, V, 4, 3), residuals[l]) by Lanczos on H_w^2, then H_w Rayleigh-Ritz.

    ``extra`` more eigenvectors of H_w^2 are computed so that a cluster of
    nearly equal |lambda| that straddles position l is complete.
    """
    from scipy.sparse.linalg import LinearOperator, eigsh

    V = lat.V
    n = 12 * V

    def hw(x):
        return api.dslash(lat, np.asarray(x).reshape(V, 4, 3), 1).ravel()

    A = LinearOperator((n, n), matvec=lambda x: hw(hw(x)), dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    nev = l + extra
    _, vecs = eigsh(A, k=nev, which="SA", tol=tol, v0=v0, ncv=max(2 * nev + 1, 40))
    q, _ = np.linalg.qr(vecs)
    Hq = np.stack([hw(q[:, i]) for i in range(nev)], axis=1)
    Hs = q.conj().T @ Hq
    th, Z = np.linalg.eigh(0.5 * (Hs + Hs.conj().T))
    order = np.argsort(np.abs(th), kind="stable")[:l]
    X = q @ Z[:, order]
    lam = th[order]
    vecs_out = np.ascontiguousarray(X.T.reshape(l, V, 4, 3))
    res = np.array([np.linalg.norm(hw(X[:, i]) - lam[i] * X[:, i]) for i in range(l)])
    return lam, vecs_out, res


def residuals(lat: api.Lattice, lam, vecs):
    """||H_w v_j - lambda_j v_j|| / ||v_j|| with the C oracle's H_w."""
    out = []
    for lj, v in zip(lam, vecs):
        r = api.dslash(lat, v, 1) - lj * v
        out.append(np.linalg.norm(r) / np.linalg.norm(v))
    return np.array(out)


def dov_sector_low_modes_dense(S, chi, l):
    """Lowest eigenpairs of D_ov^dag D_ov restricted to the chirality-chi sector (dense).

    D_ov = 1 + gamma5 S with S a dense (approximate) sign matrix; the sector
    holds the components with gamma5 = chi (spins 0, 1 for +1 in the chiral
    basis).  Returns (lambda[l] ascending, W (l, V, 4, 3) with zeros in the
    other sector).
    """
    n = S.shape[0]
    V = n // 12
    g5 = np.diag(dense.gamma5_full(V)).real
    D = np.eye(n) + dense.gamma5_full(V) @ S
    A = D.conj().T @ D
    idx = np.nonzero(g5 == chi)[0]
    w, v = np.linalg.eigh(A[np.ix_(idx, idx)])
    W = np.zeros((l, n), np.complex128)
    W[:, idx] = v[:, :l].T
    return w[:l], W.reshape(l, V, 4, 3)
