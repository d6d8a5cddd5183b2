"""Pins of the eigen-oracle (lowest-|lambda| eigenpairs of H_w), CPU only.

* The Lanczos route (H_w^2 by ARPACK, then Rayleigh-Ritz with H_w) agrees
  with the dense eigendecomposition of the explicit 4^4 matrix.
* Free field: the smallest |lambda| of H_w are the closed forms
  sqrt(M(p)^2 + |sin p|^2), 12-fold per momentum (H_w^2 = D_w^dag D_w is
  diagonal in momentum space).
* Residuals ||H_w v - lambda v|| are at rounding level with the C stencil.
* The library's host Jacobi routine used by the GPU Rayleigh-Ritz agrees with
  numpy's eigh (the routine needs no GPU).
"""
import numpy as np
import pytest

import synth
from oracle import api, dense, eig

MW = -1.5


def _lat(L, bc, alpha, seed, qeta=0.0):
    U = synth.su3_links(L, alpha, seed)
    return api.Lattice(L, bc, MW, U, qeta), U


def test_lanczos_route_matches_dense_4x4():
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    lat, U = _lat(L, bc, 0.3, 1111, qeta=0.2)
    l = 10
    lam_d, V_d = eig.hw_low_modes_dense(L, bc, MW, U, 0.2, l + 4)
    gaps = np.abs(np.diff(np.abs(lam_d)))
    assert gaps[l - 1] > 1e-6, "choose l at a gap"
    lam, V, res = eig.hw_low_modes(lat, l)
    assert np.abs(lam - lam_d[:l]).max() < 1e-10
    assert res.max() < 1e-10
    # same subspace: projectors agree
    A = V.reshape(l, -1)
    B = V_d[:l].reshape(l, -1)
    P = A.T @ A.conj() - B.T @ B.conj()
    assert np.abs(P).max() < 1e-8


def test_free_field_closed_form():
    """Dense route (the free spectrum is highly degenerate, which a single-vector Krylov
    method cannot resolve; the Lanczos route is pinned to dense on random fields above)."""
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.0, 0)
    lat = api.Lattice(L, bc, MW, U)
    ps = []
    for mu in range(4):
        n = np.arange(L[mu])
        ps.append(2 * np.pi * n / L[mu] if bc[mu] == 0 else np.pi * (2 * n + 1) / L[mu])
    P = np.meshgrid(*ps, indexing="ij")
    mag = np.sqrt((MW + sum(1 - np.cos(p) for p in P)) ** 2 + sum(np.sin(p) ** 2 for p in P)).ravel()
    mags = np.sort(np.repeat(mag, 12))
    lam, V = eig.hw_low_modes_dense(L, bc, MW, U, 0.0, 30)
    assert np.abs(np.abs(lam) - mags[:30]).max() < 1e-10
    assert eig.residuals(lat, lam, V).max() < 1e-10


def test_residual_helper_catches_a_wrong_pair():
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    lat, U = _lat(L, bc, 0.3, 5)
    lam, V = eig.hw_low_modes_dense(L, bc, MW, U, 0.0, 4)
    r = eig.residuals(lat, lam, V)
    assert r.max() < 1e-11
    assert eig.residuals(lat, -lam, V).min() > 1e-3      # wrong sign of lambda is caught
    assert eig.residuals(lat, lam, V[::-1]).max() > 1e-6  # pairs mixed up are caught


def test_library_host_jacobi_against_numpy():
    ov = pytest.importorskip("paper_1111_6288_amd.ov")
    rng = np.random.default_rng(3)
    for n in (1, 3, 17, 64):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = A + A.conj().T
        w, Z = ov.dense_heev(A)
        assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1.0, np.abs(w).max())
        assert np.abs(A @ Z - Z * w).max() < 1e-12 * max(1.0, np.abs(w).max())
        assert np.abs(Z.conj().T @ Z - np.eye(n)).max() < 1e-12
    # degenerate spectrum: still an orthonormal basis
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))
    A = (Q * np.array([1, 1, 1, 2, 2, 3, 3, 3.0])) @ Q.conj().T
    w, Z = ov.dense_heev(A)
    assert np.abs(w - [1, 1, 1, 2, 2, 3, 3, 3]).max() < 1e-13
    assert np.abs(Z.conj().T @ Z - np.eye(8)).max() < 1e-13


def test_dov_sector_modes_reproduce_the_overlap_spectrum():
    """With the exact sign: D_ov is normal, D^dag D commutes with gamma5, and the two sectors'
    eigenvalues together are |eigenvalues of D_ov|^2; the sector operator is 2 + 2 P S P."""
    L, bc = (2, 2, 2, 4), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.5, 4)
    H = dense.dense_hw(L, bc, MW, U, 0.1)
    S = dense.exact_sign(H)
    n = H.shape[0]
    ev_d = np.linalg.eigvals(np.eye(n) + dense.gamma5_full(n // 12) @ S)
    mags = np.sort(np.abs(ev_d) ** 2)
    half = n // 2
    lp, Wp = eig.dov_sector_low_modes_dense(S, +1, half)
    lm, Wm = eig.dov_sector_low_modes_dense(S, -1, half)
    assert np.abs(np.sort(np.concatenate([lp, lm])) - mags).max() < 1e-10
    # sector operator 2 + 2 P S P on the + sector
    g5 = np.diag(dense.gamma5_full(n // 12)).real
    P = np.diag((1 + g5) / 2)
    Asec = 2 * P + 2 * P @ S @ P
    for j in range(4):
        w = Wp[j].ravel()
        assert np.linalg.norm(Asec @ w - lp[j] * w) < 1e-10
