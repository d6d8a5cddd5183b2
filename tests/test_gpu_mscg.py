"""GPU parity of the multi-mass chirality-sector CG (ov_multishift_cg).

Reference: x = D(m)^{-1} b by a dense direct solve of D(m) = (1 - m/2)(1 +
gamma5 S) + m, with S the dense spectral image of the same polynomial sign
and small space (dense.spectral_sign, pinned on the CPU to the C oracle's
Clenshaw sign at 1e-13).  The solution is unique, so it is compared directly:
bar 1e-8 relative (tol 1e-10 times the condition number of D(m), <= 1/m =
20).  The polynomial (n = 140, eps from the 17th |lambda|) keeps s^2 = 1 far
below tol, so the sector identity the solver relies on holds.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import api, dense

pytestmark = pytest.mark.gpu
MW = -1.5
NORM = 6.5
L, BC = (4, 4, 4, 4), (0, 0, 0, 1)
MASSES = (0.05, 0.1, 0.3)


def _ov():
    from paper_1111_6288_amd import ov
    return ov


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def setup():
    U = synth.su3_links(L, 0.3, 1111)
    qeta = 2 / 3 * 0.15
    H = dense.dense_hw(L, BC, MW, U, qeta)
    l = 16
    Vs, lam = dense.small_space(H, l)
    w = np.sort(np.abs(np.linalg.eigvalsh(H)))
    eps = (w[l] / NORM) ** 2 * 0.9
    n = 140
    c = api.cheb_coeffs(n, eps)
    S, _, _, _ = dense.spectral_sign(H, NORM, n, eps, c, l)
    # sources: point sources of both chiralities (spin 0, 1 -> gamma5 = +1; 2, 3 -> -1)
    P = synth.point_sources(L, (1, 2, 0, 3))
    b = P[[0, 4, 7, 11]]
    ref = {m: np.stack([np.linalg.solve(dense.dense_dm(S, m), bj.ravel()).reshape(b.shape[1:]) for bj in b])
           for m in MASSES}
    ov = _ov()
    ctx = ov.Context(L, BC, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields([2 / 3], [0.15])
    ctx.set_sign_params(n, eps, NORM)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    return ctx, b, ref, n


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("inner_prec,adaptive", [("fp64", False), ("fp64", True), ("fp32", True)])
def test_multishift_matches_dense_solve(setup, inner_prec, adaptive):
    ctx, b, ref, n = setup
    x, rel, rep = ctx.multishift_cg(_t(b), MASSES, tol=1e-10, adaptive=adaptive, min_order=20,
                                    inner_prec=inner_prec)
    x = x.cpu().numpy()
    assert rel.max() <= 1e-10
    for i, m in enumerate(MASSES):
        for j in range(len(b)):
            assert _rel(x[i, j], ref[m][j]) < 1e-8, (m, j)
    assert rep["iters"] > 0 and rep["sign_applies"] == rep["iters"] * len(b)
    if inner_prec == "fp32":
        assert rep["refine_iters"] > 0


def test_adaptive_order_saves_dslash(setup):
    ctx, b, ref, n = setup
    _, rel_f, rep_f = ctx.multishift_cg(_t(b), MASSES, tol=1e-10, adaptive=False)
    _, rel_a, rep_a = ctx.multishift_cg(_t(b), MASSES, tol=1e-10, adaptive=True, min_order=20)
    assert rel_f.max() <= 1e-10 and rel_a.max() <= 1e-10
    assert rep_f["dslash_applies"] == rep_f["sign_applies"] * (2 * n + 1)
    assert rep_a["dslash_applies"] < rep_f["dslash_applies"]


def test_multishift_equals_single_mass_cg(setup):
    """Against the library's own per-mass deflated CG (the two paths share no solver code)."""
    ctx, b, ref, n = setup
    x, rel, rep = ctx.multishift_cg(_t(b), MASSES, tol=1e-10)
    for i, m in enumerate(MASSES):
        xs, report = ctx.deflated_cg(_t(b), mass=[m] * len(b), tol=1e-10)
        assert _rel(x[i].cpu().numpy(), xs.cpu().numpy()) < 1e-8


def test_non_chiral_source_rejected(setup):
    ctx, b, ref, n = setup
    ov = _ov()
    mixed = b[0] + b[3]          # spin 0 and spin 3 components
    with pytest.raises(ov.OvError, match="OV_EINVAL"):
        ctx.multishift_cg(_t(mixed[None]), MASSES)
    with pytest.raises(ov.OvError, match="OV_EINVAL"):
        ctx.multishift_cg(_t(b), (0.1, 2.5))
