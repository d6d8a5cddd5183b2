"""GPU parity of the correlator path: time-slice norms, and R(t) = G_E(t) / G_0(t) end to end.

End to end at 4^4, Dirichlet in the field direction (x) and in time as in
Sec. 4: five operators (no field; u and d at +E and -E), 12 point-source
propagators each by the multi-mass sector CG, correlators on the GPU.  The
reference solves D(m) densely for each operator (dense spectral sign with the
same polynomial and small space, pinned to the C oracle) and contracts with
the correlator oracle.  Bars: time-slice norms 1e-13 relative; R(t) 1e-8
(propagators to 1e-10 times the condition number of D(m)).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import api, corr, dense

pytestmark = pytest.mark.gpu
MW = -1.5
NORM = 6.5


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_timeslice_norm2_matches_oracle():
    from paper_1111_6288_amd import ov
    L = (6, 4, 6, 10)
    ctx = ov.Context(L, (2, 0, 0, 2), MW)
    x = synth.gaussian_spinors(L, 5, 3)
    got = ctx.timeslice_norm2(_t(x))
    ref = corr.slice_norm2(x, L)
    assert np.abs(got - ref).max() < 1e-13 * ref.max()
    assert np.array_equal(ctx.timeslice_norm2(_t(x)), got)      # deterministic


def test_pion_correlator_matches_oracle():
    """G(t) summed over the sources on the device (ov_pion_correlator) against the correlator
    oracle, on a ragged Dirichlet lattice with 12 sources."""
    from paper_1111_6288_amd import ov
    L = (6, 4, 6, 10)
    ctx = ov.Context(L, (2, 0, 0, 2), MW)
    x = synth.gaussian_spinors(L, 12, 13)
    got = ctx.pion_correlator(_t(x))
    ref = corr.pion_correlator(x, L)
    assert got.shape == (10,)
    assert np.abs(got - ref).max() < 1e-13 * ref.max()
    assert np.array_equal(ctx.pion_correlator(_t(x)), got)


def test_ratio_R_end_to_end():
    from paper_1111_6288_amd import ov
    L, bc = (4, 4, 4, 4), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.3, 77)
    eta = 0.3
    ops = [(0.0, 0.0), (2 / 3, eta), (2 / 3, -eta), (-1 / 3, eta), (-1 / 3, -eta)]
    m = 0.1
    n, l = 140, 16
    ctx = ov.Context(L, bc, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields([q for q, _ in ops], [e for _, e in ops])
    Hs = [dense.dense_hw(L, bc, MW, U, q * e) for q, e in ops]
    w = min(np.sort(np.abs(np.linalg.eigvalsh(H)))[l] for H in Hs)
    eps = (w / NORM) ** 2 * 0.9
    ctx.set_sign_params(n, eps, NORM)
    c = api.cheb_coeffs(n, eps)
    b = synth.point_sources(L, (2, 0, 0, 1))
    G_ref, G_gpu = [], []
    for f, H in enumerate(Hs):
        Vs, lam = dense.small_space(H, l)
        ctx.upload_eigvecs(f, _t(Vs), lam)
        S, _, _, _ = dense.spectral_sign(H, NORM, n, eps, c, l)
        D = dense.dense_dm(S, m)
        props = np.stack([np.linalg.solve(D, bj.ravel()).reshape(bj.shape) for bj in b])
        G_ref.append(corr.pion_correlator(props, L))
    x, rel, rep = ctx.multishift_cg(_t(np.concatenate([b] * len(ops))), [m],
                                    fields=[f for f in range(len(ops)) for _ in range(12)], tol=1e-10)
    assert rel.max() <= 1e-10
    for f in range(len(ops)):
        G_gpu.append(ctx.pion_correlator(x[0, 12 * f:12 * (f + 1)]))
    R_ref = corr.ratio(np.mean(G_ref[1:], axis=0), G_ref[0])
    R_gpu = ov.ratio_R(G_gpu[1:], G_gpu[0])
    assert np.abs(R_gpu - R_ref).max() < 1e-8 * np.abs(R_ref).max()
    # the field changes the correlator (R is not identically 1)
    assert np.abs(R_ref - 1).max() > 1e-6


def test_correlator_derivative_against_finite_differences():
    """dF/deta for F = sum_t w_t C(t) through the solve and the sign adjoint, against central
    differences of the dense construction with the small space and polynomial held fixed
    (the same reading as the adjoint); C(t) itself against the dense solve."""
    from paper_1111_6288_amd import ov
    L, bc = (4, 4, 4, 4), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.3, 31)
    q, eta0, m = 2 / 3, 0.3, 0.1
    n, l = 140, 16
    H0 = dense.dense_hw(L, bc, MW, U, q * eta0)
    Vs, lam = dense.small_space(H0, l)
    w = np.sort(np.abs(np.linalg.eigvalsh(H0)))
    eps = (w[l] / NORM) ** 2 * 0.9
    c = api.cheb_coeffs(n, eps)
    Vm = Vs.reshape(l, -1).T
    Pi = np.eye(Vm.shape[0]) - Vm @ Vm.conj().T
    Sg = Vm @ np.diag(np.where(np.asarray(lam) >= 0, 1.0, -1.0)) @ Vm.conj().T
    b = synth.point_sources(L, (2, 0, 0, 1))[[0, 5, 7, 10]]
    wts = np.array([0.0, 1.0, 0.6, 0.3])

    def F_dense(eta):
        H = dense.dense_hw(L, bc, MW, U, q * eta)
        Qp, _, _, _ = dense.spectral_sign(H, NORM, n, eps, c, 0)
        D = dense.dense_dm(Sg + Pi @ Qp @ Pi, m)
        props = np.stack([np.linalg.solve(D, bj.ravel()).reshape(bj.shape) for bj in b])
        Ct = corr.pion_correlator(props, L)
        return Ct, float(wts @ Ct)

    C0, _ = F_dense(eta0)
    h = 1e-4
    dF_fd = (F_dense(eta0 + h)[1] - F_dense(eta0 - h)[1]) / (2 * h)
    ctx = ov.Context(L, bc, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields([q], [eta0])
    ctx.set_sign_params(n, eps, NORM)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    Cg, dF = ctx.correlator_deta(_t(b), 0, m, wts, tol=1e-11)
    assert np.abs(Cg - C0).max() < 1e-8 * np.abs(C0).max()
    assert abs(dF - dF_fd) < 1e-5 * abs(dF_fd), (dF, dF_fd)
    assert abs(dF_fd) > 1e-6
