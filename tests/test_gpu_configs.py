"""Solves and the sign adjoint at the sizes of the 16^3x32 and 24^3x48 workloads, checked by
the FP64 oracle (Sec. 3.2: CG for propagators with FP64 defect correction; the adjoint of
the polynomial sign with Clenshaw checkpoints).

The oracle cannot solve at these sizes; it checks the GPU solution with its own operator:
the true residual rho = ||D^dag b - D^dag D x|| / ||D^dag b|| of the normal equations that
the CG solves (three order-n oracle D(m) applications per sampled RHS).  Bars: rho <= 3 tol
(the library stops on its own FP64 rho <= tol; the factor covers the two FP64 evaluations'
rounding).  At these lattice sizes the reductions that drive alpha, beta and the stop test
run their grid-stride loops over many elements per thread.

Polynomial interval: eps = 0.5 / n^2, so that with seeded random small spaces (16 vectors)
almost no H_w mode of these near-free fields lies below sqrt(eps) N (0.023 at n = 200, 0.015
at n = 300; the lowest |lambda| of the 24^3x48 field is about 0.015).  The sign is then a
coarse approximation (eq. (2) gives delta ~ 0.1) of a well-conditioned operator, the same
operator on both sides, which is all that parity needs.

* 16^3x32 (Dirichlet x and t), order 200, two field groups (q eta = 2/3 x 1e-3, -1/3 x 1e-3)
  x masses {0.02, 0.05}: FP64 inner CG to 1e-11; two of four RHS sampled.
* 24^3x48, order 300, FP32 inner / FP64 outer to 1e-10, two point sources at mass 0.05;
  one sampled.
* 16^3x32, order 200, checkpoint every 32: ov_sign_backward against the oracle adjoint
  (all Clenshaw vectors stored) on gU, d/d eta and gx, 1e-12 relative to the largest
  modulus (measured on MI355X: 1.7e-13, 2.5e-13, 2.7e-14).  The bar needs the spectrum
  inside [-1, 1]: with eps from eq. (2) instead, random small spaces leave modes outside,
  where the recursion's growth (cosh(n acosh((1+eps)/(1-eps))), ~1e8 at n = 200) multiplies
  the rounding of both sides, and they differ at ~1e-11.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import api

pytestmark = pytest.mark.gpu
MW, NORM = -1.5, 6.5


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _oracle_rho(lat, sp, b, x, m):
    rhs = api.dov(lat, sp, b, m, dagger=True)
    Ax = api.dov(lat, sp, api.dov(lat, sp, x, m), m, dagger=True)
    return np.linalg.norm(rhs - Ax) / np.linalg.norm(rhs)


def _ctx(L, bc, U, q, eta, n, l, seed):
    from paper_1111_6288_amd import ov
    ctx = ov.Context(L, bc, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields(q, eta)
    ctx.set_sign_params(n, 0.5 / n ** 2, NORM)
    Vs = synth.random_orthonormal_torch(L, l, seed, "cuda")
    lam = [(-1.0) ** i * (0.05 + 0.001 * i) for i in range(l)]
    for f in range(len(q)):
        ctx.upload_eigvecs(f, Vs, lam)
    return ctx, Vs.cpu().numpy(), np.array(lam)


@pytest.mark.timeout(600)
def test_fp64_deflated_cg_16x32_order200():
    L, bc, n, l = (16, 16, 16, 32), (2, 0, 0, 2), 200, 16
    U = synth.su3_links(L, 0.2, 2016)
    q, eta = [2 / 3, -1 / 3], [1e-3, 1e-3]
    ctx, Vs, lam = _ctx(L, bc, U, q, eta, n, l, 700)
    src = synth.point_sources(L, (8, 0, 0, 16))
    picks = [0, 5, 7, 11]
    fields, mass = [0, 1, 0, 1], [0.02, 0.05, 0.05, 0.02]
    tol = 1e-11
    x, rep = ctx.deflated_cg(_t(src[picks]), fields=fields, mass=mass, tol=tol, inner_prec="fp64",
                             inner_tol=1e-10)
    assert all(r["status"] == 0 and r["relres"] <= tol for r in rep), rep
    x = x.cpu().numpy()
    sp = api.SignParams(n, 0.5 / n ** 2, NORM, Vs, lam)
    for j in (0, 3):
        lat = api.Lattice(L, bc, MW, U, q[fields[j]] * eta[fields[j]])
        rho = _oracle_rho(lat, sp, src[picks[j]], x[j], mass[j])
        assert rho <= 3 * tol, (j, rho)
    ctx.close()


@pytest.mark.timeout(900)
def test_mixed_deflated_cg_24x48_order300():
    L, bc, n, l = (24, 24, 24, 48), (2, 0, 0, 2), 300, 16
    U = synth.su3_links(L, 0.2, 2022)
    ctx, Vs, lam = _ctx(L, bc, U, [2 / 3], [1e-3], n, l, 800)
    src = synth.point_sources(L, (12, 0, 0, 24))[[0, 7]]
    tol = 1e-10
    x, rep = ctx.deflated_cg(_t(src), mass=[0.05, 0.05], tol=tol, inner_prec="fp32", inner_tol=1e-5)
    assert all(r["status"] == 0 and r["relres"] <= tol for r in rep), rep
    assert all(r["restarts"] >= 2 for r in rep)        # FP64 defect correction was needed
    sp = api.SignParams(n, 0.5 / n ** 2, NORM, Vs, lam)
    lat = api.Lattice(L, bc, MW, U, 2 / 3 * 1e-3)
    rho = _oracle_rho(lat, sp, src[1], x[1].cpu().numpy(), 0.05)
    assert rho <= 3 * tol, rho
    ctx.close()


@pytest.mark.timeout(600)
def test_sign_backward_16x32_order200_against_oracle():
    L, bc, n, l = (16, 16, 16, 32), (2, 0, 0, 2), 200, 16
    q, eta = 2 / 3, 1e-3
    U = synth.su3_links(L, 0.2, 2016)
    from paper_1111_6288_amd import ov
    ctx = ov.Context(L, bc, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields([q], [eta])
    eps = 0.5 / n ** 2
    ctx.set_sign_params(n, eps, NORM)
    Vs = synth.random_orthonormal(L, l, 901)
    lam = np.linspace(-1, 1, l)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    x, g = synth.gaussian_spinors(L, 2, 902)
    gU, ge, gx = ctx.sign_backward(0, _t(x), _t(g), ckpt_every=32)
    lat = api.Lattice(L, bc, MW, U, q * eta)
    rU, re, rx = api.sign_backward(lat, api.SignParams(n, eps, NORM, Vs, lam), q, x, g)
    gU, gx = gU.cpu().numpy(), gx.cpu().numpy()
    eU = np.abs(gU - rU).max() / np.abs(rU).max()
    ex = np.abs(gx - rx).max() / np.abs(rx).max()
    ee = abs(ge - re) / max(abs(re), 1e-12 * np.abs(rU).max())
    print(f"adjoint 16^3x32 n=200: gU {eU:.2e}, d/d eta {ee:.2e}, gx {ex:.2e}")
    assert eU < 1e-12 and ee < 1e-12 and ex < 1e-12, (eU, ee, ex)
    ctx.close()
