"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every comparison is element by element on the same seeded inputs.  Bars:
FP64 dslash 1e-14 and FP64 sign / D_ov / adjoint 1e-12 (relative to the max
modulus of the oracle result); FP32 and BF16 results are checked against
error budgets derived from their unit roundoff (FP32: 2^-24 per operation
over O(10) accumulated terms in a dslash, amplified by the Clenshaw
recursion; BF16 storage: 2^-9 per stored component).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import api, dense

pytestmark = pytest.mark.gpu
MW = -1.5


def _ov():
    from paper_1111_6288_amd import ov
    return ov


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    return t.cpu().numpy()


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def make_ctx(L, bc, U, q=(0.0,), eta=(0.0,)):
    ov = _ov()
    ctx = ov.Context(L, bc, MW)
    ctx.upload_gauge(_t(U))
    ctx.set_fields(q, eta)
    return ctx


# ------------------------------------------------------------------ dslash
DSLASH_CASES = [
    ((2, 2, 2, 2), (0, 0, 0, 1)),        # forward and backward neighbours coincide; V < one wavefront
    ((4, 4, 4, 4), (0, 0, 0, 1)),
    ((6, 4, 6, 10), (2, 0, 0, 2)),       # ragged: 1440 sites, Dirichlet in x and t
    ((8, 8, 8, 16), (1, 2, 0, 1)),
]


@pytest.mark.parametrize("L,bc", DSLASH_CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("fp32", 2e-6), ("bf16", 2e-2)])
def test_dslash_parity(L, bc, prec, tol):
    U = synth.su3_links(L, 0.5, 101)
    q, eta = (2 / 3, -1 / 3, 2 / 3), (0.0, 0.31, -0.12)
    ctx = make_ctx(L, bc, U, q, eta)
    nrhs = 7
    x = synth.gaussian_spinors(L, nrhs, 5)
    fields = [j % 3 for j in range(nrhs)]
    for op, opc in (("HW", 1), ("DW", 0)):
        y = _np(ctx.dslash(_t(x), fields, op=op, prec=prec))
        for j in range(nrhs):
            lat = api.Lattice(L, bc, MW, U, q[fields[j]] * eta[fields[j]])
            ref = api.dslash(lat, x[j], opc)
            assert _rel(y[j], ref) < tol, (op, j, _rel(y[j], ref))


@pytest.mark.parametrize("nr", [1, 2, 4, 8])
@pytest.mark.parametrize("block", [64, 128, 256])
def test_dslash_every_tuning_variant(nr, block):
    """Each launch shape of the autotuner space gives the oracle's answer."""
    L, bc = (6, 4, 6, 10), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.5, 7)
    ctx = make_ctx(L, bc, U, (2 / 3,), (0.2,))
    x = synth.gaussian_spinors(L, 11, 9)
    for prec, tol in (("fp32", 2e-6), ("fp64", 1e-14)):
        if prec == "fp64" and nr == 8:
            continue
        ctx.set_tuning(prec, nr, block)
        y = _np(ctx.dslash(_t(x), [0] * 11, prec=prec))
        lat = api.Lattice(L, bc, MW, U, 2 / 3 * 0.2)
        for j in (0, 5, 10):
            assert _rel(y[j], api.dslash(lat, x[j], 1)) < tol


def test_dslash_deterministic_and_batch_equals_single():
    L, bc = (4, 4, 4, 8), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.4, 3)
    ctx = make_ctx(L, bc, U, (2 / 3, -1 / 3), (1e-3, 2e-3))
    x = synth.gaussian_spinors(L, 6, 1)
    f = [0, 1, 0, 1, 1, 0]
    y1 = _np(ctx.dslash(_t(x), f))
    y2 = _np(ctx.dslash(_t(x), f))
    assert np.array_equal(y1, y2)
    for j in range(6):
        ys = _np(ctx.dslash(_t(x[j:j + 1]), [f[j]]))
        assert _rel(ys[0], y1[j]) < 1e-15


# ------------------------------------------------------------------ sign / D_ov
@pytest.fixture(scope="module")
def exact44():
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.3, 1111)
    H = dense.dense_hw(L, bc, MW, U)
    Vs, lam = dense.small_space(H, 8)
    return L, bc, U, H, Vs, lam


def test_sign_parity_4444_exact_small_space(exact44):
    """4^4 workload: n = 100, eps = 0.01, 8 exact eigenvectors, 12 point sources."""
    L, bc, U, H, Vs, lam = exact44
    n, eps, norm = 100, 0.01, 6.5
    ctx = make_ctx(L, bc, U)
    ctx.set_sign_params(n, eps, norm)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    src = synth.point_sources(L, (0, 0, 0, 0))
    sp = api.SignParams(n, eps, norm, Vs, lam)
    lat = api.Lattice(L, bc, MW, U)
    ref = api.sign(lat, sp, src)
    y64 = _np(ctx.sign_apply(_t(src), prec="fp64"))
    for j in range(12):
        assert _rel(y64[j], ref[j]) < 1e-12
    y32 = _np(ctx.sign_apply(_t(src), prec="fp32"))
    assert max(_rel(y32[j], ref[j]) for j in range(12)) < 1e-5
    # D_ov = 1 + gamma5 s and its dagger, several masses
    mass = [0.0, 0.01, 0.05] * 4
    d64 = _np(ctx.dov_apply(_t(src), mass=mass, prec="fp64"))
    dd64 = _np(ctx.dov_apply(_t(src), mass=mass, dagger=True, prec="fp64"))
    for j in range(12):
        assert _rel(d64[j], api.dov(lat, sp, src[j], mass[j])) < 1e-12
        assert _rel(dd64[j], api.dov(lat, sp, src[j], mass[j], dagger=True)) < 1e-12


@pytest.mark.parametrize("L,bc,n,l", [((6, 4, 6, 10), (2, 0, 0, 2), 40, 6),
                                      ((8, 8, 8, 16), (2, 0, 0, 2), 200, 16)])
def test_sign_parity_random_small_space_mixed_fields(L, bc, n, l):
    """Several field groups, each with its own small space, in one batch."""
    U = synth.su3_links(L, 0.2, 77)
    q, eta = (0.0, 2 / 3, 2 / 3), (0.0, 1e-3, -1e-3)
    ctx = make_ctx(L, bc, U, q, eta)
    eps = api.eq2_eps(1e-10, n)
    ctx.set_sign_params(n, eps, 6.5)
    Vs = [synth.random_orthonormal(L, l, 100 + f) for f in range(3)]
    lams = [np.linspace(-1, 1, l) + 0.01 * f for f in range(3)]
    for f in range(3):
        ctx.upload_eigvecs(f, _t(Vs[f]), lams[f])
    x = synth.gaussian_spinors(L, 5, 3)
    fields = [0, 1, 2, 1, 0]
    mass = [0.01, 0.02, 0.05, 0.01, 0.02]
    y = _np(ctx.sign_apply(_t(x), fields, prec="fp64"))
    d = _np(ctx.dov_apply(_t(x), fields, mass, dagger=True, prec="fp64"))
    y32 = _np(ctx.sign_apply(_t(x), fields, prec="fp32"))
    for j in (0, 1, 2):
        f = fields[j]
        lat = api.Lattice(L, bc, MW, U, q[f] * eta[f])
        sp = api.SignParams(n, eps, 6.5, Vs[f], lams[f])
        ref = api.sign(lat, sp, x[j])
        assert _rel(y[j], ref) < 1e-12
        assert _rel(y32[j], ref) < 2e-5
        assert _rel(d[j], api.dov(lat, sp, x[j], mass[j], dagger=True)) < 1e-12


def test_sign_no_small_space_and_q_eta_invariance():
    L, bc = (4, 4, 4, 8), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.2, 5)
    ctx = make_ctx(L, bc, U, (2 / 3, 4 / 3), (1e-3, 0.5e-3))
    ctx.set_sign_params(30, 0.02, 6.5)
    x = synth.gaussian_spinors(L, 2, 8)
    y = _np(ctx.sign_apply(_t(x), [0, 1]))
    assert _rel(y[0], y[1] * 0 + _np(ctx.sign_apply(_t(x[:1]), [1]))[0]) < 1e-14
    lat = api.Lattice(L, bc, MW, U, 2 / 3 * 1e-3)
    assert _rel(y[0], api.sign(lat, api.SignParams(30, 0.02, 6.5), x[0])) < 1e-12


def test_sign_bf16_storage_error_budget(exact44):
    L, bc, U, H, Vs, lam = exact44
    ctx = make_ctx(L, bc, U)
    ctx.set_sign_params(100, 0.01, 6.5 * (1 + 2 ** -6))
    ctx.upload_eigvecs(0, _t(Vs), lam)
    x = synth.gaussian_spinors(L, 2, 4)
    sp = api.SignParams(100, 0.01, 6.5 * (1 + 2 ** -6), Vs, lam)
    ref = api.sign(api.Lattice(L, bc, MW, U), sp, x)
    y = _np(ctx.sign_apply(_t(x), prec="bf16"))
    err = max(np.linalg.norm(y[j] - ref[j]) / np.linalg.norm(ref[j]) for j in range(2))
    assert err < 3e-2, err


# ------------------------------------------------------------------ CG
@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_deflated_cg_solution(inner):
    L, bc = (2, 2, 2, 4), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.5, 31)
    qeta = 2 / 3 * 1e-3
    lat = api.Lattice(L, bc, MW, U, qeta)
    H = dense.dense_hw(L, bc, MW, U, qeta)
    n, eps, norm, l = 60, 0.02, 6.5, 6
    c = api.cheb_coeffs(n, eps)
    Vs, lam = dense.small_space(H, l)
    S, _, _, _ = dense.spectral_sign(H, norm, n, eps, c, l)
    ctx = make_ctx(L, bc, U, (2 / 3,), (1e-3,))
    ctx.set_sign_params(n, eps, norm)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    src = synth.point_sources(L, (1, 0, 0, 2))
    mass = [0.01, 0.02, 0.05] * 4
    tol = 1e-12 if inner == "fp64" else 1e-10
    x, rep = ctx.deflated_cg(_t(src), mass=mass, tol=tol, inner_prec=inner, inner_tol=1e-5 if inner == "fp32" else 1e-13)
    x = _np(x)
    for j in range(12):
        assert rep[j]["status"] == 0 and rep[j]["relres"] <= tol
        # oracle's own true residual of the GPU solution
        rhs = api.dov(lat, api.SignParams(n, eps, norm, Vs, lam), src[j], mass[j], dagger=True)
        sp = api.SignParams(n, eps, norm, Vs, lam)
        Ax = api.dov(lat, sp, api.dov(lat, sp, x[j], mass[j]), mass[j], dagger=True)
        assert np.linalg.norm(rhs - Ax) / np.linalg.norm(rhs) <= 3 * tol
        xd = np.linalg.solve(dense.dense_dm(S, mass[j]), src[j].ravel())
        assert np.linalg.norm(x[j].ravel() - xd) / np.linalg.norm(xd) < 1e-7


def test_deflated_cg_with_deflation_basis():
    L, bc = (2, 2, 2, 4), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.5, 31)
    H = dense.dense_hw(L, bc, MW, U, 0.0)
    n, eps, norm, l = 60, 0.02, 6.5, 6
    c = api.cheb_coeffs(n, eps)
    Vs, lam = dense.small_space(H, l)
    S, _, _, _ = dense.spectral_sign(H, norm, n, eps, c, l)
    Dm0 = dense.dense_dm(S, 0.0)
    w, v = np.linalg.eigh(Dm0.conj().T @ Dm0)
    W = np.ascontiguousarray(v[:, :16].T.reshape(16, -1, 4, 3))
    ctx = make_ctx(L, bc, U)
    ctx.set_sign_params(n, eps, norm)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    b = synth.gaussian_spinors(L, 3, 2)
    mass = [0.01, 0.02, 0.05]
    x0, r0 = ctx.deflated_cg(_t(b), mass=mass, tol=1e-11, inner_prec="fp64", inner_tol=1e-12, use_deflation=False)
    ctx.upload_deflation(0, _t(W))
    x1, r1 = ctx.deflated_cg(_t(b), mass=mass, tol=1e-11, inner_prec="fp64", inner_tol=1e-12, use_deflation=True)
    for j in range(3):
        assert r1[j]["iters"] < r0[j]["iters"]
        assert _rel(_np(x1)[j], _np(x0)[j]) < 1e-8


def test_cg_reports_noconv_and_keeps_iterate():
    L, bc = (2, 2, 2, 4), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.5, 3)
    ctx = make_ctx(L, bc, U)
    ctx.set_sign_params(20, 0.05, 6.5)
    b = synth.gaussian_spinors(L, 2, 2)
    x, rep = ctx.deflated_cg(_t(b), mass=[0.01, 0.01], tol=1e-14, maxiter=3, inner_prec="fp64", inner_tol=1e-3,
                             raise_on_noconv=False)
    assert all(r["status"] == -4 for r in rep)
    assert np.isfinite(_np(x)).all() and np.abs(_np(x)).max() > 0


# ------------------------------------------------------------------ adjoint
@pytest.mark.parametrize("L,bc,l,K", [((2, 2, 2, 4), (2, 0, 0, 2), 4, 5), ((4, 4, 4, 4), (0, 0, 0, 1), 0, 1),
                                      ((4, 4, 2, 6), (2, 0, 0, 2), 3, 64)])
def test_sign_backward_parity(L, bc, l, K):
    q, eta = 2 / 3, 0.05
    U = synth.su3_links(L, 0.4, 41)
    n, eps, norm = 24, 0.03, 6.5
    Vs = synth.random_orthonormal(L, l, 2) if l else None
    lam = np.linspace(-1, 1, l) if l else None
    ctx = make_ctx(L, bc, U, (q,), (eta,))
    ctx.set_sign_params(n, eps, norm)
    if l:
        ctx.upload_eigvecs(0, _t(Vs), lam)
    x, g = synth.gaussian_spinors(L, 2, 13)
    gU, ge, gx = ctx.sign_backward(0, _t(x), _t(g), ckpt_every=K)
    lat = api.Lattice(L, bc, MW, U, q * eta)
    rU, re, rx = api.sign_backward(lat, api.SignParams(n, eps, norm, Vs, lam), q, x, g)
    assert _rel(_np(gU), rU) < 1e-12
    assert abs(ge - re) <= 1e-12 * max(abs(re), 1e-12 * np.abs(rU).max())
    assert _rel(_np(gx), rx) < 1e-12


# ------------------------------------------------------------------ errors
def test_error_paths_leave_context_usable():
    ov = _ov()
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    U = synth.su3_links(L, 0.3, 1)
    ctx = ov.Context(L, bc, MW)
    x = _t(synth.gaussian_spinors(L, 1, 1))
    with pytest.raises(ov.OvError) as e:
        ctx.dslash(x)
    assert e.value.code == ov.OV_ESTATE
    bad = U.copy()
    bad[1, 3, 0, 0] = np.nan
    with pytest.raises(ov.OvError) as e:
        ctx.upload_gauge(_t(bad))
    assert e.value.code == ov.OV_ENAN
    ctx.upload_gauge(_t(U))
    ctx.set_fields((0.0,), (0.0,))
    with pytest.raises(ov.OvError):
        ctx.dslash(x, [3])
    with pytest.raises(ov.OvError):
        ctx.upload_eigvecs(0, _t(2 * synth.random_orthonormal(L, 2, 1)), [1.0, -1.0])
    lat = api.Lattice(L, bc, MW, U)
    assert _rel(_np(ctx.dslash(x))[0], api.dslash(lat, _np(x)[0], 1)) < 1e-14
