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


@pytest.mark.parametrize("nr", [1, 4])
def test_dslash_zslab_site_order(nr):
    """Site order 1 (each XCD walks a z-slab) gives the oracle's answer, with padding-free V."""
    L, bc = (4, 6, 8, 6), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.5, 17)
    ctx = make_ctx(L, bc, U, (2 / 3, -1 / 3), (0.2, 0.1))
    x = synth.gaussian_spinors(L, 5, 2)
    f = [0, 1, 1, 0, 1]
    for prec, tol in (("fp32", 2e-6), ("fp64", 1e-14)):
        ctx.set_tuning(prec, nr, 64)
        ctx.set_site_order(prec, 1)
        y = _np(ctx.dslash(_t(x), f, prec=prec))
        for j in range(5):
            lat = api.Lattice(L, bc, MW, U, (2 / 3, -1 / 3)[f[j]] * (0.2, 0.1)[f[j]])
            assert _rel(y[j], api.dslash(lat, x[j], 1)) < tol


@pytest.mark.parametrize("L,bc", [((4, 4, 4, 4), (0, 0, 0, 1)), ((4, 6, 8, 6), (2, 0, 0, 2)),
                                  ((8, 8, 8, 16), (1, 2, 0, 0))])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("fp32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("block", [256, 512])
def test_dslash_tmarch_order(L, bc, prec, tol, block):
    """Site order 2 (threads march along t with the time neighbours in registers),
    4 or 8 right-hand sides per workgroup; 11 RHS leave a partial group."""
    U = synth.su3_links(L, 0.5, 23)
    q, eta = (2 / 3, -1 / 3, 2 / 3), (0.0, 0.31, -0.12)
    ctx = make_ctx(L, bc, U, q, eta)
    ctx.set_site_order(prec, 2)
    ctx.set_tuning(prec, 1, block)
    nrhs = 11
    x = synth.gaussian_spinors(L, nrhs, 5)
    fields = [j % 3 for j in range(nrhs)]
    for op, opc in (("HW", 1), ("DW", 0)):
        y = _np(ctx.dslash(_t(x), fields, op=op, prec=prec))
        for j in range(nrhs):
            lat = api.Lattice(L, bc, MW, U, q[fields[j]] * eta[fields[j]])
            assert _rel(y[j], api.dslash(lat, x[j], opc)) < tol, (op, j)


def test_sign_with_tmarch_order():
    """The fused Clenshaw epilogue under site order 2."""
    L, bc = (8, 8, 8, 16), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.2, 77)
    ctx = make_ctx(L, bc, U, (2 / 3,), (1e-3,))
    n = 60
    eps = 0.5 / n ** 2
    ctx.set_sign_params(n, eps, 6.5)
    Vs = synth.random_orthonormal(L, 6, 5)
    lam = np.linspace(-1, 1, 6)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    x = synth.gaussian_spinors(L, 5, 3)
    ref = api.sign(api.Lattice(L, bc, MW, U, 2 / 3 * 1e-3), api.SignParams(n, eps, 6.5, Vs, lam), x[:2])
    for prec, tol, block in (("fp64", 1e-12, 256), ("fp32", 2e-5, 256), ("fp32", 2e-5, 512)):
        ctx.set_site_order(prec, 2)
        ctx.set_tuning(prec, 1, block)
        y = _np(ctx.sign_apply(_t(x), [0] * 5, prec=prec))
        for j in range(2):
            assert _rel(y[j], ref[j]) < tol, (prec, block)


@pytest.mark.parametrize("L,bc", DSLASH_CASES)
@pytest.mark.parametrize("split,nr,block", [(2, 1, 64), (4, 2, 128), (4, 1, 256), (2, 2, 192), (8, 1, 64),
                                            (8, 2, 256)])
def test_dslash_rhs_split(L, bc, split, nr, block):
    """Sub-wave RHS split: each wavefront covers 64/split sites for split RHS groups
    (ragged volumes need the padding rewritten by blocks of 16 or 32 sites)."""
    U = synth.su3_links(L, 0.4, 17)
    q, eta = (2 / 3, -1 / 3), (0.1, -0.3)
    ctx = make_ctx(L, bc, U, q, eta)
    nrhs = 7
    x = synth.gaussian_spinors(L, nrhs, 12)
    f = [(j * 5) % 2 for j in range(nrhs)]
    for prec, tol in (("fp64", 1e-14), ("fp32", 2e-6), ("bf16", 2e-2)):
        if prec == "bf16" and split == 8:
            with pytest.raises(_ov().OvError):
                ctx.set_launch_config(prec, "dslash", rhs_split=8, rhs_per_thread=nr)
            continue
        for order, cols in ((0, 1), (1, 1), (3, 1), (1, 2), (1, L[1])):
            if L[1] % cols:
                continue
            ctx.set_launch_config(prec, "dslash", rhs_per_thread=nr, block=block, site_order=order,
                                  blocks_per_cu=0, stream_hint=order % 2, rhs_split=split, cols=cols)
            for op, opc in (("HW", 1), ("DW", 0)):
                y = _np(ctx.dslash(_t(x), f, op=op, prec=prec))
                for j in range(nrhs):
                    lat = api.Lattice(L, bc, MW, U, q[f[j]] * eta[f[j]])
                    assert _rel(y[j], api.dslash(lat, x[j], opc)) < tol, (prec, order, op, j)


@pytest.mark.parametrize("order,block,nr,split", [(0, 128, 2, 1), (1, 64, 1, 4), (0, 256, 2, 2), (2, 256, 1, 1),
                                                  (2, 512, 1, 1), (3, 256, 1, 4), (3, 128, 2, 8)])
def test_stream_hint_and_per_kind_shapes(order, block, nr, split):
    """Non-temporal epilogue/output accesses and separate plain / fused launch shapes give
    the oracle's dslash and sign (the hint changes cache policy only)."""
    L, bc = (8, 8, 8, 16), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.3, 41)
    ctx = make_ctx(L, bc, U, (2 / 3, -1 / 3), (1e-3, 0.2))
    n = 40
    eps = 0.5 / n ** 2
    ctx.set_sign_params(n, eps, 6.5)
    x = synth.gaussian_spinors(L, 9, 8)
    f = [j % 2 for j in range(9)]
    for prec, dtol, stol in (("fp64", 1e-14, 1e-12), ("fp32", 2e-6, 2e-5), ("bf16", 2e-2, 3e-2)):
        if (prec == "fp64" and block == 512) or (prec == "bf16" and split == 8):
            continue
        # plain launches in one shape, fused launches in another, both with the hint
        ctx.set_launch_config(prec, "dslash", rhs_per_thread=nr, block=block, site_order=order,
                              blocks_per_cu=0, stream_hint=1, rhs_split=split)
        ctx.set_launch_config(prec, "clenshaw", rhs_per_thread=2, block=128, site_order=(order + 1) % 4,
                              blocks_per_cu=2, stream_hint=1, rhs_split=4 if order != 1 else 1)
        got = ctx.get_launch_config(prec, "dslash")
        assert got == dict(rhs_per_thread=nr, block=block, site_order=order, blocks_per_cu=0, stream_hint=1,
                           rhs_split=split, cols=1, wshare=1)
        y = _np(ctx.dslash(_t(x), f, prec=prec))
        for j in (0, 1, 8):
            lat = api.Lattice(L, bc, MW, U, (2 / 3 * 1e-3, -1 / 3 * 0.2)[f[j]])
            assert _rel(y[j], api.dslash(lat, x[j], 1)) < dtol, (prec, j)
        if prec == "bf16":
            continue
        s = _np(ctx.sign_apply(_t(x[:3]), f[:3], prec=prec))
        for j in range(2):
            lat = api.Lattice(L, bc, MW, U, (2 / 3 * 1e-3, -1 / 3 * 0.2)[f[j]])
            ref = api.sign(lat, api.SignParams(n, eps, 6.5), x[j:j + 1])[0]
            assert _rel(s[j], ref) < stol, (prec, j)


def test_launch_config_rejects_bad_values():
    L, bc = (4, 4, 4, 4), (0, 0, 0, 1)
    ctx = make_ctx(L, bc, synth.su3_links(L, 0.3, 1))
    ov = _ov()
    good = ctx.get_launch_config("fp32", "clenshaw")
    for bad in (dict(rhs_per_thread=3), dict(block=96), dict(site_order=4), dict(blocks_per_cu=-1),
                dict(stream_hint=2), dict(rhs_split=3), dict(rhs_per_thread=4, rhs_split=2), dict(cols=3),
                dict(cols=0)):
        with pytest.raises(ov.OvError):
            ctx.set_launch_config("fp32", "clenshaw", **bad)
        assert ctx.get_launch_config("fp32", "clenshaw") == good


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


def clenshaw_growth(n, eps):
    """Worst amplification of the recursion on Q^2 in [0, 1]: |T_n| at t = -(1+eps)/(1-eps).

    Modes with Q^2 < eps map outside [-1, 1], where Chebyshev polynomials grow
    like cosh(n acosh|t|); rounding errors committed inside the recursion are
    amplified by up to this factor.
    """
    return float(np.cosh(n * np.arccosh((1 + eps) / (1 - eps))))


def _sign_mixed_fields(L, bc, n, l, eps, tol32):
    U = synth.su3_links(L, 0.2, 77)
    q, eta = (0.0, 2 / 3, 2 / 3), (0.0, 1e-3, -1e-3)
    ctx = make_ctx(L, bc, U, q, eta)
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
    out = []
    for j in (0, 1, 2):
        f = fields[j]
        lat = api.Lattice(L, bc, MW, U, q[f] * eta[f])
        sp = api.SignParams(n, eps, 6.5, Vs[f], lams[f])
        ref = api.sign(lat, sp, x[j])
        out.append((_rel(y[j], ref), _rel(y32[j], ref), _rel(d[j], api.dov(lat, sp, x[j], mass[j], dagger=True))))
    return out


@pytest.mark.parametrize("L,bc,n,l", [((6, 4, 6, 10), (2, 0, 0, 2), 40, 6),
                                      ((8, 8, 8, 16), (2, 0, 0, 2), 200, 16)])
def test_sign_parity_random_small_space_mixed_fields(L, bc, n, l):
    """Several field groups, each with its own small space, in one batch.

    eps = 0.5/n^2 keeps the recursion within a growth of cosh(sqrt 2) for any
    spectrum, the regime the method prescribes (the small space holds every
    mode below sqrt(eps)), so FP64 rounding stays O(n u) and the 1e-12 bar holds.
    """
    eps = 0.5 / n ** 2
    assert clenshaw_growth(n, eps) < 2.3
    for e64, e32, ed in _sign_mixed_fields(L, bc, n, l, eps, 2e-5):
        assert e64 < 1e-12 and ed < 1e-12
        assert e32 < 2e-5


def test_sign_parity_outside_the_interval():
    """eps from eq. (2) with a random small space leaves modes below sqrt(eps) in the
    polynomial part; there the recursion is evaluated outside [-1, 1] and both sides'
    rounding is amplified by up to clenshaw_growth(n, eps).  Bar: 10 n u growth."""
    L, bc, n, l = (6, 4, 6, 10), (2, 0, 0, 2), 40, 6
    eps = api.eq2_eps(1e-10, n)
    bar = 10 * n * 2.0 ** -53 * clenshaw_growth(n, eps)
    for e64, e32, ed in _sign_mixed_fields(L, bc, n, l, eps, 1e-3):
        assert e64 < bar and ed < bar


def test_sign_no_small_space_and_q_eta_invariance():
    L, bc = (4, 4, 4, 8), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.2, 5)
    ctx = make_ctx(L, bc, U, (2 / 3, 4 / 3), (1e-3, 0.5e-3))
    ctx.set_sign_params(30, 0.02, 6.5)
    x = synth.gaussian_spinors(L, 2, 8)
    y = _np(ctx.sign_apply(_t(x), [0, 1]))
    # (q, eta) and (2q, eta/2) give the same operator
    assert _rel(y[0], _np(ctx.sign_apply(_t(x[:1]), [1]))[0]) < 1e-14
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


# ------------------------------------------------------------------ autograd
def test_sign_apply_autograd_gradcheck():
    """torch.autograd.gradcheck of SignApply w.r.t. links, eta and x at 2^4."""
    from paper_1111_6288_amd.autograd import sign_apply
    L, bc = (2, 2, 2, 2), (2, 0, 0, 2)
    q = 2 / 3
    U0 = synth.su3_links(L, 0.4, 3)
    ctx = make_ctx(L, bc, U0, (q,), (0.1,))
    ctx.set_sign_params(8, 0.05, 6.5)
    Vs = synth.random_orthonormal(L, 2, 1)
    ctx.upload_eigvecs(0, _t(Vs), [0.3, -0.4])
    U = _t(U0).requires_grad_(True)
    eta = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    x = _t(synth.gaussian_spinors(L, 1, 4)[0]).requires_grad_(True)
    f = lambda U_, e_, x_: sign_apply(ctx, 0, U_, e_, x_, q, ckpt_every=3)
    assert torch.autograd.gradcheck(f, (U, eta, x), eps=1e-6, atol=1e-7, rtol=1e-5, fast_mode=True)


def test_backward_vs_finite_differences_c5_shape():
    """Adjoint at 8^3 x 16 (order 200, checkpoint 32) against central differences on the GPU forward."""
    L, bc = (8, 8, 8, 16), (2, 0, 0, 2)
    q, eta = 2 / 3, 1e-3
    U = synth.su3_links(L, 0.2, 55)
    ctx = make_ctx(L, bc, U, (q,), (eta,))
    n = 200
    eps = api.eq2_eps(1e-10, n)
    ctx.set_sign_params(n, eps, 6.5)
    Vs = synth.random_orthonormal(L, 8, 3)
    ctx.upload_eigvecs(0, _t(Vs), np.linspace(-1, 1, 8))
    x, g = synth.gaussian_spinors(L, 2, 21)
    gU, ge, gx = ctx.sign_backward(0, _t(x), _t(g), ckpt_every=32)
    xt, gt = _t(x)[None], _t(g)

    def loss(eta_, Ut=None):
        if Ut is not None:
            ctx.upload_gauge(Ut)
        ctx.set_field_eta(0, q, eta_)
        return float(torch.vdot(gt.reshape(-1), ctx.sign_apply(xt, [0])[0].reshape(-1)).real)

    h = 1e-6
    fd = (loss(eta + h) - loss(eta - h)) / (2 * h)
    assert abs(fd - ge) <= 1e-6 * max(abs(ge), 1e-3)
    from scipy.linalg import expm
    X = synth.random_algebra_field(L, 99)
    V = synth.volume(L)
    Ep = np.stack([[expm(1j * h * X[m, i]) for i in range(V)] for m in range(4)])
    Em = np.stack([[expm(-1j * h * X[m, i]) for i in range(V)] for m in range(4)])
    fdU = (loss(eta, _t(Ep @ U)) - loss(eta, _t(Em @ U))) / (2 * h)
    an = float(np.sum(np.real(np.conj(_np(gU)) * (1j * X @ U))))
    assert abs(fdU - an) <= 1e-6 * abs(an)


# ------------------------------------------------------------------ graphs
def test_graph_replays_match_eager():
    """Captured D(m) pipelines: every replay equals the eager result bit for bit."""
    L, bc = (6, 4, 6, 10), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.2, 8)
    ctx = make_ctx(L, bc, U, (2 / 3, 2 / 3), (1e-3, -1e-3))
    ctx.set_sign_params(20, 0.05, 6.5)
    for f in range(2):
        ctx.upload_eigvecs(f, _t(synth.random_orthonormal(L, 4, 30 + f)), [0.2, -0.1, 0.3, -0.4])
    x = _t(synth.gaussian_spinors(L, 4, 2))
    fields, mass = [0, 1, 1, 0], [0.01, 0.02, 0.05, 0.01]
    for prec in ("fp64", "fp32"):
        ctx.set_graphs(False)
        ref = _np(ctx.dov_apply(x, fields, mass, dagger=True, prec=prec))
        ctx.set_graphs(True)
        other = _t(synth.gaussian_spinors(L, 2, 3))
        for rep in range(5):   # eager, capture+launch, then three replays
            y = _np(ctx.dov_apply(x, fields, mass, dagger=True, prec=prec))
            assert np.array_equal(y, ref), (prec, rep)
            ctx.dslash(other, [0, 1])      # unrelated eager work between replays
            torch.cuda.synchronize()


def test_workspace_reuse_across_precisions_keeps_padding_zero():
    """Regression: planes are padded to a multiple of 64 sites and the workspace is
    reused across precisions; padding must read as zeros in every call (2x2x2x4 is
    half padding)."""
    L, bc = (2, 2, 2, 4), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.5, 31)
    ctx = make_ctx(L, bc, U, (2 / 3,), (1e-3,))
    ctx.set_sign_params(20, 0.5 / 400, 6.5)
    Vs = synth.random_orthonormal(L, 3, 4)
    ctx.upload_eigvecs(0, _t(Vs), [0.1, -0.2, 0.3])
    x = synth.gaussian_spinors(L, 3, 6)
    lat = api.Lattice(L, bc, MW, U, 2 / 3 * 1e-3)
    sp = api.SignParams(20, 0.5 / 400, 6.5, Vs, [0.1, -0.2, 0.3])
    ref = [api.dov(lat, sp, x[j], 0.02) for j in range(3)]
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-5), ("fp64", 1e-12), ("bf16", 3e-2), ("fp32", 2e-5)):
        y = _np(ctx.dov_apply(_t(x), mass=[0.02] * 3, prec=prec))
        assert np.isfinite(y).all(), prec
        for j in range(3):
            assert _rel(y[j], ref[j]) < tol, (prec, j)


@pytest.mark.parametrize("l,nrhs", [(129, 37), (200, 17), (256, 48), (200, 29), (64, 14), (33, 3)])
def test_sign_large_small_space(l, nrhs):
    """Small spaces of more than 8 tiles of 16 vectors (the V^dag X kernel then spreads the
    tiles over several workgroups per K-chunk), ragged l and RHS counts, against the oracle.
    The RHS counts reach every compiled group count of 4 columns (3 -> 1, 14 -> 4, 17 -> 6,
    29 -> 8, 37 and 48 -> 12; 36 per group is the full-size test's)."""
    L, bc = (4, 4, 4, 6), (2, 0, 0, 2)
    U = synth.su3_links(L, 0.3, 61)
    ctx = make_ctx(L, bc, U, (2 / 3,), (0.2,))
    n = 30
    eps = 0.5 / n ** 2   # bounded Chebyshev growth for any spectrum (random small space)
    ctx.set_sign_params(n, eps, 6.5)
    Vs = synth.random_orthonormal(L, l, 7 + l)
    lam = np.linspace(-1, 1, l)
    ctx.upload_eigvecs(0, _t(Vs), lam)
    x = synth.gaussian_spinors(L, nrhs, 3)
    lat = api.Lattice(L, bc, MW, U, 2 / 3 * 0.2)
    sp = api.SignParams(n, eps, 6.5, Vs, lam)
    y64 = _np(ctx.sign_apply(_t(x), [0] * nrhs, prec="fp64"))
    y32 = _np(ctx.sign_apply(_t(x), [0] * nrhs, prec="fp32"))
    y16 = _np(ctx.sign_apply(_t(x), [0] * nrhs, prec="bf16"))   # the projection reads BF16 X
    # BF16 storage rounds every stored vector to 2^-9 relative; with eps = 0.5/n^2 the
    # polynomial's slope near the origin, up to 1/sqrt(eps) ~ 42, amplifies that for the modes
    # the random small space leaves there
    bf_bar = 1.25 * 2.0 ** -9 / np.sqrt(eps)
    for j in sorted({0, nrhs // 2, nrhs - 1}):
        ref = api.sign(lat, sp, x[j])
        assert _rel(y64[j], ref) < 1e-12, (j, _rel(y64[j], ref))
        assert _rel(y32[j], ref) < 2e-5, (j, _rel(y32[j], ref))
        assert _rel(y16[j], ref) < bf_bar, (j, _rel(y16[j], ref), bf_bar)
