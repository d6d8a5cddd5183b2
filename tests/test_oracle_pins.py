"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests needs a GPU.  Each one is chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign, a transposed link, a
missing boundary factor, an off-by-one in the Clenshaw indices) fails it:

* gamma matrices: Clifford algebra, hermiticity, gamma5 = g1 g2 g3 g4;
* D_w: free-field closed-form spectrum (dense) and plane waves (C stencil),
  C stencil against the explicit dense matrix, gamma5-hermiticity, gauge
  covariance, the norm bound |4 + m_w| + 4 and its attainment;
* polynomial: interpolation at the Chebyshev-Gauss nodes, the paper's error
  law eq. (2) and its worked example (Sec. 2);
* sign: exact spectral image (dense eigendecomposition), accuracy against the
  exact sign, Ginsparg-Wilson identity, D_ov spectrum on the unit circle
  around 1, small-space wiring;
* CG: dense direct solve, deflation, restarts;
* backward: central finite differences.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import api, dense

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")
MW = -1.5


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.fixture(scope="module")
def lat44():
    L = (4, 4, 4, 4)
    U = synth.su3_links(L, 0.3, 1111)
    return api.Lattice(L, (0, 0, 0, 1), MW, U)


@pytest.fixture(scope="module")
def dense44(lat44):
    H = dense.dense_hw(lat44.L, lat44.bc, MW, lat44.U)
    return H


# ---------------------------------------------------------------- gammas
@pytest.mark.parametrize("src", ["c", "dense"])
def test_gamma_algebra(src):
    g = [api.gamma(m) for m in range(5)] if src == "c" else dense.gammas()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * np.eye(4) * (a == b))
    assert np.allclose(g[4], g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))


def test_gamma_c_equals_dense():
    for m in range(5):
        assert np.array_equal(api.gamma(m), dense.gammas()[m])


# ---------------------------------------------------------------- D_w
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (0, 0, 0, 1)])
def test_free_field_spectrum_dense(bc):
    L = (4, 4, 4, 4)
    D = dense.dense_dw(L, bc, MW, synth.su3_links(L, 0.0, 1))
    ev = np.sort_complex(np.round(np.linalg.eigvals(D), 9))
    ff = np.sort_complex(np.round(dense.free_field_eigs(L, bc, MW), 9))
    assert np.abs(ev - ff).max() < 1e-8


@pytest.mark.parametrize("L,bc", [((4, 4, 4, 8), (0, 0, 0, 1)), ((6, 4, 2, 4), (1, 0, 0, 0))])
def test_free_field_plane_wave_stencil(L, bc):
    """D_w e^{ipx} u = (M(p) + i sum gamma_mu sin p_mu) e^{ipx} u for unit links."""
    rng = np.random.default_rng(5)
    g = dense.gammas()
    lat = api.Lattice(L, bc, MW, synth.su3_links(L, 0.0, 1))
    X = synth.coords(L)
    for _ in range(3):
        p = []
        for mu in range(4):
            k = rng.integers(L[mu])
            p.append(2 * np.pi * k / L[mu] if bc[mu] == 0 else np.pi * (2 * k + 1) / L[mu])
        p = np.array(p)
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        wave = np.exp(1j * X @ p)
        psi = wave[:, None, None] * u[None]
        Dp = (MW + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = wave[:, None, None] * (Dp @ u)[None]
        assert _rel(api.dslash(lat, psi), expect) < 1e-13


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 2, 4)])
@pytest.mark.parametrize("bc,qeta", [((0, 0, 0, 1), 0.0), ((2, 0, 0, 2), 0.3), ((1, 2, 0, 1), -0.7)])
def test_stencil_equals_dense(L, bc, qeta):
    U = synth.su3_links(L, 0.6, 17)
    lat = api.Lattice(L, bc, MW, U, qeta)
    x = synth.gaussian_spinors(L, 1, 3)[0]
    D = dense.dense_dw(L, bc, MW, U, qeta)
    assert np.abs(api.dslash(lat, x).ravel() - D @ x.ravel()).max() < 1e-13
    G5 = dense.gamma5_full(lat.V)
    assert np.abs(api.dslash(lat, x, op=1).ravel() - G5 @ D @ x.ravel()).max() < 1e-13


@pytest.mark.parametrize("bc,qeta", [((0, 0, 0, 1), 0.0), ((2, 0, 0, 2), 2e-3 * 2 / 3)])
def test_gamma5_hermiticity(bc, qeta):
    L = (4, 4, 4, 8)
    lat = api.Lattice(L, bc, MW, synth.su3_links(L, 0.3, 2), qeta)
    x, y = synth.gaussian_spinors(L, 2, 4)
    lhs = api.vdot(y, api.dslash(lat, x, 1))
    rhs = api.vdot(api.dslash(lat, y, 1), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_hw_norm_bound(dense44):
    w = np.linalg.eigvalsh(dense44)
    assert np.abs(w).max() <= abs(4 + MW) + 4
    # attained exactly by the free field with periodic boundaries at p = (pi,pi,pi,pi)
    L = (4, 4, 4, 4)
    Hf = dense.dense_hw(L, (0, 0, 0, 0), MW, synth.su3_links(L, 0.0, 1))
    assert abs(np.abs(np.linalg.eigvalsh(Hf)).max() - 6.5) < 1e-12


def _gauge_rotate(L, U, x_list, seed):
    V = synth.volume(L)
    Om = synth.su3_field(V, 1.0, np.random.default_rng(seed))
    X = synth.coords(L)
    Up = np.empty_like(U)
    for mu in range(4):
        Xn = X.copy()
        Xn[:, mu] = (Xn[:, mu] + 1) % L[mu]
        jn = Xn[:, 0] + L[0] * (Xn[:, 1] + L[1] * (Xn[:, 2] + L[2] * Xn[:, 3]))
        Up[mu] = Om @ U[mu] @ Om[jn].conj().transpose(0, 2, 1)
    xs = [np.einsum("iab,isb->isa", Om, x) for x in x_list]
    return Up, xs


def test_gauge_covariance_dslash_and_sign():
    L = (4, 4, 2, 4)
    bc = (2, 0, 0, 1)
    U = synth.su3_links(L, 0.4, 9)
    x = synth.gaussian_spinors(L, 1, 1)[0]
    Vs = synth.random_orthonormal(L, 3, 8)
    Up, (xp, *Vp) = _gauge_rotate(L, U, [x, *Vs], 21)
    lat, latp = api.Lattice(L, bc, MW, U, 0.2), api.Lattice(L, bc, MW, Up, 0.2)
    _, (Dx_rot,) = _gauge_rotate(L, U, [api.dslash(lat, x)], 21)
    assert _rel(api.dslash(latp, xp), Dx_rot) < 1e-13
    lam = np.array([0.3, -0.2, 0.1])
    sp, spp = api.SignParams(20, 0.05, 6.5, Vs, lam), api.SignParams(20, 0.05, 6.5, np.stack(Vp), lam)
    _, (sx_rot,) = _gauge_rotate(L, U, [api.sign(lat, sp, x)], 21)
    assert _rel(api.sign(latp, spp, xp), sx_rot) < 1e-12


# ---------------------------------------------------------------- polynomial
@pytest.mark.parametrize("n,eps", [(13, 0.0036), (100, 0.01), (300, 1.234e-3)])
def test_cheb_interpolates_at_nodes(n, eps):
    c = api.cheb_coeffs(n, eps)
    j = np.arange(n + 1)
    y = ((1 - eps) * np.cos(np.pi * (j + 0.5) / (n + 1)) + 1 + eps) / 2
    P = np.array([api.cheb_eval(n, eps, c, yy) for yy in y])
    assert np.abs(P * np.sqrt(y) - 1).max() < 1e-11
    # the scalar Clenshaw agrees with numpy's Chebyshev series
    t = (2 * y - 1 - eps) / (1 - eps)
    assert np.allclose(P, np.polynomial.chebyshev.chebval(t, c), rtol=1e-12)


def test_eq2_error_law_and_fit():
    """delta(n, eps) of the interpolant follows eq. (2): within 3x, slope b in [1.9, 2.2]."""
    gold = json.load(open(GOLD))["eq2_constants"]
    xs, ys = [], []
    for se in (0.03, 0.06, 0.1):
        for n in (20, 40, 60, 80, 100):
            if n * se > 10.5:
                continue
            d = api.cheb_delta(n, se * se, npts=1501)
            bound = api.eq2_delta(n, se * se, gold["A"], gold["b"])
            assert d <= 3 * bound, (n, se, d, bound)
            xs.append(n * se)
            ys.append(np.log(d))
    slope = -np.polyfit(xs, ys, 1)[0]
    assert 1.9 <= slope <= 2.2, slope


def test_paper_worked_example():
    gold = json.load(open(GOLD))
    A, b = gold["eq2_constants"]["A"], gold["eq2_constants"]["b"]
    we = gold["worked_example"]
    n = api.eq2_order(we["delta"], we["lambda_min"], A, b)
    assert 0.5 * we["order_of_magnitude_n"] < n < 2 * we["order_of_magnitude_n"]
    f1 = gold["fig1"]
    d = api.eq2_delta(f1["n"], f1["sqrt_eps"] ** 2, A, b)
    assert 0.5 * f1["delta"] < d < 2 * f1["delta"]
    # the workload parameters target delta ~ 1e-10 as the worked example does
    assert abs(api.eq2_eps(1e-10, 100, A, b) - 0.0111) < 2e-4
    assert abs(api.eq2_eps(1e-10, 300, A, b) - 1.234e-3) < 1e-5


# ---------------------------------------------------------------- sign
def test_clenshaw_equals_spectral_image(lat44, dense44):
    n, eps, norm, l = 100, 0.01, 6.5, 8
    c = api.cheb_coeffs(n, eps)
    S, w, v, small = dense.spectral_sign(dense44, norm, n, eps, c, l)
    Vs, lam = dense.small_space(dense44, l)
    sp = api.SignParams(n, eps, norm, Vs, lam, c)
    x = synth.gaussian_spinors(lat44.L, 1, 7)[0]
    y = api.sign(lat44, sp, x)
    assert _rel(y, S @ x.ravel()) < 1e-13


def test_projection_with_non_eigen_basis():
    """s = V S V^dag + Pi Q P(Q^2) Pi for an arbitrary orthonormal V."""
    L = (2, 2, 2, 4)
    U = synth.su3_links(L, 0.5, 4)
    lat = api.Lattice(L, (2, 0, 0, 2), MW, U, 0.1)
    H = dense.dense_hw(L, lat.bc, MW, U, 0.1)
    n, eps, norm = 40, 0.02, 6.5
    c = api.cheb_coeffs(n, eps)
    Vs = synth.random_orthonormal(L, 5, 3)
    lam = np.array([0.5, -0.1, 0.0, -2.0, 1.0])
    Qp, _, _, _ = dense.spectral_sign(H, norm, n, eps, c, 0)
    Vm = Vs.reshape(5, -1).T
    Pi = np.eye(Vm.shape[0]) - Vm @ Vm.conj().T
    S = Vm @ np.diag(np.where(lam >= 0, 1.0, -1.0)) @ Vm.conj().T + Pi @ Qp @ Pi
    x = synth.gaussian_spinors(L, 1, 9)[0]
    assert _rel(api.sign(lat, api.SignParams(n, eps, norm, Vs, lam, c), x), S @ x.ravel()) < 1e-13
    assert np.allclose(S, S.conj().T, atol=1e-13)


def _delta_eff(H, norm, n, eps, c, l):
    w = np.linalg.eigvalsh(H)
    big = np.argsort(np.abs(w))[l:]
    q = w[big] / norm
    t = (2 * q * q - 1 - eps) / (1 - eps)
    return np.abs(1 - np.abs(q) * np.polynomial.chebyshev.chebval(t, c)).max()


def test_sign_accuracy_and_gw(lat44, dense44):
    n, eps, norm, l = 100, 0.01, 6.5, 8
    c = api.cheb_coeffs(n, eps)
    Vs, lam = dense.small_space(dense44, l)
    sp = api.SignParams(n, eps, norm, Vs, lam, c)
    x = synth.gaussian_spinors(lat44.L, 1, 11)[0]
    s = api.sign(lat44, sp, x)
    d = _delta_eff(dense44, norm, n, eps, c, l)
    # the 9th |lambda| sits just below sqrt(eps)*norm, so delta_eff is ~2e-9 here
    assert d < 1e-8
    err = np.linalg.norm(s.ravel() - dense.exact_sign(dense44) @ x.ravel()) / np.linalg.norm(x)
    assert err <= 1.01 * d
    s2 = api.sign(lat44, sp, s)
    assert np.linalg.norm(s2 - x) / np.linalg.norm(x) <= 2.1 * d
    # Ginsparg-Wilson: g5 D + D g5 - D g5 D = g5 (1 - s^2) for D = 1 + g5 s
    D = lambda v: api.dov(lat44, sp, v)
    g5 = api.gamma5
    gw = g5(D(x)) + D(g5(x)) - D(g5(D(x)))
    # identity up to rounding, measured against |x| (both sides are O(delta))
    assert np.linalg.norm(gw - g5(x - s2)) / np.linalg.norm(x) < 1e-13
    assert np.linalg.norm(gw) / np.linalg.norm(x) <= 2.1 * d


def test_dov_spectrum_on_circle():
    L = (2, 2, 2, 2)
    U = synth.su3_links(L, 0.5, 12)
    lat = api.Lattice(L, (0, 0, 0, 1), MW, U)
    H = dense.dense_hw(L, lat.bc, MW, U)
    n, eps, norm, l = 60, 0.02, 6.5, 4
    c = api.cheb_coeffs(n, eps)
    Vs, lam = dense.small_space(H, l)
    sp = api.SignParams(n, eps, norm, Vs, lam, c)
    N = 12 * lat.V
    E = np.eye(N, dtype=complex).reshape(N, lat.V, 4, 3)
    Dm = api.dov(lat, sp, E).reshape(N, N).T
    ev = np.linalg.eigvals(Dm)
    d = _delta_eff(H, norm, n, eps, c, l)
    assert np.abs(np.abs(ev - 1) - 1).max() <= 2 * d + 1e-12
    # dagger is the adjoint
    Dd = api.dov(lat, sp, E, dagger=True).reshape(N, N).T
    assert np.abs(Dd - Dm.conj().T).max() < 1e-12
    # massive operator
    Dmm = api.dov(lat, sp, E, mass=0.05).reshape(N, N).T
    assert np.abs(Dmm - ((1 - 0.025) * Dm + 0.05 * np.eye(N))).max() < 1e-12


def test_small_space_is_wired_in():
    """alpha = 1 gives many modes with q^2 < eps: l = 8 misses them, l = 160 fixes them."""
    L = (4, 4, 4, 4)
    U = synth.su3_links(L, 1.0, 1111)
    lat = api.Lattice(L, (0, 0, 0, 1), MW, U)
    H = dense.dense_hw(L, lat.bc, MW, U)
    w = np.linalg.eigvalsh(H)
    n, eps, norm = 100, 0.01, 6.5
    assert np.sum((w / norm) ** 2 < eps) > 50
    c = api.cheb_coeffs(n, eps)
    Se = dense.exact_sign(H)
    x = synth.gaussian_spinors(L, 1, 2)[0]
    errs = {}
    for l in (8, 160):
        Vs, lam = dense.small_space(H, l)
        s = api.sign(lat, api.SignParams(n, eps, norm, Vs, lam, c), x)
        errs[l] = np.linalg.norm(s.ravel() - Se @ x.ravel()) / np.linalg.norm(x)
    d160 = _delta_eff(H, norm, n, eps, c, 160)
    assert errs[8] > 1e3 * d160
    assert errs[160] <= 1.01 * d160 + 1e-13


# ---------------------------------------------------------------- CG
@pytest.fixture(scope="module")
def cg_setup():
    L = (2, 2, 2, 4)
    U = synth.su3_links(L, 0.5, 31)
    lat = api.Lattice(L, (2, 0, 0, 2), MW, U, 2 / 3 * 1e-3)
    H = dense.dense_hw(L, lat.bc, MW, U, lat.qeta)
    n, eps, norm, l = 60, 0.02, 6.5, 6
    c = api.cheb_coeffs(n, eps)
    Vs, lam = dense.small_space(H, l)
    sp = api.SignParams(n, eps, norm, Vs, lam, c)
    S, _, _, _ = dense.spectral_sign(H, norm, n, eps, c, l)
    return lat, sp, S


@pytest.mark.parametrize("mass", [0.02, 0.1])
def test_cg_equals_dense_solve(cg_setup, mass):
    lat, sp, S = cg_setup
    b = synth.point_sources(lat.L, (1, 0, 0, 2))[4]
    x, it, rr = api.cg(lat, sp, b, mass, tol=1e-12)
    assert rr <= 1e-12 and it > 0
    Dm = dense.dense_dm(S, mass)
    xd = np.linalg.solve(Dm, b.ravel())
    assert _rel(x, xd) < 1e-9


def test_cg_deflation_and_restart(cg_setup):
    lat, sp, S = cg_setup
    mass = 0.02
    b = synth.gaussian_spinors(lat.L, 1, 5)[0]
    Dm = dense.dense_dm(S, mass)
    A = Dm.conj().T @ Dm
    w, v = np.linalg.eigh(A)
    W = np.ascontiguousarray(v[:, :8].T.reshape(8, lat.V, 4, 3))
    x0, it0, _ = api.cg(lat, sp, b, mass, tol=1e-11)
    x1, it1, rr1 = api.cg(lat, sp, b, mass, W=W, tol=1e-11)
    assert rr1 <= 1e-11 and it1 < it0
    assert _rel(x1, x0) < 1e-8
    # restart from a partially converged iterate gives the same solution
    xh, _, _ = api.cg(lat, sp, b, mass, tol=1e-3)
    x2, _, rr2 = api.cg(lat, sp, b, mass, x0=xh, tol=1e-11)
    assert rr2 <= 1e-11 and _rel(x2, x0) < 1e-8


# ---------------------------------------------------------------- backward
@pytest.mark.parametrize("L,bc,l", [((2, 2, 2, 2), (0, 0, 0, 1), 0), ((2, 2, 2, 4), (2, 0, 0, 2), 4)])
def test_sign_backward_finite_differences(L, bc, l):
    q, eta = 2 / 3, 0.05
    U = synth.su3_links(L, 0.4, 41)
    lat = api.Lattice(L, bc, MW, U, q * eta)
    n, eps, norm = 24, 0.03, 6.5
    Vs = synth.random_orthonormal(L, l, 2) if l else None
    lam = np.linspace(-1, 1, l) if l else None
    sp = api.SignParams(n, eps, norm, Vs, lam)
    x, g = synth.gaussian_spinors(L, 2, 13)
    gU, geta, gx = api.sign_backward(lat, sp, q, x, g)

    def loss(U_, eta_):
        return np.real(api.vdot(g, api.sign(api.Lattice(L, bc, MW, U_, q * eta_), sp, x)))

    h = 1e-6
    fd_eta = (loss(U, eta + h) - loss(U, eta - h)) / (2 * h)
    assert abs(fd_eta - geta) <= 1e-7 * max(abs(geta), 1e-3)
    X = synth.random_algebra_field(L, 77)
    from scipy.linalg import expm
    E = np.stack([[expm(1j * h * X[mu, i]) for i in range(lat.V)] for mu in range(4)])
    Em = np.stack([[expm(-1j * h * X[mu, i]) for i in range(lat.V)] for mu in range(4)])
    fd_U = (loss(E @ U, eta) - loss(Em @ U, eta)) / (2 * h)
    an_U = np.sum(np.real(np.einsum("mvab,mvab->", gU.conj(), 1j * X @ U)))
    assert abs(fd_U - an_U) <= 1e-7 * abs(an_U)
    # d/dx of Re<g, s x> is s g
    assert _rel(gx, api.sign(lat, sp, g)) < 1e-14
