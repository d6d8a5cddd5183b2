"""ctypes front end of the FP64 C oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use this module; the HIP product path never imports it.

All arrays are numpy complex128 in canonical layout (see ``synth``):
links (4, V, 3, 3), spinors (V, 4, 3), small space (l, V, 4, 3).
Boundary codes: 0 periodic, 1 antiperiodic, 2 Dirichlet.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OrField(C.Structure):
    _fields_ = [("L", C.c_int * 4), ("bc", C.c_int * 4), ("mw", C.c_double),
                ("qeta", C.c_double), ("U", C.c_void_p)]


class OrSignParams(C.Structure):
    _fields_ = [("n", C.c_int), ("eps", C.c_double), ("norm", C.c_double),
                ("c", C.c_void_p), ("l", C.c_int), ("V", C.c_void_p), ("lam", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=True)
        L = C.CDLL(path)
        vp, i, d = C.c_void_p, C.c_int, C.c_double
        L.or_gamma.argtypes = [i, vp]
        L.or_dslash.argtypes = [C.POINTER(OrField), i, vp, vp]
        L.or_gamma5.argtypes = [C.c_long, vp, vp]
        L.or_cheb_coeffs.argtypes = [i, d, vp]
        L.or_cheb_eval.argtypes = [i, d, vp, d]
        L.or_cheb_eval.restype = d
        L.or_sign.argtypes = [C.POINTER(OrField), C.POINTER(OrSignParams), vp, vp]
        L.or_dov.argtypes = [C.POINTER(OrField), C.POINTER(OrSignParams), d, i, vp, vp]
        L.or_cg.argtypes = [C.POINTER(OrField), C.POINTER(OrSignParams), d, i, vp, vp, vp,
                            d, i, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_sign_backward.argtypes = [C.POINTER(OrField), C.POINTER(OrSignParams), d,
                                       vp, vp, vp, C.POINTER(C.c_double), vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


class Lattice:
    """A gauge background: lattice size, boundary codes, Wilson mass, links, q*eta."""

    def __init__(self, L, bc, mw, U, qeta=0.0):
        self.L = tuple(int(v) for v in L)
        self.bc = tuple(int(v) for v in bc)
        self.mw = float(mw)
        self.U = _c128(U)
        self.qeta = float(qeta)
        self.V = int(np.prod(self.L))
        assert self.U.shape == (4, self.V, 3, 3)

    def with_qeta(self, qeta):
        return Lattice(self.L, self.bc, self.mw, self.U, qeta)

    def with_links(self, U):
        return Lattice(self.L, self.bc, self.mw, U, self.qeta)

    def cfield(self):
        f = OrField()
        f.L[:] = self.L
        f.bc[:] = self.bc
        f.mw = self.mw
        f.qeta = self.qeta
        f.U = _ptr(self.U)
        return f


class SignParams:
    """Polynomial degree n, interval eps, norm, coefficients and small space."""

    def __init__(self, n, eps, norm, V=None, lam=None, c=None):
        self.n, self.eps, self.norm = int(n), float(eps), float(norm)
        self.c = np.ascontiguousarray(c if c is not None else cheb_coeffs(n, eps), dtype=np.float64)
        if V is None or len(V) == 0:
            self.V = np.zeros((1, 1), np.complex128)
            self.lam = np.zeros(1)
            self.l = 0
        else:
            self.V = _c128(V)
            self.lam = np.ascontiguousarray(lam, dtype=np.float64)
            self.l = int(self.V.shape[0])

    def cparams(self):
        p = OrSignParams()
        p.n, p.eps, p.norm = self.n, self.eps, self.norm
        p.c = _ptr(self.c)
        p.l = self.l
        p.V = _ptr(self.V)
        p.lam = _ptr(self.lam)
        return p


def gamma(mu):
    g = np.zeros((4, 4), np.complex128)
    lib().or_gamma(mu, _ptr(g))
    return g


def dslash(lat: Lattice, x, op=0):
    """op=0: D_w x ; op=1: H_w x = gamma5 D_w x.  x: (V,4,3) or (n,V,4,3)."""
    x = _c128(x)
    if x.ndim == 4:
        return np.stack([dslash(lat, xi, op) for xi in x])
    y = np.empty_like(x)
    f = lat.cfield()
    lib().or_dslash(C.byref(f), op, _ptr(x), _ptr(y))
    return y


def gamma5(x):
    x = _c128(x)
    y = np.empty_like(x)
    lib().or_gamma5(x.size // 12, _ptr(x), _ptr(y))
    return y


def cheb_coeffs(n, eps):
    c = np.zeros(n + 1)
    lib().or_cheb_coeffs(int(n), float(eps), _ptr(c))
    return c


def cheb_eval(n, eps, c, y):
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().or_cheb_eval(int(n), float(eps), _ptr(c), float(y))


def sign(lat: Lattice, sp: SignParams, x):
    x = _c128(x)
    if x.ndim == 4:
        return np.stack([sign(lat, sp, xi) for xi in x])
    y = np.empty_like(x)
    f, p = lat.cfield(), sp.cparams()
    rc = lib().or_sign(C.byref(f), C.byref(p), _ptr(x), _ptr(y))
    if rc:
        raise RuntimeError(f"or_sign failed ({rc})")
    return y


def dov(lat: Lattice, sp: SignParams, x, mass=0.0, dagger=False):
    """D(m) x = (1 - m/2)(x + gamma5 s x) + m x, or its dagger gamma5 D(m) gamma5 x."""
    x = _c128(x)
    if x.ndim == 4:
        return np.stack([dov(lat, sp, xi, mass, dagger) for xi in x])
    y = np.empty_like(x)
    f, p = lat.cfield(), sp.cparams()
    rc = lib().or_dov(C.byref(f), C.byref(p), float(mass), int(bool(dagger)), _ptr(x), _ptr(y))
    if rc:
        raise RuntimeError(f"or_dov failed ({rc})")
    return y


def cg(lat: Lattice, sp: SignParams, b, mass, x0=None, W=None, tol=1e-12, maxiter=10000):
    """Solve D(m)^dag D(m) x = D(m)^dag b.  Returns (x, iterations, true relative residual)."""
    b = _c128(b)
    x = _c128(np.zeros_like(b) if x0 is None else x0).copy()
    k = 0 if W is None else int(len(W))
    Wa = _c128(W) if k else None
    it, rr = C.c_int(0), C.c_double(0)
    f, p = lat.cfield(), sp.cparams()
    lib().or_cg(C.byref(f), C.byref(p), float(mass), k, _ptr(Wa), _ptr(b), _ptr(x),
                float(tol), int(maxiter), C.byref(it), C.byref(rr))
    return x, it.value, rr.value


def sign_backward(lat: Lattice, sp: SignParams, q, x, g, want_U=True, want_eta=True, want_x=True):
    """Gradients of L = Re<g, s(U, eta) x>: (gU, geta, gx); geta is dL/deta for charge q."""
    x, g = _c128(x), _c128(g)
    gU = np.zeros((4, lat.V, 3, 3), np.complex128) if want_U else None
    gx = np.zeros_like(x) if want_x else None
    ge = C.c_double(0)
    f, p = lat.cfield(), sp.cparams()
    rc = lib().or_sign_backward(C.byref(f), C.byref(p), float(q), _ptr(x), _ptr(g), _ptr(gU),
                                C.byref(ge) if want_eta else None, _ptr(gx))
    if rc:
        raise RuntimeError(f"or_sign_backward failed ({rc})")
    return gU, (ge.value if want_eta else None), gx


def vdot(a, b):
    """<a, b> = sum conj(a) b over all components."""
    return np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel())


def eq2_delta(n, eps, A=0.41, b=2.1):
    """Empirical error law delta = A exp(-b n sqrt(eps)) (Sec. 2, eq. 2)."""
    return A * np.exp(-b * n * np.sqrt(eps))


def eq2_order(delta, sqrt_eps, A=0.41, b=2.1):
    """Polynomial order n for a target delta from eq. 2, inverted."""
    return np.log(A / delta) / (b * sqrt_eps)


def eq2_eps(delta, n, A=0.41, b=2.1):
    """Interval parameter eps for (delta, n) from eq. 2, inverted."""
    return (np.log(A / delta) / (b * n)) ** 2


def cheb_delta(n, eps, c=None, npts=4001):
    """max over y in [eps, 1] of |1 - sqrt(y) P(y)| on a Chebyshev-spaced grid."""
    c = cheb_coeffs(n, eps) if c is None else c
    t = np.cos(np.linspace(0, np.pi, npts))
    ys = ((1 - eps) * t + 1 + eps) / 2
    return max(abs(1 - np.sqrt(y) * cheb_eval(n, eps, c, y)) for y in ys)
