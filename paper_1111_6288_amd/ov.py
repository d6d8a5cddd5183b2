"""Thin ctypes binding of ``libov.so`` (the C ABI declared in include/ov.h).

Argument marshalling only: every operation runs in the HIP library.  Torch
supplies device memory (complex128 CUDA tensors in the canonical layouts) and
the stream.  If ``libov.so`` is missing this module raises at import time;
there is no fallback path.

Two layers:

* ``lib`` -- the raw ``ov_*`` functions with ctypes signatures;
* ``Context`` -- one lattice context, methods named like the C entry points
  without the ``ov_`` prefix (``ctx.dslash``, ``ctx.sign_apply``,
  ``ctx.dov_apply``, ``ctx.deflated_cg``, ``ctx.sign_backward`` ...).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libov.so")

OV_OK, OV_EINVAL, OV_ENOMEM, OV_EHIP, OV_ENOCONV, OV_ENAN, OV_ESTATE, OV_ENORM = 0, -1, -2, -3, -4, -5, -6, -7
OV_EBREAKDOWN = -8
OV_FP64, OV_FP32, OV_BF16 = 0, 1, 2
OV_PERIODIC, OV_ANTIPERIODIC, OV_DIRICHLET = 0, 1, 2
OV_OP_DW, OV_OP_HW = 0, 1
PREC = {"fp64": OV_FP64, "fp32": OV_FP32, "bf16": OV_BF16}
STATUS = {0: "OV_OK", -1: "OV_EINVAL", -2: "OV_ENOMEM", -3: "OV_EHIP", -4: "OV_ENOCONV",
          -5: "OV_ENAN", -6: "OV_ESTATE", -7: "OV_ENORM", -8: "OV_EBREAKDOWN"}


class OvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("inner_prec", C.c_int),
                ("inner_tol", C.c_double), ("max_restarts", C.c_int), ("use_deflation", C.c_int)]


class CgReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("relres", C.c_double), ("status", C.c_int)]


class EigOpts(C.Structure):
    _fields_ = [("l", C.c_int), ("k", C.c_int), ("cheb_order", C.c_int), ("cutoff", C.c_double),
                ("max_iter", C.c_int), ("tol", C.c_double), ("prec", C.c_int)]


class EigReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("hw_applies", C.c_long), ("max_resid", C.c_double)]


class MscgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("adaptive", C.c_int), ("min_order", C.c_int),
                ("refine", C.c_int), ("inner_prec", C.c_int)]


class MscgReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("sign_applies", C.c_long), ("dslash_applies", C.c_long),
                ("refine_iters", C.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libov.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_1111_6288_amd.build` (needs hipcc)")
    L = C.CDLL(LIB_PATH)
    vp, i, d, cp = C.c_void_p, C.c_int, C.c_double, C.POINTER
    sig = {
        "ov_create": ([cp(C.c_int32), cp(C.c_int32), d, i, cp(vp)], i),
        "ov_destroy": ([vp], i),
        "ov_set_stream": ([vp, vp], i),
        "ov_last_error": ([vp], C.c_char_p),
        "ov_upload_gauge": ([vp, vp], i),
        "ov_set_link_reconstruct": ([vp, i], i),
        "ov_get_link_format": ([vp, cp(i), cp(d)], i),
        "ov_set_fields": ([vp, i, cp(d), cp(d)], i),
        "ov_set_field_eta": ([vp, i, d, d], i),
        "ov_set_sign_params": ([vp, i, d, d, cp(d)], i),
        "ov_upload_eigvecs": ([vp, i, i, vp, cp(d)], i),
        "ov_upload_deflation": ([vp, i, i, vp], i),
        "ov_dslash": ([vp, i, i, i, cp(i), vp, vp], i),
        "ov_sign_apply": ([vp, i, i, cp(i), vp, vp], i),
        "ov_dov_apply": ([vp, i, i, cp(i), cp(d), i, vp, vp], i),
        "ov_deflated_cg": ([vp, i, cp(i), cp(d), vp, vp, cp(CgOpts), cp(CgReport)], i),
        "ov_sign_backward": ([vp, i, vp, vp, vp, cp(d), vp, i], i),
        "ov_hw_eigensolve": ([vp, i, cp(EigOpts), vp, vp, cp(d), cp(d), i, cp(EigReport)], i),
        "ov_dense_heev": ([i, cp(d), cp(d), cp(d)], i),
        "ov_multishift_cg": ([vp, i, cp(i), i, cp(d), vp, vp, cp(MscgOpts), cp(MscgReport), cp(d)], i),
        "ov_dov_eigensolve": ([vp, i, i, cp(EigOpts), vp, vp, cp(d), cp(d), i, cp(EigReport)], i),
        "ov_timeslice_norm2": ([vp, i, vp, cp(d)], i),
        "ov_correlator_deta": ([vp, i, d, i, vp, cp(d), cp(d), cp(d), cp(CgOpts)], i),
        "ov_prof_enable": ([vp, i], i),
        "ov_prof_query": ([vp, C.c_char_p, cp(C.c_long), cp(d), cp(d)], i),
        "ov_set_tuning": ([vp, i, i, i], i),
        "ov_get_tuning": ([vp, i, cp(i), cp(i)], i),
        "ov_autotune": ([vp, i, i, C.c_char_p], i),
        "ov_memory_used": ([vp, cp(C.c_int64)], i),
        "ov_set_graphs": ([vp, i], i),
        "ov_set_site_order": ([vp, i, i], i),
        "ov_set_occupancy": ([vp, i, i], i),
        "ov_get_launch_config": ([vp, i, i, cp(i)], i),
        "ov_set_launch_config": ([vp, i, i, cp(i)], i),
        "ov_dslash_noalloc": ([vp, i, i, i, cp(i), vp, vp], i),
        "ov_set_norm_check": ([vp, i], i),
        "ov_norm_status": ([vp], i),
        "ov_get_sign_norm": ([vp, i, cp(d)], i),
        "ov_pion_correlator": ([vp, i, vp, cp(d)], i),
        "ov_ratio_R": ([i, i, cp(d), cp(d), cp(d)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()
EXPORTED = ("ov_create", "ov_destroy", "ov_set_stream", "ov_last_error", "ov_upload_gauge", "ov_set_fields",
            "ov_set_field_eta",
            "ov_set_sign_params", "ov_upload_eigvecs", "ov_upload_deflation", "ov_dslash", "ov_sign_apply",
            "ov_dov_apply", "ov_deflated_cg", "ov_sign_backward", "ov_prof_enable", "ov_prof_query",
            "ov_set_tuning", "ov_get_tuning", "ov_autotune", "ov_memory_used", "ov_set_graphs",
            "ov_set_site_order", "ov_set_occupancy", "ov_get_launch_config",
            "ov_set_launch_config", "ov_hw_eigensolve", "ov_dense_heev", "ov_multishift_cg",
            "ov_dov_eigensolve", "ov_timeslice_norm2", "ov_correlator_deta", "ov_set_link_reconstruct",
            "ov_get_link_format", "ov_dslash_noalloc", "ov_set_norm_check", "ov_norm_status", "ov_get_sign_norm",
            "ov_pion_correlator", "ov_ratio_R")


def _ints(v):
    v = [int(a) for a in v]
    return (C.c_int * len(v))(*v)


def _doubles(v):
    v = [float(a) for a in v]
    return (C.c_double * len(v))(*v)


def _dev(t, shape_tail, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128 (canonical layout)")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected (..., {shape_tail})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def dense_heev(A):
    """Eigen-decomposition of a Hermitian matrix by the library's host Jacobi routine
    (ov_dense_heev): returns (ascending eigenvalues, eigenvectors as columns)."""
    import numpy as np
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Af = np.ascontiguousarray(A.T).view(np.float64)          # column-major, interleaved
    w = np.zeros(n)
    Z = np.zeros(2 * n * n)
    rc = lib.ov_dense_heev(n, Af.ctypes.data_as(C.POINTER(C.c_double)), w.ctypes.data_as(C.POINTER(C.c_double)),
                           Z.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError("ov_dense_heev: bad argument")
    return w, Z.view(np.complex128).reshape(n, n).T.copy()


def ratio_R(G_E_all, G_0):
    """R(t) = mean_e G_E_all[e](t) / G_0(t) (ov_ratio_R, Sec. 4): G_E_all holds the correlators of the
    field runs (u and d at +E and -E), G_0 the one without field."""
    import numpy as np
    ge = np.ascontiguousarray(np.atleast_2d(np.asarray(G_E_all, dtype=np.float64)))
    g0 = np.ascontiguousarray(np.asarray(G_0, dtype=np.float64))
    lt = int(g0.shape[0])
    if ge.shape[1] != lt:
        raise ValueError(f"G_E_all has {ge.shape[1]} time slices, G_0 has {lt}")
    out = np.zeros(lt)
    pd = C.POINTER(C.c_double)
    rc = lib.ov_ratio_R(lt, int(ge.shape[0]), ge.ctypes.data_as(pd), g0.ctypes.data_as(pd), out.ctypes.data_as(pd))
    if rc != OV_OK:
        raise OvError(rc, "ov_ratio_R: bad correlators")
    return out


class Context:
    """One lattice on one GPU: links, background fields, sign parameters, small spaces."""

    def __init__(self, L, bc, mw, device=0, stream=None):
        self.L = tuple(int(v) for v in L)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.device = int(device)
        h = C.c_void_p()
        rc = lib.ov_create((C.c_int32 * 4)(*self.L), (C.c_int32 * 4)(*[int(b) for b in bc]), float(mw),
                           self.device, C.byref(h))
        if rc != OV_OK or not h.value:
            raise OvError(rc, f"ov_create failed for L={self.L}, bc={tuple(bc)}")
        self._h = h
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.set_stream(stream)

    # ------------------------------------------------------------ plumbing
    def _chk(self, rc):
        if rc != OV_OK:
            raise OvError(rc, lib.ov_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            lib.ov_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        return self._chk(lib.ov_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def set_graphs(self, on):
        return self._chk(lib.ov_set_graphs(self._h, int(bool(on))))

    def memory_used(self):
        b = C.c_int64()
        self._chk(lib.ov_memory_used(self._h, C.byref(b)))
        return b.value

    # ------------------------------------------------------------ setup
    def upload_gauge(self, U):
        return self._chk(lib.ov_upload_gauge(self._h, _dev(U, (4, self.V, 3, 3), "U")))

    def set_link_reconstruct(self, enable=True):
        """Allow (default) or forbid the two-row SU(3) link kernels."""
        return self._chk(lib.ov_set_link_reconstruct(self._h, 1 if enable else 0))

    def link_format(self):
        """(two-row kernels in use, measured max |u_2 - conj(u_0 x u_1)| of the links)."""
        r, dev = C.c_int(0), C.c_double(0)
        self._chk(lib.ov_get_link_format(self._h, C.byref(r), C.byref(dev)))
        return bool(r.value), dev.value

    def set_fields(self, q, eta):
        q, eta = list(q), list(eta)
        return self._chk(lib.ov_set_fields(self._h, len(q), _doubles(q), _doubles(eta)))

    def set_field_eta(self, field, q, eta):
        return self._chk(lib.ov_set_field_eta(self._h, int(field), float(q), float(eta)))

    def set_sign_params(self, n, eps, norm=0.0, coeffs=None):
        cp = _doubles(coeffs) if coeffs is not None else None
        return self._chk(lib.ov_set_sign_params(self._h, int(n), float(eps), float(norm), cp))

    def upload_eigvecs(self, field, V, lam):
        l = 0 if V is None else int(V.shape[0])
        ptr = _dev(V, (self.V, 4, 3), "V") if l else None
        return self._chk(lib.ov_upload_eigvecs(self._h, int(field), l, ptr, _doubles(lam) if l else None))

    def upload_deflation(self, field, W):
        k = 0 if W is None else int(W.shape[0])
        ptr = _dev(W, (self.V, 4, 3), "W") if k else None
        return self._chk(lib.ov_upload_deflation(self._h, int(field), k, ptr))

    # ------------------------------------------------------------ operators
    def _io(self, x, fields):
        if x.dim() == 3:
            x = x.unsqueeze(0)
        n = int(x.shape[0])
        fields = [0] * n if fields is None else list(fields)
        if len(fields) != n:
            raise ValueError("fields must have one entry per RHS")
        return x, n, fields

    def dslash(self, x, fields=None, op="HW", prec="fp64"):
        x, n, fields = self._io(x, fields)
        y = torch.empty_like(x)
        opc = OV_OP_HW if op == "HW" else OV_OP_DW
        self._chk(lib.ov_dslash(self._h, PREC[prec], opc, n, _ints(fields), _dev(x, (self.V, 4, 3), "x"),
                                _dev(y, (self.V, 4, 3), "y")))
        return y

    def sign_apply(self, x, fields=None, prec="fp64"):
        x, n, fields = self._io(x, fields)
        y = torch.empty_like(x)
        self._chk(lib.ov_sign_apply(self._h, PREC[prec], n, _ints(fields), _dev(x, (self.V, 4, 3), "x"),
                                    _dev(y, (self.V, 4, 3), "y")))
        return y

    def dov_apply(self, x, fields=None, mass=None, dagger=False, prec="fp64", out=None):
        x, n, fields = self._io(x, fields)
        mass = [0.0] * n if mass is None else list(mass)
        y = torch.empty_like(x) if out is None else out
        self._chk(lib.ov_dov_apply(self._h, PREC[prec], n, _ints(fields), _doubles(mass), int(bool(dagger)),
                                   _dev(x, (self.V, 4, 3), "x"), _dev(y, (self.V, 4, 3), "y")))
        return y

    def deflated_cg(self, b, fields=None, mass=None, x0=None, tol=1e-10, maxiter=10000, inner_prec="fp32",
                    inner_tol=1e-5, max_restarts=50, use_deflation=True, raise_on_noconv=True):
        b, n, fields = self._io(b, fields)
        mass = [0.0] * n if mass is None else list(mass)
        x = torch.zeros_like(b) if x0 is None else x0.clone().reshape(b.shape).contiguous()
        opts = CgOpts(float(tol), int(maxiter), PREC[inner_prec], float(inner_tol), int(max_restarts),
                      int(bool(use_deflation)))
        rep = (CgReport * n)()
        rc = lib.ov_deflated_cg(self._h, n, _ints(fields), _doubles(mass), _dev(b, (self.V, 4, 3), "b"),
                                _dev(x, (self.V, 4, 3), "x"), C.byref(opts), rep)
        report = [dict(iters=r.iters, restarts=r.restarts, relres=r.relres, status=r.status) for r in rep]
        if rc != OV_OK and not (rc == OV_ENOCONV and not raise_on_noconv):
            self._chk(rc)
        return x, report

    def sign_backward(self, field, x, g, want_U=True, want_eta=True, want_x=True, ckpt_every=32):
        x = x.reshape(self.V, 4, 3).contiguous()
        g = g.reshape(self.V, 4, 3).contiguous()
        gU = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device=x.device) if want_U else None
        gx = torch.empty_like(x) if want_x else None
        ge = C.c_double(0.0)
        self._chk(lib.ov_sign_backward(self._h, int(field), _dev(x, (self.V, 4, 3), "x"),
                                       _dev(g, (self.V, 4, 3), "g"),
                                       _dev(gU, (4, self.V, 3, 3), "gU") if want_U else None,
                                       C.byref(ge) if want_eta else None,
                                       _dev(gx, (self.V, 4, 3), "gx") if want_x else None, int(ckpt_every)))
        return gU, (ge.value if want_eta else None), gx

    def multishift_cg(self, b, masses, fields=None, tol=1e-10, maxiter=5000, adaptive=True, min_order=20,
                      refine=True, inner_prec="fp64", raise_on_noconv=True):
        """x[i] = D(masses[i])^{-1} b for chiral sources b (ov_multishift_cg).
        Returns (x (nmass, nrhs, V, 4, 3), relres (nmass, nrhs), report)."""
        b, n, fields = self._io(b, fields)
        nm = len(masses)
        x = torch.empty((nm,) + tuple(b.shape), dtype=torch.complex128, device=b.device)
        rel = (C.c_double * (nm * n))()
        rep = MscgReport()
        opts = MscgOpts(float(tol), int(maxiter), int(bool(adaptive)), int(min_order), int(bool(refine)),
                        PREC[inner_prec])
        rc = lib.ov_multishift_cg(self._h, n, _ints(fields), nm, _doubles(masses), _dev(b, (self.V, 4, 3), "b"),
                                  C.c_void_p(x.data_ptr()), C.byref(opts), C.byref(rep), rel)
        if rc != OV_OK and not (rc == OV_ENOCONV and not raise_on_noconv):
            self._chk(rc)
        report = dict(iters=rep.iters, sign_applies=rep.sign_applies, dslash_applies=rep.dslash_applies,
                      refine_iters=rep.refine_iters, status=rc)
        import numpy as np
        return x, np.array(list(rel)).reshape(nm, n), report

    def dov_eigensolve(self, field, chirality, l, k=None, cheb_order=12, cutoff=0.0, max_iter=30, tol=1e-10,
                       prec="fp64", x0=None, seed=0, install=False, raise_on_noconv=True):
        """Lowest eigenpairs of D_ov^dag D_ov in one chirality sector (ov_dov_eigensolve).
        Returns (lambda, resid, W (l, V, 4, 3), report)."""
        k = int(k if k is not None else l + max(4, l // 4))
        if x0 is None:
            dev = f"cuda:{self.device}"
            gen = torch.Generator(device=dev)
            gen.manual_seed(int(seed))
            x0 = torch.randn((k, self.V, 4, 3), dtype=torch.complex128, device=dev, generator=gen)
        x0 = x0.reshape(k, self.V, 4, 3).contiguous()
        W = torch.empty((l, self.V, 4, 3), dtype=torch.complex128, device=x0.device)
        lam = (C.c_double * l)()
        res = (C.c_double * l)()
        rep = EigReport()
        opts = EigOpts(int(l), k, int(cheb_order), float(cutoff), int(max_iter), float(tol), PREC[prec])
        rc = lib.ov_dov_eigensolve(self._h, int(field), int(chirality), C.byref(opts),
                                   _dev(x0, (self.V, 4, 3), "x0"), _dev(W, (self.V, 4, 3), "W"), lam, res,
                                   int(bool(install)), C.byref(rep))
        if rc != OV_OK and not (rc == OV_ENOCONV and not raise_on_noconv):
            self._chk(rc)
        report = dict(iters=rep.iters, sign_applies=rep.hw_applies, max_resid=rep.max_resid, status=rc)
        return list(lam), list(res), W, report

    def timeslice_norm2(self, x):
        """out[j, t] = sum over time slice t of |x_j|^2 (ov_timeslice_norm2); numpy (nrhs, Lt)."""
        import numpy as np
        x = x.reshape(-1, self.V, 4, 3).contiguous()
        n = int(x.shape[0])
        out = np.zeros(n * self.L[3])
        self._chk(lib.ov_timeslice_norm2(self._h, n, _dev(x, (self.V, 4, 3), "x"),
                                         out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(n, self.L[3])

    def correlator_deta(self, b, field, mass, weights, tol=1e-10, inner_prec="fp32"):
        """(C(t), dF/deta) with F = sum_t weights[t] C(t) for the propagators of sources b
        (ov_correlator_deta)."""
        import numpy as np
        b = b.reshape(-1, self.V, 4, 3).contiguous()
        n = int(b.shape[0])
        Ct = np.zeros(self.L[3])
        w = np.ascontiguousarray(weights, dtype=np.float64)
        dF = C.c_double(0.0)
        opts = CgOpts(float(tol), 10000, PREC[inner_prec], 1e-5, 50, 1)
        self._chk(lib.ov_correlator_deta(self._h, int(field), float(mass), n, _dev(b, (self.V, 4, 3), "b"),
                                         w.ctypes.data_as(C.POINTER(C.c_double)),
                                         Ct.ctypes.data_as(C.POINTER(C.c_double)), C.byref(dF), C.byref(opts)))
        return Ct, dF.value

    def pion_correlator(self, props):
        """Connected pseudoscalar correlator of one flavour (ov_pion_correlator): G(t) = sum over the
        point-source propagators (props: (nsrc, V, 4, 3)) and the sink spin-colour of |S|^2."""
        import numpy as np
        props = props.reshape(-1, self.V, 4, 3).contiguous()
        G = np.zeros(self.L[3])
        self._chk(lib.ov_pion_correlator(self._h, int(props.shape[0]), _dev(props, (self.V, 4, 3), "props"),
                                         G.ctypes.data_as(C.POINTER(C.c_double))))
        return G

    def dslash_noalloc(self, x, fields=None, op="HW", prec="fp64", out=None):
        """ov_dslash on the library's fixed scratch array (no device allocation inside the call)."""
        x, n, fields = self._io(x, fields)
        y = torch.empty_like(x) if out is None else out
        opc = OV_OP_HW if op == "HW" else OV_OP_DW
        self._chk(lib.ov_dslash_noalloc(self._h, PREC[prec], opc, n, _ints(fields), _dev(x, (self.V, 4, 3), "x"),
                                        _dev(y, (self.V, 4, 3), "y")))
        return y

    def set_norm_check(self, mode):
        """0: off; 1: breaches reported by synchronising calls and norm_status(); 2 (default): sign and
        D(m) applies also synchronise and raise OV_ENORM."""
        return self._chk(lib.ov_set_norm_check(self._h, int(mode)))

    def norm_status(self):
        """Raise OvError(OV_ENORM) if a sign application since the last check exceeded its growth bound."""
        return self._chk(lib.ov_norm_status(self._h))

    def sign_norm(self, prec="fp64"):
        """Norm the sign pipeline of `prec` divides H_w by (the set norm plus the link-rounding margin)."""
        v = C.c_double(0.0)
        self._chk(lib.ov_get_sign_norm(self._h, PREC[prec], C.byref(v)))
        return v.value

    def hw_eigensolve(self, field, l, k=None, cheb_order=60, cutoff=0.0, max_iter=20, tol=1e-10, prec="fp64",
                      x0=None, seed=0, install=True, want_vectors=True, raise_on_noconv=True):
        """Lowest-|lambda| eigenpairs of H_w for field group `field` (ov_hw_eigensolve).

        x0: (k, V, 4, 3) complex128 start block on the device; by default seeded Gaussian
        numbers drawn here.  Returns (lambda, resid, V or None, report)."""
        k = int(k if k is not None else l + max(4, l // 4))
        if x0 is None:
            dev = f"cuda:{self.device}"
            gen = torch.Generator(device=dev)
            gen.manual_seed(int(seed))
            x0 = torch.randn((k, self.V, 4, 3), dtype=torch.complex128, device=dev, generator=gen)
        x0 = x0.reshape(k, self.V, 4, 3).contiguous()
        V = torch.empty((l, self.V, 4, 3), dtype=torch.complex128, device=x0.device) if want_vectors else None
        lam = (C.c_double * l)()
        res = (C.c_double * l)()
        rep = EigReport()
        opts = EigOpts(int(l), k, int(cheb_order), float(cutoff), int(max_iter), float(tol), PREC[prec])
        rc = lib.ov_hw_eigensolve(self._h, int(field), C.byref(opts), _dev(x0, (self.V, 4, 3), "x0"),
                                  _dev(V, (self.V, 4, 3), "V") if want_vectors else None, lam, res,
                                  int(bool(install)), C.byref(rep))
        if rc != OV_OK and not (rc == OV_ENOCONV and not raise_on_noconv):
            self._chk(rc)
        report = dict(iters=rep.iters, hw_applies=rep.hw_applies, max_resid=rep.max_resid, status=rc)
        return list(lam), list(res), V, report

    # ------------------------------------------------------------ measurement and tuning
    def prof_enable(self, on=True):
        return self._chk(lib.ov_prof_enable(self._h, int(bool(on))))

    def prof_query(self, cls):
        n, ms, by = C.c_long(), C.c_double(), C.c_double()
        self._chk(lib.ov_prof_query(self._h, cls.encode(), C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def set_tuning(self, prec, rhs_per_thread, block):
        return self._chk(lib.ov_set_tuning(self._h, PREC[prec], int(rhs_per_thread), int(block)))

    def set_site_order(self, prec, order):
        return self._chk(lib.ov_set_site_order(self._h, PREC[prec], int(order)))

    def set_occupancy(self, prec, blocks_per_cu):
        return self._chk(lib.ov_set_occupancy(self._h, PREC[prec], int(blocks_per_cu)))

    _KIND = {"dslash": 0, "clenshaw": 1}
    _CFG = ("rhs_per_thread", "block", "site_order", "blocks_per_cu", "stream_hint", "rhs_split", "cols", "wshare")

    def get_launch_config(self, prec, kind="dslash"):
        """Launch shape of the plain ("dslash") or fused-epilogue ("clenshaw") launches of prec."""
        cfg = (C.c_int * len(self._CFG))()
        self._chk(lib.ov_get_launch_config(self._h, PREC[prec], self._KIND[kind], cfg))
        return dict(zip(self._CFG, list(cfg)))

    def set_launch_config(self, prec, kind, **cfg):
        """Set fields of one kind's launch shape; fields not given keep their value."""
        cur = self.get_launch_config(prec, kind)
        for k, v in cfg.items():
            if k not in cur:
                raise KeyError(k)
            cur[k] = int(v)
        arr = (C.c_int * len(self._CFG))(*[cur[k] for k in self._CFG])
        return self._chk(lib.ov_set_launch_config(self._h, PREC[prec], self._KIND[kind], arr))

    def get_tuning(self, prec):
        a, b = C.c_int(), C.c_int()
        self._chk(lib.ov_get_tuning(self._h, PREC[prec], C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, prec, nrhs, cache_path=None):
        return self._chk(lib.ov_autotune(self._h, PREC[prec], int(nrhs),
                                         cache_path.encode() if cache_path else None))

    def load_tuning(self, path, prec, nrhs):
        """Apply the launch shapes recorded by autotune (one JSON object per line) for this
        lattice, precision, batch size and link format (records without a format match
        either); returns the kinds applied (empty if none match)."""
        import json
        applied = []
        two_row = self.link_format()[0]
        try:
            lines = open(path).read().splitlines()
        except OSError:
            return applied
        for line in lines:
            if not line.strip():
                continue
            e = json.loads(line)
            if (e.get("arch") != "gfx950" or tuple(e.get("L", ())) != self.L or e.get("prec") != PREC[prec]
                    or e.get("nrhs") != int(nrhs) or e.get("kind") not in self._KIND
                    or bool(e.get("two_row_links", two_row)) != two_row):
                continue
            defaults = {"stream_hint": 0, "rhs_split": 1, "cols": 1, "wshare": 1}
            self.set_launch_config(prec, e["kind"], **{k: e.get(k, defaults.get(k)) for k in self._CFG
                                                       if k in e or k in defaults})
            applied.append(e["kind"])
        return applied
