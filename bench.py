#!/usr/bin/env python3
"""Throughput of the overlap operator on one MI355X: D_ov applies per second.

Workload (24^3 x 48, the batched multi-RHS configuration): Dirichlet
boundaries in x and t, periodic in y and z; SU(3) links exp(i 0.2 H);
Wilson mass -1.5; sign(H_w) by an order-300 Chebyshev polynomial on
[1.234e-3, 1] (delta ~ 1e-10 by eq. (2)) with a 200-vector small space per
background field; 108 right-hand sides = 12 spin-colour point sources x
3 field strengths (q = 2/3, eta in {0, +1e-3, -1e-3}) x 3 quark masses
{0.01, 0.02, 0.05}.

One step = one D(m) application (alternately D and D^dag) to all 108 RHS in
the mixed path: FP32 Wilson dslash and Clenshaw recursion, FP64 small-space
projection.  value = 108 * steps / seconds.  The same batch is then run on
the FP64 path for the speedup at matched work, and the mixed result is
compared with the FP64 one per RHS.  The dominant kernel (dslash with the
fused Clenshaw epilogue) is timed live with HIP events on the library's
stream during the timed steps, for the roofline figure.

Small spaces are seeded random orthonormal bases (the eigensolver that would
produce real ones is not part of this path); they cost the same as
eigenvectors.  All data are synthetic.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# launch shapes recorded by ov_autotune for this workload on gfx950
TUNING_FILE = os.path.join(ROOT, "paper_1111_6288_amd", "tuning_gfx950.jsonl")
L = (24, 24, 24, 48)
BC = (2, 0, 0, 2)
MW = -1.5
NPOLY = 300
EPS = 1.234e-3
NORM = 6.5
LSMALL = 200
Q = 2.0 / 3.0
ETAS = (0.0, 1e-3, -1e-3)
MASSES = (0.01, 0.02, 0.05)
SRC = (12, 0, 0, 24)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--fp64-steps", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--lsmall", type=int, default=LSMALL)
    p.add_argument("--npoly", type=int, default=NPOLY)
    p.add_argument("--eig", action="store_true",
                   help="also time the H_w low-mode eigensolver at 24^3x48 (adds an 'eigensolver' object)")
    p.add_argument("--eig-l", type=int, default=LSMALL)
    p.add_argument("--no-tts", action="store_true",
                   help="skip the default time-to-solution comparison (mixed vs FP64 inner CG at 1e-10)")
    p.add_argument("--tts", action="store_true",
                   help="also time propagator methods at 16^3x32: per-mass CG vs multi-mass sector CG")
    p.add_argument("--tts-l", type=int, default=100)
    p.add_argument("--tts-ldov", type=int, default=16)
    p.add_argument("--eig-order", type=int, default=100)
    p.add_argument("--eig-k", type=int, default=256)
    p.add_argument("--eig-maxiter", type=int, default=12)
    p.add_argument("--autotune", action="store_true",
                   help="search the dslash launch shapes instead of applying the recorded ones")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 4 GiB device copy (3 times) to scale PMC byte counters")
    return p.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dslash.hip", "spin.h", "ov_device.h", "ov_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1111_6288_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def synth_volume():
    return L[0] * L[1] * L[2] * L[3]


def measured_traffic(prec, nrhs, tuned, two_row):
    """HBM bytes per launch of the Clenshaw kernel from committed rocprofv3 PMC runs, if they were
    taken on the current kernel source in the same launch configuration and link format."""
    path = os.path.join(ROOT, "profiles", "clenshaw_dslash_24x48_108rhs_pmc.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("prec") != prec or rec.get("nrhs") != nrhs:
        return None
    if bool(rec.get("two_row_links")) != bool(two_row):
        return None
    rt = dict(rec.get("tuning") or {})
    rt.setdefault("cols", 1)
    rt.setdefault("wshare", 1)
    if rt != tuned:
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_bandwidth(torch, nbytes=4 << 30, reps=5):
    """Best device bandwidth (bytes read + written per second) of a plain copy: the runtime's
    device-to-device copy and torch's elementwise neg over the same buffers, timed with events."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    srcf, dstf = src.view(torch.float32), dst.view(torch.float32)
    best = 0.0
    for op in (lambda: dst.copy_(src), lambda: torch.neg(srcf, out=dstf)):
        op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3))
    del src, dst, srcf, dstf
    torch.cuda.empty_cache()
    return best


def build_inputs(torch, ov, args):
    import synth

    V = synth.volume(L)
    t0 = time.time()
    U = synth.su3_links(L, 0.2, 2022)
    ctx = ov.Context(L, BC, MW, device=0)
    ctx.upload_gauge(torch.from_numpy(U).cuda())
    ctx.set_fields([Q] * len(ETAS), list(ETAS))
    ctx.set_sign_params(args.npoly, EPS, NORM)
    for f in range(len(ETAS)):
        Vs = synth.random_orthonormal_torch(L, args.lsmall, 500 + f, "cuda")
        lam = [(-1.0) ** i * (0.05 + 0.001 * i) for i in range(args.lsmall)]
        ctx.upload_eigvecs(f, Vs, lam)
        del Vs
        torch.cuda.empty_cache()
    fields, masses, idx = [], [], []
    for f in range(len(ETAS)):
        for m in MASSES:
            for s in range(12):
                fields.append(f)
                masses.append(m)
                idx.append(s)
    n = len(fields)
    x = torch.zeros((n, V, 4, 3), dtype=torch.complex128, device="cuda")
    site = synth.site_index(L, *SRC)
    for j, s in enumerate(idx):
        x[j, site, s // 3, s % 3] = 1.0
    torch.cuda.synchronize()
    return ctx, U, x, fields, masses, time.time() - t0


def timed_applies(torch, ctx, x, y, fields, masses, prec, steps, warmup, prof):
    """Times `steps` D(m) / D(m)^dag applications on the production path (each pipeline
    replayed from its captured HIP graph after its first two calls, no event records), then, with
    prof, runs one more application eagerly with per-kernel HIP events for the kernel statistics."""
    for w in range(warmup):
        ctx.dov_apply(x, fields, masses, dagger=bool(w % 2), prec=prec, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ctx.dov_apply(x, fields, masses, dagger=bool(k % 2), prec=prec, out=y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = {}
    if prof:
        ctx.prof_enable(True)
        ctx.dov_apply(x, fields, masses, dagger=False, prec=prec, out=y)
        for cls in ("clenshaw", "dslash", "proj_dot", "proj_expand", "blas"):
            stats[cls] = ctx.prof_query(cls)
        ctx.prof_enable(False)
    return dt, stats


def eig_measurement(torch, ov, U, args):
    """Lowest-|lambda| eigenpairs of H_w at 24^3 x 48 for one field group (q eta = 2/3 x 1e-3):
    Chebyshev-filtered subspace iteration, FP32 filter then FP64, to 1e-10 of the norm bound."""
    ctx = ov.Context(L, BC, MW)
    ctx.upload_gauge(torch.from_numpy(U).cuda())
    ctx.set_fields([Q] * len(ETAS), list(ETAS))
    ctx.set_sign_params(args.npoly, EPS, NORM)
    ctx.load_tuning(TUNING_FILE, "fp32", 108)
    ctx.load_tuning(TUNING_FILE, "fp64", 108)
    l, k = args.eig_l, max(args.eig_k, args.eig_l)
    print(f"[bench] eigensolver: l={l}, k={k}, order {args.eig_order}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.prof_enable(True)
    t0 = time.perf_counter()
    lam, res, _, rep = ctx.hw_eigensolve(1, l, k=k, cheb_order=args.eig_order, tol=1e-10, prec="fp32", seed=11,
                                         max_iter=args.eig_maxiter, install=False, want_vectors=False,
                                         raise_on_noconv=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = {cls: ctx.prof_query(cls) for cls in ("clenshaw", "dslash", "proj_dot", "proj_expand", "blas")}
    ctx.prof_enable(False)
    ctx.close()
    print(f"[bench] eigensolver: {rep['iters']} passes, {dt:.1f} s, max resid {rep['max_resid']:.2e}",
          file=sys.stderr, flush=True)
    return {"l": l, "k": k, "cheb_order": args.eig_order, "seconds": round(dt, 2), "passes": rep["iters"],
            "hw_applies": rep["hw_applies"], "hw_applies_per_s": round(rep["hw_applies"] / dt, 1),
            "converged": rep["status"] == 0, "max_resid_rel": rep["max_resid"] / NORM,
            "lambda_min_abs": min(abs(v) for v in lam), "lambda_max_abs": max(abs(v) for v in lam),
            "kernels_ms": {c: round(v[1], 1) for c, v in prof.items()}}


def tts_mixed_vs_fp64(torch, ov):
    """Time to solution at 1e-10 (Sec. 3.2: FP32 late in the solve, FP64 defect correction).

    16^3 x 32, Dirichlet x and t, one operator (q eta = 2/3 x 1e-3): the 64 lowest H_w modes
    from the eigensolver (timed apart), eps and the order n from eq. (2) for delta = 1e-10 at
    0.95 |lambda_64|, then 12 propagators (4 point sources x masses 0.05, 0.1, 0.2) in one batch
    to an FP64 true residual of 1e-10: with FP32 inner / FP64 outer CG, with BF16-storage inner /
    FP64 outer CG, and with FP64 inner CG.  Reports the times, the inner iterations, and per
    propagator the relative difference of the mixed and FP64 solutions and the FP64 residuals
    reached."""
    import math

    import synth

    Lt = (16, 16, 16, 32)
    U = synth.su3_links(Lt, 0.2, 2016)
    ctx = ov.Context(Lt, BC, MW)
    ctx.upload_gauge(torch.from_numpy(U).cuda())
    ctx.set_fields([Q], [1e-3])
    ctx.set_sign_params(100, 0.01, NORM)
    l = 64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, res, _, rep = ctx.hw_eigensolve(0, l, k=80, cheb_order=100, tol=1e-10, prec="fp32", seed=3,
                                         install=True, want_vectors=False)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    lam_l = max(abs(v) for v in lam)
    eps = (0.95 * lam_l / NORM) ** 2
    n = int(math.ceil(math.log(0.41 / 1e-10) / (2.1 * math.sqrt(eps))))
    ctx.set_sign_params(n, eps, NORM)
    src = synth.point_sources(Lt, (8, 0, 0, 16))[[0, 4, 7, 11]]
    masses = (0.05, 0.1, 0.2)
    b = torch.from_numpy(np.concatenate([src] * len(masses))).cuda()
    mvec = [m for m in masses for _ in range(len(src))]
    print(f"[bench] tts: eigensolve {t_eig:.1f}s, n = {n}, eps = {eps:.3e}", file=sys.stderr, flush=True)
    out = {}
    # inner tolerance per precision: FP32 to 1e-6 (its operator is accurate to a few 1e-7), BF16
    # storage to 1e-3 (its operator to ~1e-2); the FP64 outer loop corrects both to 1e-10
    inner_tols = {"fp32": 1e-6, "bf16": 1e-3, "fp64": 1e-11}
    for inner in ("fp32", "bf16", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, report = ctx.deflated_cg(b, mass=mvec, tol=1e-10, inner_prec=inner, inner_tol=inner_tols[inner],
                                    use_deflation=False)
        torch.cuda.synchronize()
        out[inner] = (time.perf_counter() - t0, x, report)
        print(f"[bench] tts: {inner} inner CG {out[inner][0]:.1f}s", file=sys.stderr, flush=True)
    x64 = out["fp64"][1]
    diff = {k: ((out[k][1] - x64).reshape(len(mvec), -1).norm(dim=1) / x64.reshape(len(mvec), -1).norm(dim=1)).tolist()
            for k in ("fp32", "bf16")}
    ctx.close()

    def summary(k):
        t, _, r = out[k]
        return {"seconds": round(t, 2), "inner_tol": inner_tols[k], "inner_iters_summed": sum(e["iters"] for e in r),
                "max_inner_iters": max(e["iters"] for e in r), "fp64_restarts_max": max(e["restarts"] for e in r),
                "max_relres": max(e["relres"] for e in r)}

    return {"workload": "16^3x32 Dirichlet x,t; q eta = 2/3 x 1e-3; 64 H_w low modes; 12 propagators "
                        "(4 point sources x masses 0.05, 0.1, 0.2) in one batch to FP64 true residual 1e-10",
            "npoly": n, "eps": eps, "eig_seconds": round(t_eig, 2), "lambda_64": lam_l,
            "mixed_fp32_inner": summary("fp32"), "bf16_storage_inner": summary("bf16"), "fp64_inner": summary("fp64"),
            "speedup_mixed_vs_fp64": round(out["fp64"][0] / out["fp32"][0], 3),
            "speedup_bf16_inner_vs_fp64": round(out["fp64"][0] / out["bf16"][0], 3),
            "mixed_vs_fp64_solution_rel_diff": {"max": max(diff["fp32"]),
                                                "per_propagator": [float(f"{d:.3e}") for d in diff["fp32"]]},
            "bf16_inner_vs_fp64_solution_rel_diff_max": max(diff["bf16"])}


def tts_measurement(torch, ov, args):
    """Time to solution at 16^3 x 32, one operator (q eta = 2/3 x 1e-3): H_w low modes by the
    eigensolver, eps and n from lambda_l by eq. (2) for delta = 1e-10, then propagators of
    4 point sources (both chiralities) for 3 masses to 1e-10, once by the per-mass deflated CG and
    once by the multi-mass chirality-sector CG with adaptive order."""
    import math

    import synth

    Lt = (16, 16, 16, 32)
    U = synth.su3_links(Lt, 0.2, 2016)
    ctx = ov.Context(Lt, BC, MW)
    ctx.upload_gauge(torch.from_numpy(U).cuda())
    ctx.set_fields([Q], [1e-3])
    ctx.set_sign_params(100, 0.01, NORM)
    l = args.tts_l
    t0 = time.perf_counter()
    lam, res, V, rep = ctx.hw_eigensolve(0, l, k=min(256, l + max(16, l // 4)), cheb_order=100, tol=1e-10,
                                         prec="fp32", seed=3, install=True, want_vectors=False)
    torch.cuda.synchronize()
    t_eig = time.perf_counter() - t0
    lam_l = max(abs(v) for v in lam)
    eps = (0.95 * lam_l / NORM) ** 2
    n = int(math.ceil(math.log(2 * 0.41 / 1e-10) / (2.1 * math.sqrt(eps))))
    ctx.set_sign_params(n, eps, NORM)
    src = synth.point_sources(Lt, (8, 0, 0, 16))[[0, 4, 7, 11]]
    b = torch.from_numpy(src.copy()).cuda()
    masses = (0.05, 0.1, 0.2)
    print(f"[bench] tts: eigensolve {t_eig:.1f}s (|lambda_l| = {lam_l:.3f}), n = {n}, eps = {eps:.3e}",
          file=sys.stderr, flush=True)
    def per_mass(deflate):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it_pm, rel_pm = 0, 0.0
        for m in masses:
            x, report = ctx.deflated_cg(b, mass=[m] * len(src), tol=1e-10, use_deflation=deflate)
            it_pm += sum(r["iters"] for r in report)
            rel_pm = max(rel_pm, max(r["relres"] for r in report))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, it_pm, rel_pm

    t_pm, it_pm, rel_pm = per_mass(False)
    print(f"[bench] tts: per-mass CG {t_pm:.1f}s", file=sys.stderr, flush=True)
    # D_ov low modes in both chirality sectors -> deflation basis
    ld = args.tts_ldov
    t0 = time.perf_counter()
    # a deflation basis needs no 1e-10 eigenvectors: the outer FP64 loop absorbs the rest
    lam_p, _, Wp, rp = ctx.dov_eigensolve(0, 1, ld, k=ld + 8, cheb_order=24, tol=1e-6, prec="fp32", seed=5,
                                          max_iter=20, raise_on_noconv=False)
    print(f"[bench] tts: D_ov modes, + sector: {rp['iters']} passes, {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    lam_m, _, Wm, rm = ctx.dov_eigensolve(0, -1, ld, k=ld + 8, cheb_order=24, tol=1e-6, prec="fp32", seed=6,
                                          max_iter=20, raise_on_noconv=False)
    ctx.upload_deflation(0, torch.cat([Wp, Wm]))
    del Wp, Wm
    torch.cuda.synchronize()
    t_deig = time.perf_counter() - t0
    print(f"[bench] tts: D_ov eigensolve 2 x {ld} modes {t_deig:.1f}s", file=sys.stderr, flush=True)
    t_pmd, it_pmd, rel_pmd = per_mass(True)
    print(f"[bench] tts: deflated per-mass CG {t_pmd:.1f}s", file=sys.stderr, flush=True)
    mres = {}
    for adaptive in (False, True):
        t0 = time.perf_counter()
        x, rel, rep2 = ctx.multishift_cg(b, masses, tol=1e-10, adaptive=adaptive, min_order=max(10, n // 10),
                                         inner_prec="fp64", refine=True)
        torch.cuda.synchronize()
        t_ms = time.perf_counter() - t0
        mres[adaptive] = (t_ms, rel, rep2)
        print(f"[bench] tts: multi-mass CG (adaptive={adaptive}) {t_ms:.1f}s", file=sys.stderr, flush=True)
    ctx.close()
    t_ms, rel, rep2 = mres[True]
    return {"workload": "16^3x32, q eta = 2/3 x 1e-3, 4 point sources x masses (0.05, 0.1, 0.2), tol 1e-10",
            "eig_l": l, "eig_seconds": round(t_eig, 2), "eig_passes": rep["iters"], "lambda_l": lam_l,
            "npoly": n, "eps": eps,
            "per_mass_cg": {"seconds": round(t_pm, 2), "inner_iters_summed": it_pm, "max_relres": rel_pm},
            "dov_eig": {"modes_per_sector": ld, "seconds": round(t_deig, 2), "passes": [rp["iters"], rm["iters"]],
                        "tol": 1e-6, "max_resid": max(rp["max_resid"], rm["max_resid"]),
                        "lambda_min": min(lam_p[0], lam_m[0]), "lambda_max": max(lam_p[-1], lam_m[-1])},
            "deflated_per_mass_cg": {"seconds": round(t_pmd, 2), "inner_iters_summed": it_pmd,
                                     "max_relres": rel_pmd},
            "multi_mass_cg": {"seconds": round(t_ms, 2), "iters": rep2["iters"],
                              "sign_applies": rep2["sign_applies"], "dslash_applies": rep2["dslash_applies"],
                              "refine_inner_iters": rep2["refine_iters"], "max_relres": float(rel.max())},
            "multi_mass_cg_fixed_order": {"seconds": round(mres[False][0], 2),
                                          "dslash_applies": mres[False][2]["dslash_applies"],
                                          "refine_inner_iters": mres[False][2]["refine_iters"]},
            "speedup_multi_mass_vs_per_mass": round(t_pm / t_ms, 2),
            "speedup_deflation": round(t_pm / t_pmd, 2)}


CPU_SAMPLE = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import synth
from oracle import api
L, BC, MW, EPS, NORM, QE, M, SRC = json.loads(sys.argv[2])
runs = json.loads(sys.argv[3])
U = synth.su3_links(L, 0.2, 2022)
lat = api.Lattice(L, BC, MW, U, QE)
x = synth.point_sources(L, SRC)[0]
lmax = max(l for _, l in runs)
Vs = synth.random_orthonormal(L, lmax, 9) if lmax else None
api.dov(lat, api.SignParams(1, EPS, NORM), x, M)
out = []
for n, l in runs:
    sp = api.SignParams(n, EPS, NORM, Vs[:l] if l else None, np.linspace(-1, 1, l) if l else None)
    t0 = time.perf_counter()
    api.dov(lat, sp, x, M)
    out.append(time.perf_counter() - t0)
api.dslash(lat, x, 1)
td = []
for _ in range(3):
    t0 = time.perf_counter()
    api.dslash(lat, x, 1)
    td.append(time.perf_counter() - t0)
print(json.dumps({"runs": out, "hw": min(td)}))
"""


def _oracle_dov_seconds(runs, threads):
    """Wall times of FP64 oracle D(m) applications (order n, l small-space vectors, for each
    (n, l) in runs) on one point source at 24^3 x 48, and the best of three H_w applications on
    it, in a child process with `threads` OpenMP threads (the oracle's thread count is fixed when
    it loads)."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cfg = json.dumps([list(L), list(BC), MW, EPS, NORM, Q * ETAS[1], MASSES[1], list(SRC)])
    r = subprocess.run([sys.executable, "-c", CPU_SAMPLE, ROOT, cfg, json.dumps(runs)], env=env,
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"oracle sample failed: {r.stderr[-2000:]}")
    res = json.loads(r.stdout.strip().splitlines()[-1])
    return res["runs"], res["hw"]


def cpu_baseline():
    """The FP64 oracle on the host cores: one measured order-300 D(m) at 24^3 x 48.

    Measured: D(m) with n = 300 and an 8-vector small space on one point source, all host
    threads (the workload's order; only the small space is smaller).  The 200-vector small
    space is added from two short runs (n = 1 with l = 0 and l = 8: the per-vector projection
    cost, linear in l).  A 1-thread run of the n = 1, l = 0 sample gives the speed of one core.
    """
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    (t300, t1_0, t1_8), t_hw = _oracle_dov_seconds([[NPOLY, 8], [1, 0], [1, 8]], threads)
    per_vec = max(t1_8 - t1_0, 0.0) / 8.0
    t_apply = t300 + (LSMALL - 8) * per_vec
    (one,), t_hw1 = _oracle_dov_seconds([[1, 0]], 1)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 1.0 / t_apply, "unit": "D_ov applies/s", "cores": threads, "kind": "oracle",
        "sample": (f"FP64 oracle D(m), n=300, l=8, 1 point source at 24^3x48 on {threads} threads: "
                   f"{t300:.1f} s measured; + 192 small-space vectors at {per_vec:.3f} s each "
                   f"(n=1 runs with l=0/8: {t1_0:.2f}/{t1_8:.2f} s) = {t_apply:.1f} s per apply"),
        "cpu_model": model, "nproc": os.cpu_count(),
        "one_thread": {"n1_l0_seconds": round(one, 3), "n1_l0_seconds_all_threads": round(t1_0, 3),
                       "parallel_speedup": round(one / max(t1_0, 1e-9), 2),
                       "est_seconds_per_apply": round(t_apply * one / max(t1_0, 1e-9), 1)},
        "hw_dslash_seconds": {"all_threads": round(t_hw, 4), "one_thread": round(t_hw1, 4)},
        "seconds_per_apply": round(t_apply, 2),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "gpus_requested": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_1111_6288_amd import ov

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)

    copy_bw = copy_bandwidth(torch)
    print(f"[bench] plain copy: {copy_bw / 1e9:.0f} GB/s (read + write)", file=sys.stderr, flush=True)
    print(f"[bench] building inputs: L={L}, n={args.npoly}, l={args.lsmall}", file=sys.stderr, flush=True)
    ctx, U, x, fields, masses, t_setup = build_inputs(torch, ov, args)
    nrhs = len(fields)
    applied = [] if args.autotune else ctx.load_tuning(TUNING_FILE, "fp32", nrhs)
    if sorted(applied) != ["clenshaw", "dslash"]:
        ctx.autotune("fp32", nrhs)
    if not args.autotune:
        ctx.load_tuning(TUNING_FILE, "fp64", nrhs)
        ctx.load_tuning(TUNING_FILE, "bf16", nrhs)
    tuned = {k: ctx.get_launch_config("fp32", k) for k in ("dslash", "clenshaw")}
    print(f"[bench] setup {t_setup:.1f}s, fp32 tuning {tuned}", file=sys.stderr, flush=True)

    y32 = torch.empty_like(x)
    dt, stats = timed_applies(torch, ctx, x, y32, fields, masses, "fp32", args.steps, args.warmup, True)
    applies = nrhs * args.steps
    value = applies / dt
    print(f"[bench] mixed: {args.steps} steps in {dt:.2f}s -> {value:.2f} applies/s", file=sys.stderr, flush=True)

    # last step applied D^dag when steps is even, D otherwise; recompute D on a fixed slice for the error check
    ctx.dov_apply(x, fields, masses, dagger=False, prec="fp32", out=y32)
    fp64 = None
    err = None
    extra = {}
    if not args.no_fp64:
        y64 = torch.empty_like(x)
        dt64, _ = timed_applies(torch, ctx, x, y64, fields, masses, "fp64", args.fp64_steps, 1, False)
        fp64 = nrhs * args.fp64_steps / dt64
        ctx.dov_apply(x, fields, masses, dagger=False, prec="fp64", out=y64)
        d = (y32 - y64).reshape(nrhs, -1).norm(dim=1) / y64.reshape(nrhs, -1).norm(dim=1)
        err = float(d.max())
        print(f"[bench] fp64: {fp64:.2f} applies/s; mixed vs fp64 max rel err {err:.2e}", file=sys.stderr,
              flush=True)
        # BF16 storage (FP32 arithmetic) on the same 108 RHS, and FP64 on a single RHS
        y16 = torch.empty_like(x)
        dt16, _ = timed_applies(torch, ctx, x, y16, fields, masses, "bf16", 1, 1, False)
        extra["bf16_applies_per_s"] = round(nrhs / dt16, 3)
        ctx.dov_apply(x, fields, masses, dagger=False, prec="bf16", out=y16)
        d16 = (y16 - y64).reshape(nrhs, -1).norm(dim=1) / y64.reshape(nrhs, -1).norm(dim=1)
        extra["bf16_vs_fp64_max_rel_err"] = float(d16.max())
        del y16, y64
        x1 = x[:1].clone()
        y1 = torch.empty_like(x1)
        dt1, _ = timed_applies(torch, ctx, x1, y1, fields[:1], masses[:1], "fp64", 3, 1, False)
        extra["fp64_single_rhs_applies_per_s"] = round(3 / dt1, 3)
        print(f"[bench] bf16: {extra['bf16_applies_per_s']} applies/s, fp64 single RHS: "
              f"{extra['fp64_single_rhs_applies_per_s']} applies/s", file=sys.stderr, flush=True)

    n_launch, ms, by = stats["clenshaw"]
    avg_ms = ms / max(n_launch, 1)
    bytes_per_launch = by / max(n_launch, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    two_row = ctx.link_format()[0]
    traffic_bytes = measured_traffic("fp32", nrhs, tuned["clenshaw"], two_row)
    traffic = None if traffic_bytes is None else round(traffic_bytes / (avg_ms * 1e-3) / 1e9, 1)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "copy_GBps": round(copy_bw / 1e9, 1), "frac_of_copy": round(achieved / (copy_bw / 1e9), 4),
                "traffic": traffic, "traffic_bytes_per_launch": traffic_bytes,
                "kernel": ("k_dslash_tm<float2,HW,EPI,W,REC> (t-marching dslash + fused Clenshaw epilogue)"
                           if tuned["clenshaw"]["site_order"] == 2
                           else "k_dslash_lds<float2,NR,Q,HW,EPI,REC> (dslash with LDS-shared links + fused "
                                "Clenshaw epilogue)" if tuned["clenshaw"].get("wshare", 1) > 1
                           else "k_dslash<float2,NR,Q,HW,EPI,REC> (dslash + fused Clenshaw epilogue)"),
                "two_row_links": two_row,
                "launches": n_launch, "avg_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": bytes_per_launch}
    kernels = {k: {"launches": v[0], "ms": round(v[1], 2), "GBps": round(v[2] / max(v[1], 1e-9) / 1e6, 1)}
               for k, v in stats.items()}
    # V^dag X on the matrix cores: 8 l n K flops per launch (one field group of n RHS, K = 12 Vp)
    n_pd, ms_pd, _ = stats["proj_dot"]
    n_grp = nrhs // len(ETAS)
    Vp = (synth_volume() + 63) // 64 * 64
    flops = n_pd * 8.0 * args.lsmall * n_grp * 12 * Vp
    tf = flops / max(ms_pd * 1e-3, 1e-12) / 1e12 if n_pd else None
    projection = {"kernel": "k_proj_dot_mfma<float2> (V^dag X, FP64 MFMA)", "tflops": None if tf is None else round(tf, 2),
                  "peak_tflops": 78.6, "frac": None if tf is None else round(tf / 78.6, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on host cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
        # host cores one GPU stands for: CPU seconds x cores per GPU second, per apply
        cpu["equivalent_cores"] = round(cpu["seconds_per_apply"] * cpu["cores"] * value)

    line = {
        "metric": "D_ov applies/s at 24^3x48 (dslash HBM GB/s), mixed+multiRHS vs FP64 at 1e-10",
        "value": round(value, 3), "unit": "D_ov applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "24^3x48 overlap D(m) apply, 108 RHS (12 point sources x 3 eta x 3 masses), "
                               "order-300 Chebyshev sign, 200-vector small space per field, mixed FP32/FP64",
                   "lattice": list(L), "nrhs": nrhs, "npoly": args.npoly, "lsmall": args.lsmall,
                   "bc": "Dirichlet x,t; periodic y,z", "projection_dtype": "f64",
                   "tuning_fp32": tuned},
        "fp64_applies_per_s": None if fp64 is None else round(fp64, 3),
        "speedup_vs_fp64": None if fp64 is None else round(value / fp64, 3),
        "mixed_vs_fp64_max_rel_err": err,
        "roofline": roofline,
        "kernels": kernels,
        "projection": projection,
        **extra,
        "cpu_baseline": cpu,
    }
    ctx.close()
    del x, y32
    torch.cuda.empty_cache()
    if not args.no_tts:
        line["time_to_solution"] = tts_mixed_vs_fp64(torch, ov)
    if args.eig:
        line["eigensolver"] = eig_measurement(torch, ov, U, args)
    if args.tts:
        line["propagator_methods"] = tts_measurement(torch, ov, args)
    print(json.dumps(line), flush=True)
    if args.calibrate_copy:
        src = torch.empty(4 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        # the same 4 GiB through an elementwise kernel (torch's own, not the runtime's copy)
        srcf, dstf = src.view(torch.float32), dst.view(torch.float32)
        for _ in range(3):
            torch.neg(srcf, out=dstf)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 3 x 4 GiB device-to-device copies, 3 x 4 GiB elementwise neg",
              file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
