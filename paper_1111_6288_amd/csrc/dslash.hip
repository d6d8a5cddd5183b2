// Wilson dslash / H_w for a batch of right-hand sides, with an optional
// fused linear epilogue used by the Clenshaw recursion of the sign function.
//
//   y_r = a * G (D_w x_r)  +  c1 e1_r + c2 e2_r + c3 e3_r          (own site)
//   D_w x(s) = (4 + m_w) x(s)
//        - 1/2 sum_mu [ (1 - gamma_mu) U~_mu(s) x(s+mu) + (1 + gamma_mu) U~_mu(s-mu)^dag x(s-mu) ]
//   G = gamma5 for H_w = gamma5 D_w (Sec. 2), identity for D_w.
//
// U~_0 carries the background-field phase exp(i q eta t) of the RHS's field
// group (Sec. 4, eq. (3)), applied to the projected half spinor so that the
// links stay shared by every RHS in the batch.  Hops that wrap around the
// lattice take the boundary multiplier (+1, -1, 0; Dirichlet hops are skipped).
//
// Spin projection uses the chiral basis: each (1 -/+ gamma_mu) has rank two,
// so the neighbour spinor is reduced to a half spinor h0, h1 (2 x 3 complex),
// multiplied by the 3x3 link and expanded back.  One thread owns one site and
// NR right-hand sides: the link is loaded once and applied to all NR spinors.
#include "ov_device.h"
#include "ov_internal.h"
#include "spin.h"

namespace ov {

// Loads address a plane through a wave-uniform base pointer plus a 32-bit
// per-lane site offset, so that the compiler can use scalar-base addressing
// instead of per-lane 64-bit address arithmetic.
template <class S, class R>
__device__ __forceinline__ cx<R> ldp(const S *__restrict__ plane, unsigned site)
{
    const unsigned boff = site * (unsigned)sizeof(S);   // < 4 GiB: a plane holds at most 2^31/64 sites
    return ldc<R>((const S *)((const char *)plane + boff), 0u);
}

template <class S, class R>
__device__ __forceinline__ void stp(S *__restrict__ plane, unsigned site, cx<R> v)
{
    const unsigned boff = site * (unsigned)sizeof(S);
    stc<R>((S *)((char *)plane + boff), 0u, v);
}

template <class S, class R>
__device__ __forceinline__ void load_link(const S *__restrict__ U, int mu, int Vp, unsigned s, cx<R> (&u)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = ldp<S, R>(U + (size_t)(mu * 9 + a * 3 + b) * (unsigned)Vp, s);
}

template <class S, class R>
__device__ __forceinline__ void load_spinor(const S *__restrict__ x, int Vp, unsigned s, cx<R> (&p)[4][3])
{
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) p[sp][c] = ldp<S, R>(x + (size_t)(sp * 3 + c) * (unsigned)Vp, s);
}

// One direction, both hops, for all NR right-hand sides of this thread.
template <int MU, int NR, class S, class R>
__device__ __forceinline__ void hop_dir(const DsArgs<S> &a, int site, int cmu, int Lmu, int stride,
                                        const size_t (&off)[NR], const bool (&act)[NR],
                                        const cx<R> (&ph)[NR], cx<R> (&acc)[NR][4][3])
{
    const int Vp = a.g.Vp;
    // forward hop: -1/2 (1 - gamma_mu) U~_mu(s) x(s + mu)
    {
        const bool wrap = (cmu == Lmu - 1);
        const int j = wrap ? site - (Lmu - 1) * stride : site + stride;
        const R bf = wrap ? (R)a.g.bcf[MU] : (R)1;
        if (bf != (R)0) {
            cx<R> u[3][3];
            load_link<S, R>(a.U, MU, Vp, (unsigned)site, u);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (!act[r]) continue;
                cx<R> p[4][3], h[2][3], g[2][3];
                load_spinor<S, R>(a.x + off[r], Vp, (unsigned)j, p);
                project<MU, -1>(p, h);
                if (MU == 0 || wrap) {
                    cx<R> f = (MU == 0) ? cscale(ph[r], bf) : cmk(bf, (R)0);
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) h[k][c] = cmul(f, h[k][c]);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        cx<R> t = cmul(u[aa][0], h[k][0]);
                        cfma(t, u[aa][1], h[k][1]);
                        cfma(t, u[aa][2], h[k][2]);
                        g[k][aa] = t;
                    }
                expand_add<MU, -1>(acc[r], g);
            }
        }
    }
    // backward hop: -1/2 (1 + gamma_mu) U~_mu(s - mu)^dag x(s - mu)
    {
        const bool wrap = (cmu == 0);
        const int j = wrap ? site + (Lmu - 1) * stride : site - stride;
        const R bf = wrap ? (R)a.g.bcf[MU] : (R)1;
        if (bf != (R)0) {
            cx<R> u[3][3];
            load_link<S, R>(a.U, MU, Vp, (unsigned)j, u);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (!act[r]) continue;
                cx<R> p[4][3], h[2][3], g[2][3];
                load_spinor<S, R>(a.x + off[r], Vp, (unsigned)j, p);
                project<MU, +1>(p, h);
                if (MU == 0 || wrap) {
                    cx<R> f = (MU == 0) ? cmk(ph[r].x * bf, -ph[r].y * bf) : cmk(bf, (R)0);
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) h[k][c] = cmul(f, h[k][c]);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        cx<R> t = cmulc(u[0][aa], h[k][0]);
                        cfmac(t, u[1][aa], h[k][1]);
                        cfmac(t, u[2][aa], h[k][2]);
                        g[k][aa] = t;
                    }
                expand_add<MU, +1>(acc[r], g);
            }
        }
    }
}

// Workgroups are handed to the 8 XCDs round-robin; remap so that each XCD
// receives a contiguous run of sites, which keeps stencil neighbours in the
// same XCD's L2.  nblk must be a multiple of 8 (the launcher pads).
__device__ __forceinline__ int xcd_block(int b, int nblk)
{
    const int per = nblk >> 3;
    return (b & 7) * per + (b >> 3);
}

// Site of this thread.  order 0: blocks walk the sites in canonical order,
// each XCD taking a contiguous run (t-chunks).  order 1: XCD x owns the
// z-slab [x Lz/8, (x+1) Lz/8) and walks it plane by plane, (z, t) planes of
// Lx*Ly sites in t-major order, so the cross-section an XCD sweeps is 1/8 of
// a time slice and t-neighbours are re-read soon after their first use.
// order 1 needs Lz % 8 == 0 and V % 64 == 0 (no padding); the launcher checks.
__device__ __forceinline__ int dslash_site(const Geo &g, int order, int xcd_remap)
{
    if (order == 1) {
        const int xcd = blockIdx.x & 7;
        const int u = (blockIdx.x >> 3) * blockDim.x + threadIdx.x;
        const int nz = g.Lz >> 3;
        const int q = u / g.Lxy, o = u - q * g.Lxy;
        if (q >= nz * g.Lt) return g.Vp;   // beyond the slab: no work
        const int zl = q % nz, t = q / nz;
        return o + g.Lxy * (xcd * nz + zl + g.Lz * t);
    }
    const int blk = xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    return blk * blockDim.x + threadIdx.x;
}

template <class S, int NR, bool HW, bool EPI>
__global__ __launch_bounds__(256) void k_dslash(DsArgs<S> a)
{
    using R = typename StoreT<S>::real;
    const Geo &g = a.g;
    const int site = dslash_site(g, a.order, a.xcd_remap);
    if (site >= g.Vp) return;
    const int j0 = blockIdx.y * NR;

    size_t off[NR];
    bool act[NR];
    int grp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int j = j0 + r;
        act[r] = j < a.n;
        const int jj = act[r] ? j : j0;
        // the storage index depends on blockIdx.y only: make the compiler see it as uniform
        const int s = __builtin_amdgcn_readfirstlane(a.slots ? a.slots[jj] : jj);
        off[r] = (size_t)s * (size_t)a.fstride;
        grp[r] = __builtin_amdgcn_readfirstlane(a.fgroup ? a.fgroup[s] : 0);
    }
    if (site >= g.V) {   // padding sites hold zeros in every field
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!act[r]) continue;
#pragma unroll
            for (int k = 0; k < 12; ++k)
                stp<S, R>(a.y + off[r] + (size_t)k * (unsigned)g.Vp, (unsigned)site, cmk((R)0, (R)0));
        }
        return;
    }

    int rem = site;
    const int xc = rem % g.Lx; rem /= g.Lx;
    const int yc = rem % g.Ly; rem /= g.Ly;
    const int zc = rem % g.Lz;
    const int tc = rem / g.Lz;

    cx<R> ph[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const cx<double> p = a.phase[grp[r] * g.Lt + tc];
        ph[r] = cmk((R)p.x, (R)p.y);
    }

    cx<R> acc[NR][4][3];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][sp][c] = cmk((R)0, (R)0);

    hop_dir<0, NR, S, R>(a, site, xc, g.Lx, 1, off, act, ph, acc);
    hop_dir<1, NR, S, R>(a, site, yc, g.Ly, g.Lx, off, act, ph, acc);
    hop_dir<2, NR, S, R>(a, site, zc, g.Lz, g.Lxy, off, act, ph, acc);
    hop_dir<3, NR, S, R>(a, site, tc, g.Lt, g.Lxyz, off, act, ph, acc);

    const R diag = (R)a.diag, sc = (R)a.a;
    const R c1 = (R)a.c1, c2 = (R)a.c2, c3 = (R)a.c3;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (!act[r]) continue;
        cx<R> p[4][3];
        load_spinor<S, R>(a.x + off[r], g.Vp, (unsigned)site, p);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cx<R> v = cmk(diag * p[sp][c].x - (R)0.5 * acc[r][sp][c].x,
                              diag * p[sp][c].y - (R)0.5 * acc[r][sp][c].y);
                R s = (HW && sp >= 2) ? -sc : sc;
                v = cscale(v, s);
                const size_t po = off[r] + (size_t)(sp * 3 + c) * (unsigned)g.Vp;
                const unsigned us = (unsigned)site;
                if (EPI) {
                    if (a.e1) { cx<R> e = ldp<S, R>(a.e1 + po, us); v.x = fma(c1, e.x, v.x); v.y = fma(c1, e.y, v.y); }
                    if (a.e2) { cx<R> e = ldp<S, R>(a.e2 + po, us); v.x = fma(c2, e.x, v.x); v.y = fma(c2, e.y, v.y); }
                    if (a.e3) { cx<R> e = ldp<S, R>(a.e3 + po, us); v.x = fma(c3, e.x, v.x); v.y = fma(c3, e.y, v.y); }
                }
                stp<S, R>(a.y + po, us, v);
            }
    }
}

// ---------------------------------------------------------------------------
// t-marching variant.  Each thread owns one (x, y, z) site and one RHS and
// walks t over a chunk [t0, t1), keeping psi(t-1), psi(t), psi(t+1) and the
// backward time link in registers: the two time neighbours cost no loads and
// every input spinor is fetched once per chunk.  A wave covers 64 consecutive
// sites of one (z, t) plane, so x and y neighbours come from lines the wave
// itself touches in the same step (L1); the 4 waves of a workgroup are 4 RHS
// on the same sites, so link loads are shared through L1; blocks walk z
// fastest within an XCD, so z neighbours are loaded by workgroups running at
// the same time on the same XCD (L2).
//
// Block b: XCD b & 7, local index m = b >> 3 decomposed as
//   m = z + Lz (ob + nob (tc + ntc rg))
// with ob the 64-site block of the (x, y) plane, tc the t-chunk and rg the
// group of 4 RHS.  Needs V % 64 == 0 (no padding); the launcher checks.
template <class S, bool HW, bool EPI>
__global__ __launch_bounds__(256) void k_dslash_tm(DsArgs<S> a)
{
    using R = typename StoreT<S>::real;
    const Geo &g = a.g;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nob = (g.Lxy + 63) >> 6;
    const int ntc = (g.Lt + a.tchunk - 1) / a.tchunk;
    // XCD k takes the contiguous range of m starting at k * gridDim.x / 8; its
    // successive blocks walk z fastest
    int m = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int z = m % g.Lz;
    m /= g.Lz;
    const int ob = m % nob;
    m /= nob;
    const int tc = m % ntc;
    const int rg = m / ntc;
    const int j = rg * 4 + wave;
    const int o = ob * 64 + lane;
    if (j >= a.n || o >= g.Lxy) return;

    const int s = __builtin_amdgcn_readfirstlane(a.slots ? a.slots[j] : j);
    const size_t off = (size_t)s * (size_t)a.fstride;
    const int grp = __builtin_amdgcn_readfirstlane(a.fgroup ? a.fgroup[s] : 0);
    const int xc = o % g.Lx, yc = o / g.Lx;
    const int t0 = tc * a.tchunk;
    const int t1 = (t0 + a.tchunk < g.Lt) ? t0 + a.tchunk : g.Lt;
    const int Vp = g.Vp;
    const int base_zt = o + g.Lxy * z;          // site of (x, y, z, t) = base_zt + Lxyz t
    const S *x = a.x + off;

    auto site_at = [&](int t) { return base_zt + g.Lxyz * t; };
    const int tm1 = (t0 == 0) ? g.Lt - 1 : t0 - 1;

    cx<R> pm[4][3], pc[4][3], pn[4][3], utm[3][3];
    load_spinor<S, R>(x, Vp, (unsigned)site_at(tm1), pm);
    load_spinor<S, R>(x, Vp, (unsigned)site_at(t0), pc);
    load_link<S, R>(a.U, 3, Vp, (unsigned)site_at(tm1), utm);

    const size_t offs[1] = {off};
    const bool acts[1] = {true};
    const R diag = (R)a.diag, sc = (R)a.a;
    const R c1 = (R)a.c1, c2 = (R)a.c2, c3 = (R)a.c3;
    const R bt = (R)g.bcf[3];

    for (int t = t0; t < t1; ++t) {
        const int site = site_at(t);
        const int tp1 = (t == g.Lt - 1) ? 0 : t + 1;
        load_spinor<S, R>(x, Vp, (unsigned)site_at(tp1), pn);
        cx<R> utc[3][3];
        load_link<S, R>(a.U, 3, Vp, (unsigned)site, utc);
        const cx<double> pd = a.phase[grp * g.Lt + t];
        const cx<R> ph[1] = {cmk((R)pd.x, (R)pd.y)};

        cx<R> acc[1][4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[0][sp][c] = cmk((R)0, (R)0);

        hop_dir<0, 1, S, R>(a, site, xc, g.Lx, 1, offs, acts, ph, acc);
        hop_dir<1, 1, S, R>(a, site, yc, g.Ly, g.Lx, offs, acts, ph, acc);
        hop_dir<2, 1, S, R>(a, site, z, g.Lz, g.Lxy, offs, acts, ph, acc);

        // time hops from registers
        {
            const R bf = (t == g.Lt - 1) ? bt : (R)1;
            if (bf != (R)0) {
                cx<R> h[2][3], gg[2][3];
                project<3, -1>(pn, h);
                if (bf != (R)1) {
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) h[k][c] = cscale(h[k][c], bf);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        cx<R> tt = cmul(utc[aa][0], h[k][0]);
                        cfma(tt, utc[aa][1], h[k][1]);
                        cfma(tt, utc[aa][2], h[k][2]);
                        gg[k][aa] = tt;
                    }
                expand_add<3, -1>(acc[0], gg);
            }
            const R bb = (t == 0) ? bt : (R)1;
            if (bb != (R)0) {
                cx<R> h[2][3], gg[2][3];
                project<3, +1>(pm, h);
                if (bb != (R)1) {
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int c = 0; c < 3; ++c) h[k][c] = cscale(h[k][c], bb);
                }
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        cx<R> tt = cmulc(utm[0][aa], h[k][0]);
                        cfmac(tt, utm[1][aa], h[k][1]);
                        cfmac(tt, utm[2][aa], h[k][2]);
                        gg[k][aa] = tt;
                    }
                expand_add<3, +1>(acc[0], gg);
            }
        }

#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cx<R> v = cmk(diag * pc[sp][c].x - (R)0.5 * acc[0][sp][c].x,
                              diag * pc[sp][c].y - (R)0.5 * acc[0][sp][c].y);
                const R sg = (HW && sp >= 2) ? -sc : sc;
                v = cscale(v, sg);
                const size_t po = off + (size_t)(sp * 3 + c) * (unsigned)Vp;
                if (EPI) {
                    if (a.e1) { cx<R> e = ldp<S, R>(a.e1 + po, (unsigned)site); v.x = fma(c1, e.x, v.x); v.y = fma(c1, e.y, v.y); }
                    if (a.e2) { cx<R> e = ldp<S, R>(a.e2 + po, (unsigned)site); v.x = fma(c2, e.x, v.x); v.y = fma(c2, e.y, v.y); }
                    if (a.e3) { cx<R> e = ldp<S, R>(a.e3 + po, (unsigned)site); v.x = fma(c3, e.x, v.x); v.y = fma(c3, e.y, v.y); }
                }
                stp<S, R>(a.y + po, (unsigned)site, v);
            }

#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pm[sp][c] = pc[sp][c];
                pc[sp][c] = pn[sp][c];
            }
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb2 = 0; bb2 < 3; ++bb2) utm[aa][bb2] = utc[aa][bb2];
    }
}

template <class S>
static hipError_t launch_tm(const DsArgs<S> &a, bool hw, bool epi, hipStream_t st)
{
    DsArgs<S> b = a;
    if (b.tchunk <= 0 || b.tchunk > a.g.Lt) b.tchunk = a.g.Lt;
    const int nob = (a.g.Lxy + 63) / 64;
    const int ntc = (a.g.Lt + b.tchunk - 1) / b.tchunk;
    const long nblk = (long)a.g.Lz * nob * ntc * ((a.n + 3) / 4);
    const long padded = (nblk + 7) / 8 * 8;
    if (padded > 0x7fffffffL) return hipErrorInvalidValue;
    if (epi)
        hipLaunchKernelGGL((k_dslash_tm<S, true, true>), dim3((unsigned)padded), dim3(256), 0, st, b);
    else if (hw)
        hipLaunchKernelGGL((k_dslash_tm<S, true, false>), dim3((unsigned)padded), dim3(256), 0, st, b);
    else
        hipLaunchKernelGGL((k_dslash_tm<S, false, false>), dim3((unsigned)padded), dim3(256), 0, st, b);
    return hipGetLastError();
}

template <class S, int NR>
static hipError_t launch_nr(const DsArgs<S> &a, bool hw, bool epi, int block, hipStream_t st)
{
    // Occupancy cap: reserving LDS the kernel does not use limits the number of
    // resident workgroups per CU (160 KiB of LDS per CU on gfx950), which
    // narrows the window of sites in flight so that stencil neighbours are
    // re-read while still in L2.
    const size_t lds = a.blocks_per_cu > 0 ? (size_t)(160 * 1024) / (size_t)a.blocks_per_cu - 256 : 0;
    int nbx = (a.g.V + block - 1) / block;
    DsArgs<S> b = a;
    b.xcd_remap = 0;
    if (b.order == 1 && (a.g.Lz % 8 != 0 || a.g.V % 64 != 0)) b.order = 0;
    if (b.order == 1) {
        const int per_xcd = (a.g.Lz / 8) * a.g.Lt * a.g.Lxy;
        nbx = 8 * ((per_xcd + block - 1) / block);
    } else if (nbx >= 64) {   // pad to a multiple of 8 for the XCD remap
        nbx = (nbx + 7) & ~7;
        b.xcd_remap = 1;
    }
    dim3 grid(nbx, (a.n + NR - 1) / NR);
    if (lds > 0) {   // allow more than the default 64 KiB of dynamic LDS (once per kernel)
        static bool raised[3] = {false, false, false};
        const int ki = epi ? 0 : (hw ? 1 : 2);
        if (!raised[ki]) {
            hipError_t e;
            if (epi) e = hipFuncSetAttribute((const void *)k_dslash<S, NR, true, true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            else if (hw) e = hipFuncSetAttribute((const void *)k_dslash<S, NR, true, false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            else e = hipFuncSetAttribute((const void *)k_dslash<S, NR, false, false>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            raised[ki] = true;
        }
    }
    if (epi)
        hipLaunchKernelGGL((k_dslash<S, NR, true, true>), grid, dim3(block), lds, st, b);
    else if (hw)
        hipLaunchKernelGGL((k_dslash<S, NR, true, false>), grid, dim3(block), lds, st, b);
    else
        hipLaunchKernelGGL((k_dslash<S, NR, false, false>), grid, dim3(block), lds, st, b);
    return hipGetLastError();
}

template <class S>
hipError_t launch_dslash(const DsArgs<S> &a, bool hw, bool epi, int nr, int block, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    if (block < 64 || block > 256 || (block & 63)) return hipErrorInvalidValue;
    if (a.order == 2 && a.g.V % 64 == 0) return launch_tm<S>(a, hw, epi, st);
    switch (nr) {
    case 1: return launch_nr<S, 1>(a, hw, epi, block, st);
    case 2: return launch_nr<S, 2>(a, hw, epi, block, st);
    case 4: return launch_nr<S, 4>(a, hw, epi, block, st);
    case 8: return launch_nr<S, 8>(a, hw, epi, block, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_dslash<double2>(const DsArgs<double2> &, bool, bool, int, int, hipStream_t);
template hipError_t launch_dslash<float2>(const DsArgs<float2> &, bool, bool, int, int, hipStream_t);
template hipError_t launch_dslash<uint32_t>(const DsArgs<uint32_t> &, bool, bool, int, int, hipStream_t);

}  // namespace ov
