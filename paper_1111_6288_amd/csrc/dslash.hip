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

// Components k = 2p and 2p+1 of one site: a single 16-byte load for the
// paired FP32 layout, two plane loads otherwise.
template <class S, class R>
__device__ __forceinline__ void ldpair(const S *__restrict__ f, int Vp, int p, unsigned site, cx<R> &a, cx<R> &b)
{
    if constexpr (Pair<S>::E == 2) {
        const float4 v = *(const float4 *)((const char *)(f + (size_t)(2 * p) * (unsigned)Vp) + site * 16u);
        a = cmk((R)v.x, (R)v.y);
        b = cmk((R)v.z, (R)v.w);
    } else {
        a = ldp<S, R>(f + (size_t)(2 * p) * (unsigned)Vp, site);
        b = ldp<S, R>(f + (size_t)(2 * p + 1) * (unsigned)Vp, site);
    }
}

template <class S, class R>
__device__ __forceinline__ void stpair(S *__restrict__ f, int Vp, int p, unsigned site, cx<R> a, cx<R> b)
{
    if constexpr (Pair<S>::E == 2) {
        *(float4 *)((char *)(f + (size_t)(2 * p) * (unsigned)Vp) + site * 16u) =
            make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
    } else {
        stp<S, R>(f + (size_t)(2 * p) * (unsigned)Vp, site, a);
        stp<S, R>(f + (size_t)(2 * p + 1) * (unsigned)Vp, site, b);
    }
}

// Non-temporal variants for operands that are touched once per launch (the
// epilogue inputs and the output): the loads and stores carry the
// non-temporal hint so that they do not displace the stencil's neighbour
// spinors and links from L2.
typedef float ov_f4 __attribute__((ext_vector_type(4)));
typedef double ov_d2 __attribute__((ext_vector_type(2)));

template <class S, class R>
__device__ __forceinline__ cx<R> ldp_nt(const S *__restrict__ plane, unsigned site)
{
    const char *p = (const char *)plane + site * (unsigned)sizeof(S);
    if constexpr (sizeof(S) == 16) {
        const ov_d2 v = __builtin_nontemporal_load((const ov_d2 *)p);
        return cmk((R)v.x, (R)v.y);
    } else if constexpr (sizeof(S) == 4) {
        const uint32_t v = __builtin_nontemporal_load((const uint32_t *)p);
        return cmk((R)bf16_lo(v), (R)bf16_hi(v));
    } else {
        return ldp<S, R>(plane, site);
    }
}

template <class S, class R>
__device__ __forceinline__ void stp_nt(S *__restrict__ plane, unsigned site, cx<R> v)
{
    char *p = (char *)plane + site * (unsigned)sizeof(S);
    if constexpr (sizeof(S) == 16) {
        ov_d2 w = {(double)v.x, (double)v.y};
        __builtin_nontemporal_store(w, (ov_d2 *)p);
    } else if constexpr (sizeof(S) == 4) {
        const uint32_t w = f2bf((float)v.x) | (f2bf((float)v.y) << 16);
        __builtin_nontemporal_store(w, (uint32_t *)p);
    } else {
        stp<S, R>(plane, site, v);
    }
}

template <class S, class R>
__device__ __forceinline__ void ldpair_nt(const S *__restrict__ f, int Vp, int p, unsigned site, cx<R> &a, cx<R> &b)
{
    if constexpr (Pair<S>::E == 2) {
        const ov_f4 v = __builtin_nontemporal_load(
            (const ov_f4 *)((const char *)(f + (size_t)(2 * p) * (unsigned)Vp) + site * 16u));
        a = cmk((R)v.x, (R)v.y);
        b = cmk((R)v.z, (R)v.w);
    } else {
        a = ldp_nt<S, R>(f + (size_t)(2 * p) * (unsigned)Vp, site);
        b = ldp_nt<S, R>(f + (size_t)(2 * p + 1) * (unsigned)Vp, site);
    }
}

template <class S, class R>
__device__ __forceinline__ void stpair_nt(S *__restrict__ f, int Vp, int p, unsigned site, cx<R> a, cx<R> b)
{
    if constexpr (Pair<S>::E == 2) {
        const ov_f4 w = {(float)a.x, (float)a.y, (float)b.x, (float)b.y};
        __builtin_nontemporal_store(w, (ov_f4 *)((char *)(f + (size_t)(2 * p) * (unsigned)Vp) + site * 16u));
    } else {
        stp_nt<S, R>(f + (size_t)(2 * p) * (unsigned)Vp, site, a);
        stp_nt<S, R>(f + (size_t)(2 * p + 1) * (unsigned)Vp, site, b);
    }
}

// Link U_mu(s): components 0..7 as pairs, component 8 on its own plane.
// REC: only the first two rows are read (components 0..5, three pairs) and
// the third is rebuilt as u_2a = conj(u_0b u_1c - u_0c u_1b), (a, b, c)
// cyclic, the identity that an SU(3) matrix (unitary, det 1) satisfies.  The
// gauge upload measures how far the stored links are from it and selects
// these kernels only where it holds to FP64 rounding; they read two thirds of
// the link bytes.
template <class R>
__device__ __forceinline__ void rebuild_row2(cx<R> (&u)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b1 = (a + 1) % 3, c1 = (a + 2) % 3;
        const cx<R> t = csub(cmul(u[0][b1], u[1][c1]), cmul(u[0][c1], u[1][b1]));
        u[2][a] = cmk(t.x, -t.y);
    }
}

template <class S, class R, bool REC>
__device__ __forceinline__ void load_link(const S *__restrict__ U, int mu, int Vp, unsigned s, cx<R> (&u)[3][3])
{
    const S *b = U + (size_t)(mu * 9) * (unsigned)Vp;
    if constexpr (REC) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
            ldpair<S, R>(b, Vp, p, s, u[(2 * p) / 3][(2 * p) % 3], u[(2 * p + 1) / 3][(2 * p + 1) % 3]);
        rebuild_row2(u);
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p)
            ldpair<S, R>(b, Vp, p, s, u[(2 * p) / 3][(2 * p) % 3], u[(2 * p + 1) / 3][(2 * p + 1) % 3]);
        u[2][2] = ldp<S, R>(b + (size_t)8 * (unsigned)Vp, s);
    }
}

template <class S, class R>
__device__ __forceinline__ void load_spinor(const S *__restrict__ x, int Vp, unsigned s, cx<R> (&p)[4][3])
{
#pragma unroll
    for (int q = 0; q < 6; ++q)
        ldpair<S, R>(x, Vp, q, s, p[(2 * q) / 3][(2 * q) % 3], p[(2 * q + 1) / 3][(2 * q + 1) % 3]);
}

// Output of one site: v_k = a G (diag x_k - acc_k / 2) + c1 e1_k + c2 e2_k + c3 e3_k.
template <class S, class R, bool HW, bool EPI>
__device__ __forceinline__ void write_site(const DsArgs<S> &a, size_t off, unsigned site, const cx<R> (&x)[4][3],
                                           const cx<R> (&acc)[4][3])
{
    const int Vp = a.g.Vp;
    const R diag = (R)a.diag, sc = (R)a.a;
    const R cc[3] = {(R)a.c1, (R)a.c2, (R)a.c3};
    const S *ep[3] = {a.e1, a.e2, a.e3};
    const bool nt = a.stream_hint != 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        cx<R> v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * q + h, sp = k / 3, c = k % 3;
            v[h] = cmk(diag * x[sp][c].x - (R)0.5 * acc[sp][c].x, diag * x[sp][c].y - (R)0.5 * acc[sp][c].y);
            v[h] = cscale(v[h], (HW && sp >= 2) ? -sc : sc);
        }
        if (EPI) {
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                if (!ep[t]) continue;
                cx<R> e[2];
                if (nt) ldpair_nt<S, R>(ep[t] + off, Vp, q, site, e[0], e[1]);
                else ldpair<S, R>(ep[t] + off, Vp, q, site, e[0], e[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    v[h].x = fma(cc[t], e[h].x, v[h].x);
                    v[h].y = fma(cc[t], e[h].y, v[h].y);
                }
            }
        }
        if (nt) stpair_nt<S, R>(a.y + off, Vp, q, site, v[0], v[1]);
        else stpair<S, R>(a.y + off, Vp, q, site, v[0], v[1]);
    }
}

// Where hop_dir takes its links from.  Slot mu is U_mu(s) (forward hop),
// slot 4 + mu is U_mu(s - mu) (backward hop); `site` is the site whose link
// is wanted (s or s - mu).
template <class S, class R, bool REC>
struct GlobalLinks {   // straight from the packed link field
    const S *U;
    int Vp;
    __device__ __forceinline__ void operator()(int mu, int, unsigned site, cx<R> (&u)[3][3]) const
    {
        load_link<S, R, REC>(U, mu, Vp, site, u);
    }
};

// Staged in LDS by the workgroup: [slot][component][site slot], SL site
// slots, E components per link (9, or 6 when the third row is rebuilt at
// each read: RB).
template <class R, int E, bool RB, int SL>
struct LdsLinks {
    const cx<R> *base;
    int sl;   // this thread's site slot
    __device__ __forceinline__ void operator()(int, int slot, unsigned, cx<R> (&u)[3][3]) const
    {
        const cx<R> *p = base + slot * E * SL + sl;
#pragma unroll
        for (int k = 0; k < E; ++k) u[k / 3][k % 3] = p[k * SL];
        if constexpr (RB) rebuild_row2(u);
    }
};

// Components a link occupies in the LDS stage.  Links with FP32 arithmetic
// are rebuilt once, when the workgroup stages them, and stored whole (every
// wave of the workgroup would otherwise repeat the six complex products of
// the third row for each of its eight links); FP64 keeps two rows (nine FP64
// components per link would halve the resident workgroups).
template <class R, bool REC>
__host__ __device__ constexpr int lds_link_components()
{
    return (REC && sizeof(R) == 8) ? 6 : 9;
}

// One direction, both hops, for all NR right-hand sides of this thread.
template <int MU, int NR, class S, class R, class LF>
__device__ __forceinline__ void hop_dir(const DsArgs<S> &a, const LF &links, int site, int cmu, int Lmu,
                                        int stride, const size_t (&off)[NR], const bool (&act)[NR],
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
            links(MU, MU, (unsigned)site, u);
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
            links(MU, 4 + MU, (unsigned)j, u);
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

// Site of this thread.  A wave is split into Q sub-waves of 64/Q lanes that
// cover the same 64/Q consecutive sites for Q different groups of
// right-hand sides, so a workgroup of B threads covers B/Q sites.  order 0:
// blocks walk the sites in canonical order, each XCD taking a contiguous run
// (t-chunks).  order 1: XCD x owns the z-slab [x Lz/8, (x+1) Lz/8) and walks
// it plane by plane, (z, t) planes of Lx*Ly sites in t-major order, so the
// cross-section an XCD sweeps is 1/8 of a time slice and t-neighbours are
// re-read soon after their first use.  order 3: XCD x owns the t-slab
// [x Lt/8, (x+1) Lt/8) and walks its (z, t) planes with t fastest, so t
// neighbours are one plane away and z neighbours Lt/8 planes away; only the
// two boundary slices of a slab read neighbours another XCD fetched (2/(Lt/8)
// per site, against 2/(Lz/8) for order 1).  orders 1 and 3 need Lz % 8 == 0
// (Lt % 8 == 0) and V % 64 == 0 (no padding); the launcher checks.
//
// site_in_block gives the site of position tb (0 <= tb < spb) in workgroup
// blockIdx.x when every workgroup covers spb sites.
__device__ __forceinline__ int site_in_block(const Geo &g, int order, int xcd_remap, int cols, int tb, int spb)
{
    if (order == 3) {
        const int xcd = blockIdx.x & 7;
        const int u = (blockIdx.x >> 3) * spb + tb;
        const int nt = g.Lt >> 3;
        const int q = u / g.Lxy, o = u - q * g.Lxy;
        if (q >= nt * g.Lz) return g.Vp;   // beyond the slab: no work
        const int tl = q % nt, z = q / nt;
        return o + g.Lxy * (z + g.Lz * (xcd * nt + tl));
    }
    if (order == 1) {
        // with cols > 1 the slab is walked one y-column (Ly/cols rows) at a time,
        // which shortens the distance between a site and its t neighbours
        const int xcd = blockIdx.x & 7;
        const int u = (blockIdx.x >> 3) * spb + tb;
        const int nz = g.Lz >> 3;
        const int P = g.Lxy / cols;                 // sites of one column in one (z, t) plane
        const int per_col = P * nz * g.Lt;
        const int col = u / per_col;
        if (col >= cols) return g.Vp;               // beyond the slab: no work
        const int rem = u - col * per_col;
        const int q = rem / P, o = rem - q * P + col * P;
        const int zl = q % nz, t = q / nz;
        return o + g.Lxy * (xcd * nz + zl + g.Lz * t);
    }
    const int blk = xcd_remap ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    return blk * spb + tb;
}

template <int Q>
__device__ __forceinline__ int dslash_site(const Geo &g, int order, int xcd_remap, int cols)
{
    constexpr int SL = 64 / Q;   // sites per wave
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int spb = (int)(blockDim.x >> 6) * SL;
    const int tb = wave * SL + (lane & (SL - 1));
    return site_in_block(g, order, xcd_remap, cols, tb, spb);
}

// Work of one thread after its site and first right-hand side are known:
// padding sites write zeros; other sites gather the 8 hops for NR RHS
// (links from `lf`) and write the output with the optional epilogue.
// Q == 1 means j0 is uniform over the wave, which lets the RHS offsets live
// in scalar registers.
template <class S, int NR, int Q, bool HW, bool EPI, class LF>
__device__ __forceinline__ void dslash_body_at(const DsArgs<S> &a, int site, int xc, int yc, int zc, int tc, int j0,
                                               const LF &lf);

template <class S, int NR, int Q, bool HW, bool EPI, class LF>
__device__ __forceinline__ void dslash_body(const DsArgs<S> &a, int site, int j0, const LF &lf)
{
    int rem = site;
    const int xc = rem % a.g.Lx; rem /= a.g.Lx;
    const int yc = rem % a.g.Ly; rem /= a.g.Ly;
    const int zc = rem % a.g.Lz;
    const int tc = rem / a.g.Lz;
    dslash_body_at<S, NR, Q, HW, EPI>(a, site, xc, yc, zc, tc, j0, lf);
}

// The body for a site whose coordinates are known.
template <class S, int NR, int Q, bool HW, bool EPI, class LF>
__device__ __forceinline__ void dslash_body_at(const DsArgs<S> &a, int site, int xc, int yc, int zc, int tc, int j0,
                                               const LF &lf)
{
    using R = typename StoreT<S>::real;
    const Geo &g = a.g;
    size_t off[NR];
    bool act[NR];
    int grp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int j = j0 + r;
        act[r] = j < a.n;
        const int jj = act[r] ? j : 0;
        int s = a.slots ? a.slots[jj] : jj;
        if (Q == 1) s = __builtin_amdgcn_readfirstlane(s);   // uniform over the wave
        off[r] = (size_t)s * (size_t)a.fstride;
        int gr = a.fgroup ? a.fgroup[s] : 0;
        if (Q == 1) gr = __builtin_amdgcn_readfirstlane(gr);
        grp[r] = gr;
    }
    if (site >= g.V) {   // padding sites hold zeros in every field
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!act[r]) continue;
#pragma unroll
            for (int q = 0; q < 6; ++q)
                stpair<S, R>(a.y + off[r], g.Vp, q, (unsigned)site, cmk((R)0, (R)0), cmk((R)0, (R)0));
        }
        return;
    }

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

    hop_dir<0, NR, S, R>(a, lf, site, xc, g.Lx, 1, off, act, ph, acc);
    hop_dir<1, NR, S, R>(a, lf, site, yc, g.Ly, g.Lx, off, act, ph, acc);
    hop_dir<2, NR, S, R>(a, lf, site, zc, g.Lz, g.Lxy, off, act, ph, acc);
    hop_dir<3, NR, S, R>(a, lf, site, tc, g.Lt, g.Lxyz, off, act, ph, acc);

#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (!act[r]) continue;
        cx<R> p[4][3];
        load_spinor<S, R>(a.x + off[r], g.Vp, (unsigned)site, p);
        write_site<S, R, HW, EPI>(a, off[r], (unsigned)site, p, acc[r]);
    }
}

// Q > 1: the Q sub-waves load the same link addresses in one instruction, so
// a link line is fetched once for Q NR right-hand sides while every lane keeps
// the registers of NR.
template <class S, int NR, int Q, bool HW, bool EPI, bool REC>
__global__ __launch_bounds__(256) void k_dslash(DsArgs<S> a)
{
    using R = typename StoreT<S>::real;
    const int site = dslash_site<Q>(a.g, a.order, a.xcd_remap, a.cols);
    if (site >= a.g.Vp) return;
    const int sub = (int)(threadIdx.x & 63) / (64 / Q);
    const GlobalLinks<S, R, REC> lf{a.U, a.g.Vp};
    dslash_body<S, NR, Q, HW, EPI>(a, site, (blockIdx.y * Q + sub) * NR, lf);
}

// ---------------------------------------------------------------------------
// Link-sharing variant.  The W waves of a workgroup (W = blockDim / 64: 2, 4
// or 8) cover the same 64/Q sites, each for its own Q NR right-hand sides, so
// a workgroup covers 64/Q sites for W Q NR RHS.  Before the stencil the
// workgroup copies the eight links its sites use (U_mu(s) and U_mu(s - mu))
// into LDS; every wave then reads them there, so a link crosses HBM once per
// W Q NR RHS rather than once per Q NR, without narrowing the run of
// consecutive sites each load instruction covers.  With two-row links and
// FP32 arithmetic the stage holds whole links: the third row is rebuilt once
// per workgroup instead of once per wave.  Threads of padding sites take
// part in the copy and the barrier and only then leave.
//
// Copy one link (site s, its coordinates given; slot 0..3 = U_mu(s), 4..7 =
// U_mu(s - mu)) into LDS, E components, rebuilding the third row when the
// stored rows are two (REC) and the stage holds nine (E == 9).
template <class S, class R, bool REC, int E, int SL>
__device__ __forceinline__ void stage_link(const DsArgs<S> &a, int slot, int s, int xc, int yc, int zc, int tc,
                                           cx<R> *dst)
{
    const Geo &g = a.g;
    const int mu = slot & 3;
    int src = s;
    if (slot >= 4) {   // backward neighbour s - mu, wrapping
        const int c = mu == 0 ? xc : mu == 1 ? yc : mu == 2 ? zc : tc;
        const int L = mu == 0 ? g.Lx : mu == 1 ? g.Ly : mu == 2 ? g.Lz : g.Lt;
        const int stride = mu == 0 ? 1 : mu == 1 ? g.Lx : mu == 2 ? g.Lxy : g.Lxyz;
        src = (c == 0) ? s + (L - 1) * stride : s - stride;
    }
    // the same 16-byte pair loads as the other kernels (full cache lines over a
    // run of consecutive sites)
    const S *ub = a.U + (size_t)(mu * 9) * (unsigned)g.Vp;
    if constexpr (REC && E == 9) {
        cx<R> u[3][3];
        load_link<S, R, true>(a.U, mu, g.Vp, (unsigned)src, u);   // two rows read, third rebuilt
#pragma unroll
        for (int k = 0; k < 9; ++k) dst[k * SL] = u[k / 3][k % 3];
    } else {
#pragma unroll
        for (int p = 0; p < E / 2; ++p) {   // components 0..5 (two rows) or 0..7
            cx<R> c0, c1;
            ldpair<S, R>(ub, g.Vp, p, (unsigned)src, c0, c1);
            dst[(2 * p) * SL] = c0;
            dst[(2 * p + 1) * SL] = c1;
        }
        if constexpr (E == 9) dst[8 * SL] = ldp<S, R>(ub + (size_t)8 * (unsigned)g.Vp, (unsigned)src);
    }
}

__device__ __forceinline__ void site_coords(const Geo &g, int s, int &xc, int &yc, int &zc, int &tc)
{
    int rem = s;
    xc = rem % g.Lx; rem /= g.Lx;
    yc = rem % g.Ly; rem /= g.Ly;
    zc = rem % g.Lz;
    tc = rem / g.Lz;
}

template <class S, int NR, int Q, bool HW, bool EPI, bool REC>
__global__ __launch_bounds__(512) void k_dslash_lds(DsArgs<S> a)
{
    using R = typename StoreT<S>::real;
    constexpr int SL = 64 / Q, E = lds_link_components<R, REC>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<R> *lk = reinterpret_cast<cx<R> *>(lds_raw);   // [8][E][SL]
    const Geo &g = a.g;
    const int W = (int)(blockDim.x >> 6), wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int sl = lane & (SL - 1);
    const int site = site_in_block(g, a.order, a.xcd_remap, a.cols, sl, SL);
    int xc = 0, yc = 0, zc = 0, tc = 0;
    if (site < g.V) site_coords(g, site, xc, yc, zc, tc);

    if constexpr (Q == 1) {
        // thread (wave w, lane l) stages slots w, w + W, ... of its own site
        for (int slot = wave; slot < 8; slot += W) {
            cx<R> *dst = lk + slot * E * SL + sl;
            if (site >= g.V) {   // padding or beyond the slab: never read
#pragma unroll
                for (int k = 0; k < E; ++k) dst[k * SL] = cmk((R)0, (R)0);
            } else {
                stage_link<S, R, REC, E, SL>(a, slot, site, xc, yc, zc, tc, dst);
            }
        }
    } else {
        for (int idx = (int)threadIdx.x; idx < 8 * SL; idx += (int)blockDim.x) {
            const int slot = idx / SL, ss = idx - slot * SL;
            const int s = site_in_block(g, a.order, a.xcd_remap, a.cols, ss, SL);
            cx<R> *dst = lk + slot * E * SL + ss;
            if (s >= g.V) {
#pragma unroll
                for (int k = 0; k < E; ++k) dst[k * SL] = cmk((R)0, (R)0);
                continue;
            }
            int x2, y2, z2, t2;
            site_coords(g, s, x2, y2, z2, t2);
            stage_link<S, R, REC, E, SL>(a, slot, s, x2, y2, z2, t2, dst);
        }
    }
    __syncthreads();

    if (site >= g.Vp) return;
    const int sub = lane / SL;
    const int j0 = ((blockIdx.y * W + wave) * Q + sub) * NR;
    const LdsLinks<R, E, REC && E == 6, SL> lf{lk, sl};
    dslash_body_at<S, NR, Q, HW, EPI>(a, site, xc, yc, zc, tc, j0, lf);
}

// ---------------------------------------------------------------------------
// t-marching variant.  Each thread owns one (x, y, z) site and one RHS and
// walks t over a chunk [t0, t1), keeping psi(t-1), psi(t), psi(t+1) and the
// backward time link in registers: the two time neighbours cost no loads and
// every input spinor is fetched once per chunk.  A wave covers 64 consecutive
// sites of one (z, t) plane, so x and y neighbours come from lines the wave
// itself touches in the same step (L1); the W waves of a workgroup (W = 4 or
// 8) are W RHS on the same sites, so link loads are shared through L1: the
// links stream from memory once per W right-hand sides.  Blocks walk z
// fastest within an XCD, so z neighbours are loaded by workgroups running at
// the same time on the same XCD (L2).
//
// Block b: XCD b & 7, local index m = b >> 3 decomposed as
//   m = z + Lz (ob + nob (tc + ntc rg))
// with ob the 64-site block of the (x, y) plane, tc the t-chunk and rg the
// group of W RHS.  Needs V % 64 == 0 (no padding); the launcher checks.
template <class S, bool HW, bool EPI, int W, bool REC>
__global__ __launch_bounds__(64 * W) void k_dslash_tm(DsArgs<S> a)
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
    const int j = rg * W + wave;
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
    load_link<S, R, REC>(a.U, 3, Vp, (unsigned)site_at(tm1), utm);

    const size_t offs[1] = {off};
    const bool acts[1] = {true};
    const R bt = (R)g.bcf[3];

    for (int t = t0; t < t1; ++t) {
        const int site = site_at(t);
        const int tp1 = (t == g.Lt - 1) ? 0 : t + 1;
        load_spinor<S, R>(x, Vp, (unsigned)site_at(tp1), pn);
        cx<R> utc[3][3];
        load_link<S, R, REC>(a.U, 3, Vp, (unsigned)site, utc);
        const cx<double> pd = a.phase[grp * g.Lt + t];
        const cx<R> ph[1] = {cmk((R)pd.x, (R)pd.y)};

        cx<R> acc[1][4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[0][sp][c] = cmk((R)0, (R)0);

        const GlobalLinks<S, R, REC> lf{a.U, Vp};
        hop_dir<0, 1, S, R>(a, lf, site, xc, g.Lx, 1, offs, acts, ph, acc);
        hop_dir<1, 1, S, R>(a, lf, site, yc, g.Ly, g.Lx, offs, acts, ph, acc);
        hop_dir<2, 1, S, R>(a, lf, site, z, g.Lz, g.Lxy, offs, acts, ph, acc);

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

        write_site<S, R, HW, EPI>(a, off, (unsigned)site, pc, acc[0]);

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

template <class S, int W>
static hipError_t launch_tm_w(const DsArgs<S> &a, bool hw, bool epi, hipStream_t st)
{
    DsArgs<S> b = a;
    if (b.tchunk <= 0 || b.tchunk > a.g.Lt) b.tchunk = a.g.Lt;
    const int nob = (a.g.Lxy + 63) / 64;
    const int ntc = (a.g.Lt + b.tchunk - 1) / b.tchunk;
    const long nblk = (long)a.g.Lz * nob * ntc * ((a.n + W - 1) / W);
    const long padded = (nblk + 7) / 8 * 8;
    if (padded > 0x7fffffffL) return hipErrorInvalidValue;
    const dim3 blk(64 * W), grid((unsigned)padded);
    if (a.recon) {
        if (epi) hipLaunchKernelGGL((k_dslash_tm<S, true, true, W, true>), grid, blk, 0, st, b);
        else if (hw) hipLaunchKernelGGL((k_dslash_tm<S, true, false, W, true>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_dslash_tm<S, false, false, W, true>), grid, blk, 0, st, b);
    } else {
        if (epi) hipLaunchKernelGGL((k_dslash_tm<S, true, true, W, false>), grid, blk, 0, st, b);
        else if (hw) hipLaunchKernelGGL((k_dslash_tm<S, true, false, W, false>), grid, blk, 0, st, b);
        else hipLaunchKernelGGL((k_dslash_tm<S, false, false, W, false>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

// block = 64 W threads, W = 8 right-hand sides per workgroup for block 512, else 4.
template <class S>
static hipError_t launch_tm(const DsArgs<S> &a, bool hw, bool epi, int block, hipStream_t st)
{
    if (block == 512) return launch_tm_w<S, 8>(a, hw, epi, st);
    return launch_tm_w<S, 4>(a, hw, epi, st);
}

// One site-parallel kernel: the three operator kinds (fused epilogue, H_w,
// D_w) for a link format.  With an occupancy cap the kernel is allowed more
// than the default 64 KiB of dynamic LDS (once per kernel).
template <class S, int NR, int Q, bool REC>
static hipError_t launch_site(const DsArgs<S> &b, bool hw, bool epi, dim3 grid, int block, size_t lds,
                              hipStream_t st)
{
    const void *fn = epi  ? (const void *)k_dslash<S, NR, Q, true, true, REC>
                     : hw ? (const void *)k_dslash<S, NR, Q, true, false, REC>
                          : (const void *)k_dslash<S, NR, Q, false, false, REC>;
    if (lds > 0) {
        static bool raised[3] = {false, false, false};
        const int ki = epi ? 0 : (hw ? 1 : 2);
        if (!raised[ki]) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
            raised[ki] = true;
        }
    }
    if (epi)
        hipLaunchKernelGGL((k_dslash<S, NR, Q, true, true, REC>), grid, dim3(block), lds, st, b);
    else if (hw)
        hipLaunchKernelGGL((k_dslash<S, NR, Q, true, false, REC>), grid, dim3(block), lds, st, b);
    else
        hipLaunchKernelGGL((k_dslash<S, NR, Q, false, false, REC>), grid, dim3(block), lds, st, b);
    return hipGetLastError();
}

template <class S, int NR, int Q>
static hipError_t launch_nr(const DsArgs<S> &a, bool hw, bool epi, int block, hipStream_t st)
{
    // Occupancy cap: reserving LDS the kernel does not use limits the number of
    // resident workgroups per CU (160 KiB of LDS per CU on gfx950), which
    // narrows the window of sites in flight so that stencil neighbours are
    // re-read while still in L2.
    const size_t lds = a.blocks_per_cu > 0 ? (size_t)(160 * 1024) / (size_t)a.blocks_per_cu - 256 : 0;
    const int spb = block / Q;   // sites per workgroup
    // cover every padded site: the padding [V, Vp) is rewritten with zeros
    int nbx = (a.g.Vp + spb - 1) / spb;
    DsArgs<S> b = a;
    b.xcd_remap = 0;
    if (b.order == 1 && (a.g.Lz % 8 != 0 || a.g.V % 64 != 0)) b.order = 0;
    if (b.cols < 1 || a.g.Ly % b.cols != 0) b.cols = 1;
    if (b.order == 3 && (a.g.Lt % 8 != 0 || a.g.V % 64 != 0)) b.order = 0;
    if (b.order == 2) b.order = 0;   // t-marching shapes that cannot march use order 0
    if (b.order == 1 || b.order == 3) {
        const int per_xcd = a.g.V / 8;
        nbx = 8 * ((per_xcd + spb - 1) / spb);
    } else if (nbx >= 64) {   // pad to a multiple of 8 for the XCD remap
        nbx = (nbx + 7) & ~7;
        b.xcd_remap = 1;
    }
    const dim3 grid(nbx, (a.n + NR * Q - 1) / (NR * Q));
    if (a.recon) return launch_site<S, NR, Q, true>(b, hw, epi, grid, block, lds, st);
    return launch_site<S, NR, Q, false>(b, hw, epi, grid, block, lds, st);
}

template <class S, int NR, int Q, bool REC>
static hipError_t launch_lds_kernel(const DsArgs<S> &b, bool hw, bool epi, dim3 grid, int W, size_t lds,
                                    hipStream_t st)
{
    const void *fn = epi  ? (const void *)k_dslash_lds<S, NR, Q, true, true, REC>
                     : hw ? (const void *)k_dslash_lds<S, NR, Q, true, false, REC>
                          : (const void *)k_dslash_lds<S, NR, Q, false, false, REC>;
    static bool raised[3] = {false, false, false};
    const int ki = epi ? 0 : (hw ? 1 : 2);
    if (!raised[ki]) {   // staged links of FP64 full links exceed the default 64 KiB
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        raised[ki] = true;
    }
    const dim3 blk(64 * W);
    if (epi)
        hipLaunchKernelGGL((k_dslash_lds<S, NR, Q, true, true, REC>), grid, blk, lds, st, b);
    else if (hw)
        hipLaunchKernelGGL((k_dslash_lds<S, NR, Q, true, false, REC>), grid, blk, lds, st, b);
    else
        hipLaunchKernelGGL((k_dslash_lds<S, NR, Q, false, false, REC>), grid, blk, lds, st, b);
    return hipGetLastError();
}

// Link-sharing launch: W = a.wshare waves per workgroup on the same 64/Q
// sites; LDS holds the staged links (more if the occupancy cap asks for it).
template <class S, int NR, int Q>
static hipError_t launch_lds(const DsArgs<S> &a, bool hw, bool epi, hipStream_t st)
{
    using R = typename StoreT<S>::real;
    constexpr int SL = 64 / Q;
    const int W = a.wshare;
    const int E = a.recon ? lds_link_components<R, true>() : lds_link_components<R, false>();
    const size_t need = (size_t)8 * E * SL * sizeof(cx<R>);
    const size_t capr = a.blocks_per_cu > 0 ? (size_t)(160 * 1024) / (size_t)a.blocks_per_cu - 256 : 0;
    const size_t lds = need > capr ? need : capr;
    int nbx = (a.g.Vp + SL - 1) / SL;
    DsArgs<S> b = a;
    b.xcd_remap = 0;
    if (b.order == 1 && (a.g.Lz % 8 != 0 || a.g.V % 64 != 0)) b.order = 0;
    if (b.cols < 1 || a.g.Ly % b.cols != 0) b.cols = 1;
    if (b.order == 3 && (a.g.Lt % 8 != 0 || a.g.V % 64 != 0)) b.order = 0;
    if (b.order == 2) b.order = 0;
    if (b.order == 1 || b.order == 3) {
        nbx = 8 * ((a.g.V / 8 + SL - 1) / SL);
    } else if (nbx >= 64) {
        nbx = (nbx + 7) & ~7;
        b.xcd_remap = 1;
    }
    const dim3 grid(nbx, (a.n + NR * Q * W - 1) / (NR * Q * W));
    if (a.recon) return launch_lds_kernel<S, NR, Q, true>(b, hw, epi, grid, W, lds, st);
    return launch_lds_kernel<S, NR, Q, false>(b, hw, epi, grid, W, lds, st);
}

// split = Q sub-waves per wave (1, 2, 4, 8; Q > 1 with NR <= 2 only; Q = 8
// keeps whole 128-byte lines per sub-wave for 16-byte elements only).
template <class S>
hipError_t launch_dslash(const DsArgs<S> &a, bool hw, bool epi, int nr, int block, int split, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    if (block < 64 || block > 512 || (block & 63)) return hipErrorInvalidValue;
    if (a.order == 2 && a.g.V % 64 == 0) return launch_tm<S>(a, hw, epi, block, st);
    if (a.wshare == 2 || a.wshare == 4 || a.wshare == 8) {   // waves share sites and staged links
        if (nr == 1) {
            if (split == 1) return launch_lds<S, 1, 1>(a, hw, epi, st);
            if (split == 2) return launch_lds<S, 1, 2>(a, hw, epi, st);
            if (split == 4) return launch_lds<S, 1, 4>(a, hw, epi, st);
        } else if (nr == 2) {
            if (split == 1) return launch_lds<S, 2, 1>(a, hw, epi, st);
            if (split == 2) return launch_lds<S, 2, 2>(a, hw, epi, st);
            if (split == 4) return launch_lds<S, 2, 4>(a, hw, epi, st);
        }
        return hipErrorInvalidValue;
    }
    if (a.wshare != 1) return hipErrorInvalidValue;
    if (block > 256) block = 256;   // wider workgroups only for the t-marching kernel
    if (split == 2 || split == 4) {
        if (nr == 1) return split == 2 ? launch_nr<S, 1, 2>(a, hw, epi, block, st) : launch_nr<S, 1, 4>(a, hw, epi, block, st);
        if (nr == 2) return split == 2 ? launch_nr<S, 2, 2>(a, hw, epi, block, st) : launch_nr<S, 2, 4>(a, hw, epi, block, st);
        return hipErrorInvalidValue;
    }
    if (split == 8) {
        if constexpr (sizeof(S) == 4) return hipErrorInvalidValue;   // BF16: 32-byte pieces of a line
        else {
            if (nr == 1) return launch_nr<S, 1, 8>(a, hw, epi, block, st);
            if (nr == 2) return launch_nr<S, 2, 8>(a, hw, epi, block, st);
            return hipErrorInvalidValue;
        }
    }
    if (split != 1) return hipErrorInvalidValue;
    switch (nr) {
    case 1: return launch_nr<S, 1, 1>(a, hw, epi, block, st);
    case 2: return launch_nr<S, 2, 1>(a, hw, epi, block, st);
    case 4: return launch_nr<S, 4, 1>(a, hw, epi, block, st);
    case 8: return launch_nr<S, 8, 1>(a, hw, epi, block, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_dslash<double2>(const DsArgs<double2> &, bool, bool, int, int, int, hipStream_t);
template hipError_t launch_dslash<float2>(const DsArgs<float2> &, bool, bool, int, int, int, hipStream_t);
template hipError_t launch_dslash<uint32_t>(const DsArgs<uint32_t> &, bool, bool, int, int, int, hipStream_t);

}  // namespace ov
