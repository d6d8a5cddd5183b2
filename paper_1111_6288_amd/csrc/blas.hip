// Streaming kernels of the overlap path: layout packing, precision
// conversion, linear combinations (with an optional fused squared norm),
// batched inner products with a fixed-order two-stage reduction, and the
// per-RHS CG scalar updates.  All of them are HBM-bound; they read and write
// whole planes with consecutive lanes on consecutive sites.
#include <algorithm>

#include "ov_device.h"
#include "ov_internal.h"

namespace ov {

// Sum of one double over a workgroup of up to 1024 threads in a fixed order:
// a butterfly over the 64 lanes of each wave (cross-lane shuffles, no LDS),
// then the per-wave sums added by wave index.  The result is valid in
// thread 0.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum(double v)
{
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) v += __shfl_xor(v, w, 64);
    __shared__ double wsum[16];
    const int wave = (int)(threadIdx.x >> 6), nw = (int)((blockDim.x + 63) >> 6);
    if ((threadIdx.x & 63) == 0) wsum[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) s += wsum[k];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- packing
// canonical complex128 [n][V][4][3]  <->  internal field layout [slot]
template <class S>
__global__ void k_pack_spinor(const double2 *__restrict__ in, S *__restrict__ out, long fstride,
                              const int *slots, int n, int V, int Vp)
{
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (site >= Vp || j >= n) return;
    const int s = slots ? slots[j] : j;
    S *o = out + (long)s * fstride;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        cx<double> v = {0.0, 0.0};
        if (site < V) {
            double2 w = in[((long)j * V + site) * 12 + k];
            v = {w.x, w.y};
        }
        stc<double>(o, cpos<S>(k, site, Vp), v);
    }
}

template <class S>
__global__ void k_unpack_spinor(const S *__restrict__ in, double2 *__restrict__ out, long fstride,
                                const int *slots, int n, int V, int Vp)
{
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (site >= V || j >= n) return;
    const int s = slots ? slots[j] : j;
    const S *p = in + (long)s * fstride;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        cx<double> v = ldc<double>(p, cpos<S>(k, site, Vp));
        out[((long)j * V + site) * 12 + k] = make_double2(v.x, v.y);
    }
}

// canonical [4][V][3][3]  ->  internal link layout
template <class S>
__global__ void k_pack_links(const double2 *__restrict__ in, S *__restrict__ out, int V, int Vp)
{
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (site >= Vp) return;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        cx<double> v = {0.0, 0.0};
        if (site < V) {
            double2 w = in[((long)mu * V + site) * 9 + k];
            v = {w.x, w.y};
        }
        stc<double>(out, lpos<S>(mu, k, site, Vp), v);
    }
}

// ---------------------------------------------------------------- time-slice norms
// part[(j Lt + t) nb + blk] = sum over the sites of block blk of time slice t
// of sum_k |x_j(site, k)|^2, canonical complex128 input [n][V][12] (t is the
// slowest site index, so a time slice is Lxyz consecutive sites).
__global__ __launch_bounds__(256) void k_slice_norm2(const double2 *__restrict__ x, long V, int Lxyz, int Lt,
                                                     int nb, double *__restrict__ part)
{
    const int blk = blockIdx.x, t = blockIdx.y, j = blockIdx.z;
    double s = 0.0;
    for (int o = blk * blockDim.x + threadIdx.x; o < Lxyz; o += nb * blockDim.x) {
        const double2 *p = x + ((long)j * V + (long)t * Lxyz + o) * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) s += p[k].x * p[k].x + p[k].y * p[k].y;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[((long)j * Lt + t) * nb + blk] = s;
}

// out[j Lt + t] = sum_blk part[(j Lt + t) nb + blk]  (fixed order)
__global__ void k_slice_finish(const double *__restrict__ part, int nb, int m, double *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(long)e * nb + b];
    out[e] = s;
}

// out_j(x) = w[t(x)] gamma5 in_j(x), canonical complex128 [n][V][12] (spin = k / 3).
__global__ __launch_bounds__(256) void k_weight_g5(const double2 *__restrict__ in, const double *__restrict__ w,
                                                   long V, int Lxyz, int n, double2 *__restrict__ out)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * V * 12) return;
    const long site = (e / 12) % V;
    const int k = (int)(e % 12);
    const double s = w[site / Lxyz] * (k < 6 ? 1.0 : -1.0);
    const double2 v = in[e];
    out[e] = make_double2(s * v.x, s * v.y);
}

hipError_t launch_weight_g5(const double2 *in, const double *w, long V, int Lxyz, int n, double2 *out,
                            hipStream_t st)
{
    const long m = (long)n * V * 12;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_weight_g5, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, in, w, V, Lxyz, n, out);
    return hipGetLastError();
}

// Count of non-finite doubles in a buffer (result accumulated atomically).
__global__ void k_count_nonfinite(const double *__restrict__ p, long n, int *count)
{
    int bad = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        bad += !isfinite(p[i]);
    if (bad) atomicAdd(count, bad);
}

// How far each link is from the SU(3) identity u_2 = conj(u_0 x u_1) (rows
// u_0, u_1, u_2, cross product over the colour index), in FP64.  One wave
// reduces its lanes before the atomic.  Non-negative doubles order like their
// bit patterns, so an unsigned 64-bit max is a max of the values.
__global__ __launch_bounds__(256) void k_link_row3_dev(const double2 *__restrict__ U, long nl,
                                                       unsigned long long *out)
{
    double worst = 0;
    for (long l = blockIdx.x * (long)blockDim.x + threadIdx.x; l < nl; l += (long)gridDim.x * blockDim.x) {
        const double2 *m = U + 9 * l;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const double2 p = m[b], q = m[3 + c], r = m[c], s = m[3 + b];
            const double tr = (p.x * q.x - p.y * q.y) - (r.x * s.x - r.y * s.y);
            const double ti = (p.x * q.y + p.y * q.x) - (r.x * s.y + r.y * s.x);
            const double dr = m[6 + a].x - tr, di = m[6 + a].y + ti;
            worst = fmax(worst, sqrt(dr * dr + di * di));
        }
    }
    for (int w = 32; w >= 1; w >>= 1) worst = fmax(worst, __shfl_xor(worst, w, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(worst));
}

// How far the links that the FP32 and BF16 kernels apply are from the
// uploaded FP64 links: out[2 p + r] = max over links of the Frobenius norm of
// U_eff - U for p = 0 (FP32 storage), 1 (BF16 storage) and r = 0 (nine
// entries read), 1 (rows 0, 1 read, row 2 rebuilt as conj(u_0 x u_1)).  The
// stored entries are rounded exactly as the packing kernel rounds them; the
// rebuild is evaluated in FP64 here (the kernels' FP32 evaluation adds at
// most a few FP32 ulps, which the caller allows for).  Since the Frobenius
// norm bounds the spectral one, ||H_w(U_eff)|| <= ||H_w(U)|| + 4 out[.].
__device__ __forceinline__ double2 round_store(double2 v, int p)
{
    if (p == 0) return make_double2((double)(float)v.x, (double)(float)v.y);
    const uint32_t w = f2bf((float)v.x) | (f2bf((float)v.y) << 16);
    return make_double2((double)bf16_lo(w), (double)bf16_hi(w));
}

__global__ __launch_bounds__(256) void k_link_round_dev(const double2 *__restrict__ U, long nl,
                                                        unsigned long long *out)
{
    double worst[4] = {0, 0, 0, 0};
    for (long l = blockIdx.x * (long)blockDim.x + threadIdx.x; l < nl; l += (long)gridDim.x * blockDim.x) {
        const double2 *m = U + 9 * l;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            double2 r[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) r[k] = round_store(m[k], p);
            double top = 0, full = 0, reb = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double dx = r[k].x - m[k].x, dy = r[k].y - m[k].y;
                top += dx * dx + dy * dy;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double dx = r[6 + a].x - m[6 + a].x, dy = r[6 + a].y - m[6 + a].y;
                full += dx * dx + dy * dy;
                const int b = (a + 1) % 3, c = (a + 2) % 3;
                const double2 pb = r[b], qc = r[3 + c], pc = r[c], qb = r[3 + b];
                const double tr = (pb.x * qc.x - pb.y * qc.y) - (pc.x * qb.x - pc.y * qb.y);
                const double ti = (pb.x * qc.y + pb.y * qc.x) - (pc.x * qb.y + pc.y * qb.x);
                const double ex = tr - m[6 + a].x, ey = -ti - m[6 + a].y;
                reb += ex * ex + ey * ey;
            }
            worst[2 * p] = fmax(worst[2 * p], sqrt(top + full));
            worst[2 * p + 1] = fmax(worst[2 * p + 1], sqrt(top + reb));
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double v = worst[i];
        for (int w = 32; w >= 1; w >>= 1) v = fmax(v, __shfl_xor(v, w, 64));
        if ((threadIdx.x & 63) == 0) atomicMax(out + i, (unsigned long long)__double_as_longlong(v));
    }
}

hipError_t launch_link_round_dev(const double2 *U, long nl, unsigned long long *out, hipStream_t st)
{
    long nb = (nl + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_link_round_dev, dim3(nb), dim3(256), 0, st, U, nl, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- lincomb
// out_s = sum_j coef_j(s) * G_j in_j,s   (G_j = gamma5 if bit j of g5mask)
// optionally red[s][blk] = sum |out_s|^2 over this block's elements.
template <class SI, class SO>
__global__ __launch_bounds__(256) void k_lincomb(LcArgs<SI, SO> a)
{
    const int j = blockIdx.y;
    if (j >= a.n) return;
    const int s = a.slots ? a.slots[j] : j;
    cx<double> cf[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (t < a.nin) {
            const double2 c = a.coef[t] ? a.coef[t][a.coef_by_slot ? s : j] : a.cconst[t];
            cf[t] = {c.x, c.y};
        }
    }
    const long ne = 12L * a.Vp;
    const long half = 6L * a.Vp;
    double nrm = 0.0;
    auto elem = [&](long ei, long eo, bool lower) {
        cx<double> v = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            if (t < a.nin) {
                cx<double> x = ldc<double>(a.in[t] + (long)s * a.istride[t], ei);
                if (((a.g5mask >> t) & 1) && lower) x = {-x.x, -x.y};
                cfma(v, cf[t], x);
            }
        }
        stc<double>(a.out + (long)s * a.ostride, eo, v);
        if (a.red) nrm += v.x * v.x + v.y * v.y;
    };
    const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x, nth = (long)gridDim.x * blockDim.x;
    if constexpr (Pair<SI>::E == Pair<SO>::E) {
        for (long e = tid; e < ne; e += nth) elem(e, e, e >= half);
    } else {
        // layouts differ: walk pair-planes, in which both name the same numbers
        for (int p = 0; p < 6; ++p)
            for (long r = tid; r < 2L * a.Vp; r += nth) elem(ppos<SI>(p, r, a.Vp), ppos<SO>(p, r, a.Vp), p >= 3);
    }
    if (a.red) {
        nrm = block_sum(nrm);
        if (threadIdx.x == 0) a.red[(long)j * gridDim.x + blockIdx.x] = nrm;
    }
}

// ---------------------------------------------------------------- dot
// part[j][blk] = sum over block of conj(G a_s) b_s
template <class SA, class SB>
__global__ __launch_bounds__(256) void k_dot(const SA *__restrict__ a, long astride, const SB *__restrict__ b,
                                             long bstride, const int *slots, int n, int Vp, int g5a,
                                             double2 *part)
{
    const int j = blockIdx.y;
    if (j >= n) return;
    const int s = slots ? slots[j] : j;
    const long ne = 12L * Vp, half = 6L * Vp;
    cx<double> acc = {0.0, 0.0};
    const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x, nth = (long)gridDim.x * blockDim.x;
    auto elem = [&](long ea, long eb, bool lower) {
        cx<double> x = ldc<double>(a + (long)s * astride, ea);
        if (g5a && lower) x = {-x.x, -x.y};
        cfmac(acc, x, ldc<double>(b + (long)s * bstride, eb));
    };
    if constexpr (Pair<SA>::E == Pair<SB>::E) {
        for (long e = tid; e < ne; e += nth) elem(e, e, e >= half);
    } else {
        for (int p = 0; p < 6; ++p)
            for (long r = tid; r < 2L * Vp; r += nth) elem(ppos<SA>(p, r, Vp), ppos<SB>(p, r, Vp), p >= 3);
    }
    const double re = block_sum(acc.x), im = block_sum(acc.y);
    if (threadIdx.x == 0) part[(long)j * gridDim.x + blockIdx.x] = make_double2(re, im);
}

// out[slot(j)] = sum_b part[j][b] in a fixed order (one workgroup per j)
__global__ void k_reduce_c(const double2 *__restrict__ part, int nb, int n, double2 *out, const int *oslots)
{
    const int j = blockIdx.x;
    if (j >= n) return;
    double r = 0, i = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double2 v = part[(long)j * nb + b];
        r += v.x;
        i += v.y;
    }
    r = block_sum(r);
    i = block_sum(i);
    if (threadIdx.x == 0) out[oslots ? oslots[j] : j] = make_double2(r, i);
}

__global__ void k_reduce_r(const double *__restrict__ part, int nb, int n, double *out, const int *oslots)
{
    const int j = blockIdx.x;
    if (j >= n) return;
    double r = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) r += part[(long)j * nb + b];
    r = block_sum(r);
    if (threadIdx.x == 0) out[oslots ? oslots[j] : j] = r;
}

// ---------------------------------------------------------------- CG scalars
// alpha_j = active_j ? rr_j / Re(pAp_j) : 0 ; stored as complex coefficients
// +alpha (for x += alpha p) and -alpha (for r -= alpha Ap).
__global__ void k_cg_alpha(const double *rr, const double2 *pAp, const int *active, int n,
                           double2 *alpha_pos, double2 *alpha_neg)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double al = 0.0;
    if (active[j] && pAp[j].x > 0.0) al = rr[j] / pAp[j].x;
    alpha_pos[j] = make_double2(al, 0.0);
    alpha_neg[j] = make_double2(-al, 0.0);
}

// beta_j = rr_new / rr_old; rr_old <- rr_new; deactivate when rr_new <= stop_j
// (a NaN residual deactivates too).  iters_j (optional) counts the
// iterations completed while active, so the host may read the active flags
// late without losing the per-RHS counts.
__global__ void k_cg_beta(const double *rr_new, double *rr, int *active, const double *stop, int n,
                          double2 *beta, int *iters)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double be = 0.0;
    if (active[j]) {
        be = rr[j] > 0.0 ? rr_new[j] / rr[j] : 0.0;
        rr[j] = rr_new[j];
        if (!(rr_new[j] > stop[j])) active[j] = 0;
        if (iters) iters[j] += 1;
    }
    beta[j] = make_double2(be, 0.0);
}

// p[0..n) = v (a fill kernel: unlike a memset node it is safe inside a captured graph)
__global__ void k_fill_int(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Norm check of the sign pipeline.  For a Hermitian Q with spectrum in
// [-1, 1], ||Q P(Q^2) chi|| <= M ||chi|| with M = max_{|q| <= 1} |q P(q^2)|;
// bound2 = (slack M)^2.  A right-hand side whose w = Q P(Q^2) chi violates
// the bound (or whose norms are not finite) sets *flag: the polynomial was
// evaluated outside [-1, 1], i.e. the norm bound is below ||H_w||.
__global__ void k_norm_breach(const double2 *chi2, const double2 *w2, const int *oslots, int n, double bound2,
                              int *flag)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int s = oslots ? oslots[j] : j;
    const double c = chi2[s].x, w = w2[s].x;
    if (!(w <= bound2 * c) && !(w == 0.0 && c == 0.0)) *flag = 1;
}

// G[t] = sum_j part[j Lt + t] over the n rows in order j = 0, 1, ...
__global__ void k_sum_rows(const double *__restrict__ part, int n, int Lt, double *__restrict__ G)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Lt) return;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += part[(long)j * Lt + t];
    G[t] = s;
}

// ---------------------------------------------------------------- launchers
static inline int nblocks_for(long ne, int n)
{
    // about 8k workgroups in total, at least one per RHS, at most one per 256 elements
    long want = 8192 / (n > 0 ? n : 1);
    long maxb = (ne + 255) / 256;
    if (want < 1) want = 1;
    if (want > maxb) want = maxb;
    return (int)want;
}

template <class S>
hipError_t launch_pack_spinor(const double2 *in, S *out, long fstride, const int *slots, int n, int V,
                              int Vp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((Vp + 255) / 256, n);
    hipLaunchKernelGGL((k_pack_spinor<S>), grid, dim3(256), 0, st, in, out, fstride, slots, n, V, Vp);
    return hipGetLastError();
}

template <class S>
hipError_t launch_unpack_spinor(const S *in, double2 *out, long fstride, const int *slots, int n, int V,
                                int Vp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((V + 255) / 256, n);
    hipLaunchKernelGGL((k_unpack_spinor<S>), grid, dim3(256), 0, st, in, out, fstride, slots, n, V, Vp);
    return hipGetLastError();
}

template <class S>
hipError_t launch_pack_links(const double2 *in, S *out, int V, int Vp, hipStream_t st)
{
    dim3 grid((Vp + 255) / 256, 4);
    hipLaunchKernelGGL((k_pack_links<S>), grid, dim3(256), 0, st, in, out, V, Vp);
    return hipGetLastError();
}

int slice_norm2_blocks(int Lxyz) { return std::max(1, std::min(64, (Lxyz + 255) / 256)); }

hipError_t launch_slice_norm2(const double2 *x, int n, long V, int Lxyz, int Lt, double *part, double *out,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nb = slice_norm2_blocks(Lxyz);
    hipLaunchKernelGGL(k_slice_norm2, dim3(nb, Lt, n), dim3(256), 0, st, x, V, Lxyz, Lt, nb, part);
    const int m = n * Lt;
    hipLaunchKernelGGL(k_slice_finish, dim3((m + 255) / 256), dim3(256), 0, st, part, nb, m, out);
    return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double *p, long n, int *count, hipStream_t st)
{
    long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nb), dim3(256), 0, st, p, n, count);
    return hipGetLastError();
}

hipError_t launch_link_row3_dev(const double2 *U, long nl, unsigned long long *out, hipStream_t st)
{
    long nb = (nl + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_link_row3_dev, dim3(nb), dim3(256), 0, st, U, nl, out);
    return hipGetLastError();
}

template <class SI, class SO>
hipError_t launch_lincomb(LcArgs<SI, SO> a, hipStream_t st, int *nblk_out)
{
    if (a.n <= 0) return hipSuccess;
    const int nb = nblocks_for(12L * a.Vp, a.n);
    if (nblk_out) *nblk_out = nb;
    hipLaunchKernelGGL((k_lincomb<SI, SO>), dim3(nb, a.n), dim3(256), 0, st, a);
    return hipGetLastError();
}

int lincomb_blocks(int Vp, int n) { return nblocks_for(12L * Vp, n); }

template <class SA, class SB>
hipError_t launch_dot(const SA *a, long astride, const SB *b, long bstride, const int *slots, int n, int Vp,
                      int g5a, double2 *part, double2 *out, const int *oslots, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nb = nblocks_for(12L * Vp, n);
    hipLaunchKernelGGL((k_dot<SA, SB>), dim3(nb, n), dim3(256), 0, st, a, astride, b, bstride, slots, n, Vp,
                       g5a, part);
    hipLaunchKernelGGL(k_reduce_c, dim3(n), dim3(256), 0, st, part, nb, n, out, oslots);
    return hipGetLastError();
}

hipError_t launch_reduce_r(const double *part, int nb, int n, double *out, const int *oslots, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_r, dim3(n), dim3(256), 0, st, part, nb, n, out, oslots);
    return hipGetLastError();
}

hipError_t launch_cg_alpha(const double *rr, const double2 *pAp, const int *active, int n, double2 *ap,
                           double2 *an, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_alpha, dim3((n + 63) / 64), dim3(64), 0, st, rr, pAp, active, n, ap, an);
    return hipGetLastError();
}

hipError_t launch_cg_beta(const double *rr_new, double *rr, int *active, const double *stop, int n,
                          double2 *beta, int *iters, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_beta, dim3((n + 63) / 64), dim3(64), 0, st, rr_new, rr, active, stop, n, beta, iters);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_norm_breach(const double2 *chi2, const double2 *w2, const int *oslots, int n, double bound2,
                              int *flag, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_breach, dim3((n + 63) / 64), dim3(64), 0, st, chi2, w2, oslots, n, bound2, flag);
    return hipGetLastError();
}

hipError_t launch_sum_rows(const double *part, int n, int Lt, double *G, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_rows, dim3((Lt + 255) / 256), dim3(256), 0, st, part, n, Lt, G);
    return hipGetLastError();
}

#define OV_INST_S(S)                                                                                   \
    template hipError_t launch_pack_spinor<S>(const double2 *, S *, long, const int *, int, int, int,  \
                                              hipStream_t);                                            \
    template hipError_t launch_unpack_spinor<S>(const S *, double2 *, long, const int *, int, int, int, \
                                                hipStream_t);                                          \
    template hipError_t launch_pack_links<S>(const double2 *, S *, int, int, hipStream_t);
OV_INST_S(double2)
OV_INST_S(float2)
OV_INST_S(uint32_t)

#define OV_INST_2(A, B)                                                                                   \
    template hipError_t launch_lincomb<A, B>(LcArgs<A, B>, hipStream_t, int *);                           \
    template hipError_t launch_dot<A, B>(const A *, long, const B *, long, const int *, int, int, int,   \
                                         double2 *, double2 *, const int *, hipStream_t);
OV_INST_2(double2, double2)
OV_INST_2(float2, float2)
OV_INST_2(uint32_t, uint32_t)
OV_INST_2(double2, float2)
OV_INST_2(float2, double2)
OV_INST_2(double2, uint32_t)
OV_INST_2(uint32_t, double2)

}  // namespace ov
