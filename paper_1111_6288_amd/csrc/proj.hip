// Small-space projection (Sec. 2, Fig. 1: the lowest eigenvectors of H_w
// are treated exactly).  Two complex FP64 contractions with a long inner
// dimension K = 12 Vp:
//
//   proj_dot     C[j][i] = sum_k conj(V_i[k]) (G X_j)[k]        (V^dag X)
//   proj_expand  Y_j[k]  = alpha X_j[k] + sum_i V_i[k] E[j][i]   (X + V E)
//
// V is FP64 (planes [l][12][Vp], the spinor layout); k runs over V's planes.
// X and Y may be stored in FP64, FP32 (paired layout: the position of k is
// mapped) or BF16; every product and sum is FP64.  The dot runs split-K:
// each workgroup reduces one K-chunk to a partial l x n block, then a fixed-
// order pass sums the partials (deterministic).  Both use the matrix cores
// (v_mfma_f64_4x4x4f64) on tiles of 16 vectors x 4 RHS.
#include <algorithm>

#include "ov_device.h"
#include "ov_internal.h"

namespace ov {

// --------------------------------------------------------------- V^dag X (MFMA)
// The matrix-core instruction is v_mfma_f64_4x4x4f64: four independent
// 4x4x4 products per wavefront.  Its lane layout, as measured on gfx950:
// block b = (lane >> 2) & 3; A_b[i][k] comes from lane i + 4b + 16k,
// B_b[k][j] from lane j + 4b + 16k, and D_b[i][j] lands in lane 16i + 4b + j.
// The four blocks are taken as the four row groups of one 16-row tile: lane
// q holds A = V[row q%16][k q/16], B = X[k q/16][column 4g + q%4] for RHS
// group g (the same value in all four blocks) and receives
// C[row 4((q>>2)&3) + q/16][column 4g + q%4].  Four such instructions do the work of one 16x16x4 step, but on
// gfx950 they sustain ~72 TFLOP/s of FP64 against ~47 for v_mfma_f64_16x16x4f64
// (register-only loops of independent instructions), and RHS columns come in
// groups of 4, so a batch of 36 RHS wastes nothing where 16-wide tiles pad it
// to 48.
//
// Workgroup (y, c) = W waves (W = blockDim / 64) owns K-chunk c and the
// vector tiles y W MT + w + W m (m < MT) of its waves w, with all RHS (up to
// 4 NJ).  The launcher takes W = 4 and MT = 2: three waves fit per SIMD, so
// three such workgroups share a CU, where one workgroup holding all 13 tiles
// of l = 200 (7 waves) would leave it at 7 waves.  X is staged through LDS
// 64 positions at a time (at most 53 KB, so three workgroups fit a CU), with the
// g5 sign applied there: all waves of the workgroup read the same X, so one
// coalesced load per workgroup replaces a 16-row gather per wave and step.
// chunk and Vp are multiples of 64, so a slice lies in one plane (one
// pair-plane for the paired layout) and on one side of the g5 sign change.
//
// NJ is the number of 4-column RHS groups (n <= 4 NJ), a template argument so
// that the matrix-core steps of a wave form one block without branches (a
// uniform branch per group split it into short dependent chains).  Tiles past
// l are computed on zeros rather than branched around: a copy of the K loop
// for one tile, taken by the waves whose second tile lies past l, measured no
// faster.
//
// Row padding of the staged X: rows of XP elements put the four k rows a lane
// group reads at different bank offsets (XP x 16 bytes = 64 x odd mod 256).
template <int NJ>
__host__ __device__ constexpr int xpad()
{
    return 4 * NJ + ((NJ % 2 == 0) ? 4 : 8);
}

template <class S, int MT, int NJ>
__global__ __launch_bounds__(256, 3) void k_proj_dot_mfma(const double2 *__restrict__ V, int l, long vstride,
                                                       const S *__restrict__ X, long xstride,
                                                       const int *slots, int n, int Vp, int g5x, long chunk,
                                                       double2 *__restrict__ part)
{
    constexpr int XS = 64, XJ = 4 * NJ, XP = xpad<NJ>();
    __shared__ double2 xs[XS * XP];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int W = blockDim.x >> 6;
    const int row = lane & 15, kq = lane >> 4, jq = lane & 3;
    const long K = 12L * Vp, half = 6L * Vp;
    const long k0 = (long)blockIdx.y * chunk;
    const long k1 = (k0 + chunk < K) ? k0 + chunk : K;

    double are[MT][NJ], aim[MT][NJ];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int g = 0; g < NJ; ++g) are[m][g] = aim[m][g] = 0.0;

    const double2 *vp[MT];
    bool vok[MT];
    const int tile0 = blockIdx.x * W * MT + wave;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int i = (tile0 + W * m) * 16 + row;
        vok[m] = i < l;
        vp[m] = V + (long)(vok[m] ? i : 0) * vstride;
    }
    // V of step kb + 4 is requested before the matrix-core work of step kb
    double2 vn[MT];
    auto load_v = [&](long kb) {
        const long k = kb + kq;
        const bool kin = k < k1;
#pragma unroll
        for (int m = 0; m < MT; ++m) vn[m] = (kin && vok[m]) ? vp[m][k] : make_double2(0.0, 0.0);
    };
    // conj(V) X: Re vr xr + vi xi, Im vr xi - vi xr
    auto step = [&](const double2 (&vc)[MT], const double2 *xrow) {
#pragma unroll
        for (int g = 0; g < NJ; ++g) {
            const double2 x = xrow[4 * g];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const double2 v = vc[m];
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(v.x, x.x, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(v.x, x.y, aim[m][g], 0, 0, 0);
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(v.y, x.y, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(-v.y, x.x, aim[m][g], 0, 0, 0);
            }
        }
    };
    if (k0 < k1) load_v(k0);
    for (long s0 = k0; s0 < k1; s0 += XS) {
        __syncthreads();   // the previous slice has been consumed
        {
            const long pl = s0 / Vp, sst = s0 - pl * Vp;
            const double sg = (g5x && s0 >= half) ? -1.0 : 1.0;
            for (int e = (int)threadIdx.x; e < XS * XJ; e += (int)blockDim.x) {
                const int j = e / XS, ii = e - j * XS;   // k fastest: contiguous reads of one RHS
                cx<double> x = {0.0, 0.0};
                if (j < n && s0 + ii < k1) {
                    const int sj = slots ? slots[j] : j;
                    x = ldc<double>(X + (long)sj * xstride, cpos<S>((int)pl, sst + ii, Vp));
                }
                xs[ii * XP + j] = make_double2(sg * x.x, sg * x.y);
            }
        }
        __syncthreads();
        const long send = (s0 + XS < k1) ? s0 + XS : k1;
        for (long kb = s0; kb < send; kb += 4) {
            double2 vc[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) vc[m] = vn[m];
            if (kb + 4 < k1) load_v(kb + 4);
            const double2 *xrow = xs + (int)(kb - s0 + kq) * XP + jq;
            step(vc, xrow);
        }
    }

    // partial[chunk][j][i]
    double2 *pc = part + (long)blockIdx.y * n * l;
    const int irow = 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int g = 0; g < NJ; ++g) {
            const int i = (tile0 + W * m) * 16 + irow;
            const int j = 4 * g + jq;
            if (i < l && j < n) pc[(long)j * l + i] = make_double2(are[m][g], aim[m][g]);
        }
}

// The same contraction for X in the paired FP32 layout, where one 16-byte
// element holds the site's components 2p and 2p+1.  Walking k plane by plane
// would use half of every X line (the partner plane is reached a plane
// later, long after the line left L1); here each step covers four sites of
// both planes of a pair: one 16-byte X element per lane feeds the steps of
// plane 2p and of plane 2p+1.  K-chunks count pairs of planes (chunk sites of
// the 6 Vp pair positions).
template <int MT, int NJ>
__global__ __launch_bounds__(256, 3) void k_proj_dot_mfma_pair(const double2 *__restrict__ V, int l, long vstride,
                                                            const float2 *__restrict__ X, long xstride,
                                                            const int *slots, int n, int Vp, int g5x, long chunk,
                                                            double2 *__restrict__ part)
{
    constexpr int XS = 64, XJ = 4 * NJ, XP = xpad<NJ>();
    __shared__ float4 xs[XS * XP];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int W = blockDim.x >> 6;
    const int row = lane & 15, kq = lane >> 4, jq = lane & 3;
    const long K2 = 6L * Vp;
    const long k0 = (long)blockIdx.y * chunk;
    const long k1 = (k0 + chunk < K2) ? k0 + chunk : K2;

    double are[MT][NJ], aim[MT][NJ];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int g = 0; g < NJ; ++g) are[m][g] = aim[m][g] = 0.0;
    const double2 *vp[MT];
    bool vok[MT];
    const int tile0 = blockIdx.x * W * MT + wave;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int i = (tile0 + W * m) * 16 + row;
        vok[m] = i < l;
        vp[m] = V + (long)(vok[m] ? i : 0) * vstride;
    }
    // (pair-plane, site) of kb; Vp and kb are multiples of 4
    long pp = k0 / Vp, st = k0 - pp * Vp;
    double2 vn0[MT], vn1[MT];
    auto load_v = [&](long kb) {
        const bool kin = kb + kq < k1;
        const long site = st + kq;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const bool ok = kin && vok[m];
            vn0[m] = ok ? vp[m][(2 * pp) * Vp + site] : make_double2(0.0, 0.0);
            vn1[m] = ok ? vp[m][(2 * pp + 1) * Vp + site] : make_double2(0.0, 0.0);
        }
        st += 4;
        if (st >= Vp) {
            st -= Vp;
            ++pp;
        }
    };
    // conj(V) X on both planes of the pair: Re vr xr + vi xi, Im vr xi - vi xr
    auto step = [&](const double2 (&v0)[MT], const double2 (&v1)[MT], const float4 *xrow) {
#pragma unroll
        for (int g = 0; g < NJ; ++g) {
            const float4 x = xrow[4 * g];
            const double x0r = x.x, x0i = x.y, x1r = x.z, x1i = x.w;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const double2 a = v0[m], b = v1[m];
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, x0r, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, x0i, aim[m][g], 0, 0, 0);
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, x0i, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(-a.y, x0r, aim[m][g], 0, 0, 0);
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(b.x, x1r, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(b.x, x1i, aim[m][g], 0, 0, 0);
                are[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(b.y, x1i, are[m][g], 0, 0, 0);
                aim[m][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(-b.y, x1r, aim[m][g], 0, 0, 0);
            }
        }
    };
    if (k0 < k1) load_v(k0);
    for (long s0 = k0; s0 < k1; s0 += XS) {
        __syncthreads();   // the previous slice has been consumed
        {
            const long spp = s0 / Vp, sst = s0 - spp * Vp;
            const float sg = (g5x && s0 >= 3L * Vp) ? -1.f : 1.f;
            for (int e = (int)threadIdx.x; e < XS * XJ; e += (int)blockDim.x) {
                const int j = e / XS, ii = e - j * XS;   // sites fastest: contiguous reads of one RHS
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (j < n && s0 + ii < k1) {
                    const int sj = slots ? slots[j] : j;
                    v = *(const float4 *)(X + (long)sj * xstride + 2 * (spp * (long)Vp + sst + ii));
                }
                xs[ii * XP + j] = make_float4(sg * v.x, sg * v.y, sg * v.z, sg * v.w);
            }
        }
        __syncthreads();
        const long send = (s0 + XS < k1) ? s0 + XS : k1;
        for (long kb = s0; kb < send; kb += 4) {
            double2 v0[MT], v1[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                v0[m] = vn0[m];
                v1[m] = vn1[m];
            }
            if (kb + 4 < k1) load_v(kb + 4);
            const float4 *xrow = xs + (int)(kb - s0 + kq) * XP + jq;
            step(v0, v1, xrow);
        }
    }
    double2 *pc = part + (long)blockIdx.y * n * l;
    const int irow = 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int g = 0; g < NJ; ++g) {
            const int i = (tile0 + W * m) * 16 + irow;
            const int j = 4 * g + jq;
            if (i < l && j < n) pc[(long)j * l + i] = make_double2(are[m][g], aim[m][g]);
        }
}

// C[j][i] = sum_c part[c][j][i]  (fixed order)
__global__ void k_proj_reduce(const double2 *__restrict__ part, int nchunk, int nl, double2 *__restrict__ C)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nl) return;
    double r = 0, im = 0;
    for (int c = 0; c < nchunk; ++c) {
        double2 v = part[(long)c * nl + e];
        r += v.x;
        im += v.y;
    }
    C[e] = make_double2(r, im);
}

// --------------------------------------------------------------- X + V E (MFMA)
// Y = alpha X + beta (V E).  Output D[j][k] (RHS j, position k) += A[j][i] B[i][k] with A = E
// (transposed coefficients) and B = V, on v_mfma_f64_4x4x4f64 with its four blocks taken as the
// four column groups of 16 consecutive k: lane q holds B = V[i = q/16][k = q%16], A = E[j = 4jb +
// q%4][i = q/16] (the same value in all four blocks) and receives D[j = 4jb + q/16][k = q%16], so a
// store instruction writes four runs of 16 consecutive k.  Each wave owns 16 consecutive k (one
// column block) and up to 4 NJ RHS in NJ groups of 4.  The coefficients E
// are the same for every position; they are staged through LDS 16 vector indices at a time and
// the eight waves of a workgroup (128 positions) share each slice.  Every workgroup re-reads all of
// E from L2, so wider workgroups cut that traffic; 16 waves lost more to the barriers.  At most 80
// VGPRs (six waves per SIMD) keep enough V loads in flight.
template <class SX, class SY, int NJ>
__global__ __launch_bounds__(512, 6) void k_proj_expand_mfma(const double2 *__restrict__ V, int l, long vstride,
                                                          const SX *X, long xstride, double alpha,
                                                          SY *Y, long ystride, const int *slots, int n,
                                                          int Vp, const double2 *__restrict__ E, double beta)
{
    // slice of E: EI vector indices x EJ RHS (rows padded so the four rows a lane group reads sit at
    // different bank offsets)
    constexpr int EI = 16, EJ = 4 * NJ, EP = xpad<NJ>();
    __shared__ double2 es[EI * EP];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, iq = lane >> 4, jq = lane & 3;
    const long K = 12L * Vp;
    const long kbase = ((long)blockIdx.x * (blockDim.x >> 6) + wave) * 16;
    const long kk = kbase + col;          // B column handled by this lane
    const bool kok = kk < K;              // waves past the end still take part in the barriers
    // the 16 columns of a wave lie in one plane (Vp is a multiple of 16)
    const long pl = kk / Vp, st = kk - pl * Vp;
    const long xk = cpos<SX>((int)pl, st, Vp), yk = cpos<SY>((int)pl, st, Vp);

    double dre[NJ], dim[NJ];
#pragma unroll
    for (int g = 0; g < NJ; ++g) dre[g] = dim[g] = 0.0;
    // V of step ib + 4 is requested before the matrix-core work of step ib
    double2 vn = (iq < l && kok) ? V[(long)iq * vstride + kk] : make_double2(0.0, 0.0);
    for (int i0 = 0; i0 < l; i0 += EI) {
        __syncthreads();   // the previous slice has been consumed
        for (int e = (int)threadIdx.x; e < EI * EJ; e += (int)blockDim.x) {
            const int j = e / EI, ii = e - j * EI;   // ii fastest: contiguous reads of a row of E
            es[ii * EP + j] = (i0 + ii < l && j < n) ? E[(long)j * l + i0 + ii] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const int iend = (i0 + EI < l) ? i0 + EI : l;
        for (int ib = i0; ib < iend; ib += 4) {
            const int i = ib + iq;
            const double2 v = vn;
            if (ib + 4 < l) {
                const int i2 = i + 4;
                vn = (i2 < l && kok) ? V[(long)i2 * vstride + kk] : make_double2(0.0, 0.0);
            }
            const double2 *erow = es + (ib - i0 + iq) * EP + jq;
#pragma unroll
            for (int g = 0; g < NJ; ++g) {
                // A element of this lane: j = 4g + q%4, i = q/16 (zero beyond l and n: the slice is padded)
                const double2 e = erow[4 * g];
                // (e * v): Re = er vr - ei vi ; Im = er vi + ei vr
                dre[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(e.x, v.x, dre[g], 0, 0, 0);
                dim[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(e.x, v.y, dim[g], 0, 0, 0);
                dre[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(-e.y, v.y, dre[g], 0, 0, 0);
                dim[g] = __builtin_amdgcn_mfma_f64_4x4x4f64(e.y, v.x, dim[g], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < NJ; ++g) {
        const int j = 4 * g + iq;
        if (j < n && kok) {
            const int s = slots ? slots[j] : j;
            cx<double> y = {beta * dre[g], beta * dim[g]};
            if (X) {
                cx<double> x = ldc<double>(X + (long)s * xstride, xk);
                y.x = fma(alpha, x.x, y.x);
                y.y = fma(alpha, x.y, y.y);
            }
            stc<double>(Y + (long)s * ystride, yk, y);
        }
    }
}

// E[j][i] = sgn(lambda_i) C[j][i] - D[j][i]
__global__ void k_small_combine(const double2 *C, const double2 *D, const double *sgn, int l, int n,
                                double2 *E)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= l * n) return;
    const int i = e % l;
    const double s = sgn[i];
    E[e] = make_double2(s * C[e].x - D[e].x, s * C[e].y - D[e].y);
}

// E[j][i] = C[j][i] * w[j][i]  (real weights, e.g. inverse Galerkin diagonal)
__global__ void k_mul_coef(const double2 *C, const double *w, int l, int n, double2 *E)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= l * n) return;
    E[e] = make_double2(C[e].x * w[e], C[e].y * w[e]);
}

// ------------------------------------------------------------------ launchers
// RHS column groups of 4 the kernels are built for (n <= 48); a batch takes the
// smallest that holds it.
#define OV_NJ_LIST(M) \
    OV_DOT_CASE(M, 1) OV_DOT_CASE(M, 2) OV_DOT_CASE(M, 3) OV_DOT_CASE(M, 4) OV_DOT_CASE(M, 6) OV_DOT_CASE(M, 8) \
    OV_DOT_CASE(M, 9) OV_DOT_CASE(M, 12)
static int proj_groups(int n)
{
    const int g = (n + 3) / 4;
    return g <= 4 ? g : g <= 6 ? 6 : g <= 8 ? 8 : g <= 9 ? 9 : 12;
}

long proj_dot_chunk(long K)
{
    // split K into about 1024 chunks (each a multiple of 128); with the tile split
    // along y that is 2048 workgroups for l = 200
    long c = (K + 1023) / 1024;
    c = (c + 127) & ~127L;   // a multiple of 128: the kernels stage X 64 positions at a time
    if (c < 64) c = 64;
    return c;
}

template <class S, int MT, int NJ>
static void launch_dot_mt(const double2 *V, int l, long vstride, const S *X, long xstride, const int *slots,
                          int n, int Vp, int g5x, long chunk, int nchunk, double2 *part, int waves, hipStream_t st)
{
    const int tiles = (l + 15) / 16;
    const int ny = (tiles + waves * MT - 1) / (waves * MT);
    // the ny workgroups of a K-chunk are consecutive in dispatch order, so they
    // run at the same time and the second one reads the chunk of X from L2
    hipLaunchKernelGGL((k_proj_dot_mfma<S, MT, NJ>), dim3(ny, nchunk), dim3(64 * waves), 0, st, V, l, vstride, X,
                       xstride, slots, n, Vp, g5x, chunk, part);
}

template <int MT, int NJ>
static void launch_dot_pair(const double2 *V, int l, long vstride, const float2 *X, long xstride, const int *slots,
                            int n, int Vp, int g5x, long chunk, int nchunk, double2 *part, int waves, hipStream_t st)
{
    const int tiles = (l + 15) / 16;
    const int ny = (tiles + waves * MT - 1) / (waves * MT);
    hipLaunchKernelGGL((k_proj_dot_mfma_pair<MT, NJ>), dim3(ny, nchunk), dim3(64 * waves), 0, st, V, l, vstride, X,
                       xstride, slots, n, Vp, g5x, chunk, part);
}

template <class S>
hipError_t launch_proj_dot(const double2 *V, int l, long vstride, const S *X, long xstride, const int *slots,
                           int n, int Vp, int g5x, double2 *part, double2 *C, hipStream_t st)
{
    if (l <= 0 || n <= 0) return hipSuccess;
    if (n > 48 || l > 256) return hipErrorInvalidValue;   // caller splits larger batches
    const long K = 12L * Vp;
    long chunk = proj_dot_chunk(K);
    int nchunk = (int)((K + chunk - 1) / chunk);
    if constexpr (Pair<S>::E == 2) {
        // chunks of pair positions: half as many positions per chunk (rounded up
        // to a multiple of 64), so at most as many chunks as the partial buffer holds
        chunk = ((chunk / 2) + 63) & ~63L;
        nchunk = (int)((6L * Vp + chunk - 1) / chunk);
    }
    // two vector tiles per wave, up to four waves per workgroup, the
    // remaining tiles in further workgroups along y
    const int tiles = (l + 15) / 16;
    const int mt = tiles >= 2 ? 2 : 1;
    const int waves = std::min(4, (tiles + mt - 1) / mt);
    const int nj = proj_groups(n);
    if constexpr (Pair<S>::E == 2) {
#define OV_DOT_CASE(M, N) \
    case N: launch_dot_pair<M, N>(V, l, vstride, X, xstride, slots, n, Vp, g5x, chunk, nchunk, part, waves, st); break;
        if (mt == 2) {
            switch (nj) { OV_NJ_LIST(2) default: return hipErrorInvalidValue; }
        } else {
            switch (nj) { OV_NJ_LIST(1) default: return hipErrorInvalidValue; }
        }
#undef OV_DOT_CASE
    } else {
#define OV_DOT_CASE(M, N) \
    case N: launch_dot_mt<S, M, N>(V, l, vstride, X, xstride, slots, n, Vp, g5x, chunk, nchunk, part, waves, st); break;
        if (mt == 2) {
            switch (nj) { OV_NJ_LIST(2) default: return hipErrorInvalidValue; }
        } else {
            switch (nj) { OV_NJ_LIST(1) default: return hipErrorInvalidValue; }
        }
#undef OV_DOT_CASE
    }
    const int nl = n * l;
    hipLaunchKernelGGL(k_proj_reduce, dim3((nl + 255) / 256), dim3(256), 0, st, part, nchunk, nl, C);
    return hipGetLastError();
}

template <class SX, class SY>
hipError_t launch_proj_expand(const double2 *V, int l, long vstride, const SX *X, long xstride, double alpha,
                              SY *Y, long ystride, const int *slots, int n, int Vp, const double2 *E, double beta,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (n > 48) return hipErrorInvalidValue;
    const long K = 12L * Vp;
    // 8 waves of 16 positions per workgroup: each staged slice of E serves 128 positions
    const int nblk = (int)((K + 127) / 128);
#define OV_DOT_CASE(M, N)                                                                                      \
    case N:                                                                                                    \
        hipLaunchKernelGGL((k_proj_expand_mfma<SX, SY, N>), dim3(nblk), dim3(512), 0, st, V, l, vstride, X,   \
                           xstride, alpha, Y, ystride, slots, n, Vp, E, beta);                                 \
        break;
    switch (proj_groups(n)) { OV_NJ_LIST(0) default: return hipErrorInvalidValue; }
#undef OV_DOT_CASE
    return hipGetLastError();
}

hipError_t launch_small_combine(const double2 *C, const double2 *D, const double *sgn, int l, int n, double2 *E,
                                hipStream_t st)
{
    if (l * n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_small_combine, dim3((l * n + 255) / 256), dim3(256), 0, st, C, D, sgn, l, n, E);
    return hipGetLastError();
}

hipError_t launch_mul_coef(const double2 *C, const double *w, int l, int n, double2 *E, hipStream_t st)
{
    if (l * n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul_coef, dim3((l * n + 255) / 256), dim3(256), 0, st, C, w, l, n, E);
    return hipGetLastError();
}

#define OV_INST_DOT(S)                                                                                       \
    template hipError_t launch_proj_dot<S>(const double2 *, int, long, const S *, long, const int *, int, int, \
                                           int, double2 *, double2 *, hipStream_t);
OV_INST_DOT(double2)
OV_INST_DOT(float2)
OV_INST_DOT(uint32_t)
#define OV_INST_EXP(A, B)                                                                                       \
    template hipError_t launch_proj_expand<A, B>(const double2 *, int, long, const A *, long, double, B *, long, \
                                                 const int *, int, int, const double2 *, double, hipStream_t);
OV_INST_EXP(double2, double2)
OV_INST_EXP(float2, float2)
OV_INST_EXP(uint32_t, uint32_t)
OV_INST_EXP(float2, double2)
OV_INST_EXP(double2, float2)
OV_INST_EXP(uint32_t, double2)
OV_INST_EXP(double2, uint32_t)

}  // namespace ov
