// Wilson force of the sign-function adjoint (background field, Sec. 4,
// eq. (3); the links U~ = exp(i q eta t) U are the differentiated variables).
//
// A term Re<u, dQ v> with dQ = gamma5 dD_w / norm contributes, per link,
//   G_mu(x) += -(w b / 2) [ sum_s ((1-gamma_mu) gamma5 u(x))_s v(x+mu)_s^dag
//                         + sum_s v(x)_s ((1+gamma_mu) gamma5 u(x+mu))_s^dag ]
// (w = coef, which carries 1/norm; b the boundary multiplier of the hop), so
// that dL = sum Re tr(G^dag dU~).  The accumulator G lives in FP64 planes
// [mu][3a+b][Vp]; one thread owns one site and its four forward links.
#include "ov_device.h"
#include "ov_internal.h"
#include "spin.h"

namespace ov {

template <int MU>
__device__ __forceinline__ void force_dir(const ForceArgs &a, int site, int cmu, int Lmu, int stride,
                                          const cx<double> (&ui)[4][3], const cx<double> (&vi)[4][3])
{
    const Geo &g = a.g;
    const bool wrap = (cmu == Lmu - 1);
    const int j = wrap ? site - (Lmu - 1) * stride : site + stride;
    const double b = wrap ? (double)g.bcf[MU] : 1.0;
    if (b == 0.0) return;
    cx<double> uj[4][3], vj[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uj[s][c] = ldc<double>(a.u, (long)(s * 3 + c) * g.Vp + j);
            vj[s][c] = ldc<double>(a.v, (long)(s * 3 + c) * g.Vp + j);
        }
    // gamma5 u: spins 2,3 negated
    cx<double> ai[4][3], aj[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ai[s][c] = s < 2 ? ui[s][c] : cmk(-ui[s][c].x, -ui[s][c].y);
            aj[s][c] = s < 2 ? uj[s][c] : cmk(-uj[s][c].x, -uj[s][c].y);
        }
    // pm = (1 - gamma_mu) ai ; pp = (1 + gamma_mu) aj  (full four-spinors)
    cx<double> h[2][3], pm[4][3], pp[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) pm[s][c] = pp[s][c] = cmk(0.0, 0.0);
    project<MU, -1>(ai, h);
    expand_add<MU, -1>(pm, h);
    project<MU, +1>(aj, h);
    expand_add<MU, +1>(pp, h);

    const double fac = -0.5 * a.coef * b;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<double> t = cmk(0.0, 0.0);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                // pm_s[r] conj(vj_s[c]) + vi_s[r] conj(pp_s[c])
                cfma(t, pm[s][r], cmk(vj[s][c].x, -vj[s][c].y));
                cfma(t, vi[s][r], cmk(pp[s][c].x, -pp[s][c].y));
            }
            const long k = (long)(MU * 9 + r * 3 + c) * g.Vp + site;
            double2 o = a.G[k];
            a.G[k] = make_double2(o.x + fac * t.x, o.y + fac * t.y);
        }
}

__global__ __launch_bounds__(256) void k_force(ForceArgs a)
{
    const Geo &g = a.g;
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    int rem = site;
    const int xc = rem % g.Lx; rem /= g.Lx;
    const int yc = rem % g.Ly; rem /= g.Ly;
    const int zc = rem % g.Lz;
    const int tc = rem / g.Lz;
    cx<double> ui[4][3], vi[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ui[s][c] = ldc<double>(a.u, (long)(s * 3 + c) * g.Vp + site);
            vi[s][c] = ldc<double>(a.v, (long)(s * 3 + c) * g.Vp + site);
        }
    force_dir<0>(a, site, xc, g.Lx, 1, ui, vi);
    force_dir<1>(a, site, yc, g.Ly, g.Lx, ui, vi);
    force_dir<2>(a, site, zc, g.Lz, g.Lxy, ui, vi);
    force_dir<3>(a, site, tc, g.Lt, g.Lxyz, ui, vi);
}

// Canonical gradient of the base links and per-block partial dL/deta:
//   gU_mu = G_mu, except gU_0 = exp(-i q eta t) G_0;
//   dL/deta = sum_x Re tr(G_0^dag i q t U~_0),  U~_0 = exp(i q eta t) U_0.
__global__ __launch_bounds__(256) void k_force_finish(const double2 *__restrict__ G, const double2 *__restrict__ U,
                                                      const cx<double> *phase_row, double q, Geo g,
                                                      double2 *gU, double *eta_part)
{
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    double et = 0.0;
    if (site < g.V) {
        const int tc = site / g.Lxyz;
        const cx<double> ph = phase_row[tc];
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < 9; ++k) {
                const double2 gk = G[(long)(mu * 9 + k) * g.Vp + site];
                cx<double> gv = {gk.x, gk.y};
                if (mu == 0) {
                    const double2 uk = U[(long)k * g.Vp + site];   // packed FP64 link planes, mu = 0
                    // Re(conj(G~) * i q t ph U)
                    cx<double> ut = cmul(ph, cmk(uk.x, uk.y));
                    cx<double> iu = cmk(-q * tc * ut.y, q * tc * ut.x);
                    et += gv.x * iu.x + gv.y * iu.y;
                    gv = cmulc(ph, gv);   // conj(ph) * G~
                }
                if (gU) gU[((long)mu * g.V + site) * 9 + k] = make_double2(gv.x, gv.y);
            }
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = et;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) eta_part[blockIdx.x] = sh[0];
}

hipError_t launch_force(const ForceArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_force, dim3((a.g.V + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_force_finish(const double2 *G, const double2 *U, const cx<double> *phase_row, double q, Geo g,
                               double2 *gU, double *eta_part, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_force_finish, dim3(nb), dim3(256), 0, st, G, U, phase_row, q, g, gU, eta_part);
    return hipGetLastError();
}

}  // namespace ov
