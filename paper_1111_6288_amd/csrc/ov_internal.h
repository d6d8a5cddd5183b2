// Internal declarations shared by the libov translation units: kernel
// argument blocks and launcher entry points.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ov_device.h"

namespace ov {

// ---------------------------------------------------------------- dslash
template <class S>
struct DsArgs {
    const S *x;              // input batch (planes), read at the 8 neighbours and the own site
    S *y;                    // output batch, must not alias x
    long fstride;            // storage elements between consecutive fields
    const S *U;              // links [4][9][Vp]
    const int *slots;        // storage index of batch entry j (NULL: j)
    int n;                   // batch size
    const int *fgroup;       // field group of a storage index (NULL: 0)
    const cx<double> *phase; // [nfield][Lt] background phase exp(i q eta t)
    Geo g;
    double diag;             // 4 + m_w
    double a;                // scale of G D_w x
    const S *e1, *e2, *e3;   // epilogue inputs at the own site (same fstride), NULL if unused
    double c1, c2, c3;
    int order;               // 0 canonical t-chunks per XCD, 1 z-slabs per XCD, 2 t-marching threads
    int tchunk;              // t-chunk length of order 2 (0: whole Lt)
    int blocks_per_cu;       // occupancy cap (0: none), enforced through reserved LDS
    int xcd_remap;           // set by the launcher
    int stream_hint;         // 1: epilogue inputs and the output bypass cache retention (non-temporal)
    int cols;                // order 1: the slab is walked as `cols` y-columns, one after the other
    int recon;               // 1: links are SU(3); read two rows and rebuild the third
    int wshare;              // 1, or W = 2, 4, 8 waves per workgroup sharing sites and LDS-staged links
};

template <class S>
hipError_t launch_dslash(const DsArgs<S> &a, bool hw, bool epi, int nr, int block, int split, hipStream_t st);

// ---------------------------------------------------------------- lincomb
template <class SI, class SO>
struct LcArgs {
    const SI *in[3];
    long istride[3];
    int nin;                 // 1..3 terms
    int g5mask;              // bit t: apply gamma5 to term t
    const double2 *coef[3];  // per-RHS complex coefficients (NULL: use cconst)
    int coef_by_slot;        // index coef by storage index instead of batch position
    double2 cconst[3];
    SO *out;
    long ostride;
    const int *slots;
    int n;
    int Vp;
    double *red;             // optional partial |out|^2 [n][nblk]
};

template <class SI, class SO>
hipError_t launch_lincomb(LcArgs<SI, SO> a, hipStream_t st, int *nblk_out);
int lincomb_blocks(int Vp, int n);

template <class SA, class SB>
hipError_t launch_dot(const SA *a, long astride, const SB *b, long bstride, const int *slots, int n, int Vp,
                      int g5a, double2 *part, double2 *out, const int *oslots, hipStream_t st);
hipError_t launch_reduce_r(const double *part, int nb, int n, double *out, const int *oslots, hipStream_t st);
hipError_t launch_cg_alpha(const double *rr, const double2 *pAp, const int *active, int n, double2 *ap,
                           double2 *an, hipStream_t st);
hipError_t launch_cg_beta(const double *rr_new, double *rr, int *active, const double *stop, int n,
                          double2 *beta, int *iters, hipStream_t st);
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st);
// *flag = 1 if some RHS j has w2[slot j] > bound2 * chi2[slot j] (or a non-finite norm)
hipError_t launch_norm_breach(const double2 *chi2, const double2 *w2, const int *oslots, int n, double bound2,
                              int *flag, hipStream_t st);
// G[t] = sum_{j < n} part[j Lt + t] in order of j
hipError_t launch_sum_rows(const double *part, int n, int Lt, double *G, hipStream_t st);

template <class S>
hipError_t launch_pack_spinor(const double2 *in, S *out, long fstride, const int *slots, int n, int V, int Vp,
                              hipStream_t st);
template <class S>
hipError_t launch_unpack_spinor(const S *in, double2 *out, long fstride, const int *slots, int n, int V, int Vp,
                                hipStream_t st);
template <class S>
hipError_t launch_pack_links(const double2 *in, S *out, int V, int Vp, hipStream_t st);
hipError_t launch_count_nonfinite(const double *p, long n, int *count, hipStream_t st);
// max over the nl links of canonical complex128 [nl][3][3] of
// max_a |u_2a - conj(u_0b u_1c - u_0c u_1b)|, as the bits of a non-negative
// double atomically maxed into *out (which the caller clears).
hipError_t launch_link_row3_dev(const double2 *U, long nl, unsigned long long *out, hipStream_t st);
// out[2 p + r]: max Frobenius distance between the stored links and the links
// the kernels apply for p = 0 FP32 / 1 BF16 storage, r = 0 nine entries /
// 1 two rows and the rebuilt third; maxed atomically (caller clears).
hipError_t launch_link_round_dev(const double2 *U, long nl, unsigned long long *out, hipStream_t st);

// ---------------------------------------------------------------- projection
long proj_dot_chunk(long K);
template <class S>
hipError_t launch_proj_dot(const double2 *V, int l, long vstride, const S *X, long xstride, const int *slots,
                           int n, int Vp, int g5x, double2 *part, double2 *C, hipStream_t st);
template <class SX, class SY>
hipError_t launch_proj_expand(const double2 *V, int l, long vstride, const SX *X, long xstride, double alpha,
                              SY *Y, long ystride, const int *slots, int n, int Vp, const double2 *E, double beta,
                              hipStream_t st);
hipError_t launch_small_combine(const double2 *C, const double2 *D, const double *sgn, int l, int n, double2 *E,
                                hipStream_t st);
hipError_t launch_mul_coef(const double2 *C, const double *w, int l, int n, double2 *E, hipStream_t st);

// ---------------------------------------------------------------- backward
struct ForceArgs {
    const double2 *u;        // planes [12][Vp]
    const double2 *v;        // planes [12][Vp]
    double2 *G;              // force accumulator [4][9][Vp] (phased links)
    double coef;             // weight of Re<u, dQ v>, includes 1/norm
    Geo g;
};
hipError_t launch_force(const ForceArgs &a, hipStream_t st);
int slice_norm2_blocks(int Lxyz);
hipError_t launch_weight_g5(const double2 *in, const double *w, long V, int Lxyz, int n, double2 *out,
                            hipStream_t st);
hipError_t launch_slice_norm2(const double2 *x, int n, long V, int Lxyz, int Lt, double *part, double *out,
                              hipStream_t st);
hipError_t launch_force_finish(const double2 *G, const double2 *U, const cx<double> *phase_row, double q,
                               Geo g, double2 *gU_canon, double *eta_part, int nb, hipStream_t st);

}  // namespace ov
