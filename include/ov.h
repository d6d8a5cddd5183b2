/*
 * libov -- overlap fermion operator D_ov = 1 + gamma5 sign(H_w) on one AMD
 * MI355X (gfx950).  Plain C ABI: opaque context, plain pointers and sizes.
 *
 * Paper: "Electric polarizability of hadrons with overlap fermions on
 * multi-GPUs" (Lattice 2011).  Every entry point names the passage that
 * defines the operation it performs.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Lattice L = (Lx, Ly, Lz, Lt), V = Lx*Ly*Lz*Lt sites, canonical site index
 * i = x + Lx*(y + Ly*(z + Lz*t)).  Directions mu = 0,1,2,3 are x,y,z,t.
 *
 * Canonical device layouts (complex128 = interleaved re,im doubles):
 *   spinor batch  [nrhs][V][4 spin][3 colour]
 *   gauge field   [4 mu][V][3][3]     (row a, column b; U_mu(i) links i -> i+mu)
 *   small space   [l][V][4][3]        (orthonormal columns)
 * Every pointer argument named *_dev is a device pointer that the caller owns
 * and keeps alive for the duration of the call (stream-ordered on the stream
 * set with ov_set_stream).  Host arrays are read before the call returns.
 * The context owns every internal buffer (packed links, small spaces,
 * deflation basis, workspaces); its memory is released by ov_destroy.
 *
 * Gamma matrices (chiral basis): gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 * gamma_4 = [[0,1],[1,0]], gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1,1,-1,-1).
 * Wilson operator:
 *   D_w psi(x) = (4 + m_w) psi(x)
 *     - 1/2 sum_mu [ (1 - gamma_mu) U~_mu(x) psi(x+mu) + (1 + gamma_mu) U~_mu(x-mu)^dag psi(x-mu) ]
 * with U~_0(x) = exp(i q eta t) U_0(x) (background field, Sec. 4 eq. (3)) and
 * the boundary multiplier b_mu (+1 periodic, -1 antiperiodic, 0 Dirichlet)
 * on hops that wrap around the lattice (Sec. 4: Dirichlet in the field
 * direction and in time).  H_w = gamma5 D_w (Sec. 2).
 *
 * Precision codes select the INTERNAL arithmetic and storage; I/O is always
 * complex128.  OV_FP64: double.  OV_FP32: float links and spinors, float
 * Clenshaw recursion, FP64 small-space projection.  OV_BF16: bfloat16 storage
 * of links and spinors, float arithmetic, FP64 projection.
 *
 * Errors: every entry point returns OV_OK (0) or a negative status; no
 * exception or abort crosses the ABI.  After an error the context stays
 * usable, outputs are unspecified, and ov_last_error() describes the cause.
 * One context per host thread.
 */
#ifndef OV_H
#define OV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ov_ctx ov_ctx;

enum {
    OV_OK = 0,
    OV_EINVAL = -1,   /* bad argument (shape, range, null pointer)           */
    OV_ENOMEM = -2,   /* device allocation failed or over the memory budget   */
    OV_EHIP = -3,     /* HIP runtime error                                    */
    OV_ENOCONV = -4,  /* CG reached maxiter; best iterate and report written  */
    OV_ENAN = -5,     /* NaN/Inf detected in an input or a residual           */
    OV_ESTATE = -6,   /* call out of order (e.g. no gauge field uploaded)     */
    OV_ENORM = -7,    /* norm bound below ||H_w|| detected (Clenshaw growth)  */
    OV_EBREAKDOWN = -8 /* numerical breakdown (e.g. a Gram matrix not positive) */
};

enum { OV_FP64 = 0, OV_FP32 = 1, OV_BF16 = 2 };
enum { OV_PERIODIC = 0, OV_ANTIPERIODIC = 1, OV_DIRICHLET = 2 };
enum { OV_OP_DW = 0, OV_OP_HW = 1 };

/*
 * Create a context for lattice L with boundary codes bc (per direction) and
 * Wilson mass m_w on HIP device `device`.  Sizes must be >= 2 (Lt >= 2) and
 * V < 2^31.  On success *out owns the context.
 */
int ov_create(const int32_t L[4], const int32_t bc[4], double m_w, int device, ov_ctx **out);

/* Free every device buffer and the context.  Accepts NULL. */
int ov_destroy(ov_ctx *ctx);

/* Run all further work on this hipStream_t (NULL = the null stream, the default). */
int ov_set_stream(ov_ctx *ctx, void *hip_stream);

/* Human-readable description of the last error on this context. */
const char *ov_last_error(const ov_ctx *ctx);

/*
 * Upload the base SU(3)-valued links (canonical [4][V][3][3] complex128 on
 * the device).  Packed into the context's internal layouts for every
 * precision.  Sec. 2 (D_w) and Sec. 4 (links that the background field
 * multiplies).  Returns OV_ENAN if the field holds NaN/Inf.
 */
int ov_upload_gauge(ov_ctx *ctx, const void *U_dev);

/*
 * Link storage read by the dslash kernels.  Every SU(3) matrix satisfies
 * u_2a = conj(u_0b u_1c - u_0c u_1b) for (a, b, c) cyclic (its third row is
 * the conjugated cross product of the first two), so the kernels can read
 * two rows and rebuild the third, two thirds of the link bytes.  The upload
 * measures, in FP64, the largest deviation of the uploaded links from this
 * identity; the two-row kernels are used while reconstruction is enabled
 * (the default) and that deviation is at most 1e-14; otherwise all nine
 * entries are read.  The result of either path is the operator of the
 * uploaded links to within that bound.
 *
 * ov_set_link_reconstruct: enable (1, default) or disable (0) the two-row
 * path for this context; OV_EINVAL for other values.
 * ov_get_link_format: *reconstruct = 1 if the two-row kernels are in use;
 * *row3_dev = the measured deviation (-1 before the first upload).  Either
 * pointer may be NULL.
 */
int ov_set_link_reconstruct(ov_ctx *ctx, int enable);
int ov_get_link_format(ov_ctx *ctx, int *reconstruct, double *row3_dev);

/*
 * Define nfield background-field groups: group f multiplies the mu = 0 links
 * by exp(i q[f] eta[f] t) (Sec. 4, eq. (3); the operator depends on q*eta
 * only).  Host arrays of length nfield (1 <= nfield <= 64).  Resets any small
 * space and deflation basis uploaded before.
 */
int ov_set_fields(ov_ctx *ctx, int nfield, const double *q, const double *eta);

/*
 * Change the charge and field strength of one existing group (Sec. 4,
 * eq. (3)) without touching its small space or deflation basis; used when
 * those are held fixed while eta varies (adjoint, finite differences).
 */
int ov_set_field_eta(ov_ctx *ctx, int field, double q, double eta);

/*
 * Polynomial parameters of sign(H_w) ~ Q P(Q^2), Q = H_w / norm (Sec. 2):
 * degree n >= 1 in Q^2, interval [eps, 1] for Q^2 (0 < eps < 1), and
 * norm >= ||H_w|| (the default bound |4+m_w| + 4 is valid for any links;
 * pass norm <= 0 to use it).  coeffs: host array of n+1 Chebyshev
 * coefficients c_k of P(y) = sum c_k T_k((2y-1-eps)/(1-eps)), or NULL to use
 * the Chebyshev interpolant of y^{-1/2} at the n+1 Chebyshev-Gauss nodes.
 */
int ov_set_sign_params(ov_ctx *ctx, int n, double eps, double norm, const double *coeffs);

/*
 * Small space of group `field` (Sec. 2, Fig. 1: lowest |lambda| eigenvectors
 * of H_w, treated exactly): l orthonormal vectors V_dev [l][V][4][3]
 * complex128 and their H_w eigenvalues lambda (host, length l; only the sign
 * is used, sgn(0) := +1).  l = 0 clears it.  Orthonormality is checked in
 * FP64: returns OV_EINVAL if max |V^dag V - 1| > 1e-8.
 */
int ov_upload_eigvecs(ov_ctx *ctx, int field, int l, const void *V_dev, const double *lambda);

/*
 * Deflation basis of group `field` for the CG (Sec. 2 end, Sec. 3.1: low
 * modes of the overlap operator speed up CG): k orthonormal vectors W_dev
 * [k][V][4][3].  The library computes a_i = ||D_ov w_i||^2 and
 * b_i = Re<w_i, D_ov w_i> in FP64 so that the Galerkin diagonal for mass m
 * is (1-m/2)^2 a_i + 2 m (1-m/2) b_i + m^2.  Needs the gauge field, the sign
 * parameters and the small space first (OV_ESTATE otherwise).
 */
int ov_upload_deflation(ov_ctx *ctx, int field, int k, const void *W_dev);

/*
 * y = D_w x (op = OV_OP_DW) or y = H_w x = gamma5 D_w x (op = OV_OP_HW) for
 * nrhs fields, RHS j using background group field_of_rhs[j] (host array).
 * x_dev, y_dev: [nrhs][V][4][3] complex128, must not overlap.  Sec. 2 (H_w).
 */
int ov_dslash(ov_ctx *ctx, int prec, int op, int nrhs, const int *field_of_rhs,
              const void *x_dev, void *y_dev);

/*
 * ov_dslash for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same operation, arguments and kernels as ov_dslash, with the packed
 * input, the packed output and the field-group list held in one fixed
 * device array of 64 MiB per GPU (file-scope in the library, resident until
 * the process ends) instead of the context's workspace.  It calls no
 * hipMalloc / hipFree and records no profiling events; it copies
 * field_of_rhs to the device and synchronises the stream once before the
 * launch.  Size limit: 256 + 2 * nrhs * 12 * Vp * S bytes <= 64 MiB, with
 * Vp = V rounded up to a multiple of 64 and S = 16 (FP64), 8 (FP32),
 * 4 (BF16); larger requests return OV_EINVAL and touch nothing.  Every call
 * on a GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other threads, other streams) race; calls ordered on one stream do not.
 */
int ov_dslash_noalloc(ov_ctx *ctx, int prec, int op, int nrhs, const int *field_of_rhs, const void *x_dev,
                      void *y_dev);

/*
 * y = s(x) = V sgn(lambda) V^dag x + Pi Q P(Q^2) Pi x with Pi = 1 - V V^dag
 * (Sec. 2: small space exact, polynomial on the rest), per RHS with the small
 * space of its group.  Cost: 2n+1 H_w applications.  x_dev, y_dev as in
 * ov_dslash; may alias.
 */
int ov_sign_apply(ov_ctx *ctx, int prec, int nrhs, const int *field_of_rhs,
                  const void *x_dev, void *y_dev);

/*
 * Norm safety of the polynomial sign (Sec. 2: Q = H_w / ||H_w|| must have
 * its spectrum in [-1, 1], where the Chebyshev recursion is bounded).
 *
 * Every sign application compares, per RHS, w = Q P(Q^2) chi with the bound
 * ||w|| <= 1.02 M ||chi||, M = max_{|q| <= 1} |q P(q^2)| of the current
 * coefficients (M is within 1e-5 of 1 for the built-in interpolant).  The
 * bound holds whenever the norm passed to ov_set_sign_params is at least
 * ||H_w|| of the applied links; when it is too small the recursion grows
 * like T_n outside [-1, 1] (at degree 300 a spectrum 1 % beyond the bound
 * amplifies components by ~1e25) and the comparison fails.  A failure sets
 * a sticky flag on the device; the result of that application is then not
 * the polynomial sign.
 *   mode 0: no check;
 *   mode 1: the flag is reported as OV_ENORM by the synchronising entry
 *           points that apply the sign (deflated CG, multi-mass CG, D_ov
 *           eigensolver, sign adjoint, correlator derivative), which clear it
 *           on entry, and by ov_norm_status;
 *   mode 2 (default): as 1, and ov_sign_apply / ov_dov_apply synchronise
 *           and return OV_ENORM themselves.
 * After OV_ENORM the context stays usable: set a larger norm and repeat.
 * ov_norm_status synchronises, returns OV_ENORM if the flag is set (and
 * clears it), OV_OK otherwise.
 *
 * The FP32 and BF16 kernels apply links rounded to their storage (two-row
 * links: with the rebuilt third row), whose H_w norm may exceed that of the
 * uploaded links by 4 max_x ||U_eff(x) - U(x)||_2 (four directions, one
 * link norm each).  ov_upload_gauge measures that distance (Frobenius norm,
 * an upper bound of the spectral one) and the sign pipeline of those
 * precisions divides by norm + 4 (distance + 1e-6) (the 1e-6 covers the
 * FP32 evaluation of the rebuilt row).  ov_get_sign_norm returns the norm
 * used for precision prec.
 */
int ov_set_norm_check(ov_ctx *ctx, int mode);
int ov_norm_status(ov_ctx *ctx);
int ov_get_sign_norm(ov_ctx *ctx, int prec, double *norm);

/*
 * y = D(m) x with D(m) = (1 - m/2) D_ov + m, D_ov = 1 + gamma5 s (Sec. 2,
 * eq. (1); m = 0 is eq. (1) itself), or y = D(m)^dag x = gamma5 D(m) gamma5 x
 * when dagger != 0.  mass: host array of nrhs quark masses.
 */
int ov_dov_apply(ov_ctx *ctx, int prec, int nrhs, const int *field_of_rhs, const double *mass,
                 int dagger, const void *x_dev, void *y_dev);

typedef struct {
    double tol;        /* stop when ||D^dag b - A x|| / ||D^dag b|| <= tol (FP64 true residual) */
    int maxiter;       /* cap on inner iterations summed over restarts                         */
    int inner_prec;    /* OV_FP64, OV_FP32 or OV_BF16 arithmetic of the inner CG               */
    double inner_tol;  /* relative residual reduction per inner solve (e.g. 1e-5 for FP32); an  */
                       /* inner solve also stops once its residual is below 0.1 tol ||D^dag b|| */
    int max_restarts;  /* cap on FP64 defect-correction restarts                               */
    int use_deflation; /* apply the uploaded deflation basis at each restart                   */
} ov_cg_opts;

typedef struct {
    int iters;         /* inner CG iterations (each = 2 D_ov applies per active RHS)           */
    int restarts;      /* FP64 residual evaluations                                            */
    double relres;     /* final FP64 true relative residual                                    */
    int status;        /* OV_OK or OV_ENOCONV                                                  */
} ov_cg_rhs_report;

/*
 * Solve D(m)^dag D(m) x = D(m)^dag b, i.e. x = D(m)^{-1} b, for nrhs right-hand
 * sides (Sec. 3.2: CG for overlap propagators; single precision late in the
 * solve; deflation by overlap low modes).  Outer loop in FP64 (true residual,
 * deflation step x += W Lambda^{-1} W^dag r), inner CG in opts->inner_prec,
 * x += e in FP64.  x_dev holds the initial guess on entry (zero is fine) and
 * the solution on return.  report: host array of nrhs entries (may be NULL).
 * Returns OV_ENOCONV if any RHS did not converge (its best iterate is kept).
 * Synchronises the stream.
 */
int ov_deflated_cg(ov_ctx *ctx, int nrhs, const int *field_of_rhs, const double *mass,
                   const void *b_dev, void *x_dev, const ov_cg_opts *opts,
                   ov_cg_rhs_report *report);

/*
 * Quark propagators for several masses at once (Sec. 3.2: adaptive
 * multi-mass CG, with the polynomial order following the CG residual).  For
 * a source of definite chirality (gamma5 b = chi b; point sources are), and
 * with s^2 = 1, D(m)^dag D(m) restricted to that chirality is
 *   (1 - m^2/4) (A + sigma),  A = 2 + 2 P s P,  sigma = m^2 / (1 - m^2/4),
 * P = (1 + chi gamma5)/2, so one sign application per iteration serves every
 * mass: shifted CG on A (base system = smallest shift), y_i = (A +
 * sigma_i)^{-1} b / (1 - m_i^2/4), x_i = D(m_i)^dag y_i, which solves
 * D(m_i) x_i = b because D is normal.  With opts->adaptive the degree of the
 * polynomial for an iteration is the smallest whose error bound (twice the
 * law of eq. (2)) stays below 0.01 tol ||b|| / ||r|| (a less accurate operator
 * is enough while the residual is large), at least min_order; the context's
 * polynomial is restored afterwards.  The shifted solve runs in
 * opts->inner_prec (FP64, or FP32 down to max(tol, 1e-5)) and stops early if
 * its residual fails to halve within 200 iterations; then every x_i
 * gets its FP64 true residual ||b - D(m_i) x_i|| / ||b|| with the full
 * polynomial, and with opts->refine pairs above tol are finished by the
 * FP64-outer deflated CG of ov_deflated_cg, starting from x_i.
 *   b_dev  [nrhs][V][4][3] complex128 chiral sources;
 *   x_dev  [nmass][nrhs][V][4][3] complex128 solutions (written);
 *   relres host [nmass][nrhs] final relative residuals (may be NULL).
 * OV_EINVAL for a source with both chiralities.  Synchronises.
 */
typedef struct {
    double tol;        /* FP64 true relative residual per (mass, RHS)                           */
    int maxiter;       /* shifted CG iterations (one sign application per RHS each)             */
    int adaptive;      /* polynomial order follows the residual                                 */
    int min_order;     /* lower bound of the adaptive order                                      */
    int refine;        /* finish pairs above tol with the deflated CG                            */
    int inner_prec;    /* precision of the shifted solve: OV_FP64 or OV_FP32                     */
} ov_mscg_opts;

typedef struct {
    int iters;          /* shifted CG iterations                                                 */
    long sign_applies;  /* single-vector sign applications in the shifted solve                  */
    long dslash_applies;/* single-vector H_w applications in the shifted solve                    */
    int refine_iters;   /* inner CG iterations spent in refinement (summed over RHS)              */
} ov_mscg_report;

int ov_multishift_cg(ov_ctx *ctx, int nrhs, const int *field_of_rhs, int nmass, const double *mass,
                     const void *b_dev, void *x_dev, const ov_mscg_opts *opts, ov_mscg_report *report,
                     double *relres);

/*
 * Lowest-|lambda| eigenpairs of H_w for field group `field`: the low modes
 * that the sign function treats exactly (Sec. 2, Fig. 1), which the paper
 * computes by Arnoldi with Chebyshev acceleration (Sec. 3.1).  Here:
 * Chebyshev-filtered subspace iteration on a block of k >= l vectors.  Each
 * pass
 *   1. filters the block with the degree-m Chebyshev polynomial in H_w^2
 *      that damps [a, norm^2] (scaled recurrence, normalised at the lowest
 *      Ritz value of H_w^2; 2m H_w applications per vector).  opts->prec
 *      OV_FP64: FP64 filter; OV_FP32: FP32 filter until the wanted residuals
 *      are below 1e-6 * norm or fall less than 3x in a pass, FP64 after that;
 *   2. orthonormalises it in FP64 (shifted Cholesky QR, then two plain
 *      Cholesky QR passes; Gram matrices on the matrix cores);
 *   3. Rayleigh-Ritz on its span (FP64) with H_w^2, whose wanted values are
 *      the smallest (with H_w they would be interior ones), then with H_w
 *      inside the l lowest to separate +lambda from -lambda; pairs sorted by
 *      |theta|; residuals r_j = ||H_w x_j - theta_j x_j|| (unit x_j).
 * It stops when the l lowest satisfy r_j <= tol * norm, or after max_iter
 * passes.  The first pass uses a = opts->cutoff (in units of H_w^2; <= 0:
 * norm^2 / 100), later passes the largest Ritz value of H_w^2 in the block.
 * norm is the bound of ov_set_sign_params (required).
 *   X0_dev  [k][V][4][3] complex128 start block (read only; e.g. Gaussian).
 *   V_dev   [l][V][4][3] complex128 eigenvectors out, or NULL.
 *   lambda  host [l] eigenvalues (ascending |lambda|); resid host [l] or NULL.
 *   install != 0: the pairs become the group's small space, as by
 *           ov_upload_eigvecs.
 * Workspace: 4 FP64 blocks of k fields (+ 4 FP32 blocks for an FP32 filter).
 * Synchronises.  OV_ENOCONV: not converged (outputs hold the last pass);
 * OV_EBREAKDOWN: the start block is numerically rank deficient.
 */
typedef struct {
    int l;             /* wanted eigenpairs, 1 <= l <= k                                      */
    int k;             /* block size, k <= 256 (a few more than l speeds convergence)         */
    int cheb_order;    /* m, degree of the filter in H_w^2                                     */
    double cutoff;     /* first-pass lower end a of the damped interval, in units of H_w^2     */
    int max_iter;      /* passes                                                               */
    double tol;        /* residual bound relative to the norm bound                            */
    int prec;          /* OV_FP64, or OV_FP32: FP32 filter down to 1e-6 * norm, then FP64       */
} ov_eig_opts;

typedef struct {
    int iters;         /* passes run                                                           */
    long hw_applies;   /* H_w applications on single vectors                                   */
    double max_resid;  /* max_j r_j over the l wanted pairs                                    */
} ov_eig_report;

int ov_hw_eigensolve(ov_ctx *ctx, int field, const ov_eig_opts *opts, const void *X0_dev, void *V_dev,
                     double *lambda, double *resid, int install, ov_eig_report *report);

/*
 * Low modes of D_ov for deflation (Sec. 3.1: eigensystem of D_ov with
 * Chebyshev acceleration of order 12; Sec. 2 end: deflation).  D_ov^dag D_ov
 * commutes with gamma5 and equals A = 2 + 2 P s P on the sector
 * P = (1 + chi gamma5)/2 (s^2 = 1), a Hermitian operator with spectrum in
 * [0, 4] whose wanted eigenvalues are the smallest.  The same filtered
 * subspace iteration as ov_hw_eigensolve runs on A in the sector chirality
 * = +1 or -1 (one sign application per filter degree and vector; the filter
 * damps [a, 4], first a = opts->cutoff, default 0.1), with Rayleigh-Ritz on
 * A; residuals ||A w - lambda w|| <= tol * 4.  lambda[l] are eigenvalues of
 * D_ov^dag D_ov (= |eigenvalue of D_ov|^2), ascending.  W_dev [l][V][4][3]
 * complex128 (needed when install != 0, which makes the basis the field
 * group's deflation basis as by ov_upload_deflation).  report->hw_applies
 * counts sign applications here.  Synchronises.
 */
int ov_dov_eigensolve(ov_ctx *ctx, int field, int chirality, const ov_eig_opts *opts, const void *X0_dev,
                      void *W_dev, double *lambda, double *resid, int install, ov_eig_report *report);

/*
 * Time-slice norms for the pion correlator (Sec. 4: G_E(t), G_0(t) and
 * R(t) = G_E(t) / G_0(t)): out[j][t] = sum over the sites of time slice t
 * and the 12 spin-colour components of |x_j|^2, for nrhs canonical
 * complex128 fields x_dev [nrhs][V][4][3].  With gamma5-hermiticity the
 * connected pseudoscalar correlator of one flavour from the 12 point-source
 * propagators S_j is G(t) = sum_j out[j][t].  Fixed-order (deterministic)
 * reduction.  out: host [nrhs][Lt].  Synchronises.
 */
int ov_timeslice_norm2(ov_ctx *ctx, int nrhs, const void *x_dev, double *out);

/*
 * Connected pseudoscalar (pion) correlator of one flavour (Sec. 4, eq. (4):
 * two-point functions from which R(t) is formed): with gamma5-hermiticity,
 *   G[t] = sum_j sum over the sites of time slice t and the 12 spin-colour
 *          components of |S_j|^2,
 * for the nsrc point-source propagators S_dev [nsrc][V][4][3] complex128
 * (normally the 12 spin-colour sources of one operator).  The per-slice sums
 * and the sum over j run on the device in a fixed order (deterministic).
 * G: host [Lt].  Synchronises.
 */
int ov_pion_correlator(ov_ctx *ctx, int nsrc, const void *S_dev, double *G);

/*
 * R(t) = G_E(t) / G_0(t) (Sec. 4): G_E is the mean of the nE field
 * correlators G_E_all [nE][Lt] (u and d quarks at +E and -E: nE = 4) and G_0
 * the correlator without field [Lt].  Host utility, no context, no GPU.
 * R: host [Lt].  OV_EINVAL for Lt < 1, nE < 1, a null pointer or a G_0[t]
 * that is not a positive finite number; OV_ENAN for a non-finite G_E sum.
 */
int ov_ratio_R(int Lt, int nE, const double *G_E_all, const double *G_0, double *R);

/*
 * Derivative of a correlator with respect to the background field (Sec. 4:
 * the pion's energy shift comes from G_E(t) / G_0(t); the polarizability is a
 * derivative in the field strength).  For field group `field` and mass m:
 *   S_j = D(m)^{-1} b_j (deflated CG with *opts),
 *   C[t] = sum_j sum over time slice t of |S_j|^2   (host [Lt], may be NULL),
 *   F = sum_t w[t] C[t],  *dF = dF/deta with the charge q held fixed,
 * through the solve: mu_j = D(m)^{-1} (gamma5 W S_j) (W = w by time slice),
 * dF/deta = -2 (1 - m/2) sum_j d/deta Re<mu_j, s(eta) S_j>, the last factor
 * from the sign adjoint (as ov_sign_backward: small space and polynomial held
 * fixed).  2 nsrc solves and nsrc sign adjoints.  b_dev [nsrc][V][4][3]
 * complex128.  Allocates its temporaries.  Synchronises.
 */
int ov_correlator_deta(ov_ctx *ctx, int field, double mass, int nsrc, const void *b_dev, const double *w,
                       double *C, double *dF, const ov_cg_opts *opts);

/*
 * Host utility (no context, no GPU): eigen-decomposition of a Hermitian
 * n x n matrix by cyclic Jacobi rotations, as the eigensolver's
 * Rayleigh-Ritz step uses it.  A: column-major complex (interleaved re, im),
 * only its Hermitian part is used; w: n ascending eigenvalues; Z:
 * column-major complex eigenvectors.  Returns 0, or -1 on a bad argument.
 */
int ov_dense_heev(int n, const double *A, double *w, double *Z);

/*
 * Adjoint of the sign function for L = Re<g, s(U, eta) x> with the small
 * space, the polynomial and the norm held fixed (background field, Sec. 4,
 * eq. (3)).  One RHS of group `field`.  Outputs (any may be NULL):
 *   gU_dev   [4][V][3][3] complex128, dL/dRe U + i dL/dIm U of the BASE links;
 *   geta     host double, dL/d eta of this group (charge q held fixed);
 *   gx_dev   [V][4][3] complex128, dL/dRe x + i dL/dIm x = s g.
 * The forward Clenshaw vectors are checkpointed every ckpt_every terms
 * (>= 1) and replayed segment by segment.  FP64 throughout.  Synchronises.
 */
int ov_sign_backward(ov_ctx *ctx, int field, const void *x_dev, const void *g_dev,
                     void *gU_dev, double *geta, void *gx_dev, int ckpt_every);

/*
 * Per-kernel timing with HIP events recorded on the context's stream around
 * every launch of the named kernel class ("dslash", "clenshaw", "proj_dot",
 * "proj_expand", "blas", "force").  ov_prof_enable(ctx, 1) starts a fresh
 * window; ov_prof_query synchronises and returns the launch count, the summed
 * duration in ms and the summed algorithmic HBM bytes of those launches.
 */
int ov_prof_enable(ov_ctx *ctx, int on);
int ov_prof_query(ov_ctx *ctx, const char *kernel_class, long *launches, double *total_ms,
                  double *bytes);

/*
 * Kernel launch tuning of the dslash family: RHS per thread (1, 2, 4, 8) and
 * threads per workgroup (64, 128, 192, 256 or 512) for precision prec.  The
 * t-marching site order (ov_set_site_order 2) ignores rhs_per_thread and
 * reads block as 64 threads per right-hand side of a workgroup: 512 puts 8
 * RHS in a workgroup, any other value 4.  The other orders use at most 256.
 * ov_autotune times the candidates on the current context for nrhs RHS,
 * separately for plain launches and for launches with the fused Clenshaw
 * epilogue, keeps the fastest of each and, with a non-NULL cache_path,
 * appends one JSON line per kind there.  ov_get_tuning reports the plain
 * kind.
 */
int ov_set_tuning(ov_ctx *ctx, int prec, int rhs_per_thread, int block);
int ov_get_tuning(ov_ctx *ctx, int prec, int *rhs_per_thread, int *block);
/* Site order of the dslash launches: 0 = each XCD walks a contiguous run of
 * time slices; 1 = each XCD walks a z-slab plane by plane (needs Lz % 8 == 0
 * and V % 64 == 0); 2 = every thread owns one (x, y, z) site and one RHS and
 * marches along t, keeping the time neighbours in registers (needs
 * V % 64 == 0); 3 = each XCD walks a t-slab, t fastest (needs Lt % 8 == 0
 * and V % 64 == 0).  Where a requirement fails, order 0 is used.
 * ov_autotune searches all four. */
int ov_set_site_order(ov_ctx *ctx, int prec, int order);
/* Cap on resident dslash workgroups per CU (0 = no cap).  A small cap keeps
 * the set of sites in flight narrow enough for stencil neighbours to be
 * re-read from L2 instead of HBM. */
int ov_set_occupancy(ov_ctx *ctx, int prec, int blocks_per_cu);
/* Launch shape of precision prec for kind 0 (plain H_w / D_w launches) or
 * kind 1 (launches with the fused Clenshaw epilogue), which ov_autotune tunes
 * separately; the three setters above set both kinds.  cfg is
 * {rhs_per_thread, block, site_order, blocks_per_cu, stream_hint, rhs_split,
 * cols}, the first four with the meaning and range given above.  stream_hint 1
 * marks the operands a launch touches once (epilogue inputs, output)
 * non-temporal so that they do not displace stencil neighbours from L2.
 * rhs_split Q in {1, 2, 4, 8} (Q > 1 only with rhs_per_thread <= 2 and
 * site orders 0, 1; Q = 8 not for BF16 storage) splits each wavefront into Q
 * parts that cover the same 64/Q sites for Q groups of right-hand sides, so
 * each link is fetched once per Q * rhs_per_thread RHS.  cols (a divisor of
 * Ly; site order 1 only) walks each XCD's z-slab as cols y-columns one after
 * the other, which shortens the distance between a site and its t
 * neighbours in the walk.  wshare W in {1, 2, 4, 8}: with W > 1 (rhs_per_thread
 * <= 2, rhs_split <= 4) a workgroup is W waves that cover the same 64/Q sites
 * for W different groups of Q * rhs_per_thread RHS; the workgroup copies the
 * links of its sites into LDS once and every wave reads them there, so a link
 * is fetched once per W * Q * rhs_per_thread RHS (block is then unused; the
 * t-marching order ignores wshare).  ov_set_tuning resets wshare to 1.  Set:
 * OV_EINVAL on a value out of range (nothing changed). */
int ov_get_launch_config(ov_ctx *ctx, int prec, int kind, int cfg[8]);
int ov_set_launch_config(ov_ctx *ctx, int prec, int kind, const int cfg[8]);
int ov_autotune(ov_ctx *ctx, int prec, int nrhs, const char *cache_path);

/*
 * Capture of the sign / D(m) pipelines in HIP graphs (default on): the first
 * call with a given batch signature runs eagerly, the second captures the
 * launch sequence, later identical calls replay it.  Any change of links
 * packing, fields, small spaces, polynomial, tuning or workspace size drops
 * the captured graphs.  on = 0 runs every launch eagerly.
 */
int ov_set_graphs(ov_ctx *ctx, int on);

/* Bytes of device memory the context holds right now. */
int ov_memory_used(const ov_ctx *ctx, int64_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* OV_H */
