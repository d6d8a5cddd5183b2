/*
 * FP64 CPU oracle for the overlap operator D_ov = 1 + gamma5 sign(H_w).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP library against a plain,
 * slow, obviously correct implementation.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * Everything is double precision, std C99 complex, OpenMP over lattice sites
 * only where a loop is trivially parallel.  No blocking, fusion or reordering
 * beyond what the definitions state.
 *
 * Paper: "Electric polarizability of hadrons with overlap fermions on
 * multi-GPUs" (Lattice 2011).  Sections cited:
 *   Sec. 2, eq. (1)     D_ov = 1 + gamma5 sign(H_w), H_w = gamma5 D_w
 *   Sec. 2 (text)       sign(H_w) ~ Q P(Q^2), Q = H_w/||H_w||, P ~ x^{-1/2}
 *   Sec. 2, eq. (2)     delta = A exp(-b n sqrt(eps))   (used by the tests)
 *   Sec. 2 (text, Fig.1) small space treated exactly, polynomial elsewhere
 *   Sec. 3.2            CG for D_ov^{-1} psi, deflation (Sec. 2 end)
 *   Sec. 4, eq. (3)     U(1) background field: links times a phase
 *   Sec. 4 (text)       Dirichlet boundary conditions in field dir. and time
 * The paper leaves the gamma basis, the Wilson normalisation, the polynomial
 * construction and the massive operator open; the readings taken here are:
 *   - chiral basis gamma_k = [[0,-i s_k],[i s_k,0]], gamma_4 = [[0,1],[1,0]],
 *     gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1,1,-1,-1);
 *   - D_w psi(x) = (4+m_w) psi(x)
 *       - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu) + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ];
 *   - boundary multiplier b_mu in {+1 periodic, -1 antiperiodic, 0 Dirichlet}
 *     on hops that wrap around the lattice;
 *   - U(1) phase exp(i q eta t) multiplying the mu = 0 (x) links;
 *   - P = Chebyshev interpolant of y^{-1/2} on [eps, 1] at the n+1
 *     Chebyshev-Gauss nodes, degree n in y = Q^2, evaluated by Clenshaw;
 *   - two-sided projection: s = V sgn(lam) V^dag + Pi Q P(Q^2) Pi, Pi = 1 - V V^dag;
 *   - massive operator D(m) = (1 - m/2) D_ov + m, D(m)^dag = gamma5 D(m) gamma5.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Problem description, mirrored by ctypes structures in oracle/api.py.     */

typedef struct {
    int L[4];          /* Lx, Ly, Lz, Lt                                      */
    int bc[4];         /* 0 periodic, 1 antiperiodic, 2 Dirichlet             */
    double mw;         /* Wilson mass m_w                                     */
    double qeta;       /* q*eta: phase exp(i q eta t) on the mu = 0 links     */
    const cplx *U;     /* links [4][V][3][3]                                  */
} or_field;

typedef struct {
    int n;             /* polynomial degree in Q^2                            */
    double eps;        /* approximation interval [eps, 1] for y = Q^2         */
    double norm;       /* N_norm >= ||H_w||, Q = H_w / N_norm                 */
    const double *c;   /* Chebyshev coefficients c_0..c_n                     */
    int l;             /* small-space dimension                               */
    const cplx *V;     /* small-space vectors [l][V][4][3], orthonormal       */
    const double *lam; /* their H_w eigenvalues (only the sign is used)       */
} or_sign_params;

static long or_volume(const or_field *f)
{
    return (long)f->L[0] * f->L[1] * f->L[2] * f->L[3];
}

/* ------------------------------------------------------------------------ */
/* Gamma matrices (chiral basis), built from the Pauli matrices.            */

static void or_pauli(int k, cplx s[2][2])
{
    memset(s, 0, sizeof(cplx) * 4);
    if (k == 1) { s[0][1] = 1; s[1][0] = 1; }
    if (k == 2) { s[0][1] = -I; s[1][0] = I; }
    if (k == 3) { s[0][0] = 1; s[1][1] = -1; }
}

/* mu = 0,1,2,3 -> gamma_1..gamma_4 ; mu = 4 -> gamma5 = g1 g2 g3 g4. */
void or_gamma(int mu, cplx *g /* [4][4] row-major */)
{
    cplx G[4][4];
    memset(G, 0, sizeof G);
    if (mu >= 0 && mu <= 2) {
        cplx s[2][2];
        or_pauli(mu + 1, s);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[a][2 + b] = -I * s[a][b];
                G[2 + a][b] = I * s[a][b];
            }
    } else if (mu == 3) {
        G[0][2] = G[1][3] = G[2][0] = G[3][1] = 1;
    } else {
        cplx A[4][4], B[4][4], T[4][4];
        or_gamma(0, &A[0][0]);
        for (int m = 1; m < 4; ++m) {
            or_gamma(m, &B[0][0]);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    cplx acc = 0;
                    for (int k = 0; k < 4; ++k) acc += A[i][k] * B[k][j];
                    T[i][j] = acc;
                }
            memcpy(A, T, sizeof A);
        }
        memcpy(G, A, sizeof G);
    }
    memcpy(g, G, sizeof G);
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                        */

static void or_coords(const int L[4], long i, int c[4])
{
    c[0] = (int)(i % L[0]); i /= L[0];
    c[1] = (int)(i % L[1]); i /= L[1];
    c[2] = (int)(i % L[2]); i /= L[2];
    c[3] = (int)i;
}

static long or_index(const int L[4], const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static double or_bc_factor(int bc)
{
    return bc == 0 ? 1.0 : (bc == 1 ? -1.0 : 0.0);
}

/* Neighbour j = i +/- mu-hat; returns the boundary multiplier of the hop. */
static double or_hop(const or_field *f, long i, int mu, int dir, long *j)
{
    int c[4];
    or_coords(f->L, i, c);
    double b = 1.0;
    c[mu] += dir;
    if (c[mu] >= f->L[mu]) { c[mu] -= f->L[mu]; b = or_bc_factor(f->bc[mu]); }
    if (c[mu] < 0)         { c[mu] += f->L[mu]; b = or_bc_factor(f->bc[mu]); }
    *j = or_index(f->L, c);
    return b;
}

/* Link U_mu(i) including the U(1) background phase on mu = 0. */
static void or_link(const or_field *f, int mu, long i, cplx W[3][3])
{
    long V = or_volume(f);
    const cplx *u = f->U + ((long)mu * V + i) * 9;
    cplx ph = 1.0;
    if (mu == 0) {
        int c[4];
        or_coords(f->L, i, c);
        ph = cexp(I * f->qeta * (double)c[3]);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) W[a][b] = ph * u[a * 3 + b];
}

/* ------------------------------------------------------------------------ */
/* Wilson Dirac operator and H_w = gamma5 D_w                              */

/* y = D_w x (op = 0) or y = gamma5 D_w x (op = 1).  x, y: [V][4][3]. */
void or_dslash(const or_field *f, int op, const cplx *x, cplx *y)
{
    long V = or_volume(f);
    cplx G[4][4][4], Gm[4][4][4], G5[4][4];
    for (int mu = 0; mu < 4; ++mu) {
        or_gamma(mu, &G[mu][0][0]);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx one = (a == b) ? 1.0 : 0.0;
                Gm[mu][a][b] = one - G[mu][a][b];  /* 1 - gamma_mu */
                G[mu][a][b] = one + G[mu][a][b];   /* 1 + gamma_mu */
            }
    }
    or_gamma(4, &G5[0][0]);

#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        cplx acc[4][3];
        for (int s = 0; s < 4; ++s)
            for (int c = 0; c < 3; ++c) acc[s][c] = (4.0 + f->mw) * x[(i * 4 + s) * 3 + c];
        for (int mu = 0; mu < 4; ++mu) {
            long j;
            double b = or_hop(f, i, mu, +1, &j);
            if (b != 0.0) {   /* -1/2 (1 - gamma_mu) U_mu(i) x(i+mu) */
                cplx W[3][3], u[4][3];
                or_link(f, mu, i, W);
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int c = 0; c < 3; ++c) t += W[a][c] * x[(j * 4 + s) * 3 + c];
                        u[s][a] = t;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int r = 0; r < 4; ++r) t += Gm[mu][s][r] * u[r][a];
                        acc[s][a] -= 0.5 * b * t;
                    }
            }
            b = or_hop(f, i, mu, -1, &j);
            if (b != 0.0) {   /* -1/2 (1 + gamma_mu) U_mu(i-mu)^dag x(i-mu) */
                cplx W[3][3], u[4][3];
                or_link(f, mu, j, W);
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int c = 0; c < 3; ++c) t += conj(W[c][a]) * x[(j * 4 + s) * 3 + c];
                        u[s][a] = t;
                    }
                for (int s = 0; s < 4; ++s)
                    for (int a = 0; a < 3; ++a) {
                        cplx t = 0;
                        for (int r = 0; r < 4; ++r) t += G[mu][s][r] * u[r][a];
                        acc[s][a] -= 0.5 * b * t;
                    }
            }
        }
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx v = acc[s][a];
                if (op == 1) {
                    cplx t = 0;
                    for (int r = 0; r < 4; ++r) t += G5[s][r] * acc[r][a];
                    v = t;
                }
                y[(i * 4 + s) * 3 + a] = v;
            }
    }
}

/* y = gamma5 x */
void or_gamma5(long V, const cplx *x, cplx *y)
{
    cplx G5[4][4];
    or_gamma(4, &G5[0][0]);
    for (long i = 0; i < V; ++i)
        for (int s = 0; s < 4; ++s)
            for (int a = 0; a < 3; ++a) {
                cplx t = 0;
                for (int r = 0; r < 4; ++r) t += G5[s][r] * x[(i * 4 + r) * 3 + a];
                y[(i * 4 + s) * 3 + a] = t;
            }
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers (plain loops)                                       */

static cplx or_dot(long n, const cplx *a, const cplx *b)   /* sum conj(a) b */
{
    cplx s = 0;
    for (long k = 0; k < n; ++k) s += conj(a[k]) * b[k];
    return s;
}

static cplx *or_alloc(long n)
{
    return (cplx *)calloc((size_t)n, sizeof(cplx));
}

/* ------------------------------------------------------------------------ */
/* Chebyshev coefficients of y^{-1/2} on [eps, 1]                          */
/*
 * Interpolation at the n+1 Chebyshev-Gauss nodes t_j = cos(pi (j+1/2)/(n+1)),
 * mapped to y_j = ((1-eps) t_j + 1 + eps)/2:
 *   c_k = 2/(n+1) sum_j y_j^{-1/2} cos(pi k (j+1/2)/(n+1)),  c_0 halved,
 * so that P(y) = sum_k c_k T_k(t(y)), t(y) = (2y - 1 - eps)/(1 - eps).
 */
void or_cheb_coeffs(int n, double eps, double *c)
{
    int m = n + 1;
    for (int k = 0; k <= n; ++k) {
        double s = 0;
        for (int j = 0; j < m; ++j) {
            double th = M_PI * (j + 0.5) / m;
            double y = ((1.0 - eps) * cos(th) + 1.0 + eps) / 2.0;
            s += cos(k * th) / sqrt(y);
        }
        c[k] = 2.0 * s / m;
    }
    c[0] *= 0.5;
}

/* Scalar P(y) by the same Clenshaw recursion (used for error curves). */
double or_cheb_eval(int n, double eps, const double *c, double y)
{
    double t = (2.0 * y - 1.0 - eps) / (1.0 - eps);
    double b1 = 0, b2 = 0;
    for (int k = n; k >= 1; --k) {
        double b0 = c[k] + 2.0 * t * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + t * b1 - b2;
}

/* ------------------------------------------------------------------------ */
/* Sign function: exact small space + Q P(Q^2) on the rest                  */

/* y = T v with T = (2 Q^2 - (1+eps)) / (1-eps), Q = H_w / norm. */
static void or_apply_T(const or_field *f, const or_sign_params *p, const cplx *v,
                       cplx *y, cplx *tmp)
{
    long N = or_volume(f) * 12;
    or_dslash(f, 1, v, tmp);
    or_dslash(f, 1, tmp, y);
    double a = 2.0 / ((1.0 - p->eps) * p->norm * p->norm);
    double b = (1.0 + p->eps) / (1.0 - p->eps);
    for (long k = 0; k < N; ++k) y[k] = a * y[k] - b * v[k];
}

/* out[k] = sum_i C_i V_i[k]   (C: [l]) */
static void or_combine(long N, int l, const cplx *V, const cplx *C, cplx *out)
{
    for (long k = 0; k < N; ++k) out[k] = 0;
    for (int i = 0; i < l; ++i)
        for (long k = 0; k < N; ++k) out[k] += C[i] * V[(long)i * N + k];
}

/* y = s(x), the approximate sign(H_w) applied to x.  Returns 0 on success. */
int or_sign(const or_field *f, const or_sign_params *p, const cplx *x, cplx *y)
{
    long N = or_volume(f) * 12;
    int l = p->l;
    cplx *C = or_alloc(l > 0 ? l : 1), *D = or_alloc(l > 0 ? l : 1);
    cplx *chi = or_alloc(N), *b1 = or_alloc(N), *b2 = or_alloc(N), *b0 = or_alloc(N);
    cplx *tb = or_alloc(N), *tmp = or_alloc(N), *proj = or_alloc(N);
    if (!C || !D || !chi || !b1 || !b2 || !b0 || !tb || !tmp || !proj) return -2;

    /* C = V^dag x ; chi = Pi x = x - V C */
    for (int i = 0; i < l; ++i) C[i] = or_dot(N, p->V + (long)i * N, x);
    or_combine(N, l, p->V, C, proj);
    for (long k = 0; k < N; ++k) chi[k] = x[k] - proj[k];

    /* Clenshaw: b_{n+1} = b_{n+2} = 0, b_k = c_k chi + 2 T b_{k+1} - b_{k+2} */
    for (int k = p->n; k >= 1; --k) {
        or_apply_T(f, p, b1, tb, tmp);
        for (long q = 0; q < N; ++q) b0[q] = p->c[k] * chi[q] + 2.0 * tb[q] - b2[q];
        cplx *r = b2; b2 = b1; b1 = b0; b0 = r;
    }
    /* z = c_0 chi + T b_1 - b_2  (= P(Q^2) chi) -> stored in b0 */
    or_apply_T(f, p, b1, tb, tmp);
    for (long q = 0; q < N; ++q) b0[q] = p->c[0] * chi[q] + tb[q] - b2[q];

    /* w = Q z ; w <- Pi w */
    or_dslash(f, 1, b0, tmp);
    for (long q = 0; q < N; ++q) tmp[q] /= p->norm;
    for (int i = 0; i < l; ++i) D[i] = or_dot(N, p->V + (long)i * N, tmp);
    or_combine(N, l, p->V, D, proj);
    for (long q = 0; q < N; ++q) tmp[q] -= proj[q];

    /* y = w + V sgn(lam) C  (sgn(0) := +1) */
    for (int i = 0; i < l; ++i) D[i] = (p->lam[i] >= 0 ? 1.0 : -1.0) * C[i];
    or_combine(N, l, p->V, D, proj);
    for (long q = 0; q < N; ++q) y[q] = tmp[q] + proj[q];

    free(C); free(D); free(chi); free(b1); free(b2); free(b0); free(tb); free(tmp); free(proj);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Overlap operator                                                         */

/* y = D(m) x = (1 - m/2)(x + gamma5 s(x)) + m x ; dagger: gamma5 D(m) gamma5 x. */
int or_dov(const or_field *f, const or_sign_params *p, double m, int dagger,
           const cplx *x, cplx *y)
{
    long V = or_volume(f), N = V * 12;
    cplx *u = or_alloc(N), *s = or_alloc(N), *g = or_alloc(N);
    if (!u || !s || !g) return -2;
    const cplx *in = x;
    if (dagger) { or_gamma5(V, x, u); in = u; }
    int rc = or_sign(f, p, in, s);
    if (rc) return rc;
    or_gamma5(V, s, g);
    for (long k = 0; k < N; ++k) y[k] = (1.0 - 0.5 * m) * (in[k] + g[k]) + m * in[k];
    if (dagger) { or_gamma5(V, y, u); memcpy(y, u, sizeof(cplx) * N); }
    free(u); free(s); free(g);
    return 0;
}

/* y = A x with A = D(m)^dag D(m) */
static int or_normal_op(const or_field *f, const or_sign_params *p, double m,
                        const cplx *x, cplx *y, cplx *tmp)
{
    int rc = or_dov(f, p, m, 0, x, tmp);
    if (rc) return rc;
    return or_dov(f, p, m, 1, tmp, y);
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient on A = D(m)^dag D(m), A x = D(m)^dag b                */
/*
 * Textbook CG.  With k > 0 deflation vectors W (orthonormal), the initial
 * guess is corrected by the Galerkin step x += W Lambda^{-1} W^dag r with
 * Lambda_i = <w_i, A w_i> computed here.  Stops when the recursive residual
 * reaches tol; then the true residual ||D^dag b - A x|| / ||D^dag b|| is
 * computed and, if still above tol, CG restarts from it.
 * Returns 0 on convergence, -4 if maxiter was reached.
 */
int or_cg(const or_field *f, const or_sign_params *p, double m, int k,
          const cplx *W, const cplx *b, cplx *x, double tol, int maxiter,
          int *iters_out, double *relres_out)
{
    long N = or_volume(f) * 12;
    cplx *rhs = or_alloc(N), *r = or_alloc(N), *pp = or_alloc(N), *Ap = or_alloc(N);
    cplx *tmp = or_alloc(N);
    if (!rhs || !r || !pp || !Ap || !tmp) return -2;
    int rc = or_dov(f, p, m, 1, b, rhs);
    if (rc) return rc;
    double rhs_norm = sqrt(creal(or_dot(N, rhs, rhs)));
    if (rhs_norm == 0) {
        for (long q = 0; q < N; ++q) x[q] = 0;
        *iters_out = 0; *relres_out = 0;
        free(rhs); free(r); free(pp); free(Ap); free(tmp);
        return 0;
    }

    if (k > 0) {
        or_normal_op(f, p, m, x, Ap, tmp);
        for (long q = 0; q < N; ++q) r[q] = rhs[q] - Ap[q];
        for (int i = 0; i < k; ++i) {
            const cplx *w = W + (long)i * N;
            or_normal_op(f, p, m, w, Ap, tmp);
            double lam = creal(or_dot(N, w, Ap));
            cplx coef = or_dot(N, w, r) / lam;
            for (long q = 0; q < N; ++q) x[q] += coef * w[q];
        }
    }

    int it = 0;
    double relres = 0;
    for (;;) {
        or_normal_op(f, p, m, x, Ap, tmp);
        for (long q = 0; q < N; ++q) r[q] = rhs[q] - Ap[q];
        double rr = creal(or_dot(N, r, r));
        relres = sqrt(rr) / rhs_norm;
        if (relres <= tol || it >= maxiter) break;
        memcpy(pp, r, sizeof(cplx) * N);
        while (it < maxiter && sqrt(rr) / rhs_norm > tol) {
            or_normal_op(f, p, m, pp, Ap, tmp);
            double pAp = creal(or_dot(N, pp, Ap));
            double alpha = rr / pAp;
            for (long q = 0; q < N; ++q) { x[q] += alpha * pp[q]; r[q] -= alpha * Ap[q]; }
            double rr_new = creal(or_dot(N, r, r));
            double beta = rr_new / rr;
            rr = rr_new;
            for (long q = 0; q < N; ++q) pp[q] = r[q] + beta * pp[q];
            ++it;
        }
    }
    *iters_out = it;
    *relres_out = relres;
    free(rhs); free(r); free(pp); free(Ap); free(tmp);
    return relres <= tol ? 0 : -4;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the sign function                                             */
/*
 * L = Re <g, s(U, eta) x> with V, lam, norm, eps, c held fixed.  With
 * chi = Pi x, the Clenshaw vectors b_k, z = P(Q^2) chi, w-bar = Pi g,
 * z-bar = Q w-bar and the adjoint Chebyshev vectors bb_k = T_k(T) z-bar:
 *   dL = Re<wbar, dQ z> + Re<zbar, dT b_1> + sum_{k=1..n} 2 Re<bb_k, dT b_{k+1}>,
 *   dT = (2/(1-eps)) (dQ Q + Q dQ),  dQ = gamma5 dD_w / norm.
 * Each Re<u, dQ v> adds the Wilson force
 *   G_mu(x) += -(b/(2 norm)) [ sum_s ((1-gamma_mu) gamma5 u)(x)_s v(x+mu)_s^dag
 *                           + sum_s v(x)_s ((1+gamma_mu) gamma5 u(x+mu))_s^dag ]
 * (b the boundary multiplier of the hop), for the phased links, with
 * dL = sum Re tr(G^dag dU).  The gradient w.r.t. the base links is
 * exp(-i q eta t) G_0 on mu = 0, and dL/deta = sum_x Re tr(G_0^dag i q t U~_0).
 * The gradient w.r.t. x is s g (s is Hermitian).
 */

/* G[mu][x] += coef * force(u, v) for the phased links */
static void or_force_acc(const or_field *f, double coef, const cplx *u, const cplx *v,
                         cplx *G /* [4][V][3][3] */)
{
    long V = or_volume(f);
    cplx Gm[4][4][4], Gp[4][4][4], G5[4][4];
    for (int mu = 0; mu < 4; ++mu) {
        cplx g[4][4];
        or_gamma(mu, &g[0][0]);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx one = (a == b) ? 1.0 : 0.0;
                Gm[mu][a][b] = one - g[a][b];
                Gp[mu][a][b] = one + g[a][b];
            }
    }
    or_gamma(4, &G5[0][0]);
    double fac = -0.5 * coef;

#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        for (int mu = 0; mu < 4; ++mu) {
            long j;
            double b = or_hop(f, i, mu, +1, &j);
            if (b == 0.0) continue;
            /* a = gamma5 u at i and at j */
            cplx ai[4][3], aj[4][3], pm[4][3], pp[4][3];
            for (int s = 0; s < 4; ++s)
                for (int c = 0; c < 3; ++c) {
                    cplx ti = 0, tj = 0;
                    for (int r = 0; r < 4; ++r) {
                        ti += G5[s][r] * u[(i * 4 + r) * 3 + c];
                        tj += G5[s][r] * u[(j * 4 + r) * 3 + c];
                    }
                    ai[s][c] = ti; aj[s][c] = tj;
                }
            for (int s = 0; s < 4; ++s)
                for (int c = 0; c < 3; ++c) {
                    cplx tm = 0, tp = 0;
                    for (int r = 0; r < 4; ++r) {
                        tm += Gm[mu][s][r] * ai[r][c];
                        tp += Gp[mu][s][r] * aj[r][c];
                    }
                    pm[s][c] = tm; pp[s][c] = tp;
                }
            cplx *g = G + ((long)mu * V + i) * 9;
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    cplx t = 0;
                    for (int s = 0; s < 4; ++s) {
                        t += pm[s][a] * conj(v[(j * 4 + s) * 3 + bb]);
                        t += v[(i * 4 + s) * 3 + a] * conj(pp[s][bb]);
                    }
                    g[a * 3 + bb] += fac * b * t;
                }
        }
    }
}

/*
 * Gradients of L = Re<g, s x>:  gU [4][V][3][3] (w.r.t. the base links, torch
 * convention grad = dL/dRe + i dL/dIm), geta = dL/deta for the charge q
 * (qeta = q * eta), gx = s g.  Any output may be NULL.
 */
int or_sign_backward(const or_field *f, const or_sign_params *p, double q,
                     const cplx *x, const cplx *g, cplx *gU, double *geta, cplx *gx)
{
    long V = or_volume(f), N = V * 12;
    int n = p->n, l = p->l;
    double kap = 2.0 / (1.0 - p->eps);
    double invN = 1.0 / p->norm;
    cplx *C = or_alloc(l > 0 ? l : 1);
    cplx *chi = or_alloc(N), *tmp = or_alloc(N), *tb = or_alloc(N), *proj = or_alloc(N);
    cplx *z = or_alloc(N), *wbar = or_alloc(N), *zbar = or_alloc(N);
    cplx *bb0 = or_alloc(N), *bb1 = or_alloc(N), *bb2 = or_alloc(N);
    cplx *Qu = or_alloc(N), *Qv = or_alloc(N);
    cplx *bk = or_alloc((long)(n + 3) * N);   /* b_0 .. b_{n+2}; b_{n+1} = b_{n+2} = 0 */
    cplx *G = or_alloc(4 * V * 9);
    if (!C || !chi || !tmp || !tb || !proj || !z || !wbar || !zbar || !bb0 || !bb1 ||
        !bb2 || !Qu || !Qv || !bk || !G)
        return -2;

    if (gx) or_sign(f, p, g, gx);
    if (!gU && !geta) goto done;

    /* forward: chi, all b_k, z */
    for (int i = 0; i < l; ++i) C[i] = or_dot(N, p->V + (long)i * N, x);
    or_combine(N, l, p->V, C, proj);
    for (long k = 0; k < N; ++k) chi[k] = x[k] - proj[k];
    for (int k = n; k >= 1; --k) {
        cplx *b1 = bk + (long)(k + 1) * N, *b2 = bk + (long)(k + 2) * N, *b0 = bk + (long)k * N;
        or_apply_T(f, p, b1, tb, tmp);
        for (long q2 = 0; q2 < N; ++q2) b0[q2] = p->c[k] * chi[q2] + 2.0 * tb[q2] - b2[q2];
    }
    or_apply_T(f, p, bk + N, tb, tmp);
    for (long q2 = 0; q2 < N; ++q2) z[q2] = p->c[0] * chi[q2] + tb[q2] - bk[2 * N + q2];

    /* wbar = Pi g ; zbar = Q wbar */
    for (int i = 0; i < l; ++i) C[i] = or_dot(N, p->V + (long)i * N, g);
    or_combine(N, l, p->V, C, proj);
    for (long k = 0; k < N; ++k) wbar[k] = g[k] - proj[k];
    or_dslash(f, 1, wbar, zbar);
    for (long k = 0; k < N; ++k) zbar[k] *= invN;

    /* Re<wbar, dQ z> */
    or_force_acc(f, invN, wbar, z, G);

    /* Re<zbar, dT b_1> = kap (Re<zbar, dQ Q b_1> + Re<Q zbar, dQ b_1>) */
    or_dslash(f, 1, bk + N, Qv);
    for (long k = 0; k < N; ++k) Qv[k] *= invN;
    or_force_acc(f, kap * invN, zbar, Qv, G);
    or_dslash(f, 1, zbar, Qu);
    for (long k = 0; k < N; ++k) Qu[k] *= invN;
    or_force_acc(f, kap * invN, Qu, bk + N, G);

    /* adjoint Chebyshev vectors bb_k = T_k(T) zbar, k = 1..n-1 (b_{n+1} = 0) */
    memcpy(bb0, zbar, sizeof(cplx) * N);           /* bb_0 */
    or_apply_T(f, p, zbar, bb1, tmp);                /* bb_1 */
    for (int k = 1; k <= n - 1; ++k) {
        const cplx *v = bk + (long)(k + 1) * N;     /* b_{k+1} */
        or_dslash(f, 1, v, Qv);
        for (long q2 = 0; q2 < N; ++q2) Qv[q2] *= invN;
        or_force_acc(f, 2.0 * kap * invN, bb1, Qv, G);
        or_dslash(f, 1, bb1, Qu);
        for (long q2 = 0; q2 < N; ++q2) Qu[q2] *= invN;
        or_force_acc(f, 2.0 * kap * invN, Qu, v, G);
        /* bb_{k+1} = 2 T bb_k - bb_{k-1} */
        or_apply_T(f, p, bb1, tb, tmp);
        for (long q2 = 0; q2 < N; ++q2) bb2[q2] = 2.0 * tb[q2] - bb0[q2];
        cplx *r = bb0; bb0 = bb1; bb1 = bb2; bb2 = r;
    }

    /* base-link gradient and d/deta */
    {
        double ge = 0;
        for (long i = 0; i < V; ++i) {
            int c[4];
            or_coords(f->L, i, c);
            double t = (double)c[3];
            cplx ph = cexp(I * f->qeta * t);
            const cplx *u0 = f->U + i * 9;
            cplx *g0 = G + i * 9;
            /* Re tr(G~^dag i q t U~) with U~ = ph U */
            cplx tr = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) tr += conj(g0[a * 3 + b]) * (I * q * t * ph * u0[a * 3 + b]);
            ge += creal(tr);
            for (int a = 0; a < 9; ++a) g0[a] *= conj(ph);
        }
        if (geta) *geta = ge;
        if (gU) memcpy(gU, G, sizeof(cplx) * 4 * V * 9);
    }

done:
    free(C); free(chi); free(tmp); free(tb); free(proj); free(z); free(wbar); free(zbar);
    free(bb0); free(bb1); free(bb2); free(Qu); free(Qv); free(bk); free(G);
    return 0;
}
