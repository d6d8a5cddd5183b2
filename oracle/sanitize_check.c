/*
 * Sanitizer driver for the FP64 oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Compiled together with oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py, it runs every
 * oracle entry point on tiny lattices (including 2^4, where forward and
 * backward neighbours coincide, and a Dirichlet lattice) and exits 0 when no
 * sanitizer reports an error.  Inputs come from a fixed linear congruential
 * generator; the numbers themselves are not checked here (the pins do that).
 */
#include "oracle.c"

#include <stdio.h>

static unsigned long long lcg_state = 12345u;
static double lcg_uniform(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) / 9007199254740992.0 - 0.5;
}

static void fill(cplx *a, long n)
{
    for (long i = 0; i < n; ++i) a[i] = lcg_uniform() + I * lcg_uniform();
}

/* Gram-Schmidt on l random vectors of length N. */
static void orthonormal(cplx *v, int l, long N)
{
    fill(v, (long)l * N);
    for (int i = 0; i < l; ++i) {
        for (int j = 0; j < i; ++j) {
            cplx d = or_dot(N, v + (long)j * N, v + (long)i * N);
            for (long k = 0; k < N; ++k) v[(long)i * N + k] -= d * v[(long)j * N + k];
        }
        double nn = sqrt(creal(or_dot(N, v + (long)i * N, v + (long)i * N)));
        for (long k = 0; k < N; ++k) v[(long)i * N + k] /= nn;
    }
}

static int run(const int L[4], const int bc[4])
{
    long V = (long)L[0] * L[1] * L[2] * L[3], N = 12 * V;
    cplx *U = malloc(sizeof(cplx) * 36 * V), *x = malloc(sizeof(cplx) * N), *y = malloc(sizeof(cplx) * N);
    cplx *g = malloc(sizeof(cplx) * N), *gx = malloc(sizeof(cplx) * N), *gU = malloc(sizeof(cplx) * 36 * V);
    cplx *Vs = malloc(sizeof(cplx) * 3 * N), *W = malloc(sizeof(cplx) * 2 * N), *xs = malloc(sizeof(cplx) * N);
    double c[9], lam[3] = {0.3, -0.2, 0.1}, geta = 0, rr = 0;
    int it = 0;
    if (!U || !x || !y || !g || !gx || !gU || !Vs || !W || !xs) return 2;
    fill(U, 36 * V);
    for (long i = 0; i < 36 * V; ++i) U[i] *= 0.4;   /* norm well below 6.5 / 4 per link */
    fill(x, N);
    fill(g, N);
    orthonormal(Vs, 3, N);
    orthonormal(W, 2, N);
    or_field f = {{L[0], L[1], L[2], L[3]}, {bc[0], bc[1], bc[2], bc[3]}, -1.5, 0.01, U};
    or_cheb_coeffs(8, 0.05, c);
    (void)or_cheb_eval(8, 0.05, c, 0.3);
    or_sign_params p = {8, 0.05, 6.5, c, 3, Vs, lam};
    cplx gm[16];
    for (int mu = 0; mu < 5; ++mu) or_gamma(mu, gm);
    or_dslash(&f, 0, x, y);
    or_dslash(&f, 1, x, y);
    or_gamma5(V, x, y);
    if (or_sign(&f, &p, x, y)) return 3;
    if (or_dov(&f, &p, 0.05, 0, x, y) || or_dov(&f, &p, 0.05, 1, x, y)) return 4;
    memset(xs, 0, sizeof(cplx) * N);
    (void)or_cg(&f, &p, 0.1, 2, W, x, xs, 1e-8, 30, &it, &rr);
    if (or_sign_backward(&f, &p, 2.0 / 3.0, x, g, gU, &geta, gx)) return 5;
    free(U); free(x); free(y); free(g); free(gx); free(gU); free(Vs); free(W); free(xs);
    return 0;
}

int main(void)
{
    const int L1[4] = {2, 2, 2, 2}, bc1[4] = {0, 0, 0, 1};
    const int L2[4] = {2, 4, 2, 6}, bc2[4] = {2, 0, 0, 2};
    int rc = run(L1, bc1);
    if (!rc) rc = run(L2, bc2);
    printf("sanitize_check rc=%d\n", rc);
    return rc;
}
