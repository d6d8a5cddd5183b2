// Small dense complex linear algebra on the host for the eigensolver's
// Rayleigh-Ritz and orthonormalisation steps (matrices of order <= 256, so
// O(n^3) host work is a few milliseconds next to the field operations).
// Column-major storage, element (i, j) at i + n j.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace ov {

using cd = std::complex<double>;

// Cyclic Jacobi for a Hermitian matrix.  Each rotation zeroes one
// off-diagonal pair: with b = a_pq = |b| e^{i phi}, U = diag(1, e^{-i phi}) R
// (R the real symmetric Jacobi rotation of [[a_pp, |b|], [|b|, a_qq]]) makes
// the (p, q) block of U^H A U diagonal.
int heev_jacobi(int n, cd *A, double *w, cd *Z)
{
    if (n <= 0) return 0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) Z[i + (size_t)n * j] = (i == j) ? 1.0 : 0.0;
    double fro = 0;
    for (size_t e = 0; e < (size_t)n * n; ++e) fro += std::norm(A[e]);
    fro = std::sqrt(fro);
    if (fro == 0) {
        for (int i = 0; i < n; ++i) w[i] = 0;
        return 0;
    }
    const int max_sweeps = 60;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0;
        for (int q = 0; q < n; ++q)
            for (int p = 0; p < q; ++p) off += std::norm(A[p + (size_t)n * q]);
        if (std::sqrt(2 * off) <= 1e-16 * fro) break;
        for (int q = 1; q < n; ++q)
            for (int p = 0; p < q; ++p) {
                const cd b = A[p + (size_t)n * q];
                const double ab = std::abs(b);
                if (ab <= 1e-300) continue;
                const double app = A[p + (size_t)n * p].real(), aqq = A[q + (size_t)n * q].real();
                const double zeta = (aqq - app) / (2 * ab);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
                const double c = 1 / std::sqrt(1 + t * t), s = t * c;
                const cd ph = b / ab;                  // e^{i phi}
                // U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
                const cd u_pp = c, u_pq = s, u_qp = -s * std::conj(ph), u_qq = c * std::conj(ph);
                // A <- A U (columns p, q)
                for (int i = 0; i < n; ++i) {
                    const cd x = A[i + (size_t)n * p], y = A[i + (size_t)n * q];
                    A[i + (size_t)n * p] = x * u_pp + y * u_qp;
                    A[i + (size_t)n * q] = x * u_pq + y * u_qq;
                }
                // A <- U^H A (rows p, q)
                for (int j = 0; j < n; ++j) {
                    const cd x = A[p + (size_t)n * j], y = A[q + (size_t)n * j];
                    A[p + (size_t)n * j] = std::conj(u_pp) * x + std::conj(u_qp) * y;
                    A[q + (size_t)n * j] = std::conj(u_pq) * x + std::conj(u_qq) * y;
                }
                A[p + (size_t)n * q] = 0;
                A[q + (size_t)n * p] = 0;
                A[p + (size_t)n * p] = A[p + (size_t)n * p].real();
                A[q + (size_t)n * q] = A[q + (size_t)n * q].real();
                for (int i = 0; i < n; ++i) {
                    const cd x = Z[i + (size_t)n * p], y = Z[i + (size_t)n * q];
                    Z[i + (size_t)n * p] = x * u_pp + y * u_qp;
                    Z[i + (size_t)n * q] = x * u_pq + y * u_qq;
                }
            }
    }
    // ascending eigenvalues, columns of Z permuted alike
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(),
              [&](int a, int b) { return A[a + (size_t)n * a].real() < A[b + (size_t)n * b].real(); });
    std::vector<cd> Zs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = A[idx[j] + (size_t)n * idx[j]].real();
        for (int i = 0; i < n; ++i) Zs[i + (size_t)n * j] = Z[i + (size_t)n * idx[j]];
    }
    std::copy(Zs.begin(), Zs.end(), Z);
    return 0;
}

// G = R^H R with R upper triangular; R overwrites the upper triangle of G and
// the strict lower triangle is zeroed.  Returns the first non-positive pivot
// (1-based) or 0.
int potrf_upper(int n, cd *G)
{
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i <= j; ++i) {
            cd s = G[i + (size_t)n * j];
            for (int k = 0; k < i; ++k) s -= std::conj(G[k + (size_t)n * i]) * G[k + (size_t)n * j];
            if (i == j) {
                const double d = s.real();
                if (!(d > 0)) return j + 1;
                G[j + (size_t)n * j] = std::sqrt(d);
            } else {
                G[i + (size_t)n * j] = s / G[i + (size_t)n * i].real();
            }
        }
        for (int i = j + 1; i < n; ++i) G[i + (size_t)n * j] = 0;
    }
    return 0;
}

// R <- R^{-1} for upper triangular R (back substitution column by column).
int trinv_upper(int n, cd *R)
{
    for (int i = 0; i < n; ++i)
        if (R[i + (size_t)n * i] == cd(0)) return i + 1;
    std::vector<cd> X((size_t)n * n, cd(0));
    for (int j = 0; j < n; ++j) {
        X[j + (size_t)n * j] = 1.0 / R[j + (size_t)n * j];
        for (int i = j - 1; i >= 0; --i) {
            cd s = 0;
            for (int k = i + 1; k <= j; ++k) s += R[i + (size_t)n * k] * X[k + (size_t)n * j];
            X[i + (size_t)n * j] = -s / R[i + (size_t)n * i];
        }
    }
    std::copy(X.begin(), X.end(), R);
    return 0;
}

}  // namespace ov

extern "C" int ov_dense_heev(int n, const double *A, double *w, double *Z)
{
    if (n < 0 || n > 4096 || (n > 0 && (!A || !w || !Z))) return -1;
    std::vector<std::complex<double>> a((size_t)n * n), z((size_t)n * n);
    for (size_t e = 0; e < (size_t)n * n; ++e) a[e] = {A[2 * e], A[2 * e + 1]};
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < j; ++i) {   // Hermitian part
            const std::complex<double> h = 0.5 * (a[i + (size_t)n * j] + std::conj(a[j + (size_t)n * i]));
            a[i + (size_t)n * j] = h;
            a[j + (size_t)n * i] = std::conj(h);
        }
    for (int i = 0; i < n; ++i) a[i + (size_t)n * i] = a[i + (size_t)n * i].real();
    ov::heev_jacobi(n, a.data(), w, z.data());
    for (size_t e = 0; e < (size_t)n * n; ++e) {
        Z[2 * e] = z[e].real();
        Z[2 * e + 1] = z[e].imag();
    }
    return 0;
}
