// Small dense complex linear algebra on the host (column-major, order <= 256).
#pragma once

#include <complex>

namespace ov {

// Hermitian A (overwritten): eigenvalues w ascending, orthonormal eigenvectors
// in the columns of Z.
int heev_jacobi(int n, std::complex<double> *A, double *w, std::complex<double> *Z);
// G = R^H R, R upper triangular, in place; nonzero: index of a failed pivot.
int potrf_upper(int n, std::complex<double> *G);
// R <- R^{-1}, R upper triangular.
int trinv_upper(int n, std::complex<double> *R);

}  // namespace ov
