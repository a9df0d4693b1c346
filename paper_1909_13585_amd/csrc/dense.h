// Small dense FP64 host linear algebra (row-major).
#pragma once

namespace mlb {

bool cholesky(int n, double* A);
// eigenvalues w descending, eigenvectors as columns of V (row-major n x n)
bool sym_eig(int n, const double* A, double* w, double* V);
// B y = mu A y, A SPD; mu descending, Y columns A-orthonormal
bool gen_eig(int n, const double* A, const double* B, double* mu, double* Y);

}  // namespace mlb
