// Small dense FP64 linear algebra on the host (Rayleigh-Ritz problems of
// size <= ~100): Cholesky, symmetric eigendecomposition by Householder
// tridiagonalisation followed by implicit-shift QL iterations (Golub & Van
// Loan, Sec. 8.3), and the symmetric-definite generalized problem.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace mlb {

// Lower Cholesky factor in place (row-major n x n, upper part zeroed).
bool cholesky(int n, double* A) {
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double l = std::sqrt(d);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / l;
        }
        for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
    }
    return true;
}

// Householder reduction of symmetric A (row-major, overwritten by the
// accumulated orthogonal transform Q) to tridiagonal form: diag d, sub e
// (e[0] unused), with A_in = Q T Q^T.
static void tridiagonalize(int n, double* Q, double* d, double* e) {
    std::vector<double> a(Q, Q + (size_t)n * n);
    auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
    // Q starts as identity, accumulate H_1 H_2 ... applied on the right
    std::vector<double> q((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), w(n);
    for (int k = 0; k < n - 2; ++k) {
        // column below the diagonal: x = A[k+1:, k]
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += A(i, k) * A(i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        const double x0 = A(k + 1, k);
        if (x0 > 0) alpha = -alpha;  // avoid cancellation: v = x - alpha e1
        std::fill(v.begin(), v.end(), 0.0);
        v[k + 1] = x0 - alpha;
        for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // A <- H A H with H = I - beta v v^T:  p = beta A v, K = beta/2 v^T p, w = p - K v
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
            p[i] = beta * s;
        }
        double Kc = 0.0;
        for (int i = k + 1; i < n; ++i) Kc += v[i] * p[i];
        Kc *= 0.5 * beta;
        for (int i = 0; i < n; ++i) w[i] = p[i] - Kc * v[i];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) A(i, j) -= v[i] * w[j] + w[i] * v[j];
        // Q <- Q H
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += q[(size_t)i * n + j] * v[j];
            s *= beta;
            for (int j = k + 1; j < n; ++j) q[(size_t)i * n + j] -= s * v[j];
        }
    }
    for (int i = 0; i < n; ++i) {
        d[i] = A(i, i);
        e[i] = i > 0 ? A(i, i - 1) : 0.0;
    }
    std::copy(q.begin(), q.end(), Q);
}

// Implicit-shift QL on the tridiagonal (d, e), accumulating rotations into
// the columns of Q.  Returns false if an eigenvalue fails to converge.
static bool tql(int n, double* d, double* e, double* Q) {
    for (int i = 1; i < n; ++i) e[i - 1] = e[i];
    if (n > 0) e[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        int m;
        do {
            for (m = l; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-300 || std::fabs(e[m]) <= 2.2e-16 * dd) break;
            }
            if (m != l) {
                if (++iter > 60) return false;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = std::hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i];
                    const double b = c * e[i];
                    r = std::hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    for (int k = 0; k < n; ++k) {
                        f = Q[(size_t)k * n + i + 1];
                        Q[(size_t)k * n + i + 1] = s * Q[(size_t)k * n + i] + c * f;
                        Q[(size_t)k * n + i] = c * Q[(size_t)k * n + i] - s * f;
                    }
                }
                if (r == 0.0 && i >= l) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    return true;
}

bool sym_eig(int n, const double* A, double* w, double* V) {
    std::vector<double> Q(A, A + (size_t)n * n), d(n), e(n);
    // symmetrise input
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            const double v = 0.5 * (Q[(size_t)i * n + j] + Q[(size_t)j * n + i]);
            Q[(size_t)i * n + j] = Q[(size_t)j * n + i] = v;
        }
    if (n == 1) {
        w[0] = Q[0];
        V[0] = 1.0;
        return true;
    }
    tridiagonalize(n, Q.data(), d.data(), e.data());
    if (!tql(n, d.data(), e.data(), Q.data())) return false;
    // sort descending, eigenvectors as columns (row-major V[i*n + j]: row i of column j)
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] > d[b]; });
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Q[(size_t)i * n + idx[j]];
    }
    return true;
}

// B y = mu A y with A SPD: A = L L^T, C = L^-1 B L^-T, C z = mu z, y = L^-T z.
// Eigenvalues descending; Y columns A-orthonormal (row-major n x n).
bool gen_eig(int n, const double* A, const double* B, double* mu, double* Y) {
    std::vector<double> L(A, A + (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            const double v = 0.5 * (L[(size_t)i * n + j] + L[(size_t)j * n + i]);
            L[(size_t)i * n + j] = L[(size_t)j * n + i] = v;
        }
    if (!cholesky(n, L.data())) return false;
    // W = L^-1 B  (forward substitution on columns)
    std::vector<double> W(B, B + (size_t)n * n), C((size_t)n * n);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            double s = W[(size_t)i * n + c];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * W[(size_t)k * n + c];
            W[(size_t)i * n + c] = s / L[(size_t)i * n + i];
        }
    // C = W L^-T  = (L^-1 W^T)^T
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) {
            double s = W[(size_t)r * n + i];
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * C[(size_t)r * n + k];
            C[(size_t)r * n + i] = s / L[(size_t)i * n + i];
        }
    std::vector<double> Z((size_t)n * n);
    if (!sym_eig(n, C.data(), mu, Z.data())) return false;
    // Y = L^-T Z  (back substitution)
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double s = Z[(size_t)i * n + c];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * Y[(size_t)k * n + c];
            Y[(size_t)i * n + c] = s / L[(size_t)i * n + i];
        }
    return true;
}

}  // namespace mlb
