// Small dense FP64 linear algebra on the host (Rayleigh-Ritz problems of
// size <= ~100): Cholesky, symmetric eigendecomposition by Householder
// tridiagonalisation followed by the implicit symmetric QR algorithm with
// Wilkinson shifts (Golub & Van Loan, Sec. 8.3), and the symmetric-definite
// generalized problem.
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

// Symmetric QR algorithm on the tridiagonal matrix T = tridiag(e, d, e)
// (Golub & Van Loan, Matrix Computations, 4th ed., Alg. 8.3.2 "implicit
// symmetric QR step with Wilkinson shift" inside the deflation loop of
// Alg. 8.3.3).  d: diagonal (n); off: off[i] = T(i, i+1) (n - 1 used).
// Every Givens rotation G_k of plane (k, k+1) is accumulated as Q <- Q G_k
// (Q row-major n x n), so on exit T = diag(d) and the columns of Q are the
// eigenvectors of the matrix whose tridiagonal form T was.  Returns false
// if the active block has not split after 30 n sweeps.
namespace {

// c, s with [c s; -s c]^T [a; b] = [r; 0] (Golub & Van Loan, Alg. 5.1.3)
void givens(double a, double b, double* c, double* s) {
    if (b == 0.0) {
        *c = 1.0;
        *s = 0.0;
        return;
    }
    const double r = std::hypot(a, b);
    *c = a / r;
    *s = -b / r;
}

// One implicit QR step with Wilkinson shift on the unreduced block [p, q].
void qr_step(int n, int p, int q, double* d, double* off, double* Q) {
    // shift: eigenvalue of the trailing 2 x 2 block closer to d[q]
    const double half = 0.5 * (d[q - 1] - d[q]);
    const double b2 = off[q - 1] * off[q - 1];
    const double den = half + (half >= 0.0 ? 1.0 : -1.0) * std::hypot(half, off[q - 1]);
    const double mu = den != 0.0 ? d[q] - b2 / den : d[q];
    double x = d[p] - mu;   // first column of T - mu I ...
    double z = off[p];      // ... and, after the first rotation, the bulge
    for (int k = p; k < q; ++k) {
        double c, s;
        givens(x, z, &c, &s);
        if (k > p) off[k - 1] = c * x - s * z;   // the bulge moves down
        const double a = d[k], b = off[k], cc = d[k + 1];
        d[k] = c * c * a - 2.0 * c * s * b + s * s * cc;
        d[k + 1] = s * s * a + 2.0 * c * s * b + c * c * cc;
        off[k] = c * s * (a - cc) + (c * c - s * s) * b;
        if (k + 1 < q) {
            z = -s * off[k + 1];
            off[k + 1] *= c;
        }
        x = off[k];
        for (int i = 0; i < n; ++i) {
            double* row = Q + (size_t)i * n;
            const double u = row[k], v = row[k + 1];
            row[k] = c * u - s * v;
            row[k + 1] = s * u + c * v;
        }
    }
}

bool tridiagonal_qr(int n, double* d, double* off, double* Q) {
    const double eps = 2.220446049250313e-16;
    int q = n - 1;
    long sweeps = 0;
    while (q > 0) {
        // deflate converged eigenvalues at the bottom
        if (std::fabs(off[q - 1]) <= eps * (std::fabs(d[q - 1]) + std::fabs(d[q])) ||
            std::fabs(off[q - 1]) < 1e-300) {
            off[q - 1] = 0.0;
            --q;
            continue;
        }
        // largest unreduced block ending at q
        int p = q - 1;
        while (p > 0) {
            if (std::fabs(off[p - 1]) <= eps * (std::fabs(d[p - 1]) + std::fabs(d[p])) ||
                std::fabs(off[p - 1]) < 1e-300) {
                off[p - 1] = 0.0;
                break;
            }
            --p;
        }
        if (++sweeps > 30L * n) return false;
        qr_step(n, p, q, d, off, Q);
    }
    return true;
}

}  // namespace

bool sym_eig(int n, const double* A, double* w, double* V) {
    for (size_t i = 0; i < (size_t)n * n; ++i)
        if (!std::isfinite(A[i])) return false;
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
    // e[i] = T(i, i-1) -> off[i] = T(i, i+1)
    std::vector<double> off(n, 0.0);
    for (int i = 0; i + 1 < n; ++i) off[i] = e[i + 1];
    if (!tridiagonal_qr(n, d.data(), off.data(), Q.data())) return false;
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
