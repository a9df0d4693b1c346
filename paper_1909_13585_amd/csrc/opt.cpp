// Host runtime of the optimisation layer (mlb_opt.h): continuation of the
// SIMP exponent and the projection sharpness (Secs. 3, 6), the problem
// functions of P1 / P2 with the bound formulation of the buckling constraint
// (Sec. 3), and the method of moving asymptotes (Svanberg 1987).
//
// The MMA subproblem
//   min f~_0(x) + sum_i (c y_i + d y_i^2 / 2)
//   s.t. f~_i(x) - y_i <= 0,  alpha <= x <= beta,  y >= 0,
//   f~_i(x) = r_i + sum_j p_ij / (U_j - x_j) + q_ij / (x_j - L_j),
// is strictly convex and separable, so it is solved exactly through its dual
// in the m multipliers lam >= 0:
//   W(lam) = f~_0(x(lam)) + sum_i lam_i (f~_i(x(lam)) - y_i(lam))
//            + sum_i (c y_i + d y_i^2 / 2),
//   y_i(lam) = max(0, (lam_i - c) / d),
//   grad W = f~_i(x(lam)) - y_i,   Hess W = -B^T B - diag(lam_i > c) / d,
// with x(lam) and the sums on the device (kernels_mma.hip) and the
// m-dimensional Newton iteration here: projected Newton steps on the set of
// multipliers that are positive or pushed up, damped in the
// Levenberg-Marquardt way (a step is kept only if W does not drop; the
// damping falls tenfold after a kept step and rises tenfold after a refused
// one).  The damping handles the stretches where every x_j sits on its box
// and W is piecewise linear.  The iteration stops when the projected
// gradient is below 1e-13 (1 + max |r_i|), or when no damped step raises W
// any more (the rounding floor of the sums) with the projected gradient
// below 1e-9 (1 + max |r_i|); a stall above that is MLB_ENOTCONV.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/mlb_opt.h"
#include "kernels.h"

using namespace mlb;

struct mlb_mma {
    int64_t n = 0;
    int m = 0;
    int dev = 0;
    int it = 0;
    MmaParams pr{};
    double c = 1000.0, d = 1.0;
    std::string err;
    double *low = nullptr, *upp = nullptr, *xold1 = nullptr, *xold2 = nullptr, *alo = nullptr, *bhi = nullptr;
    double *B = nullptr, *part = nullptr, *gpart = nullptr, *sums = nullptr;
    int nparts = 0, gparts = 0;
    int evals = 0;
};

namespace {

int mfail(mlb_mma* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define MHIPC(call)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return mfail(h, MLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Solves (A + mu I) d = g for symmetric positive semidefinite A (k x k,
// row-major) by Cholesky; false if the shifted matrix is not positive
// definite in floating point.
bool shifted_solve(int k, const std::vector<double>& A, double mu, const std::vector<double>& g,
                   std::vector<double>& d) {
    std::vector<double> Lm((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[(size_t)i * k + j] + (i == j ? mu : 0.0);
            for (int t = 0; t < j; ++t) s -= Lm[(size_t)i * k + t] * Lm[(size_t)j * k + t];
            if (i == j) {
                if (!(s > 0.0)) return false;
                Lm[(size_t)i * k + i] = std::sqrt(s);
            } else {
                Lm[(size_t)i * k + j] = s / Lm[(size_t)j * k + j];
            }
        }
    }
    d.assign(k, 0.0);
    for (int i = 0; i < k; ++i) {
        double s = g[i];
        for (int t = 0; t < i; ++t) s -= Lm[(size_t)i * k + t] * d[t];
        d[i] = s / Lm[(size_t)i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = d[i];
        for (int t = i + 1; t < k; ++t) s -= Lm[(size_t)t * k + i] * d[t];
        d[i] = s / Lm[(size_t)i * k + i];
    }
    return true;
}

// One dual evaluation at lam: W, grad, Hessian (row-major m x m), y.
struct DualPoint {
    std::vector<double> lam, g, H, y;
    double W = 0.0, pg = 0.0;
};

struct Dual {
    mlb_mma* h;
    const double* df0;
    const double* dfdx;
    int64_t ldg;
    hipStream_t st;
    std::vector<double> r;      // r_0 .. r_m
    std::vector<double> host;   // sums (m + 1) then Gram (m x m, column-major)

    int eval(const std::vector<double>& lam, DualPoint& P) {
        const int m = h->m;
        MmaLam L{};
        for (int i = 0; i < m; ++i) L.v[i] = lam[i];
        launch_mma_dual(h->n, m, L, h->pr, h->xold1, h->low, h->upp, h->alo, h->bhi, df0, dfdx, ldg, h->nparts,
                        h->part, h->B, nullptr, st);
        launch_sum_parts(m + 1, h->nparts, h->part, h->sums, st);
        if (launch_gram(h->n, m, h->n, h->B, m, h->n, h->B, 0, 0, nullptr, h->gparts, h->gpart, h->sums + m + 1,
                        st) != 0)
            return mfail(h, MLB_EINVAL, "too many constraints for the Gram kernel");
        MHIPC(hipGetLastError());
        MHIPC(hipMemcpyAsync(host.data(), h->sums, sizeof(double) * host.size(), hipMemcpyDeviceToHost, st));
        MHIPC(hipStreamSynchronize(st));
        ++h->evals;
        for (double v : host)
            if (!std::isfinite(v)) return mfail(h, MLB_EINVAL, "non-finite MMA sums (check the gradients)");
        P.lam = lam;
        P.y.assign(m, 0.0);
        P.g.assign(m, 0.0);
        P.H.assign((size_t)m * m, 0.0);
        const double h0 = r[0] + host[0];
        double W = h0;
        for (int i = 0; i < m; ++i) {
            const double yi = std::max(0.0, (lam[i] - h->c) / h->d);
            const double hi = r[i + 1] + host[i + 1];
            P.y[i] = yi;
            P.g[i] = hi - yi;
            W += lam[i] * (hi - yi) + h->c * yi + 0.5 * h->d * yi * yi;
        }
        P.W = W;
        const double* G = host.data() + m + 1;
        for (int i = 0; i < m; ++i)
            for (int k = 0; k < m; ++k) P.H[(size_t)i * m + k] = -G[i + (size_t)m * k];
        for (int i = 0; i < m; ++i)
            if (lam[i] > h->c) P.H[(size_t)i * m + i] -= 1.0 / h->d;
        double pg = 0.0;
        for (int i = 0; i < m; ++i) pg = std::max(pg, std::fabs(lam[i] > 0.0 ? P.g[i] : std::max(P.g[i], 0.0)));
        P.pg = pg;
        return MLB_OK;
    }
};

}  // namespace

extern "C" {

int mlb_continuation(int step, double p0, double dp, int p_every, double p_max, double beta0, int beta_every,
                     double beta_max, double* p, double* beta) {
    if (!p || !beta || step < 0 || !(dp > 0.0) || p_every < 1 || !(p_max >= p0) || !(beta0 > 0.0) || beta_every < 0 ||
        (beta_every > 0 && !(beta_max >= beta0)))
        return MLB_EINVAL;
    *p = std::min(p0 + dp * (double)(step / p_every), p_max);
    *beta = beta0;
    if (beta_every == 0) return MLB_OK;
    const int inc = std::max(0, (int)std::ceil((p_max - p0) / dp - 1e-12));
    const long long k_p = (long long)inc * p_every;
    if (step < k_p) return MLB_OK;
    const long long dbl = (step - k_p) / beta_every;
    *beta = dbl >= 60 ? beta_max : std::min(beta0 * std::ldexp(1.0, (int)dbl), beta_max);
    return MLB_OK;
}

}  // extern "C"

namespace {

int problem_functions(int kind, int64_t m, int nb, const double* x, double J, const double* dJ, const double* lam,
                      const double* dlam, int64_t ld, double Jscale, double lam_bar, double f_bar, double alpha,
                      double* f0, double* fval, double* grad, void* stream) {
    if (m < 1 || nb < 1 || nb > kMmaMaxCon - 2 || !x || !dJ || !lam || !dlam || !f0 || !fval || !grad || ld < m)
        return MLB_EINVAL;
    if (!(Jscale > 0.0) || !(lam_bar > 0.0) || !(alpha > 0.0) || !(alpha <= 1.0) || !std::isfinite(J) ||
        (kind == 1 && !(f_bar > 0.0)))
        return MLB_EINVAL;
    for (int i = 0; i < nb; ++i)
        if (!std::isfinite(lam[i])) return MLB_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    MmaLam w{};
    double a = 1.0;
    for (int i = 0; i < nb; ++i) {
        a *= alpha;
        w.v[i] = a / lam_bar;
    }
    const int np = mma_parts(m);
    double* buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * (np + 1)) != hipSuccess) return MLB_ENOMEM;
    const double vcol = kind == 1 ? 1.0 / ((double)m * f_bar) : 1.0 / (double)m;
    launch_opt_cols(m, kind, nb, x, dJ, 1.0 / Jscale, vcol, dlam, ld, w, grad, np, buf, st);
    launch_sum_parts(1, np, buf, buf + np, st);
    double vsum = 0.0;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&vsum, buf + np, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(buf);
    if (e != hipSuccess) return MLB_EDEVICE;
    const double vol = vsum / (double)m;
    if (kind == 1) {
        *f0 = J / Jscale;
        fval[0] = vol / f_bar - 1.0;
    } else {
        *f0 = vol;
        fval[0] = J / Jscale - 1.0;
    }
    for (int i = 0; i < nb; ++i) fval[1 + i] = 1.0 - w.v[i] * lam[i];
    return MLB_OK;
}

}  // namespace

extern "C" {

int mlb_p1_functions_dev(int64_t m, int nb, const double* x, double J, const double* dJ, const double* lam,
                         const double* dlam, int64_t ld, double J0, double lam_bar, double f_bar, double alpha,
                         double* f0, double* fval, double* grad, void* stream) {
    return problem_functions(1, m, nb, x, J, dJ, lam, dlam, ld, J0, lam_bar, f_bar, alpha, f0, fval, grad, stream);
}

int mlb_p2_functions_dev(int64_t m, int nb, const double* x, double J, const double* dJ, const double* lam,
                         const double* dlam, int64_t ld, double J_max, double lam_bar, double alpha, double* f0,
                         double* fval, double* grad, void* stream) {
    return problem_functions(2, m, nb, x, J, dJ, lam, dlam, ld, J_max, lam_bar, 1.0, alpha, f0, fval, grad, stream);
}

int mlb_mma_create(int64_t n, int m, const mlb_mma_opts* o, int device, mlb_mma** out) {
    if (!out || n < 1 || m < 1 || m > kMmaMaxCon) return MLB_EINVAL;
    *out = nullptr;
    mlb_mma_opts op{};
    if (o) op = *o;
    MmaParams pr{};
    pr.xmin = op.xmax > op.xmin ? op.xmin : 0.0;
    pr.xmax = op.xmax > op.xmin ? op.xmax : 1.0;
    pr.move = op.move > 0.0 ? op.move : 0.2;
    pr.asyinit = op.asyinit > 0.0 ? op.asyinit : 0.5;
    pr.asyincr = op.asyincr > 0.0 ? op.asyincr : 1.2;
    pr.asydecr = op.asydecr > 0.0 ? op.asydecr : 0.7;
    const double c = op.c > 0.0 ? op.c : 1000.0, d = op.d > 0.0 ? op.d : 1.0;
    for (double v : {pr.xmin, pr.xmax, pr.move, pr.asyinit, pr.asyincr, pr.asydecr, c, d})
        if (!std::isfinite(v)) return MLB_EINVAL;
    if (pr.asydecr >= 1.0 || pr.asyincr < 1.0) return MLB_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return MLB_EDEVICE;
    mlb_mma* h = new mlb_mma();
    h->n = n;
    h->m = m;
    h->dev = device;
    h->pr = pr;
    h->c = c;
    h->d = d;
    h->nparts = mma_parts(n);
    h->gparts = gram_parts(n, m, m);
    const size_t vec = sizeof(double) * (size_t)n;
    bool ok = true;
    for (double** p : {&h->low, &h->upp, &h->xold1, &h->xold2, &h->alo, &h->bhi})
        ok = ok && hipMalloc(p, vec) == hipSuccess;
    ok = ok && hipMalloc(&h->B, vec * m) == hipSuccess;
    ok = ok && hipMalloc(&h->part, sizeof(double) * (size_t)h->nparts * (m + 1)) == hipSuccess;
    ok = ok && hipMalloc(&h->gpart, sizeof(double) * (size_t)h->gparts * m * m) == hipSuccess;
    ok = ok && hipMalloc(&h->sums, sizeof(double) * (size_t)(m + 1 + m * m)) == hipSuccess;
    if (!ok) {
        mlb_mma_destroy(h);
        return MLB_ENOMEM;
    }
    *out = h;
    return MLB_OK;
}

void mlb_mma_destroy(mlb_mma* h) {
    if (!h) return;
    for (double* p : {h->low, h->upp, h->xold1, h->xold2, h->alo, h->bhi, h->B, h->part, h->gpart, h->sums})
        if (p) hipFree(p);
    delete h;
}

const char* mlb_mma_last_error(const mlb_mma* h) { return h ? h->err.c_str() : "null MMA handle"; }

int mlb_mma_update_dev(mlb_mma* h, double* x, double f0, const double* df0, const double* fval, const double* dfdx,
                       int64_t ldg, mlb_mma_info* info, void* stream) {
    if (!h || !x || !df0 || !fval || !dfdx) return h ? mfail(h, MLB_EINVAL, "null argument") : MLB_EINVAL;
    if (ldg < h->n) return mfail(h, MLB_EINVAL, "ldg must be >= n");
    if (!std::isfinite(f0)) return mfail(h, MLB_EINVAL, "non-finite objective");
    const int m = h->m;
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(fval[i])) return mfail(h, MLB_EINVAL, "non-finite constraint value");
    const double t0 = now_s();
    hipStream_t st = (hipStream_t)stream;
    h->evals = 0;
    // asymptotes, move limits, history; the sums that fix r
    launch_mma_prep(h->n, m, h->it, h->pr, x, h->xold1, h->xold2, h->low, h->upp, h->alo, h->bhi, df0, dfdx, ldg,
                    h->nparts, h->part, st);
    launch_sum_parts(m + 1, h->nparts, h->part, h->sums, st);
    MHIPC(hipGetLastError());
    Dual D{h, df0, dfdx, ldg, st, std::vector<double>(m + 1), std::vector<double>((size_t)(m + 1 + m * m))};
    MHIPC(hipMemcpyAsync(D.host.data(), h->sums, sizeof(double) * (m + 1), hipMemcpyDeviceToHost, st));
    MHIPC(hipStreamSynchronize(st));
    ++h->it;
    D.r[0] = f0 - D.host[0];
    for (int i = 0; i < m; ++i) D.r[i + 1] = fval[i] - D.host[i + 1];
    double rmax = 0.0;
    for (double v : D.r) rmax = std::max(rmax, std::fabs(v));
    if (!std::isfinite(rmax)) return mfail(h, MLB_EINVAL, "non-finite MMA sums (check the gradients)");
    const double tol = 1e-13 * (1.0 + rmax);
    // a stall (no damped step raises W) counts as converged below this: the
    // dual sums over n variables carry rounding far above 1e-13 for large n
    const double stall_tol = 1e-9 * (1.0 + rmax);
    // projected Newton on the dual
    DualPoint P, T;
    int rc = D.eval(std::vector<double>(m, 0.0), P);
    if (rc != MLB_OK) return rc;
    double tr = 0.0;
    for (int i = 0; i < m; ++i) tr -= P.H[(size_t)i * m + i];
    double mu = 1e-10 * (1.0 + tr / m);
    int its = 0;
    bool converged = false;
    const int max_it = 500;
    for (; its < max_it; ++its) {
        if (P.pg <= tol) {
            converged = true;
            break;
        }
        std::vector<int> F;
        for (int i = 0; i < m; ++i)
            if (P.lam[i] > 0.0 || P.g[i] > 0.0) F.push_back(i);
        const int k = (int)F.size();
        std::vector<double> A((size_t)k * k), gF(k), dF;
        for (int a = 0; a < k; ++a) {
            gF[a] = P.g[F[a]];
            for (int b = 0; b < k; ++b) A[(size_t)a * k + b] = -P.H[(size_t)F[a] * m + F[b]];
        }
        bool taken = false;
        for (int tries = 0; tries < 100; ++tries) {
            if (shifted_solve(k, A, mu, gF, dF)) {
                std::vector<double> lt = P.lam;
                for (int a = 0; a < k; ++a) lt[F[a]] = std::max(0.0, P.lam[F[a]] + dF[a]);
                rc = D.eval(lt, T);
                if (rc != MLB_OK) return rc;
                if (T.W > P.W || (T.W >= P.W - 1e-15 * std::fabs(P.W) && T.pg < P.pg)) {
                    taken = true;
                    break;
                }
            }
            mu *= 10.0;
        }
        if (!taken) {
            // no step raises W: the sums' rounding floor is reached
            converged = P.pg <= stall_tol;
            break;
        }
        P = T;
        mu = std::max(mu * 0.1, 1e-300);
    }
    // the final minimiser into x
    MmaLam L{};
    for (int i = 0; i < m; ++i) L.v[i] = P.lam[i];
    launch_mma_dual(h->n, m, L, h->pr, h->xold1, h->low, h->upp, h->alo, h->bhi, df0, dfdx, ldg, h->nparts, h->part,
                    nullptr, x, st);
    MHIPC(hipGetLastError());
    MHIPC(hipStreamSynchronize(st));
    if (info) {
        *info = mlb_mma_info{};
        info->dual_iterations = its;
        info->dual_evaluations = h->evals;
        info->proj_grad = P.pg;
        info->dual_value = P.W;
        for (int i = 0; i < m; ++i) {
            info->lam[i] = P.lam[i];
            info->y[i] = P.y[i];
        }
        info->seconds = now_s() - t0;
    }
    if (!converged) return mfail(h, MLB_ENOTCONV, "MMA dual solve stopped before its tolerance");
    return MLB_OK;
}

}  // extern "C"
