// Per-variable work of the method of moving asymptotes (Svanberg 1987) and
// of the design problems' gradient columns (Secs. 3 and 6).
//
// One MMA update is a handful of passes over the n design variables, each a
// grid-stride loop with per-block partial sums (partial b of value i at
// part[i nparts + b], summed by k_sum_parts in a fixed order):
//   k_mma_prep   asymptotes L, U and move limits alpha, beta from the last
//                two steps; the history shift; the sums that fix r_i;
//   k_mma_dual   for given multipliers lam: each variable's minimiser of the
//                subproblem Lagrangian, the sums sum_j p_ij / (U - x) +
//                q_ij / (x - L) of every approximation, and (optionally) the
//                scaled columns B whose Gram product gives the dual Hessian,
//                or the minimiser itself (the final pass).
// The approximation coefficients are never stored: with g = df_i/dx_j at x^k,
//   p_ij = (U - x^k)^2 (1.001 g+ + 0.001 g- + reg),
//   q_ij = (x^k - L)^2 (0.001 g+ + 1.001 g- + reg),   reg = 1e-5 / (xmax - xmin),
// are rebuilt from the gradient rows in each pass.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace mlb {

namespace {

__device__ inline double mma_wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums acc[0..cnt) over the block and writes partial b of value i to
// part[i nparts + b]; sh holds (blockDim / 64) x M doubles.
template <int M>
__device__ inline void mma_block_parts(const double (&acc)[M], int cnt, double* sh, int64_t nparts, double* part) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        if (i < cnt) {
            const double v = mma_wsum(acc[i]);
            if (lane == 0) sh[wid * M + i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w * M + threadIdx.x];
        part[(int64_t)threadIdx.x * nparts + blockIdx.x] = s;
    }
}

__device__ inline void mma_pq(double g, double reg, double& pc, double& qc) {
    const double gp = fmax(g, 0.0), gm = fmax(-g, 0.0);
    pc = 1.001 * gp + 0.001 * gm + reg;
    qc = 0.001 * gp + 1.001 * gm + reg;
}

__device__ inline double mma_grad(int i, int64_t j, const double* __restrict__ df0, const double* __restrict__ dfdx,
                                  int64_t ldg) {
    return i == 0 ? df0[j] : dfdx[(int64_t)(i - 1) * ldg + j];
}

// Asymptotes and move limits (it = number of earlier updates), then the
// history shift xold2 <- xold1 <- x, and the sums S_i = sum_j [(U - x) pc_ij
// + (x - L) qc_ij] (= sum_j p_ij/(U - x) + q_ij/(x - L) at x^k).
template <int M>
__global__ __launch_bounds__(kBlock) void k_mma_prep(int64_t n, int m, int it, MmaParams pr,
                                                     const double* __restrict__ x, double* __restrict__ xold1,
                                                     double* __restrict__ xold2, double* __restrict__ low,
                                                     double* __restrict__ upp, double* __restrict__ alo,
                                                     double* __restrict__ bhi, const double* __restrict__ df0,
                                                     const double* __restrict__ dfdx, int64_t ldg,
                                                     double* __restrict__ part) {
    __shared__ double sh[(kBlock / 64) * M];
    const double dx = pr.xmax - pr.xmin, reg = 1e-5 / dx;
    double acc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) acc[i] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double xj = x[j];
        double L, U;
        if (it < 2) {
            L = xj - pr.asyinit * dx;
            U = xj + pr.asyinit * dx;
        } else {
            const double x1 = xold1[j], x2 = xold2[j];
            const double trend = (xj - x1) * (x1 - x2);
            const double f = trend > 0.0 ? pr.asyincr : (trend < 0.0 ? pr.asydecr : 1.0);
            L = xj - f * (x1 - low[j]);
            U = xj + f * (upp[j] - x1);
            L = fmin(fmax(L, xj - 10.0 * dx), xj - 0.01 * dx);
            U = fmin(fmax(U, xj + 0.01 * dx), xj + 10.0 * dx);
        }
        const double a = fmax(fmax(pr.xmin, L + 0.1 * (xj - L)), xj - pr.move * dx);
        const double b = fmin(fmin(pr.xmax, U - 0.1 * (U - xj)), xj + pr.move * dx);
        low[j] = L;
        upp[j] = U;
        alo[j] = a;
        bhi[j] = b;
        xold2[j] = it >= 1 ? xold1[j] : xj;
        xold1[j] = xj;
        const double ux = U - xj, xl = xj - L;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i <= m) {
                double pc, qc;
                mma_pq(mma_grad(i, j, df0, dfdx, ldg), reg, pc, qc);
                acc[i] += ux * pc + xl * qc;
            }
        }
    }
    mma_block_parts<M>(acc, m + 1, sh, gridDim.x, part);
}

// Dual pass for multipliers lam (lam.v[0..m)): x_j(lam) minimises
//   P_j / (U - x) + Q_j / (x - L) over [alpha_j, beta_j],
//   P_j = p_0j + sum_i lam_i p_ij,  Q_j likewise,
// at x = (L sqrt(P) + U sqrt(Q)) / (sqrt(P) + sqrt(Q)) clipped to the box.
// Sums h_i = sum_j p_ij / (U - x) + q_ij / (x - L) for i = 0..m.  With B,
// B[(i-1) n + j] = a_ij / sqrt(c_j) for variables strictly inside their box
// (0 otherwise), a_ij = p_ij / (U - x)^2 - q_ij / (x - L)^2 and c_j =
// 2 P / (U - x)^3 + 2 Q / (x - L)^3, so that the dual Hessian is -B^T B
// (plus the elastic variables' diagonal).  With xout, writes x_j(lam).
template <int M>
__global__ __launch_bounds__(kBlock) void k_mma_dual(int64_t n, int m, MmaLam lam, MmaParams pr,
                                                     const double* __restrict__ xk, const double* __restrict__ low,
                                                     const double* __restrict__ upp, const double* __restrict__ alo,
                                                     const double* __restrict__ bhi, const double* __restrict__ df0,
                                                     const double* __restrict__ dfdx, int64_t ldg,
                                                     double* __restrict__ part, double* __restrict__ B,
                                                     double* __restrict__ xout) {
    __shared__ double sh[(kBlock / 64) * M];
    const double reg = 1e-5 / (pr.xmax - pr.xmin);
    double acc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) acc[i] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double x0 = xk[j], L = low[j], U = upp[j], a = alo[j], b = bhi[j];
        const double u0 = (U - x0) * (U - x0), l0 = (x0 - L) * (x0 - L);
        double P = 0.0, Q = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i <= m) {
                double pc, qc;
                mma_pq(mma_grad(i, j, df0, dfdx, ldg), reg, pc, qc);
                const double w = i == 0 ? 1.0 : lam.v[i - 1];
                P += w * pc;
                Q += w * qc;
            }
        }
        P *= u0;
        Q *= l0;
        const double sp = sqrt(P), sq = sqrt(Q);
        const double xs = (L * sp + U * sq) / (sp + sq);
        const double xj = fmin(fmax(xs, a), b);
        const double ux = 1.0 / (U - xj), xl = 1.0 / (xj - L);
        const bool inside = xj > a && xj < b;
        const double rc = B && inside ? 1.0 / sqrt(2.0 * P * ux * ux * ux + 2.0 * Q * xl * xl * xl) : 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (i <= m) {
                double pc, qc;
                mma_pq(mma_grad(i, j, df0, dfdx, ldg), reg, pc, qc);
                const double p = u0 * pc, q = l0 * qc;
                acc[i] += p * ux + q * xl;
                if (B && i >= 1) B[(int64_t)(i - 1) * n + j] = (p * ux * ux - q * xl * xl) * rc;
            }
        }
        if (xout) xout[j] = xj;
    }
    mma_block_parts<M>(acc, m + 1, sh, gridDim.x, part);
}

// Gradient columns of problems P1 / P2 (see mlb_opt.h) and the partial sums
// of x (the volume).  kind 1: [dJ sJ, vcol, -w_i dlam_i]; kind 2: [vcol,
// dJ sJ, -w_i dlam_i].  Column c at c m of grad.
__global__ __launch_bounds__(kBlock) void k_opt_cols(int64_t m, int kind, int nb, const double* __restrict__ x,
                                                     const double* __restrict__ dJ, double sJ, double vcol,
                                                     const double* __restrict__ dlam, int64_t ld, MmaLam w,
                                                     double* __restrict__ grad, double* __restrict__ part) {
    __shared__ double sh[kBlock / 64];
    double acc[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        acc[0] += x[e];
        const double gJ = dJ[e] * sJ;
        grad[(kind == 1 ? 0 : 1) * m + e] = gJ;
        grad[(kind == 1 ? 1 : 0) * m + e] = vcol;
        for (int i = 0; i < nb; ++i) grad[(int64_t)(2 + i) * m + e] = -w.v[i] * dlam[(int64_t)i * ld + e];
    }
    mma_block_parts<1>(acc, 1, sh, gridDim.x, part);
}

}  // namespace

int mma_parts(int64_t n) {
    int64_t p = (n + 4 * kBlock - 1) / (4 * kBlock);
    if (p < 1) p = 1;
    if (p > kMaxPartials) p = kMaxPartials;
    return (int)p;
}

#define MLB_MMA_DISPATCH(KER, ...)                                                                        \
    do {                                                                                                  \
        if (m + 1 <= 8) hipLaunchKernelGGL(KER<8>, dim3(nparts), dim3(kBlock), 0, st, __VA_ARGS__);        \
        else if (m + 1 <= 16) hipLaunchKernelGGL(KER<16>, dim3(nparts), dim3(kBlock), 0, st, __VA_ARGS__); \
        else hipLaunchKernelGGL(KER<kMmaMaxCon + 1>, dim3(nparts), dim3(kBlock), 0, st, __VA_ARGS__);      \
    } while (0)

void launch_mma_prep(int64_t n, int m, int it, const MmaParams& pr, const double* x, double* xold1, double* xold2,
                     double* low, double* upp, double* alo, double* bhi, const double* df0, const double* dfdx,
                     int64_t ldg, int nparts, double* part, hipStream_t st) {
    MLB_MMA_DISPATCH(k_mma_prep, n, m, it, pr, x, xold1, xold2, low, upp, alo, bhi, df0, dfdx, ldg, part);
}

void launch_mma_dual(int64_t n, int m, const MmaLam& lam, const MmaParams& pr, const double* xk, const double* low,
                     const double* upp, const double* alo, const double* bhi, const double* df0, const double* dfdx,
                     int64_t ldg, int nparts, double* part, double* B, double* xout, hipStream_t st) {
    MLB_MMA_DISPATCH(k_mma_dual, n, m, lam, pr, xk, low, upp, alo, bhi, df0, dfdx, ldg, part, B, xout);
}
#undef MLB_MMA_DISPATCH

void launch_opt_cols(int64_t m, int kind, int nb, const double* x, const double* dJ, double sJ, double vcol,
                     const double* dlam, int64_t ld, const MmaLam& w, double* grad, int nparts, double* part,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_opt_cols, dim3(nparts), dim3(kBlock), 0, st, m, kind, nb, x, dJ, sJ, vcol, dlam, ld, w, grad,
                       part);
}

}  // namespace mlb
