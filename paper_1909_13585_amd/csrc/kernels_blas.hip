// Block-vector kernels of the Krylov solvers and the eigensolver.
//
// Reductions are two-stage and deterministic: each block writes one partial
// per column (fixed-order wavefront trees), then a single block per output
// sums the partials in index order.  No atomics.
#include <algorithm>

#include "kernels.h"

namespace mlb {

__device__ inline double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// block of kBlock threads (1D); result valid in thread 0
__device__ inline double bsum(double v, double* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wsum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

__device__ inline double bmax(double v, double* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = fmax(s, sh[w]);
    return s;
}

static inline unsigned nb1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int reduction_parts(int64_t n) {
    int64_t p = (n + 4 * kBlock - 1) / (4 * kBlock);
    if (p < 1) p = 1;
    if (p > kMaxPartials) p = kMaxPartials;
    return (int)p;
}

// ---- elementwise

template <typename T>
__global__ void k_jacobi0(int64_t n, int ncols, int64_t ld, const T* __restrict__ dinv, T omega,
                          const T* __restrict__ r, T* __restrict__ z) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T d = omega * dinv[i];
    for (int c = 0; c < ncols; ++c) z[c * ld + i] = d * r[c * ld + i];
}

// b = (float) a and z = (omega D^-1) b in one pass: the right-hand side of a
// mixed-precision cycle and its first Jacobi sweep from zero (the same
// products as k_d2f followed by k_jacobi0<float>)
__global__ void k_d2f_jacobi0(int64_t n, int ncols, int64_t ld, const double* __restrict__ a,
                              const float* __restrict__ dinv, float omega, float* __restrict__ b,
                              float* __restrict__ z) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float d = omega * dinv[i];
    for (int c = 0; c < ncols; ++c) {
        const float v = (float)a[c * ld + i];
        b[c * ld + i] = v;
        z[c * ld + i] = d * v;
    }
}

__global__ void k_d2f(int64_t n, int ncols, int64_t ld, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) b[c * ld + i] = (float)a[c * ld + i];
}

__global__ void k_f2d(int64_t n, int ncols, int64_t ld, const float* __restrict__ a, double* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) b[c * ld + i] = (double)a[c * ld + i];
}

// ---- dots: grid (nparts, ncols)

__global__ void k_dot_part(int64_t n, int64_t lda, const double* __restrict__ a, int64_t ldb,
                           const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double sh[16];
    const int col = blockIdx.y;
    const double* ac = a + col * lda;
    const double* bc = b + col * ldb;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += ac[i] * bc[i];
    s = bsum(s, sh);
    if (threadIdx.x == 0) part[col * gridDim.x + blockIdx.x] = s;
}

// out[col] = sum_b part[col*nparts + b]  (one block per column)
__global__ void k_sum_parts(int64_t nparts, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[16];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) s += part[col * nparts + i];
    s = bsum(s, sh);
    if (threadIdx.x == 0) out[col] = s;
}

// Convergence test on the device after a CG update: an active column counts
// the iteration, and stops at rr <= thr (or with flags |= 2 when rr is not
// finite).  Inactive columns get alpha = 0 afterwards, so iterations run
// past convergence leave their x and r bitwise unchanged.
__global__ void k_cg_check(int ncols, const double* __restrict__ rr, const double* __restrict__ thr,
                           int* __restrict__ active, int* __restrict__ iters, int* __restrict__ flags) {
    const int c = threadIdx.x;
    if (c >= ncols || !active[c]) return;
    iters[c] += 1;
    const double v = rr[c];
    if (!(v == v) || v >= __builtin_huge_val()) {
        flags[c] |= 2;
        active[c] = 0;
    } else if (v <= thr[c]) {
        active[c] = 0;
    }
}

// alpha = rz / pq per active column; flags[col] = 1 on breakdown (pq <= 0 / non-finite)
__global__ void k_cg_alpha(int ncols, const double* __restrict__ rz, const double* __restrict__ pq,
                           const int* __restrict__ active, double* __restrict__ alpha, int* __restrict__ flags) {
    const int c = threadIdx.x;
    if (c >= ncols) return;
    double a = 0.0;
    if (active[c]) {
        const double d = pq[c];
        if (d > 0.0 && isfinite(d) && isfinite(rz[c])) a = rz[c] / d;
        else flags[c] = 1;
    }
    alpha[c] = a;
}

__global__ void k_cg_beta(int ncols, const double* __restrict__ rz_new, double* __restrict__ rz,
                          const int* __restrict__ active, double* __restrict__ beta) {
    const int c = threadIdx.x;
    if (c >= ncols) return;
    double b = 0.0;
    if (active[c] && rz[c] != 0.0) b = rz_new[c] / rz[c];
    beta[c] = b;
    rz[c] = rz_new[c];
}

// x += alpha p; r -= alpha q; partial r.r  (grid (nparts, ncols))
// flexible (Polak-Ribiere) beta = (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / (r_k.z_k)
__global__ void k_cg_beta_flex(int ncols, const double* __restrict__ rz_new, const double* __restrict__ rz_cross,
                               double* __restrict__ rz, const int* __restrict__ active, double* __restrict__ beta) {
    const int c = threadIdx.x;
    if (c >= ncols) return;
    double b = 0.0;
    if (active[c] && rz[c] != 0.0) b = (rz_new[c] - rz_cross[c]) / rz[c];
    beta[c] = b;
    rz[c] = rz_new[c];
}

// generic y = a*x + b*y over a contiguous array
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// out[i] = 1/sqrt(in[i]) (0 if in <= 0)
__global__ void k_rsqrt(int ncols, const double* __restrict__ in, double* __restrict__ out) {
    const int c = threadIdx.x;
    if (c < ncols) out[c] = in[c] > 0.0 ? 1.0 / sqrt(in[c]) : 0.0;
}

__global__ void k_cg_update_xr(int64_t n, int64_t ld, const double* __restrict__ alpha, const double* __restrict__ p,
                               const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
                               double* __restrict__ part) {
    __shared__ double sh[16];
    const int col = blockIdx.y;
    const double a = alpha[col];
    const int64_t o = col * ld;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[o + i] += a * p[o + i];
        const double rv = r[o + i] - a * q[o + i];
        r[o + i] = rv;
        s += rv * rv;
    }
    s = bsum(s, sh);
    if (threadIdx.x == 0) part[col * gridDim.x + blockIdx.x] = s;
}

__global__ void k_cg_update_p(int64_t n, int ncols, int64_t ld, const double* __restrict__ beta,
                              const double* __restrict__ z, double* __restrict__ p) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) p[c * ld + i] = z[c * ld + i] + beta[c] * p[c * ld + i];
}

__global__ void k_copy_cols(int64_t n, int ncols, int64_t lds, const double* __restrict__ s, int64_t ldd,
                            double* __restrict__ d) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) d[c * ldd + i] = s[c * lds + i];
}

// y[:,c] += sign * coef[c] * x[:,c]
__global__ void k_axpy_cols(int64_t n, int ncols, int64_t ld, const double* __restrict__ coef, double sign,
                            const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) y[c * ld + i] += sign * coef[c] * x[c * ld + i];
}

// ---- Gram products
// Gram matrices G = A^T [B1 B2] (A: n x k1, B1: n x k2a, B2: n x k2b, all
// column-major).  Bandwidth-bound: every block streams slabs of `rows`
// consecutive rows of all operands into LDS (coalesced, one wave per column),
// then each thread accumulates a TS x TS tile of G over a strided subset of
// the slab rows in registers.  Where the slab fits 12 values per thread (FP64
// operands), the next slab is loaded into registers while the current one is
// multiplied.  B may be FP32 (converted on load; exact).  Tiles x row-groups fill the 256 threads; the
// row groups are summed through LDS in a fixed order at the end and every
// block writes one partial G, reduced by k_gram_reduce in block order, so
// the result is deterministic.
constexpr int kGramThreads = 256;
constexpr int kGramMaxCols = 192;   // k1 + k2a + k2b

template <int TS, typename TB>
__global__ __launch_bounds__(kGramThreads) void k_gram(int64_t n, int rows, int k1, int64_t lda,
                                                       const double* __restrict__ A, int k2a, int64_t ldb1,
                                                       const TB* __restrict__ B1, int k2b, int64_t ldb2,
                                                       const TB* __restrict__ B2, double* __restrict__ part) {
    extern __shared__ double sm[];
    const int k2 = k2a + k2b;
    const int stride = rows + 1;            // padded column stride (bank spread)
    double* sa = sm;
    double* sb = sm + (size_t)k1 * stride;
    const int ti_n = (k1 + TS - 1) / TS, tj_n = (k2 + TS - 1) / TS;
    const int ntile = ti_n * tj_n;
    const int rg_n = max(1, min(rows, kGramThreads / ntile));
    const int t = threadIdx.x;
    const bool active = t < ntile * rg_n;
    const int tile = active ? t / rg_n : 0, rg = active ? t % rg_n : 0;
    const int ti = tile % ti_n, tj = tile / ti_n;
    int ca[TS], cb[TS];
#pragma unroll
    for (int u = 0; u < TS; ++u) {
        ca[u] = min(ti * TS + u, k1 - 1) * stride;   // clamped: extra rows/cols are discarded
        cb[u] = min(tj * TS + u, k2 - 1) * stride;
    }
    double acc[TS][TS];
#pragma unroll
    for (int u = 0; u < TS; ++u)
#pragma unroll
        for (int v = 0; v < TS; ++v) acc[u][v] = 0.0;
    const int64_t nslab = (n + rows - 1) / rows;
    // the next slab's share of this thread is loaded into registers while
    // the current one is multiplied (when (k1 + k2) rows <= PF x 256)
    constexpr int PF = TS == 4 ? 12 : 1;
    const int tot = (k1 + k2) * rows;
    const bool pf_ok = sizeof(TB) == 8 && tot <= PF * kGramThreads;
    double pv[PF];
    // rows divides the block size: a thread keeps its row r = t % rows and
    // takes columns c0, c0 + cstep, ...
    const int prow = t % rows, pc0 = t / rows, pcs = kGramThreads / rows;
    auto fetch = [&](int64_t sl) {
        const int64_t row = sl * rows + prow;
        const bool rok = sl < nslab && row < n;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int cc = pc0 + q * pcs;
            double v = 0.0;
            if (rok && cc < k1 + k2) {
                if (cc < k1) {
                    v = A[cc * lda + row];
                } else {
                    const TB* src = cc - k1 < k2a ? B1 + (cc - k1) * ldb1 : B2 + (cc - k1 - k2a) * ldb2;
                    v = (double)src[row];
                }
            }
            pv[q] = v;
        }
    };
    if (pf_ok) fetch(blockIdx.x);
    for (int64_t sl = blockIdx.x; sl < nslab; sl += gridDim.x) {
        const int64_t r0 = sl * rows;
        __syncthreads();
        if (pf_ok) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int cc = pc0 + q * pcs;
                if (cc < k1 + k2) sa[cc * stride + prow] = pv[q];   // sb follows sa
            }
            __syncthreads();
            fetch(sl + gridDim.x);
        } else {
            for (int e = t; e < k1 * rows; e += kGramThreads) {
                const int r = e % rows, cc = e / rows;
                const int64_t row = r0 + r;
                sa[cc * stride + r] = row < n ? A[cc * lda + row] : 0.0;
            }
            for (int e = t; e < k2 * rows; e += kGramThreads) {
                const int r = e % rows, cc = e / rows;
                const int64_t row = r0 + r;
                double v = 0.0;
                if (row < n) v = cc < k2a ? (double)B1[cc * ldb1 + row] : (double)B2[(cc - k2a) * ldb2 + row];
                sb[cc * stride + r] = v;
            }
            __syncthreads();
        }
        if (active) {
            for (int r = rg; r < rows; r += rg_n) {
                double av[TS], bv[TS];
#pragma unroll
                for (int u = 0; u < TS; ++u) {
                    av[u] = sa[ca[u] + r];
                    bv[u] = sb[cb[u] + r];
                }
#pragma unroll
                for (int u = 0; u < TS; ++u)
#pragma unroll
                    for (int v = 0; v < TS; ++v) acc[u][v] += av[u] * bv[v];
            }
        }
    }
    // sum the row groups of each tile entry, one entry position at a time
    const int nout = k1 * k2;
    double* red = sm;
#pragma unroll
    for (int u = 0; u < TS; ++u)
#pragma unroll
        for (int v = 0; v < TS; ++v) {
            __syncthreads();
            red[t] = active ? acc[u][v] : 0.0;
            __syncthreads();
            if (t < ntile) {
                const int tti = t % ti_n, ttj = t / ti_n;
                const int i = tti * TS + u, j = ttj * TS + v;
                double s = 0.0;
                for (int g = 0; g < rg_n; ++g) s += red[t * rg_n + g];
                if (i < k1 && j < k2) part[(int64_t)blockIdx.x * nout + i + (int64_t)k1 * j] = s;
            }
        }
}

// out[o] = sum_b part[b * nout + o], b ascending within each of 16 waves and
// the 16 wave sums added in wave order.
__global__ __launch_bounds__(1024) void k_gram_reduce(int nout, int nparts, const double* __restrict__ part,
                                                      double* __restrict__ out) {
    __shared__ double red[16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    double s0 = 0.0, s1 = 0.0;
    if (o < nout) {
        int b = w;
        for (; b + 16 < nparts; b += 32) {
            s0 += part[(int64_t)b * nout + o];
            s1 += part[(int64_t)(b + 16) * nout + o];
        }
        if (b < nparts) s0 += part[(int64_t)b * nout + o];
    }
    red[w][lane] = s0 + s1;
    __syncthreads();
    if (w == 0 && o < nout) {
        double s = 0.0;
        for (int q = 0; q < 16; ++q) s += red[q][lane];
        out[o] = s;
    }
}

// ---------------------------------------------------------------------------
// Row-wise block updates of block CG (thread per row; small coefficient
// matrices staged in LDS; rows are independent, so updates are in place).
constexpr int kBcgMax = 32;

// X += P alpha, R -= Q alpha (P, Q: n x sp; alpha: sp x nc), and the block
// partials of the column norms |R_q|^2.  MC bounds sp and nc.  The search
// block's orthonormalising transform is folded into alpha by the caller, so
// P and Q are only read.
template <int MC>
__global__ __launch_bounds__(256) void k_bcg_step(int64_t n, int sp, int nc, const double* __restrict__ alpha,
                                                  const double* __restrict__ P, const double* __restrict__ Q,
                                                  double* __restrict__ X, double* __restrict__ R,
                                                  double* __restrict__ rr_part) {
    __shared__ double sA[MC * MC];
    __shared__ double sred[4][MC];
    for (int e = threadIdx.x; e < sp * nc; e += blockDim.x) sA[e] = alpha[e];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const int64_t ii = ok ? i : 0;
    double v[MC];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < MC; ++a) v[a] = a < sp ? P[a * n + ii] : 0.0;
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        if (q >= nc) break;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < MC; ++a)
            if (a < sp) s += v[a] * sA[a + sp * q];
        if (ok) X[q * n + i] += s;
    }
#pragma unroll
    for (int a = 0; a < MC; ++a) v[a] = a < sp ? Q[a * n + ii] : 0.0;
    // R -= Q alpha with the wave sums of |R_q|^2 (fixed-order trees)
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        if (q >= nc) break;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < MC; ++a)
            if (a < sp) s += v[a] * sA[a + sp * q];
        double e = 0.0;
        if (ok) {
            const double nr = R[q * n + i] - s;
            R[q * n + i] = nr;
            e = nr * nr;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
        if (lane == 0) sred[wv][q] = e;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int q = threadIdx.x;
        rr_part[(int64_t)q * gridDim.x + blockIdx.x] = sred[0][q] + sred[1][q] + sred[2][q] + sred[3][q];
    }
}

// P <- Z + P beta  (P: n x sp in, n x nc out; beta sp x nc).
template <int MC, typename TZ>
__global__ __launch_bounds__(256) void k_bcg_dir(int64_t n, int sp, int nc, const double* __restrict__ beta,
                                                 const TZ* __restrict__ Z, double* __restrict__ P) {
    __shared__ double sB[MC * MC];
    for (int e = threadIdx.x; e < sp * nc; e += blockDim.x) sB[e] = beta[e];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[MC];
#pragma unroll
    for (int a = 0; a < MC; ++a) v[a] = a < sp ? P[a * n + i] : 0.0;
#pragma unroll
    for (int q = 0; q < MC; ++q) {
        if (q >= nc) break;
        double s = (double)Z[q * n + i];
#pragma unroll
        for (int a = 0; a < MC; ++a)
            if (a < sp) s += v[a] * sB[a + sp * q];
        P[q * n + i] = s;
    }
}

// Y (n x k2) = S (n x k1) C (k1 x k2, column-major), k1 <= 96, k2 <= 32;
// C staged in LDS; thread per (row, group of 8 output columns).
__global__ void k_gemm_small(int64_t n, int k1, int64_t lds, const double* __restrict__ S, int k2,
                             const double* __restrict__ C, int64_t ldy, double* __restrict__ Y) {
    __shared__ double sc[96 * 32];
    for (int t = threadIdx.x; t < k1 * k2; t += blockDim.x) sc[t] = C[t];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j0 = blockIdx.y * 8;
    const int nj = min(8, k2 - j0);
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0;
    for (int a = 0; a < k1; ++a) {
        const double sv = S[a * lds + i];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < nj) acc[j] += sv * sc[(j0 + j) * k1 + a];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < nj) Y[(j0 + j) * ldy + i] = acc[j];
}

// Y = alpha Y + [A1 A2] C  (A1: n x k1a, A2: n x k1b, C: (k1a + k1b) x k2
// column-major, k1a + k1b <= 96, k2 <= 32); Y must not overlap A1 or A2.
// Thread per (row, group of 8 output columns); alpha == 0 never reads Y.
__global__ void k_gemm_cat(int64_t n, int k1a, int64_t lda1, const double* __restrict__ A1, int k1b, int64_t lda2,
                           const double* __restrict__ A2, int k2, const double* __restrict__ C, double alpha,
                           int64_t ldy, double* __restrict__ Y) {
    __shared__ double sc[96 * 32];
    const int k1 = k1a + k1b;
    for (int t = threadIdx.x; t < k1 * k2; t += blockDim.x) sc[t] = C[t];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j0 = blockIdx.y * 8;
    const int nj = min(8, k2 - j0);
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0;
    for (int a = 0; a < k1; ++a) {
        const double sv = a < k1a ? A1[a * lda1 + i] : A2[(a - k1a) * lda2 + i];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < nj) acc[j] += sv * sc[(j0 + j) * k1 + a];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < nj) {
            const int64_t o = (j0 + j) * ldy + i;
            Y[o] = alpha == 0.0 ? acc[j] : alpha * Y[o] + acc[j];
        }
}

// V[:, 0:k2] = V[:, 0:k1] T in place (T: k1 x k2 column-major, both <= MC):
// every thread reads its whole row before writing it.
template <int MC>
__global__ __launch_bounds__(256) void k_xform_inplace(int64_t n, int k1, int k2, const double* __restrict__ Tm,
                                                       int64_t ld, double* __restrict__ V) {
    __shared__ double sT[MC * MC];
    for (int e = threadIdx.x; e < k1 * k2; e += blockDim.x) sT[e] = Tm[e];
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[MC];
#pragma unroll
    for (int a = 0; a < MC; ++a) v[a] = a < k1 ? V[a * ld + i] : 0.0;
#pragma unroll
    for (int j = 0; j < MC; ++j) {
        if (j >= k2) break;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < MC; ++a)
            if (a < k1) s += v[a] * sT[a + k1 * j];
        V[j * ld + i] = s;
    }
}

// R = AX - KX diag(mu)
__global__ void k_residual_block(int64_t n, int ncols, int64_t ld, const double* __restrict__ AX,
                                 const double* __restrict__ KX, const double* __restrict__ mu, double* __restrict__ R) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) R[c * ld + i] = AX[c * ld + i] - mu[c] * KX[c * ld + i];
}

// Counter-based uniform(-1, 1) from splitmix64 of (seed, column, row); zero at fixed DOFs.
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_random_fill(int64_t n, int ncols, int64_t ld, uint64_t seed, const uint8_t* __restrict__ nmask,
                              int dim, double* __restrict__ X) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fixed = (nmask[i / dim] >> (i % dim)) & 1;
    for (int c = 0; c < ncols; ++c) {
        const uint64_t h = splitmix64(seed ^ splitmix64((uint64_t)c * 0x100000001B3ull + (uint64_t)i));
        const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
        X[c * ld + i] = fixed ? 0.0 : 2.0 * u - 1.0;
    }
}

// Zero the Dirichlet entries of a block (restores the free-subspace invariant).
__global__ void k_mask_fixed(int64_t n, int ncols, int64_t ld, const uint8_t* __restrict__ nmask, int dim,
                             double* __restrict__ X) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!((nmask[i / dim] >> (i % dim)) & 1)) return;
    for (int c = 0; c < ncols; ++c) X[c * ld + i] = 0.0;
}

// Column-wise argmax |x| (ties: lowest index) -> signed value of that entry.
__global__ void k_absmax_part(int64_t n, int64_t ld, const double* __restrict__ X, double* __restrict__ pval,
                              int64_t* __restrict__ pidx) {
    __shared__ double sv[kBlock];
    __shared__ int64_t si[kBlock];
    const int col = blockIdx.y;
    double best = -1.0, bval = 0.0;
    int64_t bidx = INT64_MAX;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = X[col * ld + i];
        if (fabs(v) > best) {   // strictly greater keeps the lowest index on ties
            best = fabs(v);
            bval = v;
            bidx = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bidx;
    __shared__ double sval[kBlock];
    sval[threadIdx.x] = bval;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const int o = threadIdx.x + s;
            if (sv[o] > sv[threadIdx.x] || (sv[o] == sv[threadIdx.x] && si[o] < si[threadIdx.x])) {
                sv[threadIdx.x] = sv[o];
                si[threadIdx.x] = si[o];
                sval[threadIdx.x] = sval[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pval[(int64_t)col * gridDim.x + blockIdx.x] = sval[0];
        pidx[(int64_t)col * gridDim.x + blockIdx.x] = sv[0] >= 0.0 ? si[0] : INT64_MAX;
    }
}

__global__ void k_absmax_sum(int ncols, int nparts, const double* __restrict__ pval, const int64_t* __restrict__ pidx,
                             double* __restrict__ out) {
    const int col = threadIdx.x;
    if (col >= ncols) return;
    double best = -1.0, val = 0.0;
    int64_t bi = INT64_MAX;
    for (int b = 0; b < nparts; ++b) {
        const double v = pval[(int64_t)col * nparts + b];
        const int64_t ix = pidx[(int64_t)col * nparts + b];
        if (fabs(v) > best || (fabs(v) == best && ix < bi)) {
            best = fabs(v);
            val = v;
            bi = ix;
        }
    }
    out[col] = val;
}

__global__ void k_infnorm_part(int64_t n, int64_t ld, const double* __restrict__ X, double* __restrict__ part) {
    __shared__ double sh[16];
    const int col = blockIdx.y;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s = fmax(s, fabs(X[col * ld + i]));
    s = bmax(s, sh);
    if (threadIdx.x == 0) part[col * gridDim.x + blockIdx.x] = s;
}

__global__ void k_max_parts(int nparts, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[16];
    const int col = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s = fmax(s, part[col * nparts + i]);
    s = bmax(s, sh);
    if (threadIdx.x == 0) out[col] = s;
}

__global__ void k_scale_cols(int64_t n, int ncols, int64_t ld, const double* __restrict__ s, double* __restrict__ X) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < ncols; ++c) X[c * ld + i] *= s[c];
}

// ---- launchers

template <typename T>
void launch_jacobi0(int64_t n, int ncols, int64_t ld, const T* dinv, T omega, const T* r, T* z, hipStream_t st) {
    hipLaunchKernelGGL((k_jacobi0<T>), dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, dinv, omega, r, z);
}
template void launch_jacobi0<double>(int64_t, int, int64_t, const double*, double, const double*, double*, hipStream_t);
template void launch_jacobi0<float>(int64_t, int, int64_t, const float*, float, const float*, float*, hipStream_t);

void launch_d2f_jacobi0(int64_t n, int ncols, int64_t ld, const double* a, const float* dinv, float omega, float* b,
                        float* z, hipStream_t st) {
    hipLaunchKernelGGL(k_d2f_jacobi0, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, a, dinv, omega, b, z);
}
void launch_d2f(int64_t n, int ncols, int64_t ld, const double* a, float* b, hipStream_t st) {
    hipLaunchKernelGGL(k_d2f, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, a, b);
}
void launch_f2d(int64_t n, int ncols, int64_t ld, const float* a, double* b, hipStream_t st) {
    hipLaunchKernelGGL(k_f2d, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, a, b);
}
void launch_dot_part(int64_t n, int ncols, int64_t lda, const double* a, int64_t ldb, const double* b, int nparts,
                     double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_part, dim3(nparts, ncols), dim3(kBlock), 0, st, n, lda, a, ldb, b, part);
}
void launch_sum_parts(int ncols, int64_t nparts, const double* part, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_parts, dim3(ncols), dim3(kBlock), 0, st, nparts, part, out);
}
void launch_cg_alpha(int ncols, const double* rz, const double* pq, const int* active, double* alpha, int* flags,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, rz, pq, active, alpha, flags);
}
void launch_cg_check(int ncols, const double* rr, const double* thr, int* active, int* iters, int* flags,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, rr, thr, active, iters,
                       flags);
}
// out[a + k2 q] = sign G[q + k1 a] (a < k2, q < k1): the transposed Gram
// block, scaled, as a column-major coefficient matrix for k_gemm_cat.
__global__ void k_gram_transpose(int k1, int k2, double sign, const double* __restrict__ G,
                                 double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k1 * k2) return;
    const int a = t % k2, q = t / k2;
    out[a + k2 * q] = sign * G[q + k1 * a];
}
void launch_gram_transpose(int k1, int k2, double sign, const double* G, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_gram_transpose, dim3((k1 * k2 + 255) / 256), dim3(256), 0, st, k1, k2, sign, G, out);
}
void launch_cg_beta(int ncols, const double* rz_new, double* rz, const int* active, double* beta, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, rz_new, rz, active, beta);
}
void launch_cg_beta_flex(int ncols, const double* rz_new, const double* rz_cross, double* rz, const int* active,
                         double* beta, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_beta_flex, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, rz_new, rz_cross, rz,
                       active, beta);
}
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(nb1(n)), dim3(kBlock), 0, st, n, a, x, b, y);
}
void launch_rsqrt(int ncols, const double* in, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_rsqrt, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, in, out);
}
void launch_cg_update_xr(int64_t n, int ncols, int64_t ld, const double* alpha, const double* p, const double* q,
                         double* x, double* r, int nparts, double* rr_part, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_xr, dim3(nparts, ncols), dim3(kBlock), 0, st, n, ld, alpha, p, q, x, r, rr_part);
}
void launch_cg_update_p(int64_t n, int ncols, int64_t ld, const double* beta, const double* z, double* p,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_cg_update_p, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, beta, z, p);
}
void launch_copy_cols(int64_t n, int ncols, int64_t lds, const double* s, int64_t ldd, double* d, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_cols, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, lds, s, ldd, d);
}
void launch_axpy_cols(int64_t n, int ncols, int64_t ld, const double* coef, double sign, const double* x, double* y,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_cols, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, coef, sign, x, y);
}
int gram_parts(int64_t n, int k1, int k2) {
    const int rows = k1 + k2 > 120 ? 32 : 64;
    const int64_t nslab = (n + rows - 1) / rows;
    return (int)std::max<int64_t>(1, std::min<int64_t>(nslab, 1024));
}

template <typename TB>
static int launch_gram_t(int64_t n, int k1, int64_t lda, const double* A, int k2a, int64_t ldb1, const TB* B1, int k2b,
                         int64_t ldb2, const TB* B2, int nparts, double* part, double* out, hipStream_t st) {
    const int k2 = k2a + k2b;
    if (k1 < 1 || k2 < 1 || k1 + k2 > kGramMaxCols) return -1;
    const int rows = k1 + k2 > 120 ? 32 : 64;
    const size_t lds = std::max<size_t>((size_t)(k1 + k2) * (rows + 1), kGramThreads) * sizeof(double);
    const int t4 = ((k1 + 3) / 4) * ((k2 + 3) / 4);
    if (t4 <= kGramThreads)
        hipLaunchKernelGGL((k_gram<4, TB>), dim3(nparts), dim3(kGramThreads), lds, st, n, rows, k1, lda, A, k2a, ldb1,
                           B1, k2b, ldb2, B2, part);
    else
        hipLaunchKernelGGL((k_gram<6, TB>), dim3(nparts), dim3(kGramThreads), lds, st, n, rows, k1, lda, A, k2a, ldb1,
                           B1, k2b, ldb2, B2, part);
    const int nout = k1 * k2;
    hipLaunchKernelGGL(k_gram_reduce, dim3((nout + 63) / 64), dim3(1024), 0, st, nout, nparts, part, out);
    return 0;
}
int launch_gram(int64_t n, int k1, int64_t lda, const double* A, int k2a, int64_t ldb1, const double* B1, int k2b,
                int64_t ldb2, const double* B2, int nparts, double* part, double* out, hipStream_t st) {
    return launch_gram_t<double>(n, k1, lda, A, k2a, ldb1, B1, k2b, ldb2, B2, nparts, part, out, st);
}
int launch_gram_f32b(int64_t n, int k1, int64_t lda, const double* A, int k2, int64_t ldb, const float* B, int nparts,
                     double* part, double* out, hipStream_t st) {
    return launch_gram_t<float>(n, k1, lda, A, k2, ldb, B, 0, 0, (const float*)nullptr, nparts, part, out, st);
}

void launch_bcg_step(int64_t n, int sp, int nc, const double* alpha, const double* P, const double* Q, double* X,
                     double* R, double* rr_part, hipStream_t st) {
    const int mc = std::max(sp, nc);
#define MLB_BS(M) hipLaunchKernelGGL(k_bcg_step<M>, dim3(nb1(n)), dim3(256), 0, st, n, sp, nc, alpha, P, Q, X, R, rr_part)
    if (mc <= 4) MLB_BS(4);
    else if (mc <= 8) MLB_BS(8);
    else if (mc <= 12) MLB_BS(12);
    else if (mc <= 16) MLB_BS(16);
    else if (mc <= 24) MLB_BS(24);
    else MLB_BS(32);
#undef MLB_BS
}

int bcg_step_parts(int64_t n) { return nb1(n); }

template <typename TZ>
static void launch_bcg_dir_t(int64_t n, int sp, int nc, const double* beta, const TZ* Z, double* P, hipStream_t st) {
    const int mc = std::max(sp, nc);
#define MLB_BD(M) hipLaunchKernelGGL((k_bcg_dir<M, TZ>), dim3(nb1(n)), dim3(256), 0, st, n, sp, nc, beta, Z, P)
    if (mc <= 4) MLB_BD(4);
    else if (mc <= 8) MLB_BD(8);
    else if (mc <= 12) MLB_BD(12);
    else if (mc <= 16) MLB_BD(16);
    else if (mc <= 24) MLB_BD(24);
    else MLB_BD(32);
#undef MLB_BD
}
void launch_bcg_dir(int64_t n, int sp, int nc, const double* beta, const double* Z, double* P, hipStream_t st) {
    launch_bcg_dir_t<double>(n, sp, nc, beta, Z, P, st);
}
void launch_bcg_dir(int64_t n, int sp, int nc, const double* beta, const float* Z, double* P, hipStream_t st) {
    launch_bcg_dir_t<float>(n, sp, nc, beta, Z, P, st);
}

void launch_gemm_small(int64_t n, int k1, int64_t lds, const double* S, int k2, const double* C, int64_t ldy,
                       double* Y, hipStream_t st) {
    hipLaunchKernelGGL(k_gemm_small, dim3(nb1(n), (k2 + 7) / 8), dim3(kBlock), 0, st, n, k1, lds, S, k2, C, ldy, Y);
}
void launch_gemm_cat(int64_t n, int k1a, int64_t lda1, const double* A1, int k1b, int64_t lda2, const double* A2,
                     int k2, const double* C, double alpha, int64_t ldy, double* Y, hipStream_t st) {
    hipLaunchKernelGGL(k_gemm_cat, dim3(nb1(n), (k2 + 7) / 8), dim3(kBlock), 0, st, n, k1a, lda1, A1, k1b, lda2, A2,
                       k2, C, alpha, ldy, Y);
}
void launch_xform_inplace(int64_t n, int k1, int k2, const double* T, int64_t ld, double* V, hipStream_t st) {
    const int mc = std::max(k1, k2);
#define MLB_XF(M) hipLaunchKernelGGL(k_xform_inplace<M>, dim3(nb1(n)), dim3(256), 0, st, n, k1, k2, T, ld, V)
    if (mc <= 8) MLB_XF(8);
    else if (mc <= 16) MLB_XF(16);
    else if (mc <= 24) MLB_XF(24);
    else MLB_XF(32);
#undef MLB_XF
}
void launch_residual_block(int64_t n, int ncols, int64_t ld, const double* AX, const double* KX, const double* mu,
                           double* R, hipStream_t st) {
    hipLaunchKernelGGL(k_residual_block, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, AX, KX, mu, R);
}
void launch_random_fill(int64_t n, int ncols, int64_t ld, uint64_t seed, const uint8_t* nmask, int dim, double* X,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_random_fill, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, seed, nmask, dim, X);
}
void launch_mask_fixed(int64_t n, int ncols, int64_t ld, const uint8_t* nmask, int dim, double* X, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_fixed, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, nmask, dim, X);
}
void launch_absmax_part(int64_t n, int ncols, int64_t ld, const double* X, int nparts, double* pval, int64_t* pidx,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_absmax_part, dim3(nparts, ncols), dim3(kBlock), 0, st, n, ld, X, pval, pidx);
}
void launch_absmax_sum(int ncols, int nparts, const double* pval, const int64_t* pidx, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_absmax_sum, dim3(1), dim3(64 * ((ncols + 63) / 64)), 0, st, ncols, nparts, pval, pidx, out);
}
void launch_infnorm_part(int64_t n, int ncols, int64_t ld, const double* X, int nparts, double* part,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_infnorm_part, dim3(nparts, ncols), dim3(kBlock), 0, st, n, ld, X, part);
}
void launch_max_parts(int ncols, int nparts, const double* part, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_max_parts, dim3(ncols), dim3(kBlock), 0, st, nparts, part, out);
}
void launch_scale_cols(int64_t n, int ncols, int64_t ld, const double* s, double* X, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols, dim3(nb1(n)), dim3(kBlock), 0, st, n, ncols, ld, s, X);
}

}  // namespace mlb
