// Dense FP64 linear algebra of the coarsest multigrid level on the matrix
// cores: the explicit inverse of the coarsest Galerkin matrix (blocked
// Gauss-Jordan, whose rank-b updates are FP64 MFMA GEMMs) and the coarsest
// solve z = A^-1 r as a split-K MFMA product that reads the inverse once
// for up to 32 columns.
//
// Matrix-core instruction: v_mfma_f64_16x16x4f64, D(16x16) += A(16x4) B(4x16)
// over a 64-lane wave.  Operand layout (lane l, 0..63):
//   A: element (l % 16, l / 16)            one double per lane
//   B: element (l / 16, l % 16)            one double per lane
//   D: element (l / 16 + 4 r, l % 16)      r = 0..3, four doubles per lane
#include "kernels.h"

namespace mlb {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16x16x4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C = alpha A B + beta C, all row-major FP64; M, N multiples of 64, K a
// multiple of 16.  One 256-thread block per 64 x 64 tile of C (wave w owns
// the 32 x 32 quarter (w / 2, w % 2), four 16 x 16 MFMA tiles); A and B
// stream through LDS in 16-deep slices.  beta == 0 never reads C.
constexpr int kGT = 64;   // tile edge
constexpr int kGK = 16;   // K slice
// Tile (skip_r, skip_c) of C, if any, is left untouched.
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                  int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
                                                  double* __restrict__ C, int64_t ldc, int skip_r, int skip_c) {
    __shared__ double As[kGT * kGK];   // [row][k]
    __shared__ double Bs[kGK * kGT];   // [k][col]
    if ((int)blockIdx.y == skip_r && (int)blockIdx.x == skip_c) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * kGT, c0 = (int64_t)blockIdx.x * kGT;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    // C is read before the products, so its loads overlap them (the rank-64
    // updates of the inverse are bound by streaming C in and out)
    v4d cv[2][2];
    if (beta != 0.0) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    cv[a][b][r] = C[(r0 + wr + 16 * a + (lane >> 4) + 4 * r) * ldc + c0 + wc + 16 * b + (lane & 15)];
    }
    for (int k0 = 0; k0 < K; k0 += kGK) {
        // 1024 entries of each slice, 4 per thread, coalesced along rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            const int ar = e / kGK, ak = e % kGK;          // A slice: 64 rows x 16
            As[e] = A[(r0 + ar) * lda + k0 + ak];
            const int bk = e / kGT, bc = e % kGT;          // B slice: 16 x 64 cols
            Bs[e] = B[(int64_t)(k0 + bk) * ldb + c0 + bc];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 4) {
            const int kk = ks + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[(wr + 16 * a + (lane & 15)) * kGK + kk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kk * kGT + wc + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16x16x4(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + wr + 16 * a + (lane >> 4) + 4 * r;
                const int64_t col = c0 + wc + 16 * b + (lane & 15);
                C[row * ldc + col] = beta == 0.0 ? alpha * acc[a][b][r] : fma(alpha, acc[a][b][r], beta * cv[a][b][r]);
            }
}

// Inverse of the 64 x 64 diagonal block at (k0, k0) of A (row-major,
// leading dimension ld) into P (64 x 64, row-major) by scalar Gauss-Jordan;
// the block is SPD (a Schur complement of an SPD matrix), so no pivoting.
// One block of 256 threads; thread t keeps column j = t % 64 of rows
// t / 64 + 4 r (r = 0..15) in registers.  Step k: the owners publish row k
// and column k to LDS (double-buffered by the parity of k, so one barrier
// per step), then every thread updates its 16 entries; within a wave the
// rows, hence the column-k entries read, are the same (LDS broadcasts).
__global__ __launch_bounds__(256) void k_gj_diag(const double* __restrict__ A, int64_t ld, int64_t k0,
                                                 double* __restrict__ P) {
    __shared__ double rowk[2][kGT], colk[2][kGT];
    const int tid = threadIdx.x;
    const int j = tid & (kGT - 1), i0 = tid >> 6;   // rows i0 + 4 r
    double v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = A[(k0 + i0 + 4 * r) * ld + k0 + j];
    for (int k = 0; k < kGT; ++k) {
        const int b = k & 1;
        // row k lives in the threads with i0 == k % 4 (r = k / 4), column k
        // in the threads with j == k
        if (i0 == (k & 3)) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (r == (k >> 2)) rowk[b][j] = v[r];
        }
        if (j == k) {
#pragma unroll
            for (int r = 0; r < 16; ++r) colk[b][i0 + 4 * r] = v[r];
        }
        __syncthreads();
        const double pinv = 1.0 / rowk[b][k];
        const double rj = rowk[b][j] * pinv;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + 4 * r;
            const double ci = colk[b][i];
            double w;
            if (i == k) w = j == k ? pinv : rj;
            else w = j == k ? -ci * pinv : v[r] - ci * rj;
            v[r] = w;
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) P[(i0 + 4 * r) * kGT + j] = v[r];
}

// dst (rows x cols, leading dimension ldd) = src (leading dimension lds)
__global__ void k_copy_block(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds,
                             double* __restrict__ dst, int64_t ldd) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    const int64_t i = t / cols, j = t % cols;
    dst[i * ldd + j] = src[i * lds + j];
}

// A = (A + A^T) / 2 for an N x N row-major matrix (each pair once)
__global__ void k_symmetrize(int64_t N, double* __restrict__ A) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t / N, j = t % N;
    if (j <= i) return;
    const double v = 0.5 * (A[i * N + j] + A[j * N + i]);
    A[i * N + j] = v;
    A[j * N + i] = v;
}

// Xt[k * 32 + c] = x[c * ld + k] as FP64 for k < n and c < nc, zero for
// the padding rows n <= k < N and columns nc <= c < 32 (k-major, so that the
// MFMA operand loads below read four full 128-byte lines)
template <typename T>
__global__ void k_coarse_stage(int64_t n, int64_t N, int nc, int64_t ld, const T* __restrict__ x,
                               double* __restrict__ Xt) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * 32) return;
    const int64_t k = t >> 5;
    const int c = (int)(t & 31);
    Xt[t] = (k < n && c < nc) ? (double)x[c * ld + k] : 0.0;
}

// The symmetric inverse is read from its lower triangle only, stored as
// 16 x 16 tiles: tile (R, C), R >= C, at (R (R + 1) / 2 + C) 256, each tile
// as four slabs of four columns (element (r, c) at (c / 4) 64 + 4 r + c % 4),
// so that a K step reads a tile below the diagonal as four 128-byte runs and
// one above it (the transpose of the stored tile) as one 512-byte run.  Half
// the bytes of the full matrix per coarsest solve.
__global__ void k_pack_lower(int64_t N, const double* __restrict__ A, double* __restrict__ Apk) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t row = t / N, col = t % N;
    const int64_t R = row >> 4, C = col >> 4;
    if (R < C) return;
    Apk[(R * (R + 1) / 2 + C) * 256 + ((col & 15) >> 2) * 64 + (row & 15) * 4 + (col & 3)] = A[t];
}

int64_t packed_lower_doubles(int64_t N) {
    const int64_t T = N / 16;
    return T * (T + 1) / 2 * 256;
}

// Partial products of Z = A X with A symmetric N x N (packed lower tiles)
// and X staged k-major in Xt (N x 32), computed as Z^T = X^T A: wave (tile,
// split) forms the 16 (or 32) columns x 16 rows of Z^T for rows
// j0 .. j0 + 15 over its share of the K range.  A K-tile at or below the
// diagonal is read as stored, one above it as the transpose of the stored
// tile (J, K); the loop issues the loads of four K steps before their
// products.  part[(split * 32 + c) * N + j].
template <int NCT>
__global__ __launch_bounds__(256) void k_coarse_part(int64_t N, const double* __restrict__ A,
                                                     const double* __restrict__ Xt, int nsplit,
                                                     double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ntiles = N / 16;
    if (wid >= ntiles * nsplit) return;
    const int64_t tile = wid / nsplit;
    const int split = (int)(wid % nsplit);
    const int64_t kchunk = (N / 16 + nsplit - 1) / nsplit * 16;
    const int64_t kb = split * kchunk, ke = min(N, kb + kchunk);
    const int64_t j0 = tile * 16;
    const int cl = lane & 15, kl = lane >> 4;
    v4d acc[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t J = tile;
    for (int64_t k = kb; k < ke; k += 16) {   // N and kchunk are multiples of 16
        const int64_t K = k >> 4;
        const bool below = K >= J;   // wave-uniform
        const double* At = A + (below ? K * (K + 1) / 2 + J : J * (J + 1) / 2 + K) * 256;
        double b[4], a[4][NCT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t kr = k + 4 * u + kl;
            // element (kr, j0 + cl): stored (4 u + kl, cl) below, (cl, 4 u + kl) above
            b[u] = At[below ? (cl >> 2) * 64 + (4 * u + kl) * 4 + (cl & 3) : u * 64 + cl * 4 + kl];
#pragma unroll
            for (int t = 0; t < NCT; ++t) a[u][t] = Xt[kr * 32 + 16 * t + cl];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NCT; ++t) acc[t] = mfma16x16x4(a[u][t], b[u], acc[t]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = kl + 4 * r;
#pragma unroll
        for (int t = 0; t < NCT; ++t) part[((int64_t)split * 32 + c + 16 * t) * N + j0 + cl] = acc[t][r];
    }
}

// z[c * ld + j] = sum over splits of the partials (fixed order), j < n, c < nc
template <typename T>
__global__ void k_coarse_sum(int64_t n, int64_t N, int nc, int64_t ld, int nsplit, const double* __restrict__ part,
                             T* __restrict__ z) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * nc) return;
    const int64_t c = t / n, j = t % n;
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += part[((int64_t)q * 32 + c) * N + j];
    z[c * ld + j] = (T)s;
}

static inline unsigned nbk(int64_t n) { return (unsigned)((n + 255) / 256); }

int coarse_pad(int64_t n) { return (int)((n + kGT - 1) / kGT * kGT); }

int coarse_splits(int64_t N) {
    // enough waves to cover the chip (>= ~2048) with >= 64 K steps of 4 per wave
    const int64_t tiles = N / 16;
    int s = 1;
    while (tiles * s < 2048 && N / (4 * (s * 2)) >= 64) s *= 2;
    return s;
}

int64_t coarse_stage_doubles(int64_t N) { return N * 32; }

void launch_gemm_f64(int M, int N, int K, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double beta, double* C, int64_t ldc, hipStream_t st, int skip_r, int skip_c) {
    hipLaunchKernelGGL(k_gemm_f64, dim3(N / kGT, M / kGT), dim3(256), 0, st, M, N, K, alpha, A, lda, B, ldb, beta, C,
                       ldc, skip_r, skip_c);
}

// In-place inverse of the N x N SPD matrix A (N a multiple of 64; pad with an
// identity block) by 64-wide panels: P = A_KK^-1, R = P A_K:, C = A_:K,
// A -= C R, A_:K = -C P, A_K: = R, A_KK = P; then A = (A + A^T) / 2.
// Work: P (64 x 64), R (64 x N), C (N x 64), all device.
// Panel k: P_k = inverse of the diagonal block (k, k); R = P_k A[k rows];
// A -= A[:, k cols] R; A[:, k cols] = -A[:, k cols] P_k; A[k rows] = R;
// block (k, k) = P_k.  With a second stream the next diagonal block is
// updated first and inverted there while the rest of the rank-64 update runs
// (P double-buffered: 2 x 64 x 64); the results are the same either way.
void launch_block_inverse(int64_t N, double* A, double* P, double* R, double* Cp, hipStream_t st, hipStream_t st2,
                          hipEvent_t ev_a, hipEvent_t ev_b) {
    const int n = (int)N;
    const int64_t nk = N / kGT;
    auto pbuf = [&](int64_t kb) { return P + (kb & 1) * kGT * kGT; };
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, st, A, N, (int64_t)0, pbuf(0));
    for (int64_t kb = 0; kb < nk; ++kb) {
        const int64_t k0 = kb * kGT, k1 = k0 + kGT;
        double* Pk = pbuf(kb);
        const bool more = kb + 1 < nk, ahead = more && st2;
        launch_gemm_f64(kGT, n, kGT, 1.0, Pk, kGT, A + k0 * N, N, 0.0, R, N, st);
        hipLaunchKernelGGL(k_copy_block, dim3(nbk(N * kGT)), dim3(256), 0, st, N, (int64_t)kGT, A + k0, N, Cp,
                           (int64_t)kGT);
        if (ahead) {
            // block (k + 1, k + 1) gets its update now (the same tile
            // product as in the full update) and is inverted on st2
            launch_gemm_f64(kGT, kGT, kGT, -1.0, Cp + k1 * kGT, kGT, R + k1, N, 1.0, A + k1 * N + k1, N, st);
            (void)hipEventRecord(ev_a, st);
            (void)hipStreamWaitEvent(st2, ev_a, 0);
            hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, st2, A, N, k1, pbuf(kb + 1));
            (void)hipEventRecord(ev_b, st2);
            launch_gemm_f64(n, n, kGT, -1.0, Cp, kGT, R, N, 1.0, A, N, st, (int)(kb + 1), (int)(kb + 1));
        } else {
            launch_gemm_f64(n, n, kGT, -1.0, Cp, kGT, R, N, 1.0, A, N, st);
        }
        launch_gemm_f64(n, kGT, kGT, -1.0, Cp, kGT, Pk, kGT, 0.0, A + k0, N, st);
        hipLaunchKernelGGL(k_copy_block, dim3(nbk(kGT * N)), dim3(256), 0, st, (int64_t)kGT, N, R, N, A + k0 * N, N);
        hipLaunchKernelGGL(k_copy_block, dim3(nbk(kGT * kGT)), dim3(256), 0, st, (int64_t)kGT, (int64_t)kGT, Pk,
                           (int64_t)kGT, A + k0 * N + k0, N);
        if (ahead)
            (void)hipStreamWaitEvent(st, ev_b, 0);
        else if (more)
            hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, st, A, N, k1, pbuf(kb + 1));
    }
    hipLaunchKernelGGL(k_symmetrize, dim3(nbk(N * N)), dim3(256), 0, st, N, A);
}

// part holds nsplit * 32 * N doubles followed by the N x 32 staging block
void launch_pack_lower(int64_t N, const double* A, double* Apk, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_lower, dim3(nbk(N * N)), dim3(256), 0, st, N, A, Apk);
}

template <typename T>
void launch_coarse_solve(int64_t n, int64_t N, int nc, int64_t ld, const double* A, const T* x, T* z, int nsplit,
                         double* part, hipStream_t st) {
    double* Xt = part + (int64_t)nsplit * 32 * N;
    hipLaunchKernelGGL(k_coarse_stage<T>, dim3(nbk(N * 32)), dim3(256), 0, st, n, N, nc, ld, x, Xt);
    const int64_t waves = N / 16 * nsplit;
    if (nc > 16)
        hipLaunchKernelGGL(k_coarse_part<2>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, N, A, Xt, nsplit,
                           part);
    else
        hipLaunchKernelGGL(k_coarse_part<1>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, N, A, Xt, nsplit,
                           part);
    hipLaunchKernelGGL(k_coarse_sum<T>, dim3(nbk(n * nc)), dim3(256), 0, st, n, N, nc, ld, nsplit, part, z);
}
template void launch_coarse_solve<double>(int64_t, int64_t, int, int64_t, const double*, const double*, double*, int,
                                          double*, hipStream_t);
template void launch_coarse_solve<float>(int64_t, int64_t, int, int64_t, const double*, const float*, float*, int,
                                         double*, hipStream_t);

}  // namespace mlb
