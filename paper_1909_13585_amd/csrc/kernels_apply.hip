// Operator applies, smoother epilogues, diagonals and grid transfers.
//
// All applies are node-centric gathers: one thread owns one grid node and
// sums the contributions of the (up to) 2^dim elements around it, so no
// atomics are needed and results are bitwise repeatable.  Vectors are
// interleaved (dof = dim*node + c) and blocks are column-major with leading
// dimension `ld`.  Dirichlet DOFs: K has identity rows/columns, G zero ones
// (the masked operators of the fine problem and of every Galerkin level).
#include "kernels.h"

namespace mlb {

// ---------------------------------------------------------------------------
// small helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block; valid in linear thread 0.  Uses fixed-order trees.
__device__ inline double block_sum(double v, double* sh) {
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (wid == 0) {
        r = lane < nw ? sh[lane] : 0.0;
        r = wave_sum(r);
    }
    return r;
}

template <int DIM>
struct Nb {
    static constexpr int NN = 1 << DIM;
    static constexpr int ND = DIM;
    static constexpr int NDE = DIM << DIM;
    static constexpr int NB = DIM == 2 ? 9 : 27;
    // neighbour slot of offset (dx,dy,dz) in {-1,0,1}
    static __device__ __host__ constexpr int slot(int dx, int dy, int dz) {
        return (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
    }
};

// Loads the 3^dim neighbourhood of node (i,j,k): validity, node masks, indices.
template <int DIM>
__device__ inline void neighbourhood(const Geo& g, int i, int j, int k, const uint8_t* __restrict__ nmask,
                                     int64_t* idx, uint8_t* msk) {
    using N = Nb<DIM>;
#pragma unroll
    for (int t = 0; t < N::NB; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
        const int ii = i + dx, jj = j + dy, kk = k + dz;
        const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny && kk >= 0 && kk < g.nnz;
        const int64_t n = ok ? ii + (int64_t)g.nnx * (jj + (int64_t)g.nny * kk) : 0;
        idx[t] = n;
        msk[t] = ok ? nmask[n] : (uint8_t)0xff;   // outside: treat as fixed (value 0)
    }
}

template <int DIM>
__device__ inline int64_t elem_of_slot(const Geo& g, int i, int j, int k, int s, bool& ok) {
    const int ox = s & 1, oy = (s >> 1) & 1, oz = (s >> 2) & 1;
    const int ei = i - 1 + ox, ej = j - 1 + oy, ek = DIM == 3 ? k - 1 + oz : 0;
    ok = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && (DIM == 2 || (ek >= 0 && ek < g.nz));
    return ok ? ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek) : 0;
}

template <typename T, int MODE>
__device__ inline T epilogue(T ax, T xown, T rr, T di, T omega) {
    if (MODE == kModeY) return ax;
    if (MODE == kModeResidual) return rr - ax;
    return xown + omega * di * (rr - ax);
}

// ---------------------------------------------------------------------------
// Level-1 stiffness apply, matrix free: y = sum_e E_e P_e^T K0 P_e x.
// K0 is staged in LDS (uniform-address broadcast reads).  The 3^dim
// neighbours are visited once each; every neighbour feeds the element slots
// that contain it.  Columns are processed in chunks of CB so that each K0
// entry is read once per chunk.

template <int DIM, typename T, int MODE, bool DOT, int CB>
__global__ __launch_bounds__(256) void k_apply_fine(Geo g, const T* __restrict__ E,
                                                    const uint8_t* __restrict__ nmask,
                                                    const T* __restrict__ K0, int ncols, int64_t ld,
                                                    const T* __restrict__ x, T* __restrict__ y,
                                                    const T* __restrict__ r, const T* __restrict__ dinv,
                                                    T omega, double* __restrict__ part) {
    using N = Nb<DIM>;
    __shared__ T k0s[N::NDE * N::NDE];
    __shared__ double sh[16];
    {
        const int tid = threadIdx.x + blockDim.x * threadIdx.y;
        for (int q = tid; q < N::NDE * N::NDE; q += blockDim.x * blockDim.y) k0s[q] = K0[q];
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? blockIdx.z : 0;
    const bool active = i < g.nnx && j < g.nny;
    const int ic = active ? i : 0, jc = active ? j : 0;
    const int64_t node = ic + (int64_t)g.nnx * (jc + (int64_t)g.nny * k);
    T Ee[N::NN];
#pragma unroll
    for (int s = 0; s < N::NN; ++s) {
        bool ok;
        const int64_t e = elem_of_slot<DIM>(g, ic, jc, k, s, ok);
        Ee[s] = ok ? E[e] : T(0);
    }
    const uint8_t own = nmask[node];
    const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    const int64_t nblk = (int64_t)gridDim.x * gridDim.y * gridDim.z;
    for (int c0 = 0; c0 < ncols; c0 += CB) {
        T tmp[N::NN][CB][N::ND];
#pragma unroll
        for (int s = 0; s < N::NN; ++s)
#pragma unroll
            for (int q = 0; q < CB; ++q)
#pragma unroll
                for (int c = 0; c < N::ND; ++c) tmp[s][q][c] = T(0);
        // runtime loop over neighbours (wave-uniform), compile-time slots
#pragma unroll 1
        for (int t = 0; t < N::NB; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
            const int ii = ic + dx, jj = jc + dy, kk = k + dz;
            const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny && kk >= 0 && kk < g.nnz;
            const int64_t nn = ok ? ii + (int64_t)g.nnx * (jj + (int64_t)g.nny * kk) : 0;
            const uint8_t mb = ok ? nmask[nn] : (uint8_t)0xff;
            T xv[CB][N::ND];
#pragma unroll
            for (int q = 0; q < CB; ++q)
#pragma unroll
                for (int c = 0; c < N::ND; ++c)
                    xv[q][c] = ((mb >> c) & 1) || (c0 + q >= ncols) ? T(0) : x[(c0 + q) * ld + nn * N::ND + c];
            // element slots s = (ox,oy,oz) containing this neighbour: ox in {dx, dx+1} ∩ {0,1}
#pragma unroll
            for (int s = 0; s < N::NN; ++s) {
                const int ox = s & 1, oy = (s >> 1) & 1, oz = (s >> 2) & 1;
                const int bx = dx + 1 - ox, by = dy + 1 - oy, bz = DIM == 3 ? dz + 1 - oz : 0;
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                const int b = bx + 2 * by + 4 * bz;
                const int a = (N::NN - 1) ^ s;
#pragma unroll
                for (int c = 0; c < N::ND; ++c)
#pragma unroll
                    for (int c2 = 0; c2 < N::ND; ++c2) {
                        const T kv = k0s[(a * N::ND + c) * N::NDE + b * N::ND + c2];
#pragma unroll
                        for (int q = 0; q < CB; ++q) tmp[s][q][c] += kv * xv[q][c2];
                    }
            }
        }
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            double dsum = 0.0;
            if (active && c0 + q < ncols) {
                const int col = c0 + q;
#pragma unroll
                for (int c = 0; c < N::ND; ++c) {
                    T acc = T(0);
#pragma unroll
                    for (int s = 0; s < N::NN; ++s) acc += Ee[s] * tmp[s][q][c];
                    const int64_t d = node * N::ND + c;
                    const T xown = x[col * ld + d];
                    const T ax = (own >> c) & 1 ? xown : acc;
                    const T rr = MODE == kModeY ? T(0) : r[col * ld + d];
                    const T di = MODE == kModeJacobi ? dinv[d] : T(0);
                    y[col * ld + d] = epilogue<T, MODE>(ax, xown, rr, di, omega);
                    if (DOT) dsum += (double)xown * (double)ax;
                }
            }
            if (DOT) {
                const double bs = block_sum(dsum, sh);
                if (threadIdx.x == 0 && threadIdx.y == 0 && c0 + q < ncols) part[(c0 + q) * nblk + blk] = bs;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Coarse-level applies.  SRC selects where the element matrix entries come
// from:
//   kSrcDense   dense per-element matrices (SoA, entry-major, stride m);
//   kSrcKron    dense scalar nn x nn matrices acting on each component (G);
//   kSrcChildE  level 2 on the fly: K_E = sum_c E_c Mc[c] from the fine-level
//               moduli of the 2^dim children (Mc = T_c^T K0 T_c, in LDS).
// Column chunks of CB reuse every matrix entry.

// ---------------------------------------------------------------------------
// Level-1 stress-stiffness apply from element stresses S (SoA nv x m):
// G_e = (sum_k S_k,e Hk_k) kron I.

template <int DIM>
__global__ __launch_bounds__(256) void k_apply_G_fine(Geo g, const double* __restrict__ S,
                                                      const uint8_t* __restrict__ nmask,
                                                      const double* __restrict__ Hk, int ncols, int64_t ld,
                                                      const double* __restrict__ x, double* __restrict__ y) {
    using N = Nb<DIM>;
    constexpr int NV = DIM == 2 ? 3 : 6;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? blockIdx.z : 0;
    if (i >= g.nnx || j >= g.nny) return;
    const int64_t node = i + (int64_t)g.nnx * (j + (int64_t)g.nny * k);
    int64_t idx[N::NB];
    uint8_t msk[N::NB];
    neighbourhood<DIM>(g, i, j, k, nmask, idx, msk);
    // row a of each adjacent element's scalar matrix g_e
    double grow[N::NN][N::NN];
#pragma unroll
    for (int s = 0; s < N::NN; ++s) {
        bool ok;
        const int64_t e = elem_of_slot<DIM>(g, i, j, k, s, ok);
        const int a = (N::NN - 1) ^ s;
        double sv[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) sv[q] = ok ? S[q * g.m + e] : 0.0;
#pragma unroll
        for (int b = 0; b < N::NN; ++b) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NV; ++q) v += sv[q] * Hk[q * 64 + a * N::NN + b];
            grow[s][b] = v;
        }
    }
    const uint8_t own = msk[N::slot(0, 0, 0)];
    for (int col = 0; col < ncols; ++col) {
        const double* xc = x + col * ld;
        double acc[N::ND];
#pragma unroll
        for (int c = 0; c < N::ND; ++c) acc[c] = 0.0;
#pragma unroll
        for (int s = 0; s < N::NN; ++s) {
            const int ox = s & 1, oy = (s >> 1) & 1, oz = (s >> 2) & 1;
#pragma unroll
            for (int b = 0; b < N::NN; ++b) {
                const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
                const int ts = N::slot(ox - 1 + bx, oy - 1 + by, DIM == 3 ? oz - 1 + bz : 0);
#pragma unroll
                for (int c = 0; c < N::ND; ++c) {
                    const double xv = (msk[ts] >> c) & 1 ? 0.0 : xc[idx[ts] * N::ND + c];
                    acc[c] += grow[s][b] * xv;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < N::ND; ++c) y[col * ld + node * N::ND + c] = (own >> c) & 1 ? 0.0 : acc[c];
    }
}

// ---------------------------------------------------------------------------
// Inverse diagonals (Jacobi), FP64 and FP32 copies.  The FP64 copy is 1 at
// fixed DOFs (identity rows); the FP32 copy, read only by the mixed-precision
// smoother, whose blocks are 0 at fixed DOFs, is 0 there, so that its sweeps
// leave those DOFs at 0 without reading the mask.

template <int DIM>
__global__ void k_dinv_fine(Geo g, const double* __restrict__ E, const uint8_t* __restrict__ nmask,
                            const double* __restrict__ K0, double* __restrict__ dinv, float* __restrict__ dinvf) {
    using N = Nb<DIM>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? blockIdx.z : 0;
    if (i >= g.nnx || j >= g.nny) return;
    const int64_t node = i + (int64_t)g.nnx * (j + (int64_t)g.nny * k);
    const uint8_t own = nmask[node];
#pragma unroll
    for (int c = 0; c < N::ND; ++c) {
        double d = 0.0;
#pragma unroll
        for (int s = 0; s < N::NN; ++s) {
            bool ok;
            const int64_t e = elem_of_slot<DIM>(g, i, j, k, s, ok);
            const int a = (N::NN - 1) ^ s;
            if (ok) d += E[e] * K0[(a * N::ND + c) * N::NDE + a * N::ND + c];
        }
        const bool fixed = (own >> c) & 1;
        const double v = fixed ? 1.0 : (d > 0.0 ? 1.0 / d : 0.0);
        dinv[node * N::ND + c] = v;
        dinvf[node * N::ND + c] = fixed ? 0.0f : (float)v;
    }
}

// ---------------------------------------------------------------------------
// host launchers

static dim3 node_grid(const Geo& g, dim3& block) {
    block = dim3(64, 4, 1);
    return dim3((g.nnx + 63) / 64, (g.nny + 3) / 4, g.nnz);
}

int64_t apply_fine_blocks(const Geo& g) {
    dim3 b;
    dim3 gr = node_grid(g, b);
    return (int64_t)gr.x * gr.y * gr.z;
}

template <typename T>
void launch_apply_fine(int dim, const Geo& g, const T* E, const uint8_t* nmask, const T* K0, int ncols,
                       int64_t ld, const T* x, T* y, int mode, const T* r, const T* dinv, T omega,
                       double* dot_part, hipStream_t st) {
    dim3 b;
    dim3 gr = node_grid(g, b);
#define MLB_LAUNCH(D, M, DOT, CB)                                                                         \
    hipLaunchKernelGGL((k_apply_fine<D, T, M, DOT, CB>), gr, b, 0, st, g, E, nmask, K0, ncols, ld, x, y, r, \
                       dinv, omega, dot_part)
#define MLB_MODES(D, CB)                                                       \
    if (mode == kModeY && dot_part) MLB_LAUNCH(D, kModeY, true, CB);           \
    else if (mode == kModeY) MLB_LAUNCH(D, kModeY, false, CB);                 \
    else if (mode == kModeResidual) MLB_LAUNCH(D, kModeResidual, false, CB);   \
    else MLB_LAUNCH(D, kModeJacobi, false, CB);
    if (dim == 2) {
        if (ncols == 1) { MLB_MODES(2, 1) } else { MLB_MODES(2, 4) }
    } else {
        if (ncols == 1) { MLB_MODES(3, 1) } else { MLB_MODES(3, 2) }
    }
#undef MLB_MODES
#undef MLB_LAUNCH
}

void launch_apply_G_fine(int dim, const Geo& g, const double* S, const uint8_t* nmask, const double* Hk,
                         int ncols, int64_t ld, const double* x, double* y, hipStream_t st) {
    dim3 b;
    dim3 gr = node_grid(g, b);
    if (dim == 2) hipLaunchKernelGGL(k_apply_G_fine<2>, gr, b, 0, st, g, S, nmask, Hk, ncols, ld, x, y);
    else hipLaunchKernelGGL(k_apply_G_fine<3>, gr, b, 0, st, g, S, nmask, Hk, ncols, ld, x, y);
}

void launch_dinv_fine(int dim, const Geo& g, const double* E, const uint8_t* nmask, const double* K0,
                      double* dinv, float* dinvf, hipStream_t st) {
    dim3 b;
    dim3 gr = node_grid(g, b);
    if (dim == 2) hipLaunchKernelGGL(k_dinv_fine<2>, gr, b, 0, st, g, E, nmask, K0, dinv, dinvf);
    else hipLaunchKernelGGL(k_dinv_fine<3>, gr, b, 0, st, g, E, nmask, K0, dinv, dinvf);
}

template void launch_apply_fine<double>(int, const Geo&, const double*, const uint8_t*, const double*, int,
                                        int64_t, const double*, double*, int, const double*, const double*,
                                        double, double*, hipStream_t);
template void launch_apply_fine<float>(int, const Geo&, const float*, const uint8_t*, const float*, int,
                                       int64_t, const float*, float*, int, const float*, const float*, float,
                                       double*, hipStream_t);

}  // namespace mlb
