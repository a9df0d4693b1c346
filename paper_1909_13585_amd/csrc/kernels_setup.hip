// Per-density setup: SIMP moduli, node masks, Galerkin coarse element
// matrices, and the dense FP64 inverse of the coarsest-level operator.
#include "kernels.h"

namespace mlb {

// E_kappa = E0 + x^p (E1 - E0), E_sigma = x^p E1 (eq. interpolationSIMP2-SIMP).
// Counts densities outside [0, 1] or not finite: one partial count per block
// (grid-stride loop, fixed-order block sum), summed afterwards.
__global__ void k_material(int64_t m, const double* __restrict__ x, double E1, double E0, double p,
                           double* __restrict__ Ek, float* __restrict__ Ekf, double* __restrict__ Es,
                           double* __restrict__ bad_part) {
    __shared__ double sh[16];
    double bad = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[e];
        if (!(v >= 0.0 && v <= 1.0)) bad += 1.0;   // also catches NaN
        const double xp = v > 0.0 ? pow(v, p) : 0.0;
        const double ek = E0 + xp * (E1 - E0);
        Ek[e] = ek;
        Ekf[e] = (float)ek;
        Es[e] = xp * E1;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if (lane == 0) sh[wid] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
        bad_part[blockIdx.x] = s;
    }
}

__global__ void k_node_mask(int64_t nodes, int dim, const uint8_t* __restrict__ fixed, uint8_t* __restrict__ nm) {
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nodes) return;
    uint8_t v = 0;
    for (int c = 0; c < dim; ++c)
        if (fixed[n * dim + c]) v |= (uint8_t)(1u << c);
    nm[n] = v;
}

__global__ void k_coarse_mask(Geo gf, Geo gc, const uint8_t* __restrict__ mf, uint8_t* __restrict__ mc) {
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= gc.nodes) return;
    const int I = (int)(n % gc.nnx);
    const int J = (int)((n / gc.nnx) % gc.nny);
    const int K = (int)(n / ((int64_t)gc.nnx * gc.nny));
    mc[n] = mf[2 * I + (int64_t)gf.nnx * (2 * J + (int64_t)gf.nny * 2 * K)];
}

// child c = cx + 2cy + 4cz of coarse element (I,J,K) is fine element (2I+cx, ...)
__device__ inline int64_t child_elem(const Geo& gf, int I, int J, int K, int c) {
    return (2 * I + (c & 1)) + (int64_t)gf.nx * ((2 * J + ((c >> 1) & 1)) + (int64_t)gf.ny * (2 * K + ((c >> 2) & 1)));
}

__device__ inline void coarse_ijk(const Geo& gc, int64_t E, int& I, int& J, int& K) {
    I = (int)(E % gc.nx);
    J = (int)((E / gc.nx) % gc.ny);
    K = (int)(E / ((int64_t)gc.nx * gc.ny));
}

// Level 1 -> 2: K_E = sum_c E_c Mc[c], Mc[c] = T_c^T K0 T_c.
template <int DIM>
__global__ void k_galerkin_from_E(Geo gf, Geo gc, const double* __restrict__ E, const double* __restrict__ Mc,
                                  double* __restrict__ Kc) {
    constexpr int NDE = DIM << DIM, NCH = 1 << DIM;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= gc.m * NDE * NDE) return;
    const int64_t Ec = t % gc.m;
    const int entry = (int)(t / gc.m);
    int I, J, K;
    coarse_ijk(gc, Ec, I, J, K);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += E[child_elem(gf, I, J, K, c)] * Mc[c * 576 + entry];
    Kc[(int64_t)entry * gc.m + Ec] = s;
}

// Level 1 -> 2 for G: g_E = sum_c sum_k S_k,c GHc[c][k]  (scalar nn x nn).
template <int DIM>
__global__ void k_galerkin_G_from_S(Geo gf, Geo gc, const double* __restrict__ S, const double* __restrict__ GHc,
                                    double* __restrict__ gout) {
    constexpr int NN = 1 << DIM, NCH = 1 << DIM, NV = DIM == 2 ? 3 : 6;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= gc.m * NN * NN) return;
    const int64_t Ec = t % gc.m;
    const int entry = (int)(t / gc.m);
    const int A = entry / NN, B = entry % NN;
    int I, J, K;
    coarse_ijk(gc, Ec, I, J, K);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int64_t e = child_elem(gf, I, J, K, c);
#pragma unroll
        for (int k = 0; k < NV; ++k) s += S[k * gf.m + e] * GHc[(c * 6 + k) * 64 + A * NN + B];
    }
    gout[(int64_t)entry * gc.m + Ec] = s;
}

// Level j -> j+1 from dense child matrices: K_E = sum_c T_c^T K_c T_c.
template <int DIM, bool KRON>
__global__ void k_galerkin_dense(Geo gf, Geo gc, const double* __restrict__ Kf, const double* __restrict__ T,
                                 double* __restrict__ Kc) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM, NCH = 1 << DIM;
    constexpr int W = KRON ? NN : NDE;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= gc.m * W * W) return;
    const int64_t Ec = t % gc.m;
    const int entry = (int)(t / gc.m);
    const int row = entry / W, col = entry % W;
    const int A = KRON ? row : row / ND, ca = KRON ? 0 : row % ND;
    const int B = KRON ? col : col / ND, cb = KRON ? 0 : col % ND;
    int I, J, K;
    coarse_ijk(gc, Ec, I, J, K);
    double s = 0.0;
    for (int c = 0; c < NCH; ++c) {
        const int64_t e = child_elem(gf, I, J, K, c);
        for (int b = 0; b < NN; ++b) {
            const double wa = T[(c * 8 + b) * 8 + A];
            if (wa == 0.0) continue;
            for (int b2 = 0; b2 < NN; ++b2) {
                const double wb = T[(c * 8 + b2) * 8 + B];
                if (wb == 0.0) continue;
                const int fe = KRON ? b * NN + b2 : (b * ND + ca) * NDE + b2 * ND + cb;
                s += wa * wb * Kf[(int64_t)fe * gf.m + e];
            }
        }
    }
    Kc[(int64_t)entry * gc.m + Ec] = s;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Dense (row-major n x n) coarsest operator; identity rows/cols at fixed DOFs.
// One thread per row: each thread writes only its own row.
template <int DIM>
__global__ void k_assemble_dense(Geo g, const double* __restrict__ Ke, const uint8_t* __restrict__ nmask, int64_t n,
                                 int64_t ld, double* __restrict__ A) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM;
    const int64_t rowdof = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (rowdof >= n) return;
    const int64_t node = rowdof / ND;
    const int c = (int)(rowdof % ND);
    const int i = (int)(node % g.nnx), j = (int)((node / g.nnx) % g.nny), k = (int)(node / ((int64_t)g.nnx * g.nny));
    double* Ar = A + rowdof * ld;
    if ((nmask[node] >> c) & 1) {
        Ar[rowdof] = 1.0;
        return;
    }
    for (int s = 0; s < NN; ++s) {
        const int ox = s & 1, oy = (s >> 1) & 1, oz = (s >> 2) & 1;
        const int ei = i - 1 + ox, ej = j - 1 + oy, ek = DIM == 3 ? k - 1 + oz : 0;
        if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || (DIM == 3 && (ek < 0 || ek >= g.nz))) continue;
        const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
        const int a = (NN - 1) ^ s;
        for (int b = 0; b < NN; ++b) {
            const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
            const int64_t nb = (ei + bx) + (int64_t)g.nnx * ((ej + by) + (int64_t)g.nny * (ek + (DIM == 3 ? bz : 0)));
            const uint8_t mb = nmask[nb];
            for (int c2 = 0; c2 < ND; ++c2) {
                if ((mb >> c2) & 1) continue;
                Ar[nb * ND + c2] += Ke[(int64_t)((a * ND + c) * NDE + b * ND + c2) * g.m + e];
            }
        }
    }
}

// A[i * N + i] = 1 for n <= i < N (identity padding of the coarsest matrix)
__global__ void k_pad_identity(int64_t n, int64_t N, double* __restrict__ A) {
    const int64_t i = n + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < N) A[i * N + i] = 1.0;
}

// ---- launchers
static inline unsigned nb1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_material(int64_t m, const double* x, double E1, double E0, double p, double* Ek, float* Ekf,
                     double* Es, int nparts, double* bad_part, hipStream_t st) {
    hipLaunchKernelGGL(k_material, dim3(nparts), dim3(kBlock), 0, st, m, x, E1, E0, p, Ek, Ekf, Es, bad_part);
}
void launch_node_mask(int64_t nodes, int dim, const uint8_t* fixed, uint8_t* nm, hipStream_t st) {
    hipLaunchKernelGGL(k_node_mask, dim3(nb1(nodes)), dim3(kBlock), 0, st, nodes, dim, fixed, nm);
}
void launch_coarse_mask(const Geo& gf, const Geo& gc, const uint8_t* mf, uint8_t* mc, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_mask, dim3(nb1(gc.nodes)), dim3(kBlock), 0, st, gf, gc, mf, mc);
}
void launch_galerkin_from_E(int dim, const Geo& gf, const Geo& gc, const double* E, const double* Mc, double* Kc,
                            hipStream_t st) {
    const int nde = dim << dim;
    const int64_t tot = gc.m * nde * nde;
    if (dim == 2) hipLaunchKernelGGL(k_galerkin_from_E<2>, dim3(nb1(tot)), dim3(kBlock), 0, st, gf, gc, E, Mc, Kc);
    else hipLaunchKernelGGL(k_galerkin_from_E<3>, dim3(nb1(tot)), dim3(kBlock), 0, st, gf, gc, E, Mc, Kc);
}
// Fine-grid element matrices in the layout the stencil assembly reads
// ([entry m + e]): K_e = E_e K0 (nde x nde) and the scalar stress matrix
// g_e = sum_q S_qe H_q (nn x nn).  Used only when the refinement of Alg. 2
// also visits the fine grid.
__global__ void k_fine_Ke(int64_t m, int nde2, const double* __restrict__ E, const double* __restrict__ K0,
                          double* __restrict__ Ke) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m * nde2) return;
    const int64_t e = t % m;
    const int entry = (int)(t / m);
    Ke[t] = E[e] * K0[entry];
}

__global__ void k_fine_Ge(int64_t m, int nn, int nv, const double* __restrict__ S, const double* __restrict__ Hk,
                          double* __restrict__ Ge) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= m * nn * nn) return;
    const int64_t e = t % m;
    const int entry = (int)(t / m);
    double s = 0.0;
    for (int q = 0; q < nv; ++q) s += S[q * m + e] * Hk[q * 64 + entry];
    Ge[t] = s;
}

void launch_fine_elem_mats(int dim, const Geo& g, const double* E, const double* K0, const double* S,
                           const double* Hk, double* Ke, double* Ge, hipStream_t st) {
    const int nn = 1 << dim, nde = dim << dim, nv = dim == 2 ? 3 : 6;
    const int64_t t1 = g.m * nde * nde, t2 = g.m * nn * nn;
    hipLaunchKernelGGL(k_fine_Ke, dim3(nb1(t1)), dim3(kBlock), 0, st, g.m, nde * nde, E, K0, Ke);
    hipLaunchKernelGGL(k_fine_Ge, dim3(nb1(t2)), dim3(kBlock), 0, st, g.m, nn, nv, S, Hk, Ge);
}

void launch_galerkin_G_from_S(int dim, const Geo& gf, const Geo& gc, const double* S, const double* GHc,
                              double* gout, hipStream_t st) {
    const int nn = 1 << dim;
    const int64_t tot = gc.m * nn * nn;
    if (dim == 2) hipLaunchKernelGGL(k_galerkin_G_from_S<2>, dim3(nb1(tot)), dim3(kBlock), 0, st, gf, gc, S, GHc, gout);
    else hipLaunchKernelGGL(k_galerkin_G_from_S<3>, dim3(nb1(tot)), dim3(kBlock), 0, st, gf, gc, S, GHc, gout);
}
void launch_galerkin_dense(int dim, bool kron, const Geo& gf, const Geo& gc, const double* Kf, const double* T,
                           double* Kc, hipStream_t st) {
    const int w = kron ? (1 << dim) : (dim << dim);
    const int64_t tot = gc.m * w * w;
    dim3 gr(nb1(tot)), b(kBlock);
    if (dim == 2) {
        if (kron) hipLaunchKernelGGL((k_galerkin_dense<2, true>), gr, b, 0, st, gf, gc, Kf, T, Kc);
        else hipLaunchKernelGGL((k_galerkin_dense<2, false>), gr, b, 0, st, gf, gc, Kf, T, Kc);
    } else {
        if (kron) hipLaunchKernelGGL((k_galerkin_dense<3, true>), gr, b, 0, st, gf, gc, Kf, T, Kc);
        else hipLaunchKernelGGL((k_galerkin_dense<3, false>), gr, b, 0, st, gf, gc, Kf, T, Kc);
    }
}
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t st) {
    hipLaunchKernelGGL(k_to_float, dim3(nb1(n)), dim3(kBlock), 0, st, n, a, b);
}
void launch_assemble_dense(int dim, const Geo& g, const double* Ke, const uint8_t* nmask, int64_t n, int64_t ld,
                           double* A, hipStream_t st) {
    if (dim == 2) hipLaunchKernelGGL(k_assemble_dense<2>, dim3(nb1(n)), dim3(kBlock), 0, st, g, Ke, nmask, n, ld, A);
    else hipLaunchKernelGGL(k_assemble_dense<3>, dim3(nb1(n)), dim3(kBlock), 0, st, g, Ke, nmask, n, ld, A);
}
void launch_pad_identity(int64_t n, int64_t N, double* A, hipStream_t st) {
    if (N > n) hipLaunchKernelGGL(k_pad_identity, dim3(nb1(N - n)), dim3(kBlock), 0, st, n, N, A);
}

}  // namespace mlb
