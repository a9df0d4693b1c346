// Element stresses, adjoint right-hand sides and sensitivities.
//
// Stress (Sec. 2, G_e = E_sigma(x_e) G_e0[u_e]): one Voigt stress per element
// at the centroid, s_e = E_sigma(x_e) D0 B_c u_e.
// Adjoint RHS (eq. AdjointSystem): G depends linearly on u through s_e, so
//   grad_u (phi^T G phi) = sum_e P_e^T E_sigma,e B_c^T D0 w_e,
//   w_e,k = phi_e^T (Hk_k kron I) phi_e.
// Buckling-factor sensitivity (eq. SensitivityLambda times lambda, the
// factor implied by the normalisation phi^T K phi = 1):
//   dlam/dx_e = lam [dEk phi^T K0 phi + lam (dEs phi^T G_e0[u_e] phi - dEk z^T K0 u)]
// Consistent variant (appendix, eq. consistentSensitivity, read through the
// fine solve K Phi~ = G Psi): with w = K^-1 (K + lam G) phi and psi the
// combination of interpolated coarse modes with K phi = G psi, the adjoint
// right-hand side gains (2 / lam) grad_u (w^T G psi) and the sensitivity
//   + 2 lam (dEs w^T G_e0[u_e] psi - dEk w^T K0 phi).
#include "kernels.h"

namespace mlb {

template <int DIM>
__device__ inline void elem_nodes(const Geo& g, int64_t e, int64_t* nodes) {
    const int i = (int)(e % g.nx);
    const int j = (int)((e / g.nx) % g.ny);
    const int k = DIM == 3 ? (int)(e / ((int64_t)g.nx * g.ny)) : 0;
#pragma unroll
    for (int a = 0; a < (1 << DIM); ++a)
        nodes[a] = (i + (a & 1)) + (int64_t)g.nnx * ((j + ((a >> 1) & 1)) + (int64_t)g.nny * (k + ((a >> 2) & 1)));
}

template <int DIM>
__global__ void k_stress(Geo g, const double* __restrict__ Es, const double* __restrict__ u,
                         const double* __restrict__ D0Bc, double* __restrict__ S) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM, NV = DIM == 2 ? 3 : 6;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    int64_t nodes[NN];
    elem_nodes<DIM>(g, e, nodes);
    double ue[NDE];
#pragma unroll
    for (int a = 0; a < NN; ++a)
#pragma unroll
        for (int c = 0; c < ND; ++c) ue[a * ND + c] = u[nodes[a] * ND + c];
    const double es = Es[e];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NDE; ++j) s += D0Bc[k * NDE + j] * ue[j];
        S[k * g.m + e] = es * s;
    }
}

template <int DIM>
__device__ inline double quad_K0(const double* __restrict__ K0, const double* a, const double* b) {
    constexpr int NDE = DIM << DIM;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NDE; ++i) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < NDE; ++j) t += K0[i * NDE + j] * b[j];
        s += a[i] * t;
    }
    return s;
}

// w_k = sum_c phi_c^T Hk_k phi_c for the nv Voigt components.
template <int DIM>
__device__ inline void quad_Hk(const double* __restrict__ Hk, const double* ph, double* w) {
    constexpr int NN = 1 << DIM, ND = DIM, NV = DIM == 2 ? 3 : 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NN; ++a)
#pragma unroll
            for (int b = 0; b < NN; ++b) {
                double pp = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) pp += ph[a * ND + c] * ph[b * ND + c];
                s += Hk[k * 64 + a * NN + b] * pp;
            }
        w[k] = s;
    }
}

// w_k = sum_c a_c^T Hk_k b_c (bilinear; Hk_k is symmetric).
template <int DIM>
__device__ inline void bil_Hk(const double* __restrict__ Hk, const double* a, const double* b, double* w) {
    constexpr int NN = 1 << DIM, ND = DIM, NV = DIM == 2 ? 3 : 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NN; ++i)
#pragma unroll
            for (int j = 0; j < NN; ++j) {
                double pp = 0.0;
#pragma unroll
                for (int c = 0; c < ND; ++c) pp += a[i * ND + c] * b[j * ND + c];
                s += Hk[k * 64 + i * NN + j] * pp;
            }
        w[k] = s;
    }
}

template <int DIM>
__global__ void k_dJ(Geo g, const double* __restrict__ x, double p, double dE, int ncases, int64_t ld,
                     const double* __restrict__ U, const double* __restrict__ K0, double* __restrict__ dJ) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    int64_t nodes[NN];
    elem_nodes<DIM>(g, e, nodes);
    const double xe = x[e];
    const double dEk = xe > 0.0 ? p * pow(xe, p - 1.0) * dE : (p == 1.0 ? dE : 0.0);
    for (int c0 = 0; c0 < ncases; ++c0) {
        double ue[NDE];
#pragma unroll
        for (int a = 0; a < NN; ++a)
#pragma unroll
            for (int c = 0; c < ND; ++c) ue[a * ND + c] = U[c0 * ld + nodes[a] * ND + c];
        dJ[c0 * g.m + e] = -dEk * quad_K0<DIM>(K0, ue, ue);
    }
}

// V[(i*nv + k)*m + e] = E_sigma,e (D0 w_e)_k for mode i; CONS adds
// (2 / lam_i) times the bilinear w_k(W_i, Ps_i) to w_k(Phi_i, Phi_i)
template <int DIM, bool CONS>
__global__ void k_adj_elem(Geo g, const double* __restrict__ Es, int q, int64_t ld, const double* __restrict__ Phi,
                           const double* __restrict__ Hk, const double* __restrict__ D0, double* __restrict__ V,
                           const double* __restrict__ W, const double* __restrict__ Ps, const double* __restrict__ lam) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM, NV = DIM == 2 ? 3 : 6;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    int64_t nodes[NN];
    elem_nodes<DIM>(g, e, nodes);
    const double es = Es[e];
    for (int i = 0; i < q; ++i) {
        double ph[NDE];
#pragma unroll
        for (int a = 0; a < NN; ++a)
#pragma unroll
            for (int c = 0; c < ND; ++c) ph[a * ND + c] = Phi[i * ld + nodes[a] * ND + c];
        double w[NV];
        quad_Hk<DIM>(Hk, ph, w);
        if (CONS) {
            double we[NDE], pe[NDE], wb[NV];
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    we[a * ND + c] = W[i * ld + nodes[a] * ND + c];
                    pe[a * ND + c] = Ps[i * ld + nodes[a] * ND + c];
                }
            bil_Hk<DIM>(Hk, we, pe, wb);
            const double f = 2.0 / lam[i];
#pragma unroll
            for (int k = 0; k < NV; ++k) w[k] += f * wb[k];
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < NV; ++l) s += D0[k * NV + l] * w[l];
            V[((int64_t)i * NV + k) * g.m + e] = es * s;
        }
    }
}

// b[node, c] = sum over adjacent elements of sum_k Bc[k][a*dim + c] V_k,e  (0 at fixed DOFs)
template <int DIM>
__global__ void k_adj_gather(Geo g, int q, const double* __restrict__ V, const double* __restrict__ Bc,
                             const uint8_t* __restrict__ nmask, int64_t ld, double* __restrict__ B) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM, NV = DIM == 2 ? 3 : 6;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = DIM == 3 ? blockIdx.z : 0;
    if (i >= g.nnx || j >= g.nny) return;
    const int64_t node = i + (int64_t)g.nnx * (j + (int64_t)g.nny * k);
    const uint8_t own = nmask[node];
    for (int md = 0; md < q; ++md) {
        double acc[ND];
#pragma unroll
        for (int c = 0; c < ND; ++c) acc[c] = 0.0;
#pragma unroll
        for (int s = 0; s < NN; ++s) {
            const int ox = s & 1, oy = (s >> 1) & 1, oz = (s >> 2) & 1;
            const int ei = i - 1 + ox, ej = j - 1 + oy, ek = DIM == 3 ? k - 1 + oz : 0;
            if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || (DIM == 3 && (ek < 0 || ek >= g.nz))) continue;
            const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
            const int a = (NN - 1) ^ s;
#pragma unroll
            for (int kk = 0; kk < NV; ++kk) {
                const double v = V[((int64_t)md * NV + kk) * g.m + e];
#pragma unroll
                for (int c = 0; c < ND; ++c) acc[c] += Bc[kk * NDE + a * ND + c] * v;
            }
        }
#pragma unroll
        for (int c = 0; c < ND; ++c) B[md * ld + node * ND + c] = (own >> c) & 1 ? 0.0 : acc[c];
    }
}

template <int DIM, bool CONS>
__global__ void k_dlam(Geo g, const double* __restrict__ x, double p, double E1, double E0,
                       const double* __restrict__ u, int q, int64_t ld, const double* __restrict__ Phi,
                       const double* __restrict__ Z, const double* __restrict__ lam, const double* __restrict__ K0,
                       const double* __restrict__ Hk, const double* __restrict__ D0Bc, double* __restrict__ out,
                       const double* __restrict__ W, const double* __restrict__ Ps) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM, NV = DIM == 2 ? 3 : 6;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    int64_t nodes[NN];
    elem_nodes<DIM>(g, e, nodes);
    const double xe = x[e];
    const double xp1 = xe > 0.0 ? p * pow(xe, p - 1.0) : (p == 1.0 ? 1.0 : 0.0);
    const double dEk = xp1 * (E1 - E0), dEs = xp1 * E1;
    double ue[NDE];
#pragma unroll
    for (int a = 0; a < NN; ++a)
#pragma unroll
        for (int c = 0; c < ND; ++c) ue[a * ND + c] = u[nodes[a] * ND + c];
    double s0[NV];   // unit-modulus stress D0 Bc u_e
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NDE; ++j) s += D0Bc[k * NDE + j] * ue[j];
        s0[k] = s;
    }
    double K0u[NDE];
#pragma unroll
    for (int a = 0; a < NDE; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NDE; ++b) s += K0[a * NDE + b] * ue[b];
        K0u[a] = s;
    }
    for (int i = 0; i < q; ++i) {
        double ph[NDE], ze[NDE];
#pragma unroll
        for (int a = 0; a < NN; ++a)
#pragma unroll
            for (int c = 0; c < ND; ++c) {
                ph[a * ND + c] = Phi[i * ld + nodes[a] * ND + c];
                ze[a * ND + c] = Z[i * ld + nodes[a] * ND + c];
            }
        const double pK = quad_K0<DIM>(K0, ph, ph);
        double w[NV];
        quad_Hk<DIM>(Hk, ph, w);
        double pG = 0.0;
#pragma unroll
        for (int k = 0; k < NV; ++k) pG += s0[k] * w[k];
        double zKu = 0.0;
#pragma unroll
        for (int a = 0; a < NDE; ++a) zKu += ze[a] * K0u[a];
        const double l = lam[i];
        double r = l * (dEk * pK + l * (dEs * pG - dEk * zKu));
        if (CONS) {
            double we[NDE], pe[NDE], wb[NV];
#pragma unroll
            for (int a = 0; a < NN; ++a)
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                    we[a * ND + c] = W[i * ld + nodes[a] * ND + c];
                    pe[a * ND + c] = Ps[i * ld + nodes[a] * ND + c];
                }
            bil_Hk<DIM>(Hk, we, pe, wb);
            double wGp = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) wGp += s0[k] * wb[k];
            const double wKp = quad_K0<DIM>(K0, we, ph);
            r += 2.0 * l * (dEs * wGp - dEk * wKp);
        }
        out[(int64_t)i * g.m + e] = r;
    }
}

// ---- launchers
static inline unsigned nb1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_stress(int dim, const Geo& g, const double* Es, const double* u, const double* D0Bc, double* S,
                   hipStream_t st) {
    if (dim == 2) hipLaunchKernelGGL(k_stress<2>, dim3(nb1(g.m)), dim3(kBlock), 0, st, g, Es, u, D0Bc, S);
    else hipLaunchKernelGGL(k_stress<3>, dim3(nb1(g.m)), dim3(kBlock), 0, st, g, Es, u, D0Bc, S);
}
void launch_dJ(int dim, const Geo& g, const double* x, double p, double dE, int ncases, int64_t ld, const double* U,
               const double* K0, double* dJ, hipStream_t st) {
    if (dim == 2) hipLaunchKernelGGL(k_dJ<2>, dim3(nb1(g.m)), dim3(kBlock), 0, st, g, x, p, dE, ncases, ld, U, K0, dJ);
    else hipLaunchKernelGGL(k_dJ<3>, dim3(nb1(g.m)), dim3(kBlock), 0, st, g, x, p, dE, ncases, ld, U, K0, dJ);
}
void launch_adj_elem(int dim, const Geo& g, const double* Es, int q, int64_t ld, const double* Phi, const double* Hk,
                     const double* D0, double* V, hipStream_t st, const double* W, const double* Ps,
                     const double* lam) {
    const dim3 gr(nb1(g.m)), b(kBlock);
    if (W) {
        if (dim == 2) hipLaunchKernelGGL((k_adj_elem<2, true>), gr, b, 0, st, g, Es, q, ld, Phi, Hk, D0, V, W, Ps, lam);
        else hipLaunchKernelGGL((k_adj_elem<3, true>), gr, b, 0, st, g, Es, q, ld, Phi, Hk, D0, V, W, Ps, lam);
    } else {
        if (dim == 2) hipLaunchKernelGGL((k_adj_elem<2, false>), gr, b, 0, st, g, Es, q, ld, Phi, Hk, D0, V, W, Ps, lam);
        else hipLaunchKernelGGL((k_adj_elem<3, false>), gr, b, 0, st, g, Es, q, ld, Phi, Hk, D0, V, W, Ps, lam);
    }
}
void launch_adj_gather(int dim, const Geo& g, int q, const double* V, const double* Bc, const uint8_t* nmask,
                       int64_t ld, double* B, hipStream_t st) {
    dim3 b(64, 4, 1), gr((g.nnx + 63) / 64, (g.nny + 3) / 4, g.nnz);
    if (dim == 2) hipLaunchKernelGGL(k_adj_gather<2>, gr, b, 0, st, g, q, V, Bc, nmask, ld, B);
    else hipLaunchKernelGGL(k_adj_gather<3>, gr, b, 0, st, g, q, V, Bc, nmask, ld, B);
}
void launch_dlam(int dim, const Geo& g, const double* x, double p, double E1, double E0, const double* u, int q,
                 int64_t ld, const double* Phi, const double* Z, const double* lam, const double* K0,
                 const double* Hk, const double* D0Bc, double* out, hipStream_t st, const double* W,
                 const double* Ps) {
    const dim3 gr(nb1(g.m)), b(kBlock);
#define MLB_DL(D, C)                                                                                            \
    hipLaunchKernelGGL((k_dlam<D, C>), gr, b, 0, st, g, x, p, E1, E0, u, q, ld, Phi, Z, lam, K0, Hk, D0Bc, out, W, \
                       Ps)
    if (W) {
        if (dim == 2) MLB_DL(2, true);
        else MLB_DL(3, true);
    } else {
        if (dim == 2) MLB_DL(2, false);
        else MLB_DL(3, false);
    }
#undef MLB_DL
}

}  // namespace mlb
