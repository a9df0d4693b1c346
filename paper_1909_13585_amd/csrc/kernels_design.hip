// Three-field design variables (Sec. 2): density filter, relaxed Heaviside
// projection (eq. projectionOperator) and the chain rule back to the design
// variables.
//
// Filter weights w = r_min - |offset| > 0 depend only on the offset between
// element centroids, so the host passes them as a table of (di, dj, dk, w)
// entries; every thread walks the same entries (uniform loads) and skips the
// ones that leave the grid.  Each row is normalised by its own weight sum W_e
// (truncated at the boundary):
//   xtilde_e = sum_k w_ek xhat_k / W_e,   x_e = projection(xtilde_e)
//   g_e      = df/dx_e * dx/dxtilde_e / W_e   (scratch, interleaved by column chunk)
//   df/dxhat_k = sum_e w_ek g_e           (w symmetric)
// Products and sums are not contracted into fused multiply-adds, and the
// table order is fixed, so the filtered field does not depend on the compiler.
#include <cmath>

#include "kernels.h"

namespace mlb {
namespace {

struct DesignProj {
    double eta, beta, tbe, den;   // tanh(beta eta), tanh(beta eta) + tanh(beta (1 - eta))
};

__device__ inline bool tab_inside(const Geo& g, int ci, int cj, int ck, const double* __restrict__ tab, int t,
                                  int64_t* k) {
    const int ii = ci + (int)tab[4 * t], jj = cj + (int)tab[4 * t + 1], kk = ck + (int)tab[4 * t + 2];
    if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) return false;
    *k = ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk);
    return true;
}

__global__ void k_filter_project(Geo g, int nt, const double* __restrict__ tab, DesignProj p,
                                 const double* __restrict__ xhat, double* __restrict__ xtilde,
                                 double* __restrict__ x) {
#pragma clang fp contract(off)
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int ci = (int)(e % g.nx), cj = (int)((e / g.nx) % g.ny), ck = (int)(e / ((int64_t)g.nx * g.ny));
    double s = 0.0, sw = 0.0;
    for (int t = 0; t < nt; ++t) {
        int64_t k;
        if (!tab_inside(g, ci, cj, ck, tab, t, &k)) continue;
        const double w = tab[4 * t + 3];
        s += w * xhat[k];
        sw += w;
    }
    const double xt = s / sw;
    xtilde[e] = xt;
    x[e] = (p.tbe + tanh(p.beta * (xt - p.eta))) / p.den;
}

// Columns are grouped in chunks of kChainCols; chunk q (columns 8q ...,
// width nc_q) is stored interleaved at work[8q m + e nc_q + j], so that the
// gather reads one neighbour's values of a chunk from one cache line.  The
// workspace holds exactly ncols x m doubles.
constexpr int kChainCols = 8;

// work = dfdx * dx/dxtilde / W_e for every column (W_e once per element)
__global__ void k_chain_scale(Geo g, int nt, const double* __restrict__ tab, DesignProj p, int ncols,
                              const double* __restrict__ xtilde, const double* __restrict__ dfdx,
                              double* __restrict__ gout) {
#pragma clang fp contract(off)
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int ci = (int)(e % g.nx), cj = (int)((e / g.nx) % g.ny), ck = (int)(e / ((int64_t)g.nx * g.ny));
    double sw = 0.0;
    for (int t = 0; t < nt; ++t) {
        int64_t k;
        if (tab_inside(g, ci, cj, ck, tab, t, &k)) sw += tab[4 * t + 3];
    }
    const double th = tanh(p.beta * (xtilde[e] - p.eta));
    const double dx = p.beta * (1.0 - th * th) / p.den;
    for (int c0 = 0; c0 < ncols; c0 += kChainCols) {
        const int nc = min(kChainCols, ncols - c0);
        double* dst = gout + (int64_t)c0 * g.m + e * nc;
        for (int j = 0; j < nc; ++j) dst[j] = dfdx[(int64_t)(c0 + j) * g.m + e] * dx / sw;
    }
}

// out[c*m + e] = sum over the table of w g_c[k] for the NC columns of the
// chunks starting at column c_first + NC blockIdx.y; each column's sum keeps
// the table order
template <int NC>
__global__ void k_chain_gather(Geo g, int nt, const double* __restrict__ tab, int c_first,
                               const double* __restrict__ gin, double* __restrict__ out) {
#pragma clang fp contract(off)
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int c0 = c_first + (int)blockIdx.y * NC;
    const double* gc = gin + (int64_t)c0 * g.m;
    const int ci = (int)(e % g.nx), cj = (int)((e / g.nx) % g.ny), ck = (int)(e / ((int64_t)g.nx * g.ny));
    double s[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) s[j] = 0.0;
    for (int t = 0; t < nt; ++t) {
        int64_t k;
        if (!tab_inside(g, ci, cj, ck, tab, t, &k)) continue;
        const double w = tab[4 * t + 3];
        const double* v = gc + k * NC;
#pragma unroll
        for (int j = 0; j < NC; ++j) s[j] += w * v[j];
    }
#pragma unroll
    for (int j = 0; j < NC; ++j) out[(int64_t)(c0 + j) * g.m + e] = s[j];
}

inline DesignProj make_proj(double eta, double beta) {
    DesignProj p;
    p.eta = eta;
    p.beta = beta;
    p.tbe = std::tanh(beta * eta);
    p.den = p.tbe + std::tanh(beta * (1.0 - eta));
    return p;
}

inline unsigned design_nb(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_filter_project(const Geo& g, int nt, const double* tab, double eta, double beta, const double* xhat,
                           double* xtilde, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_filter_project, dim3(design_nb(g.m)), dim3(kBlock), 0, st, g, nt, tab, make_proj(eta, beta),
                       xhat, xtilde, x);
}

void launch_filter_chain(const Geo& g, int nt, const double* tab, double eta, double beta, int ncols,
                         const double* xtilde, const double* dfdx, double* work, double* out, hipStream_t st) {
    const unsigned nb = design_nb(g.m);
    hipLaunchKernelGGL(k_chain_scale, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, make_proj(eta, beta), ncols, xtilde,
                       dfdx, work);
    const int full = ncols / kChainCols, rem = ncols % kChainCols;
    if (full > 0)
        hipLaunchKernelGGL(k_chain_gather<kChainCols>, dim3(nb, full), dim3(kBlock), 0, st, g, nt, tab, 0, work, out);
    const int c1 = full * kChainCols;
    switch (rem) {
        case 1: hipLaunchKernelGGL(k_chain_gather<1>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 2: hipLaunchKernelGGL(k_chain_gather<2>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 3: hipLaunchKernelGGL(k_chain_gather<3>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 4: hipLaunchKernelGGL(k_chain_gather<4>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 5: hipLaunchKernelGGL(k_chain_gather<5>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 6: hipLaunchKernelGGL(k_chain_gather<6>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        case 7: hipLaunchKernelGGL(k_chain_gather<7>, dim3(nb), dim3(kBlock), 0, st, g, nt, tab, c1, work, out); break;
        default: break;
    }
}

}  // namespace mlb
