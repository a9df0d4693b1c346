// Post-processing measures of local buckling (Sec. 5):
//   strain energy density  pi_{j|e} = E_kappa(x_e) phi_{j|e}^T K_e0 phi_{j|e},
//   its gradient magnitude on the element grid and total variation over the
//   solid set {x_e >= xbar} (eq. TVsed),
//   a local dilation of the densities around flagged elements
//   (eq. postProcessingDilation).
// The gradient of the element-constant field uses differences between
// neighbouring solid elements only: central when both neighbours along an
// axis are solid, one-sided when one is, none otherwise; zero off the solid
// set.  Dilation: element e takes the largest density among the flagged
// elements whose centroid lies within r_th of its own, and keeps its own
// density when that is larger or when there is none.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace mlb {
namespace {

template <int DIM>
__device__ inline void post_elem_nodes(const Geo& g, int64_t e, int64_t* nodes) {
    const int i = (int)(e % g.nx);
    const int j = (int)((e / g.nx) % g.ny);
    const int k = DIM == 3 ? (int)(e / ((int64_t)g.nx * g.ny)) : 0;
#pragma unroll
    for (int a = 0; a < (1 << DIM); ++a)
        nodes[a] = (i + (a & 1)) + (int64_t)g.nnx * ((j + ((a >> 1) & 1)) + (int64_t)g.nny * (k + ((a >> 2) & 1)));
}

__device__ inline double post_block_sum(double v, double* sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

// sed[i*m + e], one thread per element, all q modes
template <int DIM>
__global__ void k_sed(Geo g, const double* __restrict__ Ek, int q, int64_t ld, const double* __restrict__ Phi,
                      const double* __restrict__ K0, double* __restrict__ sed) {
    constexpr int NN = 1 << DIM, ND = DIM, NDE = DIM << DIM;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    int64_t nodes[NN];
    post_elem_nodes<DIM>(g, e, nodes);
    const double E = Ek[e];
    for (int i = 0; i < q; ++i) {
        double ph[NDE];
#pragma unroll
        for (int a = 0; a < NN; ++a)
#pragma unroll
            for (int c = 0; c < ND; ++c) ph[a * ND + c] = Phi[i * ld + nodes[a] * ND + c];
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NDE; ++r) {
            double t = 0.0;
#pragma unroll
            for (int cc = 0; cc < NDE; ++cc) t += K0[r * NDE + cc] * ph[cc];
            s += ph[r] * t;
        }
        sed[(int64_t)i * g.m + e] = E * s;
    }
}

// gradn[i*m + e] = |grad pi_i|_e on the solid set, 0 elsewhere; part[i*gridDim.x + b]
// = this block's sum of gradn over solid elements.  Grid (nparts, q).
template <int DIM>
__global__ void k_grad_tv(Geo g, const double* __restrict__ x, double xbar, const double* __restrict__ sed,
                          double* __restrict__ gradn, double* __restrict__ part) {
    __shared__ double sh[16];
    const int i = blockIdx.y;
    const double* P = sed + (int64_t)i * g.m;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < g.m; e += (int64_t)gridDim.x * blockDim.x) {
        double gn = 0.0;
        if (x[e] >= xbar) {
            const int ci[3] = {(int)(e % g.nx), (int)((e / g.nx) % g.ny),
                               DIM == 3 ? (int)(e / ((int64_t)g.nx * g.ny)) : 0};
            const int ext[3] = {g.nx, g.ny, g.nz};
            const int64_t stride[3] = {1, g.nx, (int64_t)g.nx * g.ny};
            const double pe = P[e];
            double g2 = 0.0;
#pragma unroll
            for (int ax = 0; ax < DIM; ++ax) {
                const bool lo = ci[ax] > 0 && x[e - stride[ax]] >= xbar;
                const bool hi = ci[ax] + 1 < ext[ax] && x[e + stride[ax]] >= xbar;
                double d = 0.0;
                if (lo && hi) d = (P[e + stride[ax]] - P[e - stride[ax]]) / 2.0;
                else if (hi) d = P[e + stride[ax]] - pe;
                else if (lo) d = pe - P[e - stride[ax]];
                g2 += d * d;
            }
            gn = sqrt(g2);
            acc += gn;
        }
        gradn[(int64_t)i * g.m + e] = gn;
    }
    acc = post_block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = acc;
}

template <int DIM>
__global__ void k_dilate(Geo g, int nsel, const double* __restrict__ gradn, const double* __restrict__ gmax,
                         double rel_thr, int R, double r2, const double* __restrict__ x, double* __restrict__ xout) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= g.m) return;
    const int ci = (int)(e % g.nx), cj = (int)((e / g.nx) % g.ny);
    const int ck = DIM == 3 ? (int)(e / ((int64_t)g.nx * g.ny)) : 0;
    const int Rz = DIM == 3 ? R : 0;
    double best = x[e];
    for (int dk = -Rz; dk <= Rz; ++dk) {
        const int kk = ck + dk;
        if (kk < 0 || kk >= g.nz) continue;
        for (int dj = -R; dj <= R; ++dj) {
            const int jj = cj + dj;
            if (jj < 0 || jj >= g.ny) continue;
            for (int di = -R; di <= R; ++di) {
                const int ii = ci + di;
                if (ii < 0 || ii >= g.nx) continue;
                if ((double)(di * di + dj * dj + dk * dk) > r2) continue;
                const int64_t k = ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk);
                bool flag = false;
                for (int s = 0; s < nsel && !flag; ++s) {
                    const double gm = gmax[s];
                    flag = gm > 0.0 && gradn[(int64_t)s * g.m + k] >= rel_thr * gm;
                }
                if (flag && x[k] > best) best = x[k];
            }
        }
    }
    xout[e] = best;
}

inline unsigned post_nb(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

void launch_sed(int dim, const Geo& g, const double* Ek, int q, int64_t ld, const double* Phi, const double* K0,
                double* sed, hipStream_t st) {
    if (dim == 2) hipLaunchKernelGGL(k_sed<2>, dim3(post_nb(g.m)), dim3(kBlock), 0, st, g, Ek, q, ld, Phi, K0, sed);
    else hipLaunchKernelGGL(k_sed<3>, dim3(post_nb(g.m)), dim3(kBlock), 0, st, g, Ek, q, ld, Phi, K0, sed);
}

int grad_tv_parts(const Geo& g) { return (int)std::min<int64_t>(post_nb(g.m), kMaxPartials); }

void launch_grad_tv(int dim, const Geo& g, const double* x, double xbar, int q, const double* sed, double* gradn,
                    double* part, hipStream_t st) {
    const dim3 gr(grad_tv_parts(g), q);
    if (dim == 2) hipLaunchKernelGGL(k_grad_tv<2>, gr, dim3(kBlock), 0, st, g, x, xbar, sed, gradn, part);
    else hipLaunchKernelGGL(k_grad_tv<3>, gr, dim3(kBlock), 0, st, g, x, xbar, sed, gradn, part);
}

void launch_dilate(int dim, const Geo& g, int nsel, const double* gradn, const double* gmax, double rel_thr,
                   double r_th, const double* x, double* xout, hipStream_t st) {
    const int R = (int)std::floor(r_th);
    const double r2 = r_th * r_th;
    if (dim == 2)
        hipLaunchKernelGGL(k_dilate<2>, dim3(post_nb(g.m)), dim3(kBlock), 0, st, g, nsel, gradn, gmax, rel_thr, R,
                           r2, x, xout);
    else
        hipLaunchKernelGGL(k_dilate<3>, dim3(post_nb(g.m)), dim3(kBlock), 0, st, g, nsel, gradn, gmax, rel_thr, R,
                           r2, x, xout);
}

}  // namespace mlb
