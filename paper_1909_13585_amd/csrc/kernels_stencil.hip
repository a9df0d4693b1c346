// Assembled node-block stencils for the Galerkin levels (j >= 2) and the
// coarse stress stiffness, plus the grid transfers.
//
// On the regular grid every row of a Galerkin operator couples a node with
// its 3^dim lattice neighbours only, so level j is stored as 3^dim dense
// dim x dim blocks per node ("node-block stencil"), entry-major with the node
// index fastest:
//     A[((nb * dim + c) * dim + c2) * nodes + node]      (vector operator K)
//     A[(nb * dim + c) * nodes + node]                   (block-diagonal G)
// nb = (dx+1) + 3 (dy+1) [+ 9 (dz+1)].  Dirichlet conditions are folded in
// when the stencil is assembled: K gets identity rows and zero columns at
// fixed DOFs, G zero rows and columns.  Entries of neighbours outside the
// grid are zero, so the apply clamps their addresses and reads no masks.
// The stored level-2 stencil of K is half the size of the element matrices
// it is summed from (3^3 x 9 vs 2^3 x 72 doubles per node).
// The FP32 copy of K's stencil that the mixed-precision cycle reads
// (assembled with af_half) keeps only the blocks nb <= NB/2 (the centre and the neighbours that come first
// in the node order): the operator is symmetric, so block nb > NB/2 of a node
// is the transpose of block NB-1-nb of that neighbour, and the apply reads
// it there.  That stores and streams 14 of 27 blocks (3D) per node.  Its
// blocks are node-major, Af[(nb * nodes + node) * dim^2 + c * dim + c2], so a
// thread reads a block with a few wide loads.
//
// Apply mapping: one thread per (node, column chunk) over all components
// (each stencil block and neighbour value loaded once for the node's rows),
// or per (node, component, column chunk) for one-column and block-diagonal
// calls, which need the threads; lanes run over consecutive nodes (coalesced
// stencil loads, stride-dim vector loads that hit the same cache lines).  Each XCD (blocks are dealt round robin
// over the 8 XCDs) works on one contiguous range of nodes with every
// component and column chunk, so the x values they share come from one L2.
#include "kernels.h"

namespace mlb {

constexpr int kXcd = 8;
constexpr int kNbThreads = 256;
constexpr int64_t kNbSplitBelow = 131072;   // (node, chunk) threads below which levels split components

template <int DIM>
struct Sten {
    static constexpr int ND = DIM;
    static constexpr int NN = 1 << DIM;
    static constexpr int NDE = DIM << DIM;
    static constexpr int NB = DIM == 2 ? 9 : 27;
};

__device__ inline void node_ijk(const Geo& g, int64_t node, int& i, int& j, int& k) {
    i = (int)(node % g.nnx);
    const int64_t r = node / g.nnx;
    j = (int)(r % g.nny);
    k = (int)(r / g.nny);
}

// XCD-aware decode of a 1-D grid into (node block, group).  Blocks are
// dealt round robin over the 8 XCDs; XCD x gets the contiguous node-block
// range [x P, (x+1) P) (P = padded node blocks / 8) with all groups of each
// node block, so neighbouring nodes' vector values are shared through one L2.
__device__ inline bool xcd_decode(int64_t nblocks_nodes, int ngroups, int64_t& nodeblk, int& grp) {
    const int64_t b = blockIdx.x;
    const int64_t xcd = b % kXcd, slot = b / kXcd;
    const int64_t per = (int64_t)gridDim.x / ngroups / kXcd;   // node blocks per XCD
    grp = (int)(slot % ngroups);
    nodeblk = xcd * per + slot / ngroups;
    return nodeblk < nblocks_nodes;
}

static dim3 xcd_grid(int64_t nodes, int ngroups) {
    const int64_t nbn = (nodes + kNbThreads - 1) / kNbThreads;
    const int64_t padded = (nbn + kXcd - 1) / kXcd * kXcd;
    return dim3((unsigned)(padded * ngroups), 1, 1);
}

// ---------------------------------------------------------------------------
// assembly from element matrices (SoA entry-major, [entry * m + e])

// Vector operator: thread per (node, c).  Row (node, c), block nb gathers
// the elements that contain both the node and its neighbour nb: along an axis
// with offset 0 the node may sit at either end of the element, with offset
// +-1 at exactly one.  Also writes the Jacobi diagonal inverse.
template <int DIM>
__global__ __launch_bounds__(kNbThreads) void k_assemble_nb(Geo g, const double* __restrict__ Ke,
                                                            const uint8_t* __restrict__ nmask, double* __restrict__ A,
                                                            float* __restrict__ Af, double* __restrict__ dinv,
                                                            float* __restrict__ dinvf, bool af_half) {
    using S = Sten<DIM>;
    const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (node >= g.nodes) return;
    int i, j, k;
    node_ijk(g, node, i, j, k);
    const uint8_t own = nmask[node];
    const bool own_fixed = (own >> c) & 1;
    const int64_t N = g.nodes;
    double diag = 0.0;
    for (int nb = 0; nb < S::NB; ++nb) {
        const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, DIM == 3 ? nb / 9 - 1 : 0};
        const int ii = i + d[0], jj = j + d[1], kk = k + d[2];
        const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny && kk >= 0 && kk < g.nnz;
        double s[DIM];
        for (int c2 = 0; c2 < DIM; ++c2) s[c2] = 0.0;
        if (ok && !own_fixed) {
            const uint8_t nm = nmask[ii + (int64_t)g.nnx * (jj + (int64_t)g.nny * kk)];
            for (int a = 0; a < S::NN; ++a) {
                const int ax = a & 1, ay = (a >> 1) & 1, az = DIM == 3 ? (a >> 2) & 1 : 0;
                const int bx = ax + d[0], by = ay + d[1], bz = az + d[2];
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                const int ei = i - ax, ej = j - ay, ek = k - az;
                if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
                const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
                const int b = bx + 2 * by + 4 * bz;
                for (int c2 = 0; c2 < DIM; ++c2)
                    s[c2] += Ke[(int64_t)((a * DIM + c) * S::NDE + b * DIM + c2) * g.m + e];
            }
            for (int c2 = 0; c2 < DIM; ++c2)
                if ((nm >> c2) & 1) s[c2] = 0.0;
        }
        if (own_fixed && nb == S::NB / 2) s[c] = 1.0;
        if (nb == S::NB / 2) diag = s[c];
        for (int c2 = 0; c2 < DIM; ++c2) {
            const int64_t at = (int64_t)((nb * DIM + c) * DIM + c2) * N + node;
            A[at] = s[c2];
            if (!af_half) Af[at] = (float)s[c2];
            else if (nb <= S::NB / 2) Af[((int64_t)nb * N + node) * (DIM * DIM) + c * DIM + c2] = (float)s[c2];
        }
    }
    const double v = own_fixed ? 1.0 : (diag > 0.0 ? 1.0 / diag : 0.0);
    dinv[node * DIM + c] = v;
    dinvf[node * DIM + c] = (float)v;
}

// Block-diagonal operator from scalar element matrices g_e (nn x nn,
// [ (a*nn + b) * m + e ]), masked on both sides per component.
template <int DIM>
__global__ __launch_bounds__(kNbThreads) void k_assemble_nb_diag(Geo g, const double* __restrict__ Ge,
                                                                 const uint8_t* __restrict__ nmask,
                                                                 double* __restrict__ A) {
    using S = Sten<DIM>;
    const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (node >= g.nodes) return;
    int i, j, k;
    node_ijk(g, node, i, j, k);
    const uint8_t own = nmask[node];
    const int64_t N = g.nodes;
    for (int nb = 0; nb < S::NB; ++nb) {
        const int d[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, DIM == 3 ? nb / 9 - 1 : 0};
        const int ii = i + d[0], jj = j + d[1], kk = k + d[2];
        const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny && kk >= 0 && kk < g.nnz;
        double s = 0.0;
        uint8_t nm = 0xff;
        if (ok) {
            nm = nmask[ii + (int64_t)g.nnx * (jj + (int64_t)g.nny * kk)];
            for (int a = 0; a < S::NN; ++a) {
                const int ax = a & 1, ay = (a >> 1) & 1, az = DIM == 3 ? (a >> 2) & 1 : 0;
                const int bx = ax + d[0], by = ay + d[1], bz = az + d[2];
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
                const int ei = i - ax, ej = j - ay, ek = k - az;
                if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
                const int64_t e = ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek);
                const int b = bx + 2 * by + 4 * bz;
                s += Ge[(int64_t)(a * S::NN + b) * g.m + e];
            }
        }
        for (int c = 0; c < DIM; ++c) {
            const bool z = ((own >> c) & 1) || ((nm >> c) & 1);
            A[(int64_t)(nb * DIM + c) * N + node] = z ? 0.0 : s;
        }
    }
}

// ---------------------------------------------------------------------------
// apply: y = A x | r - A x | x + omega D^-1 (r - A x), CB columns per thread

template <typename T, int MODE>
__device__ inline T nb_epilogue(T ax, T xown, T rr, T di, T omega) {
    if (MODE == kModeY) return ax;
    if (MODE == kModeResidual) return rr - ax;
    return xown + omega * di * (rr - ax);
}

template <int DIM, typename T, int MODE, int CB, bool DIAG, bool SPLITC>
__global__ __launch_bounds__(kNbThreads) void k_apply_nb(Geo g, int64_t nblk_nodes, int nchunks,
                                                         const T* __restrict__ A, int ncols, int64_t ld,
                                                         const T* __restrict__ x, T* __restrict__ y,
                                                         const T* __restrict__ r, const T* __restrict__ dinv,
                                                         T omega) {
    // SPLITC: thread per (node, component, column chunk), for few columns
    // (enough threads).  Otherwise thread per (node, column chunk) over all
    // DIM components of the node, so each neighbour value and stencil block
    // is loaded once for the node's rows and all columns.  Every output sums
    // the same terms in the same order either way.
    using S = Sten<DIM>;
    // FP32 operator stencils are stored by half, node-major (see the top of
    // this file); their one-component threads run DOF-major (lanes over the
    // components of consecutive nodes, so a lane's stencil row is the next
    // lane's neighbour in memory); nblk_nodes then counts blocks of DOFs
    constexpr bool HALF = sizeof(T) == 4 && !DIAG;
    constexpr bool DOFS = SPLITC && HALF;
    int64_t nbk;
    int grp;
    if (!xcd_decode(nblk_nodes, SPLITC && !DOFS ? DIM * nchunks : nchunks, nbk, grp)) return;
    const int64_t tix = nbk * kNbThreads + threadIdx.x;
    const int64_t node = DOFS ? tix / DIM : tix;
    if (node >= g.nodes) return;
    int i, j, k;
    node_ijk(g, node, i, j, k);
    const int64_t N = g.nodes;
    const int64_t sy = g.nnx, sz = (int64_t)g.nnx * g.nny;
    if constexpr (SPLITC) {
        const int c = DOFS ? (int)(tix - node * DIM) : grp % DIM;
        const int c0 = (DOFS ? grp : grp / DIM) * CB;
        const int nq = min(CB, ncols - c0);
        const T* xb = x + (int64_t)c0 * ld;
        T acc[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) acc[q] = T(0);
#pragma unroll
        for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
            const bool okz = k + dz >= 0 && k + dz < g.nnz;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const bool oky = okz && j + dy >= 0 && j + dy < g.nny;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const bool ok = oky && i + dx >= 0 && i + dx < g.nnx;
                    const int nb = (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
                    const int64_t nbn = ok ? node + dx + sy * dy + sz * dz : node;
                    if (DIAG) {
                        const T a = A[(int64_t)(nb * DIM + c) * N + node];
#pragma unroll
                        for (int q = 0; q < CB; ++q)
                            if (q < nq) acc[q] += a * xb[q * ld + nbn * DIM + c];
                    } else {
                        T a[DIM];
#pragma unroll
                        for (int c2 = 0; c2 < DIM; ++c2)
                            a[c2] = !HALF ? A[(int64_t)((nb * DIM + c) * DIM + c2) * N + node]
                                    : nb <= S::NB / 2
                                        ? A[((int64_t)nb * N + node) * (DIM * DIM) + c * DIM + c2]
                                        : (ok ? A[((int64_t)(S::NB - 1 - nb) * N + nbn) * (DIM * DIM) + c2 * DIM + c]
                                              : T(0));
#pragma unroll
                        for (int q = 0; q < CB; ++q)
                            if (q < nq)
#pragma unroll
                                for (int c2 = 0; c2 < DIM; ++c2) acc[q] += a[c2] * xb[q * ld + nbn * DIM + c2];
                    }
                }
            }
        }
        const int64_t d = node * DIM + c;
        const T di = MODE == kModeJacobi ? dinv[d] : T(0);
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            if (q >= nq) break;
            const int64_t o = (int64_t)(c0 + q) * ld + d;
            const T xown = MODE == kModeJacobi ? x[o] : T(0);
            const T rr = MODE == kModeY ? T(0) : r[o];
            y[o] = nb_epilogue<T, MODE>(acc[q], xown, rr, di, omega);
        }
    } else {
        const int c0 = grp * CB;
        const int nq = min(CB, ncols - c0);
        const T* xb = x + (int64_t)c0 * ld;
        T acc[DIM][CB];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int q = 0; q < CB; ++q) acc[c][q] = T(0);
#pragma unroll
        for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
            const bool okz = k + dz >= 0 && k + dz < g.nnz;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const bool oky = okz && j + dy >= 0 && j + dy < g.nny;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const bool ok = oky && i + dx >= 0 && i + dx < g.nnx;
                    const int nb = (dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0);
                    const int64_t nbn = ok ? node + dx + sy * dy + sz * dz : node;
                    // the neighbour's block of the stencil, once for all columns
                    T a[DIM][DIM];
#pragma unroll
                    for (int c = 0; c < DIM; ++c)
#pragma unroll
                        for (int c2 = 0; c2 < DIM; ++c2)
                            a[c][c2] = DIAG ? (c2 == c ? A[(int64_t)(nb * DIM + c) * N + node] : T(0))
                                       : !HALF ? A[(int64_t)((nb * DIM + c) * DIM + c2) * N + node]
                                       : nb <= S::NB / 2
                                           ? A[((int64_t)nb * N + node) * (DIM * DIM) + c * DIM + c2]
                                           // unconditional (nbn is the node itself off the grid),
                                           // so the block's loads merge; zero selected after
                                           : A[((int64_t)(S::NB - 1 - nb) * N + nbn) * (DIM * DIM) + c2 * DIM + c];
                    if (HALF && nb > S::NB / 2 && !ok)
#pragma unroll
                        for (int c = 0; c < DIM; ++c)
#pragma unroll
                            for (int c2 = 0; c2 < DIM; ++c2) a[c][c2] = T(0);
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        if (q >= nq) break;
                        T xv[DIM];
#pragma unroll
                        for (int c2 = 0; c2 < DIM; ++c2) xv[c2] = xb[q * ld + nbn * DIM + c2];
#pragma unroll
                        for (int c = 0; c < DIM; ++c) {
                            if (DIAG) {
                                acc[c][q] += a[c][c] * xv[c];
                            } else {
#pragma unroll
                                for (int c2 = 0; c2 < DIM; ++c2) acc[c][q] += a[c][c2] * xv[c2];
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const int64_t d = node * DIM + c;
            const T di = MODE == kModeJacobi ? dinv[d] : T(0);
#pragma unroll
            for (int q = 0; q < CB; ++q) {
                if (q >= nq) break;
                const int64_t o = (int64_t)(c0 + q) * ld + d;
                const T xown = MODE == kModeJacobi ? x[o] : T(0);
                const T rr = MODE == kModeY ? T(0) : r[o];
                y[o] = nb_epilogue<T, MODE>(acc[c][q], xown, rr, di, omega);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// transfers: nodal (bi/tri)linear interpolation P and its transpose, masked
// on both sides.  Thread per (node, column) over all DIM components: each
// neighbour's mask and its DIM contiguous vector values are loaded once for
// the node; consecutive threads take consecutive nodes of one column, so the
// fine-side (prolongation) and coarse-side (restriction) vectors are read
// and written contiguously.
template <int DIM, typename T, bool ADD>
__global__ __launch_bounds__(kNbThreads) void k_prolong_nb(Geo gf, Geo gc, int64_t nblk_nodes, int ncols,
                                                           const uint8_t* __restrict__ mf,
                                                           const uint8_t* __restrict__ mc, int64_t ldf,
                                                           int64_t ldc, const T* __restrict__ xc,
                                                           T* __restrict__ yf) {
    int64_t nbk;
    int col;
    if (!xcd_decode(nblk_nodes, ncols, nbk, col)) return;
    const int64_t node = nbk * kNbThreads + threadIdx.x;
    if (node >= gf.nodes) return;
    int i, j, k;
    node_ijk(gf, node, i, j, k);
    const uint8_t fm = mf[node];
    const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (DIM == 3 && (k & 1)) ? 2 : 1;
    const T* xcol = xc + (int64_t)col * ldc;
    T acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = T(0);
#pragma unroll
    for (int dk = 0; dk < (DIM == 3 ? 2 : 1); ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                if (di >= ni || dj >= nj || dk >= nk) continue;
                const int64_t cn = (i0 + di) + (int64_t)gc.nnx * ((j0 + dj) + (int64_t)gc.nny * (k0 + dk));
                const uint8_t cm = mc[cn];
                T v[DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) v[c] = xcol[cn * DIM + c];
#pragma unroll
                for (int c = 0; c < DIM; ++c) acc[c] += ((cm >> c) & 1) ? T(0) : v[c];
            }
    const T w = T(1) / T(ni * nj * nk);
    T* ycol = yf + (int64_t)col * ldf + node * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if ((fm >> c) & 1) {
            if (!ADD) ycol[c] = T(0);
        } else {
            ycol[c] = ADD ? ycol[c] + w * acc[c] : w * acc[c];
        }
    }
}

template <int DIM, typename T>
__global__ __launch_bounds__(kNbThreads) void k_restrict_nb(Geo gf, Geo gc, int64_t nblk_nodes, int ncols,
                                                            const uint8_t* __restrict__ mf,
                                                            const uint8_t* __restrict__ mc, int64_t ldf,
                                                            int64_t ldc, const T* __restrict__ xf,
                                                            T* __restrict__ yc) {
    int64_t nbk;
    int col;
    if (!xcd_decode(nblk_nodes, ncols, nbk, col)) return;
    const int64_t cnode = nbk * kNbThreads + threadIdx.x;
    if (cnode >= gc.nodes) return;
    int I, J, K;
    node_ijk(gc, cnode, I, J, K);
    const uint8_t cm = mc[cnode];
    const T* xcol = xf + (int64_t)col * ldf;
    T acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = T(0);
#pragma unroll
    for (int dk = (DIM == 3 ? -1 : 0); dk <= (DIM == 3 ? 1 : 0); ++dk) {
        const int kk = 2 * K + dk;
        const bool okk = kk >= 0 && kk < gf.nnz;
        const T wk = dk == 0 ? T(1) : T(0.5);
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const int jj = 2 * J + dj;
            const bool okj = okk && jj >= 0 && jj < gf.nny;
            const T wj = dj == 0 ? wk : wk * T(0.5);
#pragma unroll
            for (int di = -1; di <= 1; ++di) {
                const int ii = 2 * I + di;
                const bool ok = okj && ii >= 0 && ii < gf.nnx;
                const T w = di == 0 ? wj : wj * T(0.5);
                const int64_t fn = ok ? ii + (int64_t)gf.nnx * (jj + (int64_t)gf.nny * kk) : 0;
                const uint8_t fmk = mf[fn];
                T v[DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) v[c] = xcol[fn * DIM + c];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const bool use = ok && !((fmk >> c) & 1);
                    acc[c] += use ? w * v[c] : T(0);
                }
            }
        }
    }
    T* ycol = yc + (int64_t)col * ldc + cnode * DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) ycol[c] = ((cm >> c) & 1) ? T(0) : acc[c];
}

// ---------------------------------------------------------------------------
// host launchers

void launch_assemble_nb(int dim, const Geo& g, const double* Ke, const uint8_t* nmask, double* A, float* Af,
                        double* dinv, float* dinvf, bool af_half, hipStream_t st) {
    const dim3 gr((unsigned)((g.nodes + kNbThreads - 1) / kNbThreads), dim, 1);
    if (dim == 2)
        hipLaunchKernelGGL(k_assemble_nb<2>, gr, dim3(kNbThreads), 0, st, g, Ke, nmask, A, Af, dinv, dinvf, af_half);
    else
        hipLaunchKernelGGL(k_assemble_nb<3>, gr, dim3(kNbThreads), 0, st, g, Ke, nmask, A, Af, dinv, dinvf, af_half);
}

void launch_assemble_nb_diag(int dim, const Geo& g, const double* Ge, const uint8_t* nmask, double* A,
                             hipStream_t st) {
    const dim3 gr((unsigned)((g.nodes + kNbThreads - 1) / kNbThreads), 1, 1);
    if (dim == 2) hipLaunchKernelGGL(k_assemble_nb_diag<2>, gr, dim3(kNbThreads), 0, st, g, Ge, nmask, A);
    else hipLaunchKernelGGL(k_assemble_nb_diag<3>, gr, dim3(kNbThreads), 0, st, g, Ge, nmask, A);
}

int64_t stencil_entries(int dim, const Geo& g, bool diag, bool half) {
    const int nb = dim == 2 ? (half ? 5 : 9) : (half ? 14 : 27);
    return (int64_t)nb * dim * (diag ? 1 : dim) * g.nodes;
}

template <typename T>
void launch_apply_nb(int dim, const Geo& g, const T* A, bool diag, int ncols, int64_t ld, const T* x, T* y, int mode,
                     const T* r, const T* dinv, T omega, int cbmax, hipStream_t st) {
    const int64_t nbn = (g.nodes + kNbThreads - 1) / kNbThreads;
    // columns per thread: at most cbmax (tunable, default 6), split evenly;
    // each chunk re-reads the stencil, wider chunks run fewer threads
    const int cap = cbmax >= 1 && cbmax <= 12 ? cbmax : 6;
    const int per = (ncols + cap - 1) / cap;
    const int want = (ncols + per - 1) / per;
    const int cb = want <= 1 ? 1 : want <= 2 ? 2 : want <= 3 ? 3 : want <= 4 ? 4 : want <= 6 ? 6 : want <= 8 ? 8 : 12;
    const int nchunks = (ncols + cb - 1) / cb;
    // one-column calls, DIAG and small levels (whose node threads alone would
    // leave most SIMDs idle) keep a thread per component: enough threads
    // (FP32 operator stencils: DOF-major threads, nbn counting DOF blocks)
    const bool split = ncols == 1 || diag || g.nodes * nchunks < kNbSplitBelow;
    const bool dofs = split && sizeof(T) == 4 && !diag;
    const int64_t nbn_s = dofs ? (g.nodes * dim + kNbThreads - 1) / kNbThreads : nbn;
    const dim3 gr = dofs ? xcd_grid(g.nodes * dim, nchunks) : xcd_grid(g.nodes, split ? dim * nchunks : nchunks);
    const dim3 b(kNbThreads);
#define MLB_NB(D, M, C, DG)                                                                                         \
    do {                                                                                                            \
        if (split)                                                                                                  \
            hipLaunchKernelGGL((k_apply_nb<D, T, M, C, DG, true>), gr, b, 0, st, g, nbn_s, nchunks, A, ncols, ld,  \
                               x, y, r, dinv, omega);                                                               \
        else                                                                                                        \
            hipLaunchKernelGGL((k_apply_nb<D, T, M, C, DG, false>), gr, b, 0, st, g, nbn, nchunks, A, ncols, ld, x, \
                               y, r, dinv, omega);                                                                  \
    } while (0)
#define MLB_NB_M(D, C)                                             \
    do {                                                           \
        if (diag) MLB_NB(D, kModeY, C, true);                      \
        else if (mode == kModeY) MLB_NB(D, kModeY, C, false);      \
        else if (mode == kModeResidual) MLB_NB(D, kModeResidual, C, false); \
        else MLB_NB(D, kModeJacobi, C, false);                     \
    } while (0)
#define MLB_NB_C(D)                       \
    do {                                  \
        if (cb == 1) MLB_NB_M(D, 1);      \
        else if (cb == 2) MLB_NB_M(D, 2); \
        else if (cb == 3) MLB_NB_M(D, 3); \
        else if (cb == 4) MLB_NB_M(D, 4); \
        else if (cb == 6) MLB_NB_M(D, 6); \
        else if (cb == 8) MLB_NB_M(D, 8); \
        else MLB_NB_M(D, 12);             \
    } while (0)
    if (dim == 2) MLB_NB_C(2);
    else MLB_NB_C(3);
#undef MLB_NB_C
#undef MLB_NB_M
#undef MLB_NB
}

template <typename T>
void launch_prolong_nb(int dim, const Geo& gf, const Geo& gc, const uint8_t* mf, const uint8_t* mc, int ncols,
                       int64_t ldf, int64_t ldc, const T* xc, T* yf, bool add, hipStream_t st) {
    const int64_t nbn = (gf.nodes + kNbThreads - 1) / kNbThreads;
    const dim3 gr = xcd_grid(gf.nodes, ncols);
    const dim3 b(kNbThreads);
#define MLB_P(D, AD) \
    hipLaunchKernelGGL((k_prolong_nb<D, T, AD>), gr, b, 0, st, gf, gc, nbn, ncols, mf, mc, ldf, ldc, xc, yf)
    if (dim == 2) {
        if (add) MLB_P(2, true);
        else MLB_P(2, false);
    } else {
        if (add) MLB_P(3, true);
        else MLB_P(3, false);
    }
#undef MLB_P
}

template <typename T>
void launch_restrict_nb(int dim, const Geo& gf, const Geo& gc, const uint8_t* mf, const uint8_t* mc, int ncols,
                        int64_t ldf, int64_t ldc, const T* xf, T* yc, hipStream_t st) {
    const int64_t nbn = (gc.nodes + kNbThreads - 1) / kNbThreads;
    const dim3 gr = xcd_grid(gc.nodes, ncols);
    const dim3 b(kNbThreads);
    if (dim == 2)
        hipLaunchKernelGGL((k_restrict_nb<2, T>), gr, b, 0, st, gf, gc, nbn, ncols, mf, mc, ldf, ldc, xf, yc);
    else
        hipLaunchKernelGGL((k_restrict_nb<3, T>), gr, b, 0, st, gf, gc, nbn, ncols, mf, mc, ldf, ldc, xf, yc);
}

template void launch_apply_nb<double>(int, const Geo&, const double*, bool, int, int64_t, const double*, double*,
                                      int, const double*, const double*, double, int, hipStream_t);
template void launch_apply_nb<float>(int, const Geo&, const float*, bool, int, int64_t, const float*, float*, int,
                                     const float*, const float*, float, int, hipStream_t);
template void launch_prolong_nb<double>(int, const Geo&, const Geo&, const uint8_t*, const uint8_t*, int, int64_t,
                                        int64_t, const double*, double*, bool, hipStream_t);
template void launch_prolong_nb<float>(int, const Geo&, const Geo&, const uint8_t*, const uint8_t*, int, int64_t,
                                       int64_t, const float*, float*, bool, hipStream_t);
template void launch_restrict_nb<double>(int, const Geo&, const Geo&, const uint8_t*, const uint8_t*, int, int64_t,
                                         int64_t, const double*, double*, hipStream_t);
template void launch_restrict_nb<float>(int, const Geo&, const Geo&, const uint8_t*, const uint8_t*, int, int64_t,
                                        int64_t, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// Kaczmarz sweep for (K + sigma G) x = 0 on a Galerkin level, every column of
// X.  Rows are visited colour by colour, colour (i mod 3) + 3 (j mod 3) +
// 9 (k mod 3) in increasing order: a row couples a node to its 3^d
// neighbours only, so the rows of the nodes of one colour touch disjoint
// columns and one thread per (node, column of X) applies the node's rows
// (components in increasing order) without conflicts; the columns of X are
// independent systems.  The result equals the row-by-row sweep in that
// order.  Each free row r projects x onto a_r . x = 0; Dirichlet rows are
// skipped.  K: full node-block stencil, G: block-diagonal stencil.
constexpr int kKzThreads = 64;

template <int DIM>
__global__ __launch_bounds__(kKzThreads) void k_kaczmarz_color(Geo g, int cx, int cy, int cz,
                                                               const double* __restrict__ A,
                                                               const double* __restrict__ Gd, double sigma,
                                                               const uint8_t* __restrict__ nmask, int ncols,
                                                               int64_t ld, double* __restrict__ X) {
    constexpr int NB = DIM == 3 ? 27 : 9;
    const int mx = (g.nnx - cx + 2) / 3, my = (g.nny - cy + 2) / 3;
    const int mz = DIM == 3 ? (g.nnz - cz + 2) / 3 : 1;
    const int64_t nodes_c = (int64_t)mx * my * mz;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tid >= nodes_c * ncols) return;
    const int q = (int)(tid / nodes_c);
    const int64_t t = tid % nodes_c;
    const int i = cx + 3 * (int)(t % mx);
    const int j = cy + 3 * (int)((t / mx) % my);
    const int k = DIM == 3 ? cz + 3 * (int)(t / ((int64_t)mx * my)) : 0;
    const int64_t N = g.nodes, sy = g.nnx, sz = (int64_t)g.nnx * g.nny;
    const int64_t node = i + sy * j + sz * k;
    const unsigned m = nmask[node];
    double* Xq = X + (int64_t)q * ld;
    auto nb_ok = [&](int nb) -> bool {
        const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = DIM == 3 ? nb / 9 - 1 : 0;
        return i + dx >= 0 && i + dx < g.nnx && j + dy >= 0 && j + dy < g.nny &&
               (DIM == 2 || (k + dz >= 0 && k + dz < g.nnz));
    };
    auto nb_node = [&](int nb) -> int64_t {
        const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = DIM == 3 ? nb / 9 - 1 : 0;
        return node + dx + sy * dy + sz * dz;
    };
    auto coef = [&](int nb, int c, int c2) -> double {
        const double a = A[(int64_t)((nb * DIM + c) * DIM + c2) * N + node];
        return c2 == c ? a + sigma * Gd[(int64_t)(nb * DIM + c) * N + node] : a;
    };
    for (int c = 0; c < DIM; ++c) {
        if ((m >> c) & 1u) continue;
        double nrm = 0.0, res = 0.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            if (!nb_ok(nb)) continue;
            const int64_t o = nb_node(nb) * DIM;
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) {
                const double a = coef(nb, c, c2);
                nrm += a * a;
                res += a * Xq[o + c2];
            }
        }
        if (!(nrm > 0.0)) continue;
        const double tq = res / nrm;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            if (!nb_ok(nb)) continue;
            const int64_t o = nb_node(nb) * DIM;
#pragma unroll
            for (int c2 = 0; c2 < DIM; ++c2) Xq[o + c2] -= tq * coef(nb, c, c2);
        }
    }
}

void launch_kaczmarz_sweep(int dim, const Geo& g, const double* A, const double* Gd, double sigma,
                           const uint8_t* nmask, int ncols, int64_t ld, double* X, hipStream_t st) {
    const int ncol = dim == 3 ? 27 : 9;
    for (int col = 0; col < ncol; ++col) {
        const int cx = col % 3, cy = (col / 3) % 3, cz = col / 9;
        const int64_t mx = (g.nnx - cx + 2) / 3, my = (g.nny - cy + 2) / 3;
        const int64_t mz = dim == 3 ? (g.nnz - cz + 2) / 3 : 1;
        const int64_t th = mx * my * mz * ncols;
        if (th <= 0) continue;
        const dim3 gr((unsigned)((th + kKzThreads - 1) / kKzThreads)), b(kKzThreads);
        if (dim == 3)
            hipLaunchKernelGGL(k_kaczmarz_color<3>, gr, b, 0, st, g, cx, cy, cz, A, Gd, sigma, nmask, ncols, ld, X);
        else
            hipLaunchKernelGGL(k_kaczmarz_color<2>, gr, b, 0, st, g, cx, cy, cz, A, Gd, sigma, nmask, ncols, ld, X);
    }
}

}  // namespace mlb
