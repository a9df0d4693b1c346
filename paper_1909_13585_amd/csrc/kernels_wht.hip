// Level-1 stiffness apply, element-centric, in the symmetry-adapted
// Walsh-Hadamard basis of the unit element.
//
// The unit square/cube element is invariant under the dim mid-plane
// reflections.  Transforming each displacement component over the 2^dim
// element nodes with the Walsh-Hadamard matrix H (H[k][a] = (-1)^popcount(k&a))
// and grouping component c at index sigma ^ (1 << c) splits K0 exactly into
// 2^dim independent dim x dim blocks B_sigma:
//     K0 u = H diag(B_sigma) H u / 4^dim      (per element, times E_e)
// i.e. ~ 200 operations per element instead of the 1152 of a dense 24 x 24
// product.  Because the cell is also symmetric under axis permutations, the
// blocks are made of 9 (3D) or 5 (2D) numbers (with the 1/4^dim folded in);
// they arrive as kernel arguments and stay in scalar registers.
//
// Traversal: each thread walks a pencil of elements along the slowest axis
// (z in 3D, y in 2D), carrying the shared node plane and the partial sums of
// the next node plane in registers.  The contributions of the element columns
// that share a node are combined with lane shuffles, always in the same
// order, so the result is deterministic (no atomics) and no barriers are
// needed.  Tiles overlap by one element column/row; a thread owns the node
// at the low corner of its element column.
#include "kernels.h"

namespace mlb {

// 3D: d0, o0, d7, o7, e1, f1, g2d, g2o, h2;  2D: d0, o0, q1, d3, o3
template <typename T>
struct WhtBlocks {
    T v[9];
};

__device__ inline double shfl_up_w(double v, int d, int width) { return __shfl_up(v, d, width); }
__device__ inline float shfl_up_w(float v, int d, int width) { return __shfl_up(v, d, width); }

// In-place 2^DIM-point Walsh-Hadamard transform of s[0 .. 2^DIM).
template <int DIM, typename T>
__device__ inline void wht(T* s) {
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
        for (int a = 0; a < (1 << DIM); ++a)
            if (!((a >> b) & 1)) {
                const T p = s[a], q = s[a | (1 << b)];
                s[a] = p + q;
                s[a | (1 << b)] = p - q;
            }
}

// out[a][c] = E * (H diag(B) H u)[a][c] for one element; component c of
// block sigma sits at Walsh index sigma ^ (1 << c).
template <int DIM, typename T>
__device__ inline void element_apply(const WhtBlocks<T>& B, T Ee, T (&u)[DIM][1 << DIM]) {
    constexpr int NN = 1 << DIM;
#pragma unroll
    for (int c = 0; c < DIM; ++c) wht<DIM, T>(u[c]);
    if constexpr (DIM == 3) {
        const T d0 = B.v[0], o0 = B.v[1], d7 = B.v[2], o7 = B.v[3], e1 = B.v[4], f1 = B.v[5], g2d = B.v[6],
                g2o = B.v[7], h2 = B.v[8];
        {   // sigma = 0: components at 1, 2, 4
            const T a = u[0][1], b = u[1][2], c3 = u[2][4];
            const T sum = o0 * (a + b + c3), dd = d0 - o0;
            u[0][1] = dd * a + sum;
            u[1][2] = dd * b + sum;
            u[2][4] = dd * c3 + sum;
        }
        {   // sigma = 7: components at 6, 5, 3
            const T a = u[0][6], b = u[1][5], c3 = u[2][3];
            const T sum = o7 * (a + b + c3), dd = d7 - o7;
            u[0][6] = dd * a + sum;
            u[1][5] = dd * b + sum;
            u[2][3] = dd * c3 + sum;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            // sigma = 1 << c: component c is a rigid translation (index 0),
            // components c1, c2 at indices with bits {c, c1} and {c, c2}
            const int i1 = (1 << c) | (1 << c1), i2 = (1 << c) | (1 << c2);
            const T v1 = u[c1][i1], v2 = u[c2][i2];
            u[c1][i1] = e1 * v1 + f1 * v2;
            u[c2][i2] = f1 * v1 + e1 * v2;
            u[c][0] = T(0);
            // sigma = 7 ^ (1 << c): components c1, c2 at indices 1 << c2 and
            // 1 << c1, component c at index 7
            const T w1 = u[c1][1 << c2], w2 = u[c2][1 << c1];
            u[c1][1 << c2] = g2d * w1 + g2o * w2;
            u[c2][1 << c1] = g2o * w1 + g2d * w2;
            u[c][7] = h2 * u[c][7];
        }
    } else {
        const T d0 = B.v[0], o0 = B.v[1], q1 = B.v[2], d3 = B.v[3], o3 = B.v[4];
        {   // sigma = 0: components at 1, 2
            const T a = u[0][1], b = u[1][2];
            u[0][1] = d0 * a + o0 * b;
            u[1][2] = o0 * a + d0 * b;
        }
        {   // sigma = 3: components at 2, 1
            const T a = u[0][2], b = u[1][1];
            u[0][2] = d3 * a + o3 * b;
            u[1][1] = o3 * a + d3 * b;
        }
        // sigma = 1: component 0 is a translation, component 1 at 3;
        // sigma = 2: component 1 is a translation, component 0 at 3
        u[0][0] = T(0);
        u[1][0] = T(0);
        u[1][3] = q1 * u[1][3];
        u[0][3] = q1 * u[0][3];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        wht<DIM, T>(u[c]);
#pragma unroll
        for (int a = 0; a < NN; ++a) u[c][a] *= Ee;
    }
}

template <typename T, int MODE>
__device__ inline T wht_epilogue(T ax, T xown, T rr, T di, T omega) {
    if (MODE == kModeY) return ax;
    if (MODE == kModeResidual) return rr - ax;
    return xown + omega * di * (rr - ax);
}

__device__ inline double wht_block_sum(double v, double* sh) {
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nthreads = blockDim.x * blockDim.y;
    const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0)
        for (int w = 0; w < nw; ++w) r += sh[w];
    return r;
}

// ---------------------------------------------------------------------------
// 3D: every wavefront is an independent 8 x 8 tile of element columns
// (lane = tx + 8 ty) walking a pencil along z; tiles overlap by one column/row
// and lanes with tx, ty >= 1 own the node at the low corner of their column.
// x partners come from lane-1, y partners from lane-8 (shuffles, no
// barriers); the next node plane is prefetched one step ahead.
constexpr int kWT = 8;          // tile edge (element columns per wave edge)
constexpr int kW3 = 4;          // waves per block
constexpr int kXcd3 = 8;        // XCDs the blocks are dealt over

#ifndef MLB_WHT3_WAVES
#define MLB_WHT3_WAVES 2
#endif

// Work of one block of a 3D apply launched with `cgrid` column groups on the
// grid (gridDim.x = cgrid x tile blocks, tile blocks a multiple of kXcd3).
// Block b runs on XCD b mod kXcd3; the tile blocks of each XCD form one
// contiguous range of the tile order, and the cgrid groups of a tile block
// are consecutive there.  `slot` is the block's index in a launch with one
// group (partial dot products go to part[col * nblk + slot], so every column
// is reduced in the same order whatever cgrid is).
struct WhtSlot {
    int64_t bl, slot, nblk;
    int c0, c1;
};
__device__ inline WhtSlot wht_slot(int cgrid, int ncols) {
    WhtSlot s;
    s.nblk = gridDim.x / cgrid;
    const int64_t per_xcd = s.nblk / kXcd3;
    const int64_t li = blockIdx.x / kXcd3;
    const int grp = (int)(li % cgrid);
    s.bl = (blockIdx.x % kXcd3) * per_xcd + li / cgrid;
    s.slot = (s.bl % per_xcd) * kXcd3 + s.bl / per_xcd;
    const int per = (ncols + cgrid - 1) / cgrid;
    s.c0 = grp * per;
    s.c1 = min(ncols, s.c0 + per);
    return s;
}
// CLEAN: the caller guarantees x == 0 at every Dirichlet DOF (true for every
// vector inside the solvers), so neighbour values need no masking; only the
// owned node's mask is read (identity rows).
// PF: prefetch the next node plane one step ahead (more registers, fewer
// waves per SIMD); without it the next plane is loaded at the end of a step
// and latency is hidden by the other waves only.
template <typename T, int MODE, bool DOT, bool CLEAN, bool PF>
__global__ __launch_bounds__(64 * kW3) __attribute__((amdgpu_waves_per_eu(PF || DOT ? MLB_WHT3_WAVES : 3, 8))) void k_apply_wht3(
    Geo g, int kz_chunk, int ntiles_x, int ntiles_y, const T* __restrict__ E, const uint8_t* __restrict__ nmask,
    WhtBlocks<T> B, int ncols, int64_t ld, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ r,
    const T* __restrict__ dinv, T omega, double* __restrict__ part, int cgrid) {
    __shared__ double sh[16];
    const int lane = threadIdx.x;              // 0..63
    const int tx = lane & 7, ty = lane >> 3;
    // Blocks are dealt round robin over the 8 XCDs; each XCD gets one
    // contiguous range of the (z-chunk major) tile order, so the node planes
    // and columns that neighbouring tiles share are re-read from its own L2.
    // With cgrid column groups on the grid, the groups of one tile block are
    // consecutive on the same XCD (its modulus, masks and diagonal are read
    // from HBM once and then from that L2).
    const WhtSlot sl = wht_slot(cgrid, ncols);
    const int64_t bl = sl.bl;
    const int64_t tile = bl * kW3 + threadIdx.y;
    const int64_t ntile_xy = (int64_t)ntiles_x * ntiles_y;
    const int tzc = (int)(tile / ntile_xy);
    const int txy = (int)(tile % ntile_xy);
    const int ie = (txy % ntiles_x) * (kWT - 1) - 1 + tx;
    const int je = (txy / ntiles_x) * (kWT - 1) - 1 + ty;
    const int kz0 = tzc * kz_chunk;
    const int kend = min(kz0 + kz_chunk, g.nnz);
    const bool col_ok = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny;
    const bool owner = tx >= 1 && ty >= 1 && ie >= 0 && je >= 0 && ie <= g.nx && je <= g.ny;
    const int64_t plane = (int64_t)g.nnx * g.nny;
    const int64_t eplane = (int64_t)g.nx * g.ny;
    const int64_t nblk = sl.nblk;
    // per-lane node columns (ie+ax, je+ay): in-plane index and validity
    int64_t base[4];
    bool qok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ii = ie + (q & 1), jj = je + (q >> 1);
        qok[q] = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny;
        base[q] = qok[q] ? ii + (int64_t)g.nnx * jj : 0;
    }
    const int64_t ebase = col_ok ? ie + (int64_t)g.nx * je : 0;
    for (int col = sl.c0; col < sl.c1; ++col) {
        const T* xc = x + col * ld;
        double dsum = 0.0;
        // values (and, unless CLEAN, masks) of the 4 nodes of node plane kk;
        // clamped addresses keep every load valid and branch free
        auto fetch = [&](int kk, T (&v)[3][4], uint8_t (&mk)[4]) {
            const bool kin = kk >= 0 && kk < g.nnz;
            const int64_t off = kin ? plane * kk : 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = qok[q] && kin;
                const int64_t nd = base[q] + off;
                if (!CLEAN || q == 0) {
                    const uint8_t mraw = nmask[nd];
                    mk[q] = ok ? mraw : (uint8_t)0x07;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T xv = xc[nd * 3 + c];
                    v[c][q] = ok ? xv : T(0);
                }
            }
        };
        T lo[3][4], hi[3][4], pf[3][4];
        uint8_t mlo[4], mhi[4], mpf[4];
        T cout[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) cout[c][q] = T(0);
        fetch(kz0 - 1, lo, mlo);
        fetch(kz0, hi, mhi);
        for (int ke = kz0 - 1; ke < kend; ++ke) {
            if (PF) fetch(ke + 2, pf, mpf);   // prefetch for the next step
            const bool eok = col_ok && ke >= 0 && ke < g.nz;
            const T Eraw = E[eok ? ebase + eplane * ke : 0];
            const T Ee = eok ? Eraw : T(0);
            T u[3][8];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (CLEAN) {
                        u[c][q] = lo[c][q];
                        u[c][q + 4] = hi[c][q];
                    } else {
                        u[c][q] = ((mlo[q] >> c) & 1) ? T(0) : lo[c][q];
                        u[c][q + 4] = ((mhi[q] >> c) & 1) ? T(0) : hi[c][q];
                    }
                }
            element_apply<3, T>(B, Ee, u);
            T P[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    P[c][q] = u[c][q] + cout[c][q];
                    cout[c][q] = u[c][q + 4];
                }
            if (ke >= kz0) {
                T acc[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // x partners (lane-1), then y partners (lane-8)
                    const T q0 = P[c][0] + shfl_up_w(P[c][1], 1, kWT);
                    const T q1 = P[c][2] + shfl_up_w(P[c][3], 1, kWT);
                    acc[c] = q0 + shfl_up_w(q1, kWT, 64);
                }
                if (owner && ke < g.nnz) {
                    const int64_t nd = base[0] + plane * ke;
                    const uint8_t own = mlo[0];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int64_t d = nd * 3 + c;
                        const T xown = lo[c][0];
                        const T ax = (own >> c) & 1 ? xown : acc[c];
                        const T rr = MODE == kModeY ? T(0) : r[col * ld + d];
                        const T di = MODE == kModeJacobi ? dinv[d] : T(0);
                        y[col * ld + d] = wht_epilogue<T, MODE>(ax, xown, rr, di, omega);
                        if (DOT) dsum += (double)xown * (double)ax;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    lo[c][q] = hi[c][q];
                    if (PF) hi[c][q] = pf[c][q];
                }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                mlo[q] = mhi[q];
                if (PF) mhi[q] = mpf[q];
            }
            if (!PF) fetch(ke + 2, hi, mhi);
        }
        if (DOT) {
            const double bs = wht_block_sum(dsum, sh);
            if (lane == 0 && threadIdx.y == 0) part[col * nblk + sl.slot] = bs;
        }
    }
}

// ---------------------------------------------------------------------------
// 3D, variant 3: the wave tiles of k_apply_wht3 with far fewer instructions
// per element layer (the register-tile kernels are bound by instruction
// issue, not by memory):
//  - the 8-point transform factors as H8 = H2 (z) x H4 (xy), so each node
//    plane is transformed over its 4 column corners once, when it arrives,
//    and an element's transform is the sum and the difference of its two
//    planes' transforms;
//  - the part of an element's result that falls on its lower plane and the
//    part the element below put on the same plane are added in the
//    transformed basis, and one inverse 4-point transform per plane gives
//    the corner values;
//  - the element modulus scales the 9 block coefficients instead of the 21
//    nonzero outputs;
//  - loads and stores are buffer operations with 32-bit byte offsets: a lane
//    whose node column lies outside the grid, and a plane or element layer
//    outside the box, carry offsets beyond the buffer's size, so the
//    hardware range check returns zeros (and drops stores of lanes that own
//    no node) without per-value selects;
//  - Dirichlet masks of inputs that may be nonzero at fixed DOFs are applied
//    only in waves that see a fixed DOF (wave-uniform branch).
// Memory schedule of a step: 0 stores at the end of the step, loads placed
// by the compiler; 1 stores of plane ke issued at the start of step ke + 1;
// 2 as 1, with every load of the step issued before its arithmetic.
#ifndef MLB_WHT3R_SCHED
#define MLB_WHT3R_SCHED 2
#endif
constexpr int kW3rSched = MLB_WHT3R_SCHED;
constexpr uint32_t kOffLane = 0x80000000u;    // offset of a lane outside the grid
constexpr uint32_t kOffPlane = 0x40000000u;   // offset of a plane/layer outside the box
constexpr uint32_t kMaxBufBytes = 0x40000000u;  // largest array the offsets can address
constexpr int kBufFlags = 0x00020000;          // buffer descriptor word 3 (raw 32-bit data)

template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const T* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)bytes, kBufFlags);
}
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t off, double& v) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
}
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t off, float& v) {
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
}
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, double v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), rs, (int)off, 0, 0);
}
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, float v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(rs, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), rs, (int)off, 0, 0);
}

// The three components of one node (12 or 24 contiguous bytes) in one
// access (FP32: 96 bits) or two (FP64: 128 + 64 bits).  Out-of-range offsets
// read zeros and drop stores, like the single-word accesses.
typedef int mlb_v2i __attribute__((ext_vector_type(2)));
__device__ inline void buf_load3(__amdgpu_buffer_rsrc_t rs, uint32_t off, float& a, float& b, float& c) {
    // Components are taken out with shuffles: subscripting the 96-bit result
    // type lowers to a one-word load whose value fills all three.
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, (int)off, 0, 0);
    a = __builtin_bit_cast(float, __builtin_shufflevector(v, v, 0)[0]);
    b = __builtin_bit_cast(float, __builtin_shufflevector(v, v, 1)[0]);
    c = __builtin_bit_cast(float, __builtin_shufflevector(v, v, 2)[0]);
}
__device__ inline void buf_load3(__amdgpu_buffer_rsrc_t rs, uint32_t off, double& a, double& b, double& c) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(off + 16u), 0, 0);
    a = __builtin_bit_cast(double, mlb_v2i{(int)__builtin_shufflevector(v, v, 0)[0], (int)__builtin_shufflevector(v, v, 1)[0]});
    b = __builtin_bit_cast(double, mlb_v2i{(int)__builtin_shufflevector(v, v, 2)[0], (int)__builtin_shufflevector(v, v, 3)[0]});
    c = __builtin_bit_cast(double, w);
}
__device__ inline void buf_store3(__amdgpu_buffer_rsrc_t rs, uint32_t off, float a, float b, float c) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b96(rs, 0, 0, 0));
    V v;
    v[0] = __builtin_bit_cast(int, a);
    v[1] = __builtin_bit_cast(int, b);
    v[2] = __builtin_bit_cast(int, c);
    __builtin_amdgcn_raw_buffer_store_b96(v, rs, (int)off, 0, 0);
}
__device__ inline void buf_store3(__amdgpu_buffer_rsrc_t rs, uint32_t off, double a, double b, double c) {
    using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rs, 0, 0, 0));
    const mlb_v2i ia = __builtin_bit_cast(mlb_v2i, a), ib = __builtin_bit_cast(mlb_v2i, b);
    V4 v;
    v[0] = ia[0];
    v[1] = ia[1];
    v[2] = ib[0];
    v[3] = ib[1];
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, c), rs, (int)(off + 16u), 0, 0);
}

__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// wht_epilogue with an explicit fused multiply-add (no contraction choices)
template <typename T, int MODE>
__device__ inline T wht_epilogue_fixed(T ax, T xown, T rr, T di, T omega) {
#pragma clang fp contract(off)
    if (MODE == kModeY) return ax;
    if (MODE == kModeResidual) return rr - ax;
    return fmat(omega * di, rr - ax, xown);
}

// The 3D blocks of element_apply with coefficients already scaled by the
// element modulus: s = E * (o0, d0 - o0, o7, d7 - o7, e1, f1, g2d, g2o, h2).
// The translation entries u[c][0] are left untouched (they are zero).
// Contraction is off and the fused multiply-adds are explicit, so every
// inlined copy rounds the same way.
template <typename T>
__device__ inline void blocks3_scaled(const T (&s)[9], T (&u)[3][8]) {
#pragma clang fp contract(off)
    {
        const T a = u[0][1], b = u[1][2], c3 = u[2][4];
        const T sum = s[0] * ((a + b) + c3);
        u[0][1] = fmat(s[1], a, sum);
        u[1][2] = fmat(s[1], b, sum);
        u[2][4] = fmat(s[1], c3, sum);
    }
    {
        const T a = u[0][6], b = u[1][5], c3 = u[2][3];
        const T sum = s[2] * ((a + b) + c3);
        u[0][6] = fmat(s[3], a, sum);
        u[1][5] = fmat(s[3], b, sum);
        u[2][3] = fmat(s[3], c3, sum);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const int i1 = (1 << c) | (1 << c1), i2 = (1 << c) | (1 << c2);
        const T v1 = u[c1][i1], v2 = u[c2][i2];
        u[c1][i1] = fmat(s[4], v1, s[5] * v2);
        u[c2][i2] = fmat(s[5], v1, s[4] * v2);
        const T w1 = u[c1][1 << c2], w2 = u[c2][1 << c1];
        u[c1][1 << c2] = fmat(s[6], w1, s[7] * w2);
        u[c2][1 << c1] = fmat(s[7], w1, s[6] * w2);
        u[c][7] = s[8] * u[c][7];
    }
}

template <typename T, int MODE, bool DOT, bool CLEAN>
__global__ __launch_bounds__(64 * kW3) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && CLEAN ? 4 : MLB_WHT3_WAVES, 8))) void k_apply_wht3r(
    Geo g, int kz_chunk, int ntiles_x, int ntiles_y, const T* __restrict__ E, const uint8_t* __restrict__ nmask,
    WhtBlocks<T> B, int ncols, int64_t ld, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ r,
    const T* __restrict__ dinv, T omega, double* __restrict__ part, int cgrid) {
    // no contraction: the loop is unrolled twice and both copies must round
    // alike, so that results do not depend on the pencil length
#pragma clang fp contract(off)
    // FP32 Jacobi sweeps of clean blocks need no identity rows: their D^-1
    // copy is 0 at fixed DOFs, where x and r are 0, so y = x + 0 = 0 there
    // (the value the identity row gives) and the owned node's mask is not read
    constexpr bool NOMASK = sizeof(T) == 4 && CLEAN && MODE == kModeJacobi;
    __shared__ double sh[16];
    const int lane = threadIdx.x;
    const int tx = lane & 7, ty = lane >> 3;
    const WhtSlot sl = wht_slot(cgrid, ncols);
    const int64_t bl = sl.bl;
    // the wave's index in its block, as a wave-uniform value: everything
    // derived from it (pencil, loop bounds, plane offsets) stays scalar
    const int wib = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int64_t tile = bl * kW3 + wib;
    const int64_t ntile_xy = (int64_t)ntiles_x * ntiles_y;
    const int tzc = (int)(tile / ntile_xy);
    const int txy = (int)(tile % ntile_xy);
    const int ie = (txy % ntiles_x) * (kWT - 1) - 1 + tx;
    const int je = (txy / ntiles_x) * (kWT - 1) - 1 + ty;
    const int kz0 = tzc * kz_chunk;
    const int kend = min(kz0 + kz_chunk, g.nnz);
    const bool col_ok = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny;
    const bool owner = tx >= 1 && ty >= 1 && ie >= 0 && je >= 0 && ie <= g.nx && je <= g.ny;
    const uint32_t plane = (uint32_t)g.nnx * (uint32_t)g.nny;
    const uint32_t xnode = 3u * sizeof(T);                 // bytes per node
    const uint32_t xplane = plane * xnode;                 // bytes per node plane
    const uint32_t eplane = (uint32_t)g.nx * (uint32_t)g.ny * sizeof(T);
    const uint32_t xbytes = (uint32_t)g.nodes * xnode;
    uint32_t vo[4], mo[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int ii = ie + (q & 1), jj = je + (q >> 1);
        const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny;
        const uint32_t nd = (uint32_t)ii + (uint32_t)g.nnx * (uint32_t)jj;
        vo[q] = ok ? nd * xnode : kOffLane;
        mo[q] = ok ? nd : kOffLane;
    }
    const uint32_t eo = col_ok ? ((uint32_t)ie + (uint32_t)g.nx * (uint32_t)je) * sizeof(T) : kOffLane;
    const __amdgpu_buffer_rsrc_t rE = buf_rsrc(E, (uint32_t)g.m * sizeof(T));
    const __amdgpu_buffer_rsrc_t rM = buf_rsrc(nmask, (uint32_t)g.nodes);
    const __amdgpu_buffer_rsrc_t rD = buf_rsrc(dinv, MODE == kModeJacobi ? xbytes : 0u);
    const T dd0 = B.v[0] - B.v[1], dd7 = B.v[2] - B.v[3];
    const int64_t nblk = sl.nblk;
    // byte offsets of node plane kk / element layer ke (out of range: zeros)
    auto poff = [&](int kk) -> uint32_t { return kk >= 0 && kk < g.nnz ? (uint32_t)kk * xplane : kOffPlane; };
    auto moff = [&](int kk) -> uint32_t { return kk >= 0 && kk < g.nnz ? (uint32_t)kk * plane : kOffPlane; };
    auto eoff = [&](int ke) -> uint32_t { return ke >= 0 && ke < g.nz ? (uint32_t)ke * eplane : kOffPlane; };
    for (int col = sl.c0; col < sl.c1; ++col) {
        const __amdgpu_buffer_rsrc_t rX = buf_rsrc(x + col * ld, xbytes);
        const __amdgpu_buffer_rsrc_t rY = buf_rsrc(y + col * ld, xbytes);
        const __amdgpu_buffer_rsrc_t rR = buf_rsrc(r + col * ld, MODE == kModeY ? 0u : xbytes);
        double dsum = 0.0;
        auto load_plane = [&](int kk, T (&v)[3][4], uint8_t (&mk)[4]) {
            const uint32_t po = poff(kk), pm = moff(kk);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                buf_load3(rX, vo[q] + po, v[0][q], v[1][q], v[2][q]);
                if (!CLEAN || (q == 0 && !NOMASK)) mk[q] = __builtin_amdgcn_raw_buffer_load_b8(rM, (int)(mo[q] + pm), 0, 0);
                else if (q == 0) mk[q] = 0;
            }
        };
        // Walsh-Hadamard transform of a plane over the 4 column corners
        // (values at fixed DOFs taken as zero)
        auto transform = [&](T (&v)[3][4], const uint8_t (&mk)[4], T (&h)[3][4]) {
            if (!CLEAN) {
                if (__any((mk[0] | mk[1] | mk[2] | mk[3]) != 0)) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            if ((mk[q] >> c) & 1) v[c][q] = T(0);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int q = 0; q < 4; ++q) h[c][q] = v[c][q];
                wht<2, T>(h[c]);
            }
        };
        // Each step works on element layer ke between node planes ke (lo)
        // and ke + 1 (hi), writes plane ke, and transforms plane ke + 2 into
        // the slot that plane ke leaves free; the loop is unrolled twice so
        // that the two slots swap roles instead of being copied.
        T hA[3][4], hB[3][4], carry[3][4], oA[3], oB[3], EA, EB;
        uint8_t mA, mB;
        {
            T v[3][4];
            uint8_t mk[4];
            load_plane(kz0 - 1, v, mk);
#pragma unroll
            for (int c = 0; c < 3; ++c) oA[c] = v[c][0];
            mA = mk[0];
            transform(v, mk, hA);
            load_plane(kz0, v, mk);
#pragma unroll
            for (int c = 0; c < 3; ++c) oB[c] = v[c][0];
            mB = mk[0];
            transform(v, mk, hB);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) carry[c][q] = T(0);
        buf_load(rE, eo + eoff(kz0 - 1), EA);
        // Results of plane ke are stored at the start of step ke + 1.  Loads
        // and stores share one completion counter here, and a wait for a
        // load issued before a store still in flight waits for that store
        // too; issued after the step's first wait (the modulus) and before
        // its loads, the stores complete during the element arithmetic.
        T py[3] = {T(0), T(0), T(0)};
        uint32_t pod = kOffLane;
        auto flush = [&]() { buf_store3(rY, pod, py[0], py[1], py[2]); };
        auto step = [&](int ke, T (&hl)[3][4], const T (&hh)[3][4], T (&olo)[3], uint8_t& mlo, const T& Ecur,
                        T& Enext) {
            T s[9];
            s[0] = Ecur * B.v[1];
            s[1] = Ecur * dd0;
            s[2] = Ecur * B.v[3];
            s[3] = Ecur * dd7;
#pragma unroll
            for (int i = 4; i < 9; ++i) s[i] = Ecur * B.v[i];
            if (kW3rSched >= 1) {
                __builtin_amdgcn_sched_barrier(0);
                flush();
                __builtin_amdgcn_sched_barrier(0);
            }
            // next plane, next modulus, and this plane's right-hand data
            T pf[3][4];
            uint8_t mpf[4];
            load_plane(ke + 2, pf, mpf);
            buf_load(rE, eo + eoff(ke + 1), Enext);
            const bool out = ke >= kz0;   // wave-uniform
            const uint32_t od = owner && out ? vo[0] + poff(ke) : kOffLane;
            T rr[3] = {T(0), T(0), T(0)}, di[3] = {T(0), T(0), T(0)};
            if (MODE != kModeY) buf_load3(rR, od, rr[0], rr[1], rr[2]);
            if (MODE == kModeJacobi) buf_load3(rD, od, di[0], di[1], di[2]);
            // all of the step's loads are issued before its arithmetic
            if (kW3rSched >= 2) __builtin_amdgcn_sched_barrier(0);
            T u[3][8];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    u[c][k] = hl[c][k] + hh[c][k];
                    u[c][k + 4] = hl[c][k] - hh[c][k];
                }
            blocks3_scaled<T>(s, u);
            // plane ke: this element's lower half plus the carried upper half
            // of the element below, in the transformed basis; then back to
            // the 4 corners
            T a[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[c][0] = carry[c][0] + u[c][4];
                carry[c][0] = -u[c][4];
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    a[c][k] = carry[c][k] + (u[c][k] + u[c][k + 4]);
                    carry[c][k] = u[c][k] - u[c][k + 4];
                }
                wht<2, T>(a[c]);
            }
            // (also in the first step of a pencil, whose plane is not ours:
            // its results go to an out-of-range offset, and a branch here
            // would let the compiler sink the right-hand loads into it)
            if (kW3rSched >= 2 || out) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T q0 = a[c][0] + shfl_up_w(a[c][1], 1, kWT);
                    const T q1 = a[c][2] + shfl_up_w(a[c][3], 1, kWT);
                    const T acc = q0 + shfl_up_w(q1, kWT, 64);
                    const T xown = olo[c];
                    const T ax = !NOMASK && ((mlo >> c) & 1) ? xown : acc;
                    py[c] = wht_epilogue_fixed<T, MODE>(ax, xown, rr[c], di[c], omega);
                    if (DOT && owner && out) dsum += (double)xown * (double)ax;
                }
            }
            pod = od;
            if (kW3rSched == 0) flush();
            // plane ke + 2 takes the slot of plane ke
#pragma unroll
            for (int c = 0; c < 3; ++c) olo[c] = pf[c][0];
            mlo = mpf[0];
            transform(pf, mpf, hl);
        };
        for (int ke = kz0 - 1; ke < kend; ke += 2) {
            step(ke, hA, hB, oA, mA, EA, EB);
            if (ke + 1 >= kend) break;
            step(ke + 1, hB, hA, oB, mB, EB, EA);
        }
        if (kW3rSched >= 1) flush();
        if (DOT) {
            const double bs = wht_block_sum(dsum, sh);
            if (lane == 0 && threadIdx.y == 0) part[col * nblk + sl.slot] = bs;
        }
    }
}

// ---------------------------------------------------------------------------
// 3D, LDS variant: one block of 16 x 16 threads is a tile of 16 x 16 element
// columns (tiles overlap by one column/row, the 15 x 15 interior node columns
// are owned) walking a pencil of element layers along z.  Each node plane of
// the tile (17 x 17 nodes x 3 components, component-major) is loaded once,
// coalesced, into a ring of 3 LDS planes, one step ahead of its use; every
// thread reads its element's 8 nodes from LDS, applies the element in the
// Walsh-Hadamard basis, and writes its 4 low-plane node contributions (plus
// the carried high-plane part of the element below) to LDS, where each owned
// node sums its 4 columns in a fixed order.  Per lane this keeps no node
// planes in registers (the register-tile variant holds 3 x 12 values).
// Dirichlet masking happens when a plane is loaded; identity rows take the
// owned node's raw value.
constexpr int kLT = 16;                    // tile edge in element columns
constexpr int kLN = kLT + 1;               // tile edge in nodes
constexpr int kLP = kLN * kLN;             // nodes per tile plane
constexpr int kLThreads = kLT * kLT;
#ifndef MLB_WHTL_WAVES
#define MLB_WHTL_WAVES 2
#endif

template <typename T, int MODE, bool DOT>
__global__ __launch_bounds__(kLThreads) __attribute__((amdgpu_waves_per_eu(MLB_WHTL_WAVES, 8))) void k_apply_wht3_lds(Geo g, int kz_chunk, int ntiles_x, int ntiles_y,
                                                              const T* __restrict__ E,
                                                              const uint8_t* __restrict__ nmask, WhtBlocks<T> B,
                                                              int ncols, int64_t ld, const T* __restrict__ x,
                                                              T* __restrict__ y, const T* __restrict__ r,
                                                              const T* __restrict__ dinv, T omega,
                                                              double* __restrict__ part) {
    __shared__ T plane[3][3][kLP];         // [slot][component][node]
    __shared__ T pc[3][4][kLThreads];      // [component][corner][element column]
    __shared__ double sh[kLThreads / 64];
    const int tid = threadIdx.x;
    const int tx = tid % kLT, ty = tid / kLT;
    // blocks dealt round robin over the XCDs; each XCD takes a contiguous
    // range of the (z-chunk major) tile order
    const int64_t per_xcd = gridDim.x / kXcd3;
    const int64_t tile = (blockIdx.x % kXcd3) * per_xcd + blockIdx.x / kXcd3;
    const int64_t ntile_xy = (int64_t)ntiles_x * ntiles_y;
    const int tzc = (int)(tile / ntile_xy);
    const int txy = (int)(tile % ntile_xy);
    const int i0 = (txy % ntiles_x) * (kLT - 1) - 1;   // node / element origin of the tile
    const int j0 = (txy / ntiles_x) * (kLT - 1) - 1;
    const int kz0 = tzc * kz_chunk;
    const int kend = min(kz0 + kz_chunk, g.nnz);
    const bool live = kz0 < g.nnz;                      // padding blocks of the XCD-rounded grid
    const int ie = i0 + tx, je = j0 + ty;
    const bool col_ok = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny;
    const bool owner = tx >= 1 && ty >= 1 && ie <= g.nx && je <= g.ny;
    const int64_t pl = (int64_t)g.nnx * g.nny;
    const int64_t epl = (int64_t)g.nx * g.ny;
    const int64_t ebase = col_ok ? ie + (int64_t)g.nx * je : 0;
    const int64_t own = owner ? ie + (int64_t)g.nnx * je : 0;
    constexpr int kPer = (3 * kLP + kLThreads - 1) / kLThreads;   // plane entries per thread
    for (int col = 0; col < ncols; ++col) {
        const T* xc = x + col * ld;
        double dsum = 0.0;
        // entries e = tid + kLThreads * k of a plane: row ly, then x-major
        // interleaved (node, component), so consecutive threads read
        // consecutive addresses
        auto load = [&](int kk, T (&v)[kPer]) {
            const bool kin = kk >= 0 && kk < g.nnz;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int e = tid + kLThreads * k;
                const int ly = e / (3 * kLN), rem = e % (3 * kLN);
                const int lx = rem / 3, c = rem % 3;
                const int gi = i0 + lx, gj = j0 + ly;
                const bool ok = e < 3 * kLP && kin && gi >= 0 && gi < g.nnx && gj >= 0 && gj < g.nny;
                const int64_t nd = ok ? gi + (int64_t)g.nnx * gj + pl * kk : 0;
                const T xv = xc[nd * 3 + c];
                const uint8_t m = nmask[nd];
                v[k] = (ok && !((m >> c) & 1)) ? xv : T(0);
            }
        };
        auto stash = [&](int kk, const T (&v)[kPer]) {
            const int slot = (kk + 3) % 3;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int e = tid + kLThreads * k;
                if (e < 3 * kLP) {
                    const int ly = e / (3 * kLN), rem = e % (3 * kLN);
                    plane[slot][rem % 3][ly * kLN + rem / 3] = v[k];
                }
            }
        };
        T pf[kPer];
        if (live) {
            load(kz0 - 1, pf);
            stash(kz0 - 1, pf);
            load(kz0, pf);
            stash(kz0, pf);
        }
        __syncthreads();
        T cout[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) cout[c][q] = T(0);
        for (int ke = kz0 - 1; live && ke < kend; ++ke) {
            const bool more = ke + 2 <= kend;
            if (more) load(ke + 2, pf);   // in flight during this step
            const bool eok = col_ok && ke >= 0 && ke < g.nz;
            const T Eraw = E[eok ? ebase + epl * ke : 0];
            const T Ee = eok ? Eraw : T(0);
            const int slo = (ke + 3) % 3, shi = (ke + 4) % 3;
            T u[3][8];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ln = (ty + (q >> 1)) * kLN + tx + (q & 1);
                    u[c][q] = plane[slo][c][ln];
                    u[c][q + 4] = plane[shi][c][ln];
                }
            const T xo0 = u[0][0], xo1 = u[1][0], xo2 = u[2][0];   // owned node (masked)
            element_apply<3, T>(B, Ee, u);
            if (ke >= kz0) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q = 0; q < 4; ++q) pc[c][q][tid] = u[c][q] + cout[c][q];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) cout[c][q] = u[c][q + 4];
            if (ke >= kz0) {
                __syncthreads();
                if (owner && ke < g.nnz) {
                    const int64_t nd = own + pl * ke;
                    const uint8_t m = nmask[nd];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        // fixed order: own column, x neighbour, y neighbour, diagonal
                        const T acc = ((pc[c][0][tid] + pc[c][1][tid - 1]) + pc[c][2][tid - kLT]) +
                                      pc[c][3][tid - kLT - 1];
                        const int64_t d = nd * 3 + c;
                        const T xm = c == 0 ? xo0 : c == 1 ? xo1 : xo2;
                        const bool fixed = (m >> c) & 1;
                        const T xraw = fixed ? xc[d] : xm;
                        const T ax = fixed ? xraw : acc;
                        const T rr = MODE == kModeY ? T(0) : r[col * ld + d];
                        const T di = MODE == kModeJacobi ? dinv[d] : T(0);
                        y[col * ld + d] = wht_epilogue<T, MODE>(ax, xraw, rr, di, omega);
                        if (DOT) dsum += (double)xraw * (double)ax;
                    }
                }
            }
            if (more) stash(ke + 2, pf);   // the slot of plane ke - 1, no longer read
            __syncthreads();
        }
        if (DOT) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) dsum += __shfl_down(dsum, off, 64);
            sh[tid >> 6] = __shfl(dsum, 0, 64);
            __syncthreads();
            if (tid < 64) {
                double s2 = 0.0;
                for (int w = 0; w < kLThreads / 64; ++w) s2 += sh[w];
                part[col * (int64_t)gridDim.x + blockIdx.x] = s2;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// 2D: block = 64 x 4 threads; each wave (row of the block) is an independent
// pencil of elements along y for its own x tile.
constexpr int kTX2 = 64, kTW2 = 4;

template <typename T, int MODE, bool DOT>
__global__ __launch_bounds__(kTX2* kTW2) void k_apply_wht2(Geo g, int ky_chunk, int ntiles_x, const T* __restrict__ E,
                                                           const uint8_t* __restrict__ nmask, WhtBlocks<T> B,
                                                           int ncols, int64_t ld, const T* __restrict__ x,
                                                           T* __restrict__ y, const T* __restrict__ r,
                                                           const T* __restrict__ dinv, T omega,
                                                           double* __restrict__ part, int cgrid) {
    __shared__ double sh[16];
    const int tx = threadIdx.x;
    // cgrid column groups on the grid, the groups of one tile block
    // consecutive; partial dot products go to the block's one-group slot
    const int64_t blk = blockIdx.x / cgrid;
    const int64_t nblk = gridDim.x / cgrid;
    const int per = (ncols + cgrid - 1) / cgrid;
    const int c0 = (int)(blockIdx.x % cgrid) * per, c1 = min(ncols, c0 + per);
    const int64_t tile = blk * kTW2 + threadIdx.y;
    const int tile_x = (int)(tile % ntiles_x);
    const int tile_y = (int)(tile / ntiles_x);
    const int ie = tile_x * (kTX2 - 1) - 1 + tx;
    const int ky0 = tile_y * ky_chunk;
    const int kend = min(ky0 + ky_chunk, g.nny);
    const bool col_ok = ie >= 0 && ie < g.nx;
    const bool owner = tx >= 1 && ie >= 0 && ie <= g.nx;
    for (int col = c0; col < c1; ++col) {
        const T* xc = x + col * ld;
        T cx[2][2], craw[2], cout[2][2];
        double dsum = 0.0;
        auto load_row = [&](int jj, T (&v)[2][2], T (&raw)[2]) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int ii = ie + q;
                const bool ok = ii >= 0 && ii < g.nnx && jj >= 0 && jj < g.nny;
                const int64_t nd = ok ? ii + (int64_t)g.nnx * jj : 0;
                const uint8_t mraw = nmask[nd];
                const uint8_t mb = ok ? mraw : (uint8_t)0xff;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const T xl = xc[nd * 2 + c];
                    const T xv = ok ? xl : T(0);
                    if (q == 0) raw[c] = xv;
                    v[c][q] = ((mb >> c) & 1) ? T(0) : xv;
                }
            }
        };
        load_row(ky0 - 1, cx, craw);
#pragma unroll
        for (int c = 0; c < 2; ++c) cout[c][0] = cout[c][1] = T(0);
        const bool live = tile_y * ky_chunk < g.nny;
        for (int je = ky0 - 1; live && je < kend; ++je) {
            T nx_[2][2], nraw[2];
            load_row(je + 1, nx_, nraw);
            const bool eok = col_ok && je >= 0 && je < g.ny;
            const T Eraw = E[eok ? ie + (int64_t)g.nx * je : 0];
            const T Ee = eok ? Eraw : T(0);
            T u[2][4];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                u[c][0] = cx[c][0];
                u[c][1] = cx[c][1];
                u[c][2] = nx_[c][0];
                u[c][3] = nx_[c][1];
            }
            element_apply<2, T>(B, Ee, u);
            T P[2][2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                P[c][0] = u[c][0] + cout[c][0];
                P[c][1] = u[c][1] + cout[c][1];
                cout[c][0] = u[c][2];
                cout[c][1] = u[c][3];
            }
            if (je >= ky0) {
                T Q[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) Q[c] = P[c][0] + shfl_up_w(P[c][1], 1, kTX2);
                if (owner && je < g.nny) {
                    const int64_t nd = ie + (int64_t)g.nnx * je;
                    const uint8_t own = nmask[nd];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int64_t d = nd * 2 + c;
                        const T xown = craw[c];
                        const T ax = (own >> c) & 1 ? xown : Q[c];
                        const T rr = MODE == kModeY ? T(0) : r[col * ld + d];
                        const T di = MODE == kModeJacobi ? dinv[d] : T(0);
                        y[col * ld + d] = wht_epilogue<T, MODE>(ax, xown, rr, di, omega);
                        if (DOT) dsum += (double)xown * (double)ax;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                craw[c] = nraw[c];
                cx[c][0] = nx_[c][0];
                cx[c][1] = nx_[c][1];
            }
        }
        if (DOT) {
            const double bs = wht_block_sum(dsum, sh);
            if (tx == 0 && threadIdx.y == 0) part[col * nblk + blk] = bs;
        }
    }
}

// ---------------------------------------------------------------------------
// launch geometry

// zchunk: target pencil length in node planes (3D; tunable, results do not
// depend on it: every owned node is summed in the same order)
static void wht_geometry(int dim, const Geo& g, int zchunk, int variant, dim3& grid, dim3& block, int& chunk,
                         int& ntx, int& nty) {
    nty = 1;
    if (dim == 3 && variant == 1) {
        const int tiles_x = (g.nnx + kLT - 2) / (kLT - 1);
        const int tiles_y = (g.nny + kLT - 2) / (kLT - 1);
        const int zc = zchunk > 0 ? zchunk : 8;
        int nch = (g.nnz + zc - 1) / zc;
        chunk = (g.nnz + nch - 1) / nch;
        nch = (g.nnz + chunk - 1) / chunk;
        const int64_t tiles = (int64_t)tiles_x * tiles_y * nch;
        grid = dim3((unsigned)((tiles + kXcd3 - 1) / kXcd3 * kXcd3), 1, 1);
        block = dim3(kLThreads, 1, 1);
        ntx = tiles_x;
        nty = tiles_y;
    } else if (dim == 3) {
        const int tiles_x = (g.nnx + kWT - 2) / (kWT - 1);
        const int tiles_y = (g.nny + kWT - 2) / (kWT - 1);
        const int zc = zchunk > 0 ? zchunk : 8;
        int nch = (g.nnz + zc - 1) / zc;
        chunk = (g.nnz + nch - 1) / nch;
        nch = (g.nnz + chunk - 1) / chunk;
        const int64_t tiles = (int64_t)tiles_x * tiles_y * nch;
        const int64_t blocks = (tiles + kW3 - 1) / kW3;
        grid = dim3((unsigned)((blocks + kXcd3 - 1) / kXcd3 * kXcd3), 1, 1);
        block = dim3(64, kW3, 1);
        ntx = tiles_x;
        nty = tiles_y;
    } else {
        const int tiles_x = (g.nnx + kTX2 - 2) / (kTX2 - 1);
        int nch = (g.nny + 15) / 16;
        chunk = (g.nny + nch - 1) / nch;
        nch = (g.nny + chunk - 1) / chunk;
        const int tiles = tiles_x * nch;
        grid = dim3((tiles + kTW2 - 1) / kTW2, 1, 1);
        block = dim3(kTX2, kTW2, 1);
        ntx = tiles_x;
    }
}

int64_t apply_wht_blocks(int dim, const Geo& g, int zchunk, int variant) {
    dim3 gr, b;
    int ch, ntx, nty;
    wht_geometry(dim, g, zchunk, variant, gr, b, ch, ntx, nty);
    return (int64_t)gr.x * gr.y * gr.z;
}

template <typename T>
void launch_apply_wht(int dim, const Geo& g, const T* E, const uint8_t* nmask, const T* blocks, int ncols,
                      int64_t ld, const T* x, T* y, int mode, const T* r, const T* dinv, T omega, double* dot_part,
                      bool clean, int zchunk, int variant, hipStream_t st) {
    WhtBlocks<T> B;
    for (int i = 0; i < 9; ++i) B.v[i] = blocks[i];
    dim3 gr, b;
    int ch, ntx, nty;
    wht_geometry(dim, g, zchunk, variant, gr, b, ch, ntx, nty);
    // variant 3 addresses each array with 32-bit byte offsets
    if (dim == 3 && variant == 3 &&
        ((uint64_t)g.nodes * 3 * sizeof(T) > kMaxBufBytes || (uint64_t)g.m * sizeof(T) > kMaxBufBytes))
        variant = 0;
    // one column per block group (the LDS variant walks its columns itself)
    const int cgrid = (dim == 3 && variant == 1) ? 1 : std::max(1, ncols);
    const dim3 grc(gr.x * cgrid, gr.y, gr.z);
#define MLB_L3C(M, D, C)                                                                                          \
    do {                                                                                                          \
        if (variant == 3)                                                                                         \
            hipLaunchKernelGGL((k_apply_wht3r<T, M, D, C>), grc, b, 0, st, g, ch, ntx, nty, E, nmask, B, ncols, ld, \
                               x, y, r, dinv, omega, dot_part, cgrid);                                            \
        else if (variant == 2)                                                                                    \
            hipLaunchKernelGGL((k_apply_wht3<T, M, D, C, false>), grc, b, 0, st, g, ch, ntx, nty, E, nmask, B,     \
                               ncols, ld, x, y, r, dinv, omega, dot_part, cgrid);                                 \
        else                                                                                                      \
            hipLaunchKernelGGL((k_apply_wht3<T, M, D, C, true>), grc, b, 0, st, g, ch, ntx, nty, E, nmask, B,      \
                               ncols, ld, x, y, r, dinv, omega, dot_part, cgrid);                                 \
    } while (0)
#define MLB_L3(M, D)                       \
    do {                                   \
        if (clean) MLB_L3C(M, D, true);    \
        else MLB_L3C(M, D, false);         \
    } while (0)
#define MLB_L2(M, D)                                                                                              \
    hipLaunchKernelGGL((k_apply_wht2<T, M, D>), grc, b, 0, st, g, ch, ntx, E, nmask, B, ncols, ld, x, y, r, dinv,  \
                       omega, dot_part, cgrid)
#define MLB_LL(M, D)                                                                                              \
    hipLaunchKernelGGL((k_apply_wht3_lds<T, M, D>), gr, b, 0, st, g, ch, ntx, nty, E, nmask, B, ncols, ld, x, y, r,  \
                       dinv, omega, dot_part)
    if (dim == 3 && variant == 1) {
        if (mode == kModeY && dot_part) MLB_LL(kModeY, true);
        else if (mode == kModeY) MLB_LL(kModeY, false);
        else if (mode == kModeResidual) MLB_LL(kModeResidual, false);
        else MLB_LL(kModeJacobi, false);
    } else if (dim == 3) {
        if (mode == kModeY && dot_part) MLB_L3(kModeY, true);
        else if (mode == kModeY) MLB_L3(kModeY, false);
        else if (mode == kModeResidual) MLB_L3(kModeResidual, false);
        else MLB_L3(kModeJacobi, false);
    } else {
        if (mode == kModeY && dot_part) MLB_L2(kModeY, true);
        else if (mode == kModeY) MLB_L2(kModeY, false);
        else if (mode == kModeResidual) MLB_L2(kModeResidual, false);
        else MLB_L2(kModeJacobi, false);
    }
#undef MLB_L3
#undef MLB_L3C
#undef MLB_L2
#undef MLB_LL
}

template void launch_apply_wht<double>(int, const Geo&, const double*, const uint8_t*, const double*, int, int64_t,
                                       const double*, double*, int, const double*, const double*, double, double*,
                                       bool, int, int, hipStream_t);
template void launch_apply_wht<float>(int, const Geo&, const float*, const uint8_t*, const float*, int, int64_t,
                                      const float*, float*, int, const float*, const float*, float, double*, bool,
                                      int, int, hipStream_t);

}  // namespace mlb
