// Kernels of the batched 2D instances: every launch drains one work list of
// (segment, chunk) items that covers all instances at once.
//
// Work distribution.  In persistent mode a grid of at most a few thousand
// blocks pulls items from 8 queues, one per XCD: queue x holds the x-th
// contiguous eighth of the list, blocks are dealt round robin over the XCDs
// (block b runs on XCD b mod 8), and a block first drains its own XCD's
// queue, so neighbouring chunks (which share halo nodes) are read through one
// L2.  Then it steals from the other queues.  Every counter only grows and a
// block leaves a queue after one failed take (and after at most its length
// plus one takes in any case), so the launch always ends;
// the last block out resets the counters for the next launch.  Otherwise the
// hardware dispatcher is the queue (one block per item).
//
// Results never depend on which block takes which item: per-item partial
// sums are written to the item's own slot and every per-instance scalar is
// summed from those slots in a fixed order.
#include "batch_kernels.h"

namespace mlb {

constexpr int kBT = kBItemNodes;   // threads per block

// The ticket fetch is wave-uniform on purpose: the whole first wave executes
// the atomic (only its lane 0 adds 1) and every lane stores the same ticket,
// and the ticket read back is made scalar.  With a lane-0-only branch at the
// loop header the compiler may rotate the loop so that the other lanes of
// the first wave re-enter the barrier while lane 0 waits to fetch the next
// ticket, which never finishes; keeping every branch around the barriers
// uniform within each wave rules that out.
template <typename F>
__device__ inline void bq_drain(const BQueue& q, F&& body) {
    if (!q.persistent) {
        if ((int)blockIdx.x < q.nitems) body((int)blockIdx.x);
        return;
    }
    __shared__ int s_it;
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;
    const int home = (int)(blockIdx.x & 7);
    for (int k = 0; k < 8; ++k) {
        const int qi = (home + k) & 7;
        const int lo = (int)(((int64_t)q.nitems * qi) >> 3);
        const int hi = (int)(((int64_t)q.nitems * (qi + 1)) >> 3);
        // a block takes at most hi - lo + 1 tickets from one queue (the last
        // one fails), so the trip count is bounded whatever the counters hold
        for (int take = 0; take <= hi - lo; ++take) {
            if (wave0) {
                const unsigned t = atomicAdd(&q.ctr[qi], threadIdx.x == 0 ? 1u : 0u);
                s_it = lo + (int)__builtin_amdgcn_readfirstlane(t);
            }
            __syncthreads();
            const int it = __builtin_amdgcn_readfirstlane(s_it);
            __syncthreads();
            if (it >= hi) break;
            body(it);
        }
    }
    // No fence: each block's last ticket atomic has returned before its
    // done-count atomic is issued, so the block that counts last resets the
    // counters after every take of this launch (atomics on one counter are
    // performed in a single order).
    if (wave0) {
        const unsigned done = __builtin_amdgcn_readfirstlane(atomicAdd(&q.ctr[8], threadIdx.x == 0 ? 1u : 0u));
        if (done == gridDim.x - 1)
            for (int k = 0; k < 9; ++k) atomicExch(&q.ctr[k], 0u);
    }
}

// Sum over the 256 threads of a block in a fixed order; every thread gets it.
__device__ inline double bq_block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    sh[threadIdx.x >> 6] = __shfl(v, 0, 64);   // uniform store: every lane writes its wave's total
    __syncthreads();
    const double s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return s;
}

// Fixed-order sum of part[lo, hi) over a block (threads stride the range).
__device__ inline double bq_range_sum(const double* __restrict__ part, int lo, int hi, double* sh) {
    double v = 0.0;
    for (int k = lo + (int)threadIdx.x; k < hi; k += kBT) v += part[k];
    return bq_block_sum(v, sh);
}

// ---------------------------------------------------------------------------
// operator apply

template <typename T, typename TR, int MODE, int DOT>
__global__ __launch_bounds__(kBT) void k_bq_apply(BQueue q, const BSeg* __restrict__ segs,
                                                  const int* __restrict__ active, const T* __restrict__ Ek, BK0<T> K0,
                                                  const T* __restrict__ A, const T* __restrict__ dinv,
                                                  const T* __restrict__ omega, const uint8_t* __restrict__ nmask,
                                                  const T* __restrict__ x, T* __restrict__ y,
                                                  const TR* __restrict__ r, const double* __restrict__ dsrc,
                                                  double* __restrict__ part) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (active && !active[s.inst]) {
            if (DOT && threadIdx.x < 64) part[it] = 0.0;
            return;
        }
        const int nodes = s.nnx * s.nny;
        const int node = w.first + (int)threadIdx.x;
        double dacc = 0.0;
        if (node < nodes) {
            const int i = node % s.nnx, j = node / s.nnx;
            const T* xs = x + s.voff;
            T acc0 = T(0), acc1 = T(0);
            if (MODE != kBJac0) {
                if (s.level == 1) {
                    // matrix free: the four elements around the node, each
                    // E_e K0 restricted to the node's two rows
                    T xv[3][3][2];
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const bool ok = i + dx >= 0 && i + dx < s.nnx && j + dy >= 0 && j + dy < s.nny;
                            const int nb = ok ? node + dx + dy * s.nnx : node;
                            xv[dy + 1][dx + 1][0] = ok ? xs[2 * nb] : T(0);
                            xv[dy + 1][dx + 1][1] = ok ? xs[2 * nb + 1] : T(0);
                        }
#pragma unroll
                    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
                        for (int ox = 0; ox < 2; ++ox) {
                            const int ei = i - 1 + ox, ej = j - 1 + oy;
                            if (ei < 0 || ei >= s.nx || ej < 0 || ej >= s.ny) continue;
                            const T E = Ek[s.soff + ei + (int64_t)s.nx * ej];
                            const int a = (1 - ox) + 2 * (1 - oy);   // the node's corner in element e
                            T t0 = T(0), t1 = T(0);
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int bx = b & 1, by = b >> 1;
#pragma unroll
                                for (int c2 = 0; c2 < 2; ++c2) {
                                    const T v = xv[oy + by][ox + bx][c2];
                                    t0 += K0.k[(2 * a) * 8 + 2 * b + c2] * v;
                                    t1 += K0.k[(2 * a + 1) * 8 + 2 * b + c2] * v;
                                }
                            }
                            acc0 += E * t0;
                            acc1 += E * t1;
                        }
                } else {
                    // node-block stencil, entries of outside neighbours are zero
                    const T* As = A + s.soff;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const bool ok = i + dx >= 0 && i + dx < s.nnx && j + dy >= 0 && j + dy < s.nny;
                            const int nbn = ok ? node + dx + dy * s.nnx : node;
                            const int nb = (dx + 1) + 3 * (dy + 1);
                            const T x0 = xs[2 * nbn], x1 = xs[2 * nbn + 1];
                            acc0 += As[(int64_t)(nb * 4 + 0) * nodes + node] * x0 +
                                    As[(int64_t)(nb * 4 + 1) * nodes + node] * x1;
                            acc1 += As[(int64_t)(nb * 4 + 2) * nodes + node] * x0 +
                                    As[(int64_t)(nb * 4 + 3) * nodes + node] * x1;
                        }
                }
            }
            const uint8_t m = nmask[s.noff + node];
            const T om = omega ? omega[w.seg] : T(1);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                const bool fixed = (m >> c) & 1;
                const T ac = c == 0 ? acc0 : acc1;
                T v;
                if (MODE == kBY) v = fixed ? x[d] : ac;
                else if (fixed) v = T(0);
                else if (MODE == kBRes) v = (T)r[d] - ac;
                else if (MODE == kBJac) v = x[d] + om * dinv[d] * ((T)r[d] - ac);
                else if (MODE == kBJac0) v = om * dinv[d] * (T)r[d];
                else v = dinv[d] * ac;
                y[d] = v;
                if (DOT == 1 && !fixed) dacc += dsrc[d] * (double)v;
                if (DOT == 2 && !fixed) dacc += (double)v * (double)v;
            }
        }
        if (DOT) {
            const double sum = bq_block_sum(dacc, sh);
            if (threadIdx.x < 64) part[it] = sum;
        }
    });
}

// ---------------------------------------------------------------------------
// compensated residual of the fine level

// Error-free transformations (Knuth's two-sum, the FMA form of the exact
// product): a + b = s + e and a b = p + e exactly in floating point.
__device__ inline void bq_two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ inline void bq_two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = __builtin_fma(a, b, -p);
}

// r = f - K (x + xlo) on the free DOFs of the fine segments (zero at fixed
// DOFs), accumulated in double-double: every product E_e K0_ab x_b is formed
// exactly to second order and summed with two-sum, and the low part xlo (a
// double-double solution's tail, may be NULL) enters the low word, so r is
// the residual of x + xlo to a few units of rounding of r itself (not of
// |K||x|).  Per item: partial sums of r.r (part) and of (|K||x|).(|K||x|)
// over free DOFs (part2), the latter for the instance's representation
// floor.  r is written as zero for instances with skip[inst] != 0 (the sums
// still hold their residual).
__global__ __launch_bounds__(kBT) void k_bq_res_dd(BQueue q, const BSeg* __restrict__ segs,
                                                   const double* __restrict__ Ek, BK0<double> K0,
                                                   const uint8_t* __restrict__ nmask, const double* __restrict__ x,
                                                   const double* __restrict__ xlo, const int* __restrict__ skip,
                                                   const double* __restrict__ f, double* __restrict__ r,
                                                   double* __restrict__ part, double* __restrict__ part2) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const int nodes = s.nnx * s.nny;
        const int node = w.first + (int)threadIdx.x;
        double rr = 0.0, aa = 0.0;
        if (node < nodes) {
            const int i = node % s.nnx, j = node / s.nnx;
            const double* xs = x + s.voff;
            const double* xl = xlo ? xlo + s.voff : nullptr;
            double xv[3][3][2], xw[3][3][2];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const bool ok = i + dx >= 0 && i + dx < s.nnx && j + dy >= 0 && j + dy < s.nny;
                    const int nb = ok ? node + dx + dy * s.nnx : node;
#pragma unroll
                    for (int c2 = 0; c2 < 2; ++c2) {
                        xv[dy + 1][dx + 1][c2] = ok ? xs[2 * nb + c2] : 0.0;
                        xw[dy + 1][dx + 1][c2] = ok && xl ? xl[2 * nb + c2] : 0.0;
                    }
                }
            const uint8_t m = nmask[s.noff + node];
            const bool zero_out = skip && skip[s.inst];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                if ((m >> c) & 1) {
                    r[d] = 0.0;
                    continue;
                }
                double hi = f[d], lo = 0.0, ak = 0.0;
#pragma unroll
                for (int oy = 0; oy < 2; ++oy)
#pragma unroll
                    for (int ox = 0; ox < 2; ++ox) {
                        const int ei = i - 1 + ox, ej = j - 1 + oy;
                        if (ei < 0 || ei >= s.nx || ej < 0 || ej >= s.ny) continue;
                        const double E = Ek[s.soff + ei + (int64_t)s.nx * ej];
                        const int a = (1 - ox) + 2 * (1 - oy);
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int bx = b & 1, by = b >> 1;
#pragma unroll
                            for (int c2 = 0; c2 < 2; ++c2) {
                                const double v = xv[oy + by][ox + bx][c2];
                                double p1, e1, p2, e2, t, et;
                                bq_two_prod(K0.k[(2 * a + c) * 8 + 2 * b + c2], v, p1, e1);
                                bq_two_prod(E, p1, p2, e2);
                                e2 = __builtin_fma(E, e1, e2);   // E K0 v = p2 + e2 to second order
                                bq_two_sum(hi, -p2, t, et);
                                hi = t;
                                lo += et - e2 - E * (K0.k[(2 * a + c) * 8 + 2 * b + c2] * xw[oy + by][ox + bx][c2]);
                                ak += fabs(p2);
                            }
                        }
                    }
                double rv, re;
                bq_two_sum(hi, lo, rv, re);
                r[d] = zero_out ? 0.0 : rv;
                rr += rv * rv;
                aa += ak * ak;
            }
        }
        const double s1 = bq_block_sum(rr, sh);
        const double s2 = bq_block_sum(aa, sh);
        if (threadIdx.x < 64) {
            part[it] = s1;
            part2[it] = s2;
        }
    });
}

// ---------------------------------------------------------------------------
// transfers (bilinear interpolation P and P^T, masked on both sides)

template <typename T>
__global__ __launch_bounds__(kBT) void k_bq_restrict(BQueue q, const BSeg* __restrict__ segs,
                                                     const int* __restrict__ active,
                                                     const uint8_t* __restrict__ nmask, const T* __restrict__ xf,
                                                     T* __restrict__ yc) {
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (active && !active[s.inst]) return;
        const int node = w.first + (int)threadIdx.x;
        if (node >= s.nnx * s.nny) return;
        const BSeg f = segs[s.parent];
        const int I = node % s.nnx, J = node / s.nnx;
        const uint8_t mc = nmask[s.noff + node];
        T acc[2] = {T(0), T(0)};
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            const int jj = 2 * J + dj;
            if (jj < 0 || jj >= f.nny) continue;
            const T wj = dj == 0 ? T(1) : T(0.5);
#pragma unroll
            for (int di = -1; di <= 1; ++di) {
                const int ii = 2 * I + di;
                if (ii < 0 || ii >= f.nnx) continue;
                const T wt = di == 0 ? wj : wj * T(0.5);
                const int fn = ii + f.nnx * jj;
                const uint8_t mf = nmask[f.noff + fn];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (!((mf >> c) & 1)) acc[c] += wt * xf[f.voff + 2 * (int64_t)fn + c];
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) yc[s.voff + 2 * (int64_t)node + c] = ((mc >> c) & 1) ? T(0) : acc[c];
    });
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_bq_prolong_add(BQueue q, const BSeg* __restrict__ segs,
                                                        const int* __restrict__ active,
                                                        const uint8_t* __restrict__ nmask, const T* __restrict__ zc,
                                                        T* __restrict__ yf) {
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (active && !active[s.inst]) return;
        const int node = w.first + (int)threadIdx.x;
        if (node >= s.nnx * s.nny) return;
        const BSeg cs = segs[s.child];
        const int i = node % s.nnx, j = node / s.nnx;
        const uint8_t mf = nmask[s.noff + node];
        const int i0 = i >> 1, j0 = j >> 1, ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1;
        T acc[2] = {T(0), T(0)};
        for (int dj = 0; dj < nj; ++dj)
            for (int di = 0; di < ni; ++di) {
                const int cn = (i0 + di) + cs.nnx * (j0 + dj);
                const uint8_t mc = nmask[cs.noff + cn];
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    if (!((mc >> c) & 1)) acc[c] += zc[cs.voff + 2 * (int64_t)cn + c];
            }
        const T wt = T(1) / T(ni * nj);
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (!((mf >> c) & 1)) yf[s.voff + 2 * (int64_t)node + c] += wt * acc[c];
    });
}

// ---------------------------------------------------------------------------
// coarsest level: dense inverse, one wave per row, 4 rows per item

template <typename T>
__global__ __launch_bounds__(kBT) void k_bq_coarsest(BQueue q, const BSeg* __restrict__ segs,
                                                     const int* __restrict__ active, const double* __restrict__ Ainv,
                                                     const T* __restrict__ r, T* __restrict__ z) {
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (active && !active[s.inst]) return;
        const int n = 2 * s.nnx * s.nny;
        const int row = w.first + (int)(threadIdx.x >> 6);
        const int lane = (int)(threadIdx.x & 63);
        if (row >= n) return;   // whole wave
        const double* Ar = Ainv + s.coff + (int64_t)row * n;
        const T* rs = r + s.voff;
        double acc = 0.0;
        for (int col = lane; col < n; col += 64) acc += Ar[col] * (double)rs[col];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        z[s.voff + row] = (T)__shfl(acc, 0, 64);   // same value from every lane (uniform store)
    });
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting), one block
// per instance.  Thread (tx, ty) = (tid mod 64, tid / 64) owns the entries
// (i, j) with i = ty mod 16 and j = tx mod 64, so global memory is only ever
// touched by its owner and a wave updates 64 consecutive entries of a row;
// the pivot row and column travel through LDS: while updating step k the
// owners of row / column k+1 also write them to the next LDS buffer.  Each
// step first divides the pivot row by the pivot once (n divisions) and then
// updates every entry with one multiply-add.
constexpr int kGjThreads = 1024;
constexpr int kGjCols = 64;                       // threads along a row
constexpr int kGjRows = kGjThreads / kGjCols;     // rows updated concurrently
constexpr int kGjMax = 1024;

__global__ __launch_bounds__(kGjThreads) void k_bq_gj(const int* __restrict__ cs, const BSeg* __restrict__ segs,
                                                      double* __restrict__ Ainv) {
    __shared__ double rowb[2][kGjMax], colb[2][kGjMax], rs[kGjMax];
    const BSeg s = segs[cs[blockIdx.x]];
    const int n = 2 * s.nnx * s.nny;
    double* A = Ainv + s.coff;
    const int tx = threadIdx.x % kGjCols, ty = threadIdx.x / kGjCols;
    for (int t = threadIdx.x; t < n; t += kGjThreads) {
        rowb[0][t] = A[t];
        colb[0][t] = A[(int64_t)t * n];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double* rowk = rowb[k & 1];
        const double* colk = colb[k & 1];
        double* rown = rowb[(k + 1) & 1];
        double* coln = colb[(k + 1) & 1];
        const double p = rowk[k];
        for (int j = threadIdx.x; j < n; j += kGjThreads) rs[j] = rowk[j] / p;
        __syncthreads();
        for (int i = ty; i < n; i += kGjRows) {
            const double ci = colk[i];
            double* Ai = A + (int64_t)i * n;
            for (int j = tx; j < n; j += kGjCols) {
                double v;
                if (i == k && j == k) v = 1.0 / p;
                else if (i == k) v = rs[j];
                else if (j == k) v = -ci / p;
                else v = Ai[j] - ci * rs[j];
                Ai[j] = v;
                if (i == k + 1) rown[j] = v;
                if (j == k + 1) coln[i] = v;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// CG vector steps (fine items only)

__global__ __launch_bounds__(kBT) void k_bq_cg_init(BQueue q, const BSeg* __restrict__ segs,
                                                    const uint8_t* __restrict__ nmask, const double* __restrict__ F,
                                                    double* __restrict__ X, double* __restrict__ R,
                                                    double* __restrict__ part) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const int node = w.first + (int)threadIdx.x;
        double a = 0.0;
        if (node < s.nnx * s.nny) {
            const uint8_t m = nmask[s.noff + node];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                const double f = ((m >> c) & 1) ? 0.0 : F[d];
                X[d] = 0.0;
                R[d] = f;
                a += f * f;
            }
        }
        const double sum = bq_block_sum(a, sh);
        if (threadIdx.x < 64) part[it] = sum;
    });
}

__global__ __launch_bounds__(kBT) void k_bq_cg_update(BQueue q, const BSeg* __restrict__ segs,
                                                      const int* __restrict__ active, const int* __restrict__ ib,
                                                      const int* __restrict__ ie, const double* __restrict__ pq_part,
                                                      const double* __restrict__ rz, const double* __restrict__ P,
                                                      const double* __restrict__ Q, const double* __restrict__ Z,
                                                      double* __restrict__ X, double* __restrict__ R,
                                                      double* __restrict__ rr_part, double* __restrict__ rzx_part,
                                                      int* __restrict__ flags) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (!active[s.inst]) {
            if (threadIdx.x < 64) {
                rr_part[it] = 0.0;
                rzx_part[it] = 0.0;
            }
            return;
        }
        const double pq = bq_range_sum(pq_part, ib[s.inst], ie[s.inst], sh);
        const bool ok = pq > 0.0 && pq < __builtin_huge_val();
        if (!ok && threadIdx.x < 64) atomicOr(&flags[s.inst], 1);
        const double alpha = ok ? rz[s.inst] / pq : 0.0;
        const int node = w.first + (int)threadIdx.x;
        double a = 0.0, bx = 0.0;
        if (node < s.nnx * s.nny) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                X[d] += alpha * P[d];
                const double rv = R[d] - alpha * Q[d];
                R[d] = rv;
                a += rv * rv;
                bx += rv * Z[d];   // r_{k+1} . z_k for the flexible beta
            }
        }
        const double sum = bq_block_sum(a, sh);
        const double sumx = bq_block_sum(bx, sh);
        if (threadIdx.x < 64) {
            rr_part[it] = sum;
            rzx_part[it] = sumx;
        }
    });
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_bq_finish(BQueue q, const BSeg* __restrict__ segs,
                                                   const int* __restrict__ active, const T* __restrict__ zt,
                                                   const double* __restrict__ R, double* __restrict__ Z,
                                                   double* __restrict__ part) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (!active[s.inst]) {
            if (threadIdx.x < 64) part[it] = 0.0;
            return;
        }
        const int node = w.first + (int)threadIdx.x;
        double a = 0.0;
        if (node < s.nnx * s.nny) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                const double z = (double)zt[d];
                Z[d] = z;
                a += R[d] * z;
            }
        }
        const double sum = bq_block_sum(a, sh);
        if (threadIdx.x < 64) part[it] = sum;
    });
}

__global__ __launch_bounds__(kBT) void k_bq_cg_dir(BQueue q, const BSeg* __restrict__ segs,
                                                   const int* __restrict__ active, const double* __restrict__ beta,
                                                   int first, const double* __restrict__ Z, double* __restrict__ P) {
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        if (!active[s.inst]) return;
        const int node = w.first + (int)threadIdx.x;
        if (node >= s.nnx * s.nny) return;
        const double b = beta[s.inst];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int64_t d = s.voff + 2 * (int64_t)node + c;
            P[d] = first ? Z[d] : Z[d] + b * P[d];
        }
    });
}

// one wave per instance: fixed-order sum of the instance's partials
__device__ inline double bq_wave_range_sum(const double* __restrict__ part, int lo, int hi) {
    const int lane = (int)(threadIdx.x & 63);
    double v = 0.0;
    for (int k = lo + lane; k < hi; k += 64) v += part[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;   // lane 0
}

__global__ void k_bq_check_res(int ninst, int first, double tol2, const int* __restrict__ ib,
                               const int* __restrict__ ie, const double* __restrict__ part, double* __restrict__ ff,
                               double* __restrict__ thr, double* __restrict__ rr, int* __restrict__ active,
                               int* __restrict__ iters, int* __restrict__ flags) {
    const int inst = blockIdx.x;
    if (inst >= ninst) return;
    const double s = bq_wave_range_sum(part, ib[inst], ie[inst]);
    if (threadIdx.x != 0) return;
    const bool finite = s == s && s < __builtin_huge_val();
    if (first) {
        ff[inst] = s;
        thr[inst] = tol2 * s;
        rr[inst] = s;
        iters[inst] = 0;
        if (!finite) flags[inst] |= 2;
        active[inst] = (finite && s > 0.0) ? 1 : 0;   // zero load: u = 0
        return;
    }
    if (!active[inst]) return;
    iters[inst] += 1;
    rr[inst] = s;
    if (!finite) {
        flags[inst] |= 2;
        active[inst] = 0;
    } else if (s <= thr[inst]) {
        active[inst] = 0;
    }
}

// beta = r_{k+1}.z_{k+1} / r_k.z_k, or with flex (FP32 cycle, which is not
// exactly a fixed symmetric operator) the flexible form
// (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / r_k.z_k, as in the single-problem solver.
__global__ void k_bq_check_rz(int ninst, int first, int flex, const int* __restrict__ ib, const int* __restrict__ ie,
                              const double* __restrict__ part, const double* __restrict__ xpart,
                              const int* __restrict__ active, double* __restrict__ rz, double* __restrict__ beta,
                              int* __restrict__ flags) {
    const int inst = blockIdx.x;
    if (inst >= ninst) return;
    const double s = bq_wave_range_sum(part, ib[inst], ie[inst]);
    const double x = flex && !first ? bq_wave_range_sum(xpart, ib[inst], ie[inst]) : 0.0;
    if (threadIdx.x != 0 || !active[inst]) return;
    if (!(s > 0.0 && s < __builtin_huge_val())) flags[inst] |= 4;   // preconditioner lost definiteness
    beta[inst] = first ? 0.0 : (s - x) / rz[inst];
    rz[inst] = s;
}

__global__ __launch_bounds__(kBT) void k_bq_dot(BQueue q, const BSeg* __restrict__ segs,
                                                const uint8_t* __restrict__ nmask, const double* __restrict__ a,
                                                const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const int node = w.first + (int)threadIdx.x;
        double v = 0.0;
        if (node < s.nnx * s.nny) {
            const uint8_t m = nmask[s.noff + node];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                if (!((m >> c) & 1)) v += a[d] * b[d];
            }
        }
        const double sum = bq_block_sum(v, sh);
        if (threadIdx.x < 64) part[it] = sum;
    });
}

// ---------------------------------------------------------------------------
// power iteration for the Jacobi weights

// SplitMix64 finaliser (Steele, Lea & Flood 2014) of a counter: a uniform
// value in [-1, 1) per (seed, segment, DOF).
__device__ inline double hash_uniform(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (ctr + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ __launch_bounds__(kBT) void k_bq_random(BQueue q, const BSeg* __restrict__ segs,
                                                   const uint8_t* __restrict__ nmask, uint64_t seed,
                                                   double* __restrict__ v, double* __restrict__ part) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const int node = w.first + (int)threadIdx.x;
        double a = 0.0;
        if (node < s.nnx * s.nny) {
            const uint8_t m = nmask[s.noff + node];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int64_t d = s.voff + 2 * (int64_t)node + c;
                const double val = ((m >> c) & 1) ? 0.0 : hash_uniform(seed, (uint64_t)d);
                v[d] = val;
                a += val * val;
            }
        }
        const double sum = bq_block_sum(a, sh);
        if (threadIdx.x < 64) part[it] = sum;
    });
}

__global__ __launch_bounds__(kBT) void k_bq_normalize(BQueue q, const BSeg* __restrict__ segs,
                                                      const int* __restrict__ pb, const int* __restrict__ pe,
                                                      const double* __restrict__ part, double* __restrict__ v) {
    __shared__ double sh[4];
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const double nrm = bq_range_sum(part, pb[w.seg], pe[w.seg], sh);
        const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
        const int node = w.first + (int)threadIdx.x;
        if (node < s.nnx * s.nny) {
            const int64_t d = s.voff + 2 * (int64_t)node;
            v[d] *= inv;
            v[d + 1] *= inv;
        }
    });
}

// ---------------------------------------------------------------------------
// compliance sensitivity dJ/dx_e = -p x_e^(p-1) (E1 - E0) u_e^T K0 u_e

__global__ __launch_bounds__(kBT) void k_bq_dJ(BQueue q, const BSeg* __restrict__ segs,
                                               const double* __restrict__ x, double p, double dE, BK0<double> K0,
                                               const double* __restrict__ U, double* __restrict__ dJ) {
    bq_drain(q, [&](int it) {
        const BItem w = q.items[it];
        const BSeg s = segs[w.seg];
        const int e = w.first + (int)threadIdx.x;
        if (e >= s.nx * s.ny) return;
        const int ei = e % s.nx, ej = e / s.nx;
        double ue[8];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t nd = (ei + (b & 1)) + (int64_t)s.nnx * (ej + (b >> 1));
            ue[2 * b] = U[s.voff + 2 * nd];
            ue[2 * b + 1] = U[s.voff + 2 * nd + 1];
        }
        double quad = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) t += K0.k[a * 8 + b] * ue[b];
            quad += ue[a] * t;
        }
        const double xe = x[s.soff + e];
        const double xp1 = p == 1.0 ? 1.0 : (xe > 0.0 ? pow(xe, p - 1.0) : 0.0);
        dJ[s.soff + e] = -p * xp1 * dE * quad;
    });
}

// ---------------------------------------------------------------------------
// launchers

int bq_grid(const BQueue& q, int max_blocks) {
    if (!q.persistent) return q.nitems;
    int b = q.nitems < max_blocks ? q.nitems : max_blocks;
    if (b >= 8) b = (b + 7) / 8 * 8;
    return b;
}

template <typename T, typename TR, int MODE, int DOT>
static void apply_inst(const BQueue& q, int blocks, const BSeg* segs, const int* active, const T* Ek,
                       const BK0<T>& K0, const T* A, const T* dinv, const T* omega, const uint8_t* nmask,
                       const T* x, T* y, const TR* r, const double* dsrc, double* part, hipStream_t st) {
    hipLaunchKernelGGL((k_bq_apply<T, TR, MODE, DOT>), dim3(blocks), dim3(kBT), 0, st, q, segs, active, Ek, K0, A,
                       dinv, omega, nmask, x, y, r, dsrc, part);
}

template <typename T, typename TR, int MODE>
static void apply_dot(int dot, const BQueue& q, int blocks, const BSeg* segs, const int* active, const T* Ek,
                      const BK0<T>& K0, const T* A, const T* dinv, const T* omega, const uint8_t* nmask, const T* x,
                      T* y, const TR* r, const double* dsrc, double* part, hipStream_t st) {
    if (dot == 0) apply_inst<T, TR, MODE, 0>(q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st);
    else if (dot == 1) apply_inst<T, TR, MODE, 1>(q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st);
    else apply_inst<T, TR, MODE, 2>(q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st);
}

template <typename T, typename TR>
void launch_bq_apply(const BQueue& q, int blocks, int mode, int dot, const BSeg* segs, const int* active, const T* Ek,
                     const BK0<T>& K0, const T* A, const T* dinv, const T* omega, const uint8_t* nmask, const T* x,
                     T* y, const TR* r, const double* dsrc, double* part, hipStream_t st) {
    if (blocks <= 0) return;
    switch (mode) {
    case kBY: apply_dot<T, TR, kBY>(dot, q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st); break;
    case kBRes: apply_dot<T, TR, kBRes>(dot, q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st); break;
    case kBJac: apply_dot<T, TR, kBJac>(dot, q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st); break;
    case kBJac0: apply_dot<T, TR, kBJac0>(dot, q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st); break;
    default: apply_dot<T, TR, kBDinvY>(dot, q, blocks, segs, active, Ek, K0, A, dinv, omega, nmask, x, y, r, dsrc, part, st); break;
    }
}

template <typename T>
void launch_bq_restrict(const BQueue& q, int blocks, const BSeg* segs, const int* active, const uint8_t* nmask,
                        const T* xf, T* yc, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_restrict<T>, dim3(blocks), dim3(kBT), 0, st, q, segs, active, nmask, xf, yc);
}

template <typename T>
void launch_bq_prolong_add(const BQueue& q, int blocks, const BSeg* segs, const int* active, const uint8_t* nmask,
                           const T* zc, T* yf, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_prolong_add<T>, dim3(blocks), dim3(kBT), 0, st, q, segs, active, nmask, zc, yf);
}

template <typename T>
void launch_bq_coarsest(const BQueue& q, int blocks, const BSeg* segs, const int* active, const double* Ainv,
                        const T* r, T* z, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_coarsest<T>, dim3(blocks), dim3(kBT), 0, st, q, segs, active, Ainv, r, z);
}

void launch_bq_gj(int nseg_coarsest, const int* coarsest_segs, const BSeg* segs, double* Ainv, hipStream_t st) {
    if (nseg_coarsest <= 0) return;
    hipLaunchKernelGGL(k_bq_gj, dim3(nseg_coarsest), dim3(kGjThreads), 0, st, coarsest_segs, segs, Ainv);
}

void launch_bq_res_dd(const BQueue& q, int blocks, const BSeg* segs, const double* Ek, const BK0<double>& K0,
                      const uint8_t* nmask, const double* x, const double* xlo, const int* skip, const double* f,
                      double* r, double* part, double* part2, hipStream_t st) {
    hipLaunchKernelGGL(k_bq_res_dd, dim3(blocks), dim3(kBT), 0, st, q, segs, Ek, K0, nmask, x, xlo, skip, f, r, part,
                       part2);
}

// (hi, lo) += d as a double-double per entry (two-sum, then renormalised so
// that hi = fl(hi + lo)).
__global__ void k_dd_add(int64_t n, const double* __restrict__ d, double* __restrict__ hi, double* __restrict__ lo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s, e;
    bq_two_sum(hi[i], d[i], s, e);
    const double l = lo[i] + e;
    const double h = s + l;
    hi[i] = h;
    lo[i] = l - (h - s);
}

void launch_dd_add(int64_t n, const double* d, double* hi, double* lo, hipStream_t st) {
    hipLaunchKernelGGL(k_dd_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, d, hi, lo);
}

void launch_bq_cg_init(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, const double* F,
                       double* X, double* R, double* part, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_cg_init, dim3(blocks), dim3(kBT), 0, st, q, segs, nmask, F, X, R, part);
}

void launch_bq_cg_update(const BQueue& q, int blocks, const BSeg* segs, const int* active, const int* ib, const int* ie,
                         const double* pq_part, const double* rz, const double* P, const double* Q, const double* Z,
                         double* X, double* R, double* rr_part, double* rzx_part, int* flags, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_cg_update, dim3(blocks), dim3(kBT), 0, st, q, segs, active, ib, ie, pq_part, rz, P, Q, Z,
                       X, R, rr_part, rzx_part, flags);
}

template <typename T>
void launch_bq_finish(const BQueue& q, int blocks, const BSeg* segs, const int* active, const T* zt, const double* R,
                      double* Z, double* rz_part, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_finish<T>, dim3(blocks), dim3(kBT), 0, st, q, segs, active, zt, R, Z, rz_part);
}

void launch_bq_cg_dir(const BQueue& q, int blocks, const BSeg* segs, const int* active, const double* beta, int first,
                      const double* Z, double* P, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_cg_dir, dim3(blocks), dim3(kBT), 0, st, q, segs, active, beta, first, Z, P);
}

void launch_bq_check_res(int ninst, int first, double tol2, const int* ib, const int* ie, const double* rr_part,
                         double* ff, double* thr, double* rr, int* active, int* iters, int* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_bq_check_res, dim3(ninst), dim3(64), 0, st, ninst, first, tol2, ib, ie, rr_part, ff, thr, rr,
                       active, iters, flags);
}

void launch_bq_check_rz(int ninst, int first, int flex, const int* ib, const int* ie, const double* rz_part,
                        const double* rzx_part, const int* active, double* rz, double* beta, int* flags,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_bq_check_rz, dim3(ninst), dim3(64), 0, st, ninst, first, flex, ib, ie, rz_part, rzx_part,
                       active, rz, beta, flags);
}

void launch_bq_dot(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, const double* a,
                   const double* b, double* part, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_dot, dim3(blocks), dim3(kBT), 0, st, q, segs, nmask, a, b, part);
}

void launch_bq_random(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, uint64_t seed, double* v,
                      double* part, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_random, dim3(blocks), dim3(kBT), 0, st, q, segs, nmask, seed, v, part);
}

void launch_bq_normalize(const BQueue& q, int blocks, const BSeg* segs, const int* pb, const int* pe,
                         const double* part, double* v, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_normalize, dim3(blocks), dim3(kBT), 0, st, q, segs, pb, pe, part, v);
}

void launch_bq_dJ(const BQueue& q, int blocks, const BSeg* segs, const double* x, double p, double dE,
                  const BK0<double>& K0, const double* U, double* dJ, hipStream_t st) {
    if (blocks <= 0) return;
    hipLaunchKernelGGL(k_bq_dJ, dim3(blocks), dim3(kBT), 0, st, q, segs, x, p, dE, K0, U, dJ);
}

template void launch_bq_apply<double, double>(const BQueue&, int, int, int, const BSeg*, const int*, const double*,
                                              const BK0<double>&, const double*, const double*, const double*,
                                              const uint8_t*, const double*, double*, const double*, const double*,
                                              double*, hipStream_t);
template void launch_bq_apply<float, double>(const BQueue&, int, int, int, const BSeg*, const int*, const float*,
                                             const BK0<float>&, const float*, const float*, const float*,
                                             const uint8_t*, const float*, float*, const double*, const double*,
                                             double*, hipStream_t);
template void launch_bq_apply<float, float>(const BQueue&, int, int, int, const BSeg*, const int*, const float*,
                                            const BK0<float>&, const float*, const float*, const float*,
                                            const uint8_t*, const float*, float*, const float*, const double*,
                                            double*, hipStream_t);
template void launch_bq_restrict<double>(const BQueue&, int, const BSeg*, const int*, const uint8_t*, const double*,
                                         double*, hipStream_t);
template void launch_bq_restrict<float>(const BQueue&, int, const BSeg*, const int*, const uint8_t*, const float*,
                                        float*, hipStream_t);
template void launch_bq_prolong_add<double>(const BQueue&, int, const BSeg*, const int*, const uint8_t*,
                                            const double*, double*, hipStream_t);
template void launch_bq_prolong_add<float>(const BQueue&, int, const BSeg*, const int*, const uint8_t*, const float*,
                                           float*, hipStream_t);
template void launch_bq_coarsest<double>(const BQueue&, int, const BSeg*, const int*, const double*, const double*,
                                         double*, hipStream_t);
template void launch_bq_coarsest<float>(const BQueue&, int, const BSeg*, const int*, const double*, const float*,
                                        float*, hipStream_t);
template void launch_bq_finish<double>(const BQueue&, int, const BSeg*, const int*, const double*, const double*,
                                       double*, double*, hipStream_t);
template void launch_bq_finish<float>(const BQueue&, int, const BSeg*, const int*, const float*, const double*,
                                      double*, double*, hipStream_t);

}  // namespace mlb
