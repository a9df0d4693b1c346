// Internal declarations of the batched-instance kernels (kernels_batch.hip):
// many independent 2D Q4 problems advanced by one launch per solver step.
#pragma once

#include "common.h"

namespace mlb {

// One grid level of one instance.  Level-space vectors hold the levels of all
// instances; level-1 segments come first, in instance order, so level-1
// offsets are those of the batched user layout.
struct BSeg {
    int nx, ny;        // elements
    int nnx, nny;      // nodes
    int inst, level;   // level 1 = fine
    int parent, child; // finer / coarser segment of the same instance (-1: none)
    int64_t voff;      // DOF offset in the level space
    int64_t noff;      // node offset (node masks)
    int64_t soff;      // level 1: element offset; levels >= 2: stencil offset (36 entries per node)
    int64_t coff;      // coarsest segment: offset of its dense inverse (row-major n x n), else -1
};

// A work item: `first` node (apply, transfer, vector items), first row
// (dense items, 4 rows) or first element (element items) of a segment.
struct BItem {
    int seg;
    int first;
};

constexpr int kBItemNodes = 256;   // nodes (or elements) per item, one per thread
constexpr int kBCtr = 16;          // counters per queue slot: 8 XCD queues, 1 finished-block count

// A work list drained by one launch.  Persistent mode: a grid of `blocks`
// blocks pulls items from 8 XCD-local queues (contiguous eighths of the
// list), stealing from the other queues when its own is empty; the last
// block to finish resets the counters.  Otherwise one block per item.
struct BQueue {
    const BItem* items;
    int nitems;
    unsigned* ctr;     // kBCtr counters, zero at launch
    int persistent;
};

enum BMode { kBY = 0, kBRes = 1, kBJac = 2, kBJac0 = 3, kBDinvY = 4 };

template <typename T>
struct BK0 {
    T k[64];           // unit-modulus Q4 element stiffness, row-major 8 x 8
};

int bq_grid(const BQueue& q, int max_blocks);

// y = A x | r - A x | x + om D^-1 (r - A x) | om D^-1 r | D^-1 A x over the
// items' nodes; level 1 matrix free from the moduli, other levels from the
// node-block stencils.  dot: 0 none, 1 partial sum of dsrc . y per item,
// 2 partial sum of y . y per item (free DOFs; y is zero at fixed DOFs except
// in mode kBY, where fixed rows are identity rows).
template <typename T, typename TR>
void launch_bq_apply(const BQueue& q, int blocks, int mode, int dot, const BSeg* segs, const int* active,
                     const T* Ek, const BK0<T>& K0, const T* A, const T* dinv, const T* omega,
                     const uint8_t* nmask, const T* x, T* y, const TR* r, const double* dsrc, double* part,
                     hipStream_t st);
// restriction to the items' (coarse) segments from their parents
template <typename T>
void launch_bq_restrict(const BQueue& q, int blocks, const BSeg* segs, const int* active, const uint8_t* nmask,
                        const T* xf, T* yc, hipStream_t st);
// yf += P zc on the items' (fine) segments from their children
template <typename T>
void launch_bq_prolong_add(const BQueue& q, int blocks, const BSeg* segs, const int* active, const uint8_t* nmask,
                           const T* zc, T* yf, hipStream_t st);
// z = Ainv r on coarsest segments (items of 4 rows)
template <typename T>
void launch_bq_coarsest(const BQueue& q, int blocks, const BSeg* segs, const int* active, const double* Ainv,
                        const T* r, T* z, hipStream_t st);
// Gauss-Jordan inversion of every instance's coarsest matrix, one block each
void launch_bq_gj(int nseg_coarsest, const int* coarsest_segs, const BSeg* segs, double* Ainv, hipStream_t st);

// CG steps on the fine items (level-1 segments); per-instance sums are
// formed from the per-item partials of the instance's item range [ib, ie).
// r = f - K (x + xlo) (fine level, free DOFs; xlo may be NULL) accumulated in
// double-double; per item partial sums of r.r and of (|K||x|).(|K||x|) over
// free DOFs; r zero for instances with skip[inst] != 0 (skip may be NULL).
void launch_bq_res_dd(const BQueue& q, int blocks, const BSeg* segs, const double* Ek, const BK0<double>& K0,
                      const uint8_t* nmask, const double* x, const double* xlo, const int* skip, const double* f,
                      double* r, double* part, double* part2, hipStream_t st);
// (hi, lo) += d per entry in double-double
void launch_dd_add(int64_t n, const double* d, double* hi, double* lo, hipStream_t st);
void launch_bq_cg_init(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, const double* F,
                       double* X, double* R, double* part, hipStream_t st);
void launch_bq_cg_update(const BQueue& q, int blocks, const BSeg* segs, const int* active, const int* ib,
                         const int* ie, const double* pq_part, const double* rz, const double* P, const double* Q,
                         const double* Z, double* X, double* R, double* rr_part, double* rzx_part, int* flags,
                         hipStream_t st);
template <typename T>
void launch_bq_finish(const BQueue& q, int blocks, const BSeg* segs, const int* active, const T* zt,
                      const double* R, double* Z, double* rz_part, hipStream_t st);
void launch_bq_cg_dir(const BQueue& q, int blocks, const BSeg* segs, const int* active, const double* beta,
                      int first, const double* Z, double* P, hipStream_t st);
// per-instance convergence test on the residual partials (first: sets the
// thresholds tol^2 ||f||^2) and the CG scalars from the r.z partials (flex:
// flexible beta from the r_{k+1}.z_k partials as well)
void launch_bq_check_res(int ninst, int first, double tol2, const int* ib, const int* ie, const double* rr_part,
                         double* ff, double* thr, double* rr, int* active, int* iters, int* flags, hipStream_t st);
void launch_bq_check_rz(int ninst, int first, int flex, const int* ib, const int* ie, const double* rz_part,
                        const double* rzx_part, const int* active, double* rz, double* beta, int* flags,
                        hipStream_t st);
// partial sums of a . b per fine item (free DOFs)
void launch_bq_dot(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, const double* a,
                   const double* b, double* part, hipStream_t st);

// power iteration helpers (items of any level): random start (counter-based
// hash, zero at fixed DOFs) with y.y partials; scaling by the segment's norm
// from its item range [pb, pe) of the partials
void launch_bq_random(const BQueue& q, int blocks, const BSeg* segs, const uint8_t* nmask, uint64_t seed,
                      double* v, double* part, hipStream_t st);
void launch_bq_normalize(const BQueue& q, int blocks, const BSeg* segs, const int* pb, const int* pe,
                         const double* part, double* v, hipStream_t st);

// compliance sensitivities on element items of the level-1 segments
void launch_bq_dJ(const BQueue& q, int blocks, const BSeg* segs, const double* x, double p, double dE,
                  const BK0<double>& K0, const double* U, double* dJ, hipStream_t st);

}  // namespace mlb
