// Host launchers of the HIP kernels (all enqueue on the given stream).
#pragma once

#include "common.h"

namespace mlb {

// ---- operators and transfers (kernels_apply.hip)
int64_t apply_fine_blocks(const Geo& g);
template <typename T>
void launch_apply_fine(int dim, const Geo& g, const T* E, const uint8_t* nmask, const T* K0, int ncols,
                       int64_t ld, const T* x, T* y, int mode, const T* r, const T* dinv, T omega,
                       double* dot_part, hipStream_t st);
void launch_apply_G_fine(int dim, const Geo& g, const double* S, const uint8_t* nmask, const double* Hk,
                         int ncols, int64_t ld, const double* x, double* y, hipStream_t st);
void launch_dinv_fine(int dim, const Geo& g, const double* E, const uint8_t* nmask, const double* K0,
                      double* dinv, float* dinvf, hipStream_t st);

// ---- assembled node-block stencils and transfers (kernels_stencil.hip)
// entries of a node-block stencil (half: the FP32 copy of K's, blocks nb <= NB/2)
int64_t stencil_entries(int dim, const Geo& g, bool diag, bool half = false);
// af_half: the FP32 copy Af keeps only the blocks nb <= NB/2 (what
// launch_apply_nb<float> reads); otherwise Af is the full stencil
void launch_assemble_nb(int dim, const Geo& g, const double* Ke, const uint8_t* nmask, double* A, float* Af,
                        double* dinv, float* dinvf, bool af_half, hipStream_t st);
// One Kaczmarz sweep for (K + sigma G) x = 0 on every column of X (a
// Galerkin level: K full node-block stencil, Gd block-diagonal stencil), rows
// in colour order (i mod 3) + 3 (j mod 3) + 9 (k mod 3); Dirichlet rows skipped.
void launch_kaczmarz_sweep(int dim, const Geo& g, const double* A, const double* Gd, double sigma,
                           const uint8_t* nmask, int ncols, int64_t ld, double* X, hipStream_t st);
// fine-grid element matrices E_e K0 and sum_q S_qe H_q ([entry m + e])
void launch_fine_elem_mats(int dim, const Geo& g, const double* E, const double* K0, const double* S,
                           const double* Hk, double* Ke, double* Ge, hipStream_t st);
void launch_assemble_nb_diag(int dim, const Geo& g, const double* Ge, const uint8_t* nmask, double* A,
                             hipStream_t st);
template <typename T>
void launch_apply_nb(int dim, const Geo& g, const T* A, bool diag, int ncols, int64_t ld, const T* x, T* y, int mode,
                     const T* r, const T* dinv, T omega, int cbmax, hipStream_t st);
template <typename T>
void launch_prolong_nb(int dim, const Geo& gf, const Geo& gc, const uint8_t* mf, const uint8_t* mc, int ncols,
                       int64_t ldf, int64_t ldc, const T* xc, T* yf, bool add, hipStream_t st);
template <typename T>
void launch_restrict_nb(int dim, const Geo& gf, const Geo& gc, const uint8_t* mf, const uint8_t* mc, int ncols,
                        int64_t ldf, int64_t ldc, const T* xf, T* yc, hipStream_t st);

// ---- element-centric Walsh-Hadamard apply (kernels_wht.hip)
// variant (3D): 0 register tiles of 8 x 8 element columns per wave with the
// next node plane prefetched, 1 tiles of 16 x 16 columns per block staged in
// LDS, 2 register tiles without prefetch (fewer registers, more waves), 3
// register tiles with per-plane transforms and buffer accesses (levels whose
// vectors exceed 1 GiB run variant 0)
int64_t apply_wht_blocks(int dim, const Geo& g, int zchunk, int variant);
template <typename T>
void launch_apply_wht(int dim, const Geo& g, const T* E, const uint8_t* nmask, const T* blocks, int ncols,
                      int64_t ld, const T* x, T* y, int mode, const T* r, const T* dinv, T omega, double* dot_part,
                      bool clean, int zchunk, int variant, hipStream_t st);

// ---- setup (kernels_setup.hip)
void launch_material(int64_t m, const double* x, double E1, double E0, double p, double* Ek, float* Ekf,
                     double* Es, int nparts, double* bad_part, hipStream_t st);
void launch_node_mask(int64_t nodes, int dim, const uint8_t* fixed_dof, uint8_t* nmask, hipStream_t st);
void launch_coarse_mask(const Geo& gf, const Geo& gc, const uint8_t* mf, uint8_t* mc, hipStream_t st);
void launch_galerkin_from_E(int dim, const Geo& gf, const Geo& gc, const double* E, const double* Mc,
                            double* Kc, hipStream_t st);
void launch_galerkin_G_from_S(int dim, const Geo& gf, const Geo& gc, const double* S, const double* GHc,
                              double* gc_out, hipStream_t st);
void launch_galerkin_dense(int dim, bool kron, const Geo& gf, const Geo& gc, const double* Kf,
                           const double* T, double* Kc, hipStream_t st);
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t st);
void launch_assemble_dense(int dim, const Geo& g, const double* Ke, const uint8_t* nmask, int64_t n, int64_t ld,
                           double* A, hipStream_t st);
void launch_pad_identity(int64_t n, int64_t N, double* A, hipStream_t st);
// coarsest level on the matrix cores (kernels_dense.hip): N = n rounded up
// to a multiple of 64; the inverse is N x N row-major with an identity pad
int coarse_pad(int64_t n);
int coarse_splits(int64_t N);
int64_t coarse_stage_doubles(int64_t N);
void launch_gemm_f64(int M, int N, int K, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                     double beta, double* C, int64_t ldc, hipStream_t st, int skip_r = -1, int skip_c = -1);
// P: 2 x 64 x 64 doubles; st2 (with its two events) overlaps each diagonal
// block inversion with the previous panel's update, or null for one stream
void launch_block_inverse(int64_t N, double* A, double* P, double* R, double* Cp, hipStream_t st,
                          hipStream_t st2 = nullptr, hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr);
// the lower triangle of a symmetric N x N row-major matrix as packed 16 x 16
// tiles (tile (R, C), R >= C, row-major at (R (R + 1) / 2 + C) 256)
int64_t packed_lower_doubles(int64_t N);
void launch_pack_lower(int64_t N, const double* A, double* Apk, hipStream_t st);
// z = A x for the packed symmetric A (up to 32 columns)
template <typename T>
void launch_coarse_solve(int64_t n, int64_t N, int nc, int64_t ld, const double* Apk, const T* x, T* z, int nsplit,
                         double* part, hipStream_t st);

// ---- vector kernels (kernels_blas.hip)
template <typename T>
void launch_jacobi0(int64_t n, int ncols, int64_t ld, const T* dinv, T omega, const T* r, T* z, hipStream_t st);
void launch_d2f(int64_t n, int ncols, int64_t ld, const double* a, float* b, hipStream_t st);
void launch_d2f_jacobi0(int64_t n, int ncols, int64_t ld, const double* a, const float* dinv, float omega, float* b,
                        float* z, hipStream_t st);
void launch_f2d(int64_t n, int ncols, int64_t ld, const float* a, double* b, hipStream_t st);
int reduction_parts(int64_t n);
void launch_dot_part(int64_t n, int ncols, int64_t lda, const double* a, int64_t ldb, const double* b,
                     int nparts, double* part, hipStream_t st);
void launch_sum_parts(int ncols, int64_t nparts, const double* part, double* out, hipStream_t st);
// device convergence test after a CG update (counts iterations of active columns)
void launch_cg_check(int ncols, const double* rr, const double* thr, int* active, int* iters, int* flags,
                     hipStream_t st);
void launch_cg_alpha(int ncols, const double* rz, const double* pq, const int* active, double* alpha,
                     int* flags, hipStream_t st);
void launch_cg_beta(int ncols, const double* rz_new, double* rz, const int* active, double* beta,
                    hipStream_t st);
void launch_cg_beta_flex(int ncols, const double* rz_new, const double* rz_cross, double* rz, const int* active,
                         double* beta, hipStream_t st);
void launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st);
void launch_rsqrt(int ncols, const double* in, double* out, hipStream_t st);
void launch_cg_update_xr(int64_t n, int ncols, int64_t ld, const double* alpha, const double* p,
                         const double* q, double* x, double* r, int nparts, double* rr_part, hipStream_t st);
void launch_cg_update_p(int64_t n, int ncols, int64_t ld, const double* beta, const double* z, double* p,
                        hipStream_t st);
void launch_copy_cols(int64_t n, int ncols, int64_t lds, const double* s, int64_t ldd, double* d,
                      hipStream_t st);
void launch_axpy_cols(int64_t n, int ncols, int64_t ld, const double* coef, double sign, const double* x,
                      double* y, hipStream_t st);
// G (device, column-major k1 x (k2a + k2b)) = A^T [B1 B2]; nparts blocks of
// partials (gram_parts) in part; returns -1 if k1 + k2a + k2b > 192.
int gram_parts(int64_t n, int k1, int k2);
int launch_gram(int64_t n, int k1, int64_t lda, const double* A, int k2a, int64_t ldb1, const double* B1, int k2b,
                int64_t ldb2, const double* B2, int nparts, double* part, double* out, hipStream_t st);
// the same with B in FP32 (one operand block, read as doubles)
int launch_gram_f32b(int64_t n, int k1, int64_t lda, const double* A, int k2, int64_t ldb, const float* B, int nparts,
                     double* part, double* out, hipStream_t st);
// out (k2 x k1, column-major) = sign G^T for G (k1 x k2, column-major)
void launch_gram_transpose(int k1, int k2, double sign, const double* G, double* out, hipStream_t st);
// block CG row updates (sp, nc <= 32)
int bcg_step_parts(int64_t n);
void launch_bcg_step(int64_t n, int sp, int nc, const double* alpha, const double* P, const double* Q, double* X,
                     double* R, double* rr_part, hipStream_t st);
void launch_bcg_dir(int64_t n, int sp, int nc, const double* beta, const double* Z, double* P, hipStream_t st);
void launch_bcg_dir(int64_t n, int sp, int nc, const double* beta, const float* Z, double* P, hipStream_t st);
// Y = alpha Y + [A1 A2] C (k1a + k1b <= 96, k2 <= 32; Y disjoint from A1, A2)
void launch_gemm_cat(int64_t n, int k1a, int64_t lda1, const double* A1, int k1b, int64_t lda2, const double* A2,
                     int k2, const double* C, double alpha, int64_t ldy, double* Y, hipStream_t st);
// V[:, :k2] = V[:, :k1] T in place (k1, k2 <= 32)
void launch_xform_inplace(int64_t n, int k1, int k2, const double* T, int64_t ld, double* V, hipStream_t st);
void launch_gemm_small(int64_t n, int k1, int64_t lds, const double* S, int k2, const double* C, int64_t ldy,
                       double* Y, hipStream_t st);
void launch_residual_block(int64_t n, int ncols, int64_t ld, const double* AX, const double* KX,
                           const double* mu, double* R, hipStream_t st);
void launch_random_fill(int64_t n, int ncols, int64_t ld, uint64_t seed, const uint8_t* nmask, int dim,
                        double* X, hipStream_t st);
void launch_mask_fixed(int64_t n, int ncols, int64_t ld, const uint8_t* nmask, int dim, double* X, hipStream_t st);
void launch_absmax_part(int64_t n, int ncols, int64_t ld, const double* X, int nparts, double* pval,
                        int64_t* pidx, hipStream_t st);
void launch_absmax_sum(int ncols, int nparts, const double* pval, const int64_t* pidx, double* out_val,
                       hipStream_t st);
void launch_infnorm_part(int64_t n, int ncols, int64_t ld, const double* X, int nparts, double* part,
                         hipStream_t st);
void launch_max_parts(int ncols, int nparts, const double* part, double* out, hipStream_t st);
void launch_scale_cols(int64_t n, int ncols, int64_t ld, const double* s, double* X, hipStream_t st);

// ---- post-processing measures (kernels_post.hip)
// sed (q x m) = E_kappa phi^T K_e0 phi per element and mode
void launch_sed(int dim, const Geo& g, const double* Ek, int q, int64_t ld, const double* Phi, const double* K0,
                double* sed, hipStream_t st);
// gradn (q x m) = |grad sed| on {x >= xbar}; part (q x grad_tv_parts) block sums of gradn there
int grad_tv_parts(const Geo& g);
void launch_grad_tv(int dim, const Geo& g, const double* x, double xbar, int q, const double* sed, double* gradn,
                    double* part, hipStream_t st);
// xout = dilation of x around elements flagged by gradn >= rel_thr * gmax (nsel rows)
// device address of the fixed scratch array on `device` (which must be the
// current device); looked up once per device (scratch.hip)
hipError_t scratch_address(int device, double** out);
void launch_dilate(int dim, const Geo& g, int nsel, const double* gradn, const double* gmax, double rel_thr,
                   double r_th, const double* x, double* xout, hipStream_t st);

// ---- design variables (kernels_design.hip); tab: nt entries (di, dj, dk, w)
void launch_filter_project(const Geo& g, int nt, const double* tab, double eta, double beta, const double* xhat,
                           double* xtilde, double* x, hipStream_t st);
void launch_filter_chain(const Geo& g, int nt, const double* tab, double eta, double beta, int ncols,
                         const double* xtilde, const double* dfdx, double* work, double* out, hipStream_t st);

// ---- physics (kernels_sens.hip)
void launch_stress(int dim, const Geo& g, const double* Es, const double* u, const double* D0Bc, double* S,
                   hipStream_t st);
void launch_dJ(int dim, const Geo& g, const double* x, double p, double dE, int ncases, int64_t ld,
               const double* U, const double* K0, double* dJ, hipStream_t st);
// W, Ps, lam non-null: the consistent variant (bilinear residual terms)
void launch_adj_elem(int dim, const Geo& g, const double* Es, int q, int64_t ld, const double* Phi,
                     const double* Hk, const double* D0, double* V, hipStream_t st, const double* W = nullptr,
                     const double* Ps = nullptr, const double* lam = nullptr);
void launch_adj_gather(int dim, const Geo& g, int q, const double* V, const double* Bc, const uint8_t* nmask,
                       int64_t ld, double* B, hipStream_t st);
void launch_dlam(int dim, const Geo& g, const double* x, double p, double E1, double E0, const double* u, int q,
                 int64_t ld, const double* Phi, const double* Z, const double* lam, const double* K0,
                 const double* Hk, const double* D0Bc, double* out, hipStream_t st, const double* W = nullptr,
                 const double* Ps = nullptr);

// ---- warm-start network (kernels_nn.hip)
int launch_nn_conv3d(int N, int Ci, int Co, int D, int H, int W, int K, int trans, const float* x, const uint16_t* w,
                     const float* bias, float* y, int relu, hipStream_t st);
int launch_nn_conv3d_mfma(int N, int Ci, int Co, int D, int H, int W, const float* x, const uint16_t* w,
                          const float* bias, float* y, int relu, hipStream_t st);
int launch_nn_conv3d_wgrad(int N, int Ci, int Co, int D, int H, int W, int K, const float* x, const float* dy,
                           float* dw, float* db, hipStream_t st);
void launch_nn_relu_mask(int64_t n, const float* y, float* g, hipStream_t st);
void launch_nn_pool2(int64_t planes, int D, int H, int W, float scale, const float* x, float* y, hipStream_t st);
void launch_nn_axpy(int64_t n, float a, const float* x, float* y, hipStream_t st);
void launch_nn_unpool2(int64_t planes, int D, int H, int W, float scale, const float* gy, float* gx, hipStream_t st);
void launch_nn_concat(int N, int Ca, int Cb, int64_t V, const float* a, const float* b, float* y, hipStream_t st);
void launch_nn_split(int N, int Ca, int Cb, int64_t V, const float* y, float* a, float* b, hipStream_t st);
void launch_nn_cell2node(int64_t planes, int D, int H, int W, const float* c, float* nd, hipStream_t st);
void launch_nn_nodes_to_dofs(int nfields, int64_t nodes, const float* ch, double* b, hipStream_t st);
void launch_nn_node2cell_grad(int64_t planes, int D, int H, int W, const float* gn, float* gc, hipStream_t st);
int nn_mse_parts(int64_t n);
void launch_nn_mse(int64_t n, const float* pred, const float* target, const float* weight, float scale, float* grad,
                   int nparts, double* part, hipStream_t st);
void launch_nn_adam(int64_t n, float lr, float b1, float b2, float eps, int step, float* w, uint16_t* wb,
                    const float* g, float* m, float* v, hipStream_t st);
void launch_nn_to_bf16(int64_t n, const float* a, uint16_t* b, hipStream_t st);

// method of moving asymptotes and design-problem columns (kernels_mma.hip)
constexpr int kMmaMaxCon = 32;
struct MmaLam {
    double v[kMmaMaxCon];
};
struct MmaParams {
    double xmin, xmax, move, asyinit, asyincr, asydecr;
};
int mma_parts(int64_t n);
void launch_mma_prep(int64_t n, int m, int it, const MmaParams& pr, const double* x, double* xold1, double* xold2,
                     double* low, double* upp, double* alo, double* bhi, const double* df0, const double* dfdx,
                     int64_t ldg, int nparts, double* part, hipStream_t st);
void launch_mma_dual(int64_t n, int m, const MmaLam& lam, const MmaParams& pr, const double* xk, const double* low,
                     const double* upp, const double* alo, const double* bhi, const double* df0, const double* dfdx,
                     int64_t ldg, int nparts, double* part, double* B, double* xout, hipStream_t st);
void launch_opt_cols(int64_t m, int kind, int nb, const double* x, const double* dJ, double sJ, double vcol,
                     const double* dlam, int64_t ld, const MmaLam& w, double* grad, int nparts, double* part,
                     hipStream_t st);

}  // namespace mlb
