// Host runtime behind the C ABI: context, multigrid hierarchy, V-cycle,
// block PCG, coarse eigensolver, Rayleigh-Ritz and sensitivities.
//
// The analysis follows the paper (Alg. 1 and Sec. 2.1):
//   LA       K u = f by CG preconditioned with a geometric-multigrid V-cycle
//            on the nested grids (Alg. 2, "mgPCG");
//   step 1   Galerkin K^l = P^T K P, G^l = P^T G P (Alg. 2) and the
//            lowest k positive pairs of (K^l + lambda G^l) psi = 0;
//   step 2   Psi = P_{1<-l} Psi^l;
//   step 3   K Phi~ = G Psi as one multi-column PCG (Alg. 2);
//   step 4   Rayleigh-Ritz on span(Phi~) (Alg. 2).
// The coarse eigensolver is LOBPCG for the largest mu = 1/lambda of
// (-G^l) psi = mu K^l psi, preconditioned by the V-cycle of the levels below
// l.  (The paper uses Krylov-Schur; that choice is prior art here.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlb.h"
#include "dense.h"
#include "kernels.h"
#include "tables.h"

using namespace mlb;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Level {
    Geo g{};
    int64_t n = 0;
    uint8_t* nmask = nullptr;
    double* Ke = nullptr;     // dense element matrices (levels >= 2), SoA entry-major
    double* A = nullptr;      // assembled node-block stencil of K (levels >= 2)
    float* Af = nullptr;
    double* Ge = nullptr;     // scalar element matrices of G (levels 2 .. ell)
    double* Gs = nullptr;     // block-diagonal node stencil of G (level ell)
    double* dinv = nullptr;
    float* dinvf = nullptr;
    double omega = 0.6;
    // V-cycle work, wcols columns each
    double *vr = nullptr, *vz = nullptr, *vz2 = nullptr, *vt = nullptr;
    float *fr = nullptr, *fz = nullptr, *fz2 = nullptr, *ft = nullptr;
};

}  // namespace

struct mlb_ctx {
    mlb_desc d{};
    mlb_opts o{};
    int dim = 0, nn = 0, nde = 0, nv = 0, L = 1, ell = 1;
    hipStream_t own = nullptr, st = nullptr;
    hipStream_t cap = nullptr;   // capture stream for the preconditioner graphs
    hipStream_t aux = nullptr;   // second stream of the coarsest-level inversion
    hipEvent_t aux_ev[2] = {nullptr, nullptr};
    struct Graph {
        int j, nc;
        const void* r;
        void* z;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;   // captured preconditioner applications of this hierarchy
    // tile parameters (mlb_autotune / mlb_set_tiles); operator results do not
    // depend on them (fused dot products group their partials by tile)
    int wz[2] = {8, 8};          // fine apply, FP64 / FP32: pencil length in node planes
    int wv[2] = {0, 0};          // fine apply, FP64 / FP32: 3D variant (register / LDS tiles)
    int nb_cbmax = 6;            // stencil apply: columns per thread
    float tune_stencil_ms[5] = {};
    Tables tab{};
    double *dK0 = nullptr, *dHk = nullptr, *dBc = nullptr, *dD0Bc = nullptr, *dD0 = nullptr, *dT = nullptr,
           *dMc = nullptr, *dGHc = nullptr;
    float* fK0 = nullptr;
    float whtf[9] = {};    // FP32 copy of the Walsh-Hadamard block numbers (host; passed by value)
    std::vector<Level> lv;
    int64_t n = 0, m = 0;
    // fine-level problem data
    double *x = nullptr, *Ek = nullptr, *Es = nullptr;
    float* Ekf = nullptr;
    uint8_t* fixed = nullptr;
    std::vector<uint8_t> fixed_host;
    bool has_bc = false, has_density = false, has_static = false, has_stress = false, has_buck = false;
    bool has_adj = false;
    int ncases = 0;
    int ref_case_used = 0;
    double* F = nullptr;
    double* U = nullptr;
    std::vector<double> J;
    double tol_solve = 1e-8;
    int max_it = 1000;
    double* S = nullptr;   // element stresses of the reference case (SoA nv x m)
    // coarsest level: dense FP64 inverse (N x N, N = n_L rounded up to a
    // multiple of 64, identity pad), its block Gauss-Jordan work buffers and
    // the split-K partial products of the coarsest solve
    double* Ainv = nullptr;
    double* Apk = nullptr;   // lower triangle of Ainv in packed 16 x 16 tiles
    int64_t nA = 0;
    int nsplit = 1;
    double *gjP = nullptr, *gjR = nullptr, *gjC = nullptr, *cpart = nullptr;
    // block work (fine level, cg_cap columns)
    int cg_cap = 0;
    double *R = nullptr, *Zb = nullptr, *Pb = nullptr, *Qb = nullptr, *Zo = nullptr, *X1 = nullptr, *X2 = nullptr;
    int wcols = 0;   // columns of the level buffers
    // eigen
    int k = 0;
    double *Phi = nullptr, *Zadj = nullptr, *dlam_l = nullptr;
    // for the consistent sensitivities: the interpolated coarse modes on the
    // fine grid (right-hand side basis of K Phi~ = G Psi), the Rayleigh-Ritz
    // coefficients of the returned modes (signs included), the residual
    // adjoints w = K^-1 (K + lam G) phi
    double *Psif = nullptr, *cW = nullptr;
    // fine-grid stencils of K and G, built only when the refinement of Alg. 2
    // also visits the fine grid (mlb_opts.refine_fine)
    double *fineA = nullptr, *fineGs = nullptr, *fineDinv = nullptr;
    float *fineAf = nullptr, *fineDinvf = nullptr;
    std::vector<double> rrC;
    bool psi_ok = false;
    std::vector<double> lam, eigres;
    // coarse eigensolver work
    int eig_cap = 0;
    double *eS = nullptr, *eK = nullptr, *eA = nullptr, *eT = nullptr, *eTK = nullptr, *eTA = nullptr, *eR = nullptr;
    double *eP = nullptr, *ePK = nullptr, *ePA = nullptr;
    // reductions and scalars
    double* part = nullptr;
    int64_t part_cap = 0;
    double* scratch = nullptr;   // the device's fixed scratch array (kScratchDoubles)
    bool sweep_ready = false;    // mlb_sweep_dev has given its work blocks defined contents
    int64_t* pidx = nullptr;
    double* scal = nullptr;   // 16 blocks of kScal doubles
    double* gbuf = nullptr;   // summed Gram matrices (up to 96 x 192)
    double *cbuf = nullptr, *cbuf2 = nullptr;   // small coefficient matrices
    int* iscal = nullptr;     // active / flags / iteration counts
    double* hpin = nullptr;   // pinned host staging (96 x 192 doubles)
    double* hup = nullptr;    // pinned staging of coefficient uploads (2 x 96 x 96)
    bool up_pending = false;  // an upload from hup may still be in flight
    // warm starts
    double* warm_coarse = nullptr;   // device, n_l x warm_coarse_cols
    int warm_coarse_cols = 0;
    double* warm_static = nullptr;   // device, n x warm_static_cols
    int warm_static_cols = 0;
    size_t warm_coarse_cap = 0, warm_static_cap = 0;   // allocated doubles
    // density filter weight table (di, dj, dk, w) for the radius fw_r
    double* fw = nullptr;
    int fw_n = 0;
    double fw_r = -1.0;
    std::vector<double> fw_host;
    std::string err;
};

namespace {

constexpr int kScal = 256;
// largest coarsest level (DOFs) inverted explicitly: 16384^2 doubles = 2 GiB
constexpr int64_t kMaxCoarsest = 16384;

int fail(mlb_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPC(call)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(c, MLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define CHK(expr)               \
    do {                                \
        int r_ = (expr);        \
        if (r_ != MLB_OK) return r_;    \
    } while (0)

template <typename T>
int dalloc(mlb_ctx* c, T** p, size_t count) {
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, MLB_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return MLB_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

double* sc(mlb_ctx* c, int slot) { return c->scal + slot * kScal; }

int ensure_part(mlb_ctx* c, int64_t count) {
    if (count <= c->part_cap) return MLB_OK;
    CHK(dalloc(c, &c->part, count));
    CHK(dalloc(c, &c->pidx, count));
    c->part_cap = count;
    return MLB_OK;
}

int sync(mlb_ctx* c) {
    HIPC(hipStreamSynchronize(c->st));
    c->up_pending = false;
    HIPC(hipGetLastError());
    return MLB_OK;
}

void drop_graphs(mlb_ctx* c);

// ---- level buffers

int ensure_level_cols(mlb_ctx* c, int cols) {
    if (cols <= c->wcols) return MLB_OK;
    drop_graphs(c);   // captured cycles point at the old buffers
    c->sweep_ready = false;
    for (auto& l : c->lv) {
        const size_t s = (size_t)l.n * cols;
        CHK(dalloc(c, &l.vr, s));
        CHK(dalloc(c, &l.vz, s));
        CHK(dalloc(c, &l.vz2, s));
        CHK(dalloc(c, &l.vt, s));
        CHK(dalloc(c, &l.fr, s));
        CHK(dalloc(c, &l.fz, s));
        CHK(dalloc(c, &l.fz2, s));
        CHK(dalloc(c, &l.ft, s));
    }
    c->wcols = cols;
    return MLB_OK;
}

int ensure_cg(mlb_ctx* c, int cols) {
    CHK(ensure_level_cols(c, cols));
    if (cols <= c->cg_cap) return MLB_OK;
    drop_graphs(c);
    const size_t s = (size_t)c->n * cols;
    CHK(dalloc(c, &c->R, s));
    CHK(dalloc(c, &c->Zb, s));
    CHK(dalloc(c, &c->Pb, s));
    CHK(dalloc(c, &c->Qb, s));
    CHK(dalloc(c, &c->Zo, s));
    CHK(dalloc(c, &c->X1, s));
    CHK(dalloc(c, &c->X2, s));
    c->cg_cap = cols;
    return MLB_OK;
}

// ---- operators

template <typename T>
const T* E_of(mlb_ctx* c);
template <>
const double* E_of<double>(mlb_ctx* c) { return c->Ek; }
template <>
const float* E_of<float>(mlb_ctx* c) { return c->Ekf; }
template <typename T>
const T* K0_of(mlb_ctx* c);
template <>
const double* K0_of<double>(mlb_ctx* c) { return c->dK0; }
template <>
const float* K0_of<float>(mlb_ctx* c) { return c->fK0; }
template <typename T>
const T* A_of(Level& l);
template <>
const double* A_of<double>(Level& l) { return l.A; }
template <>
const float* A_of<float>(Level& l) { return l.Af; }
template <typename T>
const T* dinv_of(Level& l);
template <>
const double* dinv_of<double>(Level& l) { return l.dinv; }
template <>
const float* dinv_of<float>(Level& l) { return l.dinvf; }

// y = A_j x (mode Y), y = r - A_j x (residual), y = x + omega D^-1 (r - A_j x) (Jacobi)
template <typename T>
const T* wht_of(mlb_ctx* c);
template <>
const double* wht_of<double>(mlb_ctx* c) { return c->tab.whs; }
template <>
const float* wht_of<float>(mlb_ctx* c) { return c->whtf; }

template <typename T>
constexpr int tix() { return sizeof(T) == 8 ? 0 : 1; }   // per-precision tile settings

// partial-sum blocks written by the level-1 apply with a fused dot product
int64_t fine_apply_blocks(mlb_ctx* c) {
    return c->tab.wht_ok ? apply_wht_blocks(c->dim, c->lv[0].g, c->wz[0], c->wv[0]) : apply_fine_blocks(c->lv[0].g);
}

// y = A_j x (mode Y), y = r - A_j x (residual), y = x + omega D^-1 (r - A_j x) (Jacobi).
// Level 1 is matrix free; the Galerkin levels read their assembled
// node-block stencils.
// `clean`: x is zero at every Dirichlet DOF (always true inside the solvers,
// whose vectors never leave the free subspace), so the level-1 kernel may
// skip masking its inputs.
template <typename T>
void apply_K(mlb_ctx* c, int j, int nc, const T* x, T* y, int mode, const T* r, double* dot_part,
             bool clean = true) {
    Level& l = c->lv[j - 1];
    if (j == 1 && c->tab.wht_ok)
        launch_apply_wht<T>(c->dim, l.g, E_of<T>(c), l.nmask, wht_of<T>(c), nc, l.n, x, y, mode, r, dinv_of<T>(l),
                            (T)l.omega, dot_part, clean, c->wz[tix<T>()], c->wv[tix<T>()], c->st);
    else if (j == 1)
        launch_apply_fine<T>(c->dim, l.g, E_of<T>(c), l.nmask, K0_of<T>(c), nc, l.n, x, y, mode, r,
                             dinv_of<T>(l), (T)l.omega, dot_part, c->st);
    else
        launch_apply_nb<T>(c->dim, l.g, A_of<T>(l), false, nc, l.n, x, y, mode, r, dinv_of<T>(l), (T)l.omega,
                           c->nb_cbmax, c->st);
}

void apply_G(mlb_ctx* c, int j, int nc, const double* x, double* y) {
    Level& l = c->lv[j - 1];
    if (j == 1) launch_apply_G_fine(c->dim, l.g, c->S, l.nmask, c->dHk, nc, l.n, x, y, c->st);
    else launch_apply_nb<double>(c->dim, l.g, l.Gs, true, nc, l.n, x, y, kModeY, nullptr, nullptr, 0.0, c->nb_cbmax,
                                 c->st);
}

template <typename T>
T* lbuf(Level& l, int which);
template <>
double* lbuf<double>(Level& l, int w) { return w == 0 ? l.vr : w == 1 ? l.vz : w == 2 ? l.vz2 : l.vt; }
template <>
float* lbuf<float>(Level& l, int w) { return w == 0 ? l.fr : w == 1 ? l.fz : w == 2 ? l.fz2 : l.ft; }

// One V(nu,nu)-cycle with damped Jacobi, symmetric (same sweeps before and
// after, restriction = interpolation^T), so it is an SPD preconditioner.
// r, z: level-j blocks with leading dimension n_j; z is overwritten.
// first_done: the first sweep from zero (a = omega D^-1 r in the level's
// block z2) was fused into the caller's conversion of r.
template <typename T>
void vcycle(mlb_ctx* c, int j, int nc, const T* r, T* z, bool first_done = false) {
    Level& l = c->lv[j - 1];
    if (j == c->L) {
        if (c->L == 1) launch_jacobi0<T>(l.n, nc, l.n, l.dinv ? dinv_of<T>(l) : nullptr, (T)1.0, r, z, c->st);
        else
            for (int c0 = 0; c0 < nc; c0 += 32)   // the product takes up to 32 columns
                launch_coarse_solve<T>(l.n, c->nA, std::min(32, nc - c0), l.n, c->Apk, r + c0 * l.n, z + c0 * l.n,
                                       c->nsplit, c->cpart, c->st);
        return;
    }
    const int nu = std::max(1, j >= 3 && c->o.coarse_sweeps > 0 ? c->o.coarse_sweeps : c->o.smooth_steps);
    T* a = lbuf<T>(l, 2);   // current iterate alternates between a and b
    T* b = z;
    T* t = lbuf<T>(l, 3);
    // 2*nu - 1 Jacobi sweeps after the first: start in z2 so the result ends in z
    if (!first_done) launch_jacobi0<T>(l.n, nc, l.n, dinv_of<T>(l), (T)l.omega, r, a, c->st);
    for (int s = 1; s < nu; ++s) {
        apply_K<T>(c, j, nc, a, b, kModeJacobi, r, nullptr);
        std::swap(a, b);
    }
    Level& lc = c->lv[j];
    T* rc = lbuf<T>(lc, 0);
    T* zc = lbuf<T>(lc, 1);
    // gamma coarse-grid corrections (1: V-cycle, 2: W-cycle; the coarsest
    // solve is exact, so one visit suffices just above it)
    const int gamma = (j + 1 == c->L) ? 1 : std::max(1, c->o.cycle);
    for (int gi = 0; gi < gamma; ++gi) {
        apply_K<T>(c, j, nc, a, t, kModeResidual, r, nullptr);
        launch_restrict_nb<T>(c->dim, l.g, lc.g, l.nmask, lc.nmask, nc, l.n, lc.n, t, rc, c->st);
        vcycle<T>(c, j + 1, nc, rc, zc);
        launch_prolong_nb<T>(c->dim, l.g, lc.g, l.nmask, lc.nmask, nc, l.n, lc.n, zc, a, true, c->st);
    }
    for (int s = 0; s < nu; ++s) {
        apply_K<T>(c, j, nc, a, b, kModeJacobi, r, nullptr);
        std::swap(a, b);
    }
    // a now holds the result; by construction a == z
}

// z = M^-1 r at level j in FP64 or mixed precision (FP32 inside).  In mixed
// precision z == nullptr leaves the result in FP32 in the level's block fz
// (for callers that read it directly).
void precondition_eager(mlb_ctx* c, int j, int nc, const double* r, double* z) {
    Level& l = c->lv[j - 1];
    if (c->d.precision == MLB_MIXED) {
        if (j < c->L) {   // the conversion and the first sweep from zero in one pass
            launch_d2f_jacobi0(l.n, nc, l.n, r, l.dinvf, (float)l.omega, l.fr, lbuf<float>(l, 2), c->st);
            vcycle<float>(c, j, nc, l.fr, l.fz, true);
        } else {
            launch_d2f(l.n, nc, l.n, r, l.fr, c->st);
            vcycle<float>(c, j, nc, l.fr, l.fz);
        }
        if (z) launch_f2d(l.n, nc, l.n, l.fz, z, c->st);
    } else {
        vcycle<double>(c, j, nc, r, z);
    }
}

void drop_graphs(mlb_ctx* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

// z = M^-1 r.  With graphs on, each (level, columns, r, z) application is
// captured once per hierarchy as a HIP graph (its 20-50 launches then cost
// one) and replayed; the graphs hold kernel arguments such as the Jacobi
// weights, so they are dropped whenever the hierarchy or the options change.
// The cycle records kernels only (no memset or copy nodes).
int precondition(mlb_ctx* c, int j, int nc, const double* r, double* z) {
    if (c->o.graphs != 1) {
        precondition_eager(c, j, nc, r, z);
        return MLB_OK;
    }
    for (auto& g : c->graphs)
        if (g.j == j && g.nc == nc && g.r == r && g.z == z) {
            HIPC(hipGraphLaunch(g.exec, c->st));
            return MLB_OK;
        }
    if (c->graphs.size() >= 128) drop_graphs(c);
    if (!c->cap) HIPC(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipStream_t saved = c->st;
    c->st = c->cap;
    HIPC(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    precondition_eager(c, j, nc, r, z);
    hipGraph_t graph = nullptr;
    const hipError_t e1 = hipStreamEndCapture(c->cap, &graph);
    c->st = saved;
    HIPC(e1);
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPC(e2);
    c->graphs.push_back({j, nc, r, z, exec});
    HIPC(hipGraphLaunch(exec, c->st));
    return MLB_OK;
}

// ---- reductions

// out (device, slot) = column dots of a and b (n x nc)
void dots(mlb_ctx* c, int64_t n, int nc, const double* a, const double* b, double* out) {
    const int np = reduction_parts(n);
    launch_dot_part(n, nc, n, a, n, b, np, c->part, c->st);
    launch_sum_parts(nc, np, c->part, out, c->st);
}

int read_scal(mlb_ctx* c, const double* dev, int count, double* host) {
    HIPC(hipMemcpyAsync(c->hpin, dev, sizeof(double) * count, hipMemcpyDeviceToHost, c->st));
    CHK(sync(c));
    std::memcpy(host, c->hpin, sizeof(double) * count);
    return MLB_OK;
}

// Gram A^T [B B2] (n x k1; n x k2, n x k2b) -> host column-major
// k1 x (k2 + k2b) (G[i + k1*j]).
int gram(mlb_ctx* c, int64_t n, int k1, const double* A, int64_t lda, int k2, const double* B, int64_t ldb,
         std::vector<double>& G, int k2b = 0, const double* B2 = nullptr, int64_t ldb2 = 0) {
    const int kt = k2 + k2b;
    if ((int64_t)k1 * kt > 96 * 192) return fail(c, MLB_EINVAL, "Gram matrix larger than 96 x 192");
    const int np = gram_parts(n, k1, kt);
    CHK(ensure_part(c, (int64_t)np * k1 * kt));
    if (launch_gram(n, k1, lda, A, k2, ldb, B, k2b, ldb2, B2, np, c->part, c->gbuf, c->st) != 0)
        return fail(c, MLB_EINVAL, "Gram operands wider than 192 columns");
    G.resize((size_t)k1 * kt);
    HIPC(hipMemcpyAsync(c->hpin, c->gbuf, sizeof(double) * k1 * kt, hipMemcpyDeviceToHost, c->st));
    CHK(sync(c));
    std::memcpy(G.data(), c->hpin, sizeof(double) * k1 * kt);
    return MLB_OK;
}

// G = A^T B (k1 x k2) -> host, B in FP32 (n x k2, leading dimension n)
int gram_f32b(mlb_ctx* c, int64_t n, int k1, const double* A, int k2, const float* B, std::vector<double>& G) {
    if ((int64_t)k1 * k2 > 96 * 192) return fail(c, MLB_EINVAL, "Gram matrix larger than 96 x 192");
    const int np = gram_parts(n, k1, k2);
    CHK(ensure_part(c, (int64_t)np * k1 * k2));
    if (launch_gram_f32b(n, k1, n, A, k2, n, B, np, c->part, c->gbuf, c->st) != 0)
        return fail(c, MLB_EINVAL, "Gram operands wider than 192 columns");
    G.resize((size_t)k1 * k2);
    HIPC(hipMemcpyAsync(c->hpin, c->gbuf, sizeof(double) * k1 * k2, hipMemcpyDeviceToHost, c->st));
    CHK(sync(c));
    std::memcpy(G.data(), c->hpin, sizeof(double) * k1 * k2);
    return MLB_OK;
}

// out = sign (A^T B)^T (k2 x k1, column-major) in device memory, enqueued
// only (no host read): the coefficients of an orthogonalisation step.
int gram_coeffs_dev(mlb_ctx* c, int64_t n, int k1, const double* A, int64_t lda, int k2, const double* B,
                    int64_t ldb, double sign, double* out) {
    if ((int64_t)k1 * k2 > 96 * 192) return fail(c, MLB_EINVAL, "Gram matrix larger than 96 x 192");
    const int np = gram_parts(n, k1, k2);
    CHK(ensure_part(c, (int64_t)np * k1 * k2));
    if (launch_gram(n, k1, lda, A, k2, ldb, B, 0, 0, nullptr, np, c->part, c->gbuf, c->st) != 0)
        return fail(c, MLB_EINVAL, "Gram operands wider than 192 columns");
    launch_gram_transpose(k1, k2, sign, c->gbuf, out, c->st);
    return MLB_OK;
}

// G1 = A^T B1, G2 = A^T B2 (each k1 x k2) in one pass over A, or in two when
// the three operands together are wider than the Gram kernel's 192 columns.
int gram2(mlb_ctx* c, int64_t n, int k1, const double* A, int k2, const double* B1, const double* B2,
          std::vector<double>& G1, std::vector<double>& G2) {
    if (k1 + 2 * k2 > 192) {
        CHK(gram(c, n, k1, A, n, k2, B1, n, G1));
        return gram(c, n, k1, A, n, k2, B2, n, G2);
    }
    std::vector<double> G;
    CHK(gram(c, n, k1, A, n, k2, B1, n, G, k2, B2, n));
    const size_t h = (size_t)k1 * k2;
    G1.assign(G.begin(), G.begin() + h);
    G2.assign(G.begin() + h, G.begin() + 2 * h);
    return MLB_OK;
}

// ---- PCG on the fine level for nc columns: K X = B.
// X holds the initial guess when use_x0, else it is zeroed.
int pcg(mlb_ctx* c, const double* B, double* X, int nc, double tol, int max_it, bool use_x0, mlb_solve_info* info) {
    const double t0 = now_s();
    const int64_t n = c->n;
    CHK(ensure_cg(c, nc));
    const int npa = (int)fine_apply_blocks(c);
    const int np = reduction_parts(n);
    CHK(ensure_part(c, (int64_t)std::max(npa, np) * nc));
    double* bb = sc(c, 0);
    double* rr = sc(c, 1);
    double* rz = sc(c, 2);
    double* pq = sc(c, 3);
    double* alpha = sc(c, 4);
    double* beta = sc(c, 5);
    double* rzn = sc(c, 6);
    int* active = c->iscal;
    int* flags = c->iscal + kScal;
    int* dits = c->iscal + 2 * kScal;
    double* thr = sc(c, 7);
    const bool flex = c->d.precision == MLB_MIXED;

    dots(c, n, nc, B, B, bb);
    if (use_x0) {
        apply_K<double>(c, 1, nc, X, c->R, kModeResidual, B, nullptr);
    } else {
        HIPC(hipMemsetAsync(X, 0, sizeof(double) * n * nc, c->st));
        launch_copy_cols(n, nc, n, B, n, c->R, c->st);
    }
    dots(c, n, nc, c->R, c->R, rr);
    std::vector<double> hb(nc), hr(nc);
    CHK(read_scal(c, bb, nc, hb.data()));
    CHK(read_scal(c, rr, nc, hr.data()));
    std::vector<int> act(nc);
    std::vector<double> hthr(nc);
    int nact = 0;
    for (int i = 0; i < nc; ++i) {
        if (!std::isfinite(hb[i]) || !std::isfinite(hr[i]))
            return fail(c, MLB_EINVAL, "non-finite right-hand side or initial guess");
        act[i] = hr[i] > tol * tol * hb[i] ? 1 : 0;
        hthr[i] = tol * tol * hb[i];
        nact += act[i];
    }
    // the convergence test runs on the device after every iteration; the
    // host reads the flags every check_every iterations (iterations past a
    // column's convergence leave it unchanged: alpha = 0)
    HIPC(hipMemcpyAsync(active, act.data(), sizeof(int) * nc, hipMemcpyHostToDevice, c->st));
    HIPC(hipMemcpyAsync(thr, hthr.data(), sizeof(double) * nc, hipMemcpyHostToDevice, c->st));
    HIPC(hipMemsetAsync(flags, 0, sizeof(int) * nc, c->st));
    HIPC(hipMemsetAsync(dits, 0, sizeof(int) * nc, c->st));
    CHK(sync(c));   // act and hthr are host locals
    int it = 0;
    int status = MLB_OK;
    if (nact > 0) {
        CHK(precondition(c, 1, nc, c->R, c->Zb));
        dots(c, n, nc, c->R, c->Zb, rz);
        launch_copy_cols(n, nc, n, c->Zb, n, c->Pb, c->st);
        const int every = std::max(1, c->o.check_every);
        for (it = 1; it <= max_it; ++it) {
            apply_K<double>(c, 1, nc, c->Pb, c->Qb, kModeY, nullptr, c->part);
            launch_sum_parts(nc, npa, c->part, pq, c->st);
            launch_cg_alpha(nc, rz, pq, active, alpha, flags, c->st);
            launch_cg_update_xr(n, nc, n, alpha, c->Pb, c->Qb, X, c->R, np, c->part, c->st);
            launch_sum_parts(nc, np, c->part, rr, c->st);
            launch_cg_check(nc, rr, thr, active, dits, flags, c->st);
            if (it % every == 0 || it == max_it) {
                CHK(read_scal(c, rr, nc, hr.data()));
                int fl[3 * kScal];
                HIPC(hipMemcpyAsync(fl, c->iscal, sizeof(int) * 3 * kScal, hipMemcpyDeviceToHost, c->st));
                CHK(sync(c));
                nact = 0;
                for (int i = 0; i < nc; ++i) {
                    if (fl[kScal + i] & 1) return fail(c, MLB_EBREAKDOWN, "CG breakdown: p^T K p <= 0 or non-finite");
                    if (fl[kScal + i] & 2) return fail(c, MLB_EBREAKDOWN, "CG residual not finite");
                    nact += fl[i] ? 1 : 0;
                }
                if (std::getenv("MLB_VERBOSE") && (it % 10 == 0 || nact == 0)) {
                    double w = 0.0;
                    for (int i = 0; i < nc; ++i) w = std::max(w, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
                    std::fprintf(stderr, "[mlb] pcg it %d worst rel %.3e active %d\n", it, w, nact);
                }
                if (nact == 0) {
                    // the iteration count: the largest over the columns
                    int mx = 0;
                    for (int i = 0; i < nc; ++i) mx = std::max(mx, fl[2 * kScal + i]);
                    it = mx;
                    break;
                }
            }
            if (flex) dots(c, n, nc, c->R, c->Zb, sc(c, 8));   // r_{k+1} . z_k for the flexible beta
            CHK(precondition(c, 1, nc, c->R, c->Zb));
            dots(c, n, nc, c->R, c->Zb, rzn);
            if (flex) launch_cg_beta_flex(nc, rzn, sc(c, 8), rz, active, beta, c->st);
            else launch_cg_beta(nc, rzn, rz, active, beta, c->st);
            launch_cg_update_p(n, nc, n, beta, c->Zb, c->Pb, c->st);
        }
        if (it > max_it) {
            it = max_it;
            status = MLB_ENOTCONV;
        }
    }
    // true residual
    apply_K<double>(c, 1, nc, X, c->R, kModeResidual, B, nullptr);
    dots(c, n, nc, c->R, c->R, rr);
    CHK(read_scal(c, rr, nc, hr.data()));
    double worst = 0.0;
    for (int i = 0; i < nc; ++i) {
        const double rel = hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0;
        worst = std::max(worst, rel);
    }
    if (info) {
        info->iterations = it;
        info->converged = status == MLB_OK;
        info->rel_residual = worst;
        info->true_rel_residual = worst;
        info->seconds = now_s() - t0;
    }
    if (status != MLB_OK) return fail(c, status, "CG did not reach the tolerance in " + std::to_string(max_it) + " iterations");
    return MLB_OK;
}

}  // namespace


namespace {

// ---- hierarchy setup (per density)

// rho(D^-1 A_j) by 12 power iterations kept on the device (one host read),
// then omega_j = jacobi_omega / (1.05 rho).
int estimate_omega(mlb_ctx* c, int j) {
    Level& l = c->lv[j - 1];
    double* v = l.vz;
    double* w = l.vz2;
    double* nrm = sc(c, 9);
    double* inv = sc(c, 10);
    launch_random_fill(l.n, 1, l.n, 0x5eedull + (uint64_t)j, l.nmask, c->dim, v, c->st);
    dots(c, l.n, 1, v, v, nrm);
    launch_rsqrt(1, nrm, inv, c->st);
    launch_scale_cols(l.n, 1, l.n, inv, v, c->st);
    for (int it = 0; it < 12; ++it) {
        apply_K<double>(c, j, 1, v, w, kModeY, nullptr, nullptr);
        launch_jacobi0<double>(l.n, 1, l.n, l.dinv, 1.0, w, w, c->st);   // w = D^-1 A v
        dots(c, l.n, 1, w, w, nrm);
        launch_rsqrt(1, nrm, inv, c->st);
        launch_scale_cols(l.n, 1, l.n, inv, w, c->st);
        std::swap(v, w);
    }
    double h;
    CHK(read_scal(c, nrm, 1, &h));
    const double rho = std::sqrt(std::max(h, 0.0));
    if (!(rho > 0.0) || !std::isfinite(rho)) return fail(c, MLB_EINVAL, "Jacobi spectral radius estimate failed");
    l.omega = c->o.jacobi_omega / (1.05 * rho);
    return MLB_OK;
}

int build_hierarchy(mlb_ctx* c) {
    drop_graphs(c);
    const int dim = c->dim;
    Level& l1 = c->lv[0];
    launch_dinv_fine(dim, l1.g, c->Ek, l1.nmask, c->dK0, l1.dinv, l1.dinvf, c->st);
    for (int j = 2; j <= c->L; ++j) {
        Level& lf = c->lv[j - 2];
        Level& lc = c->lv[j - 1];
        if (j == 2) launch_galerkin_from_E(dim, lf.g, lc.g, c->Ek, c->dMc, lc.Ke, c->st);
        else launch_galerkin_dense(dim, false, lf.g, lc.g, lf.Ke, c->dT, lc.Ke, c->st);
        launch_assemble_nb(dim, lc.g, lc.Ke, lc.nmask, lc.A, lc.Af, lc.dinv, lc.dinvf, true, c->st);
    }
    for (int j = 1; j < c->L; ++j) CHK(estimate_omega(c, j));
    if (c->L == 1) {
        c->lv[0].omega = 1.0;
    } else {
        Level& lL = c->lv[c->L - 1];
        const int64_t nL = lL.n;
        const int64_t N = c->nA;
        HIPC(hipMemsetAsync(c->Ainv, 0, sizeof(double) * N * N, c->st));
        launch_assemble_dense(dim, lL.g, lL.Ke, lL.nmask, nL, N, c->Ainv, c->st);
        launch_pad_identity(nL, N, c->Ainv, c->st);
        if (!c->aux) {
            HIPC(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
            HIPC(hipEventCreateWithFlags(&c->aux_ev[0], hipEventDisableTiming));
            HIPC(hipEventCreateWithFlags(&c->aux_ev[1], hipEventDisableTiming));
        }
        launch_block_inverse(N, c->Ainv, c->gjP, c->gjR, c->gjC, c->st, c->aux, c->aux_ev[0], c->aux_ev[1]);
        launch_pack_lower(N, c->Ainv, c->Apk, c->st);
    }
    CHK(sync(c));
    return MLB_OK;
}

// ---- coarse eigensolver: LOBPCG for the largest mu of (-G) psi = mu K psi
// at level ell; X K-orthonormal on exit (columns eS[0..nb)).

// Enqueues a host -> device copy of a small coefficient matrix without
// waiting for it; the staging buffer is only rewritten after a sync.
int upload_cm(mlb_ctx* c, double* dev, const std::vector<double>& cm) {
    if (cm.size() > (size_t)96 * 96) return fail(c, MLB_EINVAL, "coefficient matrix larger than 96 x 96");
    if (c->up_pending) CHK(sync(c));
    std::memcpy(c->hup, cm.data(), sizeof(double) * cm.size());
    HIPC(hipMemcpyAsync(dev, c->hup, sizeof(double) * cm.size(), hipMemcpyHostToDevice, c->st));
    c->up_pending = true;
    return MLB_OK;
}

// Two coefficient matrices in one upload (both land in consecutive device
// memory starting at dev; the second at dev + a.size()).
int upload_cm2(mlb_ctx* c, double* dev, const std::vector<double>& a, const std::vector<double>& b) {
    if (a.size() + b.size() > (size_t)2 * 96 * 96) return fail(c, MLB_EINVAL, "coefficient matrices too large");
    if (c->up_pending) CHK(sync(c));
    std::memcpy(c->hup, a.data(), sizeof(double) * a.size());
    std::memcpy(c->hup + a.size(), b.data(), sizeof(double) * b.size());
    HIPC(hipMemcpyAsync(dev, c->hup, sizeof(double) * (a.size() + b.size()), hipMemcpyHostToDevice, c->st));
    c->up_pending = true;
    return MLB_OK;
}

// Rayleigh-Ritz on span(S) from its Gram matrices GK = S^T K S and
// GA = S^T A S (column-major, leading dimension ld, leading ncol x ncol
// block used): scale to unit diagonal, K-orthonormalise through the
// eigendecomposition of GK (directions with eigenvalue below 1e-12 of the
// largest are dropped as linearly dependent), solve the projected symmetric
// problem and return the top nb Ritz values and coefficients C (column-major
// ncol x nb) so that S C is K-orthonormal.
bool rayleigh_ritz_gram(int ncol, int ld, const std::vector<double>& GK, const std::vector<double>& GA, int nb,
                        std::vector<double>& ev, std::vector<double>& C) {
    std::vector<double> d(ncol);
    for (int i = 0; i < ncol; ++i) {
        const double g = GK[i + (size_t)ld * i];
        d[i] = g > 0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    std::vector<double> Ks((size_t)ncol * ncol), As((size_t)ncol * ncol);
    for (int a = 0; a < ncol; ++a)
        for (int q = 0; q < ncol; ++q) {
            Ks[(size_t)a * ncol + q] = d[a] * d[q] * 0.5 * (GK[a + (size_t)ld * q] + GK[q + (size_t)ld * a]);
            As[(size_t)a * ncol + q] = d[a] * d[q] * 0.5 * (GA[a + (size_t)ld * q] + GA[q + (size_t)ld * a]);
        }
    // Fast path: a well-conditioned basis (Cholesky pivots of the unit-diagonal
    // Gram matrix all above 1e-5) is K-orthonormalised by its Cholesky factor,
    // Ks = L L^T; the projected matrix is L^-1 As L^-T and C = diag(d) L^-T Y.
    {
        std::vector<double> L(Ks);
        bool good = cholesky(ncol, L.data());
        for (int i = 0; good && i < ncol; ++i) good = L[(size_t)i * ncol + i] > 1e-5;
        if (good) {
            // Y1 = L^-1 As (forward substitution, column by column)
            std::vector<double> Y1((size_t)ncol * ncol), Ar((size_t)ncol * ncol);
            for (int col = 0; col < ncol; ++col)
                for (int i = 0; i < ncol; ++i) {
                    double v = As[(size_t)i * ncol + col];
                    for (int q = 0; q < i; ++q) v -= L[(size_t)i * ncol + q] * Y1[(size_t)q * ncol + col];
                    Y1[(size_t)i * ncol + col] = v / L[(size_t)i * ncol + i];
                }
            // Ar = Y1 L^-T = (L^-1 Y1^T)^T ; Ar is symmetric
            for (int row = 0; row < ncol; ++row)
                for (int i = 0; i < ncol; ++i) {
                    double v = Y1[(size_t)row * ncol + i];
                    for (int q = 0; q < i; ++q) v -= L[(size_t)i * ncol + q] * Ar[(size_t)row * ncol + q];
                    Ar[(size_t)row * ncol + i] = v / L[(size_t)i * ncol + i];
                }
            for (int a = 0; a < ncol; ++a)
                for (int q = 0; q < a; ++q) {
                    const double v = 0.5 * (Ar[(size_t)a * ncol + q] + Ar[(size_t)q * ncol + a]);
                    Ar[(size_t)a * ncol + q] = Ar[(size_t)q * ncol + a] = v;
                }
            std::vector<double> ew(ncol), Y((size_t)ncol * ncol);
            if (sym_eig(ncol, Ar.data(), ew.data(), Y.data())) {
                ev.assign(ew.begin(), ew.begin() + nb);
                C.assign((size_t)ncol * nb, 0.0);
                // Z = L^-T Y (back substitution), C = diag(d) Z
                for (int qc = 0; qc < nb; ++qc)
                    for (int i = ncol - 1; i >= 0; --i) {
                        double v = Y[(size_t)i * ncol + qc];
                        for (int a = i + 1; a < ncol; ++a) v -= L[(size_t)a * ncol + i] * C[a + (size_t)ncol * qc];
                        C[i + (size_t)ncol * qc] = v / L[(size_t)i * ncol + i];
                    }
                for (int qc = 0; qc < nb; ++qc)
                    for (int a = 0; a < ncol; ++a) C[a + (size_t)ncol * qc] *= d[a];
                return true;
            }
        }
    }
    std::vector<double> w(ncol), V((size_t)ncol * ncol);
    if (!sym_eig(ncol, Ks.data(), w.data(), V.data())) return false;
    if (!(w[0] > 0)) return false;
    int r = 0;
    while (r < ncol && w[r] > 1e-12 * w[0]) ++r;
    if (r < nb) return false;
    // Bm = V_r diag(w_r^-1/2) (ncol x r); Ar = Bm^T As Bm
    std::vector<double> Bm((size_t)ncol * r), T((size_t)ncol * r), Ar((size_t)r * r);
    for (int a = 0; a < ncol; ++a)
        for (int j = 0; j < r; ++j) Bm[(size_t)a * r + j] = V[(size_t)a * ncol + j] / std::sqrt(w[j]);
    for (int a = 0; a < ncol; ++a)
        for (int j = 0; j < r; ++j) {
            double sacc = 0.0;
            for (int b = 0; b < ncol; ++b) sacc += As[(size_t)a * ncol + b] * Bm[(size_t)b * r + j];
            T[(size_t)a * r + j] = sacc;
        }
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
            double sacc = 0.0;
            for (int a = 0; a < ncol; ++a) sacc += Bm[(size_t)a * r + i] * T[(size_t)a * r + j];
            Ar[(size_t)i * r + j] = sacc;
        }
    std::vector<double> ew(r), Y((size_t)r * r);
    if (!sym_eig(r, Ar.data(), ew.data(), Y.data())) return false;
    ev.assign(ew.begin(), ew.begin() + nb);
    C.assign((size_t)ncol * nb, 0.0);
    for (int a = 0; a < ncol; ++a)
        for (int q = 0; q < nb; ++q) {
            double sacc = 0.0;
            for (int j = 0; j < r; ++j) sacc += Bm[(size_t)a * r + j] * Y[(size_t)j * r + q];
            C[a + (size_t)ncol * q] = d[a] * sacc;
        }
    return true;
}

// SVQB: given the Gram matrix G (r0 x r0, column-major) of a block V,
// returns T (column-major r0 x r) with V T orthonormal in that inner product,
// dropping directions whose Gram eigenvalue is below drop * largest, and
// r >= 1.  Returns 0 if the block is exactly zero (nothing left to add) and
// -1 if G is not a Gram matrix of finite vectors: a non-finite entry, a
// negative diagonal or largest eigenvalue, or an eigensolver failure.
static int svqb(int r0, const std::vector<double>& G, double drop, std::vector<double>& T) {
    std::vector<double> d(r0), Gs((size_t)r0 * r0), w(r0), V((size_t)r0 * r0);
    for (size_t i = 0; i < (size_t)r0 * r0; ++i)
        if (!std::isfinite(G[i])) return -1;
    for (int i = 0; i < r0; ++i) {
        const double g = G[i + (size_t)r0 * i];
        if (g < 0) return -1;
        d[i] = g > 0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    for (int a = 0; a < r0; ++a)
        for (int q = 0; q < r0; ++q)
            Gs[(size_t)a * r0 + q] = d[a] * d[q] * 0.5 * (G[a + (size_t)r0 * q] + G[q + (size_t)r0 * a]);
    if (!sym_eig(r0, Gs.data(), w.data(), V.data()) || w[0] < 0) return -1;
    if (!(w[0] > 0)) return 0;
    int r = 0;
    while (r < r0 && w[r] > drop * w[0]) ++r;
    T.assign((size_t)r0 * r, 0.0);
    for (int a = 0; a < r0; ++a)
        for (int j = 0; j < r; ++j) T[a + (size_t)r0 * j] = d[a] * V[(size_t)a * r0 + j] / std::sqrt(w[j]);
    return r;
}

// out (sp x nc) = sign T C for T (sp x r) and C (r x nc), column-major.
void fold_t(int sp, int r, int nc, const std::vector<double>& T, const std::vector<double>& Cr, double sign,
            std::vector<double>& out) {
    out.assign((size_t)sp * nc, 0.0);
    for (int q = 0; q < nc; ++q)
        for (int i = 0; i < sp; ++i) {
            double a = 0.0;
            for (int j = 0; j < r; ++j) a += T[i + (size_t)sp * j] * Cr[j + (size_t)r * q];
            out[i + (size_t)sp * q] = sign * a;
        }
}

// ---- Block PCG (O'Leary's block conjugate gradients, in the breakdown-free
// form of Ji & Li: the search block is A-orthonormalised by SVQB every
// iteration, so converged or linearly dependent directions drop out).
// Per iteration, with Q = A P:
//   [P^T Q, P^T R]     one Gram pass over P, Q, R
//   T = svqb(P^T Q),  alpha = T^T P^T R                      (host, tiny)
//   X += P (T alpha), R -= Q (T alpha), |R|^2                one fused pass
//   Z = M R,  beta = -T^T Q^T Z,  P <- Z + P (T beta),  Q = A P
// (the orthonormal block P T and its image Q T are never formed: T is
// folded into the coefficients, so P and Q are only read by the updates)
// All columns share one block Krylov space, which deflates the outlying
// eigenvalues of M A for every right-hand side at once.
int bpcg(mlb_ctx* c, const double* B, double* X, int nc, double tol, int max_it, bool use_x0, mlb_solve_info* info) {
    const double t0 = now_s();
    const int64_t n = c->n;
    if (nc > 32) return fail(c, MLB_EINVAL, "block CG supports at most 32 columns");
    CHK(ensure_cg(c, nc));
    const int np = std::max(reduction_parts(n), bcg_step_parts(n));
    CHK(ensure_part(c, (int64_t)np * nc));
    double* bb = sc(c, 0);
    double* rr = sc(c, 1);
    dots(c, n, nc, B, B, bb);
    if (use_x0) {
        apply_K<double>(c, 1, nc, X, c->R, kModeResidual, B, nullptr);
    } else {
        HIPC(hipMemsetAsync(X, 0, sizeof(double) * n * nc, c->st));
        launch_copy_cols(n, nc, n, B, n, c->R, c->st);
    }
    std::vector<double> hb(nc), hr(nc);
    CHK(read_scal(c, bb, nc, hb.data()));
    for (int i = 0; i < nc; ++i)
        if (!std::isfinite(hb[i])) return fail(c, MLB_EINVAL, "non-finite right-hand side");
    double* P = c->Pb;    // n x sp
    double* Q = c->Qb;    // A P
    double* Z = c->Zb;
    int sp = nc;
    int it = 0, status = MLB_OK;
    auto check = [&](bool* done) -> int {
        CHK(read_scal(c, rr, nc, hr.data()));
        bool all = true;
        double w = 0;
        for (int i = 0; i < nc; ++i) {
            if (!std::isfinite(hr[i])) return fail(c, MLB_EBREAKDOWN, "block CG residual not finite");
            if (hr[i] > tol * tol * hb[i]) all = false;
            w = std::max(w, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
        }
        if (std::getenv("MLB_VERBOSE") && (it % 10 == 0 || all))
            std::fprintf(stderr, "[mlb] bpcg it %d worst rel %.3e rank %d\n", it, w, sp);
        *done = all;
        return MLB_OK;
    };
    bool done = false;
    dots(c, n, nc, c->R, c->R, rr);
    CHK(check(&done));
    std::vector<double> G, Tm, Al, Cm;
    if (!done) {
        CHK(precondition(c, 1, nc, c->R, P));
        apply_K<double>(c, 1, nc, P, Q, kModeY, nullptr, nullptr);
        for (it = 1; it <= max_it; ++it) {
            // [P^T Q | P^T R]
            CHK(gram(c, n, sp, P, n, sp, Q, n, G, nc, c->R, n));
            std::vector<double> PQ(G.begin(), G.begin() + (size_t)sp * sp);
            const int r = svqb(sp, PQ, 1e-13, Tm);
            if (r < 0) return fail(c, MLB_EBREAKDOWN, "block CG: P^T K P is not a finite Gram matrix");
            if (r == 0) return fail(c, MLB_EBREAKDOWN, "block CG: search space collapsed");
            // The K-orthonormal search block is P T (r columns); it is never
            // formed: its coefficients are folded into the small matrices.
            // alpha = T^T (P^T R) (r x nc); X += P (T alpha), R -= Q (T alpha)
            Al.assign((size_t)r * nc, 0.0);
            for (int j = 0; j < r; ++j)
                for (int q = 0; q < nc; ++q) {
                    double a = 0.0;
                    for (int i = 0; i < sp; ++i) a += Tm[i + (size_t)sp * j] * G[(size_t)sp * sp + i + (size_t)sp * q];
                    Al[j + (size_t)r * q] = a;
                }
            fold_t(sp, r, nc, Tm, Al, 1.0, Cm);
            CHK(upload_cm(c, c->cbuf, Cm));
            const int nps = bcg_step_parts(n);
            launch_bcg_step(n, sp, nc, c->cbuf, P, Q, X, c->R, c->part, c->st);
            launch_sum_parts(nc, nps, c->part, rr, c->st);
            CHK(check(&done));
            if (done) break;
            // Z = M R; beta = -(Q T)^T Z (r x nc); P <- Z + P (T beta); Q = A P.
            // In mixed precision Z stays in the cycle's FP32 block (read as
            // doubles, exactly: no conversion pass).
            const float* Zf = nullptr;
            if (c->d.precision == MLB_MIXED) {
                CHK(precondition(c, 1, nc, c->R, nullptr));
                Zf = c->lv[0].fz;
                CHK(gram_f32b(c, n, sp, Q, nc, Zf, G));
            } else {
                CHK(precondition(c, 1, nc, c->R, Z));
                CHK(gram(c, n, sp, Q, n, nc, Z, n, G));
            }
            Al.assign((size_t)r * nc, 0.0);
            for (int j = 0; j < r; ++j)
                for (int q = 0; q < nc; ++q) {
                    double a = 0.0;
                    for (int i = 0; i < sp; ++i) a += Tm[i + (size_t)sp * j] * G[i + (size_t)sp * q];
                    Al[j + (size_t)r * q] = a;
                }
            fold_t(sp, r, nc, Tm, Al, -1.0, Cm);
            CHK(upload_cm(c, c->cbuf, Cm));
            if (Zf) launch_bcg_dir(n, sp, nc, c->cbuf, Zf, P, c->st);
            else launch_bcg_dir(n, sp, nc, c->cbuf, Z, P, c->st);
            sp = nc;
            apply_K<double>(c, 1, nc, P, Q, kModeY, nullptr, nullptr);
        }
        if (it > max_it) {
            it = max_it;
            status = MLB_ENOTCONV;
        }
    }
    // true residual
    apply_K<double>(c, 1, nc, X, c->R, kModeResidual, B, nullptr);
    dots(c, n, nc, c->R, c->R, rr);
    CHK(read_scal(c, rr, nc, hr.data()));
    double worst = 0.0;
    for (int i = 0; i < nc; ++i) worst = std::max(worst, hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0);
    if (info) {
        info->iterations = it;
        info->converged = status == MLB_OK;
        info->rel_residual = worst;
        info->true_rel_residual = worst;
        info->seconds = now_s() - t0;
    }
    if (status != MLB_OK) return fail(c, status, "block CG did not reach the tolerance");
    return MLB_OK;
}

// LOBPCG for the largest mu of (-G) psi = mu K psi at level ell.
// The basis S = [X P W] and its images K S, -G S live contiguously in one of
// two buffers; each iteration writes the new X and P into the other buffer.
//   R = -G X - K X diag(mu);  W = T R (multigrid preconditioner)
//   W -= [X P] ([K X, K P]^T W)  (twice);  K W, -G W;  SVQB of W^T K W
//   Rayleigh-Ritz on span(S) (rank revealing, K-orthonormal result)
//   X' = S C, P' = [P W] C_pw;  K [X' P'] and -G [X' P'] applied explicitly,
// so every Gram matrix is formed from exact operator images (updating them
// by the same recurrences drifts once the basis becomes ill-conditioned).
// On exit eS[0..nb) holds X (K-orthonormal), mu the Ritz values (descending).
int coarse_eigs(mlb_ctx* c, int k, double tol, int* iters, double* worst, double* gap, std::vector<double>& mu,
                int* warm_used, int* guard_fired) {
    const bool verbose = std::getenv("MLB_VERBOSE") != nullptr;
    const int j = c->ell;
    Level& l = c->lv[j - 1];
    const int64_t n = l.n;
    int guard = c->o.eig_guard > 0 ? c->o.eig_guard : std::max(4, k / 2);
    const int nb = std::min(k + guard, 32);
    if (nb <= k) return fail(c, MLB_EINVAL, "k must be at most 31");
    if (nb > n / 2) return fail(c, MLB_EINVAL, "eigen level too small for the requested modes");
    CHK(ensure_level_cols(c, nb));
    if (nb > c->eig_cap) {
        const size_t s3 = (size_t)n * 3 * nb, s1 = (size_t)n * nb;
        CHK(dalloc(c, &c->eS, s3));
        CHK(dalloc(c, &c->eK, s3));
        CHK(dalloc(c, &c->eA, s3));
        CHK(dalloc(c, &c->eT, s3));
        CHK(dalloc(c, &c->eTK, s3));
        CHK(dalloc(c, &c->eTA, s3));
        CHK(dalloc(c, &c->eR, s1));
        CHK(dalloc(c, &c->eP, s1));
        CHK(dalloc(c, &c->ePK, s1));
        CHK(dalloc(c, &c->ePA, s1));
        c->eig_cap = nb;
    }
    struct Buf {
        double *S, *KS, *AS;
    };
    Buf bufs[2] = {{c->eS, c->eK, c->eA}, {c->eT, c->eTK, c->eTA}};
    int cur = 0;
    auto applyKA = [&](int cols, const double* V, double* KV, double* AV) {
        apply_K<double>(c, j, cols, V, KV, kModeY, nullptr, nullptr);
        apply_G(c, j, cols, V, AV);
        launch_axpby(n * cols, -1.0, AV, 0.0, AV, c->st);
    };

    // Start block: seeded random columns, Rayleigh-Ritz on their span, the
    // Ritz block in bufs[1].  With a warm start (its columns first, random
    // guard columns after) both blocks are built and the warm one is kept
    // only if the worst initial residual of the k wanted Ritz pairs is not
    // larger than the plain block's (a rank-deficient warm block is dropped).
    std::vector<double> GK, GA, ev, C, Cpw, G, Tm, Co;
    std::vector<double> nrm(2 * nb);
    auto ritz_residual = [&](const std::vector<double>& m, double* out) -> int {
        std::memcpy(c->hpin, m.data(), sizeof(double) * nb);
        HIPC(hipMemcpyAsync(sc(c, 11), c->hpin, sizeof(double) * nb, hipMemcpyHostToDevice, c->st));
        launch_residual_block(n, nb, n, bufs[1].AS, bufs[1].KS, sc(c, 11), c->eR, c->st);
        dots(c, n, nb, c->eR, c->eR, sc(c, 12));
        dots(c, n, nb, bufs[1].KS, bufs[1].KS, sc(c, 12) + nb);
        CHK(read_scal(c, sc(c, 12), 2 * nb, nrm.data()));
        double w = 0.0;
        for (int i = 0; i < k; ++i) {
            const double den = std::fabs(m[i]) * std::sqrt(nrm[nb + i]);
            w = std::max(w, den > 0 ? std::sqrt(nrm[i]) / den : 1e300);
        }
        *out = std::isfinite(w) ? w : 1e300;
        return MLB_OK;
    };
    // build + Rayleigh-Ritz of one start block; ok = false if rank deficient
    auto start_block = [&](bool warm, bool* ok) -> int {
        double* X = bufs[0].S;
        launch_random_fill(n, nb, n, c->o.seed, l.nmask, c->dim, X, c->st);
        if (warm) {
            const int wc = std::min(c->warm_coarse_cols, nb);
            HIPC(hipMemcpyAsync(X, c->warm_coarse, sizeof(double) * n * wc, hipMemcpyDeviceToDevice, c->st));
            launch_mask_fixed(n, wc, n, l.nmask, c->dim, X, c->st);
        }
        applyKA(nb, X, bufs[0].KS, bufs[0].AS);
        CHK(gram2(c, n, nb, bufs[0].S, nb, bufs[0].KS, bufs[0].AS, GK, GA));
        *ok = rayleigh_ritz_gram(nb, nb, GK, GA, nb, ev, C);
        if (!*ok) return MLB_OK;
        CHK(upload_cm(c, c->cbuf, C));
        launch_gemm_cat(n, nb, n, bufs[0].S, 0, n, nullptr, nb, c->cbuf, 0.0, n, bufs[1].S, c->st);
        applyKA(nb, bufs[1].S, bufs[1].KS, bufs[1].AS);
        return MLB_OK;
    };
    {
        bool ok = false;
        CHK(start_block(false, &ok));
        if (!ok) return fail(c, MLB_EBREAKDOWN, "coarse eigensolver: start block is rank deficient");
        mu.assign(ev.begin(), ev.begin() + nb);
        *warm_used = 0;
        if (c->warm_coarse_cols > 0 && c->warm_coarse) {
            double w_plain = 0.0, w_warm = 0.0;
            CHK(ritz_residual(mu, &w_plain));
            // keep the plain Ritz block in the P buffers while the warm one is built
            launch_copy_cols(n, nb, n, bufs[1].S, n, c->eP, c->st);
            launch_copy_cols(n, nb, n, bufs[1].KS, n, c->ePK, c->st);
            launch_copy_cols(n, nb, n, bufs[1].AS, n, c->ePA, c->st);
            CHK(start_block(true, &ok));
            std::vector<double> mu_w;
            if (ok) {
                mu_w.assign(ev.begin(), ev.begin() + nb);
                CHK(ritz_residual(mu_w, &w_warm));
            }
            if (ok && w_warm <= w_plain) {
                mu = mu_w;
                *warm_used = 1;
            } else {
                launch_copy_cols(n, nb, n, c->eP, n, bufs[1].S, c->st);
                launch_copy_cols(n, nb, n, c->ePK, n, bufs[1].KS, c->st);
                launch_copy_cols(n, nb, n, c->ePA, n, bufs[1].AS, c->st);
            }
            if (verbose)
                std::fprintf(stderr, "[mlb] coarse start: plain %.3e warm %.3e -> %s\n", w_plain,
                             ok ? w_warm : -1.0, *warm_used ? "warm" : "plain");
        }
        cur = 1;
    }
    int rp = 0;   // columns of P
    int it = 0;
    bool stalled = false;
    std::vector<double> hist;
    double wres = 1e300;
    const int max_it = c->o.eig_max_it > 0 ? c->o.eig_max_it : 400;
    double t_host = 0.0, t_pre = 0.0;
    const double t_start = now_s();
    std::vector<double> cres(nb);
    std::vector<int> act;
    for (it = 0; it <= max_it; ++it) {
        Buf& b = bufs[cur];
        double *X = b.S, *KX = b.KS, *AX = b.AS;
        std::memcpy(c->hpin, mu.data(), sizeof(double) * nb);
        HIPC(hipMemcpyAsync(sc(c, 11), c->hpin, sizeof(double) * nb, hipMemcpyHostToDevice, c->st));
        launch_residual_block(n, nb, n, AX, KX, sc(c, 11), c->eR, c->st);
        dots(c, n, nb, c->eR, c->eR, sc(c, 12));
        dots(c, n, nb, KX, KX, sc(c, 12) + nb);
        CHK(read_scal(c, sc(c, 12), 2 * nb, nrm.data()));
        wres = 0.0;
        for (int i = 0; i < nb; ++i) {
            const double den = std::fabs(mu[i]) * std::sqrt(nrm[nb + i]);
            cres[i] = den > 0 ? std::sqrt(nrm[i]) / den : 1e300;
            if (!std::isfinite(cres[i])) cres[i] = 1e300;
            if (i < k) wres = std::max(wres, cres[i]);
        }
        if (!(wres < 1e300)) return fail(c, MLB_EBREAKDOWN, "coarse eigensolver residual not finite");
        // Soft locking: a column whose residual is already below tol keeps its
        // place in X (and in every Rayleigh-Ritz step) but adds no new
        // direction.  Its residual is then dominated by rounding, and adding
        // that noise, normalised, to the basis spoils the conditioning of the
        // Gram matrices and with it the pairs that had converged.  The active
        // set is recomputed every iteration, so a locked column whose residual
        // grows again is unlocked.
        act.clear();
        for (int i = 0; i < nb; ++i)
            if (cres[i] > tol) act.push_back(i);
        const int na = (int)act.size();
        if (verbose) std::fprintf(stderr, "[mlb] lobpcg it %d worst %.3e rp %d active %d mu0 %.12g muk %.12g\n", it,
                                  wres, rp, na, mu[0], mu[k - 1]);
        if (wres <= tol || it == max_it) break;
        // Precision floor: the residual of the k-th pair cannot fall below
        // about eps * ||K^-1 G|| / mu_k.  Accept a residual that has stopped
        // improving for 15 iterations once it (and the best of those 15) is
        // below sqrt(tol).
        hist.push_back(wres);
        if ((int)hist.size() > 15) {
            const double best_old = *std::min_element(hist.begin(), hist.end() - 15);
            const double best_new = *std::min_element(hist.end() - 15, hist.end());
            if (best_new > 0.5 * best_old && wres <= std::sqrt(tol)) {
                stalled = true;
                break;
            }
        }
        if (it >= 30 && !(mu[k - 1] > 0.0))
            return fail(c, MLB_ENOPOS, "fewer than k positive buckling factors at the coarse level");
        // compact the active residual columns (and, below, the active search
        // directions) to the front of their blocks; every move is to a lower
        // or equal column, in increasing order, so no source is overwritten
        // before it is read
        for (int a = 0; a < na; ++a)
            if (act[a] != a) launch_copy_cols(n, 1, n, c->eR + n * act[a], n, c->eR + n * a, c->st);
        if (rp > 0) {
            for (int a = 0; a < na; ++a)
                if (act[a] != a)
                    for (double* base : {b.S, b.KS, b.AS})
                        launch_copy_cols(n, 1, n, base + n * (nb + act[a]), n, base + n * (nb + a), c->st);
            rp = na;
            // K-orthonormalise the active directions against X (twice) and
            // among themselves (SVQB), updating their images by the same
            // combinations, so that [X P W] below is K-orthonormal block by
            // block and its Rayleigh-Ritz problem well conditioned
            double *P = b.S + n * nb, *KP = b.KS + n * nb, *AP = b.AS + n * nb;
            for (int pass = 0; pass < 2; ++pass) {
                // cbuf2[a, q] = -(X^T K P)[a, q], formed on the device
                CHK(gram_coeffs_dev(c, n, rp, P, n, nb, KX, n, -1.0, c->cbuf2));
                launch_gemm_cat(n, nb, n, X, 0, n, nullptr, rp, c->cbuf2, 1.0, n, P, c->st);
                launch_gemm_cat(n, nb, n, KX, 0, n, nullptr, rp, c->cbuf2, 1.0, n, KP, c->st);
                launch_gemm_cat(n, nb, n, AX, 0, n, nullptr, rp, c->cbuf2, 1.0, n, AP, c->st);
            }
            CHK(gram(c, n, rp, P, n, rp, KP, n, G));
            const int rq = svqb(rp, G, 1e-10, Tm);
            if (rq < 0) return fail(c, MLB_EBREAKDOWN, "coarse eigensolver: P^T K P is not a finite Gram matrix");
            if (rq > 0) {
                CHK(upload_cm(c, c->cbuf, Tm));
                launch_xform_inplace(n, rp, rq, c->cbuf, n, P, c->st);
                launch_xform_inplace(n, rp, rq, c->cbuf, n, KP, c->st);
                launch_xform_inplace(n, rp, rq, c->cbuf, n, AP, c->st);
            }
            rp = rq;
        }
        const int64_t oW = n * (nb + rp);
        double *W = b.S + oW, *KW = b.KS + oW, *AW = b.AS + oW;
        // W = T R
        if (verbose) {
            CHK(sync(c));
            t_pre -= now_s();
        }
        // (eig_sweeps stationary multigrid iterations from zero: a symmetric
        // preconditioner that approximates (K^l)^-1 better than one cycle)
        CHK(precondition(c, j, na, c->eR, W));
        for (int sw = 1; sw < c->o.eig_sweeps; ++sw) {   // W += B (R - K W)
            apply_K<double>(c, j, na, W, c->eP, kModeResidual, c->eR, nullptr);
            CHK(precondition(c, j, na, c->eP, c->ePK));
            launch_axpby(n * na, 1.0, c->ePK, 1.0, W, c->st);
        }
        if (verbose) {
            CHK(sync(c));
            t_pre += now_s();
        }
        // W -= [X P] ([K X, K P]^T W), twice
        const int nx = nb + rp;
        for (int pass = 0; pass < 2; ++pass) {
            // cbuf2[a, q] = ([K X, K P]^T W)[a, q], formed on the device
            CHK(gram_coeffs_dev(c, n, na, W, n, nx, KX, n, 1.0, c->cbuf2));
            launch_gemm_cat(n, nx, n, X, 0, n, nullptr, na, c->cbuf2, 0.0, n, c->eR, c->st);
            launch_axpby(n * na, -1.0, c->eR, 1.0, W, c->st);
        }
        applyKA(na, W, KW, AW);
        CHK(gram(c, n, na, W, n, na, KW, n, G));
        const int rw = svqb(na, G, 1e-10, Tm);
        if (rw < 0) return fail(c, MLB_EBREAKDOWN, "coarse eigensolver: W^T K W is not a finite Gram matrix");
        if (rw == 0) {   // the preconditioned residual vanished: nothing new to add
            stalled = true;
            break;
        }
        CHK(upload_cm(c, c->cbuf, Tm));
        launch_xform_inplace(n, na, rw, c->cbuf, n, W, c->st);
        launch_xform_inplace(n, na, rw, c->cbuf, n, KW, c->st);
        launch_xform_inplace(n, na, rw, c->cbuf, n, AW, c->st);
        int ncol = nx + rw;
        int np_ = rp;   // P columns inside the Ritz basis
        CHK(gram2(c, n, ncol, b.S, ncol, b.KS, b.AS, GK, GA));
        const double th0 = now_s();
        const bool rr_ok = rayleigh_ritz_gram(ncol, ncol, GK, GA, nb, ev, C);
        t_host += now_s() - th0;
        if (!rr_ok) {
            bool ok = false;
            if (rp > 0) {   // retry on [X W]: move W down over P
                for (int a = 0; a < 3; ++a) {
                    double* base = a == 0 ? b.S : a == 1 ? b.KS : b.AS;
                    launch_copy_cols(n, rw, n, base + oW, n, base + n * nb, c->st);
                }
                ncol = nb + rw;
                np_ = 0;
                CHK(gram2(c, n, ncol, b.S, ncol, b.KS, b.AS, GK, GA));
                ok = rayleigh_ritz_gram(ncol, ncol, GK, GA, nb, ev, C);
                if (verbose) std::fprintf(stderr, "[mlb] lobpcg it %d: dropped P\n", it);
            }
            if (!ok) return fail(c, MLB_EBREAKDOWN, "coarse eigensolver: search space collapsed");
        }
        (void)np_;
        // X' = S C, P' = S[nb:ncol] C[nb:ncol, :] into the other buffer
        Cpw.assign((size_t)(ncol - nb) * nb, 0.0);
        for (int a = nb; a < ncol; ++a)
            for (int q = 0; q < nb; ++q) Cpw[(a - nb) + (size_t)(ncol - nb) * q] = C[a + (size_t)ncol * q];
        CHK(upload_cm2(c, c->cbuf, C, Cpw));
        Buf& nbf = bufs[cur ^ 1];
        launch_gemm_cat(n, ncol, n, b.S, 0, n, nullptr, nb, c->cbuf, 0.0, n, nbf.S, c->st);
        launch_gemm_cat(n, ncol - nb, n, b.S + n * nb, 0, n, nullptr, nb, c->cbuf + C.size(), 0.0, n,
                        nbf.S + n * nb, c->st);
        applyKA(2 * nb, nbf.S, nbf.KS, nbf.AS);
        rp = nb;
        cur ^= 1;
        mu.assign(ev.begin(), ev.begin() + nb);
    }
    if (cur == 1) launch_copy_cols(n, nb, n, bufs[1].S, n, c->eS, c->st);
    if (verbose)
        std::fprintf(stderr, "[mlb] lobpcg %d its: total %.3f s, preconditioner %.3f s, host Rayleigh-Ritz %.3f s\n", it,
                     now_s() - t_start, t_pre, t_host);
    *iters = it;
    *worst = wres;
    *gap = mu[k - 1] > 0 ? (mu[k - 1] - mu[k]) / mu[k - 1] : 0.0;
    *guard_fired = wres > tol ? 1 : 0;
    // A stalled residual is accepted only below sqrt(tol); the caller
    // reports it (mlb_eig_info.coarse_guard_fired, coarse_residual).
    if (wres > tol && !(stalled && wres <= std::sqrt(tol)))
        return fail(c, MLB_ENOTCONV, "coarse eigensolver stalled at relative residual " + std::to_string(wres) +
                                         " after " + std::to_string(it) + " iterations");
    if (!(mu[k - 1] > 0.0)) return fail(c, MLB_ENOPOS, "fewer than k positive buckling factors at the coarse level");
    return MLB_OK;
}

// G element matrices at the eigen level from the reference stresses.
// Galerkin G^j = P^T G^{j-1} P for j = 2 .. ell (scalar element matrices,
// since G_e = g_e kron I), then the masked block-diagonal stencil at ell.
int build_G_levels(mlb_ctx* c) {
    if (c->ell == 1) return MLB_OK;
    const int dim = c->dim;
    for (int j = 2; j <= c->ell; ++j) {
        Level& lf = c->lv[j - 2];
        Level& lc = c->lv[j - 1];
        if (j == 2) launch_galerkin_G_from_S(dim, lf.g, lc.g, c->S, c->dGHc, lc.Ge, c->st);
        else launch_galerkin_dense(dim, true, lf.g, lc.g, lf.Ge, c->dT, lc.Ge, c->st);
    }
    Level& le = c->lv[c->ell - 1];
    launch_assemble_nb_diag(dim, le.g, le.Ge, le.nmask, le.Gs, c->st);
    // the intermediate-level refinement also needs G^j on levels 2 .. ell-1
    if (c->o.refine_sweeps > 0)
        for (int j = 2; j < c->ell; ++j) {
            Level& l = c->lv[j - 1];
            if (!l.Gs) CHK(dalloc(c, &l.Gs, (size_t)stencil_entries(dim, l.g, true)));
            launch_assemble_nb_diag(dim, l.g, l.Ge, l.nmask, l.Gs, c->st);
        }
    HIPC(hipGetLastError());
    return MLB_OK;
}

int do_buckling(mlb_ctx* c, int ref_case, int k, double tol_eig, mlb_eig_info* info) {
    if (!c->has_static) return fail(c, MLB_ESTATE, "mlb_buckling needs a converged static solve first");
    if (ref_case < 0 || ref_case >= c->ncases) return fail(c, MLB_EINVAL, "ref_case out of range");
    if (k < 1) return fail(c, MLB_EINVAL, "k must be positive");
    if (!(tol_eig > 0)) tol_eig = 1e-10;
    const double t0 = now_s();
    const int64_t n = c->n;
    c->has_buck = false;
    c->has_adj = false;
    launch_stress(c->dim, c->lv[0].g, c->Es, c->U + (int64_t)ref_case * n, c->dD0Bc, c->S, c->st);
    c->has_stress = true;
    c->ref_case_used = ref_case;
    CHK(build_G_levels(c));
    int cit = 0;
    double cres = 0, gap = 0;
    std::vector<double> mu;
    int warm_used = 0, guard = 0;
    CHK(coarse_eigs(c, k, tol_eig, &cit, &cres, &gap, mu, &warm_used, &guard));
    const double t1 = now_s();
    // step 2: interpolate the coarse modes to the fine grid
    CHK(ensure_cg(c, std::max(k, c->ncases)));
    if ((int)c->k != k) {
        CHK(dalloc(c, &c->Phi, (size_t)n * k));
        CHK(dalloc(c, &c->Zadj, (size_t)n * k));
        CHK(dalloc(c, &c->dlam_l, (size_t)k));
        CHK(dalloc(c, &c->Psif, (size_t)n * k));
        dfree(c->cW);
        c->k = k;
    }
    c->psi_ok = false;
    // Optionally (Alg. 2, intermediate levels): on every level ell-1 .. 2
    // smooth the prolonged modes by Kaczmarz sweeps on (K^j + sigma G^j) psi
    // = 0, sigma the smallest Ritz value of the coarser level, and replace
    // them by their level-j Ritz vectors.
    const int sweeps = c->o.refine_sweeps;
    int nref = 0;
    double lam1_ref[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double t_refine = 0.0;
    double sigma = mu.empty() ? 0.0 : 1.0 / mu[0];
    if (sweeps > 0) CHK(ensure_level_cols(c, k));
    const double* cur = c->eS;
    int64_t ldc = c->lv[c->ell - 1].n;
    for (int j = c->ell - 1; j >= 1; --j) {
        Level& lf = c->lv[j - 1];
        Level& lc = c->lv[j];
        double* dst = j == 1 ? c->X1 : lf.vt;
        launch_prolong_nb<double>(c->dim, lf.g, lc.g, lf.nmask, lc.nmask, k, lf.n, ldc, cur, dst, false, c->st);
        cur = dst;
        ldc = lf.n;
        if (sweeps > 0 && j >= 2) {
            const double ts = now_s();
            for (int sw = 0; sw < sweeps; ++sw)
                launch_kaczmarz_sweep(c->dim, lf.g, lf.A, lf.Gs, sigma, lf.nmask, k, lf.n, dst, c->st);
            apply_K<double>(c, j, k, dst, lf.vr, kModeY, nullptr, nullptr);
            apply_G(c, j, k, dst, lf.vz);
            std::vector<double> A, B;
            CHK(gram2(c, lf.n, k, dst, k, lf.vr, lf.vz, A, B));
            std::vector<double> A2(k * k), B2(k * k), ev(k), Y(k * k);
            for (int a = 0; a < k; ++a)
                for (int q = 0; q < k; ++q) {
                    A2[a * k + q] = 0.5 * (A[a + k * q] + A[q + k * a]);
                    B2[a * k + q] = -0.5 * (B[a + k * q] + B[q + k * a]);
                }
            if (!gen_eig(k, A2.data(), B2.data(), ev.data(), Y.data()))
                return fail(c, MLB_EBREAKDOWN, "level Rayleigh-Ritz: Psi^T K^j Psi not positive definite");
            if (!(ev[k - 1] > 0.0)) return fail(c, MLB_ENOPOS, "fewer than k positive Ritz values on a refined level");
            std::vector<double> C(k * k);
            for (int a = 0; a < k; ++a)
                for (int q = 0; q < k; ++q) C[a + k * q] = Y[a * k + q];
            CHK(upload_cm(c, c->cbuf, C));
            launch_gemm_small(lf.n, k, lf.n, dst, k, c->cbuf, lf.n, lf.vz2, c->st);
            cur = lf.vz2;
            sigma = 1.0 / ev[0];
            if (nref < 8) lam1_ref[nref] = sigma;
            ++nref;
            CHK(sync(c));
            t_refine += now_s() - ts;
        }
    }
    // Optionally the loop also visits the fine grid (it is printed down to
    // it): the same sweeps on (K + sigma G) psi = 0 with assembled fine
    // stencils, then a fine Ritz step, before the block solve.
    if (sweeps > 0 && c->o.refine_fine && c->ell > 1) {
        const double ts = now_s();
        Level& l1 = c->lv[0];
        const int dim = c->dim;
        const int nn = 1 << dim, nde = dim << dim;
        if (!c->fineA) {
            CHK(dalloc(c, &c->fineA, (size_t)stencil_entries(dim, l1.g, false)));
            CHK(dalloc(c, &c->fineAf, (size_t)stencil_entries(dim, l1.g, false, true)));
            CHK(dalloc(c, &c->fineGs, (size_t)stencil_entries(dim, l1.g, true)));
            CHK(dalloc(c, &c->fineDinv, (size_t)n));
            CHK(dalloc(c, &c->fineDinvf, (size_t)n));
        }
        double *Ke = nullptr, *Ge = nullptr;
        CHK(dalloc(c, &Ke, (size_t)l1.g.m * nde * nde));
        const int rge = dalloc(c, &Ge, (size_t)l1.g.m * nn * nn);
        if (rge != MLB_OK) {
            dfree(Ke);
            return rge;
        }
        launch_fine_elem_mats(dim, l1.g, c->Ek, c->dK0, c->S, c->dHk, Ke, Ge, c->st);
        launch_assemble_nb(dim, l1.g, Ke, l1.nmask, c->fineA, c->fineAf, c->fineDinv, c->fineDinvf, true, c->st);
        launch_assemble_nb_diag(dim, l1.g, Ge, l1.nmask, c->fineGs, c->st);
        const hipError_t es = hipStreamSynchronize(c->st);
        dfree(Ke);
        dfree(Ge);
        HIPC(es);
        for (int sw = 0; sw < sweeps; ++sw)
            launch_kaczmarz_sweep(dim, l1.g, c->fineA, c->fineGs, sigma, l1.nmask, k, n, c->X1, c->st);
        apply_K<double>(c, 1, k, c->X1, c->Phi, kModeY, nullptr, nullptr);
        apply_G(c, 1, k, c->X1, c->X2);
        std::vector<double> A, B;
        CHK(gram2(c, n, k, c->X1, k, c->Phi, c->X2, A, B));
        std::vector<double> A2(k * k), B2(k * k), ev(k), Y(k * k);
        for (int a = 0; a < k; ++a)
            for (int q = 0; q < k; ++q) {
                A2[a * k + q] = 0.5 * (A[a + k * q] + A[q + k * a]);
                B2[a * k + q] = -0.5 * (B[a + k * q] + B[q + k * a]);
            }
        if (!gen_eig(k, A2.data(), B2.data(), ev.data(), Y.data()))
            return fail(c, MLB_EBREAKDOWN, "fine Rayleigh-Ritz: Psi^T K Psi not positive definite");
        if (!(ev[k - 1] > 0.0)) return fail(c, MLB_ENOPOS, "fewer than k positive Ritz values on the fine grid");
        std::vector<double> C(k * k);
        for (int a = 0; a < k; ++a)
            for (int q = 0; q < k; ++q) C[a + k * q] = Y[a * k + q];
        CHK(upload_cm(c, c->cbuf, C));
        launch_gemm_small(n, k, n, c->X1, k, c->cbuf, n, c->Zb, c->st);
        launch_copy_cols(n, k, n, c->Zb, n, c->X1, c->st);
        sigma = 1.0 / ev[0];
        if (nref < 8) lam1_ref[nref] = sigma;
        ++nref;
        CHK(sync(c));
        t_refine += now_s() - ts;
    }
    if (c->ell == 1) launch_copy_cols(n, k, n, c->eS, n, c->X1, c->st);
    launch_copy_cols(n, k, n, c->X1, n, c->Psif, c->st);
    // step 3: K Phi~ = G Psi
    apply_G(c, 1, k, c->X1, c->X2);
    mlb_solve_info si{};
    if (c->o.block_cg) CHK(bpcg(c, c->X2, c->Phi, k, c->tol_solve, c->max_it, false, &si));
    else CHK(pcg(c, c->X2, c->Phi, k, c->tol_solve, c->max_it, false, &si));
    const double t2 = now_s();
    // step 4: Rayleigh-Ritz on span(Phi~); then, optionally, preconditioned
    // inverse iteration steps on the Ritz block (App. A, eq.
    // PInvIt-GeneralInteration), each followed by Rayleigh-Ritz again:
    // phi_i <- phi_i - M^-1 (K + lam~_i G) phi_i, M^-1 one multigrid cycle,
    // each vector shifted by its own Ritz value (the gradient step of its
    // Rayleigh quotient), or, with pinvit_shift = 2, every vector by lam~_1
    // as the step is printed.  After each Ritz step Zo holds the Ritz vectors,
    // R = K Zo, Qb = G Zo.
    const int steps = c->o.pinvit_steps;
    double lam1_before = 0.0, t_pinvit = 0.0;
    for (int s = 0; s <= steps; ++s) {
        if (s > 0) {
            const double ts = now_s();
            if (s == 1) lam1_before = c->lam[0];
            for (int i = 0; i < k; ++i) c->hpin[i] = c->o.pinvit_shift == 2 ? c->lam[0] : c->lam[i];
            HIPC(hipMemcpyAsync(c->dlam_l, c->hpin, sizeof(double) * k, hipMemcpyHostToDevice, c->st));
            launch_axpy_cols(n, k, n, c->dlam_l, 1.0, c->Qb, c->R, c->st);   // (K + lam~_i G) phi_i
            CHK(precondition(c, 1, k, c->R, c->Zb));
            launch_copy_cols(n, k, n, c->Zo, n, c->Phi, c->st);
            launch_axpby((int64_t)n * k, -1.0, c->Zb, 1.0, c->Phi, c->st);
            CHK(sync(c));
            t_pinvit += now_s() - ts;
        }
        apply_K<double>(c, 1, k, c->Phi, c->X1, kModeY, nullptr, nullptr);
        apply_G(c, 1, k, c->Phi, c->X2);
        std::vector<double> A, B;
        CHK(gram2(c, n, k, c->Phi, k, c->X1, c->X2, A, B));
        std::vector<double> A2(k * k), B2(k * k), ev(k), Y(k * k);
        for (int a = 0; a < k; ++a)
            for (int q = 0; q < k; ++q) {
                A2[a * k + q] = 0.5 * (A[a + k * q] + A[q + k * a]);
                B2[a * k + q] = -0.5 * (B[a + k * q] + B[q + k * a]);
            }
        if (!gen_eig(k, A2.data(), B2.data(), ev.data(), Y.data()))
            return fail(c, MLB_EBREAKDOWN, "Rayleigh-Ritz: Phi~^T K Phi~ not positive definite");
        if (!(ev[k - 1] > 0.0)) return fail(c, MLB_ENOPOS, "fewer than k positive Ritz values");
        c->lam.assign(k, 0.0);
        for (int i = 0; i < k; ++i) c->lam[i] = 1.0 / ev[i];
        std::vector<double> C(k * k);
        for (int a = 0; a < k; ++a)
            for (int q = 0; q < k; ++q) C[a + k * q] = Y[a * k + q];
        c->rrC = C;
        CHK(upload_cm(c, c->cbuf, C));
        launch_gemm_small(n, k, n, c->Phi, k, c->cbuf, n, c->Zo, c->st);
        launch_gemm_small(n, k, n, c->X1, k, c->cbuf, n, c->R, c->st);
        launch_gemm_small(n, k, n, c->X2, k, c->cbuf, n, c->Qb, c->st);
    }
    std::memcpy(c->hpin, c->lam.data(), sizeof(double) * k);
    HIPC(hipMemcpyAsync(c->dlam_l, c->hpin, sizeof(double) * k, hipMemcpyHostToDevice, c->st));
    launch_axpy_cols(n, k, n, c->dlam_l, 1.0, c->Qb, c->R, c->st);   // (K + lam G) phi
    const int np = reduction_parts(n);
    CHK(ensure_part(c, (int64_t)np * k));
    launch_infnorm_part(n, k, n, c->R, np, c->part, c->st);
    launch_max_parts(k, np, c->part, sc(c, 14), c->st);
    c->eigres.assign(k, 0.0);
    CHK(read_scal(c, sc(c, 14), k, c->eigres.data()));
    // sign convention: largest-magnitude entry positive (ties: lowest index)
    launch_copy_cols(n, k, n, c->Zo, n, c->Phi, c->st);
    launch_absmax_part(n, k, n, c->Phi, np, c->part, c->pidx, c->st);
    launch_absmax_sum(k, np, c->part, c->pidx, sc(c, 15), c->st);
    std::vector<double> sv(k);
    CHK(read_scal(c, sc(c, 15), k, sv.data()));
    for (int i = 0; i < k; ++i) sv[i] = sv[i] < 0 ? -1.0 : 1.0;
    // returned mode i = sv_i Phi~ C_i, so K phi_i = G (sv_i Psi C_i) when no
    // inverse-iteration step followed the Rayleigh-Ritz step
    for (int i = 0; i < k; ++i)
        for (int a = 0; a < k; ++a) c->rrC[a + (size_t)k * i] *= sv[i];
    c->psi_ok = steps == 0;
    std::memcpy(c->hpin, sv.data(), sizeof(double) * k);
    HIPC(hipMemcpyAsync(sc(c, 15), c->hpin, sizeof(double) * k, hipMemcpyHostToDevice, c->st));
    launch_scale_cols(n, k, n, sc(c, 15), c->Phi, c->st);
    CHK(sync(c));
    const double t3 = now_s();
    c->has_buck = true;
    if (info) {
        info->coarse_iterations = cit;
        info->coarse_residual = cres;
        info->coarse_gap = gap;
        info->coarse_warm_used = warm_used;
        info->coarse_guard_fired = guard;
        info->fine_iterations = si.iterations;
        info->fine_true_residual = si.true_rel_residual;
        info->seconds_coarse = t1 - t0;
        info->seconds_fine = t2 - t1;
        info->seconds_ritz = t3 - t2 - t_pinvit;
        info->pinvit_steps = steps;
        info->lambda1_before_pinvit = steps > 0 ? lam1_before : c->lam[0];
        info->seconds_pinvit = t_pinvit;
        info->refine_levels = nref;
        for (int i = 0; i < 8; ++i) info->refine_lambda1[i] = lam1_ref[i];
        info->seconds_refine = t_refine;
    }
    return MLB_OK;
}

int do_sens(mlb_ctx* c, double* dJ_dev, double* dlam_dev, mlb_solve_info* info) {
    const double t0 = now_s();
    const Geo& g = c->lv[0].g;
    if (dJ_dev) {
        if (!c->has_static) return fail(c, MLB_ESTATE, "compliance sensitivities need a static solve");
        launch_dJ(c->dim, g, c->x, c->d.penal, c->d.E1 - c->d.E0, c->ncases, c->n, c->U, c->dK0, dJ_dev, c->st);
    }
    if (info) *info = mlb_solve_info{};
    if (dlam_dev) {
        if (!c->has_buck) return fail(c, MLB_ESTATE, "buckling sensitivities need mlb_buckling first");
        const int k = c->k;
        double* V = nullptr;
        CHK(dalloc(c, &V, (size_t)g.m * c->nv * k));
        launch_adj_elem(c->dim, g, c->Es, k, c->n, c->Phi, c->dHk, c->dD0, V, c->st);
        launch_adj_gather(c->dim, g, k, V, c->dBc, c->lv[0].nmask, c->n, c->X2, c->st);
        CHK(sync(c));
        dfree(V);
        if (c->o.block_cg) CHK(bpcg(c, c->X2, c->Zadj, k, c->tol_solve, c->max_it, false, info));
        else CHK(pcg(c, c->X2, c->Zadj, k, c->tol_solve, c->max_it, false, info));
        launch_dlam(c->dim, g, c->x, c->d.penal, c->d.E1, c->d.E0, c->U + (int64_t)c->ref_case_used * c->n, k,
                    c->n, c->Phi, c->Zadj, c->dlam_l, c->dK0, c->dHk, c->dD0Bc, dlam_dev, c->st);
        c->has_adj = true;
    }
    CHK(sync(c));
    if (info) info->seconds = now_s() - t0;
    return MLB_OK;
}

// Consistent buckling sensitivities (appendix, eq. consistentSensitivity,
// read through the fine solve K Phi~ = G Psi with Psi fixed): residual
// adjoints w = K^-1 (K + lam G) phi, then K zt = b + (2 / lam) grad_u(w^T G psi)
// as one block each, then the element formula with the residual terms.
int do_sens_consistent(mlb_ctx* c, double* dlam_dev, mlb_solve_info* info) {
    const double t0 = now_s();
    if (!c->has_buck) return fail(c, MLB_ESTATE, "buckling sensitivities need mlb_buckling first");
    if (!c->psi_ok)
        return fail(c, MLB_ESTATE, "the consistent sensitivity is defined for modes from the fine solve and one "
                                   "Rayleigh-Ritz step (no inverse-iteration steps)");
    const Geo& g = c->lv[0].g;
    const int k = c->k;
    const int64_t n = c->n;
    if (!c->cW) CHK(dalloc(c, &c->cW, (size_t)n * k));
    // psi = Psi C (signs included) into X1
    CHK(upload_cm(c, c->cbuf, c->rrC));
    launch_gemm_small(n, k, n, c->Psif, k, c->cbuf, n, c->X1, c->st);
    // y = K phi + lam G phi into Zo (dlam_l holds the factors of the last call)
    apply_K<double>(c, 1, k, c->Phi, c->Zo, kModeY, nullptr, nullptr);
    apply_G(c, 1, k, c->Phi, c->X2);
    launch_axpy_cols(n, k, n, c->dlam_l, 1.0, c->X2, c->Zo, c->st);
    mlb_solve_info s1{}, s2{};
    if (c->o.block_cg) CHK(bpcg(c, c->Zo, c->cW, k, c->tol_solve, c->max_it, false, &s1));
    else CHK(pcg(c, c->Zo, c->cW, k, c->tol_solve, c->max_it, false, &s1));
    double* V = nullptr;
    CHK(dalloc(c, &V, (size_t)g.m * c->nv * k));
    launch_adj_elem(c->dim, g, c->Es, k, n, c->Phi, c->dHk, c->dD0, V, c->st, c->cW, c->X1, c->dlam_l);
    launch_adj_gather(c->dim, g, k, V, c->dBc, c->lv[0].nmask, n, c->X2, c->st);
    CHK(sync(c));
    dfree(V);
    if (c->o.block_cg) CHK(bpcg(c, c->X2, c->Zadj, k, c->tol_solve, c->max_it, false, &s2));
    else CHK(pcg(c, c->X2, c->Zadj, k, c->tol_solve, c->max_it, false, &s2));
    launch_dlam(c->dim, g, c->x, c->d.penal, c->d.E1, c->d.E0, c->U + (int64_t)c->ref_case_used * n, k, n, c->Phi,
                c->Zadj, c->dlam_l, c->dK0, c->dHk, c->dD0Bc, dlam_dev, c->st, c->cW, c->X1);
    c->has_adj = true;
    CHK(sync(c));
    if (info) {
        info->iterations = s1.iterations + s2.iterations;
        info->converged = s1.converged && s2.converged;
        info->rel_residual = std::max(s1.rel_residual, s2.rel_residual);
        info->true_rel_residual = std::max(s1.true_rel_residual, s2.true_rel_residual);
        info->seconds = now_s() - t0;
    }
    return MLB_OK;
}

hipStream_t pick(mlb_ctx* c, void* stream) { return stream ? (hipStream_t)stream : c->own; }

}  // namespace

namespace {
// Mean time (ms) of `reps` calls of f after one untimed call, HIP events on c->st.
template <typename F>
int time_ms(mlb_ctx* c, int reps, F f, float* ms) {
    hipEvent_t a, b;
    HIPC(hipEventCreate(&a));
    HIPC(hipEventCreate(&b));
    f();
    HIPC(hipEventRecord(a, c->st));
    for (int i = 0; i < reps; ++i) f();
    HIPC(hipEventRecord(b, c->st));
    HIPC(hipEventSynchronize(b));
    float t = 0.f;
    HIPC(hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / (float)reps;
    return MLB_OK;
}

// Tunes the pencil length of the fine apply and the column chunk of the
// stencil applies for blocks of ncols columns in the precision of the
// multigrid cycle, on Jacobi sweeps (the dominant launches), and keeps the
// fastest of each.
template <typename T>
// Times the fine apply for every variant and pencil length, in `mode`
// (Jacobi sweeps for the multigrid cycle, plain products for the FP64
// operator of the outer solvers in mixed precision), and keeps the fastest;
// with `stencils`, also the stencil applies of level 2.
int autotune_t(mlb_ctx* c, int ncols, bool stencils, int mode, int* zout, int* vout, float* ms_reg, float* ms_lds,
               float* ms_nopf, float* ms_v3, float* score) {
    Level& l1 = c->lv[0];
    T* x = lbuf<T>(l1, 1);
    T* y = lbuf<T>(l1, 2);
    T* r = lbuf<T>(l1, 0);
    launch_random_fill(l1.n, 1, l1.n, 77, l1.nmask, c->dim, l1.vt, c->st);
    if (sizeof(T) == 4) launch_d2f(l1.n, 1, l1.n, l1.vt, (float*)(void*)l1.ft, c->st);
    const T* src = sizeof(T) == 4 ? (const T*)(const void*)l1.ft : (const T*)(const void*)l1.vt;
    for (int q = 0; q < ncols; ++q) {
        HIPC(hipMemcpyAsync(x + (int64_t)q * l1.n, src, sizeof(T) * l1.n, hipMemcpyDeviceToDevice, c->st));
        HIPC(hipMemcpyAsync(r + (int64_t)q * l1.n, src, sizeof(T) * l1.n, hipMemcpyDeviceToDevice, c->st));
    }
    const int zc[] = {4, 6, 8, 10, 12};
    float best = 1e30f;
    int bz = c->wz[tix<T>()], bv = c->wv[tix<T>()];
    const int nvar = c->dim == 3 ? 4 : 1;
    // The solvers run the fine apply on single columns (static CG) about as
    // often as on the ncols-column blocks (block solves), so each candidate
    // is scored by one sweep of each; the reported times are the block's.
    for (int v = 0; v < nvar; ++v)
        for (int i = 0; i < 5; ++i) {
            c->wz[tix<T>()] = zc[i];
            c->wv[tix<T>()] = v;
            float ms = 0.f, ms1 = 0.f;
            CHK(time_ms(c, 5, [&] { apply_K<T>(c, 1, ncols, x, y, mode, r, nullptr); }, &ms));
            if (ncols > 1) CHK(time_ms(c, 5, [&] { apply_K<T>(c, 1, 1, x, y, mode, r, nullptr); }, &ms1));
            (v == 0 ? ms_reg : v == 1 ? ms_lds : v == 2 ? ms_nopf : ms_v3)[i] = ms;
            score[5 * v + i] = ms + ms1;
            if (ms + ms1 < best) best = ms + ms1, bz = zc[i], bv = v;
        }
    c->wz[tix<T>()] = bz;
    c->wv[tix<T>()] = bv;
    *zout = bz;
    *vout = bv;
    if (stencils && c->L > 1) {
        Level& l2 = c->lv[1];
        T* x2 = lbuf<T>(l2, 1);
        T* y2 = lbuf<T>(l2, 2);
        T* r2 = lbuf<T>(l2, 0);
        launch_restrict_nb<T>(c->dim, l1.g, l2.g, l1.nmask, l2.nmask, ncols, l1.n, l2.n, x, x2, c->st);
        launch_restrict_nb<T>(c->dim, l1.g, l2.g, l1.nmask, l2.nmask, ncols, l1.n, l2.n, r, r2, c->st);
        const int cb[] = {2, 3, 4, 6, 12};
        best = 1e30f;
        int bc = c->nb_cbmax;
        for (int i = 0; i < 5; ++i) {
            c->nb_cbmax = cb[i];
            float ms = 0.f;
            CHK(time_ms(c, 5, [&] { apply_K<T>(c, 2, ncols, x2, y2, kModeJacobi, r2, nullptr); }, &ms));
            c->tune_stencil_ms[i] = ms;
            if (ms < best) best = ms, bc = cb[i];
        }
        c->nb_cbmax = bc;
    }
    CHK(sync(c));
    return MLB_OK;
}
}  // namespace


// ============================ C ABI ======================================

extern "C" {

int mlb_create(const mlb_desc* desc, mlb_ctx** out) {
    if (!desc || !out) return MLB_EINVAL;
    *out = nullptr;
    mlb_ctx* c = new mlb_ctx();
    c->d = *desc;
    c->o.smooth_steps = 2;
    c->o.jacobi_omega = 4.0 / 3.0;
    c->o.eig_guard = 0;
    c->o.eig_max_it = 400;
    c->o.check_every = 8;
    c->o.pinvit_shift = 1;
    c->o.refine_fine = 0;
    c->o.seed = 1;
    c->o.cycle = 1;
    c->o.block_cg = 1;
    c->o.eig_sweeps = 3;
    c->o.graphs = 1;

    const int dim = desc->dim;
    auto bad = [&](const std::string& m) {
        c->err = m;
        *out = c;   // returned so mlb_last_error works; caller must destroy
        return MLB_EINVAL;
    };
    if (dim != 2 && dim != 3) return bad("dim must be 2 or 3");
    if (desc->mg_levels < 1 || desc->mg_levels > 12) return bad("mg_levels must be in 1..12");
    if (desc->eig_level < 1 || desc->eig_level > desc->mg_levels) return bad("eig_level must be in 1..mg_levels");
    if (desc->precision != MLB_FP64 && desc->precision != MLB_MIXED) return bad("unknown precision");
    if (desc->element != MLB_ELEM_CONFORMING && desc->element != MLB_ELEM_INCOMPATIBLE)
        return bad("unknown element (MLB_ELEM_CONFORMING or MLB_ELEM_INCOMPATIBLE)");
    if (!(desc->E1 > 0) || !(desc->E0 >= 0) || !(desc->E0 < desc->E1)) return bad("need 0 <= E0 < E1");
    if (!(desc->nu > -1.0 && desc->nu < 0.5)) return bad("Poisson ratio must lie in (-1, 0.5)");
    if (!(desc->penal >= 1.0)) return bad("penalty p must be >= 1");
    const int div = 1 << (desc->mg_levels - 1);
    for (int a = 0; a < dim; ++a)
        if (desc->nel[a] < div || desc->nel[a] % div)
            return bad("every nel must be a positive multiple of 2^(mg_levels-1)");
    c->dim = dim;
    c->nn = 1 << dim;
    c->nde = dim << dim;
    c->nv = dim == 2 ? 3 : 6;
    c->L = desc->mg_levels;
    c->ell = desc->eig_level;
    if (hipSetDevice(desc->device) != hipSuccess) {
        c->err = "hipSetDevice failed";
        *out = c;
        return MLB_EDEVICE;
    }
    // the fixed scratch of the no-allocation entry points, looked up once per
    // device with that device current
    if (scratch_address(desc->device, &c->scratch) != hipSuccess) {
        c->err = "no address for the device scratch array";
        *out = c;
        return MLB_EDEVICE;
    }
    *out = c;
    HIPC(hipStreamCreate(&c->own));
    c->st = c->own;
    build_tables(dim, desc->nu, desc->element, &c->tab);
    for (int i = 0; i < 9; ++i) c->whtf[i] = (float)c->tab.whs[i];
    // device tables
    CHK(dalloc(c, &c->dK0, 576));
    CHK(dalloc(c, &c->fK0, 576));
    CHK(dalloc(c, &c->dHk, 6 * 64));
    CHK(dalloc(c, &c->dBc, 6 * 24));
    CHK(dalloc(c, &c->dD0Bc, 6 * 24));
    CHK(dalloc(c, &c->dD0, 36));
    CHK(dalloc(c, &c->dT, 512));
    CHK(dalloc(c, &c->dMc, 8 * 576));
    CHK(dalloc(c, &c->dGHc, 8 * 6 * 64));
    float k0f[576];
    for (int i = 0; i < 576; ++i) k0f[i] = (float)c->tab.K0[i];
    HIPC(hipMemcpy(c->dK0, c->tab.K0, sizeof(double) * 576, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->fK0, k0f, sizeof(float) * 576, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dHk, c->tab.Hk, sizeof(double) * 6 * 64, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dBc, c->tab.Bc, sizeof(double) * 6 * 24, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dD0Bc, c->tab.D0Bc, sizeof(double) * 6 * 24, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dD0, c->tab.D0, sizeof(double) * 36, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dT, c->tab.T, sizeof(double) * 512, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dMc, c->tab.Mc, sizeof(double) * 8 * 576, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(c->dGHc, c->tab.GHc, sizeof(double) * 8 * 6 * 64, hipMemcpyHostToDevice));
    // levels
    c->lv.resize(c->L);
    int nel[3] = {desc->nel[0], desc->nel[1], dim == 3 ? desc->nel[2] : 1};
    for (int j = 0; j < c->L; ++j) {
        Level& l = c->lv[j];
        int ne[3] = {nel[0] >> j, nel[1] >> j, dim == 3 ? nel[2] >> j : 1};
        l.g = make_geo(dim, ne);
        l.n = (int64_t)dim * l.g.nodes;
        CHK(dalloc(c, &l.nmask, (size_t)l.g.nodes));
        HIPC(hipMemset(l.nmask, 0, (size_t)l.g.nodes));
        CHK(dalloc(c, &l.dinv, (size_t)l.n));
        CHK(dalloc(c, &l.dinvf, (size_t)l.n));
        if (j > 0) {
            CHK(dalloc(c, &l.Ke, (size_t)l.g.m * c->nde * c->nde));
            CHK(dalloc(c, &l.A, (size_t)stencil_entries(dim, l.g, false)));
            CHK(dalloc(c, &l.Af, (size_t)stencil_entries(dim, l.g, false, true)));
        }
        if (j > 0 && j < c->ell) CHK(dalloc(c, &l.Ge, (size_t)l.g.m * c->nn * c->nn));
    }
    c->n = c->lv[0].n;
    c->m = c->lv[0].g.m;
    if (c->L > 1) {
        const int64_t nL = c->lv[c->L - 1].n;
        if (nL > kMaxCoarsest) {
            c->err = "coarsest level has " + std::to_string(nL) + " DOFs (> " + std::to_string(kMaxCoarsest) +
                     "): use more multigrid levels";
            return MLB_EINVAL;
        }
        c->nA = coarse_pad(nL);
        c->nsplit = coarse_splits(c->nA);
        CHK(dalloc(c, &c->Ainv, (size_t)c->nA * c->nA));
        CHK(dalloc(c, &c->Apk, (size_t)packed_lower_doubles(c->nA)));
        CHK(dalloc(c, &c->gjP, (size_t)2 * 64 * 64));
        CHK(dalloc(c, &c->gjR, (size_t)64 * c->nA));
        CHK(dalloc(c, &c->gjC, (size_t)64 * c->nA));
        CHK(dalloc(c, &c->cpart, (size_t)c->nsplit * 32 * c->nA + (size_t)coarse_stage_doubles(c->nA)));
    }
    if (c->ell > 1) {
        Level& le = c->lv[c->ell - 1];
        CHK(dalloc(c, &le.Gs, (size_t)stencil_entries(dim, le.g, true)));
    }
    CHK(dalloc(c, &c->x, (size_t)c->m));
    CHK(dalloc(c, &c->Ek, (size_t)c->m));
    CHK(dalloc(c, &c->Ekf, (size_t)c->m));
    CHK(dalloc(c, &c->Es, (size_t)c->m));
    CHK(dalloc(c, &c->S, (size_t)c->m * c->nv));
    CHK(dalloc(c, &c->fixed, (size_t)c->n));
    CHK(dalloc(c, &c->scal, (size_t)16 * kScal));
    CHK(dalloc(c, &c->iscal, (size_t)3 * kScal));
    CHK(dalloc(c, &c->gbuf, (size_t)96 * 192));
    CHK(dalloc(c, &c->cbuf, (size_t)2 * 96 * 96));
    CHK(dalloc(c, &c->cbuf2, (size_t)96 * 96));
    HIPC(hipHostMalloc((void**)&c->hpin, sizeof(double) * 96 * 192, hipHostMallocDefault));
    HIPC(hipHostMalloc((void**)&c->hup, sizeof(double) * 2 * 96 * 96, hipHostMallocDefault));
    CHK(ensure_part(c, 4096));
    CHK(ensure_level_cols(c, 1));
    return MLB_OK;
}

void mlb_destroy(mlb_ctx* c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (auto& l : c->lv) {
        dfree(l.nmask); dfree(l.Ke); dfree(l.A); dfree(l.Af); dfree(l.Ge); dfree(l.Gs); dfree(l.dinv); dfree(l.dinvf);
        dfree(l.vr); dfree(l.vz); dfree(l.vz2); dfree(l.vt); dfree(l.fr); dfree(l.fz); dfree(l.fz2); dfree(l.ft);
    }
    dfree(c->dK0); dfree(c->fK0); dfree(c->dHk); dfree(c->dBc); dfree(c->dD0Bc); dfree(c->dD0); dfree(c->dT);
    dfree(c->dMc); dfree(c->dGHc); dfree(c->x); dfree(c->Ek); dfree(c->Ekf); dfree(c->Es); dfree(c->fixed);
    dfree(c->F); dfree(c->U); dfree(c->S); dfree(c->Ainv); dfree(c->Apk); dfree(c->gjP); dfree(c->gjR);
    dfree(c->gjC); dfree(c->cpart); dfree(c->R); dfree(c->Zb); dfree(c->Pb); dfree(c->Qb); dfree(c->Zo);
    dfree(c->X1); dfree(c->X2); dfree(c->Phi); dfree(c->Zadj); dfree(c->dlam_l); dfree(c->eS); dfree(c->eK);
    dfree(c->eA); dfree(c->eT); dfree(c->eTK); dfree(c->eTA); dfree(c->eR); dfree(c->eP); dfree(c->ePK); dfree(c->ePA); dfree(c->part); dfree(c->pidx);
    dfree(c->scal); dfree(c->iscal); dfree(c->gbuf); dfree(c->cbuf); dfree(c->cbuf2);
    dfree(c->fw); dfree(c->warm_coarse); dfree(c->warm_static); dfree(c->Psif); dfree(c->cW);
    dfree(c->fineA); dfree(c->fineGs); dfree(c->fineDinv); dfree(c->fineAf); dfree(c->fineDinvf);
    if (c->hpin) (void)hipHostFree(c->hpin);
    if (c->hup) (void)hipHostFree(c->hup);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    for (hipEvent_t e : c->aux_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
}

const char* mlb_last_error(const mlb_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mlb_set_opts(mlb_ctx* c, const mlb_opts* o) {
    if (!c || !o) return MLB_EINVAL;
    if (o->smooth_steps > 0) c->o.smooth_steps = o->smooth_steps;
    if (o->jacobi_omega > 0) c->o.jacobi_omega = o->jacobi_omega;
    if (o->eig_guard > 0) c->o.eig_guard = o->eig_guard;
    if (o->eig_max_it > 0) c->o.eig_max_it = o->eig_max_it;
    if (o->check_every > 0) c->o.check_every = o->check_every;
    if (o->seed > 0) c->o.seed = o->seed;
    if (o->cycle > 0) c->o.cycle = std::min(o->cycle, 2);
    if (o->block_cg > 0) c->o.block_cg = o->block_cg == 1 ? 1 : 0;
    if (o->eig_sweeps > 0) c->o.eig_sweeps = std::min(o->eig_sweeps, 8);
    if (o->graphs > 0) c->o.graphs = o->graphs == 1 ? 1 : 2;
    if (o->pinvit_steps > 0) c->o.pinvit_steps = std::min(o->pinvit_steps, 64);
    else if (o->pinvit_steps < 0) c->o.pinvit_steps = 0;
    if (o->coarse_sweeps > 0) c->o.coarse_sweeps = std::min(o->coarse_sweeps, 64);
    if (o->pinvit_shift > 0) c->o.pinvit_shift = o->pinvit_shift == 2 ? 2 : 1;
    if (o->refine_fine > 0) c->o.refine_fine = 1;
    else if (o->refine_fine < 0) c->o.refine_fine = 0;
    if (o->refine_sweeps > 0) c->o.refine_sweeps = std::min(o->refine_sweeps, 16);
    else if (o->refine_sweeps < 0) c->o.refine_sweeps = 0;
    drop_graphs(c);
    if (o->jacobi_omega > 0 && c->has_density) {
        c->st = c->own;
        for (int j = 1; j < c->L; ++j) CHK(estimate_omega(c, j));
    }
    return MLB_OK;
}

int mlb_level_size(const mlb_ctx* c, int level, int64_t* n_dofs, int64_t* n_elems) {
    if (!c || level < 1 || level > c->L) return MLB_EINVAL;
    if (n_dofs) *n_dofs = c->lv[level - 1].n;
    if (n_elems) *n_elems = c->lv[level - 1].g.m;
    return MLB_OK;
}

static int set_bc_common(mlb_ctx* c) {
    // host check of nestedness + coarse masks, then node masks on device
    const int dim = c->dim;
    std::vector<uint8_t> mf(c->lv[0].g.nodes, 0);
    for (int64_t nd = 0; nd < c->lv[0].g.nodes; ++nd)
        for (int cc = 0; cc < dim; ++cc)
            if (c->fixed_host[nd * dim + cc]) mf[nd] |= (uint8_t)(1u << cc);
    HIPC(hipMemcpyAsync(c->lv[0].nmask, mf.data(), mf.size(), hipMemcpyHostToDevice, c->st));
    CHK(sync(c));
    for (int j = 1; j < c->L; ++j) {
        const Geo& gf = c->lv[j - 1].g;
        const Geo& gc = c->lv[j].g;
        std::vector<uint8_t> mc(gc.nodes, 0);
        for (int64_t N = 0; N < gc.nodes; ++N) {
            const int I = (int)(N % gc.nnx), J = (int)((N / gc.nnx) % gc.nny), K = (int)(N / ((int64_t)gc.nnx * gc.nny));
            mc[N] = mf[2 * I + (int64_t)gf.nnx * (2 * J + (int64_t)gf.nny * 2 * K)];
        }
        // every fixed fine DOF must interpolate only from fixed coarse DOFs
        for (int64_t nd = 0; nd < gf.nodes; ++nd) {
            if (!mf[nd]) continue;
            const int i = (int)(nd % gf.nnx), jj = (int)((nd / gf.nnx) % gf.nny), k = (int)(nd / ((int64_t)gf.nnx * gf.nny));
            const int ni = (i & 1) ? 2 : 1, nj = (jj & 1) ? 2 : 1, nk = (dim == 3 && (k & 1)) ? 2 : 1;
            for (int dk = 0; dk < nk; ++dk)
                for (int dj = 0; dj < nj; ++dj)
                    for (int di = 0; di < ni; ++di) {
                        const int64_t cn = (i / 2 + di) + (int64_t)gc.nnx * ((jj / 2 + dj) + (int64_t)gc.nny * (k / 2 + dk));
                        if ((mf[nd] & ~mc[cn]) != 0)
                            return fail(c, MLB_EINVAL, "fixed DOF set is not nested across multigrid levels");
                    }
        }
        HIPC(hipMemcpyAsync(c->lv[j].nmask, mc.data(), mc.size(), hipMemcpyHostToDevice, c->st));
        CHK(sync(c));
        mf.swap(mc);
    }
    HIPC(hipMemcpyAsync(c->fixed, c->fixed_host.data(), (size_t)c->n, hipMemcpyHostToDevice, c->st));
    CHK(sync(c));
    c->has_bc = true;
    c->has_static = c->has_buck = c->has_stress = false;
    if (c->has_density) CHK(build_hierarchy(c));
    return MLB_OK;
}

int mlb_set_bc(mlb_ctx* c, const uint8_t* fixed) {
    if (!c || !fixed) return MLB_EINVAL;
    c->st = c->own;
    c->fixed_host.assign(fixed, fixed + c->n);
    for (auto& v : c->fixed_host) v = v ? 1 : 0;
    return set_bc_common(c);
}

int mlb_set_bc_dev(mlb_ctx* c, const uint8_t* fixed, void* stream) {
    if (!c || !fixed) return MLB_EINVAL;
    c->st = pick(c, stream);
    c->fixed_host.assign(c->n, 0);
    HIPC(hipMemcpyAsync(c->fixed_host.data(), fixed, (size_t)c->n, hipMemcpyDeviceToHost, c->st));
    CHK(sync(c));
    for (auto& v : c->fixed_host) v = v ? 1 : 0;
    return set_bc_common(c);
}

static int set_loads_common(mlb_ctx* c, int ncases) {
    c->ncases = ncases;
    c->J.assign(ncases, 0.0);
    c->has_static = c->has_buck = false;
    c->has_adj = false;
    CHK(ensure_cg(c, std::max(ncases, c->k)));
    return MLB_OK;
}

int mlb_set_loads(mlb_ctx* c, int ncases, const double* F) {
    if (!c || !F || ncases < 1 || ncases > 64) return fail(c, MLB_EINVAL, "need 1..64 load cases");
    if (!c->has_bc) return fail(c, MLB_ESTATE, "set the Dirichlet mask before the loads");
    c->st = c->own;
    std::vector<double> h(F, F + (size_t)c->n * ncases);
    for (int cc = 0; cc < ncases; ++cc)
        for (int64_t i = 0; i < c->n; ++i) {
            double& v = h[(size_t)cc * c->n + i];
            if (!std::isfinite(v)) return fail(c, MLB_EINVAL, "non-finite load entry");
            if (c->fixed_host[i]) v = 0.0;
        }
    CHK(dalloc(c, &c->F, h.size()));
    CHK(dalloc(c, &c->U, h.size()));
    HIPC(hipMemcpy(c->F, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
    return set_loads_common(c, ncases);
}

int mlb_set_loads_dev(mlb_ctx* c, int ncases, const double* F, void* stream) {
    if (!c || !F || ncases < 1 || ncases > 64) return fail(c, MLB_EINVAL, "need 1..64 load cases");
    if (!c->has_bc) return fail(c, MLB_ESTATE, "set the Dirichlet mask before the loads");
    c->st = pick(c, stream);
    std::vector<double> h((size_t)c->n * ncases);
    HIPC(hipMemcpyAsync(h.data(), F, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->st));
    CHK(sync(c));
    c->st = c->own;
    return mlb_set_loads(c, ncases, h.data());
}

static int set_density_common(mlb_ctx* c) {
    const int np = reduction_parts(c->m);
    CHK(ensure_part(c, np));
    launch_material(c->m, c->x, c->d.E1, c->d.E0, c->d.penal, c->Ek, c->Ekf, c->Es, np, c->part, c->st);
    launch_sum_parts(1, np, c->part, sc(c, 0), c->st);
    double nbad = 0;
    CHK(read_scal(c, sc(c, 0), 1, &nbad));
    if (nbad > 0) {
        c->has_density = false;
        return fail(c, MLB_EINVAL, "densities must be finite and lie in [0, 1]");
    }
    c->has_static = c->has_buck = c->has_stress = c->has_adj = false;
    c->has_density = true;
    if (!c->has_bc) return MLB_OK;   // the hierarchy is built when the mask arrives
    return build_hierarchy(c);
}

int mlb_set_penal(mlb_ctx* c, double penal) {
    if (!c) return MLB_EINVAL;
    if (!(penal >= 1.0) || !std::isfinite(penal)) return fail(c, MLB_EINVAL, "penalty p must be finite and >= 1");
    c->d.penal = penal;
    // the moduli were interpolated with the old exponent
    c->has_density = false;
    c->has_static = c->has_buck = c->has_stress = c->has_adj = false;
    return MLB_OK;
}

int mlb_set_density(mlb_ctx* c, const double* x) {
    if (!c || !x) return MLB_EINVAL;
    c->st = c->own;
    if (c->d.E0 == 0.0)
        for (int64_t e = 0; e < c->m; ++e)
            if (!(x[e] > 0.0)) return fail(c, MLB_EINVAL, "with E0 = 0 every density must be positive");
    HIPC(hipMemcpy(c->x, x, sizeof(double) * c->m, hipMemcpyHostToDevice));
    return set_density_common(c);
}

int mlb_set_density_dev(mlb_ctx* c, const double* x, void* stream) {
    if (!c || !x) return MLB_EINVAL;
    c->st = pick(c, stream);
    HIPC(hipMemcpyAsync(c->x, x, sizeof(double) * c->m, hipMemcpyDeviceToDevice, c->st));
    return set_density_common(c);
}

static int solve_static_common(mlb_ctx* c, double tol, int max_it, mlb_solve_info* info) {
    if (!c->has_bc || !c->has_density) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    if (c->ncases < 1 || !c->F) return fail(c, MLB_ESTATE, "set the loads first");
    if (!(tol > 0) || max_it < 1) return fail(c, MLB_EINVAL, "need tol > 0 and max_it >= 1");
    c->tol_solve = tol;
    c->max_it = max_it;
    c->has_static = c->has_buck = false;
    c->has_adj = false;
    bool x0 = false;
    if (c->warm_static && c->warm_static_cols == c->ncases) {
        // initial guess scaled per column to its energy-optimal multiple
        // alpha = f^T u0 / u0^T K u0 (the minimiser of the energy-norm error
        // along u0), so a guess of the right shape but any scale helps
        const int nc = c->ncases;
        CHK(ensure_cg(c, nc));
        HIPC(hipMemcpyAsync(c->U, c->warm_static, sizeof(double) * c->n * nc, hipMemcpyDeviceToDevice, c->st));
        launch_mask_fixed(c->n, nc, c->n, c->lv[0].nmask, c->dim, c->U, c->st);
        apply_K<double>(c, 1, nc, c->U, c->R, kModeY, nullptr, nullptr);
        dots(c, c->n, nc, c->F, c->U, sc(c, 0));
        dots(c, c->n, nc, c->U, c->R, sc(c, 0) + nc);
        std::vector<double> fu(2 * nc);
        CHK(read_scal(c, sc(c, 0), 2 * nc, fu.data()));
        // (this never does worse than the zero start in the energy norm; a
        // non-finite guess falls back to the zero start)
        bool finite = true;
        for (double v : fu) finite = finite && std::isfinite(v);
        if (finite) {
            std::vector<double> alpha(nc);
            for (int i = 0; i < nc; ++i) alpha[i] = fu[nc + i] > 0 ? fu[i] / fu[nc + i] : 0.0;
            CHK(upload_cm(c, sc(c, 1), alpha));
            launch_scale_cols(c->n, nc, c->n, sc(c, 1), c->U, c->st);
            x0 = true;
        }
    }
    if (c->ncases > 1 && c->o.block_cg) CHK(bpcg(c, c->F, c->U, c->ncases, tol, max_it, x0, info));
    else CHK(pcg(c, c->F, c->U, c->ncases, tol, max_it, x0, info));
    dots(c, c->n, c->ncases, c->F, c->U, sc(c, 0));
    CHK(read_scal(c, sc(c, 0), c->ncases, c->J.data()));
    c->has_static = true;
    return MLB_OK;
}

int mlb_solve_static(mlb_ctx* c, double tol, int max_it, double* U, double* J, mlb_solve_info* info) {
    if (!c) return MLB_EINVAL;
    c->st = c->own;
    CHK(solve_static_common(c, tol, max_it, info));
    if (U) HIPC(hipMemcpy(U, c->U, sizeof(double) * c->n * c->ncases, hipMemcpyDeviceToHost));
    if (J) std::memcpy(J, c->J.data(), sizeof(double) * c->ncases);
    return MLB_OK;
}

int mlb_solve_static_dev(mlb_ctx* c, double tol, int max_it, double* U, double* J_host, mlb_solve_info* info,
                         void* stream) {
    if (!c) return MLB_EINVAL;
    c->st = pick(c, stream);
    CHK(solve_static_common(c, tol, max_it, info));
    if (U) HIPC(hipMemcpyAsync(U, c->U, sizeof(double) * c->n * c->ncases, hipMemcpyDeviceToDevice, c->st));
    if (J_host) std::memcpy(J_host, c->J.data(), sizeof(double) * c->ncases);
    CHK(sync(c));
    return MLB_OK;
}

int mlb_buckling(mlb_ctx* c, int ref_case, int k, double tol_eig, double* lambda, double* Phi, mlb_eig_info* info) {
    if (!c) return MLB_EINVAL;
    c->st = c->own;
    CHK(do_buckling(c, ref_case, k, tol_eig, info));
    if (lambda) std::memcpy(lambda, c->lam.data(), sizeof(double) * k);
    if (Phi) HIPC(hipMemcpy(Phi, c->Phi, sizeof(double) * c->n * k, hipMemcpyDeviceToHost));
    return MLB_OK;
}

int mlb_buckling_dev(mlb_ctx* c, int ref_case, int k, double tol_eig, double* lambda_host, double* Phi,
                     mlb_eig_info* info, void* stream) {
    if (!c) return MLB_EINVAL;
    c->st = pick(c, stream);
    CHK(do_buckling(c, ref_case, k, tol_eig, info));
    if (lambda_host) std::memcpy(lambda_host, c->lam.data(), sizeof(double) * k);
    if (Phi) HIPC(hipMemcpyAsync(Phi, c->Phi, sizeof(double) * c->n * k, hipMemcpyDeviceToDevice, c->st));
    CHK(sync(c));
    return MLB_OK;
}

int mlb_eig_residuals(mlb_ctx* c, double* res) {
    if (!c || !res) return MLB_EINVAL;
    if (!c->has_buck) return fail(c, MLB_ESTATE, "no buckling result");
    std::memcpy(res, c->eigres.data(), sizeof(double) * c->eigres.size());
    return MLB_OK;
}

int mlb_eig_residuals_dev(mlb_ctx* c, double* res, void* stream) {
    if (!c || !res) return MLB_EINVAL;
    if (!c->has_buck) return fail(c, MLB_ESTATE, "no buckling result");
    c->st = pick(c, stream);
    // the norms were reduced on the device into scalar slot 14 by the last
    // buckling call (one value per mode)
    HIPC(hipMemcpyAsync(res, sc(c, 14), sizeof(double) * c->k, hipMemcpyDeviceToDevice, c->st));
    return MLB_OK;
}

int mlb_sensitivities(mlb_ctx* c, double* dJ, double* dlam, mlb_solve_info* info) {
    if (!c) return MLB_EINVAL;
    c->st = c->own;
    double *dJd = nullptr, *dld = nullptr;
    if (dJ) CHK(dalloc(c, &dJd, (size_t)c->m * std::max(1, c->ncases)));
    if (dlam) CHK(dalloc(c, &dld, (size_t)c->m * std::max(1, c->k)));
    int r = do_sens(c, dJd, dld, info);
    if (r == MLB_OK && dJ) HIPC(hipMemcpy(dJ, dJd, sizeof(double) * c->m * c->ncases, hipMemcpyDeviceToHost));
    if (r == MLB_OK && dlam) HIPC(hipMemcpy(dlam, dld, sizeof(double) * c->m * c->k, hipMemcpyDeviceToHost));
    dfree(dJd);
    dfree(dld);
    return r;
}

int mlb_sensitivities_consistent(mlb_ctx* c, double* dlam, mlb_solve_info* info) {
    if (!c || !dlam) return MLB_EINVAL;
    c->st = c->own;
    if (!c->has_buck) return fail(c, MLB_ESTATE, "buckling sensitivities need mlb_buckling first");
    double* d = nullptr;
    CHK(dalloc(c, &d, (size_t)c->m * c->k));
    const int st = do_sens_consistent(c, d, info);
    if (st == MLB_OK) HIPC(hipMemcpy(dlam, d, sizeof(double) * c->m * c->k, hipMemcpyDeviceToHost));
    dfree(d);
    return st;
}

int mlb_sensitivities_consistent_dev(mlb_ctx* c, double* dlam, mlb_solve_info* info, void* stream) {
    if (!c || !dlam) return MLB_EINVAL;
    c->st = pick(c, stream);
    return do_sens_consistent(c, dlam, info);
}

int mlb_sensitivities_dev(mlb_ctx* c, double* dJ, double* dlam, mlb_solve_info* info, void* stream) {
    if (!c) return MLB_EINVAL;
    c->st = pick(c, stream);
    return do_sens(c, dJ, dlam, info);
}

int mlb_mac_dev(mlb_ctx* c, int qa, const double* A, int qb, const double* B, double* W, double* C_host,
                void* stream) {
    if (!c || !A || !B || !W || !C_host || qa < 1 || qb < 1) return MLB_EINVAL;
    if (qa + qb > 192 || (int64_t)qa * qb > 96 * 192)
        return fail(c, MLB_EINVAL, "correlation blocks too wide (qa + qb <= 192, qa qb <= 96 x 192)");
    if (W == B) return fail(c, MLB_EINVAL, "the workspace must not overlap B");
    if (!c->has_density || !c->has_bc) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    c->st = pick(c, stream);
    apply_K<double>(c, 1, qb, B, W, kModeY, nullptr, nullptr, false);
    HIPC(hipGetLastError());
    std::vector<double> C;
    CHK(gram(c, c->n, qa, A, c->n, qb, W, c->n, C));
    std::memcpy(C_host, C.data(), sizeof(double) * qa * qb);
    return MLB_OK;
}

int mlb_sed_tv_dev(mlb_ctx* c, int q, const double* Phi, double xbar, double* sed, double* gradn,
                   double* tv_host, void* stream) {
    if (!c || !Phi || !sed || !gradn || q < 1 || q > 65535) return MLB_EINVAL;
    if (!std::isfinite(xbar)) return fail(c, MLB_EINVAL, "xbar must be finite");
    if (!c->has_density) return fail(c, MLB_ESTATE, "set the densities first");
    c->st = pick(c, stream);
    const Geo& g = c->lv[0].g;
    const int np = grad_tv_parts(g);
    CHK(ensure_part(c, (int64_t)np * q + q));
    launch_sed(c->dim, g, c->Ek, q, c->n, Phi, c->dK0, sed, c->st);
    launch_grad_tv(c->dim, g, c->x, xbar, q, sed, gradn, c->part, c->st);
    HIPC(hipGetLastError());
    if (tv_host) {
        double* tv = c->part + (int64_t)np * q;
        launch_sum_parts(q, np, c->part, tv, c->st);
        HIPC(hipGetLastError());
        for (int i0 = 0; i0 < q; i0 += 96 * 192)
            CHK(read_scal(c, tv + i0, std::min(q - i0, 96 * 192), tv_host + i0));
    }
    return MLB_OK;
}

int mlb_dilate_dev(mlb_ctx* c, int nsel, const double* gradn, double rel_thr, double r_th, const double* x,
                   double* xout, void* stream) {
    if (!c || !gradn || !x || !xout || nsel < 1 || nsel > 65535) return MLB_EINVAL;
    if (!(r_th >= 0.0 && r_th <= 8.0)) return fail(c, MLB_EINVAL, "r_th must be in [0, 8]");
    if (!(rel_thr >= 0.0) || !std::isfinite(rel_thr)) return fail(c, MLB_EINVAL, "rel_thr must be >= 0 and finite");
    const Geo& g = c->lv[0].g;
    if (x < xout + g.m && xout < x + g.m) return fail(c, MLB_EINVAL, "x and xout must not overlap");
    c->st = pick(c, stream);
    const int np = grad_tv_parts(g);
    CHK(ensure_part(c, (int64_t)np * nsel + nsel));
    double* gmax = c->part + (int64_t)np * nsel;
    launch_infnorm_part(g.m, nsel, g.m, gradn, np, c->part, c->st);
    launch_max_parts(nsel, np, c->part, gmax, c->st);
    launch_dilate(c->dim, g, nsel, gradn, gmax, rel_thr, r_th, x, xout, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_dilate_noalloc_dev(mlb_ctx* c, int nsel, const double* gradn, double rel_thr, double r_th, const double* x,
                           double* xout, void* stream) {
    if (!c || !gradn || !x || !xout || nsel < 1) return MLB_EINVAL;
    if (nsel > kNoallocMaxSel)
        return fail(c, MLB_EINVAL, "mlb_dilate_noalloc_dev takes at most " + std::to_string(kNoallocMaxSel) +
                                       " rows of gradn (the fixed scratch holds no more)");
    if (!(r_th >= 0.0 && r_th <= 8.0)) return fail(c, MLB_EINVAL, "r_th must be in [0, 8]");
    if (!(rel_thr >= 0.0) || !std::isfinite(rel_thr)) return fail(c, MLB_EINVAL, "rel_thr must be >= 0 and finite");
    const Geo& g = c->lv[0].g;
    if (x < xout + g.m && xout < x + g.m) return fail(c, MLB_EINVAL, "x and xout must not overlap");
    const int np = grad_tv_parts(g);
    if ((int64_t)np * nsel + nsel > kScratchDoubles) return fail(c, MLB_EINVAL, "scratch too small");
    c->st = pick(c, stream);
    // every slot the kernels read is written first in the same call (one
    // partial per block and row, then one maximum per row): nothing is cleared
    double* part = c->scratch;
    double* gmax = c->scratch + (int64_t)np * nsel;
    launch_infnorm_part(g.m, nsel, g.m, gradn, np, part, c->st);
    launch_max_parts(nsel, np, part, gmax, c->st);
    launch_dilate(c->dim, g, nsel, gradn, gmax, rel_thr, r_th, x, xout, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

// Filter weights w = rmin - |o| > 0 for the integer offsets o, axis 0 outermost.
static int filter_table(mlb_ctx* c, double rmin) {
    if (rmin == c->fw_r && c->fw) return MLB_OK;
    const int r = (int)std::ceil(rmin);
    const int rz = c->dim == 3 ? r : 0;
    std::vector<double> t;
    for (int oi = -r; oi <= r; ++oi)
        for (int oj = -r; oj <= r; ++oj)
            for (int ok = -rz; ok <= rz; ++ok) {
                const double w = rmin - std::sqrt((double)(oi * oi + oj * oj + ok * ok));
                if (w > 0.0) t.insert(t.end(), {(double)oi, (double)oj, (double)ok, w});
            }
    CHK(sync(c));   // the previous table may still be read
    c->fw_host = std::move(t);
    c->fw_n = (int)(c->fw_host.size() / 4);
    CHK(dalloc(c, &c->fw, c->fw_host.size()));
    HIPC(hipMemcpy(c->fw, c->fw_host.data(), sizeof(double) * c->fw_host.size(), hipMemcpyHostToDevice));
    c->fw_r = rmin;
    return MLB_OK;
}

static int check_design_args(mlb_ctx* c, double rmin, double eta, double beta) {
    if (!(rmin > 0.0 && rmin <= 16.0)) return fail(c, MLB_EINVAL, "rmin must be in (0, 16]");
    if (!(eta >= 0.0 && eta <= 1.0)) return fail(c, MLB_EINVAL, "eta must be in [0, 1]");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(c, MLB_EINVAL, "beta must be positive and finite");
    return MLB_OK;
}

int mlb_filter_project_dev(mlb_ctx* c, const double* xhat, double rmin, double eta, double beta, double* xtilde,
                           double* x, void* stream) {
    if (!c || !xhat || !xtilde || !x) return MLB_EINVAL;
    CHK(check_design_args(c, rmin, eta, beta));
    if (xtilde == x || xhat == xtilde || xhat == x) return fail(c, MLB_EINVAL, "xhat, xtilde and x must be distinct");
    c->st = pick(c, stream);
    CHK(filter_table(c, rmin));
    launch_filter_project(c->lv[0].g, c->fw_n, c->fw, eta, beta, xhat, xtilde, x, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_filter_chain_dev(mlb_ctx* c, int ncols, const double* xtilde, double rmin, double eta, double beta,
                         const double* dfdx, double* work, double* dfdxhat, void* stream) {
    if (!c || !xtilde || !dfdx || !work || !dfdxhat || ncols < 1 || ncols > 65535) return MLB_EINVAL;
    CHK(check_design_args(c, rmin, eta, beta));
    if (work == dfdxhat || work == dfdx) return fail(c, MLB_EINVAL, "the workspace must not overlap the fields");
    c->st = pick(c, stream);
    CHK(filter_table(c, rmin));
    launch_filter_chain(c->lv[0].g, c->fw_n, c->fw, eta, beta, ncols, xtilde, dfdx, work, dfdxhat, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_coarse_modes_dev(mlb_ctx* c, int k, double* Psi, void* stream) {
    if (!c || !Psi || k < 1) return MLB_EINVAL;
    if (!c->has_buck || k > c->k) return fail(c, MLB_ESTATE, "no coarse modes: call mlb_buckling with at least k modes");
    c->st = pick(c, stream);
    const int64_t nl = c->lv[c->ell - 1].n;
    HIPC(hipMemcpyAsync(Psi, c->eS, sizeof(double) * nl * k, hipMemcpyDeviceToDevice, c->st));
    return MLB_OK;
}

int mlb_set_omegas(mlb_ctx* c, int nlevels, const double* omega) {
    if (!c || !omega || nlevels < 1 || nlevels > c->L - 1)
        return c ? fail(c, MLB_EINVAL, "nlevels must be in 1 .. levels - 1") : MLB_EINVAL;
    if (!c->has_density) return fail(c, MLB_ESTATE, "set the densities first");
    for (int j = 0; j < nlevels; ++j)
        if (!(omega[j] > 0.0) || !std::isfinite(omega[j])) return fail(c, MLB_EINVAL, "Jacobi weights must be positive");
    for (int j = 0; j < nlevels; ++j) c->lv[j].omega = omega[j];
    drop_graphs(c);
    return MLB_OK;
}

int mlb_get_omegas(const mlb_ctx* c, int nlevels, double* omega) {
    if (!c || !omega || nlevels < 1 || nlevels > c->L - 1) return MLB_EINVAL;
    for (int j = 0; j < nlevels; ++j) omega[j] = c->lv[j].omega;
    return MLB_OK;
}

int mlb_set_tiles(mlb_ctx* c, int wht_zchunk, int stencil_cols, int wht_variant) {
    if (!c) return MLB_EINVAL;
    if (wht_zchunk < 0 || wht_zchunk > 64 || stencil_cols < 0 || stencil_cols > 12 || wht_variant < -1 ||
        wht_variant > 3)
        return fail(c, MLB_EINVAL,
                    "tile parameters out of range (z chunk 1..64, stencil columns 1..12, variant -1..3)");
    if (wht_zchunk > 0) c->wz[0] = c->wz[1] = wht_zchunk;
    if (wht_variant >= 0) c->wv[0] = c->wv[1] = wht_variant;
    if (stencil_cols > 0) c->nb_cbmax = stencil_cols;
    drop_graphs(c);
    return MLB_OK;
}

int mlb_autotune(mlb_ctx* c, int ncols, mlb_tune_info* info, void* stream) {
    if (!c || ncols < 1 || ncols > 32) return MLB_EINVAL;
    if (!c->has_bc || !c->has_density) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    c->st = pick(c, stream);
    CHK(ensure_level_cols(c, ncols));
    drop_graphs(c);
    mlb_tune_info t{};
    if (c->d.precision == MLB_MIXED) {
        CHK(autotune_t<float>(c, ncols, true, kModeJacobi, &t.wht_zchunk, &t.wht_variant, t.wht_ms, t.wht_lds_ms,
                              t.wht_nopf_ms, t.wht_v3_ms, t.wht_score_ms));
        CHK(autotune_t<double>(c, ncols, false, kModeY, &t.wht64_zchunk, &t.wht64_variant, t.wht64_ms, t.wht64_lds_ms,
                               t.wht64_nopf_ms, t.wht64_v3_ms, t.wht64_score_ms));
    } else {
        CHK(autotune_t<double>(c, ncols, true, kModeJacobi, &t.wht_zchunk, &t.wht_variant, t.wht_ms, t.wht_lds_ms,
                               t.wht_nopf_ms, t.wht_v3_ms, t.wht_score_ms));
        t.wht64_zchunk = t.wht_zchunk;
        t.wht64_variant = t.wht_variant;
        for (int i = 0; i < 5; ++i) {
            t.wht64_ms[i] = t.wht_ms[i];
            t.wht64_lds_ms[i] = t.wht_lds_ms[i];
            t.wht64_nopf_ms[i] = t.wht_nopf_ms[i];
            t.wht64_v3_ms[i] = t.wht_v3_ms[i];
        }
        for (int i = 0; i < 20; ++i) t.wht64_score_ms[i] = t.wht_score_ms[i];
    }
    t.stencil_cols = c->nb_cbmax;
    for (int i = 0; i < 5; ++i) t.stencil_ms[i] = c->tune_stencil_ms[i];
    if (info) *info = t;
    drop_graphs(c);
    return MLB_OK;
}

int mlb_adjoint_rhs_dev(mlb_ctx* c, int k, double* Bout, void* stream) {
    if (!c || !Bout || k < 1) return MLB_EINVAL;
    if (!c->has_adj || k > c->k) return fail(c, MLB_ESTATE, "no adjoints: call mlb_sensitivities with dlam first");
    c->st = pick(c, stream);
    HIPC(hipMemcpyAsync(Bout, c->X2, sizeof(double) * c->n * k, hipMemcpyDeviceToDevice, c->st));
    return MLB_OK;
}

int mlb_solve_block_dev(mlb_ctx* c, int ncols, const double* B, double* X, double tol, int max_it,
                        mlb_solve_info* info, void* stream) {
    if (!c || !B || !X || ncols < 1) return MLB_EINVAL;
    if (ncols > 32) return fail(c, MLB_EINVAL, "at most 32 right-hand sides per block");
    if (!c->has_bc || !c->has_density) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    if (!(tol > 0) || max_it < 1) return fail(c, MLB_EINVAL, "need tol > 0 and max_it >= 1");
    c->st = pick(c, stream);
    CHK(ensure_cg(c, ncols));
    // the solvers keep every vector zero at Dirichlet DOFs: mask a copy of B
    HIPC(hipMemcpyAsync(c->X1, B, sizeof(double) * c->n * ncols, hipMemcpyDeviceToDevice, c->st));
    launch_mask_fixed(c->n, ncols, c->n, c->lv[0].nmask, c->dim, c->X1, c->st);
    c->has_adj = false;   // X1/X2 are shared work space
    if (c->o.block_cg || ncols == 1) CHK(ncols == 1 ? pcg(c, c->X1, X, 1, tol, max_it, false, info)
                                                    : bpcg(c, c->X1, X, ncols, tol, max_it, false, info));
    else CHK(pcg(c, c->X1, X, ncols, tol, max_it, false, info));
    CHK(sync(c));
    return MLB_OK;
}

int mlb_adjoints_dev(mlb_ctx* c, int k, double* Z, void* stream) {
    if (!c || !Z || k < 1) return MLB_EINVAL;
    if (!c->has_adj || k > c->k) return fail(c, MLB_ESTATE, "no adjoints: call mlb_sensitivities with dlam first");
    c->st = pick(c, stream);
    HIPC(hipMemcpyAsync(Z, c->Zadj, sizeof(double) * c->n * k, hipMemcpyDeviceToDevice, c->st));
    return MLB_OK;
}

// Copies a warm start into the context's device buffers (host or device
// source; `stream` only for a device source).
static int set_warm_common(mlb_ctx* c, int kind, int ncols, const double* data, bool dev, void* stream) {
    if (kind == MLB_WARM_NONE) {
        dfree(c->warm_coarse);
        dfree(c->warm_static);
        c->warm_coarse_cols = c->warm_static_cols = 0;
        c->warm_coarse_cap = c->warm_static_cap = 0;
        return MLB_OK;
    }
    if (!data || ncols < 1) return fail(c, MLB_EINVAL, "warm start needs data and ncols >= 1");
    double** dst = nullptr;
    size_t* cap = nullptr;
    int64_t rows = 0;
    if (kind == MLB_WARM_COARSE) {
        if (ncols > 64) return fail(c, MLB_EINVAL, "at most 64 coarse warm-start columns");
        dst = &c->warm_coarse;
        cap = &c->warm_coarse_cap;
        rows = c->lv[c->ell - 1].n;
        c->warm_coarse_cols = 0;
    } else if (kind == MLB_WARM_STATIC) {
        if (ncols > 32) return fail(c, MLB_EINVAL, "at most 32 static warm-start columns");
        dst = &c->warm_static;
        cap = &c->warm_static_cap;
        rows = c->n;
        c->warm_static_cols = 0;
    } else {
        return fail(c, MLB_EINVAL, "unknown warm-start kind");
    }
    // the buffer is kept between calls (a design loop sets one every step)
    if (!*dst || *cap < (size_t)rows * ncols) {
        *cap = 0;
        CHK(dalloc(c, dst, (size_t)rows * ncols));
        *cap = (size_t)rows * ncols;
    }
    const size_t bytes = sizeof(double) * (size_t)rows * ncols;
    if (dev) {
        c->st = pick(c, stream);
        HIPC(hipMemcpyAsync(*dst, data, bytes, hipMemcpyDeviceToDevice, c->st));
    } else {
        HIPC(hipMemcpy(*dst, data, bytes, hipMemcpyHostToDevice));
    }
    if (kind == MLB_WARM_COARSE) c->warm_coarse_cols = ncols;
    else c->warm_static_cols = ncols;
    return MLB_OK;
}

int mlb_set_warm_start(mlb_ctx* c, int kind, int ncols, const double* data) {
    if (!c) return MLB_EINVAL;
    return set_warm_common(c, kind, ncols, data, false, nullptr);
}

int mlb_set_warm_start_dev(mlb_ctx* c, int kind, int ncols, const double* data, void* stream) {
    if (!c) return MLB_EINVAL;
    return set_warm_common(c, kind, ncols, data, true, stream);
}

// ---- kernel-level entry points

int mlb_apply_K_dev(mlb_ctx* c, int level, int ncols, const double* x, double* y, void* stream) {
    if (!c || !x || !y || ncols < 1) return MLB_EINVAL;
    if (level < 1 || level > c->L) return fail(c, MLB_EINVAL, "level out of range");
    if (!c->has_density || !c->has_bc) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    c->st = pick(c, stream);
    apply_K<double>(c, level, ncols, x, y, kModeY, nullptr, nullptr, false);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_apply_G_dev(mlb_ctx* c, int level, int ncols, const double* x, double* y, void* stream) {
    if (!c || !x || !y || ncols < 1) return MLB_EINVAL;
    if (level == 1) {
        if (!c->has_stress) return fail(c, MLB_ESTATE, "no stress state: call mlb_set_state_dev or mlb_buckling");
    } else if (level != c->ell || !c->has_buck) {
        return fail(c, MLB_ESTATE, "coarse G exists only at the eigen level after mlb_buckling");
    }
    c->st = pick(c, stream);
    apply_G(c, level, ncols, x, y);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_set_state_dev(mlb_ctx* c, const double* u, double* stress_out, void* stream) {
    if (!c || !u) return MLB_EINVAL;
    if (!c->has_density) return fail(c, MLB_ESTATE, "set the densities first");
    c->st = pick(c, stream);
    launch_stress(c->dim, c->lv[0].g, c->Es, u, c->dD0Bc, c->S, c->st);
    if (stress_out)
        HIPC(hipMemcpyAsync(stress_out, c->S, sizeof(double) * c->m * c->nv, hipMemcpyDeviceToDevice, c->st));
    c->has_stress = true;
    c->has_buck = false;
    c->has_adj = false;
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_prolong_dev(mlb_ctx* c, int level, int ncols, const double* xc, double* yf, void* stream) {
    if (!c || !xc || !yf || ncols < 1) return MLB_EINVAL;
    if (level < 1 || level >= c->L) return fail(c, MLB_EINVAL, "level out of range");
    if (!c->has_bc) return fail(c, MLB_ESTATE, "set the mask first");
    c->st = pick(c, stream);
    Level& lf = c->lv[level - 1];
    Level& lc = c->lv[level];
    launch_prolong_nb<double>(c->dim, lf.g, lc.g, lf.nmask, lc.nmask, ncols, lf.n, lc.n, xc, yf, false, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_restrict_dev(mlb_ctx* c, int level, int ncols, const double* xf, double* yc, void* stream) {
    if (!c || !xf || !yc || ncols < 1) return MLB_EINVAL;
    if (level < 1 || level >= c->L) return fail(c, MLB_EINVAL, "level out of range");
    if (!c->has_bc) return fail(c, MLB_ESTATE, "set the mask first");
    c->st = pick(c, stream);
    Level& lf = c->lv[level - 1];
    Level& lc = c->lv[level];
    launch_restrict_nb<double>(c->dim, lf.g, lc.g, lf.nmask, lc.nmask, ncols, lf.n, lc.n, xf, yc, c->st);
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_sweep_dev(mlb_ctx* c, int level, int ncols, int reps, void* stream) {
    if (!c || ncols < 1 || ncols > 32 || reps < 1) return MLB_EINVAL;
    if (level < 1 || level >= c->L) return fail(c, MLB_EINVAL, "level must be a smoothed level (1 .. levels - 1)");
    if (!c->has_density || !c->has_bc) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    c->st = pick(c, stream);
    CHK(ensure_level_cols(c, ncols));
    Level& l = c->lv[level - 1];
    const size_t cnt = (size_t)l.n * ncols;
    if (c->d.precision == MLB_MIXED) {
        if (!c->sweep_ready) {   // defined contents, once per buffer set
            HIPC(hipMemsetAsync(l.fz2, 0, cnt * sizeof(float), c->st));
            HIPC(hipMemsetAsync(l.fr, 0, cnt * sizeof(float), c->st));
        }
        for (int i = 0; i < reps; ++i)
            apply_K<float>(c, level, ncols, i % 2 ? l.fz : l.fz2, i % 2 ? l.fz2 : l.fz, kModeJacobi, l.fr, nullptr);
    } else {
        if (!c->sweep_ready) {
            HIPC(hipMemsetAsync(l.vz2, 0, cnt * sizeof(double), c->st));
            HIPC(hipMemsetAsync(l.vr, 0, cnt * sizeof(double), c->st));
        }
        for (int i = 0; i < reps; ++i)
            apply_K<double>(c, level, ncols, i % 2 ? l.vz : l.vz2, i % 2 ? l.vz2 : l.vz, kModeJacobi, l.vr, nullptr);
    }
    c->sweep_ready = true;
    HIPC(hipGetLastError());
    return MLB_OK;
}

int mlb_vcycle_dev(mlb_ctx* c, int level, int ncols, const double* r, double* z, void* stream) {
    if (!c || !r || !z || ncols < 1) return MLB_EINVAL;
    if (level < 1 || level > c->L) return fail(c, MLB_EINVAL, "level out of range");
    if (!c->has_density || !c->has_bc) return fail(c, MLB_ESTATE, "set the mask and the densities first");
    c->st = pick(c, stream);
    CHK(ensure_level_cols(c, ncols));
    // the preconditioner acts on the free subspace: mask a copy of r
    Level& lv = c->lv[level - 1];
    launch_copy_cols(lv.n, ncols, lv.n, r, lv.n, lv.vt, c->st);
    launch_mask_fixed(lv.n, ncols, lv.n, lv.nmask, c->dim, lv.vt, c->st);
    if (level == 1 && c->d.precision != MLB_MIXED) {
        // vcycle<double> at level 1 uses vt as scratch: stage through the CG buffers
        CHK(ensure_cg(c, ncols));
        launch_copy_cols(lv.n, ncols, lv.n, lv.vt, lv.n, c->R, c->st);
        CHK(precondition(c, level, ncols, c->R, z));
    } else {
        launch_copy_cols(lv.n, ncols, lv.n, lv.vt, lv.n, lv.vr, c->st);
        CHK(precondition(c, level, ncols, lv.vr, z));
    }
    HIPC(hipGetLastError());
    return MLB_OK;
}

}  // extern "C"
