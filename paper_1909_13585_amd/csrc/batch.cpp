// Host runtime of the batched 2D instances (mlb_batch.h): many independent
// static analyses (Alg. 1, the solve K[x] u = f; compliance and its
// gradient, Sec. 3) advanced together, one kernel launch per solver step.
//
// Every instance has its own multigrid hierarchy (the same construction as
// the single-problem context: Galerkin element matrices summed to node-block
// stencils, damped Jacobi with omega from a power iteration, a dense coarsest
// inverse) and its own CG scalars.  All (instance, level) pairs are
// "segments" of one level space; every launch drains the work list of the
// segments it concerns (see kernels_batch.hip), so one CG iteration of the
// whole batch is a fixed sequence of about 8 + 7 (levels - 1) launches,
// captured once as a HIP graph.  Per-instance convergence is decided on the
// device (an instance whose residual meets its tolerance is marked inactive
// and its items are skipped); the host reads the flags every few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mlb_batch.h"
#include "batch_kernels.h"
#include "kernels.h"
#include "tables.h"

using namespace mlb;

namespace {

constexpr int kSlots = 64;          // queue counter slots (one per launch of an iteration, cycled)
constexpr int kMaxBlocks = 2048;    // persistent grid cap (256 CUs x 8 blocks)
constexpr int kMaxInst = 64;
constexpr int kMaxCoarse = 1024;    // DOFs of a coarsest level (dense inverse)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct List {
    int off = 0, n = 0;
};

}  // namespace

struct mlb_batch {
    mlb_batch_desc d{};
    mlb_batch_opts o{};
    std::string err;
    int ninst = 0, Lmax = 0;
    std::vector<int> L;                      // levels per instance
    std::vector<BSeg> seg;                   // host copy of the segment table
    std::vector<std::vector<int>> seg_of;    // [instance][level - 1] -> segment
    std::vector<int64_t> keoff;              // per segment: element-matrix offset (levels >= 2)
    std::vector<int64_t> dof_off, elem_off;
    int64_t nf = 0, mf = 0, nv = 0, nodes = 0, sten = 0, ke = 0, ainv = 0;
    hipStream_t own = nullptr, st = nullptr, cap = nullptr;
    Tables tab{};
    BK0<double> K0d{};
    BK0<float> K0f{};
    double *dK0 = nullptr, *dMc = nullptr, *dT = nullptr;
    // work lists
    std::vector<BItem> items;
    List LF, LE, LC, LP;
    std::vector<List> LS, LR;                // per level j (index j - 1): smoothing items at j, restriction items at j + 1
    std::vector<int> ib, ie, pb, pe, cs;     // instance ranges in LF, segment ranges in LP, coarsest segments
    BSeg* dseg = nullptr;
    BItem* ditems = nullptr;
    int *dib = nullptr, *die = nullptr, *dpb = nullptr, *dpe = nullptr, *dcs = nullptr;
    unsigned* ctr = nullptr;
    int slot = 0;
    // problem data
    uint8_t* nmask = nullptr;                // node masks of every segment
    uint8_t* fixed = nullptr;                // batched fine DOF mask
    double *x = nullptr, *Ek = nullptr, *Es = nullptr, *F = nullptr;
    float* Ekf = nullptr;
    double* Ke = nullptr;
    double* A = nullptr;
    float* Af = nullptr;
    double* dinv = nullptr;
    float* dinvf = nullptr;
    double* om = nullptr;
    float* omf = nullptr;
    double* Ainv = nullptr;
    // V-cycle work (level space) in the preconditioner's precision, power iteration pair
    double *vr = nullptr, *vz = nullptr, *vz2 = nullptr, *vt = nullptr;
    float *fr = nullptr, *fz = nullptr, *fz2 = nullptr, *ft = nullptr;
    double *pw0 = nullptr, *pw1 = nullptr;
    // CG (batched fine layout) and per-instance scalars
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *Z = nullptr;
    double *Xacc = nullptr, *Xlo = nullptr, *Rc = nullptr;   // refined solution (hi, lo), compensated residual
    int* dskip = nullptr;                    // per instance: refinement done
    std::vector<double> res_h, floor_h, res_dd_h;   // per instance, last solve: residuals of the returned u and
                                                    // of the double-double solution, FP64 floor
    double *part = nullptr, *part2 = nullptr, *part3 = nullptr;
    double *ff = nullptr, *thr = nullptr, *rr = nullptr, *rz = nullptr, *beta = nullptr;
    int *active = nullptr, *iters = nullptr, *flags = nullptr;
    int* hpin = nullptr;                     // pinned: active + flags + iters
    double* hpart = nullptr;                 // pinned: partials
    bool has_problem = false, has_solution = false;
    hipGraphExec_t graph = nullptr;
    double setup_s = 0.0;
};

namespace {

int fail(mlb_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

#define HIPC(call)                                                                            \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(b, MLB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define CHK(expr)                    \
    do {                             \
        int r_ = (expr);             \
        if (r_ != MLB_OK) return r_; \
    } while (0)

template <typename T>
int balloc(mlb_batch* b, T** p, size_t count) {
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return fail(b, MLB_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return MLB_OK;
}

template <typename T>
void bfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_graph(mlb_batch* b) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

Geo geo_of(const BSeg& s) {
    const int ne[2] = {s.nx, s.ny};
    return make_geo(2, ne);
}

// the next queue of a launch: list + a fresh counter slot
BQueue queue(mlb_batch* b, const List& l) {
    BQueue q;
    q.items = b->ditems + l.off;
    q.nitems = l.n;
    q.ctr = b->ctr + (size_t)kBCtr * (b->slot++ % kSlots);
    q.persistent = b->o.queue;
    return q;
}

int blocks(mlb_batch* b, const BQueue& q) {
    (void)b;
    return bq_grid(q, kMaxBlocks);
}

template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static const double* E(mlb_batch* b) { return b->Ek; }
    static const BK0<double>& K0(mlb_batch* b) { return b->K0d; }
    static const double* A(mlb_batch* b) { return b->A; }
    static const double* dinv(mlb_batch* b) { return b->dinv; }
    static const double* om(mlb_batch* b) { return b->om; }
    static double* buf(mlb_batch* b, int w) { return w == 0 ? b->vr : w == 1 ? b->vz : w == 2 ? b->vz2 : b->vt; }
};
template <>
struct Prec<float> {
    static const float* E(mlb_batch* b) { return b->Ekf; }
    static const BK0<float>& K0(mlb_batch* b) { return b->K0f; }
    static const float* A(mlb_batch* b) { return b->Af; }
    static const float* dinv(mlb_batch* b) { return b->dinvf; }
    static const float* om(mlb_batch* b) { return b->omf; }
    static float* buf(mlb_batch* b, int w) { return w == 0 ? b->fr : w == 1 ? b->fz : w == 2 ? b->fz2 : b->ft; }
};

// One smoothing-type launch at level j: y = op(x) with the residual source
// r1 (FP64 CG residual) at level 1 and rc (level space) below.
template <typename T>
void level_apply(mlb_batch* b, int j, int mode, const T* x, T* y, const double* r1, const T* rc) {
    using P = Prec<T>;
    const BQueue q = queue(b, b->LS[j - 1]);
    const int nb = blocks(b, q);
    if (j == 1)
        launch_bq_apply<T, double>(q, nb, mode, 0, b->dseg, b->active, P::E(b), P::K0(b), P::A(b), P::dinv(b),
                                   P::om(b), b->nmask, x, y, r1, nullptr, nullptr, b->st);
    else
        launch_bq_apply<T, T>(q, nb, mode, 0, b->dseg, b->active, P::E(b), P::K0(b), P::A(b), P::dinv(b), P::om(b),
                              b->nmask, x, y, rc, nullptr, nullptr, b->st);
}

// Z = M^-1 R for every active instance: one V(nu,nu)-cycle, all instances
// level by level (down to each instance's own coarsest level, dense solves of
// all coarsest levels in one launch, back up), then the FP64 copy of z and
// the partial sums of r.z.  The sweep count after the first is odd, so every
// level's correction ends in buffer 1 (same schedule as the single-problem
// V-cycle).
template <typename T>
void precondition(mlb_batch* b) {
    using P = Prec<T>;
    T* Rl = P::buf(b, 0);
    T* Zl = P::buf(b, 1);
    T* Z2 = P::buf(b, 2);
    T* Tt = P::buf(b, 3);
    const int nu = std::max(1, b->o.smooth_steps);
    std::vector<T*> ca(b->Lmax + 1), cb(b->Lmax + 1);
    for (int j = 1; j < b->Lmax; ++j) {
        T* a = Z2;
        T* c = Zl;
        level_apply<T>(b, j, kBJac0, a, a, b->R, Rl);
        for (int s = 1; s < nu; ++s) {
            level_apply<T>(b, j, kBJac, a, c, b->R, Rl);
            std::swap(a, c);
        }
        level_apply<T>(b, j, kBRes, a, Tt, b->R, Rl);
        const BQueue q = queue(b, b->LR[j - 1]);
        launch_bq_restrict<T>(q, blocks(b, q), b->dseg, b->active, b->nmask, Tt, Rl, b->st);
        ca[j] = a;
        cb[j] = c;
    }
    {
        const BQueue q = queue(b, b->LC);
        launch_bq_coarsest<T>(q, blocks(b, q), b->dseg, b->active, b->Ainv, Rl, Zl, b->st);
    }
    for (int j = b->Lmax - 1; j >= 1; --j) {
        T* a = ca[j];
        T* c = cb[j];
        const BQueue q = queue(b, b->LS[j - 1]);
        launch_bq_prolong_add<T>(q, blocks(b, q), b->dseg, b->active, b->nmask, Zl, a, b->st);
        for (int s = 0; s < nu; ++s) {
            level_apply<T>(b, j, kBJac, a, c, b->R, Rl);
            std::swap(a, c);
        }
    }
    const BQueue q = queue(b, b->LF);
    launch_bq_finish<T>(q, blocks(b, q), b->dseg, b->active, Zl, b->R, b->Z, b->part, b->st);
}

// One CG iteration of every active instance (flexible beta with the FP32
// cycle, as in the single-problem solver).
template <typename T>
void iteration(mlb_batch* b) {
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_apply<double, double>(q, blocks(b, q), kBY, 1, b->dseg, b->active, b->Ek, b->K0d, nullptr,
                                        nullptr, nullptr, b->nmask, b->P, b->Q, nullptr, b->P, b->part, b->st);
    }
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_cg_update(q, blocks(b, q), b->dseg, b->active, b->dib, b->die, b->part, b->rz, b->P, b->Q, b->Z,
                            b->X, b->R, b->part2, b->part3, b->flags, b->st);
    }
    launch_bq_check_res(b->ninst, 0, 0.0, b->dib, b->die, b->part2, b->ff, b->thr, b->rr, b->active, b->iters,
                        b->flags, b->st);
    precondition<T>(b);
    launch_bq_check_rz(b->ninst, 0, b->d.precision == MLB_MIXED, b->dib, b->die, b->part, b->part3, b->active, b->rz,
                       b->beta, b->flags, b->st);
    const BQueue q = queue(b, b->LF);
    launch_bq_cg_dir(q, blocks(b, q), b->dseg, b->active, b->beta, 0, b->Z, b->P, b->st);
}

template <typename T>
int run_iteration(mlb_batch* b) {
    if (b->o.graphs != 1) {
        b->slot = 0;
        iteration<T>(b);
        return MLB_OK;
    }
    if (!b->graph) {
        if (!b->cap) HIPC(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        hipStream_t saved = b->st;
        b->st = b->cap;
        b->slot = 0;
        HIPC(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        iteration<T>(b);
        hipGraph_t g = nullptr;
        const hipError_t e1 = hipStreamEndCapture(b->cap, &g);
        b->st = saved;
        HIPC(e1);
        hipGraphExec_t exec = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPC(e2);
        b->graph = exec;
    }
    HIPC(hipGraphLaunch(b->graph, b->st));
    return MLB_OK;
}

// fixed-order per-instance sums of the LF partials on the host
int read_sums(mlb_batch* b, const double* dpart, std::vector<double>& out) {
    HIPC(hipMemcpyAsync(b->hpart, dpart, sizeof(double) * b->LF.n, hipMemcpyDeviceToHost, b->st));
    HIPC(hipStreamSynchronize(b->st));
    out.assign(b->ninst, 0.0);
    for (int i = 0; i < b->ninst; ++i)
        for (int k = b->ib[i]; k < b->ie[i]; ++k) out[i] += b->hpart[k];
    return MLB_OK;
}

// One batched CG solve K X = rhs from X = 0 for every instance (an
// instance with a zero right-hand side is done at once with X = 0).  On
// return the host holds the per-instance iteration counts (hit), whether any
// instance broke down (bad) and how many are still active (nact).
template <typename T>
int cg_pass(mlb_batch* b, const double* rhs, double tol, int max_it, int& it, bool& bad, int& nact) {
    const int ni = b->ninst;
    HIPC(hipMemsetAsync(b->flags, 0, sizeof(int) * ni, b->st));
    b->slot = 0;
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_cg_init(q, blocks(b, q), b->dseg, b->nmask, rhs, b->X, b->R, b->part2, b->st);
    }
    launch_bq_check_res(ni, 1, tol * tol, b->dib, b->die, b->part2, b->ff, b->thr, b->rr, b->active, b->iters,
                        b->flags, b->st);
    precondition<T>(b);
    launch_bq_check_rz(ni, 1, 0, b->dib, b->die, b->part, b->part3, b->active, b->rz, b->beta, b->flags, b->st);
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_cg_dir(q, blocks(b, q), b->dseg, b->active, b->beta, 1, b->Z, b->P, b->st);
    }
    int* hact = b->hpin;
    int* hflg = b->hpin + kMaxInst;
    const int every = std::max(1, b->o.check_every);
    it = 0;
    nact = ni;
    bad = false;
    auto poll = [&]() -> int {
        HIPC(hipMemcpyAsync(hact, b->active, sizeof(int) * ni, hipMemcpyDeviceToHost, b->st));
        HIPC(hipMemcpyAsync(hflg, b->flags, sizeof(int) * ni, hipMemcpyDeviceToHost, b->st));
        HIPC(hipStreamSynchronize(b->st));
        nact = 0;
        for (int i = 0; i < ni; ++i) {
            nact += hact[i] ? 1 : 0;
            bad = bad || hflg[i] != 0;
        }
        return MLB_OK;
    };
    CHK(poll());
    while (nact > 0 && !bad && it < max_it) {
        const int n = std::min(every, max_it - it);
        for (int k = 0; k < n; ++k) CHK(run_iteration<T>(b));
        it += n;
        CHK(poll());
    }
    int* hit = b->hpin + 2 * kMaxInst;
    HIPC(hipMemcpyAsync(hit, b->iters, sizeof(int) * ni, hipMemcpyDeviceToHost, b->st));
    HIPC(hipStreamSynchronize(b->st));
    return MLB_OK;
}

// Compensated residual r = f - K (u_hi + u_lo) into Rc (zero for instances
// flagged in skip): per instance ||r|| / ||f|| and the FP64 representation
// floor eps ||(|K||u_hi|)|| / ||f|| (free DOFs).  No FP64 vector does much
// better than its floor: rounding u to doubles alone moves the residual by
// about that much.
int true_residuals(mlb_batch* b, const std::vector<double>& ff0, const double* xlo, const int* skip,
                   std::vector<double>& rel, std::vector<double>& floor) {
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_res_dd(q, blocks(b, q), b->dseg, b->Ek, b->K0d, b->nmask, b->Xacc, xlo, skip, b->F, b->Rc, b->part,
                         b->part3, b->st);
    }
    std::vector<double> rr, aa;
    CHK(read_sums(b, b->part, rr));
    CHK(read_sums(b, b->part3, aa));
    const int ni = b->ninst;
    rel.assign(ni, 0.0);
    floor.assign(ni, 0.0);
    for (int i = 0; i < ni; ++i) {
        if (!(ff0[i] > 0.0)) continue;
        rel[i] = std::sqrt(std::max(rr[i], 0.0) / ff0[i]);
        floor[i] = 2.220446049250313e-16 * std::sqrt(std::max(aa[i], 0.0) / ff0[i]);
    }
    return MLB_OK;
}

template <typename T>
int solve_t(mlb_batch* b, double tol, int max_it, double* U, double* J, int* iters, mlb_batch_info* info) {
    const double t0 = now_s();
    const int ni = b->ninst;
    int it = 0, nact = 0;
    bool bad = false;
    CHK(cg_pass<T>(b, b->F, tol, max_it, it, bad, nact));
    const int* hit = b->hpin + 2 * kMaxInst;
    std::vector<int> its(hit, hit + ni);
    int conv = 0;   // instances whose recursive residual met tol in the first pass
    for (int i = 0; i < ni; ++i) conv += b->hpin[i] ? 0 : 1;
    int batch_its = it;
    std::vector<double> ff0(ni);
    HIPC(hipMemcpy(ff0.data(), b->ff, sizeof(double) * ni, hipMemcpyDeviceToHost));
    HIPC(hipMemcpyAsync(b->Xacc, b->X, sizeof(double) * b->nf, hipMemcpyDeviceToDevice, b->st));
    HIPC(hipMemsetAsync(b->Xlo, 0, sizeof(double) * b->nf, b->st));
    // iterative refinement of a double-double solution u_hi + u_lo: its
    // residual in double-double, a correction solve to 1e-4 relative, u += d
    // in double-double.  An instance is done once its residual is below
    // tol / 100 (its correction right-hand side is then zero, so it costs no
    // iterations); the steps stop when all are done or none above that gains
    // 10 % in a step.
    const double target = 1e-2 * tol;
    std::vector<double> rel, floor;
    CHK(true_residuals(b, ff0, b->Xlo, nullptr, rel, floor));
    std::vector<int> skip(ni, 0);
    int done_steps = 0;
    for (int sidx = 0; sidx < b->o.refine_steps && !bad && nact == 0; ++sidx) {
        bool any = false;
        for (int i = 0; i < ni; ++i) {
            skip[i] = rel[i] <= target ? 1 : 0;
            any = any || !skip[i];
        }
        if (!any) break;
        HIPC(hipMemcpyAsync(b->dskip, skip.data(), sizeof(int) * ni, hipMemcpyHostToDevice, b->st));
        std::vector<double> relr, floorr;
        CHK(true_residuals(b, ff0, b->Xlo, b->dskip, relr, floorr));   // correction right-hand sides
        int itc = 0, nactc = 0;
        CHK(cg_pass<T>(b, b->Rc, std::max(tol, 1e-4), max_it, itc, bad, nactc));
        if (bad) break;
        batch_its += itc;
        for (int i = 0; i < ni; ++i) its[i] += hit[i];
        launch_dd_add(b->nf, b->X, b->Xacc, b->Xlo, b->st);
        HIPC(hipGetLastError());
        std::vector<double> rel2, floor2;
        CHK(true_residuals(b, ff0, b->Xlo, nullptr, rel2, floor2));
        ++done_steps;
        bool gained = false;
        double w0 = 0.0, w1 = 0.0;
        for (int i = 0; i < ni; ++i) {
            gained = gained || (rel[i] > target && rel2[i] < 0.9 * rel[i]);
            w0 = std::max(w0, rel[i]);
            w1 = std::max(w1, rel2[i]);
        }
        if (std::getenv("MLB_VERBOSE"))
            std::fprintf(stderr, "refinement step %d: %d iterations, worst residual %.3e -> %.3e\n", done_steps, itc,
                         w0, w1);
        rel.swap(rel2);
        if (!gained) break;
    }
    // the returned FP64 solution is u_hi = fl(u_hi + u_lo); its own residual
    std::vector<double> rel_dd = rel;
    CHK(true_residuals(b, ff0, nullptr, nullptr, rel, floor));
    HIPC(hipMemcpyAsync(b->X, b->Xacc, sizeof(double) * b->nf, hipMemcpyDeviceToDevice, b->st));
    // compliances f^T u
    std::vector<double> fu;
    {
        const BQueue q = queue(b, b->LF);
        launch_bq_dot(q, blocks(b, q), b->dseg, b->nmask, b->F, b->X, b->part, b->st);
    }
    CHK(read_sums(b, b->part, fu));
    if (U) HIPC(hipMemcpyAsync(U, b->X, sizeof(double) * b->nf, hipMemcpyDeviceToDevice, b->st));
    HIPC(hipStreamSynchronize(b->st));
    b->res_h = rel;
    b->floor_h = floor;
    b->res_dd_h = rel_dd;
    double worst = 0.0, worst_floor = 0.0, worst_dd = 0.0;
    int mx = 0, tot = 0, misses = 0;
    for (int i = 0; i < ni; ++i) {
        worst = std::max(worst, rel[i]);
        worst_dd = std::max(worst_dd, rel_dd[i]);
        if (rel[i] > tol) {
            ++misses;
            worst_floor = std::max(worst_floor, floor[i]);
        }
        mx = std::max(mx, its[i]);
        tot += its[i];
        if (J) J[i] = fu[i];
        if (iters) iters[i] = its[i];
    }
    if (info) {
        info->max_iterations = mx;
        info->total_iterations = tot;
        info->batch_iterations = batch_its;
        info->converged = bad ? 0 : conv;
        info->worst_true_rel_res = worst;
        info->setup_s = b->setup_s;
        info->solve_s = now_s() - t0;
        info->refine_steps = done_steps;
        info->misses = misses;
        info->worst_floor = worst_floor;
        info->worst_refined_rel_res = worst_dd;
    }
    b->has_solution = true;
    if (bad) {
        const int* hflg = b->hpin + kMaxInst;
        for (int i = 0; i < ni; ++i)
            if (hflg[i]) return fail(b, MLB_EBREAKDOWN, "instance " + std::to_string(i) + ": CG breakdown (flags " +
                                                            std::to_string(hflg[i]) + ")");
    }
    if (nact > 0) return fail(b, MLB_ENOTCONV, std::to_string(nact) + " instances did not converge in " +
                                                   std::to_string(max_it) + " iterations");
    return MLB_OK;
}

// rho(D^-1 A_j) for every non-coarsest segment by 12 power iterations run on
// all of them at once, then omega_j = jacobi_omega / (1.05 rho).
int estimate_omegas(mlb_batch* b) {
    const BQueue q0 = queue(b, b->LP);
    double* v = b->pw0;
    double* w = b->pw1;
    launch_bq_random(q0, blocks(b, q0), b->dseg, b->nmask, 0x5eedull, v, b->part, b->st);
    {
        const BQueue q = queue(b, b->LP);
        launch_bq_normalize(q, blocks(b, q), b->dseg, b->dpb, b->dpe, b->part, v, b->st);
    }
    for (int it = 0; it < 12; ++it) {
        const BQueue q = queue(b, b->LP);
        launch_bq_apply<double, double>(q, blocks(b, q), kBDinvY, 2, b->dseg, nullptr, b->Ek, b->K0d, b->A, b->dinv,
                                        nullptr, b->nmask, v, w, nullptr, nullptr, b->part, b->st);
        const BQueue q2 = queue(b, b->LP);
        launch_bq_normalize(q2, blocks(b, q2), b->dseg, b->dpb, b->dpe, b->part, w, b->st);
        std::swap(v, w);
    }
    HIPC(hipMemcpyAsync(b->hpart, b->part, sizeof(double) * b->LP.n, hipMemcpyDeviceToHost, b->st));
    HIPC(hipStreamSynchronize(b->st));
    std::vector<double> omh(b->seg.size(), 1.0);
    std::vector<float> omfh(b->seg.size(), 1.0f);
    for (size_t s = 0; s < b->seg.size(); ++s) {
        if (b->seg[s].child < 0) continue;
        double sum = 0.0;
        for (int k = b->pb[s]; k < b->pe[s]; ++k) sum += b->hpart[k];
        const double rho = std::sqrt(std::max(sum, 0.0));
        if (!(rho > 0.0) || !std::isfinite(rho))
            return fail(b, MLB_EINVAL, "Jacobi spectral radius estimate failed (instance " +
                                           std::to_string(b->seg[s].inst) + ")");
        omh[s] = b->o.jacobi_omega / (1.05 * rho);
        omfh[s] = (float)omh[s];
    }
    HIPC(hipMemcpy(b->om, omh.data(), sizeof(double) * omh.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->omf, omfh.data(), sizeof(float) * omfh.size(), hipMemcpyHostToDevice));
    return MLB_OK;
}

// Per-problem setup: SIMP moduli, masks, Galerkin hierarchy and stencils of
// every instance, Jacobi weights, coarsest inverses.
int build(mlb_batch* b) {
    drop_graph(b);
    hipStream_t st = b->st;
    const double t0 = now_s();
    // moduli of all instances in one launch; count densities outside [0, 1]
    const int np = std::min<int64_t>(1024, std::max<int64_t>(1, (b->mf + 255) / 256));
    launch_material(b->mf, b->x, b->d.E1, b->d.E0, b->d.penal, b->Ek, b->Ekf, b->Es, np, b->part, st);
    HIPC(hipMemcpyAsync(b->hpart, b->part, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    // node masks: fine from the DOF mask, coarse from the coincident fine node
    for (int i = 0; i < b->ninst; ++i) {
        const BSeg& s1 = b->seg[b->seg_of[i][0]];
        launch_node_mask((int64_t)s1.nnx * s1.nny, 2, b->fixed + b->dof_off[i], b->nmask + s1.noff, st);
        for (int j = 1; j < b->L[i]; ++j) {
            const BSeg& sf = b->seg[b->seg_of[i][j - 1]];
            const BSeg& sc = b->seg[b->seg_of[i][j]];
            launch_coarse_mask(geo_of(sf), geo_of(sc), b->nmask + sf.noff, b->nmask + sc.noff, st);
        }
    }
    HIPC(hipStreamSynchronize(st));
    double nbad = 0.0;
    for (int k = 0; k < np; ++k) nbad += b->hpart[k];
    if (nbad > 0) return fail(b, MLB_EINVAL, "densities must be finite and lie in [0, 1]");
    // hierarchy: level-1 Jacobi diagonal, Galerkin element matrices, stencils
    HIPC(hipMemsetAsync(b->Ainv, 0, sizeof(double) * b->ainv, st));
    for (int i = 0; i < b->ninst; ++i) {
        const BSeg& s1 = b->seg[b->seg_of[i][0]];
        launch_dinv_fine(2, geo_of(s1), b->Ek + b->elem_off[i], b->nmask + s1.noff, b->dK0, b->dinv + s1.voff,
                         b->dinvf + s1.voff, st);
        for (int j = 2; j <= b->L[i]; ++j) {
            const int si = b->seg_of[i][j - 1];
            const BSeg& sc = b->seg[si];
            const BSeg& sf = b->seg[sc.parent];
            if (j == 2) launch_galerkin_from_E(2, geo_of(sf), geo_of(sc), b->Ek + b->elem_off[i], b->dMc,
                                               b->Ke + b->keoff[si], st);
            else launch_galerkin_dense(2, false, geo_of(sf), geo_of(sc), b->Ke + b->keoff[sc.parent], b->dT,
                                       b->Ke + b->keoff[si], st);
            if (j < b->L[i])
                launch_assemble_nb(2, geo_of(sc), b->Ke + b->keoff[si], b->nmask + sc.noff, b->A + sc.soff,
                                   b->Af + sc.soff, b->dinv + sc.voff, b->dinvf + sc.voff, false, st);
            else
                launch_assemble_dense(2, geo_of(sc), b->Ke + b->keoff[si], b->nmask + sc.noff,
                                      2 * (int64_t)sc.nnx * sc.nny, 2 * (int64_t)sc.nnx * sc.nny,
                                      b->Ainv + sc.coff, st);
        }
    }
    launch_bq_gj((int)b->cs.size(), b->dcs, b->dseg, b->Ainv, st);
    CHK(estimate_omegas(b));
    HIPC(hipStreamSynchronize(st));
    b->setup_s = now_s() - t0;
    b->has_problem = true;
    b->has_solution = false;
    return MLB_OK;
}

hipStream_t pick(mlb_batch* b, void* stream) { return stream ? (hipStream_t)stream : b->own; }

}  // namespace

extern "C" {

int mlb_batch_create(const mlb_batch_desc* desc, mlb_batch** out) {
    if (!desc || !out) return MLB_EINVAL;
    *out = nullptr;
    mlb_batch* b = new mlb_batch();
    *out = b;   // returned even on failure so mlb_batch_last_error works; caller destroys
    b->d = *desc;
    b->o.smooth_steps = 2;
    b->o.jacobi_omega = 4.0 / 3.0;
    b->o.queue = 0;   // the hardware dispatcher beats the atomic queue for these uniform items
    b->o.graphs = 1;
    b->o.check_every = 4;
    b->o.refine_steps = 10;
    const int ni = desc->ninst;
    if (ni < 1 || ni > kMaxInst) return fail(b, MLB_EINVAL, "ninst must be in 1..64");
    if (!(desc->E1 > 0) || !(desc->E0 >= 0) || !(desc->E0 < desc->E1)) return fail(b, MLB_EINVAL, "need 0 <= E0 < E1");
    if (!(desc->nu > -1.0 && desc->nu < 0.5)) return fail(b, MLB_EINVAL, "Poisson ratio must lie in (-1, 0.5)");
    if (!(desc->penal >= 1.0)) return fail(b, MLB_EINVAL, "penalty p must be >= 1");
    if (desc->precision != MLB_FP64 && desc->precision != MLB_MIXED) return fail(b, MLB_EINVAL, "unknown precision");
    const int64_t maxc = desc->max_coarse_dofs > 0 ? desc->max_coarse_dofs : 256;
    b->ninst = ni;
    b->L.assign(ni, 1);
    for (int i = 0; i < ni; ++i) {
        int nx = desc->nel[2 * i], ny = desc->nel[2 * i + 1];
        if (nx < 2 || ny < 2 || nx % 2 || ny % 2 || nx > (1 << 20) || ny > (1 << 20))
            return fail(b, MLB_EINVAL, "instance " + std::to_string(i) + ": element counts must be even and >= 2");
        // at least one coarsening; then while even and above the threshold
        int L = 1;
        do {
            nx /= 2;
            ny /= 2;
            ++L;
        } while (nx % 2 == 0 && ny % 2 == 0 && 2LL * (nx + 1) * (ny + 1) > maxc);
        const int64_t nc = 2LL * (nx + 1) * (ny + 1);
        if (nc > kMaxCoarse)
            return fail(b, MLB_EINVAL, "instance " + std::to_string(i) + ": coarsest level has " +
                                           std::to_string(nc) + " DOFs (> 1024); element counts need more factors of 2");
        b->L[i] = L;
        b->Lmax = std::max(b->Lmax, L);
    }
    if (hipSetDevice(desc->device) != hipSuccess) return fail(b, MLB_EDEVICE, "hipSetDevice failed");
    HIPC(hipStreamCreate(&b->own));
    b->st = b->own;
    build_tables(2, desc->nu, 0, &b->tab);
    for (int k = 0; k < 64; ++k) {
        b->K0d.k[k] = b->tab.K0[k];
        b->K0f.k[k] = (float)b->tab.K0[k];
    }
    CHK(balloc(b, &b->dK0, 576));
    CHK(balloc(b, &b->dMc, 8 * 576));
    CHK(balloc(b, &b->dT, 512));
    HIPC(hipMemcpy(b->dK0, b->tab.K0, sizeof(double) * 576, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dMc, b->tab.Mc, sizeof(double) * 8 * 576, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dT, b->tab.T, sizeof(double) * 512, hipMemcpyHostToDevice));
    // segments, level-major (level-1 segments first, in instance order)
    b->seg_of.assign(ni, {});
    b->dof_off.assign(ni + 1, 0);
    b->elem_off.assign(ni + 1, 0);
    for (int i = 0; i < ni; ++i) {
        const int nx = desc->nel[2 * i], ny = desc->nel[2 * i + 1];
        b->dof_off[i + 1] = b->dof_off[i] + 2LL * (nx + 1) * (ny + 1);
        b->elem_off[i + 1] = b->elem_off[i] + (int64_t)nx * ny;
    }
    b->nf = b->dof_off[ni];
    b->mf = b->elem_off[ni];
    for (int j = 1; j <= b->Lmax; ++j)
        for (int i = 0; i < ni; ++i) {
            if (j > b->L[i]) continue;
            BSeg s{};
            s.nx = desc->nel[2 * i] >> (j - 1);
            s.ny = desc->nel[2 * i + 1] >> (j - 1);
            s.nnx = s.nx + 1;
            s.nny = s.ny + 1;
            s.inst = i;
            s.level = j;
            s.parent = j > 1 ? b->seg_of[i][j - 2] : -1;
            s.child = -1;
            s.voff = b->nv;
            s.noff = b->nodes;
            const int64_t nn = (int64_t)s.nnx * s.nny;
            b->nv += 2 * nn;
            b->nodes += nn;
            s.coff = -1;
            int64_t keo = 0;
            if (j == 1) {
                s.soff = b->elem_off[i];
            } else {
                keo = b->ke;
                b->ke += 64LL * s.nx * s.ny;
                if (j < b->L[i]) {
                    s.soff = b->sten;
                    b->sten += 36 * nn;
                } else {
                    s.soff = 0;
                }
            }
            if (j == b->L[i]) {
                s.coff = b->ainv;
                b->ainv += 4 * nn * nn;
            }
            const int id = (int)b->seg.size();
            if (s.parent >= 0) b->seg[s.parent].child = id;
            b->seg.push_back(s);
            b->keoff.push_back(keo);
            b->seg_of[i].push_back(id);
        }
    // work lists
    auto add_nodes = [&](int sid) {
        const BSeg& s = b->seg[sid];
        const int nn = s.nnx * s.nny;
        for (int f = 0; f < nn; f += kBItemNodes) b->items.push_back({sid, f});
    };
    auto begin = [&](List& l) { l.off = (int)b->items.size(); };
    auto end = [&](List& l) { l.n = (int)b->items.size() - l.off; };
    b->ib.assign(ni, 0);
    b->ie.assign(ni, 0);
    begin(b->LF);
    for (int i = 0; i < ni; ++i) {
        b->ib[i] = (int)b->items.size();
        add_nodes(b->seg_of[i][0]);
        b->ie[i] = (int)b->items.size();
    }
    end(b->LF);
    for (int i = 0; i < ni; ++i) {   // LF ranges relative to the LF partials
        b->ib[i] -= b->LF.off;
        b->ie[i] -= b->LF.off;
    }
    begin(b->LE);
    for (int i = 0; i < ni; ++i) {
        const int sid = b->seg_of[i][0];
        const BSeg& s = b->seg[sid];
        for (int e = 0; e < s.nx * s.ny; e += kBItemNodes) b->items.push_back({sid, e});
    }
    end(b->LE);
    b->LS.assign(std::max(1, b->Lmax - 1), List{});
    b->LR.assign(std::max(1, b->Lmax - 1), List{});
    for (int j = 1; j < b->Lmax; ++j) {
        begin(b->LS[j - 1]);
        for (int i = 0; i < ni; ++i)
            if (b->L[i] > j) add_nodes(b->seg_of[i][j - 1]);
        end(b->LS[j - 1]);
        begin(b->LR[j - 1]);
        for (int i = 0; i < ni; ++i)
            if (b->L[i] > j) add_nodes(b->seg_of[i][j]);
        end(b->LR[j - 1]);
    }
    begin(b->LC);
    for (int i = 0; i < ni; ++i) {
        const int sid = b->seg_of[i][b->L[i] - 1];
        const BSeg& s = b->seg[sid];
        b->cs.push_back(sid);
        for (int r = 0; r < 2 * s.nnx * s.nny; r += 4) b->items.push_back({sid, r});
    }
    end(b->LC);
    b->pb.assign(b->seg.size(), 0);
    b->pe.assign(b->seg.size(), 0);
    begin(b->LP);
    for (size_t s = 0; s < b->seg.size(); ++s) {
        if (b->seg[s].child < 0) continue;
        b->pb[s] = (int)b->items.size();
        add_nodes((int)s);
        b->pe[s] = (int)b->items.size();
    }
    end(b->LP);
    for (size_t s = 0; s < b->seg.size(); ++s) {
        b->pb[s] -= b->LP.off;
        b->pe[s] -= b->LP.off;
    }
    int maxlist = std::max({b->LF.n, b->LP.n, b->LE.n, 1024});
    // device memory
    CHK(balloc(b, &b->dseg, b->seg.size()));
    CHK(balloc(b, &b->ditems, b->items.size()));
    CHK(balloc(b, &b->dib, ni));
    CHK(balloc(b, &b->die, ni));
    CHK(balloc(b, &b->dpb, b->seg.size()));
    CHK(balloc(b, &b->dpe, b->seg.size()));
    CHK(balloc(b, &b->dcs, b->cs.size()));
    CHK(balloc(b, &b->ctr, (size_t)kSlots * kBCtr));
    HIPC(hipMemcpy(b->dseg, b->seg.data(), sizeof(BSeg) * b->seg.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->ditems, b->items.data(), sizeof(BItem) * b->items.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dib, b->ib.data(), sizeof(int) * ni, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->die, b->ie.data(), sizeof(int) * ni, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dpb, b->pb.data(), sizeof(int) * b->pb.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dpe, b->pe.data(), sizeof(int) * b->pe.size(), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(b->dcs, b->cs.data(), sizeof(int) * b->cs.size(), hipMemcpyHostToDevice));
    HIPC(hipMemset(b->ctr, 0, sizeof(unsigned) * kSlots * kBCtr));
    CHK(balloc(b, &b->nmask, b->nodes));
    CHK(balloc(b, &b->fixed, b->nf));
    CHK(balloc(b, &b->x, b->mf));
    CHK(balloc(b, &b->Ek, b->mf));
    CHK(balloc(b, &b->Ekf, b->mf));
    CHK(balloc(b, &b->Es, b->mf));
    CHK(balloc(b, &b->F, b->nf));
    CHK(balloc(b, &b->Ke, b->ke));
    CHK(balloc(b, &b->A, b->sten));
    CHK(balloc(b, &b->Af, b->sten));
    CHK(balloc(b, &b->dinv, b->nv));
    CHK(balloc(b, &b->dinvf, b->nv));
    CHK(balloc(b, &b->om, b->seg.size()));
    CHK(balloc(b, &b->omf, b->seg.size()));
    CHK(balloc(b, &b->Ainv, b->ainv));
    if (desc->precision == MLB_FP64) {
        CHK(balloc(b, &b->vr, b->nv));
        CHK(balloc(b, &b->vz, b->nv));
        CHK(balloc(b, &b->vz2, b->nv));
        CHK(balloc(b, &b->vt, b->nv));
    } else {
        CHK(balloc(b, &b->fr, b->nv));
        CHK(balloc(b, &b->fz, b->nv));
        CHK(balloc(b, &b->fz2, b->nv));
        CHK(balloc(b, &b->ft, b->nv));
    }
    CHK(balloc(b, &b->pw0, b->nv));
    CHK(balloc(b, &b->pw1, b->nv));
    CHK(balloc(b, &b->X, b->nf));
    CHK(balloc(b, &b->Xacc, b->nf));
    CHK(balloc(b, &b->Xlo, b->nf));
    CHK(balloc(b, &b->dskip, (size_t)ni));
    CHK(balloc(b, &b->Rc, b->nf));
    CHK(balloc(b, &b->R, b->nf));
    CHK(balloc(b, &b->P, b->nf));
    CHK(balloc(b, &b->Q, b->nf));
    CHK(balloc(b, &b->Z, b->nf));
    CHK(balloc(b, &b->part, maxlist));
    CHK(balloc(b, &b->part2, maxlist));
    CHK(balloc(b, &b->part3, maxlist));
    CHK(balloc(b, &b->ff, ni));
    CHK(balloc(b, &b->thr, ni));
    CHK(balloc(b, &b->rr, ni));
    CHK(balloc(b, &b->rz, ni));
    CHK(balloc(b, &b->beta, ni));
    CHK(balloc(b, &b->active, ni));
    CHK(balloc(b, &b->iters, ni));
    CHK(balloc(b, &b->flags, ni));
    HIPC(hipMemset(b->active, 0, sizeof(int) * ni));
    HIPC(hipHostMalloc((void**)&b->hpin, sizeof(int) * 3 * kMaxInst, hipHostMallocDefault));
    HIPC(hipHostMalloc((void**)&b->hpart, sizeof(double) * maxlist, hipHostMallocDefault));
    return MLB_OK;
}

void mlb_batch_destroy(mlb_batch* b) {
    if (!b) return;
    if (b->own) (void)hipStreamSynchronize(b->own);
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    bfree(b->dK0);
    bfree(b->dMc);
    bfree(b->dT);
    bfree(b->dseg);
    bfree(b->ditems);
    bfree(b->dib);
    bfree(b->die);
    bfree(b->dpb);
    bfree(b->dpe);
    bfree(b->dcs);
    bfree(b->ctr);
    bfree(b->nmask);
    bfree(b->fixed);
    bfree(b->x);
    bfree(b->Ek);
    bfree(b->Ekf);
    bfree(b->Es);
    bfree(b->F);
    bfree(b->Ke);
    bfree(b->A);
    bfree(b->Af);
    bfree(b->dinv);
    bfree(b->dinvf);
    bfree(b->om);
    bfree(b->omf);
    bfree(b->Ainv);
    bfree(b->vr);
    bfree(b->vz);
    bfree(b->vz2);
    bfree(b->vt);
    bfree(b->fr);
    bfree(b->fz);
    bfree(b->fz2);
    bfree(b->ft);
    bfree(b->pw0);
    bfree(b->pw1);
    bfree(b->X);
    bfree(b->Xacc);
    bfree(b->Xlo);
    bfree(b->dskip);
    bfree(b->Rc);
    bfree(b->R);
    bfree(b->P);
    bfree(b->Q);
    bfree(b->Z);
    bfree(b->part);
    bfree(b->part2);
    bfree(b->part3);
    bfree(b->ff);
    bfree(b->thr);
    bfree(b->rr);
    bfree(b->rz);
    bfree(b->beta);
    bfree(b->active);
    bfree(b->iters);
    bfree(b->flags);
    if (b->hpin) (void)hipHostFree(b->hpin);
    if (b->hpart) (void)hipHostFree(b->hpart);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

const char* mlb_batch_last_error(const mlb_batch* b) { return b ? b->err.c_str() : "null batch"; }

int mlb_batch_set_opts(mlb_batch* b, const mlb_batch_opts* o) {
    if (!b || !o) return MLB_EINVAL;
    if (o->smooth_steps < 1 || o->smooth_steps > 8) return fail(b, MLB_EINVAL, "smooth_steps must be in 1..8");
    if (!(o->jacobi_omega > 0.0 && o->jacobi_omega < 2.0)) return fail(b, MLB_EINVAL, "jacobi_omega must be in (0, 2)");
    if (o->queue != 0 && o->queue != 1) return fail(b, MLB_EINVAL, "queue must be 0 or 1");
    if (o->graphs != 0 && o->graphs != 1) return fail(b, MLB_EINVAL, "graphs must be 0 or 1");
    if (o->check_every < 1) return fail(b, MLB_EINVAL, "check_every must be >= 1");
    if (o->refine_steps < 0 || o->refine_steps > 16) return fail(b, MLB_EINVAL, "refine_steps must be in 0..16");
    const bool rebuild = o->jacobi_omega != b->o.jacobi_omega;
    b->o = *o;
    drop_graph(b);
    if (rebuild && b->has_problem) return build(b);
    return MLB_OK;
}

int mlb_batch_get_opts(const mlb_batch* b, mlb_batch_opts* o) {
    if (!b || !o) return MLB_EINVAL;
    *o = b->o;
    return MLB_OK;
}

int mlb_batch_layout(const mlb_batch* b, int64_t* dof_off, int64_t* elem_off, int* levels) {
    if (!b || b->seg.empty()) return MLB_EINVAL;
    for (int i = 0; i <= b->ninst; ++i) {
        if (dof_off) dof_off[i] = b->dof_off[i];
        if (elem_off) elem_off[i] = b->elem_off[i];
        if (levels && i < b->ninst) levels[i] = b->L[i];
    }
    return MLB_OK;
}

int mlb_batch_set_problem_dev(mlb_batch* b, const uint8_t* fixed, const double* F, const double* x, void* stream) {
    if (!b || !fixed || !F || !x || b->seg.empty()) return MLB_EINVAL;
    b->st = pick(b, stream);
    HIPC(hipMemcpyAsync(b->fixed, fixed, b->nf, hipMemcpyDeviceToDevice, b->st));
    HIPC(hipMemcpyAsync(b->F, F, sizeof(double) * b->nf, hipMemcpyDeviceToDevice, b->st));
    HIPC(hipMemcpyAsync(b->x, x, sizeof(double) * b->mf, hipMemcpyDeviceToDevice, b->st));
    b->has_problem = false;
    const int r = build(b);
    b->st = b->own;
    return r;
}

int mlb_batch_solve_dev(mlb_batch* b, double tol, int max_it, double* U, double* J, int* iters, mlb_batch_info* info,
                        void* stream) {
    if (!b) return MLB_EINVAL;
    if (!b->has_problem) return fail(b, MLB_ESTATE, "set the problem before solving");
    if (!(tol > 0.0 && tol < 1.0) || max_it < 1) return fail(b, MLB_EINVAL, "need 0 < tol < 1 and max_it >= 1");
    hipStream_t s = pick(b, stream);
    if (s != b->st) drop_graph(b);   // a graph is replayed on the stream it was made for
    b->st = s;
    const int r = b->d.precision == MLB_FP64 ? solve_t<double>(b, tol, max_it, U, J, iters, info)
                                             : solve_t<float>(b, tol, max_it, U, J, iters, info);
    return r;
}

int mlb_batch_residuals(const mlb_batch* b, double* res, double* floor, double* res_refined) {
    if (!b) return MLB_EINVAL;
    if (!b->has_solution) return MLB_ESTATE;
    for (int i = 0; i < b->ninst; ++i) {
        if (res) res[i] = b->res_h[i];
        if (floor) floor[i] = b->floor_h[i];
        if (res_refined) res_refined[i] = b->res_dd_h[i];
    }
    return MLB_OK;
}

int mlb_batch_compliance_sens_dev(mlb_batch* b, double* dJ, void* stream) {
    if (!b || !dJ) return MLB_EINVAL;
    if (!b->has_solution) return fail(b, MLB_ESTATE, "solve before the sensitivities");
    hipStream_t s = pick(b, stream);
    b->slot = 0;
    const BQueue q = queue(b, b->LE);
    launch_bq_dJ(q, blocks(b, q), b->dseg, b->x, b->d.penal, b->d.E1 - b->d.E0, b->K0d, b->X, dJ, s);
    HIPC(hipGetLastError());
    return MLB_OK;
}

}  // extern "C"
