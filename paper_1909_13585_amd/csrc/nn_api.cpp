// C ABI of the warm-start network kernels (include/mlb_nn.h).
#include <hip/hip_runtime.h>

#include "../../include/mlb.h"
#include "../../include/mlb_nn.h"
#include "kernels.h"

using namespace mlb;

namespace {
hipStream_t S(void* s) { return (hipStream_t)s; }
bool dims_ok(int64_t a, int64_t b = 1, int64_t c = 1, int64_t d = 1) { return a > 0 && b > 0 && c > 0 && d > 0; }
int last() { return hipGetLastError() == hipSuccess ? MLB_OK : MLB_EDEVICE; }
}  // namespace

extern "C" {

int mlb_nn_conv3d(int N, int Ci, int Co, int D, int H, int W, int k, int trans, const float* x, const uint16_t* w,
                  const float* bias, float* y, int relu, void* stream) {
    if (!dims_ok(N, Ci, Co) || !dims_ok(D, H, W) || !x || !w || !y || (trans && bias)) return MLB_EINVAL;
    if (launch_nn_conv3d(N, Ci, Co, D, H, W, k, trans, x, w, bias, y, relu, S(stream)) != 0) return MLB_EINVAL;
    return last();
}

int mlb_nn_conv3d_mfma(int N, int Ci, int Co, int D, int H, int W, const float* x, const uint16_t* w,
                       const float* bias, float* y, int relu, void* stream) {
    if (!dims_ok(N, Ci, Co) || !dims_ok(D, H, W) || !x || !w || !y) return MLB_EINVAL;
    if ((int64_t)Ci * 27 > (1 << 30)) return MLB_EINVAL;
    launch_nn_conv3d_mfma(N, Ci, Co, D, H, W, x, w, bias, y, relu, S(stream));
    return last();
}

int mlb_nn_conv3d_wgrad(int N, int Ci, int Co, int D, int H, int W, int k, const float* x, const float* dy, float* dw,
                        float* db, void* stream) {
    if (!dims_ok(N, Ci, Co) || !dims_ok(D, H, W) || !x || !dy || !dw) return MLB_EINVAL;
    if (launch_nn_conv3d_wgrad(N, Ci, Co, D, H, W, k, x, dy, dw, db, S(stream)) != 0) return MLB_EINVAL;
    return last();
}

int mlb_nn_relu_mask(int64_t n, const float* y, float* g, void* stream) {
    if (n < 1 || !y || !g) return MLB_EINVAL;
    launch_nn_relu_mask(n, y, g, S(stream));
    return last();
}

int mlb_nn_pool2(int64_t planes, int D, int H, int W, float scale, const float* x, float* y, void* stream) {
    if (!dims_ok(planes, D, H, W) || (D | H | W) & 1 || !x || !y) return MLB_EINVAL;
    launch_nn_pool2(planes, D, H, W, scale, x, y, S(stream));
    return last();
}

int mlb_nn_axpy(int64_t n, float a, const float* x, float* y, void* stream) {
    if (n < 1 || !x || !y) return MLB_EINVAL;
    launch_nn_axpy(n, a, x, y, S(stream));
    return last();
}

int mlb_nn_unpool2(int64_t planes, int D, int H, int W, float scale, const float* gy, float* gx, void* stream) {
    if (!dims_ok(planes, D, H, W) || (D | H | W) & 1 || !gy || !gx) return MLB_EINVAL;
    launch_nn_unpool2(planes, D, H, W, scale, gy, gx, S(stream));
    return last();
}

int mlb_nn_concat(int N, int Ca, int Cb, int64_t V, const float* a, const float* b, float* y, void* stream) {
    if (!dims_ok(N, Ca, Cb, V) || !a || !b || !y) return MLB_EINVAL;
    launch_nn_concat(N, Ca, Cb, V, a, b, y, S(stream));
    return last();
}

int mlb_nn_split(int N, int Ca, int Cb, int64_t V, const float* y, float* a, float* b, void* stream) {
    if (!dims_ok(N, Ca, Cb, V) || !a || !b || !y) return MLB_EINVAL;
    launch_nn_split(N, Ca, Cb, V, y, a, b, S(stream));
    return last();
}

int mlb_nn_cell2node(int64_t planes, int D, int H, int W, const float* cells, float* nodes, void* stream) {
    if (!dims_ok(planes, D, H, W) || !cells || !nodes) return MLB_EINVAL;
    launch_nn_cell2node(planes, D, H, W, cells, nodes, S(stream));
    return last();
}

int mlb_nn_node2cell_grad(int64_t planes, int D, int H, int W, const float* gnodes, float* gcells, void* stream) {
    if (!dims_ok(planes, D, H, W) || !gnodes || !gcells) return MLB_EINVAL;
    launch_nn_node2cell_grad(planes, D, H, W, gnodes, gcells, S(stream));
    return last();
}

int mlb_nn_nodes_to_dofs(int nfields, int64_t nodes, const float* chan, double* blocks, void* stream) {
    if (nfields < 1 || nodes < 1 || !chan || !blocks) return MLB_EINVAL;
    launch_nn_nodes_to_dofs(nfields, nodes, chan, blocks, S(stream));
    return last();
}

int64_t mlb_nn_mse_work(int64_t n) { return n < 1 ? 0 : nn_mse_parts(n); }

int mlb_nn_mse(int64_t n, const float* pred, const float* target, const float* weight, float scale, float* grad,
               double* work, double* loss_dev, void* stream) {
    if (n < 1 || !pred || !target || !grad || !work || !loss_dev) return MLB_EINVAL;
    const int np = nn_mse_parts(n);
    launch_nn_mse(n, pred, target, weight, scale, grad, np, work, S(stream));
    launch_sum_parts(1, np, work, loss_dev, S(stream));
    return last();
}

int mlb_nn_adam(int64_t n, float lr, float beta1, float beta2, float eps, int step, float* w, uint16_t* wb,
                const float* g, float* m, float* v, void* stream) {
    if (n < 1 || step < 1 || !w || !g || !m || !v) return MLB_EINVAL;
    launch_nn_adam(n, lr, beta1, beta2, eps, step, w, wb, g, m, v, S(stream));
    return last();
}

int mlb_nn_to_bf16(int64_t n, const float* a, uint16_t* b, void* stream) {
    if (n < 1 || !a || !b) return MLB_EINVAL;
    launch_nn_to_bf16(n, a, b, S(stream));
    return last();
}

}  // extern "C"
