/*
 * mlb_nn.h - C ABI of the warm-start network kernels (the learned start
 * block of the coarse eigensolver and the initial guess of the static solve).
 *
 * Not part of the paper's method: a 3-D U-Net maps the density field on the
 * eigen-level grid to q start vectors of the coarse eigensolve (Sec. 2.1,
 * step 1) and to a static displacement guess; the solvers still converge to
 * their tolerances, so the learned start only changes iteration counts.
 *
 * Tensors are FP32, NCDHW (x fastest: index ((n*C + c)*D + z)*H*W + y*W + x),
 * device pointers owned by the caller; weights are BF16 (uint16_t bit
 * patterns) in [Co][Ci][k^3] with the k^3 taps z-major.  Every call only
 * enqueues work on `stream` (hipStream_t as void*, NULL = default stream).
 * Returns MLB_OK or MLB_EINVAL (bad sizes / unsupported kernel size).
 */
#ifndef MLB_NN_H
#define MLB_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3d(x, w) + b), zero padding, stride 1, k = 1 or 3.
   trans = 1: the data gradient of a convolution with Co input and Ci output
   channels, i.e. y (N x Co) = conv with the flipped, transposed filter of
   w ([Ci_fwd=Co][Co_fwd=Ci]); bias must then be NULL.  relu: 1 applies max(.,0). */
int mlb_nn_conv3d(int N, int Ci, int Co, int D, int H, int W, int k, int trans, const float* x,
                  const uint16_t* w, const float* bias, float* y, int relu, void* stream);
/* The forward 3x3x3 convolution of mlb_nn_conv3d (k = 3, trans = 0) on the
   matrix cores: both operands BF16 (the activations x rounded to nearest
   even as they are read, the weights w as stored), products accumulated in
   FP32 (v_mfma_f32_16x16x32_bf16 on gfx950), i.e. the same convolution of
   bf16(x).  Same layouts and arguments; bias may be NULL. */
int mlb_nn_conv3d_mfma(int N, int Ci, int Co, int D, int H, int W, const float* x, const uint16_t* w,
                       const float* bias, float* y, int relu, void* stream);
/* dw[Co][Ci][k^3] = sum over samples and voxels of dy * shifted x; db[Co] = sum dy (db may be NULL). */
int mlb_nn_conv3d_wgrad(int N, int Ci, int Co, int D, int H, int W, int k, const float* x, const float* dy,
                        float* dw, float* db, void* stream);
/* g[i] = 0 where y[i] <= 0 (ReLU backward through its output). */
int mlb_nn_relu_mask(int64_t n, const float* y, float* g, void* stream);
/* y = scale * (2x2x2 mean) of `planes` D x H x W planes (all even): scale 1
   is mean pooling, scale 8 the adjoint of nearest up-sampling. */
int mlb_nn_pool2(int64_t planes, int D, int H, int W, float scale, const float* x, float* y, void* stream);
/* y += a x */
int mlb_nn_axpy(int64_t n, float a, const float* x, float* y, void* stream);
/* gx (D x H x W) = scale * gy[parent]: scale 1/8 is the adjoint of pool2,
   scale 1 is nearest-neighbour up-sampling of gy (D/2 x H/2 x W/2). */
int mlb_nn_unpool2(int64_t planes, int D, int H, int W, float scale, const float* gy, float* gx, void* stream);
/* y = [a | b] along channels per sample; split is the inverse. */
int mlb_nn_concat(int N, int Ca, int Cb, int64_t V, const float* a, const float* b, float* y, void* stream);
int mlb_nn_split(int N, int Ca, int Cb, int64_t V, const float* y, float* a, float* b, void* stream);
/* node value = mean of the cells around the node (cells D x H x W, nodes
   (D+1)(H+1)(W+1)); node2cell_grad is its adjoint. */
int mlb_nn_cell2node(int64_t planes, int D, int H, int W, const float* cells, float* nodes, void* stream);
int mlb_nn_node2cell_grad(int64_t planes, int D, int H, int W, const float* gnodes, float* gcells, void* stream);
/* Node channels of one sample, (q + 1) vector fields of 3 components each
   (channel 3 f + c, node index fastest), to the solver's DOF blocks:
   blocks[f * 3 nodes + 3 node + c] = chan[(3 f + c) nodes + node] in FP64,
   i.e. q start vectors and one displacement, column-major, interleaved. */
int mlb_nn_nodes_to_dofs(int nfields, int64_t nodes, const float* chan, double* blocks, void* stream);
/* loss = sum w (p - t)^2 (w may be NULL = 1), grad = 2 w (p - t) * scale;
   the loss (FP64) is written to loss_dev[0]; work needs mlb_nn_mse_work(n) doubles. */
int64_t mlb_nn_mse_work(int64_t n);
int mlb_nn_mse(int64_t n, const float* pred, const float* target, const float* weight, float scale, float* grad,
               double* work, double* loss_dev, void* stream);
/* Adam step `step` (1-based) on FP32 master weights w with moments m, v;
   wb (may be NULL) receives the BF16 rounding of the updated weights. */
int mlb_nn_adam(int64_t n, float lr, float beta1, float beta2, float eps, int step, float* w, uint16_t* wb,
                const float* g, float* m, float* v, void* stream);
/* b = BF16 rounding (nearest even) of a. */
int mlb_nn_to_bf16(int64_t n, const float* a, uint16_t* b, void* stream);

#ifdef __cplusplus
}
#endif
#endif
