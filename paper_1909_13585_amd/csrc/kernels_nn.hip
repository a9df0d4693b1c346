// Kernels of the warm-start network: a small 3-D U-Net on the eigen-level
// grid.  Activations are FP32 in NCDHW layout (x fastest), weights are BF16
// ([Co][Ci][k^3], taps z-major), every product is accumulated in FP32.
//
// The convolutions are direct: one thread per output voxel and group of 8
// output channels; the block's weights are uniform loads (scalar cache
// reads), the input taps coalesce across the 256 consecutive voxels of a
// block.  The data-gradient is the same kernel on the flipped, transposed
// filter.  The weight gradient reduces over (sample, voxel) with one block per
// (co, ci) pair and fixed-order trees, so training is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mlb {

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even
__device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int kNnThreads = 256;
constexpr int kCoGroup = 8;

// y[n, o, p] = act(b[o] + sum_i sum_t w_eff(o, i, t) x[n, i, p + off(t)])
// Forward: w_eff(o,i,t) = w[(o*Ci + i)*KK + t].
// Transposed (data gradient of a conv with Ci_f = Co, Co_f = Ci channels):
// w_eff(o,i,t) = w[(i*Co + o)*KK + KK-1-t].
template <int K, bool TRANS>
__global__ __launch_bounds__(kNnThreads) void k_conv3d(int Ci, int Co, int D, int H, int W, const float* __restrict__ x,
                                                       const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                                       float* __restrict__ y, int relu) {
    constexpr int KK = K * K * K, R = K / 2;
    const int64_t V = (int64_t)D * H * W;
    const int64_t p = blockIdx.x * (int64_t)kNnThreads + threadIdx.x;
    const int o0 = blockIdx.y * kCoGroup;
    const int n = blockIdx.z;
    const bool live = p < V;
    const int64_t pc = live ? p : 0;
    const int wx = (int)(pc % W), hy = (int)((pc / W) % H), dz = (int)(pc / ((int64_t)W * H));
    float acc[kCoGroup];
#pragma unroll
    for (int q = 0; q < kCoGroup; ++q) acc[q] = (bias && o0 + q < Co) ? bias[o0 + q] : 0.f;
    const float* xn = x + (int64_t)n * Ci * V;
    for (int i = 0; i < Ci; ++i) {
        const float* xi = xn + (int64_t)i * V;
        // taps: rows (z, y) in a runtime loop, the K taps along x unrolled,
        // which keeps the live weights to K x 8 registers
#pragma unroll 1
        for (int r2 = 0; r2 < K * K; ++r2) {
            const int oy = r2 % K - R, oz = r2 / K - R;
            const int yy = hy + oy, zz = dz + oz;
            const bool rin = yy >= 0 && yy < H && zz >= 0 && zz < D;
#pragma unroll
            for (int tx = 0; tx < K; ++tx) {
                const int t = r2 * K + tx;
                const int xx = wx + tx - R;
                const bool in = rin && xx >= 0 && xx < W;
                const int64_t at = in ? (int64_t)zz * H * W + (int64_t)yy * W + xx : 0;
                const float xv = in ? xi[at] : 0.f;
#pragma unroll
                for (int q = 0; q < kCoGroup; ++q) {
                    const int o = min(o0 + q, Co - 1);
                    const int64_t wi =
                        TRANS ? ((int64_t)i * Co + o) * KK + (KK - 1 - t) : ((int64_t)o * Ci + i) * KK + t;
                    acc[q] += xv * bf16_to_f32(w[wi]);
                }
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int q = 0; q < kCoGroup; ++q) {
        const int o = o0 + q;
        if (o >= Co) break;
        float v = acc[q];
        if (relu) v = v > 0.f ? v : 0.f;
        y[((int64_t)n * Co + o) * V + p] = v;
    }
}

// Forward 3x3x3 convolution on the matrix cores (implicit GEMM): per sample,
// Y (Co x V) = W (Co x Ci 27) X^ (Ci 27 x V) with X^ the zero-padded taps
// of x, both operands in BF16 (activations rounded to nearest even on load,
// the weights already BF16), products accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  Its operands: lane l holds row / column l % 16
// and the 8 consecutive k = 8 (l / 16) + e; its result: column l % 16, rows
// 4 (l / 16) + r.  A wave computes MT 16-channel tiles (channel group
// blockIdx.z) for 16 consecutive voxels, gathering each tap once for all
// of them; the k index runs over (input channel, tap) in the weights' order
// and is padded with zeros to a multiple of 32.
typedef __bf16 mlb_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mlb_f32x4 __attribute__((ext_vector_type(4)));

__device__ inline __bf16 mlb_bits_bf16(uint16_t h) { return __builtin_bit_cast(__bf16, h); }

template <int MT>
__global__ __launch_bounds__(kNnThreads) void k_conv3d_mfma(int Ci, int Co, int D, int H, int W,
                                                            const float* __restrict__ x,
                                                            const uint16_t* __restrict__ w,
                                                            const float* __restrict__ bias, float* __restrict__ y,
                                                            int relu) {
    const int64_t V = (int64_t)D * H * W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int n = blockIdx.y;
    const int obase = blockIdx.z * MT * 16;
    const int64_t p = ((int64_t)blockIdx.x * (kNnThreads / 64) + wv) * 16 + col;
    const bool live = p < V;
    const int64_t pc = live ? p : 0;
    const int wx = (int)(pc % W), hy = (int)((pc / W) % H), dz = (int)(pc / ((int64_t)W * H));
    const float* xn = x + (int64_t)n * Ci * V;
    const int KT = Ci * 27;
    mlb_f32x4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = mlb_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < KT; k0 += 32) {
        mlb_bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int kk = k0 + 8 * kg + e;
            float v = 0.f;
            if (live && kk < KT) {
                const int i = kk / 27, t = kk - 27 * i;
                const int zz = dz + t / 9 - 1, yy = hy + (t / 3) % 3 - 1, xx = wx + t % 3 - 1;
                if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = xn[(int64_t)i * V + ((int64_t)zz * H + yy) * W + xx];
            }
            b[e] = mlb_bits_bf16(f32_to_bf16(v));
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int o = obase + mt * 16 + col;
            mlb_bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int kk = k0 + 8 * kg + e;
                a[e] = mlb_bits_bf16((o < Co && kk < KT) ? w[(int64_t)o * KT + kk] : (uint16_t)0);
            }
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mt], 0, 0, 0);
        }
    }
    if (!live) return;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = obase + mt * 16 + 4 * kg + r;
            if (o >= Co) continue;
            float v = acc[mt][r] + (bias ? bias[o] : 0.f);
            if (relu) v = v > 0.f ? v : 0.f;
            y[((int64_t)n * Co + o) * V + p] = v;
        }
}

// dw[o, i, t] = sum_{n,p} dy[n, o, p] x[n, i, p + off(t)]  (one block per (o, i))
template <int K>
__global__ __launch_bounds__(kNnThreads) void k_conv3d_wgrad(int N, int Ci, int Co, int D, int H, int W,
                                                             const float* __restrict__ x,
                                                             const float* __restrict__ dy, float* __restrict__ dw) {
    constexpr int KK = K * K * K, R = K / 2;
    __shared__ float red[kNnThreads / 64][KK];
    const int i = blockIdx.x, o = blockIdx.y;
    const int64_t V = (int64_t)D * H * W;
    float acc[KK];
#pragma unroll
    for (int t = 0; t < KK; ++t) acc[t] = 0.f;
    for (int n = 0; n < N; ++n) {
        const float* xi = x + ((int64_t)n * Ci + i) * V;
        const float* dyo = dy + ((int64_t)n * Co + o) * V;
        for (int64_t p = threadIdx.x; p < V; p += kNnThreads) {
            const float g = dyo[p];
            const int wx = (int)(p % W), hy = (int)((p / W) % H), dz = (int)(p / ((int64_t)W * H));
#pragma unroll
            for (int t = 0; t < KK; ++t) {
                const int xx = wx + t % K - R, yy = hy + (t / K) % K - R, zz = dz + t / (K * K) - R;
                const bool in = xx >= 0 && xx < W && yy >= 0 && yy < H && zz >= 0 && zz < D;
                const int64_t at = in ? (int64_t)zz * H * W + (int64_t)yy * W + xx : 0;
                const float xv = in ? xi[at] : 0.f;
                acc[t] += g * xv;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < KK; ++t) {
        float v = acc[t];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wv][t] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < KK; t += kNnThreads) {
        float s = 0.f;
        for (int q = 0; q < kNnThreads / 64; ++q) s += red[q][t];
        dw[((int64_t)o * Ci + i) * KK + t] = s;
    }
}

// db[o] = sum_{n,p} dy[n, o, p]
__global__ __launch_bounds__(kNnThreads) void k_bias_grad(int N, int Co, int64_t V, const float* __restrict__ dy,
                                                          float* __restrict__ db) {
    __shared__ float red[kNnThreads / 64];
    const int o = blockIdx.x;
    float s = 0.f;
    for (int n = 0; n < N; ++n)
        for (int64_t p = threadIdx.x; p < V; p += kNnThreads) s += dy[((int64_t)n * Co + o) * V + p];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int q = 0; q < kNnThreads / 64; ++q) t += red[q];
        db[o] = t;
    }
}

// g *= (y > 0)
__global__ void k_relu_mask(int64_t n, const float* __restrict__ y, float* __restrict__ g) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}

// y = scale * mean over 2x2x2 children of NC planes (D, H, W even): scale 1
// is mean pooling, scale 8 the adjoint of nearest up-sampling
__global__ void k_pool2(int64_t planes, int D, int H, int W, float scale, const float* __restrict__ x,
                        float* __restrict__ y) {
    const int d2 = D / 2, h2 = H / 2, w2 = W / 2;
    const int64_t v2 = (int64_t)d2 * h2 * w2;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= planes * v2) return;
    const int64_t pl = i / v2, r = i % v2;
    const int wx = (int)(r % w2), hy = (int)((r / w2) % h2), dz = (int)(r / ((int64_t)w2 * h2));
    const float* xp = x + pl * (int64_t)D * H * W;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        s += xp[(int64_t)(2 * dz + (c >> 2)) * H * W + (int64_t)(2 * hy + ((c >> 1) & 1)) * W + 2 * wx + (c & 1)];
    y[i] = 0.125f * scale * s;
}

// y += a x
__global__ void k_axpy(int64_t n, float a, const float* __restrict__ x, float* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

// gx[child] = gy[parent] / 8  (adjoint of k_pool2); up-sampling by
// replication is the same map times 8
__global__ void k_unpool2(int64_t planes, int D, int H, int W, float scale, const float* __restrict__ gy,
                          float* __restrict__ gx) {
    const int64_t V = (int64_t)D * H * W;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= planes * V) return;
    const int64_t pl = i / V, r = i % V;
    const int wx = (int)(r % W), hy = (int)((r / W) % H), dz = (int)(r / ((int64_t)W * H));
    const int d2 = D / 2, h2 = H / 2, w2 = W / 2;
    gx[i] = scale * gy[pl * (int64_t)d2 * h2 * w2 + (int64_t)(dz / 2) * h2 * w2 + (int64_t)(hy / 2) * w2 + wx / 2];
}

// Channel concatenation y = [a | b] per sample, and the split back.
__global__ void k_concat(int N, int Ca, int Cb, int64_t V, const float* __restrict__ a, const float* __restrict__ b,
                         float* __restrict__ y) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int C = Ca + Cb;
    if (i >= (int64_t)N * C * V) return;
    const int64_t n = i / ((int64_t)C * V), r = i % ((int64_t)C * V);
    const int c = (int)(r / V);
    const int64_t p = r % V;
    y[i] = c < Ca ? a[((int64_t)n * Ca + c) * V + p] : b[((int64_t)n * Cb + (c - Ca)) * V + p];
}

__global__ void k_split(int N, int Ca, int Cb, int64_t V, const float* __restrict__ y, float* __restrict__ a,
                        float* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int C = Ca + Cb;
    if (i >= (int64_t)N * C * V) return;
    const int64_t n = i / ((int64_t)C * V), r = i % ((int64_t)C * V);
    const int c = (int)(r / V);
    const int64_t p = r % V;
    if (c < Ca) a[((int64_t)n * Ca + c) * V + p] = y[i];
    else b[((int64_t)n * Cb + (c - Ca)) * V + p] = y[i];
}

// Node values as the mean of the (1..8) cells around each node (cells D x H x
// W, nodes (D+1)(H+1)(W+1)), and the adjoint.
__global__ void k_cell2node(int64_t planes, int D, int H, int W, const float* __restrict__ c, float* __restrict__ nd) {
    const int64_t NV = (int64_t)(D + 1) * (H + 1) * (W + 1), CV = (int64_t)D * H * W;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= planes * NV) return;
    const int64_t pl = i / NV, r = i % NV;
    const int x = (int)(r % (W + 1)), y = (int)((r / (W + 1)) % (H + 1)), z = (int)(r / ((int64_t)(W + 1) * (H + 1)));
    float s = 0.f;
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int cx = x - 1 + (q & 1), cy = y - 1 + ((q >> 1) & 1), cz = z - 1 + (q >> 2);
        if (cx < 0 || cx >= W || cy < 0 || cy >= H || cz < 0 || cz >= D) continue;
        s += c[pl * CV + (int64_t)cz * H * W + (int64_t)cy * W + cx];
        ++cnt;
    }
    nd[i] = s / (float)cnt;
}

__global__ void k_nodes_to_dofs(int nfields, int64_t nodes, const float* __restrict__ ch, double* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nfields * 3 * nodes) return;
    const int64_t f = i / (3 * nodes), r = i % (3 * nodes);
    const int64_t node = r / 3;
    const int c = (int)(r % 3);
    b[i] = (double)ch[(3 * f + c) * nodes + node];
}

__global__ void k_node2cell_grad(int64_t planes, int D, int H, int W, const float* __restrict__ gn,
                                 float* __restrict__ gc) {
    const int64_t NV = (int64_t)(D + 1) * (H + 1) * (W + 1), CV = (int64_t)D * H * W;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= planes * CV) return;
    const int64_t pl = i / CV, r = i % CV;
    const int x = (int)(r % W), y = (int)((r / W) % H), z = (int)(r / ((int64_t)W * H));
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int nx = x + (q & 1), ny = y + ((q >> 1) & 1), nz = z + (q >> 2);
        const int cntx = (nx == 0 || nx == W) ? 1 : 2, cnty = (ny == 0 || ny == H) ? 1 : 2,
                  cntz = (nz == 0 || nz == D) ? 1 : 2;
        s += gn[pl * NV + (int64_t)nz * (H + 1) * (W + 1) + (int64_t)ny * (W + 1) + nx] / (float)(cntx * cnty * cntz);
    }
    gc[i] = s;
}

// loss partials of sum w (p - t)^2 and g = 2 w (p - t) * scale
__global__ __launch_bounds__(kNnThreads) void k_mse(int64_t n, const float* __restrict__ pred,
                                                    const float* __restrict__ target,
                                                    const float* __restrict__ weight, float scale,
                                                    float* __restrict__ grad, double* __restrict__ part) {
    __shared__ double red[kNnThreads / 64];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kNnThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNnThreads) {
        const float wgt = weight ? weight[i] : 1.f;
        const float d = pred[i] - target[i];
        grad[i] = 2.f * wgt * d * scale;
        s += (double)wgt * (double)d * (double)d;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kNnThreads / 64; ++q) t += red[q];
        part[blockIdx.x] = t;
    }
}

// Adam on FP32 master weights; refreshes the BF16 copy used by the convs.
__global__ void k_adam(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float* __restrict__ w, uint16_t* __restrict__ wb, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f32_to_bf16(wi);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ a, uint16_t* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = f32_to_bf16(a[i]);
}

// ---------------------------------------------------------------------------
static inline unsigned nbk(int64_t n) { return (unsigned)((n + kNnThreads - 1) / kNnThreads); }

int launch_nn_conv3d(int N, int Ci, int Co, int D, int H, int W, int K, int trans, const float* x, const uint16_t* w,
                     const float* bias, float* y, int relu, hipStream_t st) {
    const int64_t V = (int64_t)D * H * W;
    const dim3 gr(nbk(V), (unsigned)((Co + kCoGroup - 1) / kCoGroup), (unsigned)N);
    if (K == 3 && !trans) hipLaunchKernelGGL((k_conv3d<3, false>), gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu);
    else if (K == 3 && trans) hipLaunchKernelGGL((k_conv3d<3, true>), gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu);
    else if (K == 1 && !trans) hipLaunchKernelGGL((k_conv3d<1, false>), gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu);
    else if (K == 1 && trans) hipLaunchKernelGGL((k_conv3d<1, true>), gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu);
    else return -1;
    return 0;
}

int launch_nn_conv3d_mfma(int N, int Ci, int Co, int D, int H, int W, const float* x, const uint16_t* w,
                          const float* bias, float* y, int relu, hipStream_t st) {
    const int64_t V = (int64_t)D * H * W;
    const int64_t wavesv = (V + 15) / 16;
    const unsigned gx = (unsigned)((wavesv + kNnThreads / 64 - 1) / (kNnThreads / 64));
    const int ntile = (Co + 15) / 16;
    if (ntile <= 4) {
        const dim3 gr(gx, (unsigned)N, 1);
#define MLB_CM(MT) hipLaunchKernelGGL(k_conv3d_mfma<MT>, gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu)
        if (ntile == 1) MLB_CM(1);
        else if (ntile == 2) MLB_CM(2);
        else if (ntile == 3) MLB_CM(3);
        else MLB_CM(4);
#undef MLB_CM
    } else {
        const dim3 gr(gx, (unsigned)N, (unsigned)((ntile + 3) / 4));
        hipLaunchKernelGGL(k_conv3d_mfma<4>, gr, dim3(kNnThreads), 0, st, Ci, Co, D, H, W, x, w, bias, y, relu);
    }
    return 0;
}

int launch_nn_conv3d_wgrad(int N, int Ci, int Co, int D, int H, int W, int K, const float* x, const float* dy,
                           float* dw, float* db, hipStream_t st) {
    const dim3 gr((unsigned)Ci, (unsigned)Co, 1);
    if (K == 3) hipLaunchKernelGGL(k_conv3d_wgrad<3>, gr, dim3(kNnThreads), 0, st, N, Ci, Co, D, H, W, x, dy, dw);
    else if (K == 1) hipLaunchKernelGGL(k_conv3d_wgrad<1>, gr, dim3(kNnThreads), 0, st, N, Ci, Co, D, H, W, x, dy, dw);
    else return -1;
    if (db) hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)Co), dim3(kNnThreads), 0, st, N, Co, (int64_t)D * H * W, dy, db);
    return 0;
}

void launch_nn_relu_mask(int64_t n, const float* y, float* g, hipStream_t st) {
    hipLaunchKernelGGL(k_relu_mask, dim3(nbk(n)), dim3(kNnThreads), 0, st, n, y, g);
}
void launch_nn_pool2(int64_t planes, int D, int H, int W, float scale, const float* x, float* y, hipStream_t st) {
    hipLaunchKernelGGL(k_pool2, dim3(nbk(planes * (D / 2) * (H / 2) * (W / 2))), dim3(kNnThreads), 0, st, planes, D, H,
                       W, scale, x, y);
}
void launch_nn_axpy(int64_t n, float a, const float* x, float* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy, dim3(nbk(n)), dim3(kNnThreads), 0, st, n, a, x, y);
}
void launch_nn_unpool2(int64_t planes, int D, int H, int W, float scale, const float* gy, float* gx, hipStream_t st) {
    hipLaunchKernelGGL(k_unpool2, dim3(nbk(planes * D * H * W)), dim3(kNnThreads), 0, st, planes, D, H, W, scale, gy,
                       gx);
}
void launch_nn_concat(int N, int Ca, int Cb, int64_t V, const float* a, const float* b, float* y, hipStream_t st) {
    hipLaunchKernelGGL(k_concat, dim3(nbk((int64_t)N * (Ca + Cb) * V)), dim3(kNnThreads), 0, st, N, Ca, Cb, V, a, b, y);
}
void launch_nn_split(int N, int Ca, int Cb, int64_t V, const float* y, float* a, float* b, hipStream_t st) {
    hipLaunchKernelGGL(k_split, dim3(nbk((int64_t)N * (Ca + Cb) * V)), dim3(kNnThreads), 0, st, N, Ca, Cb, V, y, a, b);
}
void launch_nn_cell2node(int64_t planes, int D, int H, int W, const float* c, float* nd, hipStream_t st) {
    hipLaunchKernelGGL(k_cell2node, dim3(nbk(planes * (D + 1) * (H + 1) * (W + 1))), dim3(kNnThreads), 0, st, planes,
                       D, H, W, c, nd);
}
void launch_nn_nodes_to_dofs(int nfields, int64_t nodes, const float* ch, double* b, hipStream_t st) {
    hipLaunchKernelGGL(k_nodes_to_dofs, dim3(nbk(nfields * 3 * nodes)), dim3(kNnThreads), 0, st, nfields, nodes, ch, b);
}
void launch_nn_node2cell_grad(int64_t planes, int D, int H, int W, const float* gn, float* gc, hipStream_t st) {
    hipLaunchKernelGGL(k_node2cell_grad, dim3(nbk(planes * D * H * W)), dim3(kNnThreads), 0, st, planes, D, H, W, gn,
                       gc);
}
int nn_mse_parts(int64_t n) {
    const int64_t b = (n + kNnThreads - 1) / kNnThreads;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}
void launch_nn_mse(int64_t n, const float* pred, const float* target, const float* weight, float scale, float* grad,
                   int nparts, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_mse, dim3((unsigned)nparts), dim3(kNnThreads), 0, st, n, pred, target, weight, scale, grad,
                       part);
}
void launch_nn_adam(int64_t n, float lr, float b1, float b2, float eps, int step, float* w, uint16_t* wb,
                    const float* g, float* m, float* v, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nbk(n)), dim3(kNnThreads), 0, st, n, lr, b1, b2, eps, c1, c2, w, wb, g, m, v);
}
void launch_nn_to_bf16(int64_t n, const float* a, uint16_t* b, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nbk(n)), dim3(kNnThreads), 0, st, n, a, b);
}

}  // namespace mlb
