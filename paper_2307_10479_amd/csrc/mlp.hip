// Training and inference kernels of the stop predictor: a 16-64-64-1 MLP
// with ReLU hidden layers and a sigmoid output, trained with the mean binary
// cross-entropy and Adam in FP32; the search evaluates it with BF16 weights.
//
// Training step on B rows:
//   mlp_block_grad  block b takes rows [32b, 32b+32): forward, backward, and
//                   the block's gradient partial sums (LDS outer products)
//   mlp_reduce      sums the block partials in block order (deterministic)
//   mlp_adam        bias-corrected Adam update
#include <hip/hip_runtime.h>

#include <math.h>

#include "deg.h"
#include "mlp_device.h"

namespace degk {

constexpr int TB = 32;              // rows per block
constexpr int NPART = MLP_NP + 1;   // gradient + loss

__device__ __forceinline__ float softplus_neg_abs(float z) { return log1pf(expf(-fabsf(z))); }

__global__ void __launch_bounds__(256) mlp_block_grad(const float *__restrict__ P,
                                                      const float *__restrict__ X,
                                                      const float *__restrict__ y, int64_t B,
                                                      float *__restrict__ part) {
    __shared__ float sW2[MLP_H * MLP_H];
    __shared__ float sx[TB][MLP_IN];
    __shared__ float sh1[TB][MLP_H];
    __shared__ float sg2[TB][MLP_H];
    __shared__ float sg1[TB][MLP_H];
    __shared__ float sdz[TB];
    __shared__ float sloss[TB];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * TB;
    for (int i = t; i < MLP_H * MLP_H; i += 256) sW2[i] = P[OFF_W2 + i];
    for (int i = t; i < TB * MLP_IN; i += 256) {
        int r = i / MLP_IN, c = i % MLP_IN;
        sx[r][c] = (r0 + r < B) ? X[(r0 + r) * MLP_IN + c] : 0.0f;
    }
    __syncthreads();
    // forward: thread (r, j) with r = t / 8, j-group = t % 8 computes 8 hidden units
    const int r = t >> 3, jg = t & 7;
    const bool valid = r0 + r < B;
    float h1v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        int j = jg * 8 + u;
        float s = P[OFF_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) s = __fmaf_rn(P[OFF_W1 + j * MLP_IN + i], sx[r][i], s);
        h1v[u] = fmaxf(s, 0.0f);
        sh1[r][j] = h1v[u];
    }
    __syncthreads();
    float h2v[8];
    float zp = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        int j = jg * 8 + u;
        float s = P[OFF_B2 + j];
        for (int i = 0; i < MLP_H; ++i) s = __fmaf_rn(sW2[j * MLP_H + i], sh1[r][i], s);
        h2v[u] = fmaxf(s, 0.0f);
        zp = __fmaf_rn(P[OFF_W3 + j], h2v[u], zp);
    }
    // sum the 8 partial logits of row r (lanes r*8 .. r*8+7 are in one wave)
    zp = __fadd_rn(zp, __shfl_xor(zp, 1));
    zp = __fadd_rn(zp, __shfl_xor(zp, 2));
    zp = __fadd_rn(zp, __shfl_xor(zp, 4));
    const float z = __fadd_rn(zp, P[OFF_B3]);
    if (jg == 0) {
        float yt = valid ? y[r0 + r] : 0.0f;
        float sg = 1.0f / (1.0f + expf(-z));
        sdz[r] = valid ? (sg - yt) / (float)B : 0.0f;
        sloss[r] = valid ? (fmaxf(z, 0.0f) - z * yt + softplus_neg_abs(z)) : 0.0f;
    }
    __syncthreads();
    const float dz = sdz[r];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        int j = jg * 8 + u;
        sg2[r][j] = h2v[u] > 0.0f ? dz * P[OFF_W3 + j] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        int i = jg * 8 + u;
        float s = 0.0f;
        for (int j = 0; j < MLP_H; ++j) s = __fmaf_rn(sg2[r][j], sW2[j * MLP_H + i], s);
        sg1[r][i] = sh1[r][i] > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * NPART;
    // dW2[j][i] = sum_r g2[r][j] h1[r][i]
    for (int e = t; e < MLP_H * MLP_H; e += 256) {
        int j = e / MLP_H, i = e % MLP_H;
        float s = 0.0f;
        for (int rr = 0; rr < TB; ++rr) s = __fmaf_rn(sg2[rr][j], sh1[rr][i], s);
        out[OFF_W2 + e] = s;
    }
    // dW1[i][c] = sum_r g1[r][i] x[r][c]
    for (int e = t; e < MLP_H * MLP_IN; e += 256) {
        int i = e / MLP_IN, c = e % MLP_IN;
        float s = 0.0f;
        for (int rr = 0; rr < TB; ++rr) s = __fmaf_rn(sg1[rr][i], sx[rr][c], s);
        out[OFF_W1 + e] = s;
    }
    if (t < MLP_H) {
        float b1 = 0.0f, b2 = 0.0f;
        for (int rr = 0; rr < TB; ++rr) {
            b1 = __fadd_rn(b1, sg1[rr][t]);
            b2 = __fadd_rn(b2, sg2[rr][t]);
        }
        out[OFF_B1 + t] = b1;
        out[OFF_B2 + t] = b2;
    }
    // dw3[j] = sum_r dz[r] h2[r][j]; thread (r, jg) holds h2 of 8 units of row r
    __shared__ float sh2[TB][MLP_H];
#pragma unroll
    for (int u = 0; u < 8; ++u) sh2[r][jg * 8 + u] = h2v[u];
    __syncthreads();
    if (t < MLP_H) {
        float s = 0.0f;
        for (int rr = 0; rr < TB; ++rr) s = __fmaf_rn(sdz[rr], sh2[rr][t], s);
        out[OFF_W3 + t] = s;
    }
    if (t == 0) {
        float s = 0.0f, l = 0.0f;
        for (int rr = 0; rr < TB; ++rr) {
            s = __fadd_rn(s, sdz[rr]);
            l = __fadd_rn(l, sloss[rr]);
        }
        out[OFF_B3] = s;
        out[MLP_NP] = l;
    }
}

__global__ void mlp_reduce(const float *__restrict__ part, int nblocks, float *__restrict__ grad,
                           float *__restrict__ loss, int64_t B) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPART) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s = __fadd_rn(s, part[(int64_t)b * NPART + e]);
    if (e < MLP_NP) grad[e] = s;
    else if (loss) *loss = s / (float)B;
}

__global__ void mlp_adam(float *P, float *m, float *v, const float *g, float lr, float c1,
                         float c2) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MLP_NP) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gg = g[e];
    float mm = b1 * m[e] + (1.0f - b1) * gg;
    float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    P[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void mlp_forward_f32(const float *__restrict__ P, const float *__restrict__ X,
                                int64_t B, float *__restrict__ out) {
    int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= B) return;
    float x[MLP_IN], h1[MLP_H];
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[row * MLP_IN + i];
    for (int j = 0; j < MLP_H; ++j) {
        float s = P[OFF_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) s = __fmaf_rn(P[OFF_W1 + j * MLP_IN + i], x[i], s);
        h1[j] = fmaxf(s, 0.0f);
    }
    float z = P[OFF_B3];
    for (int j = 0; j < MLP_H; ++j) {
        float s = P[OFF_B2 + j];
        for (int i = 0; i < MLP_H; ++i) s = __fmaf_rn(P[OFF_W2 + j * MLP_H + i], h1[i], s);
        z = __fmaf_rn(P[OFF_W3 + j], fmaxf(s, 0.0f), z);
    }
    out[row] = z;
}

// One wave per row with the same routine the search uses.
__global__ void __launch_bounds__(64) mlp_forward_bf16_kernel(const uint16_t *W, const float *X,
                                                              int64_t B, float *out) {
    __shared__ __align__(16) float hbuf[64];
    const MlpRegs M = mlp_load(W);
    for (int64_t row = blockIdx.x; row < B; row += gridDim.x) {
        const int lane = (int)threadIdx.x & 63;
        const float fs = lane < MLP_IN ? X[row * MLP_IN + lane] : 0.0f;
        float z = mlp_logit(M, W, fs, hbuf);
        if (threadIdx.x == 0) out[row] = z;
    }
}

__global__ void mlp_export_kernel(const float *P, uint16_t *out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= MLP_NP) return;
    uint32_t u = __float_as_uint(P[e]);
    out[e] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Column statistics of B rows of 16 features for the standardisation of the
// stop predictor's inputs: one block per column, FP64 sums in a fixed order
// (per-thread strided partial sums, then a tree over the block), two passes
// (mean, then the unbiased variance). inv_std = 1 / std, or 0 when std <= 1e-6.
__global__ void __launch_bounds__(256) feature_stats_kernel(const float *X, int64_t B, float *mean,
                                                            float *inv_std) {
    __shared__ double red[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < B; i += 256) s += (double)X[i * MLP_IN + c];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double mu = red[0] / (double)B;
    __syncthreads();
    s = 0.0;
    for (int64_t i = t; i < B; i += 256) {
        const double d = (double)X[i * MLP_IN + c] - mu;
        s += d * d;
    }
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) {
        const double sd = B > 1 ? sqrt(red[0] / (double)(B - 1)) : 0.0;
        mean[c] = (float)mu;
        inv_std[c] = sd > 1e-6 ? (float)(1.0 / sd) : 0.0f;
    }
}

// out = (X - mean) * inv_std, FP32 (the rounding the search applies).
__global__ void standardise_kernel(const float *X, int64_t B, const float *mean,
                                   const float *inv_std, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * MLP_IN) return;
    const int c = (int)(i % MLP_IN);
    out[i] = __fmul_rn(__fsub_rn(X[i], mean[c]), inv_std[c]);
}

}  // namespace degk

using namespace degk;

extern "C" size_t deg_mlp_workspace_bytes(int64_t B) {
    int64_t nb = (B + TB - 1) / TB;
    return (size_t)(nb > 0 ? nb : 1) * NPART * 4 + (size_t)MLP_NP * 4 + 256;
}

extern "C" deg_status deg_mlp_train_step(float *params, float *m, float *v, const float *X,
                                         const float *y, int64_t B, int64_t step, float lr,
                                         float *grad, float *loss, void *workspace,
                                         size_t ws_bytes, void *stream) {
    if (!params || !X || !y || B < 1 || B > (int64_t)1 << 30 || step < 1) return DEG_ERR_INVALID_ARG;
    if (lr != 0.0f && (!m || !v)) return DEG_ERR_INVALID_ARG;
    if (!workspace || ws_bytes < deg_mlp_workspace_bytes(B)) return DEG_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int nb = (int)((B + TB - 1) / TB);
    float *part = reinterpret_cast<float *>(workspace);
    float *g = grad ? grad : part + (size_t)nb * NPART;
    hipLaunchKernelGGL(mlp_block_grad, dim3(nb), dim3(256), 0, st, params, X, y, B, part);
    hipLaunchKernelGGL(mlp_reduce, dim3((NPART + 255) / 256), dim3(256), 0, st, part, nb, g, loss, B);
    if (lr != 0.0f) {
        float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
        hipLaunchKernelGGL(mlp_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, params, m, v, g,
                           lr, c1, c2);
    }
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_mlp_forward(const float *params, const float *X, int64_t B, float *out,
                                      void *stream) {
    if (!params || !X || !out || B < 0) return DEG_ERR_INVALID_ARG;
    if (B == 0) return DEG_OK;
    hipLaunchKernelGGL(mlp_forward_f32, dim3((unsigned)((B + 127) / 128)), dim3(128), 0,
                       static_cast<hipStream_t>(stream), params, X, B, out);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_mlp_forward_bf16(const uint16_t *w, const float *X, int64_t B,
                                           float *out, void *stream) {
    if (!w || !X || !out || B < 0) return DEG_ERR_INVALID_ARG;
    if (B == 0) return DEG_OK;
    unsigned g = (unsigned)(B < 65536 ? B : 65536);
    hipLaunchKernelGGL(mlp_forward_bf16_kernel, dim3(g), dim3(64), 0,
                       static_cast<hipStream_t>(stream), w, X, B, out);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_mlp_export_bf16(const float *params, uint16_t *out, void *stream) {
    if (!params || !out) return DEG_ERR_INVALID_ARG;
    hipLaunchKernelGGL(mlp_export_kernel, dim3((MLP_NP + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), params, out);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_mlp_feature_stats(const float *X, int64_t B, float *mean, float *inv_std,
                                           void *stream) {
    if (!X || !mean || !inv_std || B < 1) return DEG_ERR_INVALID_ARG;
    hipLaunchKernelGGL(feature_stats_kernel, dim3(MLP_IN), dim3(256), 0,
                       static_cast<hipStream_t>(stream), X, B, mean, inv_std);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_mlp_standardise(const float *X, int64_t B, const float *mean,
                                         const float *inv_std, float *out, void *stream) {
    if (!X || !mean || !inv_std || !out || B < 0) return DEG_ERR_INVALID_ARG;
    if (B == 0) return DEG_OK;
    const int64_t n = B * MLP_IN;
    hipLaunchKernelGGL(standardise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), X, B, mean, inv_std, out);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}
