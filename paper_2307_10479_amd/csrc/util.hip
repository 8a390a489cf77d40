// Device-count helpers, the autotuner table, the medoid seed (Sec. 5.4) and
// the reduced-precision store encoders.
#include <hip/hip_runtime.h>

#include <math.h>
#include <mutex>
#include <vector>

#include "deg.h"
#include "host_util.h"

namespace degk {

// ---------------------------------------------------------------- tuner table
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

int kp_bucket_of(int kp) { return kp <= 16 ? 16 : (kp <= 64 ? 64 : (kp <= 128 ? 128 : (kp <= 256 ? 256 : 512))); }

const TuneEntry *tune_lookup(int dtype, int dim, int degree, int kp) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int b = kp_bucket_of(kp);
    for (const TuneEntry &e : g_tune)
        if (e.dtype == dtype && e.dim == dim && e.degree == degree && e.kp_bucket == b) return &e;
    return nullptr;
}

// ---------------------------------------------------------------- medoid
// Column sums: block b sums rows b, b+G, ... of its column slice in FP64.
__global__ void col_partial_kernel(const float *x, int64_t n, int32_t dim, int64_t stride,
                                   double *part, int nparts) {
    int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= dim) return;
    double s = 0.0;
    for (int64_t i = blockIdx.x; i < n; i += nparts) s += (double)x[i * stride + c];
    part[(int64_t)blockIdx.x * dim + c] = s;
}

__global__ void col_mean_kernel(const double *part, int nparts, int32_t dim, int64_t n,
                                double *mean) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= dim) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * dim + c];
    mean[c] = s / (double)n;
}

// Per-block best (score, id): score = squared distance to the mean (L2) or
// minus the inner product with it (IP); ties -> smaller id.
__global__ void medoid_score_kernel(const float *x, int64_t n, int32_t dim, int64_t stride,
                                    int32_t metric, const double *mean, double *bs, int64_t *bi) {
    __shared__ double sd[256];
    __shared__ int64_t si[256];
    double best = INFINITY;
    int64_t bid = -1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        const float *r = x + i * stride;
        for (int c = 0; c < dim; ++c) {
            if (metric == DEG_METRIC_L2) {
                double t = (double)r[c] - mean[c];
                s += t * t;
            } else {
                s -= (double)r[c] * mean[c];
            }
        }
        if (s < best || (s == best && i < bid)) { best = s; bid = i; }
    }
    sd[threadIdx.x] = best;
    si[threadIdx.x] = bid;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double o = sd[threadIdx.x + w];
            int64_t oi = si[threadIdx.x + w];
            if (oi >= 0 && (si[threadIdx.x] < 0 || o < sd[threadIdx.x] ||
                            (o == sd[threadIdx.x] && oi < si[threadIdx.x]))) {
                sd[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bs[blockIdx.x] = sd[0];
        bi[blockIdx.x] = si[0];
    }
}

__global__ void medoid_final_kernel(const double *bs, const int64_t *bi, int nb, int32_t *out) {
    double best = INFINITY;
    int64_t bid = -1;
    for (int b = 0; b < nb; ++b)
        if (bi[b] >= 0 && (bid < 0 || bs[b] < best || (bs[b] == best && bi[b] < bid))) {
            best = bs[b];
            bid = bi[b];
        }
    *out = (int32_t)bid;
}

constexpr int MED_PARTS = 256;
constexpr int MED_BLOCKS = 1024;

// ---------------------------------------------------------------- encoders
__global__ void bf16_kernel(const float *x, int64_t n, int32_t dim, int64_t xs, uint16_t *out,
                            int64_t os) {
    int64_t row = blockIdx.x;
    if (row >= n) return;
    for (int c = threadIdx.x; c < os; c += blockDim.x) {
        uint16_t h = 0;
        if (c < dim) {
            uint32_t u = __float_as_uint(x[row * xs + c]);
            h = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
        }
        out[row * os + c] = h;
    }
}

// E4M3 (OCP) code of a with round-to-nearest-even, saturating at 448.
__device__ __forceinline__ uint32_t e4m3_rne(float a) {
    uint32_t sgn = (__float_as_uint(a) >> 24) & 0x80u;
    float m = fabsf(a);
    if (!(m < 448.0f)) return sgn | 0x7Eu;
    uint32_t code;
    if (m < 0.015625f) {  // below the smallest normal 2^-6: step 2^-9
        code = (uint32_t)rintf(m * 512.0f);
    } else {
        int e;
        float fr = frexpf(m, &e);  // m = fr * 2^e, fr in [0.5, 1)
        int E = e - 1;
        float q = rintf(__fmul_rn(__fsub_rn(__fmul_rn(fr, 2.0f), 1.0f), 8.0f));
        uint32_t qi = (uint32_t)q;
        if (qi == 8u) { E += 1; qi = 0u; }
        code = ((uint32_t)(E + 7) << 3) | qi;
    }
    return sgn | code;
}

// One block (64 lanes) per row: scale = max|x| / 448, codes of x / scale.
__global__ void fp8_kernel(const float *x, int64_t n, int32_t dim, int64_t xs, uint8_t *out,
                           int64_t os, float *scale) {
    int64_t row = blockIdx.x;
    if (row >= n) return;
    const float *r = x + row * xs;
    float mx = 0.0f;
    for (int c = threadIdx.x; c < dim; c += 64) mx = fmaxf(mx, fabsf(r[c]));
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
    float s = mx > 0.0f ? __fdiv_rn(mx, 448.0f) : 1.0f;
    if (threadIdx.x == 0) scale[row] = s;
    for (int c = threadIdx.x; c < os; c += 64)
        out[row * os + c] = c < dim ? (uint8_t)e4m3_rne(__fdiv_rn(r[c], s)) : (uint8_t)0;
}

}  // namespace degk

using namespace degk;

extern "C" int32_t deg_device_cu_count(void) {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (dev >= 0 && dev < 64 && cached[dev] > 0) return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 1;
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

extern "C" const char *deg_status_string(deg_status s) {
    switch (s) {
        case DEG_OK: return "ok";
        case DEG_ERR_INVALID_ARG: return "invalid argument";
        case DEG_ERR_UNSUPPORTED: return "unsupported configuration";
        case DEG_ERR_WORKSPACE: return "workspace missing or too small";
        case DEG_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

extern "C" deg_status deg_tune_register(int32_t dtype, int32_t dim, int32_t degree,
                                        int32_t kp_bucket, int32_t hash_slots,
                                        int32_t waves_per_cu) {
    if (hash_slots < 256 || hash_slots > 16384 || (hash_slots & (hash_slots - 1)) ||
        waves_per_cu < 0 || kp_bucket != kp_bucket_of(kp_bucket))
        return DEG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TuneEntry &e : g_tune)
        if (e.dtype == dtype && e.dim == dim && e.degree == degree && e.kp_bucket == kp_bucket) {
            e.hash_slots = hash_slots;
            e.waves_per_cu = waves_per_cu;
            return DEG_OK;
        }
    g_tune.push_back(TuneEntry{dtype, dim, degree, kp_bucket, hash_slots, waves_per_cu});
    return DEG_OK;
}

extern "C" void deg_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

extern "C" size_t deg_medoid_workspace_bytes(int64_t n, int32_t dim) {
    (void)n;
    return 8 * ((size_t)MED_PARTS * dim + dim + 2 * MED_BLOCKS) + 256;
}

extern "C" deg_status deg_medoid(const float *vec, int64_t n, int32_t dim, int64_t stride,
                                 int32_t metric, int32_t *out_id, void *workspace,
                                 size_t ws_bytes, void *stream) {
    if (!vec || !out_id || n < 1 || dim < 1 || stride < dim ||
        (metric != DEG_METRIC_L2 && metric != DEG_METRIC_IP))
        return DEG_ERR_INVALID_ARG;
    if (!workspace || ws_bytes < deg_medoid_workspace_bytes(n, dim)) return DEG_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = reinterpret_cast<double *>(workspace);
    double *mean = part + (size_t)MED_PARTS * dim;
    double *bs = mean + dim;
    int64_t *bi = reinterpret_cast<int64_t *>(bs + MED_BLOCKS);
    dim3 g1(MED_PARTS, (dim + 63) / 64);
    hipLaunchKernelGGL(col_partial_kernel, g1, dim3(64), 0, st, vec, n, dim, stride, part, MED_PARTS);
    hipLaunchKernelGGL(col_mean_kernel, dim3((dim + 63) / 64), dim3(64), 0, st, part, MED_PARTS, dim,
                       n, mean);
    hipLaunchKernelGGL(medoid_score_kernel, dim3(MED_BLOCKS), dim3(256), 0, st, vec, n, dim, stride,
                       metric, mean, bs, bi);
    hipLaunchKernelGGL(medoid_final_kernel, dim3(1), dim3(1), 0, st, bs, bi, MED_BLOCKS, out_id);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_encode_bf16(const float *x, int64_t n, int32_t dim, int64_t x_stride,
                                      uint16_t *out, int64_t out_stride, void *stream) {
    if (!x || !out || n < 0 || dim < 1 || x_stride < dim || out_stride < dim)
        return DEG_ERR_INVALID_ARG;
    if (n == 0) return DEG_OK;
    hipLaunchKernelGGL(bf16_kernel, dim3((unsigned)n), dim3(128), 0,
                       static_cast<hipStream_t>(stream), x, n, dim, x_stride, out, out_stride);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

extern "C" deg_status deg_encode_fp8(const float *x, int64_t n, int32_t dim, int64_t x_stride,
                                     uint8_t *out, int64_t out_stride, float *scale,
                                     void *stream) {
    if (!x || !out || !scale || n < 0 || dim < 1 || x_stride < dim || out_stride < dim)
        return DEG_ERR_INVALID_ARG;
    if (n == 0) return DEG_OK;
    hipLaunchKernelGGL(fp8_kernel, dim3((unsigned)n), dim3(64), 0,
                       static_cast<hipStream_t>(stream), x, n, dim, x_stride, out, out_stride,
                       scale);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}
