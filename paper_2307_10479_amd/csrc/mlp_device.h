// Stop-predictor MLP (16 -> 64 -> 64 -> 1, ReLU, logit) evaluated by one
// wavefront: lane j owns hidden unit j of both layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace degk {

constexpr int MLP_IN = 16, MLP_H = 64;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_H;
constexpr int MLP_NP = OFF_B3 + 1;  // 5313

__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Logit of one feature row with BF16 weights and FP32 accumulation; every
// lane returns the same value. hbuf: 64 floats of LDS owned by the wave.
__device__ __forceinline__ float mlp_logit_bf16(const uint16_t *W, const float (&f)[MLP_IN],
                                                float *hbuf) {
    const int j = (int)threadIdx.x & 63;
    float s = bf16_val(W[OFF_B1 + j]);
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) s = __fmaf_rn(bf16_val(W[OFF_W1 + j * MLP_IN + i]), f[i], s);
    hbuf[j] = fmaxf(s, 0.0f);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    s = bf16_val(W[OFF_B2 + j]);
#pragma unroll 16
    for (int i = 0; i < MLP_H; ++i) s = __fmaf_rn(bf16_val(W[OFF_W2 + j * MLP_H + i]), hbuf[i], s);
    float h2 = fmaxf(s, 0.0f);
    float z = __fmul_rn(bf16_val(W[OFF_W3 + j]), h2);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) z = __fadd_rn(z, __shfl_xor(z, m));
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return __fadd_rn(z, bf16_val(W[OFF_B3]));
}

}  // namespace degk
