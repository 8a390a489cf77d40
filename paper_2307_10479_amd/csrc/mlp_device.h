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
// lane returns the same value. Lane i < 16 holds standardised feature i in
// `fs`; the features reach every lane through readlane (no per-lane arrays).
// hbuf: 64 floats of LDS owned by the wave, 16-byte aligned. Weight rows are
// read as 16-byte vectors (8 BF16 each).
__device__ __forceinline__ void bf16x8(const uint4 u, float (&o)[8]) {
    o[0] = __uint_as_float(u.x << 16); o[1] = __uint_as_float(u.x & 0xffff0000u);
    o[2] = __uint_as_float(u.y << 16); o[3] = __uint_as_float(u.y & 0xffff0000u);
    o[4] = __uint_as_float(u.z << 16); o[5] = __uint_as_float(u.z & 0xffff0000u);
    o[6] = __uint_as_float(u.w << 16); o[7] = __uint_as_float(u.w & 0xffff0000u);
}

__device__ __forceinline__ float mlp_logit_bf16(const uint16_t *W, float fs, float *hbuf) {
    const int j = (int)threadIdx.x & 63;
    const uint4 *w1 = reinterpret_cast<const uint4 *>(W + OFF_W1 + j * MLP_IN);
    float w[8];
    float s = bf16_val(W[OFF_B1 + j]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        bf16x8(w1[h], w);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float fi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, fs), 8 * h + i));
            s = __fmaf_rn(w[i], fi, s);
        }
    }
    hbuf[j] = fmaxf(s, 0.0f);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    const uint4 *w2 = reinterpret_cast<const uint4 *>(W + OFF_W2 + j * MLP_H);
    const float4 *h4 = reinterpret_cast<const float4 *>(hbuf);
    s = bf16_val(W[OFF_B2 + j]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        bf16x8(w2[t], w);
        const float4 ha = h4[2 * t], hb = h4[2 * t + 1];
        s = __fmaf_rn(w[0], ha.x, s); s = __fmaf_rn(w[1], ha.y, s);
        s = __fmaf_rn(w[2], ha.z, s); s = __fmaf_rn(w[3], ha.w, s);
        s = __fmaf_rn(w[4], hb.x, s); s = __fmaf_rn(w[5], hb.y, s);
        s = __fmaf_rn(w[6], hb.z, s); s = __fmaf_rn(w[7], hb.w, s);
    }
    const float h2 = fmaxf(s, 0.0f);
    float z = __fmul_rn(bf16_val(W[OFF_W3 + j]), h2);
    // sum over the 64 lanes: rotations within rows of 16 (DPP), then the four
    // row sums through readlane, in a fixed order
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x128, 0xF, 0xF, false)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x124, 0xF, 0xF, false)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x122, 0xF, 0xF, false)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x121, 0xF, 0xF, false)));
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, z), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, z), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, z), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, z), 48));
    z = __fadd_rn(__fadd_rn(r0, r1), __fadd_rn(r2, r3));
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    return __fadd_rn(z, bf16_val(W[OFF_B3]));
}

}  // namespace degk
