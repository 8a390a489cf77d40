// Stop-predictor MLP (16 -> 64 -> 64 -> 1, ReLU, logit) evaluated by one
// wavefront: lane j owns hidden unit j of both layers. BF16 inference is one
// fixed FP32 computation, so that every implementation of it takes the same
// stop decisions: BF16 inputs and first-layer outputs, fused multiply-adds in
// increasing input index (a product of two BF16 values is exact in FP32), and
// a halving tree over the 64 output-layer products.
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

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_bits(x) << 16); }
// BF16 element 2t (low half) and 2t + 1 (high half) of a packed word.
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// The first-layer weights lane j needs (row j of W1 as BF16 pairs, b1[j],
// b2[j], w3[j], b3): 8 words and 4 floats, read with two 16-byte loads and four
// 2-byte loads. The second layer's row (32 words) is read in chunks while it
// is used, so that few registers are held at once.
struct MlpRegs {
    uint32_t w1[8];
    float b1, b2, w3, b3;
};

__device__ __forceinline__ MlpRegs mlp_load(const uint16_t *W) {
    const int j = (int)threadIdx.x & 63;
    MlpRegs M;
    const uint4 *w1 = reinterpret_cast<const uint4 *>(W + OFF_W1 + j * MLP_IN);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint4 u = w1[t];
        M.w1[4 * t] = u.x; M.w1[4 * t + 1] = u.y; M.w1[4 * t + 2] = u.z; M.w1[4 * t + 3] = u.w;
    }
    M.b1 = bf16_val(W[OFF_B1 + j]);
    M.b2 = bf16_val(W[OFF_B2 + j]);
    M.w3 = bf16_val(W[OFF_W3 + j]);
    M.b3 = bf16_val(W[OFF_B3]);
    return M;
}

// Logit of one feature row: x_t = bf16(fs_t); h1_j = bf16(relu(b1_j + sum_t
// W1_jt x_t)) and h2_j = relu(b2_j + sum_t W2_jt h1_t), each sum a chain of
// fused multiply-adds in increasing t; p_j = w3_j * h2_j, summed by the
// halving tree p_j += p_(j+w) for w = 32, 16, 8, 4, 2, 1; logit = p_0 + b3.
// relu(s) = s for s > 0, else +0. Every lane returns the same value. Lane
// t < 16 holds standardised feature t in `fs`. hbuf: 64 floats of LDS owned
// by the wave, 16-byte aligned. W: the BF16 weights (device).
__device__ __forceinline__ float mlp_logit(const MlpRegs &M, const uint16_t *W, float fs, float *hbuf) {
    const int j = (int)threadIdx.x & 63;
    const float xb = bf16_round(fs);
    float s = M.b1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float x0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, xb), 2 * t));
        const float x1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, xb), 2 * t + 1));
        s = __fmaf_rn(bf16_lo(M.w1[t]), x0, s);
        s = __fmaf_rn(bf16_hi(M.w1[t]), x1, s);
    }
    hbuf[j] = bf16_round(s > 0.0f ? s : 0.0f);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    const float4 *h4 = reinterpret_cast<const float4 *>(hbuf);
    const uint4 *w2 = reinterpret_cast<const uint4 *>(W + OFF_W2 + j * MLP_H);
    s = M.b2;
    uint4 wc = w2[0];  // 8 weights per chunk, the next chunk requested before this one is used
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
        const uint4 wn = c < 7 ? w2[c + 1] : wc;
        const float4 ha = h4[2 * c], hb = h4[2 * c + 1];
        s = __fmaf_rn(bf16_lo(wc.x), ha.x, s);
        s = __fmaf_rn(bf16_hi(wc.x), ha.y, s);
        s = __fmaf_rn(bf16_lo(wc.y), ha.z, s);
        s = __fmaf_rn(bf16_hi(wc.y), ha.w, s);
        s = __fmaf_rn(bf16_lo(wc.z), hb.x, s);
        s = __fmaf_rn(bf16_hi(wc.z), hb.y, s);
        s = __fmaf_rn(bf16_lo(wc.w), hb.z, s);
        s = __fmaf_rn(bf16_hi(wc.w), hb.w, s);
        wc = wn;
    }
    const float h2 = s > 0.0f ? s : 0.0f;
    float z = __fmul_rn(M.w3, h2);
    // lanes p < 32 add lane p + 32; then the 32-lane halving tree of the
    // distance reduction (swizzle for w = 16, row shifts for 8, 4, 2, 1)
    z = __fadd_rn(z, __shfl_xor(z, 32));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, z), 0x401F)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x108, 0xF, 0xF, true)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x104, 0xF, 0xF, true)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x102, 0xF, 0xF, true)));
    z = __fadd_rn(z, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, z), 0x101, 0xF, 0xF, true)));
    z = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, z), 0));
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    return __fadd_rn(z, M.b3);
}

}  // namespace degk
