// Stop-predictor MLP (16 -> 64 -> 64 -> 1, ReLU, logit) evaluated by one
// wavefront: lane j owns hidden unit j of both layers. Inference uses the
// gfx950 BF16 dot-product instruction (two products per instruction, FP32
// accumulation).
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

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// acc + a.lo * b.lo + a.hi * b.hi with BF16 pairs packed in 32-bit words
// (element 2t in the low half); the products are exact in FP32.
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a),
                                           __builtin_bit_cast(bf16x2_t, b), acc, false);
}

// The weights lane j needs (row j of W1 and W2 as BF16 pairs, b1[j], b2[j],
// w3[j], b3) in registers: 40 words and 4 floats per lane, read with ten
// 16-byte loads and four 2-byte loads.
struct MlpRegs {
    uint32_t w1[8];
    uint32_t w2[32];
    float b1, b2, w3, b3;
};

__device__ __forceinline__ MlpRegs mlp_load(const uint16_t *W) {
    const int j = (int)threadIdx.x & 63;
    MlpRegs M;
    const uint4 *w1 = reinterpret_cast<const uint4 *>(W + OFF_W1 + j * MLP_IN);
    const uint4 *w2 = reinterpret_cast<const uint4 *>(W + OFF_W2 + j * MLP_H);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint4 u = w1[t];
        M.w1[4 * t] = u.x; M.w1[4 * t + 1] = u.y; M.w1[4 * t + 2] = u.z; M.w1[4 * t + 3] = u.w;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const uint4 u = w2[t];
        M.w2[4 * t] = u.x; M.w2[4 * t + 1] = u.y; M.w2[4 * t + 2] = u.z; M.w2[4 * t + 3] = u.w;
    }
    M.b1 = bf16_val(W[OFF_B1 + j]);
    M.b2 = bf16_val(W[OFF_B2 + j]);
    M.w3 = bf16_val(W[OFF_W3 + j]);
    M.b3 = bf16_val(W[OFF_B3]);
    return M;
}

// Logit of one feature row, BF16 inference: BF16 weights, the inputs of the
// two hidden layers rounded to BF16, FP32 accumulation; the output layer
// takes the FP32 activations. Every lane returns the same value. Lane i < 16
// holds standardised feature i in `fs`. hbuf: 64 BF16 values (128 bytes) of
// LDS owned by the wave, 16-byte aligned.
__device__ __forceinline__ float mlp_logit(const MlpRegs &M, float fs, uint16_t *hbuf) {
    const int j = (int)threadIdx.x & 63;
    // layer 1: feature pairs (2t, 2t+1) gathered into lane 2t, broadcast by readlane
    const uint32_t fb = bf16_bits(fs);
    const uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)fb, 0x101, 0xF, 0xF, false);  // lane + 1
    const uint32_t pair = fb | (nb << 16);
    float s = M.b1;
#pragma unroll
    for (int t = 0; t < 8; ++t) s = dot2(M.w1[t], (uint32_t)__builtin_amdgcn_readlane((int)pair, 2 * t), s);
    hbuf[j] = (uint16_t)bf16_bits(fmaxf(s, 0.0f));
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    // layer 2: the 64 hidden values as 32 BF16 pairs from LDS
    const uint4 *h4 = reinterpret_cast<const uint4 *>(hbuf);
    s = M.b2;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const uint4 h = h4[t];
        s = dot2(M.w2[4 * t], h.x, s);
        s = dot2(M.w2[4 * t + 1], h.y, s);
        s = dot2(M.w2[4 * t + 2], h.z, s);
        s = dot2(M.w2[4 * t + 3], h.w, s);
    }
    const float h2 = fmaxf(s, 0.0f);
    float z = __fmul_rn(M.w3, h2);
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
    return __fadd_rn(z, M.b3);
}

}  // namespace degk
