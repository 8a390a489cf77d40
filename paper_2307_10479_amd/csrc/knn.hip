// Exact kNN ground truth (Eq. knn) by brute force on matrix cores.
//
// knn_tile_kernel: a workgroup (4 waves) takes 128 queries and one slice of the
//   base set, in tiles of 128 base rows. Each wave forms a 64 x 64 block of
//   inner products on the matrix cores:
//     - BF16 inputs (v_mfma_f32_32x32x16_bf16, FP32 accumulation) when every
//       query and base value is an integer of magnitude <= 255 and the
//       dimension is <= 129: every product, partial sum and norm-expanded
//       distance is then an exact integer below 2^24, so the candidates rank
//       exactly as the FP64 definition;
//     - FP32 inputs (v_mfma_f32_32x32x2f32) otherwise.
//   A device-side check decides (each kernel variant returns at once when the
//   other applies). The distances (L2: |q|^2 + |x|^2 - 2 q.x; IP: 1 - q.x) are
//   compared with each query row's running threshold in the accumulator
//   registers; the few that pass are appended to the row's list in the
//   workspace (LDS counters), and a list that is nearly full is cut to its KC
//   smallest keys, whose largest distance becomes the row's threshold.
// knn_final_kernel: one wave per query recomputes every candidate as a direct
//   FP32 difference in the fixed C32x4 order (the search's arithmetic), selects
//   the k smallest (distance, id) keys and sorts them (bitonic, in LDS).
#include <hip/hip_runtime.h>

#include "deg.h"
#include "search_kernel.h"

namespace degk {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int KQ = 128;    // queries per workgroup
constexpr int KN = 128;    // base rows per tile
constexpr int KCH = 32;    // dims per K chunk of the FP32 path
constexpr int KMARGIN = 32;
constexpr int BF16_MAX_DIM = 128;  // the exact BF16 path (it needs dims <= 129): rows of 128 BF16
constexpr int BF16_PAD = 128;
constexpr int BF16_LD = BF16_PAD + 8;  // LDS row pitch: consecutive rows start in different banks

struct KnnParams {
    const float *base;
    const float *queries;
    const uint16_t *base16;   // BF16 copy of the base rows (exact path), dpad per row
    int64_t n, nq, bstride, qstride;
    int32_t dim, dpad, k, kc, cap, nslices, metric;
    const int32_t *exclude;
    const float *bnorm, *qnorm;
    const int32_t *inexact;   // 0: the BF16 path is exact
    uint64_t *lists;   // nq x nslices x cap
    int32_t *counts;   // nq x nslices
    int32_t *out_ids;
    float *out_dists;
};

__global__ void row_norm_kernel(const float *x, int64_t n, int32_t dim, int64_t stride,
                                float *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *r = x + i * stride;
    float s = 0.0f;
    for (int c = 0; c < dim; ++c) s = __fmaf_rn(r[c], r[c], s);
    out[i] = s;
}

__global__ void flag_reset_kernel(int32_t *f) { *f = 0; }

// Sets *flag when a value of the n x dim rows is not an integer of magnitude
// <= 255 (NaN included).
__global__ void exact_check_kernel(const float *x, int64_t n, int32_t dim, int64_t stride,
                                   int32_t *flag) {
    const int64_t tot = n * dim;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = x[(i / dim) * stride + i % dim];
        bad |= !(v == rintf(v) && fabsf(v) <= 255.0f);
    }
    if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 1);
}

// BF16 copy of the base rows (exact for the values the BF16 path accepts),
// dpad elements per row, zero beyond dim; skipped when the data is inexact.
__global__ void to_bf16_kernel(const float *x, int64_t n, int32_t dim, int64_t stride, int32_t dpad,
                               uint16_t *out, const int32_t *inexact) {
    if (*inexact) return;
    const int64_t tot = n * dpad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dpad;
        const int c = (int)(i % dpad);
        const float v = c < dim ? x[r * stride + c] : 0.0f;
        out[i] = (uint16_t)(__float_as_uint(v) >> 16);  // exact: small integers
    }
}

// Cuts the `cnt` distinct keys of `buf` (global, one wave) to the kc smallest:
// the kc-th smallest key is built bit by bit from the top by counting the keys
// below each candidate prefix (the list is read from memory at each step), and
// the kept keys are written back compacted. Returns the kc-th key.
__device__ uint64_t cut_list(uint64_t *buf, int &cnt, int kc) {
    const int lane = lane_id();
    uint64_t ans = 0;
    for (int b = 63; b >= 0; --b) {
        const uint64_t cand = ans | (1ull << b);
        int c = 0;
        for (int i = lane; i < cnt; i += WAVE) c += buf[i] < cand ? 1 : 0;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
        if (c < kc) ans = cand;
    }
    int out = 0;
    for (int base = 0; base < cnt; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < cnt ? buf[i] : KEY_MAX;
        const bool keep = i < cnt && v <= ans;
        const uint64_t m = ballot(keep);
        wave_sync();
        __threadfence_block();
        if (keep) buf[out + prefix_in(m)] = v;
        out += __popcll(m);
        __threadfence_block();
    }
    cnt = out;
    return ans;
}

// cut_list with the list held in registers (R keys per lane, cnt <= 64 R): the
// same bit-by-bit construction of the kc-th key, counting with ballots instead
// of a pass over memory per bit.
template <int R>
__device__ uint64_t cut_list_regs(uint64_t *buf, int &cnt, int kc) {
    const int lane = lane_id();
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * WAVE + lane;
        v[r] = i < cnt ? buf[i] : KEY_MAX;
    }
    uint64_t ans = 0;
    for (int b = 63; b >= 0; --b) {
        const uint64_t cand = ans | (1ull << b);
        int c = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) c += __popcll(ballot(v[r] < cand));
        if (c < kc) ans = cand;
    }
    int out = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool keep = r * WAVE + lane < cnt && v[r] <= ans;
        const uint64_t m = ballot(keep);
        if (keep) buf[out + prefix_in(m)] = v[r];
        out += __popcll(m);
    }
    __threadfence_block();
    cnt = out;
    return ans;
}

__device__ __forceinline__ uint64_t cut_any(uint64_t *buf, int &cnt, int kc, int cap) {
    if (cap <= 4 * WAVE) return cut_list_regs<4>(buf, cnt, kc);
    if (cap <= 7 * WAVE) return cut_list_regs<7>(buf, cnt, kc);
    if (cap <= 16 * WAVE) return cut_list_regs<16>(buf, cnt, kc);
    if (cap <= 36 * WAVE) return cut_list_regs<36>(buf, cnt, kc);
    return cut_list(buf, cnt, kc);
}

// Tile kernel. Wave w computes queries 64 (w >> 1) + [0, 64) against base rows
// 64 (w & 1) + [0, 64) of the tile as 2 x 2 blocks of 32 x 32; in a block's
// accumulator, lane l register v holds row 8 (v / 4) + 4 (l / 32) + v % 4 and
// column l % 32.
template <int METRIC, bool BF>
__global__ void __launch_bounds__(256) knn_tile_kernel(KnnParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (BF ? (*P.inexact != 0) : (*P.inexact == 0 && P.dim <= BF16_MAX_DIM)) return;
    const int t = threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    const int wq = w >> 1, wn = w & 1;
    const int64_t q0 = (int64_t)blockIdx.x * KQ;
    const int slice = blockIdx.y;
    const int64_t per = (P.n + P.nslices - 1) / P.nslices;
    const int64_t n0 = (int64_t)slice * per;
    const int64_t n1 = min(P.n, n0 + per);
    // LDS: per-row list counters, distance thresholds and excluded ids, two block
    // flags, then the operand tiles
    int32_t *rcnt = reinterpret_cast<int32_t *>(smem);               // KQ
    float *rthr = reinterpret_cast<float *>(smem + 4 * KQ);          // KQ
    int32_t *rex = reinterpret_cast<int32_t *>(smem + 8 * KQ);       // KQ
    // block flags: [0] a list came near its capacity this tile, [1] a threshold changed
    int32_t *bflag = reinterpret_cast<int32_t *>(smem + 12 * KQ);
    unsigned char *tiles = smem + 12 * KQ + 16;
    for (int i = t; i < KQ; i += 256) {
        rcnt[i] = 0;
        rthr[i] = __builtin_inff();
        rex[i] = (P.exclude && q0 + i < P.nq) ? P.exclude[q0 + i] : -1;
    }
    if (t < 4) bflag[t] = 0;
    // the distance thresholds of this lane's accumulator rows, held in registers and
    // re-read from LDS only after a cut changed one
    float thr[2][16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = 64 * wq + 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            thr[bi][v] = q0 + row < P.nq ? __builtin_inff() : -__builtin_inff();
        }
    // query norms of the rows this lane's accumulator registers hold
    float qn[2][16];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = 64 * wq + 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int64_t qi = q0 + row;
            qn[bi][v] = (METRIC == DEG_METRIC_L2 && qi < P.nq) ? P.qnorm[qi] : 0.0f;
        }

    // ---- operand staging
    // BF16: each wave keeps the A operands of its 64 queries in registers for the
    //       whole slice (8 k-steps of 16 dims); the tile's base rows (BF16, 128
    //       per row) are loaded as 16-byte chunks one tile ahead into LDS.
    // FP32: chunks of 32 dims, k-major ([k][row + 1]), one chunk ahead.
    uint16_t *B16 = reinterpret_cast<uint16_t *>(tiles);
    float *QsT = reinterpret_cast<float *>(tiles);
    float *BsT = QsT + KCH * (KQ + 1);
    constexpr int NB16 = (KN * BF16_PAD * 2) / (256 * 16);  // 16-byte chunks per thread (8)
    constexpr int NCK = BF16_PAD / 8;                         // 16-byte chunks per row
    uint4 rb16[BF ? NB16 : 1];
    bf16x8 A16[BF ? 2 : 1][BF ? BF16_PAD / 16 : 1];
    float4 rq[4], rb[4];

    auto fetch16 = [&](int64_t bt) {
#pragma unroll
        for (int j = 0; j < NB16; ++j) {
            const int idx = t + 256 * j;           // chunk index within the tile
            const int r = idx / NCK, c = idx % NCK;
            const int64_t bi = bt + r;
            rb16[j] = bi < n1 ? reinterpret_cast<const uint4 *>(P.base16 + bi * BF16_PAD)[c]
                              : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto stage16 = [&]() {
#pragma unroll
        for (int j = 0; j < NB16; ++j) {
            const int idx = t + 256 * j;
            const int r = idx / NCK, c = idx % NCK;
            *reinterpret_cast<uint4 *>(B16 + r * BF16_LD + 8 * c) = rb16[j];
        }
    };
    auto fetch32 = [&](int64_t bt, int k0) {
        // queries: row t / 2, dims k0 + 16 (t % 2) .. +16
        {
            const int r = t >> 1, dq = (t & 1) * 16;
            const int64_t qi = q0 + r;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = k0 + dq + 4 * j + e;
                    v[e] = (qi < P.nq && c < P.dim) ? P.queries[qi * P.qstride + c] : 0.0f;
                }
                rq[j] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
        {
            const int r = t >> 1, dq = (t & 1) * 16;
            const int64_t bi = bt + r;
            if (bi < n1 && k0 + dq + 16 <= P.dim) {  // rows are 16-byte aligned (b_stride % 4 == 0)
                const float4 *src = reinterpret_cast<const float4 *>(P.base + bi * P.bstride + k0 + dq);
#pragma unroll
                for (int j = 0; j < 4; ++j) rb[j] = src[j];
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = k0 + dq + 4 * j + e;
                        v[e] = (bi < n1 && c < P.dim) ? P.base[bi * P.bstride + c] : 0.0f;
                    }
                    rb[j] = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
        }
    };
    auto stage32 = [&]() {
        const int r = t >> 1, dq = (t & 1) * 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            QsT[(dq + 4 * j + 0) * (KQ + 1) + r] = rq[j].x;
            QsT[(dq + 4 * j + 1) * (KQ + 1) + r] = rq[j].y;
            QsT[(dq + 4 * j + 2) * (KQ + 1) + r] = rq[j].z;
            QsT[(dq + 4 * j + 3) * (KQ + 1) + r] = rq[j].w;
            BsT[(dq + 4 * j + 0) * (KN + 1) + r] = rb[j].x;
            BsT[(dq + 4 * j + 1) * (KN + 1) + r] = rb[j].y;
            BsT[(dq + 4 * j + 2) * (KN + 1) + r] = rb[j].z;
            BsT[(dq + 4 * j + 3) * (KN + 1) + r] = rb[j].w;
        }
    };

    if (BF) {
        // A operands: lane l of block bi, k-step s holds query row 32 bi + l % 32 of
        // the wave, dims 16 s + 8 (l / 32) .. + 7, as BF16 (exact), zero beyond dim
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            const int64_t qi = q0 + 64 * wq + 32 * bi + (lane & 31);
#pragma unroll
            for (int ks = 0; ks < BF16_PAD / 16; ++ks) {
                uint32_t wd[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c0 = 16 * ks + 8 * (lane >> 5) + 2 * e;
                    const float v0 = (qi < P.nq && c0 < P.dim) ? P.queries[qi * P.qstride + c0] : 0.0f;
                    const float v1 = (qi < P.nq && c0 + 1 < P.dim) ? P.queries[qi * P.qstride + c0 + 1] : 0.0f;
                    wd[e] = (__float_as_uint(v0) >> 16) | (__float_as_uint(v1) & 0xffff0000u);
                }
                A16[bi][ks] = __builtin_bit_cast(bf16x8, make_uint4(wd[0], wd[1], wd[2], wd[3]));
            }
        }
        if (n0 < n1) fetch16(n0);
    } else {
        if (n0 < n1) fetch32(n0, 0);
    }
    __syncthreads();

    // the norm term of this lane's base columns (a column past the slice gets a NaN
    // term: its distance fails every test), one tile ahead
    float bnc[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int64_t c = n0 + 64 * wn + 32 * bj + (lane & 31);
        bnc[bj] = c < n1 ? (METRIC == DEG_METRIC_L2 ? P.bnorm[c] : 0.0f) : __builtin_nanf("");
    }
    for (int64_t b0 = n0; b0 < n1; b0 += KN) {
        floatx16 acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[bi][bj][v] = 0.0f;
        if (BF) {
            stage16();
            __syncthreads();
            if (b0 + KN < n1) fetch16(b0 + KN);
            const int g = lane >> 5, c32 = lane & 31;
#pragma unroll
            for (int ks = 0; ks < BF16_PAD / 16; ++ks) {
                bf16x8 b[2];
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    b[bj] = *reinterpret_cast<const bf16x8 *>(B16 + (64 * wn + 32 * bj + c32) * BF16_LD +
                                                              16 * ks + 8 * g);
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A16[bi][ks], b[bj],
                                                                              acc[bi][bj], 0, 0, 0);
            }
        } else {
            for (int k0 = 0; k0 < P.dim; k0 += KCH) {
                stage32();
                __syncthreads();
                if (k0 + KCH < P.dim)
                    fetch32(b0, k0 + KCH);
                else if (b0 + KN < n1)
                    fetch32(b0 + KN, 0);
#pragma unroll 4
                for (int kk = 0; kk < KCH; kk += 2) {
                    const int kr = kk + (lane >> 5);
                    float a[2], b[2];
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi) a[bi] = QsT[kr * (KQ + 1) + 64 * wq + 32 * bi + (lane & 31)];
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) b[bj] = BsT[kr * (KN + 1) + 64 * wn + 32 * bj + (lane & 31)];
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj)
                            acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
                }
                __syncthreads();
            }
        }

        // ---- epilogue in the accumulator layout: distance, threshold test, append
        float bn[2];
        int64_t cid[2];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cid[bj] = b0 + 64 * wn + 32 * bj + (lane & 31);
            bn[bj] = bnc[bj];
            // the next tile's norm is requested now and used a tile later
            const int64_t cn = cid[bj] + KN;
            bnc[bj] = cn < n1 ? (METRIC == DEG_METRIC_L2 ? P.bnorm[cn] : 0.0f) : __builtin_nanf("");
        }
        bool any = false;
        uint32_t passm[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                uint32_t pm = 0;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = 64 * wq + 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const float dot = acc[bi][bj][v];
                    float d;
                    if (METRIC == DEG_METRIC_L2)
                        d = __fsub_rn(__fadd_rn(qn[bi][v], bn[bj]), __fmul_rn(2.0f, dot));
                    else
                        d = __fadd_rn(__fsub_rn(1.0f, dot), bn[bj]);
                    acc[bi][bj][v] = d;
                    const bool ok = d <= thr[bi][v];  // (rows past the queries hold -inf)
                    pm |= ok ? (1u << v) : 0u;
                }
                passm[bi][bj] = pm;
                any |= pm != 0;
            }
        }
        if (ballot(any) != 0) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    for (uint32_t pm = passm[bi][bj]; pm; pm &= pm - 1) {
                        const int v = __builtin_ctz(pm);
                        const int row = 64 * wq + 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                        if ((int32_t)cid[bj] == rex[row]) continue;  // kept out of this query's answer
                        const int pos = atomicAdd(&rcnt[row], 1);
                        if (pos + 1 > P.cap - KN) bflag[0] = 1;
                        P.lists[((q0 + row) * P.nslices + slice) * P.cap + pos] =
                            make_key(acc[bi][bj][v], (int32_t)cid[bj]);
                    }
        }
        __threadfence_block();
        __syncthreads();
        // lists that another tile could overflow are cut to their KC smallest keys
        // (only when an append of this tile came that near)
        if (bflag[0] != 0) {
            for (int rr = 0; rr < KQ / 4; ++rr) {
                const int row = w * (KQ / 4) + rr;
                int c = rcnt[row];
                if (c > P.cap - KN && q0 + row < P.nq) {
                    uint64_t *lst = P.lists + ((q0 + row) * P.nslices + slice) * P.cap;
                    const uint64_t th = cut_any(lst, c, P.kc, P.cap);
                    if (lane == 0) {
                        rcnt[row] = c;
                        rthr[row] = key_dist(th);
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
            if (t == 0) bflag[0] = 0;
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = 64 * wq + 32 * bi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    thr[bi][v] = q0 + row < P.nq ? rthr[row] : -__builtin_inff();
                }
            __syncthreads();
        }
    }
    // final cut to KC and the list sizes
    for (int rr = 0; rr < KQ / 4; ++rr) {
        const int row = w * (KQ / 4) + rr;
        const int64_t qi = q0 + row;
        if (qi >= P.nq) break;
        int c = rcnt[row];
        uint64_t *lst = P.lists + (qi * P.nslices + slice) * P.cap;
        if (c > P.kc) cut_any(lst, c, P.kc, P.cap);
        if (lane == 0) P.counts[qi * P.nslices + slice] = c;
    }
}

// Sorts n8 (a power of two, >= 2) keys in LDS ascending (bitonic network, one wave).
__device__ void bitonic_sort(uint64_t *a, int n8) {
    const int lane = lane_id();
    for (int size = 2; size <= n8; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            wave_sync();
            for (int i = lane; i < n8 / 2; i += WAVE) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            wave_sync();
        }
    }
}

template <int METRIC, int QCH>
__global__ void __launch_bounds__(64) knn_final_kernel(KnnParams P, int p2) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *top = reinterpret_cast<uint64_t *>(smem);        // p2 (power of two >= k)
    int32_t *hist = reinterpret_cast<int32_t *>(top + p2);     // 256 bins
    const int lane = lane_id(), p = lane & 31;
    const int64_t qi = blockIdx.x;
    if (qi >= P.nq) return;
    SearchParams SP;
    SP.f32 = P.base;
    SP.f32_stride = (int32_t)P.bstride;
    SP.dim = P.dim;
    const int nch = (P.dim + 3) >> 2;
    const bool mask_tail = (P.dim & 3) != 0;
    float4 qv[QCH];
    const float *qp = P.queries + qi * P.qstride;
#pragma unroll
    for (int c = 0; c < QCH; ++c) {
        int b = 4 * (p + 32 * c);
        qv[c] = make_float4(b + 0 < P.dim ? qp[b + 0] : 0.f, b + 1 < P.dim ? qp[b + 1] : 0.f,
                            b + 2 < P.dim ? qp[b + 2] : 0.f, b + 3 < P.dim ? qp[b + 3] : 0.f);
    }
    // exact FP32 distances of every candidate, written back compacted at the start of
    // the query's own list region (slice s is read at s * cap, and the keys written
    // so far end at or before s * kc < s * cap: a write never overtakes a read)
    uint64_t *keys = P.lists + qi * P.nslices * P.cap;
    int tot = 0;
    for (int s = 0; s < P.nslices; ++s) {
        const uint64_t *lst = P.lists + (qi * P.nslices + s) * P.cap;
        int c = P.counts[qi * P.nslices + s];
        for (int b = 0; b < c; b += WAVE) {
            int nc = min(WAVE, c - b);
            int32_t id = lane < nc ? key_id(lst[b + lane]) : 0;
            uint64_t msk = nc == WAVE ? ~0ull : ((1ull << nc) - 1ull);
            float d = batch_dist<DT_F32, METRIC, QCH, true>(SP, qv, id, msk, nch, mask_tail);
            if (lane < nc) keys[tot + lane] = make_key(d, id);
            tot += nc;
        }
    }
    __threadfence_block();
    wave_sync();
    // the k smallest keys, then sorted: the k-th smallest key (keys are distinct) is
    // found one byte at a time, most significant first, from a 256-bin histogram of
    // the keys that share the bytes fixed so far
    const int kk = min(P.k, tot);
    uint64_t kth = KEY_MAX;
    if (tot > kk) {
        uint64_t prefix = 0;
        int need = kk;  // rank of the wanted key among those sharing `prefix`
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            const uint64_t hmask = pass == 0 ? 0ull : (~0ull << (shift + 8));
            for (int i = lane; i < 256; i += WAVE) hist[i] = 0;
            wave_sync();
            for (int i = lane; i < tot; i += WAVE) {
                const uint64_t v = keys[i];
                if ((v & hmask) == prefix) atomicAdd(&hist[(int)((v >> shift) & 255u)], 1);
            }
            wave_sync();
            // lane l holds bins 4l .. 4l + 3; an inclusive scan over the lanes
            const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1];
            const int h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
            const int own = h0 + h1 + h2 + h3;
            int inc = own;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const int t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            const int exc = inc - own;
            const uint64_t hit = ballot(exc < need && need <= inc);
            const int hl = (int)__builtin_ctzll(hit);
            int r = need - exc, dg = 4 * lane;
            if (r > h0) { r -= h0; dg += 1;
                if (r > h1) { r -= h1; dg += 1;
                    if (r > h2) { r -= h2; dg += 1; } } }
            need = __shfl(r, hl);
            prefix |= (uint64_t)__shfl(dg, hl) << shift;
            wave_sync();
        }
        kth = prefix;
    }
    int out = 0;
    for (int base = 0; base < tot; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < tot ? keys[i] : KEY_MAX;
        const bool keep = i < tot && v <= kth;
        const uint64_t m = ballot(keep);
        if (keep) top[out + prefix_in(m)] = v;
        out += __popcll(m);
    }
    for (int i = out + lane; i < p2; i += WAVE) top[i] = KEY_MAX;
    wave_sync();
    bitonic_sort(top, p2);
    for (int i = lane; i < P.k; i += WAVE) {
        const bool have = i < kk;
        P.out_ids[qi * P.k + i] = have ? key_id(top[i]) : -1;
        P.out_dists[qi * P.k + i] = have ? key_dist(top[i]) : __builtin_inff();
    }
}

static int pow2_ge(int x) {
    int p = 2;
    while (p < x) p <<= 1;
    return p;
}

// Slices of the base set: enough workgroups to fill the chip (about 4 per CU),
// at least 4 tiles per slice, and no more candidates for the final kernel
// (slices x KC keys of 8 bytes) than about 60 KiB next to the sorted top: each
// slice adds KC exact distances per query to recompute and select (at k = 1000,
// thirteen slices instead of six took the whole search from 61 to 105 ms).
static int knn_slices(int64_t n, int64_t nq, int32_t k) {
    int64_t qb = (nq + KQ - 1) / KQ;
    int64_t want = (4 * 256 + qb - 1) / qb;
    int64_t maxs = (n + 4 * KN - 1) / (4 * KN);
    int64_t maxl = (60 * 1024 - 8 * (int64_t)pow2_ge(k)) / (8 * (int64_t)(k + KMARGIN));
    if (want > maxs) want = maxs;
    if (want > maxl) want = maxl;
    if (want > 64) want = 64;
    if (want < 1) want = 1;
    return (int)want;
}

static int32_t bf16_pad(int32_t dim) { return (dim + 15) / 16 * 16; }

}  // namespace degk

using namespace degk;

extern "C" size_t deg_knn_workspace_bytes(int64_t n, int32_t dim, int64_t nq, int32_t k) {
    if (n < 1 || nq < 0 || k < 1 || dim < 1) return 0;
    int ns = knn_slices(n, nq, k);
    int64_t kc = k + KMARGIN;
    int64_t cap = 2 * kc + KN;
    size_t b16 = dim <= BF16_MAX_DIM ? (size_t)n * BF16_PAD * 2 : 0;
    size_t off = 256 + (size_t)n * 4 + (size_t)nq * 4 + (size_t)nq * ns * 4;
    off = (off + 255) / 256 * 256 + (b16 + 255) / 256 * 256;
    return off + (size_t)nq * ns * cap * 8;
}

extern "C" deg_status deg_knn_bruteforce(const float *base, int64_t n, int32_t dim,
                                         int64_t b_stride, const float *queries, int64_t nq,
                                         int64_t q_stride, int32_t k, int32_t metric,
                                         const int32_t *exclude_ids, int32_t *out_ids,
                                         float *out_dists, void *workspace, size_t ws_bytes,
                                         void *stream) {
    if (!base || n < 1 || dim < 1 || b_stride < dim || (b_stride & 3) || nq < 0 || k < 1 ||
        k > 1024 || (metric != DEG_METRIC_L2 && metric != DEG_METRIC_IP))
        return DEG_ERR_INVALID_ARG;
    if (nq > 0 && (!queries || q_stride < dim || !out_ids || !out_dists)) return DEG_ERR_INVALID_ARG;
    if (((dim + 3) / 4 + 31) / 32 > 12 || n > 0x7fffffffLL) return DEG_ERR_UNSUPPORTED;
    if (nq == 0) return DEG_OK;
    size_t need = deg_knn_workspace_bytes(n, dim, nq, k);
    if (!workspace || ws_bytes < need) return DEG_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    KnnParams P;
    P.base = base;
    P.queries = queries;
    P.n = n;
    P.nq = nq;
    P.bstride = b_stride;
    P.qstride = q_stride;
    P.dim = dim;
    P.dpad = bf16_pad(dim);
    P.k = k;
    P.kc = k + KMARGIN;
    P.cap = 2 * P.kc + KN;
    P.nslices = knn_slices(n, nq, k);
    P.metric = metric;
    P.exclude = exclude_ids;
    char *w = reinterpret_cast<char *>(workspace);
    int32_t *flag = reinterpret_cast<int32_t *>(w);
    float *bn = reinterpret_cast<float *>(w + 256);
    float *qn = bn + n;
    int32_t *counts = reinterpret_cast<int32_t *>(qn + nq);
    size_t off = 256 + (size_t)n * 4 + (size_t)nq * 4 + (size_t)nq * P.nslices * 4;
    off = (off + 255) / 256 * 256;
    const bool try16 = dim <= BF16_MAX_DIM;
    size_t b16 = try16 ? (size_t)n * BF16_PAD * 2 : 0;
    P.base16 = reinterpret_cast<const uint16_t *>(w + off);
    off += (b16 + 255) / 256 * 256;
    P.bnorm = bn;
    P.qnorm = qn;
    P.counts = counts;
    P.inexact = flag;
    P.lists = reinterpret_cast<uint64_t *>(w + off);
    if (off + (size_t)nq * P.nslices * P.cap * 8 > ws_bytes) return DEG_ERR_WORKSPACE;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    hipLaunchKernelGGL(row_norm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, base, n,
                       dim, b_stride, bn);
    hipLaunchKernelGGL(row_norm_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st,
                       queries, nq, dim, q_stride, qn);
    hipLaunchKernelGGL(flag_reset_kernel, dim3(1), dim3(1), 0, st, flag);
    dim3 g1((unsigned)((nq + KQ - 1) / KQ), (unsigned)P.nslices);
    if (try16) {
        hipLaunchKernelGGL(exact_check_kernel, dim3(2048), dim3(256), 0, st, base, n, dim, b_stride,
                           flag);
        hipLaunchKernelGGL(exact_check_kernel, dim3(256), dim3(256), 0, st, queries, nq, dim,
                           q_stride, flag);
        hipLaunchKernelGGL(to_bf16_kernel, dim3(4096), dim3(256), 0, st, base, n, dim, b_stride,
                           BF16_PAD, const_cast<uint16_t *>(P.base16), flag);
        const size_t lds16 = 12 * KQ + 16 + (size_t)KN * BF16_LD * 2;
        void (*t16)(KnnParams) = metric == DEG_METRIC_L2 ? knn_tile_kernel<DEG_METRIC_L2, true>
                                                         : knn_tile_kernel<DEG_METRIC_IP, true>;
        hipLaunchKernelGGL(t16, g1, dim3(256), lds16, st, P);
    }
    const size_t lds32 = 12 * KQ + 16 + (size_t)KCH * (KQ + 1) * 4 + (size_t)KCH * (KN + 1) * 4;
    void (*t32)(KnnParams) = metric == DEG_METRIC_L2 ? knn_tile_kernel<DEG_METRIC_L2, false>
                                                     : knn_tile_kernel<DEG_METRIC_IP, false>;
    hipLaunchKernelGGL(t32, g1, dim3(256), lds32, st, P);
    int q = ((dim + 3) / 4 + 31) / 32;
    int qch = q <= 1 ? 1 : (q <= 2 ? 2 : (q <= 4 ? 4 : 12));
    const int p2 = pow2_ge(k);
    size_t lds = (size_t)p2 * 8 + 256 * 4;
    void (*fn)(KnnParams, int) = nullptr;
    if (metric == DEG_METRIC_L2)
        fn = qch == 1 ? knn_final_kernel<DEG_METRIC_L2, 1>
                      : (qch == 2 ? knn_final_kernel<DEG_METRIC_L2, 2>
                                  : (qch == 4 ? knn_final_kernel<DEG_METRIC_L2, 4>
                                              : knn_final_kernel<DEG_METRIC_L2, 12>));
    else
        fn = qch == 1 ? knn_final_kernel<DEG_METRIC_IP, 1>
                      : (qch == 2 ? knn_final_kernel<DEG_METRIC_IP, 2>
                                  : (qch == 4 ? knn_final_kernel<DEG_METRIC_IP, 4>
                                              : knn_final_kernel<DEG_METRIC_IP, 12>));
    if (lds > 64 * 1024) return DEG_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(fn, dim3((unsigned)nq), dim3(64), lds, st, P, p2);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}
