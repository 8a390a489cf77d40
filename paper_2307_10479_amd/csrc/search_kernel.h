// Device code of the DEG range search (Algorithm 1) for gfx950.
//
// One wavefront (64 lanes) runs one query at a time; a persistent grid pulls
// queries from a device counter. Per-wave state:
//   visited set C   open-addressing int32 hash in LDS; at 3/4 load it moves to
//                   the wave's workspace tables (16384, 65536, 262144 slots,
//                   each left at 3/8 load), then to a shared table sized for
//                   all n vertices: exact for any number of checked vertices
//   candidates S    keys (orderable distance bits << 32 | id, so one 64-bit
//                   compare is the (distance, id) order) in three levels: the
//                   64 smallest sorted across the lanes' registers, the next
//                   ones unsorted in LDS, the rest in the wave's workspace;
//                   capacity L
//   results R       sorted keys in registers, RREG per lane (up to 64*RREG)
// Each hop expands one row: the adjacency row is read by `degree` lanes (two
// parts of up to 64 for longer rows), the unchecked ids are compacted through
// LDS, and each half-wave computes one distance at a time with 32 partial sums
// (lane p of the half owns chunks p, p+32, ...), reduced by a swizzle and DPP
// halving tree that pairs the partials of the fixed order, so the result is the
// exact fixed-order sum.
//
// A row is merged as one batch (or one batch per part). This gives the same
// ids, hops and evaluations as the sequential loop of Algorithm 1: R after a
// row is the top-k of R plus the row's candidates; a candidate the batch keeps
// out of S (distance above the end-of-row threshold) could never be expanded,
// because the radius only shrinks; and entries above the threshold are dropped
// from S before any live entry is evicted for capacity.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "deg.h"

namespace degk {

constexpr int WAVE = 64;
constexpr uint64_t KEY_MAX = ~0ull;

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };
enum { MODE_VEC = 0, MODE_INDEXED = 1, MODE_BATCH = 2 };

// Trace row layout (floats): 16 features, label, query index, hop, reserved.
constexpr int TRACE_W = 20;
constexpr int NFEAT = 16;

struct SearchParams {
    // vectors
    const void *vec;
    const float *scale;
    const float *f32;
    int64_t n;
    int32_t dim;
    int32_t vstride;
    int32_t f32_stride;
    // graph
    const int32_t *adj;
    int32_t degree;
    int32_t astride;
    // queries
    int32_t mode;
    const float *queries;
    int64_t qstride;
    const int32_t *seeds;
    int32_t nseeds;
    const int32_t *qids;
    const deg_query_desc *descs;
    int64_t nq;
    int32_t k;
    int32_t kpool;  // traversal pool (>= k); batch: used when > descriptor k
    float eps;
    int32_t rerank;
    // state sizes
    int32_t L;      // capacity of S
    int32_t bcap;   // LDS part of S beyond the 64 keys in registers (>= 256)
    int32_t scap;   // LDS slots of the S array (>= bcap and >= the pool, for the rerank)
    int64_t gcap;   // workspace part of S per wave (keys)
    int64_t nqrows; // rows of `queries` (batch mode bound check)
    int32_t H;      // LDS hash slots (power of 2)
    int32_t hshift; // 32 - log2(H)
    // workspace visited tables: each wave owns a region holding tables of
    // hg0, 4 hg0, 16 hg0, ... slots up to hg_priv; beyond that a query takes
    // one of npool shared tables of hg_cap slots (3/4 of hg_cap >= n)
    int32_t hg0;
    int32_t hg_priv;
    int32_t hg_cap;
    int64_t region; // slots per wave region
    int32_t npool;
    // outputs
    int32_t *out_ids;
    float *out_dists;
    int32_t *out_stats;
    // workspace
    int32_t *counter;
    int32_t *spill;      // the per-wave regions
    int32_t *pool;       // npool tables of hg_cap slots
    int32_t *pool_owner; // npool words: 0 free, 1 taken
    uint64_t *gspace;    // per wave gcap keys: the far part of S
    // per-query exclusion lists (CSR over queries; nullable)
    const int64_t *ex_off;
    const int32_t *ex_ids;
    // learned stop
    const uint16_t *stop_w;
    const float *stop_mean;
    const float *stop_istd;
    float stop_tau;
    int32_t stop_interval;
    float stop_tau_long;
    int32_t stop_long_hops;
    // trace
    float *trace;
    int64_t trace_rows;
    int32_t trace_interval;
};

// ---------------------------------------------------------------- keys
__device__ __forceinline__ uint32_t ord_of(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;  // -0 orders as +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float f_of_ord(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t make_key(float d, int32_t id) {
    return ((uint64_t)ord_of(d) << 32) | (uint32_t)id;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return f_of_ord((uint32_t)(k >> 32)); }
__device__ __forceinline__ int32_t key_id(uint64_t k) { return (int32_t)(uint32_t)k; }

// ---------------------------------------------------------------- wave helpers
// Lanes of one wavefront communicate through LDS, which executes a wave's
// instructions in order; only the compiler must not move LDS accesses across
// such a point, so wave_sync is a code-motion barrier, not a memory fence.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
}
__device__ __forceinline__ int lane_id() { return (int)threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int prefix_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t v, int l) {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor((int)(uint32_t)v, m);
    uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | (uint32_t)lo;
}
// Rotate within rows of 16 lanes by R (DPP row_ror); lanes keep their own
// value where the source is masked.
template <int R>
__device__ __forceinline__ uint64_t row_ror_u64(uint64_t v) {
    int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, 0x120 + R, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), 0x120 + R,
                                         0xF, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
// Wave minimum / maximum of a 64-bit key (idempotent: rotations within the
// four rows of 16 lanes, then the four row results through readlane).
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    uint64_t o;
    o = row_ror_u64<8>(v); v = o < v ? o : v;
    o = row_ror_u64<4>(v); v = o < v ? o : v;
    o = row_ror_u64<2>(v); v = o < v ? o : v;
    o = row_ror_u64<1>(v); v = o < v ? o : v;
    uint64_t a = read_lane_u64(v, 0), b = read_lane_u64(v, 16);
    uint64_t c = read_lane_u64(v, 32), d = read_lane_u64(v, 48);
    a = b < a ? b : a;
    c = d < c ? d : c;
    return c < a ? c : a;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    uint64_t o;
    o = row_ror_u64<8>(v); v = o > v ? o : v;
    o = row_ror_u64<4>(v); v = o > v ? o : v;
    o = row_ror_u64<2>(v); v = o > v ? o : v;
    o = row_ror_u64<1>(v); v = o > v ? o : v;
    uint64_t a = read_lane_u64(v, 0), b = read_lane_u64(v, 16);
    uint64_t c = read_lane_u64(v, 32), d = read_lane_u64(v, 48);
    a = b > a ? b : a;
    c = d > c ? d : c;
    return c > a ? c : a;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);  // row_ror:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x122, 0xF, 0xF, false);  // row_ror:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x121, 0xF, 0xF, false);  // row_ror:1
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}
__device__ __forceinline__ float thr_of(float r, float onep) {
    // r (1 + eps) of Algorithm 1; infinity stays infinity
    if (__builtin_isinf(r) || __builtin_isinf(onep)) return __builtin_inff();
    return __fmul_rn(r, onep);
}

// ---------------------------------------------------------------- FP8 E4M3 decode
// Value of an OCP E4M3 code: exponent field 0 -> m * 2^-9, else
// (8 + m) * 2^(e - 10); every such value is exact in FP32. Code 0x7f/0xff
// (NaN) never occurs in an encoded store.
typedef float f32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- chunk loads
// Raw chunk storage per dtype: 16 B of FP32, 8 B of BF16, 4 B of FP8 codes.
template <int DT> struct RawChunk;
template <> struct RawChunk<DT_F32> { using T = float4; };
template <> struct RawChunk<DT_BF16> { using T = uint2; };
template <> struct RawChunk<DT_FP8> { using T = uint32_t; };

// Loads chunk `ch` (dims 4ch..4ch+3) of row `id` without decoding, so that the
// wait for the data is not forced right after the load.
template <int DT>
__device__ __forceinline__ typename RawChunk<DT>::T load_raw(const SearchParams &P, int32_t id, int ch) {
    if constexpr (DT == DT_F32) {
        return reinterpret_cast<const float4 *>(static_cast<const float *>(P.vec) +
                                                (int64_t)id * P.vstride)[ch];
    } else if constexpr (DT == DT_BF16) {
        return reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(P.vec) +
                                               (int64_t)id * P.vstride)[ch];
    } else {
        return reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(P.vec) +
                                                  (int64_t)id * P.vstride)[ch];
    }
}

template <int DT>
__device__ __forceinline__ float4 decode_raw(typename RawChunk<DT>::T u, float sc) {
    if constexpr (DT == DT_F32) {
        return u;
    } else if constexpr (DT == DT_BF16) {
        return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                           __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
    } else {
        // gfx950 converts OCP E4M3 in hardware (two codes per instruction, exact)
        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)u, false);
        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)u, true);
        return make_float4(__fmul_rn(sc, lo.x), __fmul_rn(sc, lo.y), __fmul_rn(sc, hi.x),
                           __fmul_rn(sc, hi.y));
    }
}

template <int METRIC>
__device__ __forceinline__ float acc_chunk(float acc, float4 x, float4 q) {
    if constexpr (METRIC == DEG_METRIC_L2) {
        float t;
        t = __fsub_rn(x.x, q.x); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(x.y, q.y); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(x.z, q.z); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(x.w, q.w); acc = __fmaf_rn(t, t, acc);
    } else {
        acc = __fmaf_rn(x.x, q.x, acc);
        acc = __fmaf_rn(x.y, q.y, acc);
        acc = __fmaf_rn(x.z, q.z, acc);
        acc = __fmaf_rn(x.w, q.w, acc);
    }
    return acc;
}

// Halving tree over the 32 lanes of a half-wave: step w adds the value of
// lane p + w to lane p, for w = 16 (swizzle), 8, 4, 2, 1 (DPP row shifts), so
// lane 0 of each half ends with ((p0 + p16) + (p8 + p24)) + ... exactly as the
// fixed order prescribes. Only lanes 0 and 32 hold the sum afterwards.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, true));
}
__device__ __forceinline__ float half_reduce(float a) {
    a = __fadd_rn(a, __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, a),
                                                                           0x401F)));
    a = __fadd_rn(a, dpp_row<0x108>(a));  // row_shl:8  lane p <- p + 8
    a = __fadd_rn(a, dpp_row<0x104>(a));  // row_shl:4
    a = __fadd_rn(a, dpp_row<0x102>(a));  // row_shl:2
    a = __fadd_rn(a, dpp_row<0x101>(a));  // row_shl:1
    return a;
}

// Distances of the candidates in the lanes set in `mask` (each lane holds its
// id in `cand`); the distance of a candidate is returned in its own lane.
// Each round takes the next two set lanes: half-wave 0 evaluates the first,
// half-wave 1 the second. Ids reach the halves and results come back through
// readlane (no LDS round trip). The raw rows of G rounds are loaded first,
// unconditionally (lanes without work read a valid chunk and are masked to
// zero afterwards), so that all loads are in flight before any is decoded.
// F32ROWS reads the FP32 rows (rerank) instead of the traversal store.
// Rows in flight per half-wave at most: a register budget for the raw chunks,
// so that narrower storage keeps more rows (and memory requests) in flight.
template <int DL, int QCH>
constexpr int dist_rounds_max() {
    constexpr int WPC = DL == DT_F32 ? 4 : (DL == DT_BF16 ? 2 : 1);  // 32-bit words per chunk
    constexpr int BUDGET = QCH >= 12 ? 64 : 16;
    constexpr int G0 = BUDGET / (QCH * WPC);
    constexpr int GMAX = QCH >= 12 ? 4 : 8;
    return G0 < 1 ? 1 : (G0 > GMAX ? GMAX : G0);
}

template <int DT, int METRIC, int QCH, bool F32ROWS, int G>
__device__ __forceinline__ float batch_dist_g(const SearchParams &P, const float4 (&qv)[QCH],
                                              int32_t cand, uint64_t mask, int nch, bool mask_tail) {
    constexpr int DL = F32ROWS ? DT_F32 : DT;
    using Raw = typename RawChunk<DL>::T;
    const int lane = lane_id();
    const int half = lane >> 5, p = lane & 31;
    float res = 0.0f;
    uint64_t m = mask;
    while (m) {
        Raw raw[G][QCH];
        float sc[G];
        int b0[G], b1[G];
        bool ok[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            b0[g] = m ? (int)__builtin_ctzll(m) : -1;
            if (m) m &= m - 1;
            b1[g] = m ? (int)__builtin_ctzll(m) : -1;
            if (m) m &= m - 1;
            const int32_t id0 = b0[g] >= 0 ? __builtin_amdgcn_readlane(cand, b0[g]) : 0;
            const int32_t id1 = b1[g] >= 0 ? __builtin_amdgcn_readlane(cand, b1[g]) : 0;
            ok[g] = (half ? b1[g] : b0[g]) >= 0;
            const int32_t id = ok[g] ? (half ? id1 : id0) : 0;
            sc[g] = 1.0f;
            if constexpr (DL == DT_FP8) sc[g] = P.scale[id];
#pragma unroll
            for (int c = 0; c < QCH; ++c) {
                const int ch = p + 32 * c;
                const int che = ch < nch ? ch : 0;
                if constexpr (F32ROWS) {
                    raw[g][c] = reinterpret_cast<const float4 *>(P.f32 + (int64_t)id * P.f32_stride)[che];
                } else {
                    raw[g][c] = load_raw<DL>(P, id, che);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (b0[g] < 0) break;
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < QCH; ++c) {
                const int ch = p + 32 * c;
                float4 x = decode_raw<DL>(raw[g][c], sc[g]);
                if (!ok[g] || ch >= nch) x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (mask_tail) {
                    const int base = 4 * ch;
                    if (base + 0 >= P.dim) x.x = 0.f;
                    if (base + 1 >= P.dim) x.y = 0.f;
                    if (base + 2 >= P.dim) x.z = 0.f;
                    if (base + 3 >= P.dim) x.w = 0.f;
                }
                acc = acc_chunk<METRIC>(acc, x, qv[c]);
            }
            acc = half_reduce(acc);
            if (METRIC == DEG_METRIC_IP) acc = __fsub_rn(1.0f, acc);
            const float d0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, acc), 0));
            const float d1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, acc), 32));
            if (lane == b0[g]) res = d0;
            if (lane == b1[g]) res = d1;
        }
    }
    return res;
}

// Distances of the lanes in `mask` (candidate id in `cand`): the number of
// rows loaded per round follows the number of candidates (2 per round and
// half-wave pair), so that a hop with few new neighbours issues few loads.
template <int DT, int METRIC, int QCH, bool F32ROWS = false>
__device__ __forceinline__ float batch_dist(const SearchParams &P, const float4 (&qv)[QCH],
                                            int32_t cand, uint64_t mask, int nch, bool mask_tail) {
    constexpr int GM = dist_rounds_max<F32ROWS ? DT_F32 : DT, QCH>();
    const int cnt = __popcll(mask);
    if (GM >= 2 && cnt <= 2) return batch_dist_g<DT, METRIC, QCH, F32ROWS, 1>(P, qv, cand, mask, nch, mask_tail);
    if (GM >= 4 && cnt <= 4) return batch_dist_g<DT, METRIC, QCH, F32ROWS, 2>(P, qv, cand, mask, nch, mask_tail);
    if (GM >= 8 && cnt <= 8) return batch_dist_g<DT, METRIC, QCH, F32ROWS, 4>(P, qv, cand, mask, nch, mask_tail);
    return batch_dist_g<DT, METRIC, QCH, F32ROWS, GM>(P, qv, cand, mask, nch, mask_tail);
}

// The same distances with the candidates handed out through LDS: each
// candidate lane writes its id at its rank among the set lanes (xb[0..64)),
// half-wave h of group g in a round reads rank 2g + h, and the two sums of a
// group go back through xb[64..128) to the candidates' own lanes. This takes
// the place of the per-group bit scans and cross-lane reads of batch_dist_g.
// xb: 128 words of LDS owned by the calling wave.
struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// `hook` runs once, after the row loads of the first round are issued and
// before any of them is used (work that should overlap their latency).
template <int DT, int METRIC, int QCH, bool F32ROWS, int G, class Hook>
__device__ __forceinline__ float batch_dist_xg(const SearchParams &P, const float4 (&qv)[QCH],
                                               int32_t cand, uint64_t mask, int nch, bool mask_tail,
                                               int32_t *xb, Hook &hook) {
    constexpr int DL = F32ROWS ? DT_F32 : DT;
    using Raw = typename RawChunk<DL>::T;
    const int lane = lane_id();
    const int half = lane >> 5, p = lane & 31;
    const int cnt = __popcll(mask);
    const bool mine = (mask >> lane) & 1ull;
    const int rk = prefix_in(mask);
    float *xr = reinterpret_cast<float *>(xb + WAVE);
    if (mine) xb[rk] = cand;
    wave_sync();
    for (int base = 0; base < cnt; base += 2 * G) {
        Raw raw[G][QCH];
        float sc[G];
        bool ok[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int j = base + 2 * g + half;
            ok[g] = j < cnt;
            const int32_t id = ok[g] ? xb[j & (WAVE - 1)] : 0;
            sc[g] = 1.0f;
            if constexpr (DL == DT_FP8) sc[g] = P.scale[id];
#pragma unroll
            for (int c = 0; c < QCH; ++c) {
                const int ch = p + 32 * c;
                const int che = ch < nch ? ch : 0;
                if constexpr (F32ROWS) {
                    raw[g][c] = reinterpret_cast<const float4 *>(P.f32 + (int64_t)id * P.f32_stride)[che];
                } else {
                    raw[g][c] = load_raw<DL>(P, id, che);
                }
            }
        }
        if (base == 0) hook();
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (base + 2 * g >= cnt) break;
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < QCH; ++c) {
                const int ch = p + 32 * c;
                float4 x = decode_raw<DL>(raw[g][c], sc[g]);
                if (!ok[g] || ch >= nch) x = make_float4(0.f, 0.f, 0.f, 0.f);
                if (mask_tail) {
                    const int b4 = 4 * ch;
                    if (b4 + 0 >= P.dim) x.x = 0.f;
                    if (b4 + 1 >= P.dim) x.y = 0.f;
                    if (b4 + 2 >= P.dim) x.z = 0.f;
                    if (b4 + 3 >= P.dim) x.w = 0.f;
                }
                acc = acc_chunk<METRIC>(acc, x, qv[c]);
            }
            acc = half_reduce(acc);  // the half's sum in its lane 0
            if (METRIC == DEG_METRIC_IP) acc = __fsub_rn(1.0f, acc);
            if (p == 0 && ok[g]) xr[base + 2 * g + half] = acc;
        }
    }
    wave_sync();
    const float res = mine ? xr[rk] : 0.0f;
    wave_sync();
    return res;
}

template <int DT, int METRIC, int QCH, bool F32ROWS = false, class Hook = NoHook>
__device__ __forceinline__ float batch_dist(const SearchParams &P, const float4 (&qv)[QCH],
                                            int32_t cand, uint64_t mask, int nch, bool mask_tail,
                                            int32_t *xb, Hook &&hook = Hook{}) {
    constexpr int GM = dist_rounds_max<F32ROWS ? DT_F32 : DT, QCH>();
    const int cnt = __popcll(mask);
    if (GM >= 2 && cnt <= 2) return batch_dist_xg<DT, METRIC, QCH, F32ROWS, 1>(P, qv, cand, mask, nch, mask_tail, xb, hook);
    if (GM >= 4 && cnt <= 4) return batch_dist_xg<DT, METRIC, QCH, F32ROWS, 2>(P, qv, cand, mask, nch, mask_tail, xb, hook);
    if (GM >= 8 && cnt <= 8) return batch_dist_xg<DT, METRIC, QCH, F32ROWS, 4>(P, qv, cand, mask, nch, mask_tail, xb, hook);
    return batch_dist_xg<DT, METRIC, QCH, F32ROWS, GM>(P, qv, cand, mask, nch, mask_tail, xb, hook);
}

// ---------------------------------------------------------------- visited set
// Visited set C of one query, exact for any number of checked vertices. It
// starts in an LDS hash table; when that is 3/4 full every id moves to the
// first table of the wave's workspace region, and each time a private
// workspace table is 3/8 full the ids move to one four times larger (the next
// table of the region, or a shared table of hg_cap slots, which holds all n
// vertices below 3/4 load).
struct Visited {
    int32_t *htab;  // LDS
    int32_t *region;// the wave's workspace region
    int32_t *gtab;  // current workspace table
    int H, hshift, Hg, hgshift;
    int limit;      // move to a larger table before count exceeds this
    int64_t roff;   // offset of gtab within region
    int pslot;      // shared table held (-1: none)
    int count;      // |C| (wave-uniform)
    bool spilled;   // wave-uniform
};

__device__ __forceinline__ uint32_t hash_slot(int32_t id, int shift) {
    return ((uint32_t)id * 0x9E3779B1u) >> shift;
}

// Position, within an aligned group of four slots, of the first slot at or
// after position j0 that holds `id` or is empty: 0..3 for an empty slot, 4..7
// for the slot holding id, -1 if neither occurs. Plain selects, no branches.
__device__ __forceinline__ int group_scan(const int4 &q, uint32_t j0, int32_t id) {
    int c = -1;
    c = (q.w == id || q.w == -1) ? (q.w == id ? 7 : 3) : c;
    c = (j0 <= 2u && (q.z == id || q.z == -1)) ? (q.z == id ? 6 : 2) : c;
    c = (j0 <= 1u && (q.y == id || q.y == -1)) ? (q.y == id ? 5 : 1) : c;
    c = (j0 == 0u && (q.x == id || q.x == -1)) ? (q.x == id ? 4 : 0) : c;
    return c;
}

// The same over eight slots read as two groups of four (the aligned group
// holding position j0, then the next group, whose positions all count):
// 0..7 for the first empty slot, 8..15 for the slot holding id (offsets from
// the first group's start), -1 if neither occurs.
__device__ __forceinline__ int group_scan8(const int4 &a, const int4 &b, uint32_t j0, int32_t id) {
    const int c0 = group_scan(a, j0, id);
    const int c1 = group_scan(b, 0u, id);
    const int r1 = c1 < 0 ? -1 : (c1 >= 4 ? c1 + 8 : c1 + 4);  // 4..7 empty, 12..15 present
    const int r0 = c0 >= 4 ? c0 + 4 : c0;                        // 0..3 empty, 8..11 present
    return c0 >= 0 ? r0 : r1;
}

// Linear-probing insert of `id` into `tab` (power-of-two size msk + 1, a
// multiple of 8) starting at slot s. Eight slots are read per round (the
// aligned group of four holding s and the next group, two 16-byte loads), so
// that a probe rarely needs a second round; the first empty slot in probe
// order is claimed with compare-and-swap, so a slot only ever goes from -1 to
// an id. The probe order is the plain linear order s, s+1, ..., so the set is
// the same as with one-slot probing. A stale read can only show -1 where an id
// already is: the CAS then returns that id (done) or another one (the probe
// goes on after that slot).
// Returns true where id was not in the set.
__device__ __forceinline__ bool probe_insert(int32_t *tab, uint32_t msk, uint32_t s, int32_t id) {
    for (;;) {
        const uint32_t g = s & ~3u;
        const int4 a = *reinterpret_cast<const int4 *>(tab + g);
        const int4 b = *reinterpret_cast<const int4 *>(tab + ((g + 4u) & msk));
        const int c = group_scan8(a, b, s & 3u, id);
        if (c >= 8) return false;
        if (c < 0) {
            s = (g + 8u) & msk;
            continue;
        }
        const uint32_t t = (g + (uint32_t)c) & msk;
        const int32_t old = atomicCAS(&tab[t], -1, id);
        if (old == -1) return true;
        if (old == id) return false;
        s = (t + 1u) & msk;
    }
}

// Linear-probing insert of id v by compare-and-swap on each probed slot, from
// slot s (one round trip per probe; for moving a table).
__device__ __forceinline__ bool cas_insert(int32_t *tab, uint32_t msk, uint32_t s, int32_t v) {
    for (;;) {
        const int32_t old = atomicCAS(&tab[s], -1, v);
        if (old == -1) return true;
        if (old == v) return false;
        s = (s + 1u) & msk;
    }
}

// Insert into the query's workspace table, which only this wave touches. Each
// lane reads its next eight slots and stops at its id (present) or at the
// first empty slot (new); lanes aiming at the same empty slot are told
// apart in registers (the lowest lane takes it, the others probe on), and the
// winners claim their slots with plain stores: one memory round trip for the
// usual hop, none waiting for a store. The workgroup-scope fence at the top
// of each round waits for this wave's earlier stores, after which every lane
// of the wave reads them.
// With PF, one prefetch word per lane (pfv = *pf; pf must be a valid address
// in every lane) is loaded right after each round's table reads: vector loads
// complete in issue order, so the wait on those reads does not include it (it
// is issued in every round so that all paths into the scan wait alike). pfv is
// not consumed here.
//
// With FIRST the first round scans a0/b0, the eight slots at s read earlier
// (spec_read, after every earlier claim of this wave), instead of reading
// them: the probe's round trip then overlaps the previous hop's work.
template <bool PF, bool FIRST = false>
__device__ __forceinline__ bool global_insert(int32_t *tab, uint32_t msk, uint32_t s, int32_t id,
                                              bool act, const int32_t *pf, int32_t &pfv,
                                              const int4 &a0 = int4{},
                                              const int4 &b0 = int4{}) {
    const int lane = lane_id();
    bool isnew = false, pending = act;
    if (ballot(pending) == 0) {
        if (PF) pfv = *pf;
        return false;
    }
    bool first = FIRST;
    for (;;) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        // every lane reads (a finished lane its last group, a valid slot)
        const uint32_t g = s & ~3u;
        int4 a, b;
        if (first) {
            a = a0;
            b = b0;
        } else {
            a = *reinterpret_cast<const int4 *>(tab + g);
            b = *reinterpret_cast<const int4 *>(tab + ((g + 4u) & msk));
        }
        if (PF) {
            __asm__ volatile("" ::: "memory");  // keeps the prefetch behind the table reads
            pfv = *pf;
        }
        uint32_t target = 0xFFFFFFFFu;
        if (pending) {
            const int c = group_scan8(a, b, s & 3u, id);
            if (c >= 8) pending = false;
            else if (c >= 0) target = (g + (uint32_t)c) & msk;
            else s = (g + 8u) & msk;
        }
        // claims: lowest lane per slot wins; a loser holding the winner's id
        // (the same id twice in one adjacency row) finds it present
        const uint64_t cm = ballot(target != 0xFFFFFFFFu);
        bool win = target != 0xFFFFFFFFu, dup = false;
        for (uint64_t m = cm; m; m &= m - 1) {
            const int c = (int)__builtin_ctzll(m);
            const uint32_t tc = (uint32_t)__builtin_amdgcn_readlane((int)target, c);
            const int32_t ic = __builtin_amdgcn_readlane(id, c);
            if (lane > c && tc == target) {
                if (win && ic == id) dup = true;
                win = false;
            }
        }
        if (dup) {
            pending = false;
        } else if (win) {
            tab[target] = id;
            isnew = true;
            pending = false;
        } else if (target != 0xFFFFFFFFu) {
            s = (target + 1u) & msk;  // the slot is taken by a lower lane: probe on
        }
        if (ballot(pending) == 0) break;
        first = false;
    }
    return isnew;
}

// The eight workspace-table slots at which the probe of `id` starts (the
// aligned group of four holding its hash slot and the next group); inactive
// lanes read group 0.
__device__ __forceinline__ void spec_read(const Visited &V, int32_t id, bool act, int4 &a, int4 &b) {
    const uint32_t msk = (uint32_t)V.Hg - 1u;
    const uint32_t g = act ? (hash_slot(id, V.hgshift) & ~3u) : 0u;
    a = *reinterpret_cast<const int4 *>(V.gtab + g);
    b = *reinterpret_cast<const int4 *>(V.gtab + ((g + 4u) & msk));
}

// Lanes of `cand` whose id is on the query's exclusion list ex[0 .. nex): the
// wave reads the list 64 ids at a time and compares each candidate with every
// id read (a ballot per candidate). Only candidates that could enter the result
// are checked, so a hop without one reads nothing.
__device__ __forceinline__ uint64_t excluded_lanes(const int32_t *ex, int nex, int32_t id,
                                                   uint64_t cand) {
    const int lane = lane_id();
    uint64_t hit = 0;
    for (int b = 0; b < nex && cand != 0; b += WAVE) {
        const int32_t e = b + lane < nex ? ex[b + lane] : -1;
        for (uint64_t m = cand; m; m &= m - 1) {
            const int c = (int)__builtin_ctzll(m);
            const int32_t ic = __builtin_amdgcn_readlane(id, c);
            if (ballot(e == ic) != 0) hit |= 1ull << c;
        }
        cand &= ~hit;
    }
    return hit;
}

// Inserts `id` (lane-wise, `act` lanes); returns true where id was not in the
// set. With PF also loads
// pfv = *pf (pf valid in every lane), issued after the workspace-table reads.
template <bool PF>
__device__ __forceinline__ bool visit_insert(Visited &V, int32_t id, bool act, const int32_t *pf,
                                             int32_t &pfv) {
    if (!V.spilled) {
        if (PF) pfv = *pf;
        bool isnew = false;
        if (act) isnew = probe_insert(V.htab, (uint32_t)V.H - 1u, hash_slot(id, V.hshift), id);
        return isnew;
    }
    return global_insert<PF>(V.gtab, (uint32_t)V.Hg - 1u, hash_slot(id, V.hgshift), id, act, pf,
                             pfv);
}
__device__ __forceinline__ bool visit_insert(Visited &V, int32_t id, bool act) {
    int32_t unused = 0;
    return visit_insert<false>(V, id, act, nullptr, unused);
}

__device__ __forceinline__ int ilog2_dev(int x) { return 31 - __builtin_clz((unsigned)x); }

// Fills n slots (a multiple of 4) of a workspace table with -1.
__device__ __forceinline__ void table_clear(int32_t *t, int n) {
    int4 *t4 = reinterpret_cast<int4 *>(t);
    for (int i = lane_id(); i < (n >> 2); i += WAVE) t4[i] = make_int4(-1, -1, -1, -1);
}

// Points V at workspace table t of `slots` slots.
__device__ __forceinline__ void table_use(Visited &V, int32_t *t, int slots, int hg_cap) {
    V.gtab = t;
    V.Hg = slots;
    V.hgshift = 32 - ilog2_dev(slots);
    V.limit = slots >= hg_cap ? 0x7fffffff : (3 * slots) / 8;
}

// Moves the LDS table to the first table of the region (cleared first).
__device__ __forceinline__ void visit_spill(Visited &V, const SearchParams &P) {
    table_clear(V.region, P.hg0);
    __threadfence();
    wave_sync();
    V.roff = 0;
    table_use(V, V.region, P.hg0, P.hg_cap);
    V.spilled = true;
    for (int i = lane_id(); i < V.H; i += WAVE) {
        const int32_t v = V.htab[i];
        if (v != -1) cas_insert(V.gtab, (uint32_t)V.Hg - 1u, hash_slot(v, V.hgshift), v);
    }
    __threadfence();
    wave_sync();
}

// Takes a free shared table (waiting while all are held: holders never wait,
// their searches end, and they give the table back at the end of their query).
__device__ __forceinline__ int pool_take(int npool, int *owner) {
    int slot = -1;
    for (;;) {
        if (lane_id() == 0) {
            for (int t = 0; t < npool; ++t) {
                const int i = (int)((blockIdx.x + (unsigned)t) % (unsigned)npool);
                if (atomicCAS(&owner[i], 0, 1) == 0) {
                    slot = i;
                    break;
                }
            }
        }
        slot = uni(slot);
        if (slot >= 0) break;
        __builtin_amdgcn_s_sleep(32);
    }
    __threadfence();
    return slot;
}

__device__ __forceinline__ void pool_give(Visited &V, const SearchParams &P) {
    if (V.pslot < 0) return;
    __threadfence();
    wave_sync();
    if (lane_id() == 0) atomicExch(&P.pool_owner[V.pslot], 0);
    V.pslot = -1;
}

// Where a table moved to (returned by value: the caller's state never has its
// address taken, so it stays in registers).
struct GrowOut {
    int32_t *t;
    int64_t off;
    int slots;
    int pslot;
};

// Moves workspace table `old` (on slots, at offset roff of the region) to one
// four times larger, or to a shared table once that passes hg_priv slots.
// Kept out of line: it runs a few times per query at most.
__device__ __forceinline__ GrowOut grow_table(const int32_t *old, int on, int32_t *region, int64_t roff,
                                           int hg_priv, int hg_cap, int32_t *pool, int npool,
                                           int *owner) {
    GrowOut o;
    int ns = on * 4;
    if (ns > hg_cap) ns = hg_cap;
    o.off = roff;
    o.pslot = -1;
    if (ns <= hg_priv) {
        o.off = roff + on;
        o.t = region + o.off;
    } else {
        ns = hg_cap;
        o.pslot = pool_take(npool, owner);
        o.t = pool + (int64_t)o.pslot * hg_cap;
    }
    o.slots = ns;
    table_clear(o.t, ns);
    __threadfence();
    wave_sync();
    const uint32_t msk = (uint32_t)ns - 1u;
    const int sh = 32 - ilog2_dev(ns);
    for (int i = lane_id(); i < on; i += WAVE) {
        const int32_t v = old[i];
        if (v != -1) cas_insert(o.t, msk, hash_slot(v, sh), v);
    }
    __threadfence();
    wave_sync();
    return o;
}

__device__ __forceinline__ void visit_grow(Visited &V, const SearchParams &P) {
    const GrowOut o = grow_table(V.gtab, V.Hg, V.region, V.roff, P.hg_priv, P.hg_cap, P.pool,
                                 P.npool, P.pool_owner);
    if (o.pslot >= 0) V.pslot = o.pslot;
    V.roff = o.off;
    table_use(V, o.t, o.slots, P.hg_cap);
}

}  // namespace degk
