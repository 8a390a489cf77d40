// Exact kNN ground truth (Eq. knn) by brute force on matrix cores.
//
// Phase 1 (knn_tile_kernel): a workgroup takes 64 queries and one slice of
//   the base set. For each tile of 128 base rows it forms the 64 x 128 inner
//   products with v_mfma_f32_32x32x2f32 (FP32 inputs, FP32 accumulation),
//   turns them into distances (L2: |q|^2 + |x|^2 - 2 q.x; IP: 1 - q.x) and
//   appends every (distance, id) key below the query's running threshold to
//   a per-(query, slice) list in the workspace. When a list is nearly full it
//   is cut to its KC smallest keys (a 64-step bitwise select) and the
//   threshold becomes the KC-th key.
// Phase 2 (knn_final_kernel): one wave per query gathers the slices' lists,
//   recomputes each candidate as a direct FP32 difference in the fixed C32x4
//   order (the same arithmetic as the search), and keeps the k smallest keys.
// On integer data below 256 every product and partial sum is an exact
// integer below 2^24, so phase 1 already ranks exactly and the result equals
// the FP64 definition; on float data KC = k + margin candidates absorb the
// rounding of the norm expansion.
#include <hip/hip_runtime.h>

#include "deg.h"
#include "search_kernel.h"

namespace degk {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int KQ = 64;     // queries per workgroup
constexpr int KN = 128;    // base rows per tile
constexpr int KCH = 32;    // dims per K chunk
constexpr int KMARGIN = 32;

struct KnnParams {
    const float *base;
    const float *queries;
    int64_t n, nq, bstride, qstride;
    int32_t dim, k, kc, cap, nslices, metric;
    const int32_t *exclude;
    const float *bnorm, *qnorm;
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

// Cuts the `cnt` distinct keys of `buf` (global, one wave) to the kc smallest:
// the keys are read once into registers (up to SEL_R per lane), the kc-th
// smallest is built bit by bit from the top by counting the keys below each
// candidate prefix, and the kept keys are written back compacted. Returns the
// kc-th key; `cnt` becomes kc (or stays, if cnt <= kc).
constexpr int SEL_R = 20;  // covers cap = 2 (k + 32) + 128 for k <= 512
__device__ uint64_t cut_list(uint64_t *buf, int &cnt, int kc) {
    const int lane = lane_id();
    uint64_t v[SEL_R];
#pragma unroll
    for (int r = 0; r < SEL_R; ++r) {
        const int i = lane + WAVE * r;
        v[r] = i < cnt ? buf[i] : KEY_MAX;
    }
    uint64_t ans = 0;
    for (int b = 63; b >= 0; --b) {
        const uint64_t cand = ans | (1ull << b);
        int c = 0;
#pragma unroll
        for (int r = 0; r < SEL_R; ++r) c += v[r] < cand ? 1 : 0;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
        if (c < kc) ans = cand;
    }
    int out = 0;
#pragma unroll
    for (int r = 0; r < SEL_R; ++r) {
        const int i = lane + WAVE * r;
        const bool keep = i < cnt && v[r] <= ans;
        const uint64_t m = ballot(keep);
        if (keep) buf[out + prefix_in(m)] = v[r];
        out += __popcll(m);
    }
    cnt = out;
    return ans;
}

template <int METRIC>
__global__ void __launch_bounds__(256) knn_tile_kernel(KnnParams P) {
    __shared__ float QsT[KCH][KQ + 1];
    __shared__ float BsT[KCH][KN + 1];
    __shared__ float S[KQ][KN + 1];
    const int t = threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    const int wq = w >> 1, wn = w & 1;
    const int64_t q0 = (int64_t)blockIdx.x * KQ;
    const int slice = blockIdx.y;
    const int64_t per = (P.n + P.nslices - 1) / P.nslices;
    const int64_t n0 = (int64_t)slice * per;
    const int64_t n1 = min(P.n, n0 + per);
    // wave w owns query rows 16w .. 16w+15: lane r < 16 keeps row 16w + r's
    // list threshold and count in registers
    uint64_t thr_l = KEY_MAX;
    int cnt_l = 0;
    // Staging of one (tile, chunk): the thread's 8 query values (row t % 64,
    // dims 8 (t / 64) ..) and 16 base values (row t % 128, dims 16 (t / 128) ..)
    // are read into registers one chunk ahead (while the matrix cores work on
    // the current one, and across the epilogue), then written to LDS.
    float4 rq[2], rb[4];
    auto fetch = [&](int64_t bt, int k0) {
        {
            const int r = t & 63, dq = (t >> 6) * 8;
            const int64_t qi = q0 + r;
            if (qi < P.nq && k0 + dq + 8 <= P.dim && (P.qstride & 3) == 0) {
                const float4 *src = reinterpret_cast<const float4 *>(P.queries + qi * P.qstride + k0 + dq);
                rq[0] = src[0];
                rq[1] = src[1];
            } else {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = k0 + dq + j;
                    v[j] = (qi < P.nq && c < P.dim) ? P.queries[qi * P.qstride + c] : 0.0f;
                }
                rq[0] = make_float4(v[0], v[1], v[2], v[3]);
                rq[1] = make_float4(v[4], v[5], v[6], v[7]);
            }
        }
        {
            const int r = t & 127, dq = (t >> 7) * 16;
            const int64_t bi = bt + r;
            if (bi < n1 && k0 + dq + 16 <= P.dim) {  // rows are 16-byte aligned (b_stride % 4 == 0)
                const float4 *src = reinterpret_cast<const float4 *>(P.base + bi * P.bstride + k0 + dq);
#pragma unroll
                for (int j4 = 0; j4 < 4; ++j4) rb[j4] = src[j4];
            } else {
                float v[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int c = k0 + dq + j;
                    v[j] = (bi < n1 && c < P.dim) ? P.base[bi * P.bstride + c] : 0.0f;
                }
#pragma unroll
                for (int j4 = 0; j4 < 4; ++j4)
                    rb[j4] = make_float4(v[4 * j4], v[4 * j4 + 1], v[4 * j4 + 2], v[4 * j4 + 3]);
            }
        }
    };
    auto stage = [&]() {
        {
            const int r = t & 63, dq = (t >> 6) * 8;
            QsT[dq + 0][r] = rq[0].x; QsT[dq + 1][r] = rq[0].y; QsT[dq + 2][r] = rq[0].z; QsT[dq + 3][r] = rq[0].w;
            QsT[dq + 4][r] = rq[1].x; QsT[dq + 5][r] = rq[1].y; QsT[dq + 6][r] = rq[1].z; QsT[dq + 7][r] = rq[1].w;
        }
        {
            const int r = t & 127, dq = (t >> 7) * 16;
#pragma unroll
            for (int j4 = 0; j4 < 4; ++j4) {
                BsT[dq + 4 * j4 + 0][r] = rb[j4].x;
                BsT[dq + 4 * j4 + 1][r] = rb[j4].y;
                BsT[dq + 4 * j4 + 2][r] = rb[j4].z;
                BsT[dq + 4 * j4 + 3][r] = rb[j4].w;
            }
        }
    };
    if (n0 < n1) fetch(n0, 0);
    for (int64_t b0 = n0; b0 < n1; b0 += KN) {
        floatx16 acc0, acc1;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            acc0[v] = 0.0f;
            acc1[v] = 0.0f;
        }
        for (int k0 = 0; k0 < P.dim; k0 += KCH) {
            stage();
            __syncthreads();
            // the next chunk of this tile, or the first chunk of the next tile
            if (k0 + KCH < P.dim)
                fetch(b0, k0 + KCH);
            else if (b0 + KN < n1)
                fetch(b0 + KN, 0);
#pragma unroll
            for (int kk = 0; kk < KCH; kk += 2) {
                int kr = kk + (lane >> 5);
                float a = QsT[kr][wq * 32 + (lane & 31)];
                float b0v = BsT[kr][wn * 64 + (lane & 31)];
                float b1v = BsT[kr][wn * 64 + 32 + (lane & 31)];
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0v, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1v, acc1, 0, 0, 0);
            }
            __syncthreads();
        }
        // 32x32 accumulator layout: lane l, register v -> row 8(v/4) + 4(l/32) + v%4, col l%32
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int row = wq * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            int col = wn * 64 + (lane & 31);
            S[row][col] = acc0[v];
            S[row][col + 32] = acc1[v];
        }
        __syncthreads();
        // epilogue: wave w takes query rows 16w .. 16w+15; the base norms of the
        // tile's columns and the rows' query norms are read once per tile
        float bn[2] = {0.f, 0.f};
        if (METRIC == DEG_METRIC_L2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t bi = b0 + lane + 64 * h;
                bn[h] = P.bnorm[bi < n1 ? bi : 0];
            }
        }
        const int64_t qrow0 = q0 + w * 16 + (lane & 15);
        const float qn_l = (METRIC == DEG_METRIC_L2 && qrow0 < P.nq) ? P.qnorm[qrow0] : 0.f;
        const int32_t ex_l = (P.exclude && qrow0 < P.nq) ? P.exclude[qrow0] : -1;
        for (int rr = 0; rr < 16; ++rr) {
            int row = w * 16 + rr;
            int64_t qi = q0 + row;
            if (qi >= P.nq) break;
            const int32_t ex = __builtin_amdgcn_readlane(ex_l, rr);
            const float qn = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qn_l), rr));
            uint64_t th = read_lane_u64(thr_l, rr);
            uint64_t key[2];
            bool pass[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int col = lane + 64 * h;
                int64_t bi = b0 + col;
                float dot = S[row][col];
                float d;
                if (METRIC == DEG_METRIC_L2)
                    d = __fsub_rn(__fadd_rn(qn, bn[h]), __fmul_rn(2.0f, dot));
                else
                    d = __fsub_rn(1.0f, dot);
                key[h] = make_key(d, (int32_t)bi);
                pass[h] = bi < n1 && bi != ex && key[h] < th;
            }
            uint64_t *lst = P.lists + ((int64_t)qi * P.nslices + slice) * P.cap;
            int c = __builtin_amdgcn_readlane(cnt_l, rr);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint64_t m = ballot(pass[h]);
                if (pass[h]) lst[c + prefix_in(m)] = key[h];
                c += __popcll(m);
            }
            if (c > P.cap - KN) {
                __threadfence_block();
                wave_sync();
                th = cut_list(lst, c, P.kc);
            }
            if (lane == rr) {
                cnt_l = c;
                thr_l = th;
            }
        }
        __syncthreads();
    }
    // final cut to KC
    for (int rr = 0; rr < 16; ++rr) {
        int row = w * 16 + rr;
        int64_t qi = q0 + row;
        if (qi >= P.nq) break;
        uint64_t *lst = P.lists + ((int64_t)qi * P.nslices + slice) * P.cap;
        int c = __builtin_amdgcn_readlane(cnt_l, rr);
        __threadfence_block();
        wave_sync();
        if (c > P.kc) cut_list(lst, c, P.kc);
        if (lane == 0) P.counts[qi * P.nslices + slice] = c;
    }
}

template <int METRIC, int QCH>
__global__ void __launch_bounds__(64) knn_final_kernel(KnnParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *keys = reinterpret_cast<uint64_t *>(smem);       // nslices * kc
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
    // exact FP32 distances of every candidate
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
    wave_sync();
    // k smallest keys, sorted
    int kk = min(P.k, tot);
    uint64_t kth = KEY_MAX;
    if (tot > kk) {
        uint64_t ans = 0;
        for (int b = 63; b >= 0; --b) {
            uint64_t cand = ans | (1ull << b);
            int c = 0;
            for (int i = lane; i < tot; i += WAVE) c += keys[i] < cand ? 1 : 0;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
            if (c < kk) ans = cand;
        }
        kth = ans;
    }
    for (int i = lane; i < tot; i += WAVE) {
        uint64_t v = keys[i];
        if (v <= kth) {
            int rank = 0;
            for (int j = 0; j < tot; ++j) rank += keys[j] < v ? 1 : 0;
            if (rank < kk) {
                P.out_ids[qi * P.k + rank] = key_id(v);
                P.out_dists[qi * P.k + rank] = key_dist(v);
            }
        }
    }
    for (int i = kk + lane; i < P.k; i += WAVE) {
        P.out_ids[qi * P.k + i] = -1;
        P.out_dists[qi * P.k + i] = __builtin_inff();
    }
}

// Slices of the base set: enough workgroups to fill the chip (about 4 per CU),
// at least 4 tiles per slice, and the final kernel's candidate keys
// (slices x KC x 8 bytes) within 60 KiB of LDS.
static int knn_slices(int64_t n, int64_t nq, int32_t k) {
    int64_t qb = (nq + KQ - 1) / KQ;
    int64_t want = (4 * 256 + qb - 1) / qb;
    int64_t maxs = (n + 4 * KN - 1) / (4 * KN);
    int64_t maxl = (60 * 1024) / (8 * (int64_t)(k + KMARGIN));
    if (want > maxs) want = maxs;
    if (want > maxl) want = maxl;
    if (want > 64) want = 64;
    if (want < 1) want = 1;
    return (int)want;
}

}  // namespace degk

using namespace degk;

extern "C" size_t deg_knn_workspace_bytes(int64_t n, int32_t dim, int64_t nq, int32_t k) {
    (void)dim;
    if (n < 1 || nq < 0 || k < 1) return 0;
    int ns = knn_slices(n, nq, k);
    int64_t kc = k + KMARGIN;
    int64_t cap = 2 * kc + KN;
    return 256 + (size_t)n * 4 + (size_t)nq * 4 + (size_t)nq * ns * 4 + (size_t)nq * ns * cap * 8;
}

extern "C" deg_status deg_knn_bruteforce(const float *base, int64_t n, int32_t dim,
                                         int64_t b_stride, const float *queries, int64_t nq,
                                         int64_t q_stride, int32_t k, int32_t metric,
                                         const int32_t *exclude_ids, int32_t *out_ids,
                                         float *out_dists, void *workspace, size_t ws_bytes,
                                         void *stream) {
    if (!base || n < 1 || dim < 1 || b_stride < dim || (b_stride & 3) || nq < 0 || k < 1 ||
        k > 512 || (metric != DEG_METRIC_L2 && metric != DEG_METRIC_IP))
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
    P.k = k;
    P.kc = k + KMARGIN;
    P.cap = 2 * P.kc + KN;
    P.nslices = knn_slices(n, nq, k);
    P.metric = metric;
    P.exclude = exclude_ids;
    char *ws = reinterpret_cast<char *>(workspace) + 256;
    float *bn = reinterpret_cast<float *>(ws);
    float *qn = bn + n;
    int32_t *counts = reinterpret_cast<int32_t *>(qn + nq);
    size_t off = 256 + (size_t)n * 4 + (size_t)nq * 4 + (size_t)nq * P.nslices * 4;
    off = (off + 7) / 8 * 8;
    P.bnorm = bn;
    P.qnorm = qn;
    P.counts = counts;
    P.lists = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(workspace) + off);
    if (off + (size_t)nq * P.nslices * P.cap * 8 > ws_bytes) return DEG_ERR_WORKSPACE;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    hipLaunchKernelGGL(row_norm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, base, n,
                       dim, b_stride, bn);
    hipLaunchKernelGGL(row_norm_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st,
                       queries, nq, dim, q_stride, qn);
    dim3 g1((unsigned)((nq + KQ - 1) / KQ), (unsigned)P.nslices);
    if (metric == DEG_METRIC_L2)
        hipLaunchKernelGGL(knn_tile_kernel<DEG_METRIC_L2>, g1, dim3(256), 0, st, P);
    else
        hipLaunchKernelGGL(knn_tile_kernel<DEG_METRIC_IP>, g1, dim3(256), 0, st, P);
    int q = ((dim + 3) / 4 + 31) / 32;
    int qch = q <= 1 ? 1 : (q <= 2 ? 2 : (q <= 4 ? 4 : 12));
    size_t lds = (size_t)P.nslices * P.kc * 8 + WAVE * 4 * 2;
    void (*fn)(KnnParams) = nullptr;
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
    hipLaunchKernelGGL(fn, dim3((unsigned)nq), dim3(64), lds, st, P);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}
