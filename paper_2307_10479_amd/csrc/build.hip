// Graph construction with batched searches (Sec. 5.2, Algorithm 3).
//
// The paper builds the graph one vertex at a time: the smallest DEG (the
// complete graph on d + 1 vertices), then for every further vertex in id order
// a search for its k_ext nearest vertices followed by the edits of scheme C:
// walk the result, take each vertex b that passes the MRNG check against the
// new vertex's tentative neighbours (a second pass takes them without it), cut
// b's longest edge (b, n) with n outside the tentative set, and give the new
// vertex both ends. The search dominates the cost; the edits touch a few rows.
//
// Here the searches run on the GPU in blocks: every vertex of a block searches
// the graph as it stands when the block starts (one deg_search launch), then
// the host applies the block's edits in id order, each on the live graph, and
// the rows they changed go back to the device before the next block. A block
// holds at most `batch` vertices and at most an eighth of the graph (at least
// one), so the first blocks are single vertices and batch = 1 is the paper's
// schedule. With lag 1 a block searches before the previous block's edits are
// applied, so that the host applies them while the device searches. The
// optional optimizeEdge step (Algorithm 4) is not part of this entry point: its
// searches depend on each other's edits.
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "deg.h"

namespace {

// One FP32 distance in the library's fixed order: 32 partial sums, the
// 4-dim chunk c feeding partial c mod 32 with fused multiply-adds in
// increasing dim order, then the halving tree over the partials.
// AVX2: a block of 128 dims is four loads of 32 floats (chunks 8g .. 8g + 7,
// four dims each); an in-register 8 x 4 transpose gives, for each position j
// in a chunk, one vector of dim j of the eight chunks, so each vector FMA
// advances eight partials by one term in their own order. (The eight chunks
// come out in the order 0 2 4 6 1 3 5 7, undone before the tree.) A short last
// block is zero-padded: fma(0, 0, p) = p, and a partial sum is never -0.
template <bool L2>
inline void c32x4_block(const float *x, const float *q, __m256 acc[4]) {
    for (int g = 0; g < 4; ++g) {
        __m256 X[4], Q[4];
        for (int u = 0; u < 4; ++u) {
            X[u] = _mm256_loadu_ps(x + 32 * g + 8 * u);
            Q[u] = _mm256_loadu_ps(q + 32 * g + 8 * u);
            if (L2) X[u] = _mm256_sub_ps(X[u], Q[u]);
        }
        auto tr = [](const __m256 *V, __m256 J[4]) {
            const __m256 a = _mm256_unpacklo_ps(V[0], V[1]), b = _mm256_unpackhi_ps(V[0], V[1]);
            const __m256 c = _mm256_unpacklo_ps(V[2], V[3]), d = _mm256_unpackhi_ps(V[2], V[3]);
            J[0] = _mm256_shuffle_ps(a, c, 0x44);
            J[1] = _mm256_shuffle_ps(a, c, 0xEE);
            J[2] = _mm256_shuffle_ps(b, d, 0x44);
            J[3] = _mm256_shuffle_ps(b, d, 0xEE);
        };
        __m256 XJ[4];
        tr(X, XJ);
        if (L2) {
            for (int j = 0; j < 4; ++j) acc[g] = _mm256_fmadd_ps(XJ[j], XJ[j], acc[g]);
        } else {
            __m256 QJ[4];
            tr(Q, QJ);
            for (int j = 0; j < 4; ++j) acc[g] = _mm256_fmadd_ps(XJ[j], QJ[j], acc[g]);
        }
    }
}

template <bool L2>
float c32x4(const float *x, const float *q, int m) {
    __m256 acc[4] = {_mm256_setzero_ps(), _mm256_setzero_ps(), _mm256_setzero_ps(),
                     _mm256_setzero_ps()};
    int base = 0;
    for (; base + 128 <= m; base += 128) c32x4_block<L2>(x + base, q + base, acc);
    if (base < m) {
        alignas(32) float xt[128], qt[128];
        for (int i = 0; i < 128; ++i) {
            xt[i] = base + i < m ? x[base + i] : 0.0f;
            qt[i] = base + i < m ? q[base + i] : 0.0f;
        }
        c32x4_block<L2>(xt, qt, acc);
    }
    alignas(32) float v[32], p[32];
    for (int g = 0; g < 4; ++g) _mm256_store_ps(v + 8 * g, acc[g]);
    static constexpr int order[8] = {0, 2, 4, 6, 1, 3, 5, 7};
    for (int g = 0; g < 4; ++g)
        for (int e = 0; e < 8; ++e) p[8 * g + order[e]] = v[8 * g + e];
    for (int w = 16; w >= 1; w >>= 1)
        for (int i = 0; i < w; ++i) p[i] = p[i] + p[i + w];
    return L2 ? p[0] : 1.0f - p[0];
}

float dist_c32x4(const float *x, const float *q, int m, int metric) {
    return metric == DEG_METRIC_L2 ? c32x4<true>(x, q, m) : c32x4<false>(x, q, m);
}

// Host copy of the growing graph. A vertex owns one 64-byte aligned record of
// 32-bit words: neighbour count, block of the last change, d neighbour ids and
// d weights (filled from the front; removal keeps the order of the remaining
// entries), so one fetch brings everything an edit reads. The records live in
// pinned host memory: the device gathers the changed rows from them directly.
struct HostGraph {
    int64_t n;
    int d;
    int64_t stride;  // words per record, a multiple of 16 (64 bytes)
    int32_t *words = nullptr;
    std::vector<int32_t> dirty;  // records changed since the last upload
    int32_t block = 0;
    bool broken = false;

    HostGraph(int64_t n_, int d_) : n(n_), d(d_), stride((2 + 2 * (int64_t)d_ + 15) / 16 * 16) {
        if (hipHostMalloc((void **)&words, sizeof(int32_t) * (size_t)(n * stride)) != hipSuccess) {
            words = nullptr;
            return;
        }
        for (int64_t a = 0; a < n; ++a) {
            int32_t *x = words + a * stride;
            x[0] = 0;
            x[1] = -1;
            for (int j = 0; j < d; ++j) x[2 + j] = -1;
            float *w = reinterpret_cast<float *>(x + 2 + d);
            for (int j = 0; j < d; ++j) w[j] = 0.0f;
        }
    }
    ~HostGraph() {
        if (words) (void)hipHostFree(words);
    }
    HostGraph(const HostGraph &) = delete;
    HostGraph &operator=(const HostGraph &) = delete;

    int32_t *rec(int32_t a) { return words + (int64_t)a * stride; }
    int32_t &cnt(int32_t a) { return rec(a)[0]; }
    int32_t *ids(int32_t a) { return rec(a) + 2; }
    float *ws(int32_t a) { return reinterpret_cast<float *>(rec(a) + 2 + d); }
    void touch(int32_t a) {
        int32_t &st = rec(a)[1];
        if (st != block) {
            st = block;
            dirty.push_back(a);
        }
    }
    int find(int32_t a, int32_t b) {
        const int32_t *x = ids(a);
        const int c = cnt(a);
        for (int j = 0; j < c; ++j)
            if (x[j] == b) return j;
        return -1;
    }
    void half_add(int32_t a, int32_t b, float wt) {
        int32_t &c = cnt(a);
        if (c >= d) {
            broken = true;
            return;
        }
        ids(a)[c] = b;
        ws(a)[c] = wt;
        ++c;
        touch(a);
    }
    void half_remove(int32_t a, int32_t b) {
        int j = find(a, b);
        if (j < 0) {
            broken = true;
            return;
        }
        int32_t *x = ids(a);
        float *w = ws(a);
        int32_t &c = cnt(a);
        for (; j + 1 < c; ++j) {
            x[j] = x[j + 1];
            w[j] = w[j + 1];
        }
        --c;
        x[c] = -1;
        w[c] = 0.0f;
        touch(a);
    }
    void add_edge(int32_t a, int32_t b, float wt) {
        if (a == b || find(a, b) >= 0) {
            broken = true;
            return;
        }
        half_add(a, b, wt);
        half_add(b, a, wt);
    }
};

// Starts the fetches of the records a search result's walk will read (issued a
// few vertices ahead of the walk: the results of a block are all known).
void prefetch_result(HostGraph &G, const int32_t *ids, int k) {
    const size_t rec_bytes = sizeof(int32_t) * (size_t)(2 + 2 * G.d);
    for (int i = 0; i < k && ids[i] >= 0; ++i) {
        const char *a = reinterpret_cast<const char *>(G.rec(ids[i]));
        for (size_t o = 0; o < rec_bytes; o += 64) __builtin_prefetch(a + o);
    }
}

// Steps 3-6 of Sec. 5.2 for vertex v given its search result (sorted ids and
// distances, ns entries). Returns false when the result cannot supply d
// neighbours. `phase2` counts vertices that needed the pass without MRNG check.
bool extend_vertex(HostGraph &G, const float *vec, int64_t vs, int m, int metric, int32_t v,
                   const int32_t *ids, const float *ds, int ns, int64_t &phase2) {
    const int d = G.d;
    int32_t U[128];
    float Ud[128];
    bool pend[128];  // U[t] is a cut edge's far end whose distance is not computed yet
    int nu = 0;
    const size_t rec_bytes = sizeof(int32_t) * (size_t)(2 + 2 * d);
    // membership in U: a 256-bit filter of hashed ids answers most lookups, the
    // short list the rest
    uint64_t filt[4] = {0, 0, 0, 0};
    auto hbit = [](int32_t x) { return ((uint32_t)x * 0x9E3779B1u) >> 24; };
    auto in_u_list = [&](int32_t x) -> int {
        for (int t = 0; t < nu; ++t)
            if (U[t] == x) return t;
        return -1;
    };
    auto in_u = [&](int32_t x) -> int {
        const uint32_t h = hbit(x);
        if (!((filt[h >> 6] >> (h & 63)) & 1)) return -1;
        return in_u_list(x);
    };
    const __m256i iota8 = _mm256_setr_epi32(0, 1, 2, 3, 4, 5, 6, 7);
    const __m256i bits8 = _mm256_setr_epi32(1, 2, 4, 8, 16, 32, 64, 128);
    const __m256i golden8 = _mm256_set1_epi32((int)0x9E3779B1u);
    auto push = [&](int32_t x, float dx, bool later) {
        const uint32_t h = hbit(x);
        filt[h >> 6] |= 1ull << (h & 63);
        U[nu] = x;
        Ud[nu] = dx;
        pend[nu++] = later;
    };
    auto dist_of = [&](int t) {
        if (pend[t]) {
            Ud[t] = dist_c32x4(vec + (size_t)U[t] * vs, vec + (size_t)v * vs, m, metric);
            pend[t] = false;
        }
        return Ud[t];
    };
    for (int pass = 0; pass < 2 && nu < d; ++pass) {
        if (pass == 1) ++phase2;
        for (int i = 0; i < ns && nu < d; ++i) {
            const int32_t b = ids[i];
            const float db = ds[i];
            if (in_u(b) >= 0) continue;
            // one pass over b's row: the MRNG check of (v, b) against the
            // tentative neighbours u of v adjacent to b (the edge stays out when
            // it is longer than both other sides of such a triangle), and b's
            // longest edge to a vertex outside U (equal weights: smaller id)
            const int32_t *x = G.ids(b);
            const float *xw = G.ws(b);
            const int cb = G.cnt(b);
            bool ok = true;
            int32_t far = -1;
            float fw = -INFINITY;
            // eight entries at a time (the record holds at least round_up(d, 8) words
            // past each array, so the loads stay inside it; lanes past the count are
            // masked): the filter sorts out most entries as outside U, the rest are
            // looked up exactly; the longest edge to an entry outside U is a maximum
            // of (weight, -id), so the order of the reduction does not matter
            const __m256i filt8 = _mm256_loadu_si256(reinterpret_cast<const __m256i *>(filt));
            for (int j0 = 0; j0 < cb; j0 += 8) {
                const __m256i c = _mm256_loadu_si256(reinterpret_cast<const __m256i *>(x + j0));
                const __m256 wt = _mm256_loadu_ps(xw + j0);
                const __m256i live = _mm256_cmpgt_epi32(_mm256_set1_epi32(cb - j0), iota8);
                const __m256i h = _mm256_srli_epi32(_mm256_mullo_epi32(c, golden8), 24);
                const __m256i word = _mm256_permutevar8x32_epi32(filt8, _mm256_srli_epi32(h, 5));
                const __m256i bit = _mm256_and_si256(
                    _mm256_srlv_epi32(word, _mm256_and_si256(h, _mm256_set1_epi32(31))),
                    _mm256_set1_epi32(1));
                const int livem = _mm256_movemask_ps(_mm256_castsi256_ps(live));
                const int maybe = _mm256_movemask_ps(_mm256_castsi256_ps(
                                      _mm256_cmpeq_epi32(bit, _mm256_set1_epi32(1)))) & livem;
                int outside = livem & ~maybe;
                for (int mb = maybe; mb; mb &= mb - 1) {
                    const int e = __builtin_ctz(mb);
                    const int32_t ce = x[j0 + e];
                    const int t = in_u_list(ce);
                    if (t < 0) {
                        outside |= 1 << e;  // a false positive of the filter
                    } else if (pass == 0) {
                        const float we = xw[j0 + e];
                        const float du = dist_of(t);
                        if (db > (du > we ? du : we)) ok = false;
                    }
                }
                if (outside == 0) continue;
                // the best (largest weight, then smallest id) of the outside lanes
                const __m256i om = _mm256_cmpgt_epi32(
                    _mm256_and_si256(_mm256_set1_epi32(outside), bits8), _mm256_setzero_si256());
                __m256 w8 = _mm256_blendv_ps(_mm256_set1_ps(-INFINITY), wt, _mm256_castsi256_ps(om));
                __m256 mx = _mm256_max_ps(w8, _mm256_permute2f128_ps(w8, w8, 1));
                mx = _mm256_max_ps(mx, _mm256_shuffle_ps(mx, mx, 0x4E));
                mx = _mm256_max_ps(mx, _mm256_shuffle_ps(mx, mx, 0xB1));
                const __m256i at = _mm256_and_si256(om, _mm256_castps_si256(_mm256_cmp_ps(w8, mx, _CMP_EQ_OQ)));
                __m256i id8 = _mm256_blendv_epi8(_mm256_set1_epi32(INT32_MAX), c, at);
                id8 = _mm256_min_epi32(id8, _mm256_permute2x128_si256(id8, id8, 1));
                id8 = _mm256_min_epi32(id8, _mm256_shuffle_epi32(id8, 0x4E));
                id8 = _mm256_min_epi32(id8, _mm256_shuffle_epi32(id8, 0xB1));
                const float bw = _mm256_cvtss_f32(mx);
                const int32_t bid = _mm256_cvtsi256_si32(id8);
                if (bw > fw || (bw == fw && bid < far)) {
                    fw = bw;
                    far = bid;
                }
            }
            if ((pass == 0 && !ok) || far < 0) continue;
            // the far end's record and vector are needed only at the end (nothing
            // in between reads its row: it is in U from here on)
            const char *fr = reinterpret_cast<const char *>(G.rec(far));
            for (size_t o = 0; o < rec_bytes; o += 64) __builtin_prefetch(fr + o);
            const char *fv = reinterpret_cast<const char *>(vec + (size_t)far * vs);
            for (int o = 0; o < m * 4; o += 64) __builtin_prefetch(fv + o);
            G.half_remove(b, far);
            push(b, db, false);
            push(far, 0.0f, true);
        }
    }
    if (nu < d) {
        // (the build stops here; the cut edges are completed so that no row
        // holds half an edge)
        for (int t = 1; t < nu; t += 2) G.half_remove(U[t], U[t - 1]);
        return false;
    }
    for (int t = 1; t < nu; t += 2) G.half_remove(U[t], U[t - 1]);
    for (int j = 0; j < nu; ++j) G.add_edge(v, U[j], dist_of(j));
    return !G.broken;
}

__global__ void fill_i32(int32_t *p, int64_t n, int32_t val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// adj[row[r]] <- the neighbour ids of record row[r] (read from pinned host memory)
__global__ void gather_rows(int32_t *adj, int d, const int32_t *rows, int64_t nrows,
                            const int32_t *records, int64_t stride) {
    const int64_t total = nrows * d;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / d;
        const int64_t a = rows[r];
        adj[a * d + (i - r * d)] = records[a * stride + 2 + (i - r * d)];
    }
}

int64_t block_size(int64_t nv, int64_t batch, int64_t left) {
    int64_t b = nv / 8;
    if (b < 1) b = 1;
    if (b > batch) b = batch;
    if (b > left) b = left;
    return b;
}

// Device and pinned host buffers of one build, freed on every return path once
// the stream has drained (an error may leave work in flight).
struct Buffers {
    hipStream_t st;
    void *dev[6] = {};
    void *host[8] = {};
    hipEvent_t ev = nullptr;
    explicit Buffers(hipStream_t s) : st(s) {}
    ~Buffers() {
        (void)hipStreamSynchronize(st);
        if (ev) (void)hipEventDestroy(ev);
        for (void *p : dev)
            if (p) (void)hipFree(p);
        for (void *p : host)
            if (p) (void)hipHostFree(p);
    }
};

}  // namespace

extern "C" deg_status deg_build_graph(const deg_vectors *v, const float *host_vectors,
                                      int64_t host_stride, const deg_build_params *p,
                                      int32_t *adjacency, float *weights, int64_t *counters,
                                      void *stream) {
    if (!v || !p || !host_vectors || !adjacency || !v->data) return DEG_ERR_INVALID_ARG;
    const int d = p->degree;
    const int64_t n = v->n;
    const int m = v->dim;
    if (v->dtype != DEG_F32 || (v->metric != DEG_METRIC_L2 && v->metric != DEG_METRIC_IP))
        return DEG_ERR_INVALID_ARG;
    if (d < 4 || d > 128 || (d & 1) || n < (int64_t)d + 1 || n > INT32_MAX || m < 1 ||
        host_stride < m || p->k_ext < 1 || p->k_ext > 1024 || !(p->eps_ext >= 0.0f) ||
        p->batch < 1 || p->lag < 0 || p->lag > 1)
        return DEG_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    HostGraph G(n, d);
    if (!G.words) return DEG_ERR_HIP;
    // the smallest DEG: the complete graph on vertices 0..d
    for (int32_t a = 0; a <= d; ++a)
        for (int32_t b = a + 1; b <= d; ++b)
            G.add_edge(a, b, dist_c32x4(host_vectors + (size_t)a * host_stride,
                                        host_vectors + (size_t)b * host_stride, m, v->metric));
    if (G.broken) return DEG_ERR_INVALID_ARG;

    const int64_t cap = p->batch < n ? p->batch : n;
    const int k = p->k_ext;
    deg_graph g{adjacency, n, d, d};
    deg_search_opts o;
    memset(&o, 0, sizeof(o));
    const size_t ws = deg_search_workspace_bytes(v, &g, cap, k, &o);
    if (ws == 0) return DEG_ERR_UNSUPPORTED;

    Buffers B(st);
    int32_t *d_seeds, *d_ids, *d_stats, *d_rows;
    float *d_ds;
    int32_t *h_ids2[2], *h_stats2[2], *h_up;
    float *h_ds2[2];
    // changed records per upload: at most d + 1 per new vertex (the vertex and the
    // d distinct ends of its d/2 cut edges) of one block, of two blocks for the last
    // upload with lag 1, and the smallest DEG's before the first
    const int64_t up_cap = 2 * cap * (d + 1) + d + 1;
    if (hipMalloc((void **)&d_seeds, sizeof(int32_t) * cap) != hipSuccess) return DEG_ERR_HIP;
    B.dev[0] = d_seeds;
    if (hipMalloc((void **)&d_ids, sizeof(int32_t) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.dev[1] = d_ids;
    if (hipMalloc((void **)&d_ds, sizeof(float) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.dev[2] = d_ds;
    if (hipMalloc((void **)&d_stats, sizeof(int32_t) * cap * 4) != hipSuccess) return DEG_ERR_HIP;
    B.dev[3] = d_stats;
    const size_t rows_bytes = (sizeof(int32_t) * up_cap + 255) / 256 * 256;
    if (hipMalloc((void **)&d_rows, rows_bytes + ws) != hipSuccess) return DEG_ERR_HIP;
    B.dev[4] = d_rows;
    void *d_ws = reinterpret_cast<char *>(d_rows) + rows_bytes;
    // two sets of host results: with lag 1 one block's results are edited in while the
    // next block's arrive
    for (int b = 0; b < 2; ++b) {
        if (hipHostMalloc((void **)&h_ids2[b], sizeof(int32_t) * cap * k) != hipSuccess)
            return DEG_ERR_HIP;
        B.host[b == 0 ? 0 : 4] = h_ids2[b];
        if (hipHostMalloc((void **)&h_ds2[b], sizeof(float) * cap * k) != hipSuccess)
            return DEG_ERR_HIP;
        B.host[b == 0 ? 1 : 5] = h_ds2[b];
        if (hipHostMalloc((void **)&h_stats2[b], sizeof(int32_t) * cap * 4) != hipSuccess)
            return DEG_ERR_HIP;
        B.host[b == 0 ? 2 : 6] = h_stats2[b];
    }
    if (hipEventCreateWithFlags(&B.ev, hipEventDisableTiming) != hipSuccess) {
        B.ev = nullptr;
        return DEG_ERR_HIP;
    }
    if (hipHostMalloc((void **)&h_up, sizeof(int32_t) * up_cap) != hipSuccess) return DEG_ERR_HIP;
    B.host[3] = h_up;
    int32_t *d_records = nullptr;
    if (hipHostGetDevicePointer((void **)&d_records, G.words, 0) != hipSuccess || !d_records)
        return DEG_ERR_HIP;

    fill_i32<<<256, 256, 0, st>>>(adjacency, n * d, -1);
    fill_i32<<<64, 256, 0, st>>>(d_seeds, cap, 0);

    // the changed rows go to the device: their vertex ids are copied, the rows
    // themselves are read from the records by the gather kernel (the host edits
    // them again only after the gather has finished: `gathering` until then)
    bool gathering = false;
    auto gather_done = [&]() -> bool {
        if (!gathering) return true;
        gathering = false;
        return hipEventSynchronize(B.ev) == hipSuccess;
    };
    auto upload = [&]() -> deg_status {
        const int64_t nr = (int64_t)G.dirty.size();
        if (nr == 0) return DEG_OK;
        if (nr > up_cap) return DEG_ERR_HIP;
        memcpy(h_up, G.dirty.data(), sizeof(int32_t) * nr);
        if (hipMemcpyAsync(d_rows, h_up, sizeof(int32_t) * nr, hipMemcpyHostToDevice, st) !=
            hipSuccess)
            return DEG_ERR_HIP;
        int blocks = (int)((nr * d + 255) / 256);
        if (blocks > 8192) blocks = 8192;
        gather_rows<<<blocks, 256, 0, st>>>(adjacency, d, d_rows, nr, d_records, G.stride);
        G.dirty.clear();
        ++G.block;
        if (hipGetLastError() != hipSuccess || hipEventRecord(B.ev, st) != hipSuccess)
            return DEG_ERR_HIP;
        gathering = true;
        return DEG_OK;
    };

    int64_t blocks = 0, searches = 0, phase2 = 0, lossy = 0;
    using clk = std::chrono::steady_clock;
    clk::duration t_search{}, t_edit{};
    const float *qbase = reinterpret_cast<const float *>(v->data);
    deg_status s = DEG_OK;
    // the edits of one block (results in set r), vertex by vertex in id order
    auto edit_block = [&](int64_t first, int64_t count, int r) -> deg_status {
        const int32_t *h_ids = h_ids2[r], *h_stats = h_stats2[r];
        const float *h_ds = h_ds2[r];
        constexpr int AHEAD = 2;
        for (int64_t i = 0; i < AHEAD && i < count; ++i) prefetch_result(G, h_ids + i * k, k);
        for (int64_t i = 0; i < count; ++i) {
            if (i + AHEAD < count) prefetch_result(G, h_ids + (i + AHEAD) * k, k);
            const int32_t fl = h_stats[i * 4 + 2];
            if (fl & DEG_FLAG_BAD_ID) return DEG_ERR_HIP;  // the device graph is corrupt
            if (fl & DEG_FLAG_QUEUE_OVERFLOW) ++lossy;
            int ns = 0;
            while (ns < k && h_ids[i * k + ns] >= 0) ++ns;
            if (!extend_vertex(G, host_vectors, host_stride, m, v->metric, (int32_t)(first + i),
                               h_ids + i * k, h_ds + i * k, ns, phase2))
                return DEG_ERR_UNSUPPORTED;  // the search result cannot supply d neighbours
        }
        return DEG_OK;
    };
    const bool lag = p->lag == 1;
    int cur = 0;
    int64_t pend_s = 0, pend_n = 0;  // lag 1: the block whose edits come after the next searches
    for (int64_t s0 = (int64_t)d + 1; s0 < n || pend_n > 0;) {
        // vertices already in the graph: all but the pending block
        const int64_t bsz = s0 < n ? block_size(s0 - pend_n, cap, n - s0) : 0;
        clk::time_point t0 = clk::now();
        if (bsz > 0) {
            if ((s = upload()) != DEG_OK) return s;
            s = deg_search(v, &g, qbase + s0 * (int64_t)v->row_stride, bsz, v->row_stride, d_seeds,
                           1, k, p->eps_ext, &o, d_ids, d_ds, d_stats, d_ws, ws, st);
            if (s != DEG_OK) return s;
            if (hipMemcpyAsync(h_ids2[cur], d_ids, sizeof(int32_t) * bsz * k,
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(h_ds2[cur], d_ds, sizeof(float) * bsz * k, hipMemcpyDeviceToHost,
                               st) != hipSuccess ||
                hipMemcpyAsync(h_stats2[cur], d_stats, sizeof(int32_t) * bsz * 4,
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                return DEG_ERR_HIP;
            ++blocks;
            searches += bsz;
        }
        if (lag && pend_n > 0) {
            // the previous block's edits run while this block searches
            if (!gather_done()) return DEG_ERR_HIP;
            t_search += clk::now() - t0;
            t0 = clk::now();
            if ((s = edit_block(pend_s, pend_n, cur ^ 1)) != DEG_OK) return s;
            t_edit += clk::now() - t0;
            t0 = clk::now();
        }
        if (bsz > 0 && hipStreamSynchronize(st) != hipSuccess) return DEG_ERR_HIP;
        gathering = false;
        t_search += clk::now() - t0;
        if (lag) {
            pend_s = s0;
            pend_n = bsz;
            cur ^= 1;
        } else if (bsz > 0) {
            t0 = clk::now();
            if ((s = edit_block(s0, bsz, cur)) != DEG_OK) return s;
            t_edit += clk::now() - t0;
        }
        s0 += bsz;
    }
    if ((s = upload()) != DEG_OK) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return DEG_ERR_HIP;
    if (weights)
        for (int64_t a = 0; a < n; ++a)
            for (int j = 0; j < d; ++j) weights[a * d + j] = G.ws((int32_t)a)[j];
    if (counters) {
        counters[0] = blocks;
        counters[1] = searches;
        counters[2] = phase2;
        counters[3] = lossy;
        counters[4] = std::chrono::duration_cast<std::chrono::microseconds>(t_search).count();
        counters[5] = std::chrono::duration_cast<std::chrono::microseconds>(t_edit).count();
    }
    return DEG_OK;
}
