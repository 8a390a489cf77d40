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
// schedule. The optional optimizeEdge step (Algorithm 4) is not part of this
// entry point: its searches depend on each other's edits.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "deg.h"

namespace {

// One FP32 distance in the library's fixed order: 32 partial sums, the
// 4-dim chunk c feeding partial c mod 32 with fused multiply-adds in
// increasing dim order, then the halving tree over the partials.
float dist_c32x4(const float *x, const float *q, int m, int metric) {
    float p[32];
    for (int i = 0; i < 32; ++i) p[i] = 0.0f;
    for (int i = 0; i < m; ++i) {
        const int c = (i >> 2) & 31;
        if (metric == DEG_METRIC_L2) {
            const float t = x[i] - q[i];
            p[c] = fmaf(t, t, p[c]);
        } else {
            p[c] = fmaf(x[i], q[i], p[c]);
        }
    }
    for (int w = 16; w >= 1; w >>= 1)
        for (int i = 0; i < w; ++i) p[i] = p[i] + p[i + w];
    return metric == DEG_METRIC_L2 ? p[0] : 1.0f - p[0];
}

// Host copy of the growing graph: rows of up to d (neighbour, weight) pairs,
// filled from the front; removal keeps the order of the remaining entries.
struct HostGraph {
    int64_t n;
    int d;
    std::vector<int32_t> nbr;
    std::vector<float> w;
    std::vector<int32_t> cnt;
    std::vector<int64_t> stamp;  // block in which the row last changed
    std::vector<int32_t> dirty;  // rows changed since the last upload
    int64_t block = 0;
    bool broken = false;

    HostGraph(int64_t n_, int d_)
        : n(n_), d(d_), nbr((size_t)n_ * d_, -1), w((size_t)n_ * d_, 0.0f), cnt(n_, 0),
          stamp(n_, -1) {}

    void touch(int32_t a) {
        if (stamp[a] != block) {
            stamp[a] = block;
            dirty.push_back(a);
        }
    }
    int find(int32_t a, int32_t b) const {
        const int32_t *r = &nbr[(size_t)a * d];
        for (int j = 0; j < cnt[a]; ++j)
            if (r[j] == b) return j;
        return -1;
    }
    void half_add(int32_t a, int32_t b, float wt) {
        if (cnt[a] >= d) {
            broken = true;
            return;
        }
        nbr[(size_t)a * d + cnt[a]] = b;
        w[(size_t)a * d + cnt[a]] = wt;
        ++cnt[a];
        touch(a);
    }
    void half_remove(int32_t a, int32_t b) {
        int j = find(a, b);
        if (j < 0) {
            broken = true;
            return;
        }
        int32_t *r = &nbr[(size_t)a * d];
        float *ww = &w[(size_t)a * d];
        for (; j + 1 < cnt[a]; ++j) {
            r[j] = r[j + 1];
            ww[j] = ww[j + 1];
        }
        --cnt[a];
        r[cnt[a]] = -1;
        ww[cnt[a]] = 0.0f;
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
    void remove_edge(int32_t a, int32_t b) {
        half_remove(a, b);
        half_remove(b, a);
    }
};

// Steps 3-6 of Sec. 5.2 for vertex v given its search result (sorted ids and
// distances, ns entries). Returns false when the result cannot supply d
// neighbours. `phase2` counts vertices that needed the pass without MRNG check.
bool extend_vertex(HostGraph &G, const float *vec, int64_t vs, int m, int metric, int32_t v,
                   const int32_t *ids, const float *ds, int ns, int64_t &phase2) {
    const int d = G.d;
    std::vector<int32_t> U;
    std::vector<float> Ud;
    U.reserve(d);
    Ud.reserve(d);
    auto in_u = [&](int32_t x) {
        for (int32_t u : U)
            if (u == x) return true;
        return false;
    };
    for (int pass = 0; pass < 2 && (int)U.size() < d; ++pass) {
        if (pass == 1) ++phase2;
        for (int i = 0; i < ns && (int)U.size() < d; ++i) {
            const int32_t b = ids[i];
            const float db = ds[i];
            if (in_u(b)) continue;
            if (pass == 0) {
                // MRNG check of (v, b) against the tentative neighbours u of v
                // that are also neighbours of b: the edge is kept out when it is
                // longer than both other sides of such a triangle
                bool ok = true;
                for (size_t t = 0; t < U.size() && ok; ++t) {
                    const int j = G.find(b, U[t]);
                    if (j < 0) continue;
                    const float wbu = G.w[(size_t)b * d + j];
                    const float mx = Ud[t] > wbu ? Ud[t] : wbu;
                    if (db > mx) ok = false;
                }
                if (!ok) continue;
            }
            // b's longest edge to a vertex outside U (equal weights: smaller id)
            int32_t far = -1;
            float fw = -INFINITY;
            for (int j = 0; j < G.cnt[b]; ++j) {
                const int32_t c = G.nbr[(size_t)b * d + j];
                if (in_u(c)) continue;
                const float wt = G.w[(size_t)b * d + j];
                if (wt > fw || (wt == fw && c < far)) {
                    fw = wt;
                    far = c;
                }
            }
            if (far < 0) continue;
            G.remove_edge(b, far);
            U.push_back(b);
            Ud.push_back(db);
            U.push_back(far);
            Ud.push_back(dist_c32x4(vec + (size_t)far * vs, vec + (size_t)v * vs, m, metric));
        }
    }
    if ((int)U.size() < d) return false;
    for (size_t j = 0; j < U.size(); ++j) G.add_edge(v, U[j], Ud[j]);
    return !G.broken;
}

__global__ void fill_i32(int32_t *p, int64_t n, int32_t val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// rows[r] (d ints) -> adj[ids[r]]
__global__ void scatter_rows(int32_t *adj, int d, const int32_t *ids, const int32_t *rows,
                             int64_t nrows) {
    const int64_t total = nrows * d;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / d;
        adj[(int64_t)ids[r] * d + (i - r * d)] = rows[i];
    }
}

int64_t block_size(int64_t nv, int64_t batch, int64_t left) {
    int64_t b = nv / 8;
    if (b < 1) b = 1;
    if (b > batch) b = batch;
    if (b > left) b = left;
    return b;
}

// Device and pinned host buffers of one build, freed on every return path.
struct Buffers {
    void *dev[6] = {};
    void *host[4] = {};
    ~Buffers() {
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
        p->batch < 1)
        return DEG_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    HostGraph G(n, d);
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

    Buffers B;
    int32_t *d_seeds, *d_ids, *d_stats, *d_rowids, *d_rows;
    float *d_ds;
    int32_t *h_ids, *h_stats, *h_up;
    float *h_ds;
    // dirty rows per block: at most 3 per new vertex (the vertex and both ends of
    // each cut edge are d/2 pairs: v, and d distinct others)
    const int64_t up_cap = cap * (d + 1) + d + 1;
    if (hipMalloc((void **)&d_seeds, sizeof(int32_t) * cap) != hipSuccess) return DEG_ERR_HIP;
    B.dev[0] = d_seeds;
    if (hipMalloc((void **)&d_ids, sizeof(int32_t) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.dev[1] = d_ids;
    if (hipMalloc((void **)&d_ds, sizeof(float) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.dev[2] = d_ds;
    if (hipMalloc((void **)&d_stats, sizeof(int32_t) * cap * 4) != hipSuccess) return DEG_ERR_HIP;
    B.dev[3] = d_stats;
    if (hipMalloc((void **)&d_rows, sizeof(int32_t) * up_cap * (d + 1) + ws) != hipSuccess)
        return DEG_ERR_HIP;
    B.dev[4] = d_rows;
    d_rowids = d_rows + up_cap * d;
    void *d_ws = reinterpret_cast<char *>(d_rows) + sizeof(int32_t) * up_cap * (d + 1);
    if (hipHostMalloc((void **)&h_ids, sizeof(int32_t) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.host[0] = h_ids;
    if (hipHostMalloc((void **)&h_ds, sizeof(float) * cap * k) != hipSuccess) return DEG_ERR_HIP;
    B.host[1] = h_ds;
    if (hipHostMalloc((void **)&h_stats, sizeof(int32_t) * cap * 4) != hipSuccess)
        return DEG_ERR_HIP;
    B.host[2] = h_stats;
    if (hipHostMalloc((void **)&h_up, sizeof(int32_t) * up_cap * (d + 1)) != hipSuccess)
        return DEG_ERR_HIP;
    B.host[3] = h_up;

    fill_i32<<<256, 256, 0, st>>>(adjacency, n * d, -1);
    fill_i32<<<64, 256, 0, st>>>(d_seeds, cap, 0);

    // the changed rows go to the device: packed rows first, their ids after
    auto upload = [&]() -> deg_status {
        const int64_t nr = (int64_t)G.dirty.size();
        if (nr == 0) return DEG_OK;
        if (nr > up_cap) return DEG_ERR_HIP;
        for (int64_t r = 0; r < nr; ++r) {
            memcpy(h_up + r * d, &G.nbr[(size_t)G.dirty[r] * d], sizeof(int32_t) * d);
            h_up[up_cap * d + r] = G.dirty[r];
        }
        if (hipMemcpyAsync(d_rows, h_up, sizeof(int32_t) * nr * d, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(d_rowids, h_up + up_cap * d, sizeof(int32_t) * nr,
                           hipMemcpyHostToDevice, st) != hipSuccess)
            return DEG_ERR_HIP;
        int blocks = (int)((nr * d + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        scatter_rows<<<blocks, 256, 0, st>>>(adjacency, d, d_rowids, d_rows, nr);
        G.dirty.clear();
        ++G.block;
        return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
    };

    int64_t blocks = 0, searches = 0, phase2 = 0, lossy = 0;
    const float *qbase = reinterpret_cast<const float *>(v->data);
    deg_status s = DEG_OK;
    for (int64_t s0 = (int64_t)d + 1; s0 < n;) {
        const int64_t nv = s0;
        const int64_t bsz = block_size(nv, cap, n - s0);
        if ((s = upload()) != DEG_OK) return s;
        s = deg_search(v, &g, qbase + s0 * (int64_t)v->row_stride, bsz, v->row_stride, d_seeds, 1,
                       k, p->eps_ext, &o, d_ids, d_ds, d_stats, d_ws, ws, st);
        if (s != DEG_OK) return s;
        if (hipMemcpyAsync(h_ids, d_ids, sizeof(int32_t) * bsz * k, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(h_ds, d_ds, sizeof(float) * bsz * k, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(h_stats, d_stats, sizeof(int32_t) * bsz * 4, hipMemcpyDeviceToHost,
                           st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return DEG_ERR_HIP;
        ++blocks;
        searches += bsz;
        for (int64_t i = 0; i < bsz; ++i) {
            const int32_t fl = h_stats[i * 4 + 2];
            if (fl & DEG_FLAG_BAD_ID) return DEG_ERR_HIP;  // the device graph is corrupt
            if (fl & DEG_FLAG_QUEUE_OVERFLOW) ++lossy;
            int ns = 0;
            while (ns < k && h_ids[i * k + ns] >= 0) ++ns;
            if (!extend_vertex(G, host_vectors, host_stride, m, v->metric, (int32_t)(s0 + i),
                               h_ids + i * k, h_ds + i * k, ns, phase2))
                return DEG_ERR_UNSUPPORTED;  // the search result cannot supply d neighbours
        }
        s0 += bsz;
    }
    if ((s = upload()) != DEG_OK) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return DEG_ERR_HIP;
    if (weights) memcpy(weights, G.w.data(), sizeof(float) * (size_t)n * d);
    if (counters) {
        counters[0] = blocks;
        counters[1] = searches;
        counters[2] = phase2;
        counters[3] = lossy;
    }
    return DEG_OK;
}
