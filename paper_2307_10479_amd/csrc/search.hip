// Entry points deg_search, deg_search_indexed and deg_search_batch: argument
// checks, launch configuration and the persistent launch.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <mutex>

#include "deg.h"
#include "host_util.h"
#include "search_impl.h"

namespace degk {

// Clears the work counter and the owner words of the shared visited tables
// (a kernel, not a memset, so that the launch can be captured in a graph).
__global__ void reset_kernel(int32_t *counter, int32_t *owners, int npool) {
    if (threadIdx.x == 0) *counter = 0;
    for (int i = (int)threadIdx.x; i < npool; i += (int)blockDim.x) owners[i] = 0;
}

// Workspace visited tables: the first holds 16384 slots (64 KiB), a wave's own
// region chains 16384, 65536 and 262144 slots (1.3 MiB), and larger sets take
// one of up to 64 shared tables sized for all n vertices (a query that needs
// one waits while all are held, so they are for the rare very long search). A
// private table is left at 3/8 load, so that most probes end within the eight
// slots of one read.
constexpr int HG_FIRST = 16384;
// S: capacity 16384 by default (at these sizes no search holds that many live
// candidates, so the result is Algorithm 1's exactly), 512 keys of it in LDS.
constexpr int DEFAULT_L = 16384;
constexpr int DEFAULT_BCAP = 512;
constexpr int HG_PRIV_MAX = 262144;
constexpr int POOL_MAX = 64;

static KernelFn pick_kernel(int dt, int metric, int qch, int rreg, int mode) {
    switch (dt) {
        case DT_F32: return pick_kernel_f32(metric, qch, rreg, mode);
        case DT_BF16: return pick_kernel_bf16(metric, qch, rreg, mode);
        default: return pick_kernel_fp8(metric, qch, rreg, mode);
    }
}

struct LaunchCfg {
    KernelFn fn;
    int H, hshift, L, bcap, scap, rreg, qch;
    int64_t gcap;  // far part of S per wave (keys)
    int hg0, hg_priv, hg_cap, npool;
    int64_t region;  // slots per wave
    size_t lds;
    int grid;
    int resident;  // blocks of the kernel resident per CU at this LDS size
    size_t off_region, off_pool, off_g, ws_bytes;
};

static int64_t pow2_at_least(int64_t x) {
    int64_t p = 8;
    while (p < x) p <<= 1;
    return p;
}

// Sizes of the workspace visited tables for n vertices: the largest holds n
// ids at 3/4 load; a wave's region holds the chain hg0, 4 hg0, ... up to
// priv_max slots; npool shared tables serve longer queries.
static void size_tables(LaunchCfg &c, int64_t n, int priv_max, int pool_max) {
    c.hg_cap = (int)pow2_at_least((4 * n + 2) / 3);
    int h0 = HG_FIRST > 4 * c.H ? HG_FIRST : 4 * c.H;
    c.hg0 = h0 < c.hg_cap ? h0 : c.hg_cap;
    c.hg_priv = priv_max < c.hg_cap ? priv_max : c.hg_cap;
    if (c.hg_priv < c.hg0) c.hg_priv = c.hg0;
    int64_t region = 0, t = c.hg0;
    for (;;) {
        region += t;
        if (t >= c.hg_cap) break;
        int64_t nt = 4 * t < c.hg_cap ? 4 * t : c.hg_cap;
        if (nt > c.hg_priv) break;
        t = nt;
    }
    c.region = region;
    c.npool = t < c.hg_cap ? (c.grid < pool_max ? c.grid : pool_max) : 0;
    c.off_region = 256 + ((size_t)4 * c.npool + 255) / 256 * 256;
    c.off_pool = c.off_region + (size_t)c.grid * (size_t)region * 4;
    c.off_g = c.off_pool + (size_t)c.npool * (size_t)c.hg_cap * 4;
    c.ws_bytes = c.off_g + (size_t)c.grid * (size_t)c.gcap * 8;
}

static int ilog2(int x) {
    int s = 0;
    while ((1 << s) < x) ++s;
    return s;
}

static deg_status validate_common(const deg_vectors *v, const deg_graph *g, int32_t kmax,
                                  const deg_search_opts *o, bool need_f32) {
    if (!v || !g || !v->data || !g->adj) return DEG_ERR_INVALID_ARG;
    if (v->n <= 0 || v->n != g->n || v->n > 0x7fffffffLL) return DEG_ERR_INVALID_ARG;
    if (v->dim < 1 || v->row_stride < v->dim || (v->row_stride & 3)) return DEG_ERR_INVALID_ARG;
    if (v->dtype < DEG_F32 || v->dtype > DEG_FP8_E4M3) return DEG_ERR_INVALID_ARG;
    if (v->metric != DEG_METRIC_L2 && v->metric != DEG_METRIC_IP) return DEG_ERR_INVALID_ARG;
    if (v->dtype == DEG_FP8_E4M3 && !v->scale) return DEG_ERR_INVALID_ARG;
    if (((v->dim + 3) / 4 + 31) / 32 > 12) return DEG_ERR_UNSUPPORTED;
    if (g->degree < 4 || (g->degree & 1) || g->degree > 128 || g->row_stride < g->degree)
        return DEG_ERR_INVALID_ARG;
    // the stop features count a row as one batch: rows of up to one wave
    if (g->degree > 64 && o && (o->stop || o->trace)) return DEG_ERR_UNSUPPORTED;
    if (kmax < 1 || kmax > 1024) return DEG_ERR_INVALID_ARG;
    int kp = kmax;
    if (o && o->k_pool > kp) kp = o->k_pool;
    if (kp > 1024) return DEG_ERR_INVALID_ARG;
    if (kp > 512 && o && (o->stop || o->trace)) return DEG_ERR_UNSUPPORTED;  // stop features: k <= 512
    // rows longer than a wave: kernels for pools of up to 256 and up to 512 dims
    if (g->degree > 64 && (kp > 256 || ((v->dim + 3) / 4 + 31) / 32 > 4)) return DEG_ERR_UNSUPPORTED;
    bool rerank = v->dtype != DEG_F32 || (o && (o->rerank || o->k_pool > kmax));
    if ((rerank || need_f32) && !v->f32_data) return DEG_ERR_INVALID_ARG;
    if (v->f32_data && (v->f32_stride < v->dim || (v->f32_stride & 3))) return DEG_ERR_INVALID_ARG;
    if (o && (o->queue_cap < 0 || o->queue_cap > (1 << 24))) return DEG_ERR_INVALID_ARG;
    if (o && o->queue_lds && (o->queue_lds < 256 || o->queue_lds > 8192 || (o->queue_lds & 63)))
        return DEG_ERR_INVALID_ARG;
    if (o && o->hash_slots && (o->hash_slots < 256 || o->hash_slots > 16384 ||
                               (o->hash_slots & (o->hash_slots - 1))))
        return DEG_ERR_INVALID_ARG;
    if (o && o->stop) {
        const deg_stop_model *s = o->stop;
        if (!s->weights_bf16 || !s->feat_mean || !s->feat_inv_std || s->interval < 1)
            return DEG_ERR_INVALID_ARG;
    }
    if (o && o->trace && (o->trace_rows_per_query < 1 || o->trace_interval < 1))
        return DEG_ERR_INVALID_ARG;
    if (o && ((o->exclude_offsets == nullptr) != (o->exclude_ids == nullptr)))
        return DEG_ERR_INVALID_ARG;
    return DEG_OK;
}

static LaunchCfg make_cfg(const deg_vectors *v, const deg_graph *g, int64_t nq, int32_t kmax,
                          const deg_search_opts *o, int priv_max = HG_PRIV_MAX) {
    LaunchCfg c;
    int kp = kmax;
    if (o && o->k_pool > kp) kp = o->k_pool;
    c.rreg = kp <= 64 ? 1 : (kp <= 128 ? 2 : (kp <= 256 ? 4 : (kp <= 512 ? 8 : 16)));
    int nch = (v->dim + 3) / 4;
    int q = (nch + 31) / 32;
    c.qch = q <= 1 ? 1 : (q <= 2 ? 2 : (q <= 4 ? 4 : 12));
    int L = (o && o->queue_cap > 0) ? o->queue_cap : DEFAULT_L;
    c.L = L;
    c.bcap = (o && o->queue_lds) ? o->queue_lds : DEFAULT_BCAP;
    c.scap = ((c.bcap > kp ? c.bcap : kp) + 63) / 64 * 64;  // B / rerank buffer
    c.gcap = (int64_t)L + 4 * 64;  // S never holds more than L + a row at the end of a push
    const TuneEntry *t = tune_lookup(v->dtype, v->dim, g->degree, kp);
    // untuned default: a small LDS table and more resident waves (the workspace
    // table takes over at 3/4 load; measured best or near-best on every workload)
    int H = (o && o->hash_slots) ? o->hash_slots : (t ? t->hash_slots : 512);
    c.H = H;
    c.hshift = 32 - ilog2(H);
    c.lds = 4 * (size_t)H + 8 * (size_t)c.scap + 8 * 128 + 8 * 64 * (size_t)c.rreg + 4 * 64 + 4 * 64;
    const bool feat = o && (o->stop || o->trace);
    c.fn = pick_kernel(v->dtype, v->metric, c.qch, c.rreg, feat ? 1 : (g->degree > 64 ? 2 : 0));
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(c.fn), 64,
                                                     c.lds) != hipSuccess || nb < 1)
        nb = 1;
    c.resident = nb;
    int cus = deg_device_cu_count();
    int64_t grid = (int64_t)nb * cus;
    // (a request beyond the resident waves would only add blocks that start once the
    // queue has drained: it is capped at residency)
    if (t && t->waves_per_cu > 0 && t->waves_per_cu < nb) grid = (int64_t)t->waves_per_cu * cus;
    if (o && o->waves_per_cu > 0) grid = (int64_t)(o->waves_per_cu < nb ? o->waves_per_cu : nb) * cus;
    if (grid > nq) grid = nq;
    if (grid < 1) grid = 1;
    c.grid = (int)grid;
    size_tables(c, v->n, priv_max, POOL_MAX);
    return c;
}

static deg_status launch(const LaunchCfg &c, SearchParams &P, void *ws, size_t ws_bytes,
                         hipStream_t st) {
    if (c.lds > 64 * 1024 || c.fn == nullptr) return DEG_ERR_UNSUPPORTED;
    if (ws_bytes < c.ws_bytes || !ws) return DEG_ERR_WORKSPACE;
    char *w = reinterpret_cast<char *>(ws);
    P.counter = reinterpret_cast<int32_t *>(w);
    P.pool_owner = reinterpret_cast<int32_t *>(w + 256);
    P.spill = reinterpret_cast<int32_t *>(w + c.off_region);
    P.pool = reinterpret_cast<int32_t *>(w + c.off_pool);
    P.gspace = reinterpret_cast<uint64_t *>(w + c.off_g);
    P.L = c.L;
    P.bcap = c.bcap;
    P.scap = c.scap;
    P.gcap = c.gcap;
    P.H = c.H;
    P.hshift = c.hshift;
    P.hg0 = c.hg0;
    P.hg_priv = c.hg_priv;
    P.hg_cap = c.hg_cap;
    P.region = c.region;
    P.npool = c.npool;
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, st, P.counter, P.pool_owner, c.npool);
    hipLaunchKernelGGL(c.fn, dim3(c.grid), dim3(64), c.lds, st, P);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}

static void fill_common(SearchParams &P, const deg_vectors *v, const deg_graph *g, int32_t k,
                        const deg_search_opts *o) {
    memset(&P, 0, sizeof(P));
    P.vec = v->data;
    P.scale = v->scale;
    P.f32 = v->f32_data;
    P.n = v->n;
    P.dim = v->dim;
    P.vstride = v->row_stride;
    P.f32_stride = v->f32_stride;
    P.adj = g->adj;
    P.degree = g->degree;
    P.astride = g->row_stride;
    P.k = k;
    P.kpool = (o && o->k_pool > k) ? o->k_pool : k;
    P.rerank = (v->dtype != DEG_F32 || (o && (o->rerank || o->k_pool > k))) ? 1 : 0;
    if (o && o->stop) {
        P.stop_w = o->stop->weights_bf16;
        P.stop_mean = o->stop->feat_mean;
        P.stop_istd = o->stop->feat_inv_std;
        // sigmoid(z) >= tau  <=>  z >= log(tau / (1 - tau))
        auto logit = [](float tau) {
            return tau <= 0.f ? -__builtin_inff()
                              : (tau >= 1.f ? __builtin_inff() : logf(tau / (1.f - tau)));
        };
        P.stop_tau = logit(o->stop->tau);
        P.stop_interval = o->stop->interval;
        P.stop_long_hops = o->stop->long_hops > 0 ? o->stop->long_hops : 0x7fffffff;
        P.stop_tau_long = o->stop->long_hops > 0 ? logit(o->stop->tau_long) : P.stop_tau;
    }
    if (o) {
        P.ex_off = o->exclude_offsets;
        P.ex_ids = o->exclude_ids;
    }
    if (o && o->trace) {
        P.trace = o->trace;
        P.trace_rows = o->trace_rows_per_query;
        P.trace_interval = o->trace_interval;
    }
}

}  // namespace degk

using namespace degk;

extern "C" size_t deg_search_workspace_bytes(const deg_vectors *v, const deg_graph *g, int64_t nq,
                                             int32_t k, const deg_search_opts *o) {
    if (validate_common(v, g, k, o, false) != DEG_OK || nq < 0) return 0;
    return make_cfg(v, g, nq < 1 ? 1 : nq, k, o).ws_bytes;
}

extern "C" int32_t deg_search_resident_waves(const deg_vectors *v, const deg_graph *g, int32_t k,
                                             const deg_search_opts *o) {
    if (validate_common(v, g, k, o, false) != DEG_OK) return 0;
    const LaunchCfg c = make_cfg(v, g, 1, k, o);
    return c.fn ? c.resident : 0;
}

extern "C" deg_status deg_search(const deg_vectors *v, const deg_graph *g, const float *queries,
                                 int64_t nq, int64_t q_stride, const int32_t *seed_ids,
                                 int32_t n_seeds, int32_t k, float eps, const deg_search_opts *o,
                                 int32_t *out_ids, float *out_dists, int32_t *out_stats,
                                 void *workspace, size_t ws_bytes, void *stream) {
    deg_status s = validate_common(v, g, k, o, false);
    if (s != DEG_OK) return s;
    if (nq < 0 || (nq > 0 && (!queries || !seed_ids || !out_ids || !out_dists)))
        return DEG_ERR_INVALID_ARG;
    if (q_stride < v->dim || n_seeds < 1 || n_seeds > 64 || !(eps >= 0.f))
        return DEG_ERR_INVALID_ARG;
    if (nq == 0) return DEG_OK;
    if (nq > 0x7fffffffLL) return DEG_ERR_INVALID_ARG;
    LaunchCfg c = make_cfg(v, g, nq, k, o);
    SearchParams P;
    fill_common(P, v, g, k, o);
    P.mode = MODE_VEC;
    P.queries = queries;
    P.qstride = q_stride;
    P.seeds = seed_ids;
    P.nseeds = n_seeds;
    P.nq = nq;
    P.eps = eps;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    P.out_stats = out_stats;
    return launch(c, P, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

extern "C" deg_status deg_search_indexed(const deg_vectors *v, const deg_graph *g,
                                         const int32_t *query_ids, int64_t nq, int32_t k,
                                         float eps, const deg_search_opts *o, int32_t *out_ids,
                                         float *out_dists, int32_t *out_stats, void *workspace,
                                         size_t ws_bytes, void *stream) {
    deg_status s = validate_common(v, g, k, o, true);
    if (s != DEG_OK) return s;
    if (nq < 0 || (nq > 0 && (!query_ids || !out_ids || !out_dists))) return DEG_ERR_INVALID_ARG;
    if (!(eps >= 0.f)) return DEG_ERR_INVALID_ARG;
    if (nq == 0) return DEG_OK;
    if (nq > 0x7fffffffLL) return DEG_ERR_INVALID_ARG;
    LaunchCfg c = make_cfg(v, g, nq, k, o);
    SearchParams P;
    fill_common(P, v, g, k, o);
    P.mode = MODE_INDEXED;
    P.qids = query_ids;
    P.nseeds = 1;
    P.nq = nq;
    P.eps = eps;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    P.out_stats = out_stats;
    return launch(c, P, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

extern "C" deg_status deg_search_batch(const deg_vectors *v, const deg_graph *g,
                                       const float *queries, int64_t n_query_rows, int64_t q_stride,
                                       const deg_query_desc *descs, int64_t nq, int32_t k_max,
                                       const deg_search_opts *o, int32_t *out_ids,
                                       float *out_dists, int32_t *out_stats, void *workspace,
                                       size_t ws_bytes, void *stream) {
    deg_status s = validate_common(v, g, k_max, o, true);
    if (s != DEG_OK) return s;
    if (nq < 0 || (nq > 0 && (!descs || !out_ids || !out_dists))) return DEG_ERR_INVALID_ARG;
    if (queries && (q_stride < v->dim || n_query_rows < 0)) return DEG_ERR_INVALID_ARG;
    if (nq == 0) return DEG_OK;
    if (nq > 0x7fffffffLL) return DEG_ERR_INVALID_ARG;
    LaunchCfg c = make_cfg(v, g, nq, k_max, o);
    SearchParams P;
    fill_common(P, v, g, k_max, o);
    P.kpool = (o && o->k_pool > 0) ? o->k_pool : 0;
    P.mode = MODE_BATCH;
    P.queries = queries;
    P.nqrows = queries ? n_query_rows : 0;
    P.qstride = q_stride;
    P.descs = descs;
    P.nseeds = 1;
    P.nq = nq;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    P.out_stats = out_stats;
    return launch(c, P, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- no-allocation variant
// deg_search_noalloc keeps its workspace in one file-scope device array per
// GPU (NOALLOC_BYTES, held while the library is loaded). Host code reaches it
// only through the device address hipGetSymbolAddress returns for the current
// device, taken once per device and kept.
namespace degk {

constexpr size_t NOALLOC_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[128];

static deg_status scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 128) return DEG_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return DEG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DEG_OK;
}

// The launch shaped to fit the scratch array: each wave keeps only the first
// visited table (hg0 slots), larger sets use at most 4 shared tables, and the
// persistent grid shrinks until the regions fit (the grid size changes no
// result). False if even one wave and one shared table do not fit.
static bool fit_noalloc(LaunchCfg &c, int64_t n) {
    int pool_max = 4;
    const int grid0 = c.grid;
    for (;;) {
        size_tables(c, n, 0, pool_max);
        if (c.ws_bytes <= NOALLOC_BYTES) return true;
        const size_t fixed = c.off_region + (size_t)c.npool * (size_t)c.hg_cap * 4;
        const size_t per_wave = (size_t)c.region * 4 + (size_t)c.gcap * 8;
        if (fixed + per_wave <= NOALLOC_BYTES) {
            size_t g = (NOALLOC_BYTES - fixed) / per_wave;
            c.grid = (int)(g < (size_t)grid0 ? g : (size_t)grid0);
            if (c.grid < 1) c.grid = 1;
            size_tables(c, n, 0, pool_max);
            if (c.ws_bytes <= NOALLOC_BYTES) return true;
        }
        if (pool_max > 1) {
            pool_max = 1;
            c.grid = grid0;
            continue;
        }
        return false;
    }
}

}  // namespace degk

extern "C" deg_status deg_search_noalloc(const deg_vectors *v, const deg_graph *g,
                                         const float *queries, int64_t nq, int64_t q_stride,
                                         const int32_t *seed_ids, int32_t n_seeds, int32_t k,
                                         float eps, const deg_search_opts *o, int32_t *out_ids,
                                         float *out_dists, int32_t *out_stats, void *stream) {
    deg_status s = validate_common(v, g, k, o, false);
    if (s != DEG_OK) return s;
    if (nq < 0 || (nq > 0 && (!queries || !seed_ids || !out_ids || !out_dists)))
        return DEG_ERR_INVALID_ARG;
    if (q_stride < v->dim || n_seeds < 1 || n_seeds > 64 || !(eps >= 0.f))
        return DEG_ERR_INVALID_ARG;
    if (nq == 0) return DEG_OK;
    if (nq > 0x7fffffffLL) return DEG_ERR_INVALID_ARG;
    LaunchCfg c = make_cfg(v, g, nq, k, o, 0);
    if (!fit_noalloc(c, v->n)) return DEG_ERR_WORKSPACE;
    void *ws = nullptr;
    s = scratch_address(&ws);
    if (s != DEG_OK) return s;
    SearchParams P;
    fill_common(P, v, g, k, o);
    P.mode = MODE_VEC;
    P.queries = queries;
    P.qstride = q_stride;
    P.seeds = seed_ids;
    P.nseeds = n_seeds;
    P.nq = nq;
    P.eps = eps;
    P.out_ids = out_ids;
    P.out_dists = out_dists;
    P.out_stats = out_stats;
    return launch(c, P, ws, NOALLOC_BYTES, static_cast<hipStream_t>(stream));
}
