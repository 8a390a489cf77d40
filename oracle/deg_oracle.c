/*
 * CPU oracle for the Dynamic Exploration Graph (DEG) search path.
 *
 * TEST INFRASTRUCTURE ONLY. Plain, slow, sequential C that follows the
 * paper step by step. It shares no code with the HIP library: only tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Contents (each function cites the passage it follows):
 *   distances            -- Sec. 2.1 notation; fixed FP32 reduction order "C32x4"
 *   or_range_search      -- Algorithm 1 (RangeSearch), with the readings listed below
 *   or_knn64             -- Eq. (knn) in FP64, brute force
 *   graph construction   -- Sec. 5.2 steps 1-6, Algorithm 2 (checkMRNG),
 *                           Algorithm 3 (ExtendGraph), Algorithm 4 (optimizeEdge),
 *                           Algorithm 5 (dynamicEdgeOptimization); a batched
 *                           schedule (searches of a block on one snapshot)
 *   or_check_graph       -- Sec. 5.1 even regularity, undirected, no loops,
 *                           connectivity and 2-edge-connectivity (no bridges)
 *   encodings            -- BF16 round-to-nearest-even, OCP FP8 e4m3 with a row scale
 *   MLP reference        -- FP64 forward/backward of the 16-64-64-1 stop predictor
 *
 * Readings where the paper is silent or inconsistent (all documented in the
 * design notes):
 *   - L2 distance is the squared Euclidean distance; IP distance is 1 - <x,q>.
 *   - Every ordering uses (distance, vertex id) ascending.
 *   - FP32 distances use 32 partial sums over 4-element chunks assigned
 *     round-robin (chunk c -> partial c mod 32), fmaf inside each partial in
 *     increasing index order, then a halving tree p += p + w for w = 16..1.
 *   - Algorithm 1 starts with the checked set C equal to the seeds (the
 *     printed C = {} would let a seed be checked twice).
 *   - The candidate set S may be bounded by a capacity L (0 = unbounded):
 *     a push into a full S evicts the (distance, id)-largest entry.
 *   - The learned stop's state features, its BF16 inference (FP32 in a fixed
 *     order) and its trace rows are defined next to range_search_core.
 *   - threshold = fl32(r * fl32(1 + eps)); r = inf gives inf.
 *   - Exploratory (indexed) search: excluded ids enter S and C but never R.
 *
 * Build: gcc -O3 -mavx2 -mfma -ffp-contract=off -fPIC -shared -pthread
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define OR_L2 0
#define OR_IP 1

/* ------------------------------------------------------------------------ */
/* distances (Sec. 2.1)                                                     */
/* ------------------------------------------------------------------------ */

/*
 * FP32 distance in the fixed C32x4 order, written straight from its
 * definition: chunk c (dims 4c..4c+3) goes to partial c mod 32; inside a
 * partial the products are fused in increasing index order; then a halving
 * tree part[p] += part[p+w] for w = 16, 8, 4, 2, 1.
 */
float or_dist32_def(const float *x, const float *q, int64_t m, int32_t metric) {
    float part[32];
    for (int p = 0; p < 32; ++p) part[p] = 0.0f;
    int64_t nch = (m + 3) / 4;
    for (int64_t c = 0; c < nch; ++c) {
        int p = (int)(c % 32);
        for (int64_t i = 4 * c; i < 4 * c + 4 && i < m; ++i) {
            if (metric == OR_L2) {
                float t = x[i] - q[i];
                part[p] = fmaf(t, t, part[p]);
            } else {
                part[p] = fmaf(x[i], q[i], part[p]);
            }
        }
    }
    for (int w = 16; w >= 1; w >>= 1)
        for (int p = 0; p < w; ++p) part[p] = part[p] + part[p + w];
    return metric == OR_L2 ? part[0] : 1.0f - part[0];
}

/*
 * The same arithmetic, grouped so the compiler can vectorise it: a block of
 * 128 dims holds exactly one chunk per partial (chunk 32r+p -> partial p), so
 * it is applied as four passes j = 0..3 over the 32 partials. Each partial
 * still receives its products in increasing index order. A last partial block
 * is zero-padded: fmaf(0, 0, a) == a exactly and a partial sum is never -0,
 * so padding changes nothing. The result equals or_dist32_def (a test checks
 * this on every dimension used here).
 */
static inline void c32x4_block(const float *xr, const float *qr, float *part, int32_t metric) {
    float a[4][32], b[4][32];
    for (int p = 0; p < 32; ++p)
        for (int j = 0; j < 4; ++j) {
            a[j][p] = xr[4 * p + j];
            b[j][p] = qr[4 * p + j];
        }
    if (metric == OR_L2) {
        for (int j = 0; j < 4; ++j)
            for (int p = 0; p < 32; ++p) {
                float t = a[j][p] - b[j][p];
                part[p] = fmaf(t, t, part[p]);
            }
    } else {
        for (int j = 0; j < 4; ++j)
            for (int p = 0; p < 32; ++p) part[p] = fmaf(a[j][p], b[j][p], part[p]);
    }
}

float or_dist32(const float *x, const float *q, int64_t m, int32_t metric) {
    float part[32];
    for (int p = 0; p < 32; ++p) part[p] = 0.0f;
    int64_t full = m / 128;
    for (int64_t r = 0; r < full; ++r) c32x4_block(x + 128 * r, q + 128 * r, part, metric);
    int64_t rest = m - 128 * full;
    if (rest > 0) {
        float xt[128], qt[128];
        for (int i = 0; i < 128; ++i) {
            xt[i] = i < rest ? x[128 * full + i] : 0.0f;
            qt[i] = i < rest ? q[128 * full + i] : 0.0f;
        }
        c32x4_block(xt, qt, part, metric);
    }
    for (int w = 16; w >= 1; w >>= 1)
        for (int p = 0; p < w; ++p) part[p] = part[p] + part[p + w];
    return metric == OR_L2 ? part[0] : 1.0f - part[0];
}

/* FP64 distance, summed in index order. */
double or_dist64(const float *x, const float *q, int64_t m, int32_t metric) {
    double s = 0.0;
    if (metric == OR_L2) {
        for (int64_t i = 0; i < m; ++i) {
            double t = (double)x[i] - (double)q[i];
            s += t * t;
        }
        return s;
    }
    for (int64_t i = 0; i < m; ++i) s += (double)x[i] * (double)q[i];
    return 1.0 - s;
}

/* ------------------------------------------------------------------------ */
/* the total order (distance, id)                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    float d;
    int32_t id;
} Ent;

static int ent_less(Ent a, Ent b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

/* ------------------------------------------------------------------------ */
/* search state                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *stamp; /* checked set C: stamp[v] == epoch */
    uint32_t epoch;
    int64_t n;
    Ent *heap; /* candidate set S as a binary min-heap */
    int64_t hsize, hcap;
    Ent *R; /* result list, sorted ascending, room for k+1 */
    int64_t rcap;
    int32_t *nbuf; /* unchecked neighbours of the current vertex */
    float *dbuf;
    int64_t ncap;
} Ctx;

static void ctx_init(Ctx *c, int64_t n) {
    memset(c, 0, sizeof(*c));
    c->n = n;
    c->stamp = (uint32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    c->epoch = 0;
    c->hcap = 1024;
    c->heap = (Ent *)malloc(sizeof(Ent) * c->hcap);
    c->rcap = 0;
    c->R = NULL;
    c->ncap = 0;
}

static void ctx_free(Ctx *c) {
    free(c->stamp);
    free(c->heap);
    free(c->R);
    free(c->nbuf);
    free(c->dbuf);
    memset(c, 0, sizeof(*c));
}

static void ctx_new_epoch(Ctx *c) {
    c->epoch++;
    if (c->epoch == 0) {
        memset(c->stamp, 0, sizeof(uint32_t) * (size_t)c->n);
        c->epoch = 1;
    }
}

static void heap_push(Ctx *c, Ent e) {
    if (c->hsize == c->hcap) {
        c->hcap *= 2;
        c->heap = (Ent *)realloc(c->heap, sizeof(Ent) * c->hcap);
    }
    int64_t i = c->hsize++;
    c->heap[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!ent_less(c->heap[i], c->heap[p])) break;
        Ent t = c->heap[i];
        c->heap[i] = c->heap[p];
        c->heap[p] = t;
        i = p;
    }
}

static void heap_sift(Ctx *c, int64_t i) {
    /* restore the heap property at i, moving up or down */
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!ent_less(c->heap[i], c->heap[p])) break;
        Ent t = c->heap[i];
        c->heap[i] = c->heap[p];
        c->heap[p] = t;
        i = p;
    }
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        if (l < c->hsize && ent_less(c->heap[l], c->heap[b])) b = l;
        if (r < c->hsize && ent_less(c->heap[r], c->heap[b])) b = r;
        if (b == i) break;
        Ent t = c->heap[i];
        c->heap[i] = c->heap[b];
        c->heap[b] = t;
        i = b;
    }
}

static Ent heap_pop_at(Ctx *c, int64_t i) {
    Ent e = c->heap[i];
    c->hsize--;
    if (i != c->hsize) {
        c->heap[i] = c->heap[c->hsize];
        heap_sift(c, i);
    }
    return e;
}

static inline float thr_of(float r, float onep) {
    /* threshold r(1+eps) of Algorithm 1; inf stays inf */
    if (isinf(r) || isinf(onep)) return INFINITY;
    return r * onep;
}

/* Views of the data the search reads. */
typedef struct {
    const float *vec;
    int64_t n, m, vs; /* rows, dims, row stride (elements) */
    int32_t metric;
} VecView;

typedef struct {
    const int32_t *adj;
    int64_t stride; /* elements per row */
    const int32_t *cnt; /* optional per-row counts (construction); NULL = `d` each */
    int32_t d;
} AdjView;

typedef struct {
    int64_t hops, evals, max_live, overflow, flags;
} SearchStats;

static inline int is_excluded(int32_t id, const int32_t *ex, int nex) {
    for (int i = 0; i < nex; ++i)
        if (ex[i] == id) return 1;
    return 0;
}

/* Insert into the sorted result list; keep at most k; update r (Alg. 1). */
static void insert_R(Ctx *c, int64_t *rsize, int32_t k, Ent e, float *r) {
    int64_t i = *rsize;
    while (i > 0 && ent_less(e, c->R[i - 1])) {
        c->R[i] = c->R[i - 1];
        --i;
    }
    c->R[i] = e;
    (*rsize)++;
    if (*rsize > k) {
        (*rsize) = k; /* drop the largest entry */
        *r = c->R[k - 1].d;
    }
}

static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Layout of the stop network's parameters (16 -> 64 -> 64 -> 1). */
#define MLP_IN_ 16
#define MLP_H_ 64
#define MOFF_W1 0
#define MOFF_B1 (MOFF_W1 + MLP_H_ * MLP_IN_)
#define MOFF_W2 (MOFF_B1 + MLP_H_)
#define MOFF_B2 (MOFF_W2 + MLP_H_ * MLP_H_)
#define MOFF_W3 (MOFF_B2 + MLP_H_)
#define MOFF_B3 (MOFF_W3 + MLP_H_)

/*
 * Push into S with capacity L (a reading; the paper's S is unbounded): when S
 * already holds L entries, the (distance, id)-largest of S and the new entry
 * is evicted (the new one itself if it is the largest). `ev` receives the
 * smallest distance evicted so far in the current hop, so that the caller can
 * tell whether an entry within the end-of-hop threshold was lost.
 */
static void push_capped(Ctx *c, Ent e, int64_t L, float *ev) {
    if (L <= 0 || c->hsize < L) {
        heap_push(c, e);
        return;
    }
    int64_t mx = 0;
    for (int64_t i = 1; i < c->hsize; ++i)
        if (ent_less(c->heap[mx], c->heap[i])) mx = i;
    if (ent_less(e, c->heap[mx])) {
        Ent out = heap_pop_at(c, mx);
        if (out.d < *ev) *ev = out.d;
        heap_push(c, e);
    } else if (e.d < *ev) {
        *ev = e.d;
    }
}

/* ------------------------------------------------------------------------ */
/* stop-predictor inference (BF16 weights, FP32 arithmetic in a fixed order) */
/* ------------------------------------------------------------------------ */
static inline float bf16_round(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u; /* nearest, ties to even (finite x) */
    memcpy(&x, &u, 4);
    return x;
}

static inline float bf16_value(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

/*
 * Logit of the 16-64-64-1 stop network from BF16 weights w (layout W1[64][16],
 * b1[64], W2[64][64], b2[64], w3[64], b3) and 16 standardised features fs.
 * Definition, all in FP32 with round-to-nearest-even:
 *   x_j  = bf16(fs_j)
 *   h1_i = bf16(relu(b1_i (+) W1_i0 x_0 (+) ... (+) W1_i15 x_15))   fused
 *          multiply-adds in increasing j (each product of two BF16 values is exact)
 *   h2_i = relu(b2_i (+) W2_i0 h1_0 (+) ... (+) W2_i63 h1_63)          same
 *   t_i  = fl(w3_i * h2_i); then the halving tree t_i = fl(t_i + t_{i+w}) for
 *          w = 32, 16, 8, 4, 2, 1; logit = fl(t_0 + b3)
 * relu(s) = s if s > 0, else +0.
 */
float or_mlp_logit_bf16(const uint16_t *w, const float *fs) {
    float x[MLP_IN_], h1[MLP_H_], t[MLP_H_];
    for (int j = 0; j < MLP_IN_; ++j) x[j] = bf16_round(fs[j]);
    for (int i = 0; i < MLP_H_; ++i) {
        float s = bf16_value(w[MOFF_B1 + i]);
        for (int j = 0; j < MLP_IN_; ++j) s = fmaf(bf16_value(w[MOFF_W1 + i * MLP_IN_ + j]), x[j], s);
        h1[i] = bf16_round(s > 0.0f ? s : 0.0f);
    }
    for (int i = 0; i < MLP_H_; ++i) {
        float s = bf16_value(w[MOFF_B2 + i]);
        for (int j = 0; j < MLP_H_; ++j) s = fmaf(bf16_value(w[MOFF_W2 + i * MLP_H_ + j]), h1[j], s);
        float h2 = s > 0.0f ? s : 0.0f;
        t[i] = bf16_value(w[MOFF_W3 + i]) * h2;
    }
    for (int wd = MLP_H_ / 2; wd >= 1; wd /= 2)
        for (int i = 0; i < wd; ++i) t[i] = t[i] + t[i + wd];
    return t[0] + bf16_value(w[MOFF_B3]);
}

/* Logits of B rows (B x 16 standardised features). */
void or_mlp_logits_bf16_rows(const uint16_t *w, const float *X, int64_t B, float *out) {
    for (int64_t b = 0; b < B; ++b) out[b] = or_mlp_logit_bf16(w, X + b * MLP_IN_);
}

/* Per-search options beyond Algorithm 1's own inputs. */
typedef struct {
    int64_t cap_L;      /* capacity of S, 0 = unbounded */
    int order_mode;     /* 0 row order, 1 reversed, 2 shuffled (the result must not depend on it) */
    uint64_t order_seed;
    int want_live;      /* report the largest number of live S entries */
    /* state features (learned stop, trace rows) */
    int32_t k_user;     /* the caller's k (R itself holds the pool of size k) */
    int32_t kind;       /* 0 vector query, 1 exploratory */
    const uint16_t *stop_w; /* NULL = plain rule only */
    const float *stop_mean, *stop_istd;
    float stop_z, stop_z_long; /* logit thresholds */
    int32_t stop_interval, stop_long_hops;
    float *trace;       /* NULL = no trace rows; else trace_rows rows of OR_TRACE_W floats */
    int64_t trace_rows;
    int32_t trace_interval;
} SearchOpts;

#define OR_NFEAT 16
#define OR_TRACE_W 20
#define OR_FLAG_QUEUE_OVERFLOW 1
#define OR_FLAG_LEARNED_STOP 16

/*
 * The 16 search-state features of the stop predictor at a checkpoint (after
 * the pop of hop h passed the threshold test, before its row is expanded).
 * Every quantity is a function of Algorithm 1's state, so any exact
 * implementation computes the same values; all arithmetic is FP32 with
 * correctly rounded division and square root. With kq = min(k, |R|), d1 and
 * dk the distances of R's first and kq-th entries:
 *   0 sqrt(h)                        1 sqrt(evaluations)
 *   2 d1 / dk                        3 d1 / (smallest seed distance)
 *   4 r / (r at the previous checkpoint)
 *   5 sqrt(hops since the first min(pool, 10) entries of R last changed)
 *   6 sqrt(hops since R's first entry last changed)
 *   7 (new candidates of the last expanded row within the end-of-row range r(1+eps)) / d
 *   8 (new candidates of the last expanded row that are in R after it) / d
 *   9 min(64, entries of S that precede R's kq-th entry) / 64
 *  10 min(4, popped distance / dk)    11 min(eps, 4)
 *  12 sqrt(k)                        13 1 for an exploratory query, else 0
 *  14 sqrt(hops since r last changed) 15 constant 1
 * A ratio whose divisor is zero or not finite (or whose dividend is not) is 1.
 */
typedef struct {
    int64_t hops, evals;
    float dseed, rprev;
    int64_t last_top, last_d1, last_r;
    int32_t n_s, n_r;
} FeatState;

static void state_features(const Ctx *c, const FeatState *F, int64_t rsize, float r, float ds,
                           float eps, const SearchOpts *o, int32_t d, float *f) {
    int64_t kq = o->k_user < rsize ? o->k_user : rsize;
    float d1 = rsize > 0 ? c->R[0].d : 0.0f;
    float dk = kq > 0 ? c->R[kq - 1].d : 0.0f;
    int fin_k = kq > 0 && dk > 0.0f;
    int64_t closer = 0;
    for (int64_t i = 0; i < c->hsize; ++i)
        if (kq == 0 || ent_less(c->heap[i], c->R[kq - 1])) closer++;
    if (closer > 64) closer = 64;
    f[0] = sqrtf((float)F->hops);
    f[1] = sqrtf((float)F->evals);
    f[2] = fin_k ? d1 / dk : 1.0f;
    f[3] = (rsize > 0 && F->dseed > 0.0f && isfinite(F->dseed)) ? d1 / F->dseed : 1.0f;
    f[4] = (isfinite(r) && isfinite(F->rprev) && F->rprev > 0.0f) ? r / F->rprev : 1.0f;
    f[5] = sqrtf((float)(F->hops - F->last_top));
    f[6] = sqrtf((float)(F->hops - F->last_d1));
    f[7] = (float)F->n_s / (float)d;
    f[8] = (float)F->n_r / (float)d;
    f[9] = (float)closer / 64.0f;
    f[10] = fin_k ? fminf(4.0f, ds / dk) : 1.0f;
    f[11] = fminf(eps, 4.0f);
    f[12] = sqrtf((float)o->k_user);
    f[13] = (float)o->kind;
    f[14] = sqrtf((float)(F->hops - F->last_r));
    f[15] = 1.0f;
}

/*
 * RangeSearch (Algorithm 1) for one query.
 *   seeds/ns : seed vertices (distinct)
 *   ex/nex   : ids never placed in R (exploratory search excludes the query vertex
 *              and any vertices already shown); they still enter S and C
 *   k        : size of R (the traversal pool)
 *   o        : capacity, row order, features / learned stop / trace rows
 * Output R sorted by (dist, id), returned size; st gets the counters and flags.
 * Capacity: S keeps at most L entries, a push into a full S evicting the
 * (distance, id)-largest. The overflow flag is set when an evicted entry lies
 * within the threshold r(1+eps) at the end of its hop (a live entry was lost;
 * whether that happens does not depend on the order of a row's neighbours).
 */
static int64_t range_search_core(Ctx *c, const VecView *V, const AdjView *G, const float *q,
                                 const int32_t *seeds, int ns, const int32_t *ex, int nex,
                                 int32_t k, float eps, const SearchOpts *o, SearchStats *st) {
    if (c->rcap < (int64_t)k + 1) {
        c->rcap = (int64_t)k + 1;
        c->R = (Ent *)realloc(c->R, sizeof(Ent) * c->rcap);
    }
    if (c->ncap < G->d) {
        c->ncap = G->d;
        c->nbuf = (int32_t *)realloc(c->nbuf, sizeof(int32_t) * c->ncap);
        c->dbuf = (float *)realloc(c->dbuf, sizeof(float) * c->ncap);
    }
    ctx_new_epoch(c);
    c->hsize = 0;
    int64_t rsize = 0;
    float r = INFINITY;
    float onep = 1.0f + eps; /* fl32(1 + eps) */
    SearchStats s = {0, 0, 0, 0, 0};
    uint64_t rs = o->order_seed;
    const int64_t L = o->cap_L;
    const int feat = o->stop_w != NULL || o->trace != NULL;
    const int t10 = k < 10 ? k : 10;
    FeatState F = {0, 0, INFINITY, INFINITY, 0, 0, 0, 0, 0};
    int64_t nrow = 0;
    int32_t to_stop = o->stop_interval, to_trace = o->trace_interval;

    /* C <- seeds; every seed is evaluated once, enters S, and enters R unless excluded */
    float ev = INFINITY;
    for (int i = 0; i < ns; ++i) c->stamp[seeds[i]] = c->epoch;
    for (int i = 0; i < ns; ++i) {
        int32_t t = seeds[i];
        Ent e = {or_dist32(V->vec + (int64_t)t * V->vs, q, V->m, V->metric), t};
        s.evals++;
        if (e.d < F.dseed) F.dseed = e.d;
        push_capped(c, e, L, &ev);
        if (!is_excluded(t, ex, nex)) insert_R(c, &rsize, k, e, &r);
    }
    if (isfinite(ev) && ev <= thr_of(r, onep)) s.overflow = 1;

    while (c->hsize > 0) {
        Ent sv = heap_pop_at(c, 0); /* argmin of S */
        if (sv.d > thr_of(r, onep)) break; /* too far away: return R */
        s.hops++;

        if (feat) { /* checkpoints of the learned stop and of the trace rows */
            int want_stop = 0, want_trace = 0;
            if (o->stop_w) {
                if (--to_stop == 0) {
                    want_stop = 1;
                    to_stop = o->stop_interval;
                }
            }
            if (o->trace) {
                if (--to_trace == 0) {
                    want_trace = nrow < o->trace_rows;
                    to_trace = o->trace_interval;
                }
            }
            if (want_stop || want_trace) {
                float f[OR_NFEAT];
                F.hops = s.hops;
                F.evals = s.evals;
                state_features(c, &F, rsize, r, sv.d, eps, o, G->d, f);
                F.rprev = r;
                if (want_trace) {
                    float *row = o->trace + nrow * OR_TRACE_W;
                    for (int i = 0; i < OR_NFEAT; ++i) row[i] = f[i];
                    row[17] = 0.0f; /* query index: set by the caller */
                    row[18] = (float)s.hops;
                    row[19] = 0.0f;
                    nrow++;
                }
                if (want_stop) {
                    float fs[OR_NFEAT];
                    for (int i = 0; i < OR_NFEAT; ++i)
                        fs[i] = (f[i] - o->stop_mean[i]) * o->stop_istd[i];
                    float z = or_mlp_logit_bf16(o->stop_w, fs);
                    float zt = s.hops >= o->stop_long_hops ? o->stop_z_long : o->stop_z;
                    if (z >= zt) {
                        s.flags |= OR_FLAG_LEARNED_STOP;
                        break;
                    }
                }
            }
        }

        /* N <- N(G,s) \ C ; C <- C u N */
        const int32_t *row = G->adj + (int64_t)sv.id * G->stride;
        int32_t deg = G->cnt ? G->cnt[sv.id] : G->d;
        int nn = 0;
        for (int j = 0; j < deg; ++j) {
            int32_t nb = row[j];
            if (c->stamp[nb] != c->epoch) {
                c->stamp[nb] = c->epoch;
                c->nbuf[nn++] = nb;
            }
        }
        if (o->order_mode == 1) {
            for (int a = 0, b = nn - 1; a < b; ++a, --b) {
                int32_t t = c->nbuf[a];
                c->nbuf[a] = c->nbuf[b];
                c->nbuf[b] = t;
            }
        } else if (o->order_mode == 2) {
            for (int a = nn - 1; a > 0; --a) {
                int b = (int)(splitmix64(&rs) % (uint64_t)(a + 1));
                int32_t t = c->nbuf[a];
                c->nbuf[a] = c->nbuf[b];
                c->nbuf[b] = t;
            }
        }
        Ent top_before[10], first_before = {INFINITY, -1};
        int64_t top_n = rsize < t10 ? rsize : t10;
        float r_before = r;
        if (feat) {
            for (int64_t i = 0; i < top_n; ++i) top_before[i] = c->R[i];
            if (rsize > 0) first_before = c->R[0];
        }
        ev = INFINITY;
        for (int j = 0; j < nn; ++j) {
            int32_t nb = c->nbuf[j];
            float dn = or_dist32(V->vec + (int64_t)nb * V->vs, q, V->m, V->metric);
            c->dbuf[j] = dn;
            s.evals++;
            if (dn <= thr_of(r, onep)) { /* close enough to be analysed later */
                push_capped(c, (Ent){dn, nb}, L, &ev);
                if (dn <= r && !is_excluded(nb, ex, nex)) insert_R(c, &rsize, k, (Ent){dn, nb}, &r);
            }
        }
        if (isfinite(ev) && ev <= thr_of(r, onep)) s.overflow = 1;
        if (feat) {
            /* what the row changed: the front of R, R's first entry, r, acceptances */
            int64_t tn = rsize < t10 ? rsize : t10;
            int changed = tn != top_n;
            for (int64_t i = 0; i < tn && !changed; ++i)
                changed = c->R[i].id != top_before[i].id || c->R[i].d != top_before[i].d;
            if (changed) F.last_top = s.hops;
            if (rsize > 0 && (c->R[0].id != first_before.id || c->R[0].d != first_before.d))
                F.last_d1 = s.hops;
            if (r != r_before) F.last_r = s.hops;
            float te = thr_of(r, onep);
            F.n_s = 0;
            F.n_r = 0;
            for (int j = 0; j < nn; ++j) {
                if (c->dbuf[j] <= te) F.n_s++;
                for (int64_t i = 0; i < rsize; ++i)
                    if (c->R[i].id == c->nbuf[j]) {
                        F.n_r++;
                        break;
                    }
            }
        }
        if (o->want_live) {
            int64_t live = 0;
            float t = thr_of(r, onep);
            for (int64_t i = 0; i < c->hsize; ++i) live += (c->heap[i].d <= t);
            if (live > s.max_live) s.max_live = live;
        }
    }
    if (o->trace) { /* labels: 1 where the front of R does not change after the row's hop */
        for (int64_t i = 0; i < o->trace_rows; ++i) {
            float *row = o->trace + i * OR_TRACE_W;
            if (i < nrow) {
                row[16] = ((int64_t)o->trace_interval * (i + 1) > F.last_top) ? 1.0f : 0.0f;
            } else {
                for (int j = 0; j < OR_TRACE_W; ++j) row[j] = 0.0f;
                row[16] = -1.0f;
            }
        }
    }
    if (s.overflow) s.flags |= OR_FLAG_QUEUE_OVERFLOW;
    if (st) *st = s;
    return rsize;
}

/* ------------------------------------------------------------------------ */
/* batched search with threads (Algorithm 1 per query)                      */
/* ------------------------------------------------------------------------ */

/* Learned stop: BF16 weights, feature standardisation, thresholds (probabilities). */
typedef struct {
    const uint16_t *w;
    const float *mean, *istd;
    float tau, tau_long;
    int32_t interval, long_hops; /* long_hops 0: tau throughout */
} OrStop;

typedef struct {
    const VecView *V;
    const AdjView *G;
    const float *queries;
    int64_t qstride, nq;
    const int32_t *seeds;
    int32_t ns;
    const int64_t *ex_off;
    const int32_t *ex_ids;
    const int32_t *k_arr;
    const float *eps_arr;
    const int32_t *kind_arr;
    int32_t k, k_pool;
    float eps;
    int64_t cap_L;
    int32_t order_mode;
    const OrStop *stop;
    float stop_z, stop_z_long;
    float *trace;
    int64_t trace_rows;
    int32_t trace_interval;
    int32_t *out_ids;
    float *out_dists;
    int64_t out_stride;
    int64_t *out_stats;
    int64_t next;
    pthread_mutex_t mu;
} SearchJob;

/* sigmoid(z) >= tau  <=>  z >= log(tau / (1 - tau)) */
static float tau_logit(float tau) {
    if (tau <= 0.0f) return -INFINITY;
    if (tau >= 1.0f) return INFINITY;
    return logf(tau / (1.0f - tau));
}

static void *search_worker(void *arg) {
    SearchJob *J = (SearchJob *)arg;
    Ctx c;
    ctx_init(&c, J->V->n);
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t qi = J->next;
        J->next += 16;
        pthread_mutex_unlock(&J->mu);
        if (qi >= J->nq) break;
        int64_t qe = qi + 16 < J->nq ? qi + 16 : J->nq;
        for (; qi < qe; ++qi) {
            int32_t k = J->k_arr ? J->k_arr[qi] : J->k;
            int32_t kp = J->k_pool > k ? J->k_pool : k;
            float eps = J->eps_arr ? J->eps_arr[qi] : J->eps;
            const int32_t *ex = J->ex_off ? J->ex_ids + J->ex_off[qi] : NULL;
            int nex = J->ex_off ? (int)(J->ex_off[qi + 1] - J->ex_off[qi]) : 0;
            SearchOpts o;
            memset(&o, 0, sizeof(o));
            o.cap_L = J->cap_L;
            o.order_mode = J->order_mode;
            o.order_seed = 0x1234567ull + (uint64_t)qi;
            o.want_live = J->out_stats != NULL;
            o.k_user = k;
            o.kind = J->kind_arr ? J->kind_arr[qi] : 0;
            if (J->stop) {
                o.stop_w = J->stop->w;
                o.stop_mean = J->stop->mean;
                o.stop_istd = J->stop->istd;
                o.stop_z = J->stop_z;
                o.stop_z_long = J->stop_z_long;
                o.stop_interval = J->stop->interval;
                o.stop_long_hops = J->stop->long_hops > 0 ? J->stop->long_hops : 0x7fffffff;
            }
            if (J->trace) {
                o.trace = J->trace + qi * J->trace_rows * OR_TRACE_W;
                o.trace_rows = J->trace_rows;
                o.trace_interval = J->trace_interval;
            }
            SearchStats st;
            int64_t rs = range_search_core(&c, J->V, J->G, J->queries + qi * J->qstride,
                                           J->seeds + qi * J->ns, J->ns, ex, nex, kp, eps, &o, &st);
            if (J->trace)
                for (int64_t i = 0; i < J->trace_rows; ++i)
                    o.trace[i * OR_TRACE_W + 17] = (float)qi;
            int32_t *oi = J->out_ids + qi * J->out_stride;
            float *od = J->out_dists + qi * J->out_stride;
            for (int64_t j = 0; j < J->out_stride; ++j) {
                if (j < rs) {
                    oi[j] = c.R[j].id;
                    od[j] = c.R[j].d;
                } else {
                    oi[j] = -1;
                    od[j] = INFINITY;
                }
            }
            if (J->out_stats) {
                int64_t *o4 = J->out_stats + qi * 4;
                o4[0] = st.hops;
                o4[1] = st.evals;
                o4[2] = st.max_live;
                o4[3] = st.flags;
            }
        }
    }
    ctx_free(&c);
    return NULL;
}

/*
 * RangeSearch over a batch of queries.
 *   vec        n x m FP32 rows (row stride vs)
 *   adj        n x d int32 neighbour ids (row stride adj_stride)
 *   queries    nq x m FP32 (row stride qstride)
 *   seeds      nq x ns seed ids
 *   ex_off/ex_ids  nullable; CSR lists (nq + 1 offsets) of ids never placed in R
 *   k_arr/eps_arr/kind_arr  nullable per-query k, eps and kind (1 = exploratory)
 *   k_pool     R holds max(k, k_pool) entries (the traversal pool)
 *   stop       nullable learned stop; trace (nullable) nq x trace_rows rows of 20
 *              floats: 16 features, label, query index, hop, 0
 *   out_ids/out_dists  nq x out_stride: the first out_stride entries of R sorted by
 *              (dist,id), padded with (-1, +inf)
 *   out_stats  nullable; nq x {hops, evals, max live |S|, flags (1 overflow, 16 learned stop)}
 * Returns 0, or -1 on invalid arguments.
 */
int or_range_search(const float *vec, int64_t n, int64_t m, int64_t vs, int32_t metric,
                    const int32_t *adj, int32_t d, int64_t adj_stride, const float *queries,
                    int64_t nq, int64_t qstride, const int32_t *seeds, int32_t ns,
                    const int64_t *ex_off, const int32_t *ex_ids, const int32_t *k_arr,
                    const float *eps_arr, const int32_t *kind_arr, int32_t k, int32_t k_pool,
                    float eps, int64_t cap_L, int32_t order_mode, const OrStop *stop, float *trace,
                    int64_t trace_rows, int32_t trace_interval, int32_t *out_ids,
                    float *out_dists, int64_t out_stride, int64_t *out_stats, int32_t nthreads) {
    if (n <= 0 || m <= 0 || d <= 0 || nq < 0 || ns <= 0 || k < 1 || out_stride < 1) return -1;
    if (stop && (!stop->w || !stop->mean || !stop->istd || stop->interval < 1)) return -1;
    if (trace && (trace_rows < 1 || trace_interval < 1)) return -1;
    VecView V = {vec, n, m, vs, metric};
    AdjView G = {adj, adj_stride, NULL, d};
    SearchJob J;
    memset(&J, 0, sizeof(J));
    J.V = &V;
    J.G = &G;
    J.queries = queries;
    J.qstride = qstride;
    J.nq = nq;
    J.seeds = seeds;
    J.ns = ns;
    J.ex_off = ex_off;
    J.ex_ids = ex_ids;
    J.k_arr = k_arr;
    J.eps_arr = eps_arr;
    J.kind_arr = kind_arr;
    J.k = k;
    J.k_pool = k_pool;
    J.eps = eps;
    J.cap_L = cap_L;
    J.order_mode = order_mode;
    J.stop = stop;
    if (stop) {
        J.stop_z = tau_logit(stop->tau);
        J.stop_z_long = stop->long_hops > 0 ? tau_logit(stop->tau_long) : J.stop_z;
    }
    J.trace = trace;
    J.trace_rows = trace_rows;
    J.trace_interval = trace_interval;
    J.out_ids = out_ids;
    J.out_dists = out_dists;
    J.out_stride = out_stride;
    J.out_stats = out_stats;
    J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, search_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return 0;
}

/* FP32 rerank of a candidate pool: C32x4 distances, sorted by (dist, id), top k. */
int or_rerank(const float *vec, int64_t vs, int64_t m, int32_t metric, const float *q,
              const int32_t *pool, int32_t npool, int32_t k, int32_t *out_ids,
              float *out_dists) {
    Ent *e = (Ent *)malloc(sizeof(Ent) * (npool > 0 ? npool : 1));
    int ne = 0;
    for (int i = 0; i < npool; ++i) {
        if (pool[i] < 0) continue;
        e[ne].id = pool[i];
        e[ne].d = or_dist32(vec + (int64_t)pool[i] * vs, q, m, metric);
        ne++;
    }
    for (int i = 1; i < ne; ++i) { /* insertion sort by (dist, id) */
        Ent t = e[i];
        int j = i;
        while (j > 0 && ent_less(t, e[j - 1])) {
            e[j] = e[j - 1];
            --j;
        }
        e[j] = t;
    }
    for (int i = 0; i < k; ++i) {
        out_ids[i] = i < ne ? e[i].id : -1;
        out_dists[i] = i < ne ? e[i].d : INFINITY;
    }
    free(e);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exact kNN in FP64 (Eq. knn)                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double d;
    int32_t id;
} Ent64;

static int e64_less(Ent64 a, Ent64 b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

typedef struct {
    const float *base, *queries;
    int64_t n, m, bs, nq, qs;
    int32_t metric, k;
    const int32_t *exclude;
    int32_t *out_ids;
    double *out_d;
    int64_t next;
    pthread_mutex_t mu;
} KnnJob;

static void *knn_worker(void *arg) {
    KnnJob *J = (KnnJob *)arg;
    Ent64 *top = (Ent64 *)malloc(sizeof(Ent64) * ((size_t)J->k + 1));
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t qi = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (qi >= J->nq) break;
        const float *q = J->queries + qi * J->qs;
        int32_t ex = J->exclude ? J->exclude[qi] : -1;
        int nt = 0;
        for (int64_t v = 0; v < J->n; ++v) {
            if (v == ex) continue;
            Ent64 e = {or_dist64(J->base + v * J->bs, q, J->m, J->metric), (int32_t)v};
            if (nt == J->k && !e64_less(e, top[nt - 1])) continue;
            int j = nt < J->k ? nt++ : nt - 1;
            while (j > 0 && e64_less(e, top[j - 1])) {
                top[j] = top[j - 1];
                --j;
            }
            top[j] = e;
        }
        for (int j = 0; j < J->k; ++j) {
            J->out_ids[qi * J->k + j] = j < nt ? top[j].id : -1;
            J->out_d[qi * J->k + j] = j < nt ? top[j].d : INFINITY;
        }
    }
    free(top);
    return NULL;
}

/* Exact k nearest neighbours by (FP64 distance, id); exclude: nullable per-query id. */
int or_knn64(const float *base, int64_t n, int64_t m, int64_t bs, int32_t metric,
             const float *queries, int64_t nq, int64_t qs, int32_t k, const int32_t *exclude,
             int32_t *out_ids, double *out_d, int32_t nthreads) {
    if (n <= 0 || m <= 0 || k < 1) return -1;
    KnnJob J = {base, queries, n, m, bs, nq, qs, metric, k, exclude, out_ids, out_d, 0};
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, knn_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* graph construction (Sec. 5.2, 5.3)                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    VecView V;
    int32_t d;
    int64_t nv; /* vertices 0..nv-1 are in the graph */
    int32_t *nbr; /* n x d */
    float *w; /* n x d edge weights w(u,v) = delta(u,v) */
    int32_t *cnt; /* current degree (d except while edges are being edited) */
    Ctx ctx;
    /* undo log of Algorithm 4: first-touch snapshots of whole rows */
    int64_t *snap_v;
    int32_t *snap_nbr;
    float *snap_w;
    int32_t *snap_cnt;
    int64_t nsnap, snapcap;
    /* counters */
    int64_t n_phase2, n_opt_calls, n_opt_commit, n_opt_revert, n_case_a, n_case_b, n_searches;
    int64_t err;
    uint64_t rng;
} Graph;

Graph *or_graph_create(const float *vec, int64_t n, int64_t m, int64_t vs, int32_t metric,
                       int32_t d) {
    if (d < 4 || (d & 1) || n < d + 1) return NULL;
    Graph *g = (Graph *)calloc(1, sizeof(Graph));
    g->V = (VecView){vec, n, m, vs, metric};
    g->d = d;
    g->nv = 0;
    g->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * d);
    g->w = (float *)malloc(sizeof(float) * (size_t)n * d);
    g->cnt = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    for (int64_t i = 0; i < n * d; ++i) {
        g->nbr[i] = -1;
        g->w[i] = 0.0f;
    }
    ctx_init(&g->ctx, n);
    g->snapcap = 16;
    g->snap_v = (int64_t *)malloc(sizeof(int64_t) * g->snapcap);
    g->snap_nbr = (int32_t *)malloc(sizeof(int32_t) * g->snapcap * d);
    g->snap_w = (float *)malloc(sizeof(float) * g->snapcap * d);
    g->snap_cnt = (int32_t *)malloc(sizeof(int32_t) * g->snapcap);
    g->rng = 0x243F6A8885A308D3ull;
    return g;
}

void or_graph_free(Graph *g) {
    if (!g) return;
    free(g->nbr);
    free(g->w);
    free(g->cnt);
    ctx_free(&g->ctx);
    free(g->snap_v);
    free(g->snap_nbr);
    free(g->snap_w);
    free(g->snap_cnt);
    free(g);
}

static inline float gdist(const Graph *g, int64_t a, int64_t b) {
    return or_dist32(g->V.vec + a * g->V.vs, g->V.vec + b * g->V.vs, g->V.m, g->V.metric);
}

static int has_edge(const Graph *g, int32_t a, int32_t b) {
    const int32_t *r = g->nbr + (int64_t)a * g->d;
    for (int j = 0; j < g->cnt[a]; ++j)
        if (r[j] == b) return 1;
    return 0;
}

static float edge_w(const Graph *g, int32_t a, int32_t b) {
    const int32_t *r = g->nbr + (int64_t)a * g->d;
    for (int j = 0; j < g->cnt[a]; ++j)
        if (r[j] == b) return g->w[(int64_t)a * g->d + j];
    return NAN;
}

static void half_add(Graph *g, int32_t a, int32_t b, float wt) {
    if (g->cnt[a] >= g->d) {
        g->err = 1;
        return;
    }
    int64_t o = (int64_t)a * g->d + g->cnt[a];
    g->nbr[o] = b;
    g->w[o] = wt;
    g->cnt[a]++;
}

static void half_remove(Graph *g, int32_t a, int32_t b) {
    int32_t *r = g->nbr + (int64_t)a * g->d;
    float *w = g->w + (int64_t)a * g->d;
    int j = 0;
    while (j < g->cnt[a] && r[j] != b) ++j;
    if (j == g->cnt[a]) {
        g->err = 2;
        return;
    }
    for (; j + 1 < g->cnt[a]; ++j) { /* keep the order of the remaining entries */
        r[j] = r[j + 1];
        w[j] = w[j + 1];
    }
    g->cnt[a]--;
    r[g->cnt[a]] = -1;
    w[g->cnt[a]] = 0.0f;
}

static void add_edge(Graph *g, int32_t a, int32_t b, float wt) {
    if (a == b || has_edge(g, a, b)) {
        g->err = 3;
        return;
    }
    half_add(g, a, b, wt);
    half_add(g, b, a, wt);
}

static void remove_edge(Graph *g, int32_t a, int32_t b) {
    half_remove(g, a, b);
    half_remove(g, b, a);
}

/* Search the current graph (Algorithm 1). Results are copied into `out` (sorted). */
static int64_t graph_search(Graph *g, const int32_t *seeds, int ns, int64_t qv, int32_t k,
                            float eps, Ent *out) {
    AdjView G = {g->nbr, g->d, g->cnt, g->d};
    g->n_searches++;
    SearchOpts o;
    memset(&o, 0, sizeof(o)); /* unbounded S, row order, no features */
    int64_t rs = range_search_core(&g->ctx, &g->V, &G, g->V.vec + qv * g->V.vs, seeds, ns, NULL,
                                   0, k, eps, &o, NULL);
    memcpy(out, g->ctx.R, sizeof(Ent) * (size_t)rs);
    return rs;
}

/* K_{d+1} on vertices 0..d (Sec. 5.1: the smallest DEG_d). */
int or_graph_init(Graph *g) {
    int32_t d = g->d;
    for (int32_t a = 0; a <= d; ++a)
        for (int32_t b = a + 1; b <= d; ++b) add_edge(g, a, b, gdist(g, a, b));
    g->nv = d + 1;
    return g->err ? -1 : 0;
}

/*
 * checkMRNG (Algorithm 2) for an existing edge (v1, v2): the edge is rejected
 * if a common neighbour u has max(w(v1,u), w(v2,u)) < delta(v1,v2).
 */
int or_graph_check_mrng(Graph *g, int32_t v1, int32_t v2) {
    float dv = edge_w(g, v1, v2);
    if (isnan(dv)) dv = gdist(g, v1, v2);
    const int32_t *r1 = g->nbr + (int64_t)v1 * g->d;
    for (int j = 0; j < g->cnt[v1]; ++j) {
        int32_t u = r1[j];
        if (u == v2) continue;
        float w2u = edge_w(g, v2, u);
        if (isnan(w2u)) continue; /* not a common neighbour */
        float w1u = g->w[(int64_t)v1 * g->d + j];
        float mx = w1u > w2u ? w1u : w2u;
        if (dv > mx) return 0;
    }
    return 1;
}

/* checkMRNG for the new vertex v whose tentative neighbours are U (weights Ud). */
static int check_mrng_new(const Graph *g, const int32_t *U, const float *Ud, int nu, int32_t b,
                          float db) {
    for (int i = 0; i < nu; ++i) {
        float wbu = edge_w(g, b, U[i]);
        if (isnan(wbu)) continue; /* U[i] is not a neighbour of b */
        float mx = Ud[i] > wbu ? Ud[i] : wbu;
        if (db > mx) return 0;
    }
    return 1;
}

/* undo log */
static void snap(Graph *g, int32_t v) {
    for (int64_t i = 0; i < g->nsnap; ++i)
        if (g->snap_v[i] == v) return;
    if (g->nsnap == g->snapcap) {
        g->snapcap *= 2;
        g->snap_v = (int64_t *)realloc(g->snap_v, sizeof(int64_t) * g->snapcap);
        g->snap_nbr = (int32_t *)realloc(g->snap_nbr, sizeof(int32_t) * g->snapcap * g->d);
        g->snap_w = (float *)realloc(g->snap_w, sizeof(float) * g->snapcap * g->d);
        g->snap_cnt = (int32_t *)realloc(g->snap_cnt, sizeof(int32_t) * g->snapcap);
    }
    int64_t i = g->nsnap++;
    g->snap_v[i] = v;
    memcpy(g->snap_nbr + i * g->d, g->nbr + (int64_t)v * g->d, sizeof(int32_t) * g->d);
    memcpy(g->snap_w + i * g->d, g->w + (int64_t)v * g->d, sizeof(float) * g->d);
    g->snap_cnt[i] = g->cnt[v];
}

static void revert_all(Graph *g) {
    for (int64_t i = g->nsnap - 1; i >= 0; --i) {
        int64_t v = g->snap_v[i];
        memcpy(g->nbr + v * g->d, g->snap_nbr + i * g->d, sizeof(int32_t) * g->d);
        memcpy(g->w + v * g->d, g->snap_w + i * g->d, sizeof(float) * g->d);
        g->cnt[v] = g->snap_cnt[i];
    }
    g->nsnap = 0;
}

static int in_list(const Ent *S, int64_t ns, int32_t id) {
    for (int64_t i = 0; i < ns; ++i)
        if (S[i].id == id) return 1;
    return 0;
}

/*
 * optimizeEdge (Algorithm 4 / Sec. 5.3 steps 1-6). Readings:
 *   case (a) adds (v1,v5) and (v1,v6) and removes (v5,v6), and requires v6 not
 *     adjacent to v1 (the prose of step 4a);
 *   case (b) requires v4 != v1, v4 not adjacent to v1 and gain - delta(v1,v4) > 0,
 *     and accepts the path test if the search from {v2,v3} reaches v1 or v4;
 *   i_opt bounds the number of recorded changes, the first removal included.
 * Returns 1 if the change was committed, 0 if it was reverted, -1 if (v1,v2) is no edge.
 */
int or_graph_optimize_edge(Graph *g, int32_t v1, int32_t v2, int32_t i_opt, int32_t k_opt,
                           float eps_opt) {
    if (!has_edge(g, v1, v2)) return -1;
    g->n_opt_calls++;
    int32_t kk = k_opt;
    Ent *S = (Ent *)malloc(sizeof(Ent) * ((size_t)kk + 1));
    Ent *S4 = (Ent *)malloc(sizeof(Ent) * ((size_t)kk + 1));
    g->nsnap = 0;
    int changes = 0;
    double gain = edge_w(g, v1, v2);
    snap(g, v1);
    snap(g, v2);
    remove_edge(g, v1, v2);
    changes++;
    int32_t v3 = v1, v4 = v1;
    int result = 0;
    while (changes < i_opt) {
        /* step 2: a good new neighbour v3 of v2 whose edge (v3,v4) is given up */
        double best = gain;
        int32_t seeds[2] = {v3, v4};
        int64_t ns = graph_search(g, seeds, v3 == v4 ? 1 : 2, v2, kk, eps_opt, S);
        int32_t n3 = -1, n4 = -1;
        float d23 = 0.0f;
        for (int64_t i = 0; i < ns; ++i) {
            int32_t s = S[i].id;
            if (s == v1 || s == v2 || has_edge(g, v2, s)) continue;
            const int32_t *row = g->nbr + (int64_t)s * g->d;
            for (int j = 0; j < g->cnt[s]; ++j) {
                int32_t nb = row[j];
                if (nb == v2) continue;
                double cand = gain - (double)S[i].d + (double)g->w[(int64_t)s * g->d + j];
                if (best < cand) {
                    best = cand;
                    n3 = s;
                    n4 = nb;
                    d23 = S[i].d;
                }
            }
        }
        if (n3 < 0) break; /* no improving swap */
        gain = best;
        v3 = n3;
        v4 = n4;
        /* step 3: replace (v3,v4) by (v2,v3) */
        snap(g, v2);
        snap(g, v3);
        snap(g, v4);
        remove_edge(g, v3, v4);
        changes++;
        add_edge(g, v2, v3, d23);
        changes++;
        if (v1 == v4) {
            /* step 4a: v1 misses two edges; replace some (v5,v6) by (v1,v5),(v1,v6) */
            double bb = 0.0;
            int32_t v5 = -1, v6 = -1;
            float d15 = 0.0f, d16 = 0.0f;
            int32_t sd[2] = {v2, v3};
            int64_t n2 = graph_search(g, sd, 2, v1, kk, eps_opt, S);
            for (int64_t i = 0; i < n2; ++i) {
                int32_t s = S[i].id;
                if (s == v1 || has_edge(g, v1, s)) continue;
                const int32_t *row = g->nbr + (int64_t)s * g->d;
                for (int j = 0; j < g->cnt[s]; ++j) {
                    int32_t nb = row[j];
                    if (nb == v1 || has_edge(g, v1, nb)) continue;
                    /* squared L2 distances are >= 0: a pair that cannot beat bb is skipped
                       without computing delta(n, v1) (same outcome, fewer evaluations) */
                    if (g->V.metric == OR_L2 &&
                        !(bb < gain + (double)g->w[(int64_t)s * g->d + j] - (double)S[i].d))
                        continue;
                    float dn1 = gdist(g, nb, v1);
                    double cand = gain + (double)g->w[(int64_t)s * g->d + j] - (double)S[i].d -
                                  (double)dn1;
                    if (bb < cand) {
                        bb = cand;
                        v5 = s;
                        v6 = nb;
                        d15 = S[i].d;
                        d16 = dn1;
                    }
                }
            }
            if (bb > 0.0) {
                gain = bb;
                snap(g, v1);
                snap(g, v5);
                snap(g, v6);
                remove_edge(g, v5, v6);
                add_edge(g, v1, v5, d15);
                add_edge(g, v1, v6, d16);
                g->n_case_a++;
                result = 1;
                break;
            }
        } else if (!has_edge(g, v1, v4)) {
            /* step 4b: connect v1 and v4 if that keeps the gain positive and a path exists */
            float d14 = gdist(g, v1, v4);
            if (gain - (double)d14 > 0.0) {
                int32_t sd[2] = {v2, v3};
                int64_t n1 = graph_search(g, sd, 2, v1, kk, eps_opt, S);
                int found = in_list(S, n1, v1);
                if (!found) {
                    int64_t n4s = graph_search(g, sd, 2, v4, kk, eps_opt, S4);
                    found = in_list(S4, n4s, v4);
                }
                if (found) {
                    snap(g, v1);
                    snap(g, v4);
                    add_edge(g, v1, v4, d14);
                    g->n_case_b++;
                    result = 1;
                    break;
                }
            }
        }
        /* step 5: continue from the vertex that lost an edge */
        int32_t t = v4;
        v4 = v3;
        v3 = v2;
        v2 = t;
    }
    if (result) {
        g->n_opt_commit++;
        g->nsnap = 0;
    } else {
        g->n_opt_revert++;
        revert_all(g); /* step 6 */
    }
    free(S);
    free(S4);
    return result;
}

/*
 * Add vertex v (Sec. 5.2 steps 2-6, Algorithm 3 with scheme C and the MRNG
 * pass; the check for the new vertex uses its tentative neighbours U).
 * Then optionally optimizeEdge for the new edges whose far end was not in the
 * search result. Returns 0 on success.
 */
static int extend_apply(Graph *g, int64_t v, const Ent *S, int64_t ns, int32_t k_opt,
                        float eps_opt, int32_t i_opt, int32_t do_opt);

int or_graph_extend(Graph *g, int64_t v, int32_t k_ext, float eps_ext, int32_t k_opt,
                    float eps_opt, int32_t i_opt, int32_t do_opt) {
    if (v != g->nv) return -1;
    Ent *S = (Ent *)malloc(sizeof(Ent) * ((size_t)k_ext + 1));
    int32_t seed = 0;
    int64_t ns = graph_search(g, &seed, 1, v, k_ext, eps_ext, S);
    int rc = extend_apply(g, v, S, ns, k_opt, eps_opt, i_opt, do_opt);
    free(S);
    return rc;
}

/* The edits for vertex v (== nv) given a search result computed elsewhere
 * (ids and distances sorted by (distance, id)). */
int or_graph_extend_with(Graph *g, int64_t v, const int32_t *ids, const float *dists, int64_t ns,
                         int32_t k_opt, float eps_opt, int32_t i_opt, int32_t do_opt) {
    Ent *S = (Ent *)malloc(sizeof(Ent) * ((size_t)ns + 1));
    for (int64_t i = 0; i < ns; ++i) S[i] = (Ent){dists[i], ids[i]};
    int rc = extend_apply(g, v, S, ns, k_opt, eps_opt, i_opt, do_opt);
    free(S);
    return rc;
}

/* The edits of Sec. 5.2 steps 3-6 for vertex v (== nv), given the result S of
 * its search (sorted by (distance, id)). */
static int extend_apply(Graph *g, int64_t v, const Ent *S, int64_t ns, int32_t k_opt,
                        float eps_opt, int32_t i_opt, int32_t do_opt) {
    int32_t d = g->d;
    if (v != g->nv) return -1;
    int32_t U[512];
    float Ud[512];
    int nu = 0;
    for (int phase = 0; phase < 2 && nu < d; ++phase) {
        if (phase == 1) g->n_phase2++;
        for (int64_t i = 0; i < ns && nu < d; ++i) {
            int32_t b = S[i].id;
            int inU = 0;
            for (int j = 0; j < nu; ++j) inU |= (U[j] == b);
            if (inU) continue;
            if (phase == 0 && !check_mrng_new(g, U, Ud, nu, b, S[i].d)) continue;
            /* neighbour n of b outside U with the longest edge (ties: smallest id) */
            const int32_t *row = g->nbr + (int64_t)b * d;
            int32_t nb = -1;
            float bw = -INFINITY;
            for (int j = 0; j < g->cnt[b]; ++j) {
                int32_t c = row[j];
                int cu = 0;
                for (int t = 0; t < nu; ++t) cu |= (U[t] == c);
                if (cu) continue;
                float wt = g->w[(int64_t)b * d + j];
                if (wt > bw || (wt == bw && c < nb)) {
                    bw = wt;
                    nb = c;
                }
            }
            if (nb < 0) continue;
            remove_edge(g, b, nb);
            U[nu] = b;
            Ud[nu] = S[i].d;
            nu++;
            U[nu] = nb;
            Ud[nu] = gdist(g, nb, v);
            nu++;
        }
    }
    if (nu < d) {
        g->err = 10;
        return -2;
    }
    for (int j = 0; j < nu; ++j) add_edge(g, (int32_t)v, U[j], Ud[j]);
    g->nv = v + 1;
    if (do_opt) {
        /* new neighbours not in the search result, ascending by (delta(v,u), u) */
        Ent cand[512];
        int nc = 0;
        for (int j = 0; j < nu; ++j)
            if (!in_list(S, ns, U[j])) cand[nc++] = (Ent){Ud[j], U[j]};
        for (int i = 1; i < nc; ++i) {
            Ent t = cand[i];
            int j = i;
            while (j > 0 && ent_less(t, cand[j - 1])) {
                cand[j] = cand[j - 1];
                --j;
            }
            cand[j] = t;
        }
        for (int i = 0; i < nc; ++i)
            if (has_edge(g, (int32_t)v, cand[i].id))
                or_graph_optimize_edge(g, (int32_t)v, cand[i].id, i_opt, k_opt, eps_opt);
    }
    return g->err ? -3 : 0;
}

/* dynamicEdgeOptimization (Algorithm 5), `rounds` times with a seeded generator. */
int or_graph_refine(Graph *g, int64_t rounds, uint64_t seed, int32_t i_opt, int32_t k_opt,
                    float eps_opt) {
    g->rng = seed;
    int32_t nbuf[512];
    for (int64_t it = 0; it < rounds; ++it) {
        int32_t v1 = (int32_t)(splitmix64(&g->rng) % (uint64_t)g->nv);
        int nn = g->cnt[v1];
        memcpy(nbuf, g->nbr + (int64_t)v1 * g->d, sizeof(int32_t) * nn);
        for (int j = 0; j < nn; ++j) {
            int32_t v2 = nbuf[j];
            if (!has_edge(g, v1, v2)) continue;
            if (!or_graph_check_mrng(g, v1, v2))
                or_graph_optimize_edge(g, v1, v2, i_opt, k_opt, eps_opt);
        }
        /* the neighbour with the longest edge */
        int32_t best = -1;
        float bw = -INFINITY;
        for (int j = 0; j < g->cnt[v1]; ++j) {
            float wt = g->w[(int64_t)v1 * g->d + j];
            int32_t c = g->nbr[(int64_t)v1 * g->d + j];
            if (wt > bw || (wt == bw && c < best)) {
                bw = wt;
                best = c;
            }
        }
        if (best >= 0) or_graph_optimize_edge(g, v1, best, i_opt, k_opt, eps_opt);
        if (g->err) return -1;
    }
    return 0;
}

int64_t or_graph_nv(const Graph *g) { return g->nv; }

void or_graph_export(const Graph *g, int32_t *adj, float *w, int32_t *cnt) {
    int64_t n = g->V.n;
    if (adj) memcpy(adj, g->nbr, sizeof(int32_t) * (size_t)n * g->d);
    if (w) memcpy(w, g->w, sizeof(float) * (size_t)n * g->d);
    if (cnt) memcpy(cnt, g->cnt, sizeof(int32_t) * (size_t)n);
}

int or_graph_import(Graph *g, const int32_t *adj, const float *w, const int32_t *cnt, int64_t nv) {
    int64_t n = g->V.n;
    memcpy(g->nbr, adj, sizeof(int32_t) * (size_t)n * g->d);
    memcpy(g->w, w, sizeof(float) * (size_t)n * g->d);
    memcpy(g->cnt, cnt, sizeof(int32_t) * (size_t)n);
    g->nv = nv;
    return 0;
}

/* counters: phase-2 passes, optimizeEdge calls/commits/reverts, case a, case b, searches, err */
void or_graph_counters(const Graph *g, int64_t *out) {
    out[0] = g->n_phase2;
    out[1] = g->n_opt_calls;
    out[2] = g->n_opt_commit;
    out[3] = g->n_opt_revert;
    out[4] = g->n_case_a;
    out[5] = g->n_case_b;
    out[6] = g->n_searches;
    out[7] = g->err;
}

/* Whole build: K_{d+1}, then every vertex in id order, then `refine` rounds of Algorithm 5. */
int or_build(const float *vec, int64_t n, int64_t m, int64_t vs, int32_t metric, int32_t d,
             int32_t k_ext, float eps_ext, int32_t k_opt, float eps_opt, int32_t i_opt,
             int32_t do_opt, int64_t refine_rounds, uint64_t seed, int32_t *out_adj,
             float *out_w, int64_t *out_counters, int32_t verbose) {
    Graph *g = or_graph_create(vec, n, m, vs, metric, d);
    if (!g) return -1;
    if (or_graph_init(g)) {
        or_graph_free(g);
        return -2;
    }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t v = d + 1; v < n; ++v) {
        int rc = or_graph_extend(g, v, k_ext, eps_ext, k_opt, eps_opt, i_opt, do_opt);
        if (rc) {
            if (verbose) fprintf(stderr, "extend failed at %lld rc=%d err=%lld\n", (long long)v, rc, (long long)g->err);
            or_graph_free(g);
            return -3;
        }
        if (verbose && (v % verbose == 0)) {
            clock_gettime(CLOCK_MONOTONIC, &t1);
            double el = (t1.tv_sec - t0.tv_sec) + 1e-9 * (t1.tv_nsec - t0.tv_nsec);
            fprintf(stderr, "[or_build] %lld / %lld vertices, %.1f s, commits %lld reverts %lld\n",
                    (long long)v, (long long)n, el, (long long)g->n_opt_commit,
                    (long long)g->n_opt_revert);
            fflush(stderr);
        }
    }
    if (refine_rounds > 0 && or_graph_refine(g, refine_rounds, seed, i_opt, k_opt, eps_opt)) {
        or_graph_free(g);
        return -4;
    }
    or_graph_export(g, out_adj, out_w, NULL);
    if (out_counters) or_graph_counters(g, out_counters);
    or_graph_free(g);
    return 0;
}

/*
 * Batched construction: the paper adds one vertex at a time (Sec. 5.2), each
 * search seeing every earlier edit. Here vertices are added in blocks: the
 * searches of a block all run on the graph as it stands when the block starts
 * (its earlier vertices are not yet in it), then the block's vertices take
 * their edits (steps 3-6 and, with do_opt, optimizeEdge with its own searches
 * on the live graph) one by one in id order. A block holds at most `batch`
 * vertices and at most an eighth of the vertices already in the graph (at
 * least one), so early blocks stay small. batch = 1 is the one-at-a-time
 * build. With lag 1 a block's searches run while the previous block's edits
 * are still pending (they see neither block's vertices); the edits still go
 * in id order. This schedule is the framework's reading, not the paper's.
 */
int64_t or_build_block_size(int64_t nv, int64_t batch, int64_t left) {
    int64_t b = nv / 8;
    if (b < 1) b = 1;
    if (b > batch) b = batch;
    if (b > left) b = left;
    return b;
}

int or_build_batched(const float *vec, int64_t n, int64_t m, int64_t vs, int32_t metric,
                     int32_t d, int32_t k_ext, float eps_ext, int32_t k_opt, float eps_opt,
                     int32_t i_opt, int32_t do_opt, int64_t batch, int32_t lag,
                     int32_t *out_adj, float *out_w, int64_t *out_counters) {
    if (batch < 1 || k_ext < 1 || lag < 0 || lag > 1) return -1;
    Graph *g = or_graph_create(vec, n, m, vs, metric, d);
    if (!g) return -1;
    if (or_graph_init(g)) {
        or_graph_free(g);
        return -2;
    }
    const int64_t stride = (int64_t)k_ext + 1;
    const int64_t cap = batch < n ? batch : n;
    /* two result buffers: with lag 1 a block's results wait while the next block searches */
    Ent *res[2];
    int64_t *cnt[2];
    for (int b = 0; b < 2; ++b) {
        res[b] = (Ent *)malloc(sizeof(Ent) * (size_t)(stride * cap));
        cnt[b] = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    }
    int rc = 0;
    int64_t pend_s = 0, pend_n = 0; /* the block whose edits are still to come (lag 1) */
    int cur = 0;
    for (int64_t s = d + 1; (s < n || pend_n > 0) && rc == 0;) {
        int64_t bsz = 0;
        if (s < n) {
            /* the block's searches see the graph as it stands now: with lag 1 the
               previous block's vertices are not in it yet */
            bsz = or_build_block_size(g->nv, batch, n - s);
            for (int64_t i = 0; i < bsz; ++i) {
                int32_t seed = 0;
                cnt[cur][i] = graph_search(g, &seed, 1, s + i, k_ext, eps_ext, res[cur] + i * stride);
            }
        }
        if (lag == 1) {
            const int prv = cur ^ 1;
            for (int64_t i = 0; i < pend_n && rc == 0; ++i)
                if (extend_apply(g, pend_s + i, res[prv] + i * stride, cnt[prv][i], k_opt, eps_opt,
                                 i_opt, do_opt))
                    rc = -3;
            pend_s = s;
            pend_n = bsz;
            cur = prv;
        } else {
            for (int64_t i = 0; i < bsz && rc == 0; ++i)
                if (extend_apply(g, s + i, res[cur] + i * stride, cnt[cur][i], k_opt, eps_opt,
                                 i_opt, do_opt))
                    rc = -3;
        }
        s += bsz;
    }
    for (int b = 0; b < 2; ++b) {
        free(res[b]);
        free(cnt[b]);
    }
    if (rc == 0) {
        or_graph_export(g, out_adj, out_w, NULL);
        if (out_counters) or_graph_counters(g, out_counters);
    }
    or_graph_free(g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* graph checker (Sec. 5.1)                                                 */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Checks: ids in range, no self loops, no duplicate edges, symmetric edges,
 * connectivity (BFS from 0) and bridges (iterative low-link DFS); optionally
 * that stored weights equal the FP32 distance.
 * out[0] flags (1 bad row, 2 asymmetric, 4 disconnected, 8 bridge, 16 weight),
 * out[1] undirected edge count, out[2] vertices reached from 0, out[3] bridges,
 * out[4] in-degree min, out[5] in-degree max.
 */
int or_check_graph(const int32_t *adj, int64_t n, int32_t d, const float *w, const float *vec,
                   int64_t m, int64_t vs, int32_t metric, int64_t *out) {
    int64_t flags = 0, half = 0;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * d);
    int32_t *indeg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) {
        const int32_t *r = adj + v * d;
        for (int j = 0; j < d; ++j) {
            if (r[j] < 0 || r[j] >= n || r[j] == v) {
                flags |= 1;
                continue;
            }
            indeg[r[j]]++;
            half++;
        }
        memcpy(tmp, r, sizeof(int32_t) * d);
        qsort(tmp, d, sizeof(int32_t), cmp_i32);
        for (int j = 1; j < d; ++j)
            if (tmp[j] == tmp[j - 1]) flags |= 1;
    }
    free(tmp);
    if (flags & 1) {
        out[0] = flags;
        free(indeg);
        return (int)flags;
    }
    for (int64_t v = 0; v < n && !(flags & 2); ++v) {
        const int32_t *r = adj + v * d;
        for (int j = 0; j < d; ++j) {
            const int32_t *s = adj + (int64_t)r[j] * d;
            int ok = 0;
            for (int t = 0; t < d; ++t) ok |= (s[t] == v);
            if (!ok) {
                flags |= 2;
                break;
            }
            if (w && vec) {
                float e = or_dist32(vec + v * vs, vec + (int64_t)r[j] * vs, m, metric);
                if (w[v * d + j] != e) flags |= 16;
            }
        }
    }
    int32_t mn = d, mx = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (indeg[v] < mn) mn = indeg[v];
        if (indeg[v] > mx) mx = indeg[v];
    }
    free(indeg);
    /* BFS + bridges via iterative DFS with low-links */
    int64_t *disc = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *low = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * n);
    int32_t *it = (int32_t *)malloc(sizeof(int32_t) * n);
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t v = 0; v < n; ++v) {
        disc[v] = -1;
        it[v] = 0;
    }
    int64_t timer = 0, reached = 0, bridges = 0, sp = 0;
    disc[0] = low[0] = timer++;
    par[0] = -1;
    stk[sp++] = 0;
    reached = 1;
    while (sp > 0) {
        int64_t v = stk[sp - 1];
        if (it[v] < d) {
            int64_t u = adj[v * d + it[v]];
            it[v]++;
            if (disc[u] < 0) {
                disc[u] = low[u] = timer++;
                par[u] = v;
                stk[sp++] = u;
                reached++;
            } else if (u != par[v]) {
                if (disc[u] < low[v]) low[v] = disc[u];
            }
        } else {
            sp--;
            int64_t p = par[v];
            if (p >= 0) {
                if (low[v] < low[p]) low[p] = low[v];
                if (low[v] > disc[p]) bridges++;
            }
        }
    }
    if (reached != n) flags |= 4;
    if (bridges) flags |= 8;
    free(disc);
    free(low);
    free(par);
    free(it);
    free(stk);
    out[0] = flags;
    out[1] = half / 2;
    out[2] = reached;
    out[3] = bridges;
    out[4] = mn;
    out[5] = mx;
    return (int)flags;
}

/* ------------------------------------------------------------------------ */
/* encodings                                                                */
/* ------------------------------------------------------------------------ */

/* FP32 -> BF16 by round-to-nearest-even on the upper 16 bits. */
uint16_t or_bf16_encode(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

float or_bf16_decode(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

/*
 * OCP FP8 E4M3 ("e4m3fn"): 1 sign bit, 4 exponent bits (bias 7), 3 mantissa
 * bits; exponent field 0 is subnormal (value m * 2^-9); S.1111.111 is NaN,
 * so the largest finite magnitude is 1.75 * 2^8 = 448; there is no infinity.
 */
float or_e4m3_decode(uint8_t c) {
    int s = c >> 7, e = (c >> 3) & 15, mant = c & 7;
    if (e == 15 && mant == 7) return NAN;
    double v = e == 0 ? mant * ldexp(1.0, -9) : (1.0 + mant / 8.0) * ldexp(1.0, e - 7);
    return (float)(s ? -v : v);
}

/* Round to the nearest finite E4M3 value, ties to the even code, saturating at 448. */
uint8_t or_e4m3_encode(float x) {
    static float tab[127];
    static int init = 0;
    if (!init) {
        for (int c = 0; c < 127; ++c) tab[c] = or_e4m3_decode((uint8_t)c);
        init = 1;
    }
    uint8_t sgn = (signbit(x) ? 0x80 : 0x00);
    double a = fabs((double)x);
    if (isnan(x)) return 0x7F;
    if (a >= tab[126]) return sgn | 126;
    int lo = 0, hi = 126; /* tab[lo] <= a < tab[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (tab[mid] <= a) lo = mid; else hi = mid;
    }
    double dl = a - tab[lo], dh = tab[hi] - a;
    int c;
    if (dl < dh) c = lo;
    else if (dh < dl) c = hi;
    else c = (lo % 2 == 0) ? lo : hi;
    return sgn | (uint8_t)c;
}

/* Per-row FP8 encoding: s = max|x| / 448 (1 for an all-zero row), code = e4m3(x / s). */
void or_fp8_encode_rows(const float *x, int64_t n, int64_t m, int64_t xs, uint8_t *codes,
                        int64_t cs, float *scale) {
    for (int64_t i = 0; i < n; ++i) {
        const float *r = x + i * xs;
        float mx = 0.0f;
        for (int64_t j = 0; j < m; ++j) {
            float a = fabsf(r[j]);
            if (a > mx) mx = a;
        }
        float s = mx > 0.0f ? mx / 448.0f : 1.0f;
        scale[i] = s;
        for (int64_t j = 0; j < m; ++j) codes[i * cs + j] = or_e4m3_encode(r[j] / s);
        for (int64_t j = m; j < cs; ++j) codes[i * cs + j] = 0;
    }
}

/* Decoded FP8 rows: fl32(s * value(code)). */
void or_fp8_decode_rows(const uint8_t *codes, int64_t n, int64_t m, int64_t cs,
                        const float *scale, float *out, int64_t os) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) out[i * os + j] = scale[i] * or_e4m3_decode(codes[i * cs + j]);
}

void or_bf16_encode_array(const float *x, int64_t cnt, uint16_t *out) {
    for (int64_t i = 0; i < cnt; ++i) out[i] = or_bf16_encode(x[i]);
}

/* ------------------------------------------------------------------------ */
/* MLP reference in FP64 (16 -> 64 -> 64 -> 1, ReLU, sigmoid, mean BCE)     */
/* ------------------------------------------------------------------------ */
#define MLP_IN 16
#define MLP_H 64
/* parameter layout: W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3 */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NP (OFF_B3 + 1)

int32_t or_mlp_nparams(void) { return MLP_NP; }

/* Forward (logits) and, if grad != NULL, the gradient of the mean BCE loss. */
int or_mlp_fwd_bwd(const double *P, const float *X, const float *y, int64_t B, double *loss,
                   double *grad, double *logits) {
    if (grad) memset(grad, 0, sizeof(double) * MLP_NP);
    double L = 0.0;
    double h1[MLP_H], h2[MLP_H], g1[MLP_H], g2[MLP_H];
    for (int64_t b = 0; b < B; ++b) {
        const float *x = X + b * MLP_IN;
        for (int j = 0; j < MLP_H; ++j) {
            double s = P[OFF_B1 + j];
            for (int i = 0; i < MLP_IN; ++i) s += P[OFF_W1 + j * MLP_IN + i] * (double)x[i];
            h1[j] = s > 0.0 ? s : 0.0;
        }
        for (int j = 0; j < MLP_H; ++j) {
            double s = P[OFF_B2 + j];
            for (int i = 0; i < MLP_H; ++i) s += P[OFF_W2 + j * MLP_H + i] * h1[i];
            h2[j] = s > 0.0 ? s : 0.0;
        }
        double z = P[OFF_B3];
        for (int j = 0; j < MLP_H; ++j) z += P[OFF_W3 + j] * h2[j];
        if (logits) logits[b] = z;
        if (y) {
            double t = y[b];
            L += (z > 0 ? z : 0.0) - z * t + log1p(exp(-fabs(z)));
            if (grad) {
                double dz = (1.0 / (1.0 + exp(-z)) - t) / (double)B;
                grad[OFF_B3] += dz;
                for (int j = 0; j < MLP_H; ++j) {
                    grad[OFF_W3 + j] += dz * h2[j];
                    g2[j] = h2[j] > 0.0 ? dz * P[OFF_W3 + j] : 0.0;
                }
                for (int i = 0; i < MLP_H; ++i) g1[i] = 0.0;
                for (int j = 0; j < MLP_H; ++j) {
                    grad[OFF_B2 + j] += g2[j];
                    for (int i = 0; i < MLP_H; ++i) {
                        grad[OFF_W2 + j * MLP_H + i] += g2[j] * h1[i];
                        g1[i] += g2[j] * P[OFF_W2 + j * MLP_H + i];
                    }
                }
                for (int i = 0; i < MLP_H; ++i) {
                    if (h1[i] <= 0.0) continue;
                    grad[OFF_B1 + i] += g1[i];
                    for (int t2 = 0; t2 < MLP_IN; ++t2) grad[OFF_W1 + i * MLP_IN + t2] += g1[i] * (double)x[t2];
                }
            }
        }
    }
    if (loss) *loss = B > 0 ? L / (double)B : 0.0;
    return 0;
}

/* One Adam step (Kingma & Ba): m,v moments, step t >= 1, bias-corrected. */
void or_adam_step(double *P, const double *g, double *mo, double *ve, int64_t np, int64_t t,
                  double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        mo[i] = b1 * mo[i] + (1.0 - b1) * g[i];
        ve[i] = b2 * ve[i] + (1.0 - b2) * g[i] * g[i];
        P[i] -= lr * (mo[i] / c1) / (sqrt(ve[i] / c2) + eps);
    }
}

/* Medoid seed: the vertex nearest (FP64) to the coordinate-wise mean; IP: largest dot. */
int64_t or_medoid(const float *vec, int64_t n, int64_t m, int64_t vs, int32_t metric) {
    double *mean = (double *)calloc((size_t)m, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) mean[j] += vec[i * vs + j];
    for (int64_t j = 0; j < m; ++j) mean[j] /= (double)n;
    int64_t best = -1;
    double bd = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            if (metric == OR_L2) {
                double t = vec[i * vs + j] - mean[j];
                s += t * t;
            } else {
                s -= vec[i * vs + j] * mean[j];
            }
        }
        if (s < bd) {
            bd = s;
            best = i;
        }
    }
    free(mean);
    return best;
}
