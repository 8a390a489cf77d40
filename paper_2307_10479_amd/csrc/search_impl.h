// Kernel template of the DEG range search (Algorithm 1); instantiated per
// storage type in search_f32.hip, search_bf16.hip and search_fp8.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "deg.h"
#include "search_kernel.h"
#include "mlp_device.h"

namespace degk {

// ---------------------------------------------------------------- S (candidates)
// S is kept in three parts ordered by key: F < B < G. F, the smallest keys (up
// to 64), is sorted in registers, lane i holding F[i]: a pop reads lane 0 and
// shifts the wave by one lane. B is an unsorted LDS array (capacity bcap) of
// keys in [beta, phi); G, the farthest keys (>= phi), is an unsorted array in
// the wave's workspace region. New keys below beta are rank-merged into F (the
// overflow beyond 64 moves to B and lowers beta); the others are appended to
// B or, from phi on, to G. When B is nearly full its dead keys are dropped and
// its larger half moves to G (phi drops to the median). When F runs empty it is
// refilled with the 64 smallest live keys of B, found by an exact histogram
// select; when B runs empty it takes back the smallest live keys of G.
// Capacity L: at the end of a hop, if S holds more than L keys, the dead ones
// are dropped and, if more than L live keys remain, only the L smallest stay.
// This keeps the same live keys as evicting the largest key at every push into
// a full S: dead keys are larger than every live one and are never expanded.
struct SQueue {
    uint64_t f;        // per lane: F[lane], KEY_MAX beyond fcnt
    int fcnt;          // wave-uniform
    uint64_t beta;     // wave-uniform: every key of B and G is >= beta > every key of F
    uint64_t *B;       // LDS
    int bcnt, bcap;    // wave-uniform
    uint64_t phi;      // wave-uniform: every key of G is >= phi > every key of B
    uint64_t *G;       // workspace
    int gcnt;          // wave-uniform
    uint64_t *stage;   // LDS, 128 keys
    uint32_t *hist;    // LDS, 64 counters
};

__device__ __forceinline__ uint64_t lane_shift_down1(uint64_t v) {
    // lane i <- lane i + 1 (DPP wave_shl:1); lane 63 <- KEY_MAX
    int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, 0x130, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), 0x130, 0xF, 0xF, true);
    uint64_t r = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    return lane_id() == WAVE - 1 ? KEY_MAX : r;
}

// In-place forward compaction of an array of this wave (LDS or its workspace)
// keeping keys with distance <= thr.
__device__ __forceinline__ int b_drop_dead(uint64_t *B, int n, float thr) {
    const int lane = lane_id();
    const uint32_t othr = ord_of(thr);
    int out = 0;
    for (int base = 0; base < n; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < n ? B[i] : KEY_MAX;
        const bool keep = i < n && (uint32_t)(v >> 32) <= othr;
        const uint64_t m = ballot(keep);
        wave_sync();
        if (keep) B[out + prefix_in(m)] = v;
        out += __popcll(m);
        wave_sync();
    }
    return out;
}

// The k-th smallest (1 <= k <= n) of the n distinct keys in B (LDS or this
// wave's workspace): each round splits the current key range into 64
// power-of-two buckets, counts them with LDS atomics and keeps the bucket that
// holds rank k; at most 64 keys are finally ranked directly.
__device__ uint64_t b_kth(const uint64_t *B, int n, int k, uint64_t *stage, uint32_t *hist) {
    const int lane = lane_id();
    uint64_t mn = KEY_MAX, mx = 0;
    for (int i = lane; i < n; i += WAVE) {
        const uint64_t v = B[i];
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
    uint64_t lo = wave_min_u64(mn), hi = wave_max_u64(mx);
    int kk = k, cnt = n;
    for (;;) {
        if (cnt <= WAVE) {
            int c = 0;
            for (int base = 0; base < n; base += WAVE) {
                const int i = base + lane;
                const uint64_t v = i < n ? B[i] : KEY_MAX;
                const bool in = i < n && v >= lo && v <= hi;
                const uint64_t m = ballot(in);
                if (in) stage[c + prefix_in(m)] = v;
                c += __popcll(m);
            }
            wave_sync();
            const uint64_t mine = lane < c ? stage[lane] : KEY_MAX;
            int rank = 0;
            for (int t = 0; t < c; ++t) rank += stage[t] < mine ? 1 : 0;
            const uint64_t m = ballot(lane < c && rank == kk - 1);
            wave_sync();
            return read_lane_u64(mine, (int)__builtin_ctzll(m));
        }
        const uint64_t w0 = (hi - lo) / WAVE + 1;
        const int sh = w0 <= 1 ? 0 : 64 - __builtin_clzll(w0 - 1);
        hist[lane] = 0;
        wave_sync();
        for (int i = lane; i < n; i += WAVE) {
            const uint64_t v = B[i];
            if (v >= lo && v <= hi) atomicAdd(&hist[(uint32_t)((v - lo) >> sh)], 1u);
        }
        wave_sync();
        const int h = (int)hist[lane];
        int incl = h;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        const uint64_t m = ballot(incl >= kk);
        const int bk = (int)__builtin_ctzll(m);
        const int below = __builtin_amdgcn_readlane(incl, bk) - __builtin_amdgcn_readlane(h, bk);
        cnt = __builtin_amdgcn_readlane(h, bk);
        kk -= below;
        lo = lo + ((uint64_t)bk << sh);
        const uint64_t top = lo + ((1ull << sh) - 1ull);
        hi = top < hi ? top : hi;
        wave_sync();
    }
}

// Moves the keys of `src` (n keys) that are > T to the end of `dst` (which
// holds *dn keys) and compacts the others in place; returns how many stay.
__device__ __forceinline__ int split_above(uint64_t *src, int n, uint64_t T, uint64_t *dst, int &dn) {
    const int lane = lane_id();
    int out = 0;
    for (int base = 0; base < n; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < n ? src[i] : KEY_MAX;
        const bool stay = i < n && v <= T;
        const bool move = i < n && v > T;
        const uint64_t ms = ballot(stay), mm = ballot(move);
        wave_sync();
        if (stay) src[out + prefix_in(ms)] = v;
        if (move) dst[dn + prefix_in(mm)] = v;
        out += __popcll(ms);
        dn += __popcll(mm);
        wave_sync();
    }
    return out;
}

// Rank-sorts the c <= 64 keys in stage[0..c) into F.
__device__ __forceinline__ void f_from_stage(SQueue &S, int c) {
    const int lane = lane_id();
    const uint64_t mine = lane < c ? S.stage[lane] : KEY_MAX;
    int rank = 0;
    for (int t = 0; t < c; ++t) rank += S.stage[t] < mine ? 1 : 0;
    wave_sync();
    if (lane < c) S.stage[64 + rank] = mine;
    wave_sync();
    S.f = lane < c ? S.stage[64 + lane] : KEY_MAX;
    S.fcnt = c;
    wave_sync();
}

// B is empty: it takes back the smallest live keys of G (up to half its capacity).
__device__ __forceinline__ void b_from_g(SQueue &S, float thr) {
    S.gcnt = b_drop_dead(S.G, S.gcnt, thr);
    if (S.gcnt == 0) {
        S.phi = KEY_MAX;
        return;
    }
    const int want = S.bcap / 2;
    const uint64_t T = S.gcnt <= want ? KEY_MAX : b_kth(S.G, S.gcnt, want, S.stage, S.hist);
    // keys <= T go to B, the rest stay in G
    int moved = 0;
    const int lane = lane_id();
    int out = 0;
    for (int base = 0; base < S.gcnt; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < S.gcnt ? S.G[i] : KEY_MAX;
        const bool take = i < S.gcnt && v <= T;
        const bool stay = i < S.gcnt && v > T;
        const uint64_t mt = ballot(take), ms = ballot(stay);
        wave_sync();
        if (take) S.B[moved + prefix_in(mt)] = v;
        if (stay) S.G[out + prefix_in(ms)] = v;
        moved += __popcll(mt);
        out += __popcll(ms);
        wave_sync();
    }
    S.bcnt = moved;
    S.gcnt = out;
    S.phi = out > 0 ? T + 1ull : KEY_MAX;
}

// F is empty: move the (up to) 64 smallest live keys of B (refilled from G when
// it is empty) into F.
__device__ __forceinline__ void s_refill(SQueue &S, float thr) {
    const int lane = lane_id();
    S.bcnt = b_drop_dead(S.B, S.bcnt, thr);
    if (S.bcnt == 0 && S.gcnt > 0) b_from_g(S, thr);
    const int n = S.bcnt;
    if (n == 0) {
        S.fcnt = 0;
        S.beta = S.gcnt > 0 ? S.phi : KEY_MAX;
        return;
    }
    const uint64_t T = n <= WAVE ? KEY_MAX : b_kth(S.B, n, WAVE, S.stage, S.hist);
    int c = 0, out = 0;
    for (int base = 0; base < n; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < n ? S.B[i] : KEY_MAX;
        const bool sel = i < n && v <= T;
        const bool rest = i < n && v > T;
        const uint64_t ms = ballot(sel), mr = ballot(rest);
        wave_sync();
        if (sel) S.stage[c + prefix_in(ms)] = v;
        if (rest) S.B[out + prefix_in(mr)] = v;
        c += __popcll(ms);
        out += __popcll(mr);
        wave_sync();
    }
    S.bcnt = out;
    S.beta = out > 0 ? T + 1ull : (S.gcnt > 0 ? S.phi : KEY_MAX);
    f_from_stage(S, c);
}

// Pops the smallest key if it lies within thr; false ends the search.
__device__ __forceinline__ bool s_pop(SQueue &S, float thr, uint64_t &key) {
    if (S.fcnt == 0) {
        if (S.bcnt == 0 && S.gcnt == 0) return false;
        s_refill(S, thr);
        if (S.fcnt == 0) return false;
    }
    key = read_lane_u64(S.f, 0);
    if (key_dist(key) > thr) return false;
    S.f = lane_shift_down1(S.f);
    S.fcnt -= 1;
    return true;
}

// B keeps room for one hop (a row's keys plus F's overflow): when it is nearly
// full its dead keys are dropped and, if still needed, its larger half moves to G.
__device__ __forceinline__ void b_make_room(SQueue &S, float thr) {
    if (S.bcnt <= S.bcap - 2 * WAVE) return;
    S.bcnt = b_drop_dead(S.B, S.bcnt, thr);
    if (S.bcnt <= S.bcap / 2) return;
    const uint64_t T = b_kth(S.B, S.bcnt, S.bcnt / 2, S.stage, S.hist);
    S.bcnt = split_above(S.B, S.bcnt, T, S.G, S.gcnt);
    S.phi = T + 1ull;
}

// Adds the keys of the lanes in pm (all within the threshold thr).
__device__ __forceinline__ void s_push(SQueue &S, uint64_t ck, uint64_t pm, float thr) {
    const int lane = lane_id();
    const uint64_t sm = pm & ballot(ck < S.beta);
    const uint64_t bg = pm & ~sm;
    if (bg) {
        const uint64_t bb = bg & ballot(ck < S.phi);
        const uint64_t gg = bg & ~bb;
        if ((bb >> lane) & 1ull) S.B[S.bcnt + prefix_in(bb)] = ck;
        if ((gg >> lane) & 1ull) S.G[S.gcnt + prefix_in(gg)] = ck;
        S.bcnt += __popcll(bb);
        S.gcnt += __popcll(gg);
    }
    if (sm) {
        int shift = 0, rank = 0, posF = 0;
        for (uint64_t m = sm; m; m &= m - 1) {
            const int t = (int)__builtin_ctzll(m);
            const uint64_t kt = read_lane_u64(ck, t);
            shift += kt < S.f ? 1 : 0;
            rank += kt < ck ? 1 : 0;
            const int pf = __popcll(ballot(S.f < kt));
            if (lane == t) posF = pf;
        }
        const int tot = S.fcnt + __popcll(sm);
        if (lane < S.fcnt) S.stage[lane + shift] = S.f;
        if ((sm >> lane) & 1ull) S.stage[posF + rank] = ck;
        wave_sync();
        const int keep = tot < WAVE ? tot : WAVE;
        S.f = lane < keep ? S.stage[lane] : KEY_MAX;
        if (tot > WAVE) {
            const int sp = tot - WAVE;
            if (lane < sp) S.B[S.bcnt + lane] = S.stage[WAVE + lane];
            S.beta = read_lane_u64(S.stage[WAVE], 0);
            S.bcnt += sp;
        }
        S.fcnt = keep;
        wave_sync();
    }
    b_make_room(S, thr);
}

// Keeps the keys <= T of an array of this wave (LDS or workspace); returns the count.
__device__ __forceinline__ int keep_upto(uint64_t *A, int n, uint64_t T) {
    const int lane = lane_id();
    int out = 0;
    for (int base = 0; base < n; base += WAVE) {
        const int i = base + lane;
        const uint64_t v = i < n ? A[i] : KEY_MAX;
        const bool k2 = i < n && v <= T;
        const uint64_t m = ballot(k2);
        wave_sync();
        if (k2) A[out + prefix_in(m)] = v;
        out += __popcll(m);
        wave_sync();
    }
    return out;
}

// State after a cut of S (returned by value, see GrowOut).
struct CutOut {
    uint64_t f;
    int fcnt, bcnt, gcnt;
    bool b_cleared;  // B emptied by the cut (beta returns to KEY_MAX)
    bool dropped;    // live keys were dropped
};

// More than L keys are held: drops the dead ones, then keeps the L smallest
// live keys (F < B < G). Out of line: most hops never get here.
__device__ __forceinline__ CutOut s_cut(uint64_t f, int fcnt, uint64_t *B, int bcnt, uint64_t *G,
                                     int gcnt, uint64_t *stage, uint32_t *hist, float thr, int L) {
    const int lane = lane_id();
    CutOut o;
    o.b_cleared = false;
    o.dropped = false;
    const uint32_t othr = ord_of(thr);
    const int fl = __popcll(ballot(lane < fcnt && (uint32_t)(f >> 32) <= othr));
    f = lane < fl ? f : KEY_MAX;
    fcnt = fl;
    bcnt = b_drop_dead(B, bcnt, thr);
    gcnt = b_drop_dead(G, gcnt, thr);
    if (fcnt + bcnt + gcnt > L) {
        o.dropped = true;
        if (fcnt + bcnt < L) {
            const uint64_t T = b_kth(G, gcnt, L - fcnt - bcnt, stage, hist);
            gcnt = keep_upto(G, gcnt, T);
        } else {
            gcnt = 0;
            if (L <= fcnt) {
                f = lane < L ? f : KEY_MAX;
                fcnt = L;
                bcnt = 0;
                o.b_cleared = true;
            } else if (fcnt + bcnt > L) {
                const uint64_t T = b_kth(B, bcnt, L - fcnt, stage, hist);
                bcnt = keep_upto(B, bcnt, T);
            }
        }
    }
    o.f = f;
    o.fcnt = fcnt;
    o.bcnt = bcnt;
    o.gcnt = gcnt;
    return o;
}

// End-of-hop capacity rule. Returns true if live keys were dropped.
__device__ __forceinline__ bool s_capacity(SQueue &S, float thr, int L) {
    if (S.fcnt + S.bcnt + S.gcnt <= L) return false;
    const CutOut o = s_cut(S.f, S.fcnt, S.B, S.bcnt, S.G, S.gcnt, S.stage, S.hist, thr, L);
    S.f = o.f;
    S.fcnt = o.fcnt;
    S.bcnt = o.bcnt;
    S.gcnt = o.gcnt;
    if (S.gcnt == 0) S.phi = KEY_MAX;
    if (o.b_cleared) S.beta = KEY_MAX;
    return o.dropped;
}

// ---------------------------------------------------------------- R (results)
template <int RREG>
__device__ __forceinline__ uint64_t r_at(const uint64_t (&R)[RREG], int i) {
    uint64_t v = KEY_MAX;
#pragma unroll
    for (int r = 0; r < RREG; ++r)
        if (r == (i >> 6)) v = R[r];
    return read_lane_u64(v, i & 63);
}

// Merges the offered candidate keys (lanes set in `om`, key `ck`) into the
// sorted result list (top-kp by key). `total` counts every key ever offered;
// once it exceeds kp the radius r is the kp-th distance (Algorithm 1: r
// changes when R overflows). Returns true if an accepted key landed in the
// first `t10` positions; `nkept` gets the number of offered keys that are in
// R after the merge.
template <int RREG>
__device__ __forceinline__ bool r_merge(uint64_t (&R)[RREG], int &rcnt, int &total, bool &ovf,
                                        int kp, uint64_t ck, uint64_t om, uint64_t *mbuf, int t10,
                                        int &nkept) {
    const int lane = lane_id();
    const uint64_t rlast = ovf ? r_at<RREG>(R, kp - 1) : KEY_MAX;
    const bool offer = (om >> lane) & 1ull;
    const bool acc = offer && ck < rlast;
    uint64_t am = ballot(acc);
    const int na = __popcll(am);
    if (!ovf) {
        total += __popcll(om);
        if (total > kp) ovf = true;
    }
    nkept = 0;
    if (na == 0) return false;
    int rank_new = 0, myposR = 0;
    int cntR[RREG];
#pragma unroll
    for (int r = 0; r < RREG; ++r) cntR[r] = 0;
    for (uint64_t m = am; m; m &= m - 1) {
        const int t = (int)__builtin_ctzll(m);
        const uint64_t kt = read_lane_u64(ck, t);
        rank_new += (kt < ck) ? 1 : 0;
        int posR = 0;
#pragma unroll
        for (int r = 0; r < RREG; ++r) {
            cntR[r] += (kt < R[r]) ? 1 : 0;
            posR += __popcll(ballot(R[r] < kt));
        }
        if (lane == t) myposR = posR;
    }
#pragma unroll
    for (int r = 0; r < RREG; ++r) {
        int i = r * WAVE + lane;
        if (i < rcnt) {
            int pos = i + cntR[r];
            if (pos < kp) mbuf[pos] = R[r];
        }
    }
    const int newpos = myposR + rank_new;
    if (acc && newpos < kp) mbuf[newpos] = ck;
    const bool top = ballot(acc && newpos < t10) != 0;
    nkept = __popcll(ballot(acc && newpos < kp));
    rcnt = min(kp, rcnt + na);
    wave_sync();
#pragma unroll
    for (int r = 0; r < RREG; ++r) {
        int i = r * WAVE + lane;
        R[r] = i < rcnt ? mbuf[i] : KEY_MAX;
    }
    wave_sync();
    return top;
}

// ---------------------------------------------------------------- the kernel
// The stop variant's checkpoint needs more registers than a hop: with one or two
// result registers it is held to 128 VGPRs (four waves per SIMD; the few spills
// fall outside the hop loop), with more to 256 (two), and wide rows (QCH 12)
// are left to the compiler.
// MODE: 0 the plain search, 1 with the stop features (learned stop, trace rows),
// 2 the plain search on rows of up to 128 neighbours (two parts per hop).
template <int DT, int METRIC, int QCH, int RREG, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE == 1 ? (QCH >= 12 ? 1 : (RREG >= 4 ? 2 : 4)) : 1)))
search_kernel(SearchParams P) {
    constexpr bool FEAT = MODE == 1;
    constexpr int MAX_PARTS = MODE == 2 ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = lane_id();
    const int p = lane & 31;
    int32_t *htab = reinterpret_cast<int32_t *>(smem);
    uint64_t *Sq = reinterpret_cast<uint64_t *>(smem + 4 * (size_t)P.H);  // B, P.scap keys
    uint64_t *stg = Sq + P.scap;                                             // 128 keys
    uint64_t *mbuf = stg + 2 * WAVE;
    uint32_t *hist = reinterpret_cast<uint32_t *>(mbuf + RREG * WAVE);
    float *hbuf = reinterpret_cast<float *>(hist + WAVE);
    // candidate hand-out area of the distance batches: the staging keys, which
    // only live inside one S operation
    int32_t *xb = reinterpret_cast<int32_t *>(stg);

    Visited V;
    V.htab = htab;
    V.region = P.spill + (int64_t)blockIdx.x * P.region;
    V.gtab = V.region;
    V.H = P.H;
    V.hshift = P.hshift;
    V.Hg = P.hg0;
    V.hgshift = 32;
    V.limit = 0;
    V.roff = 0;
    V.pslot = -1;

    const int nch = (P.dim + 3) >> 2;
    const bool mask_tail = (P.dim & 3) != 0;
    const int deg = P.degree;
    const int hlimit = (3 * P.H) / 4;

    // stop model: the feature standardisation stays in registers for the whole
    // launch; the weights (10.6 KB shared by every wave, so they stay in L2) are
    // read at each checkpoint, which keeps 44 registers per lane free between
    // checkpoints (more resident waves)
    float f_mean = 0.f, f_istd = 0.f;
    if (FEAT && P.stop_w != nullptr) {
        if (lane < NFEAT) {
            f_mean = P.stop_mean[lane];
            f_istd = P.stop_istd[lane];
        }
    }

    for (;;) {
        int qi = 0;
        if (lane == 0) qi = atomicAdd(P.counter, 1);
        qi = uni(qi);
        if ((int64_t)qi >= P.nq) break;

        // ---- query descriptor
        int kind = P.mode == MODE_INDEXED ? 1 : 0;
        int k = P.k;
        float eps = P.eps;
        int64_t out_off = (int64_t)qi * P.k;
        int64_t qrow = qi;
        int32_t vtx = -1;
        int ns = P.nseeds;
        int32_t seed_l = -1;
        if (P.mode == MODE_VEC) {
            seed_l = lane < ns ? P.seeds[(int64_t)qi * ns + lane] : -1;
        } else if (P.mode == MODE_INDEXED) {
            vtx = P.qids[qi];
            ns = 1;
            seed_l = lane == 0 ? vtx : -1;
        } else {
            const deg_query_desc *D = P.descs + qi;
            kind = D->kind;
            k = D->k;
            eps = D->eps;
            out_off = D->out_offset;
            qrow = D->query_row;
            ns = 1;
            if (kind == 1) vtx = D->seed_or_vertex;
            seed_l = lane == 0 ? D->seed_or_vertex : -1;
            // a descriptor outside what the launch was sized for is skipped
            if (k < 1 || k > P.k || (kind != 0 && kind != 1) || !(eps >= 0.f) ||
                (kind == 0 && (P.queries == nullptr || qrow < 0 || qrow >= P.nqrows))) {
                if (P.out_stats != nullptr && lane == 0) {
                    int32_t *st = P.out_stats + (int64_t)qi * 4;
                    st[0] = 0;
                    st[1] = 0;
                    st[2] = DEG_FLAG_BAD_ID;
                    st[3] = 0;
                }
                if (FEAT && P.trace != nullptr)  // no row of a skipped query is a training row
                    for (int i = lane; i < P.trace_rows; i += WAVE)
                        P.trace[((int64_t)qi * P.trace_rows + i) * TRACE_W + 16] = -1.0f;
                continue;
            }
        }
        int kp = k;
        if (P.kpool > kp) kp = P.kpool;
        if (kp > RREG * WAVE) kp = RREG * WAVE;
        const bool do_rerank = P.rerank && P.f32 != nullptr;
        const float onep = __fadd_rn(1.0f, eps);
        int flags = 0;
        bool bad_query = kind == 1 && (vtx < 0 || (int64_t)vtx >= P.n);
        if (bad_query) flags |= DEG_FLAG_BAD_ID;

        // ---- query vector in registers (zero beyond dim)
        const float *qp = kind == 1 ? (bad_query ? nullptr : P.f32 + (int64_t)vtx * P.f32_stride)
                                    : P.queries + qrow * P.qstride;
        float4 qv[QCH];
#pragma unroll
        for (int c = 0; c < QCH; ++c) {
            int b = 4 * (p + 32 * c);
            float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f;
            if (qp) {
                if (b + 0 < P.dim) e0 = qp[b + 0];
                if (b + 1 < P.dim) e1 = qp[b + 1];
                if (b + 2 < P.dim) e2 = qp[b + 2];
                if (b + 3 < P.dim) e3 = qp[b + 3];
            }
            qv[c] = make_float4(e0, e1, e2, e3);
        }

        // ---- reset state
        for (int i = lane; i < P.H; i += WAVE) htab[i] = -1;
        V.count = 0;
        V.spilled = false;
        wave_sync();
        uint64_t R[RREG];
#pragma unroll
        for (int r = 0; r < RREG; ++r) R[r] = KEY_MAX;
        int rcnt = 0, total = 0;
        bool ovf = false;
        float r = __builtin_inff();
        SQueue S;
        S.f = KEY_MAX;
        S.fcnt = 0;
        S.beta = KEY_MAX;
        S.B = Sq;
        S.bcnt = 0;
        S.bcap = P.bcap;
        S.phi = KEY_MAX;
        S.G = P.gspace + (int64_t)blockIdx.x * P.gcap;
        S.gcnt = 0;
        S.stage = stg;
        S.hist = hist;
        int hops = 0, evals = 0;
        const int t10 = kp < 10 ? kp : 10;
        int last_chg = 0, last_d1 = 0, last_r = 0;
        float dseed = __builtin_inff(), rprev = __builtin_inff();
        int n_acc_s = 0, n_acc_r = 0;
        int nrow = 0;
        int to_stop = P.stop_interval, to_trace = P.trace_interval;  // hops until the next checkpoint
        // adjacency rows requested ahead: run_v is the smallest key of S after the
        // previous pop (the next pop in about nine hops of ten), nxt_v the one after
        // it (usually run_v of the next hop: its row is requested a hop early), and
        // spec_v the closest new candidate of the previous hop
        int32_t run_v = -1, run_nb = -1, spec_v = -1, spec_nb = -1, nxt_v = -1, nxt_nb = -1;
        // workspace-table slots of run_v's neighbours, read during the previous hop
        // (after its claims) for the probe of the next pop if that is run_v
        int32_t pv = -1;
        const int32_t *pv_tab = nullptr;
        int4 pa = make_int4(-1, -1, -1, -1), pb = pa;

        // ---- exclusion list of this query: its ids are checked, enter S and are
        // expanded like any other, but never enter R (tested where a candidate
        // could enter R)
        const int32_t *exl = nullptr;
        int nex = 0;
        if (!bad_query && P.ex_off != nullptr) {
            const int64_t e0 = P.ex_off[qi], e1 = P.ex_off[qi + 1];
            exl = P.ex_ids + e0;
            nex = e1 > e0 ? (int)(e1 - e0) : 0;
            if (e1 < e0) flags |= DEG_FLAG_BAD_ID;
            bool badx = false;
            for (int i = lane; i < nex; i += WAVE) {
                const int32_t id = exl[i];
                badx |= id < 0 || (int64_t)id >= P.n;
            }
            if (ballot(badx) != 0) flags |= DEG_FLAG_BAD_ID;
        }

        // ---- seeds: C <- seeds, each evaluated once, all enter S, non-excluded enter R
        if (!bad_query) {
            bool sv = lane < ns && seed_l >= 0 && (int64_t)seed_l < P.n;
            if (ballot(lane < ns && !sv) != 0) flags |= DEG_FLAG_BAD_ID;
            bool isnew = visit_insert(V, seed_l, sv);
            uint64_t nm = ballot(isnew);
            int cnt = __popcll(nm);
            V.count += cnt;
            evals += cnt;
            float cd = batch_dist<DT, METRIC, QCH>(P, qv, seed_l, nm, nch, mask_tail, xb);
            uint64_t ck = isnew ? make_key(cd, seed_l) : KEY_MAX;
            if (cnt > 0) dseed = key_dist(wave_min_u64(ck));
            int na;
            uint64_t rm = ballot(isnew && seed_l != vtx);
            if (nex > 0) rm &= ~excluded_lanes(exl, nex, seed_l, rm);
            r_merge<RREG>(R, rcnt, total, ovf, kp, ck, rm, mbuf, t10, na);
            r = ovf ? key_dist(r_at<RREG>(R, kp - 1)) : __builtin_inff();
            if (cnt > 0) s_push(S, ck, nm, thr_of(r, onep));
            if (s_capacity(S, thr_of(r, onep), P.L)) flags |= DEG_FLAG_QUEUE_OVERFLOW;
        }

        // ---- hop loop (Algorithm 1)
        for (;;) {
            // s <- argmin of S; S <- S \ {s}; stop when S is empty or s is too far away
            const float thr0 = thr_of(r, onep);
            uint64_t gmin;
            if (!s_pop(S, thr0, gmin)) break;
            const float ds = key_dist(gmin);
            hops += 1;
            // long queries set the batch's makespan: their waves get issue priority
            if (hops == 1024) __builtin_amdgcn_s_setprio(2);
            if (hops == 3072) __builtin_amdgcn_s_setprio(3);

            // learned stop / trace rows every `interval` hops
            bool want_stop = false, want_trace = false;
            if (FEAT) {
                to_stop -= 1;
                to_trace -= 1;
                want_stop = P.stop_w != nullptr && to_stop == 0;
                want_trace = P.trace != nullptr && to_trace == 0 && nrow < P.trace_rows;
                if (to_stop == 0) to_stop = P.stop_interval;
                if (to_trace == 0) to_trace = P.trace_interval;
            }
            if (want_stop || want_trace) {
                // lane i < 16 computes state feature i from the wave-uniform state:
                // sqrt of a count, a ratio (correctly rounded), or a plain value
                const int kq = min(k, rcnt);
                const float d1 = rcnt > 0 ? key_dist(r_at<RREG>(R, 0)) : 0.f;
                const uint64_t kkey = kq > 0 ? r_at<RREG>(R, kq - 1) : KEY_MAX;
                const float dk = kq > 0 ? key_dist(kkey) : 0.f;
                // entries of S before the kq-th result (F holds the smallest keys of S;
                // B is counted only when every key of F is before it)
                // (only the first 64 count: B is read while fewer are found, G only
                // when its keys can precede the k-th result and F and B hold < 64)
                int closer = __popcll(ballot(lane < S.fcnt && S.f < kkey));
                if (closer == S.fcnt && closer < WAVE && S.bcnt > 0) {
                    if (kkey >= S.beta && S.fcnt + S.bcnt >= WAVE && kkey > S.phi) {
                        closer = WAVE;  // every key of F and B precedes it
                    } else {
                        for (int base = 0; base < S.bcnt && closer < WAVE; base += WAVE) {
                            const int i = base + lane;
                            closer += __popcll(ballot(i < S.bcnt && S.B[i] < kkey));
                        }
                    }
                }
                if (closer < WAVE && S.gcnt > 0 && kkey > S.phi) {
                    for (int base = 0; base < S.gcnt && closer < WAVE; base += WAVE) {
                        const int i = base + lane;
                        closer += __popcll(ballot(i < S.gcnt && S.G[i] < kkey));
                    }
                }
                closer = closer < WAVE ? closer : WAVE;
                const bool fin_r = !__builtin_isinf(r) && !__builtin_isinf(rprev) && rprev > 0.f;
                const bool fin_s = rcnt > 0 && dseed > 0.f && !__builtin_isinf(dseed);
                const bool fin_k = kq > 0 && dk > 0.f;
                // mode: 0 plain a, 1 sqrt(a), 2 a / b (1 when the divisor is not usable)
                int ai = 0;
                ai = lane == 0 ? hops : ai;
                ai = lane == 1 ? evals : ai;
                ai = lane == 2 ? __float_as_int(d1) : ai;
                ai = lane == 3 ? __float_as_int(d1) : ai;
                ai = lane == 4 ? __float_as_int(r) : ai;
                ai = lane == 5 ? hops - last_chg : ai;
                ai = lane == 6 ? hops - last_d1 : ai;
                ai = lane == 7 ? n_acc_s : ai;
                ai = lane == 8 ? n_acc_r : ai;
                ai = lane == 9 ? closer : ai;
                ai = lane == 10 ? __float_as_int(ds) : ai;
                ai = lane == 11 ? __float_as_int(fminf(eps, 4.0f)) : ai;
                ai = lane == 12 ? k : ai;
                ai = lane == 13 ? kind : ai;
                ai = lane == 14 ? hops - last_r : ai;
                ai = lane == 15 ? 1 : ai;
                float fb = 1.0f;
                fb = lane == 2 ? dk : fb;
                fb = lane == 3 ? dseed : fb;
                fb = lane == 4 ? rprev : fb;
                fb = (lane == 7 || lane == 8) ? (float)deg : fb;
                fb = lane == 9 ? 64.0f : fb;
                fb = lane == 10 ? dk : fb;
                const uint32_t lb = 1u << (lane & 31);
                const bool lane_lo = lane < 16;
                const bool is_int = lane_lo && (0xF3E3u & lb) != 0;  // 0,1,5,6,7,8,9,12,13,14,15
                const bool is_sqrt = lane_lo && (0x5063u & lb) != 0; // 0,1,5,6,12,14
                const bool is_div = lane_lo && (0x079Cu & lb) != 0;  // 2,3,4,7,8,9,10
                const uint32_t okm = (fin_k ? 0x404u : 0u) | (fin_s ? 0x8u : 0u) | (fin_r ? 0x10u : 0u) | 0x380u;
                const float fa = is_int ? (float)ai : __int_as_float(ai);
                float fv = fa;
                // correctly rounded square root and division (the library is built
                // with -fhip-fp32-correctly-rounded-divide-sqrt)
                if (is_sqrt) fv = __builtin_sqrtf(fa);
                if (is_div) fv = (okm & lb) != 0 ? fa / fb : 1.0f;
                if (lane == 10) fv = fminf(fv, 4.0f);
                rprev = r;
                if (want_trace) {
                    float *row = P.trace + ((int64_t)qi * P.trace_rows + nrow) * TRACE_W;
                    if (lane < NFEAT) row[lane] = fv;
                    if (lane == 17) row[17] = (float)qi;
                    if (lane == 18) row[18] = (float)hops;
                    if (lane == 19) row[19] = 0.f;
                    nrow += 1;
                }
                if (want_stop) {
                    const float fs = lane < NFEAT ? __fmul_rn(__fsub_rn(fv, f_mean), f_istd) : 0.0f;
                    // the weights are read here, not held across hops
                    const float z = mlp_logit(mlp_load(P.stop_w), P.stop_w, fs, hbuf);
                    if (z >= (hops >= P.stop_long_hops ? P.stop_tau_long : P.stop_tau)) {
                        flags |= DEG_FLAG_LEARNED_STOP;
                        break;
                    }
                }
            }

            if constexpr (MAX_PARTS == 1) {
                // N <- N(G,s) \ C ; C <- C u N
                const int32_t s = key_id(gmin);
                // (uniform branches: only the row used is waited for)
                int32_t nb;
                if (s == run_v) nb = run_nb;
                else if (s == nxt_v) nb = nxt_nb;
                else if (s == spec_v) nb = spec_nb;
                else nb = lane < deg ? P.adj[(int64_t)s * P.astride + lane] : -1;
                if (lane >= deg) nb = -1;
                // the likely next pop and its row, if requested before (early: a hop ago
                // or more, so it has arrived; the row of a candidate that took the lead
                // in the previous hop was requested at its end and may still be in flight)
                const int32_t rv = S.fcnt > 0 ? key_id(read_lane_u64(S.f, 0)) : -1;
                const bool early = rv >= 0 && (rv == nxt_v || rv == run_v);
                const bool have_row = early || (rv >= 0 && rv == spec_v);
                if (rv >= 0 && rv != run_v) {
                    if (rv == nxt_v) run_nb = nxt_nb;
                    else if (rv == spec_v) run_nb = spec_nb;
                }
                run_v = rv;
                // (its lanes below the degree are read only when the next pop is run_v)
                const int32_t *pf = P.adj + ((run_v >= 0 && lane < deg) ? (int64_t)run_v * P.astride + lane : 0);
                const bool bad = lane < deg && (nb < 0 || (int64_t)nb >= P.n);
                if (bad) nb = -1;
                if (ballot(bad) != 0) flags |= DEG_FLAG_BAD_ID;
                if (!V.spilled && V.count + deg > hlimit) {
                    visit_spill(V, P);
                    flags |= DEG_FLAG_HASH_SPILL;
                } else if (V.spilled && V.count + deg > V.limit) {
                    visit_grow(V, P);
                }
                bool isnew;
                if (V.spilled && s == pv && V.gtab == pv_tab) {
                    // the first probe round was read ahead: no table round trip here
                    if (!have_row) run_nb = *pf;
                    int32_t unused = 0;
                    isnew = global_insert<false, true>(V.gtab, (uint32_t)V.Hg - 1u,
                                                       hash_slot(nb, V.hgshift), nb, nb >= 0, nullptr,
                                                       unused, pa, pb);
                } else if (have_row) {
                    isnew = visit_insert(V, nb, nb >= 0);
                } else {
                    // the next pop's row is requested inside the check, after its table reads
                    isnew = visit_insert<true>(V, nb, nb >= 0, pf, run_nb);
                }
                // read ahead the table slots of run_v's neighbours for the next hop's
                // check: issued after this hop's claims, so nothing is inserted between
                // these reads and their use; right away when run_v's row is at hand,
                // else once this hop's rows are in
                auto spec = [&]() {
                    if (V.spilled && run_v >= 0) {
                        spec_read(V, run_nb, lane < deg && run_nb >= 0 && (int64_t)run_nb < P.n, pa, pb);
                        pv = run_v;
                        pv_tab = V.gtab;
                    } else {
                        pv = -1;
                    }
                };
                if (early) spec();
                // the pop after run_v: its row is requested now, for the next hop
                const int32_t nv = S.fcnt > 1 ? key_id(read_lane_u64(S.f, 1)) : -1;
                if (nv != nxt_v) {
                    nxt_v = nv;
                    nxt_nb = (nv >= 0 && lane < deg) ? P.adj[(int64_t)nv * P.astride + lane] : -1;
                }
                const uint64_t nm = ballot(isnew);
                const int cnt = __popcll(nm);
                V.count += cnt;
                evals += cnt;
                n_acc_s = 0;
                n_acc_r = 0;
                if (cnt == 0) {
                    if (!early) spec();
                    continue;
                }
                const float cd = batch_dist<DT, METRIC, QCH>(P, qv, nb, nm, nch, mask_tail, xb);
                if (!early) spec();
                const uint64_t ck = isnew ? make_key(cd, nb) : KEY_MAX;

                // R <- top-k of R and the row (Algorithm 1: accepted if delta <= r)
                const uint64_t old_first = read_lane_u64(R[0], 0);
                int na;
                uint64_t rm = ballot(isnew && nb != vtx);
                if (nex > 0) rm &= ~excluded_lanes(exl, nex, nb, rm & ballot(cd <= r));
                const bool chg = r_merge<RREG>(R, rcnt, total, ovf, kp, ck, rm, mbuf, t10, na);
                if (chg) last_chg = hops;
                if (read_lane_u64(R[0], 0) != old_first) last_d1 = hops;
                const float r_old = r;
                r = ovf ? key_dist(r_at<RREG>(R, kp - 1)) : __builtin_inff();
                if (r != r_old) last_r = hops;

                // S <- S u {n : delta(n,q) <= r (1 + eps)}
                const float thr = thr_of(r, onep);
                const bool push = isnew && cd <= thr;
                const uint64_t pm = ballot(push);
                const int np = __popcll(pm);
                n_acc_s = np;
                n_acc_r = na;
                if (np > 0) s_push(S, ck, pm, thr);
                if (s_capacity(S, thr, P.L)) flags |= DEG_FLAG_QUEUE_OVERFLOW;
                // a new candidate that now leads S is the next pop: its row is requested
                // here (the only read left in flight at the end of a hop, so the next
                // hop's first waits need not include it otherwise)
                if (np > 0 && S.fcnt > 0) {
                    const int32_t lead = key_id(read_lane_u64(S.f, 0));
                    if (lead != run_v && lead != nxt_v && lead != spec_v) {
                        spec_v = lead;
                        spec_nb = lane < deg ? P.adj[(int64_t)lead * P.astride + lane] : -1;
                    }
                }
            } else {
                // N <- N(G,s) \ C ; C <- C u N
                const int32_t s = key_id(gmin);
                // (uniform branches: only the row used is waited for)
                int32_t nb;
                if (s == run_v) nb = run_nb;
                else if (s == nxt_v) nb = nxt_nb;
                else if (s == spec_v) nb = spec_nb;
                else nb = lane < deg ? P.adj[(int64_t)s * P.astride + lane] : -1;
                if (lane >= deg) nb = -1;
                // a row longer than a wave is expanded in two parts of up to 64
                // neighbours (a batch per part; the result does not depend on the
                // grouping, see the order independence of a row); the second part is
                // requested now
                const int nparts = (MAX_PARTS == 2 && deg > WAVE) ? 2 : 1;
                int32_t nb2 = -1;
                if (nparts == 2) nb2 = lane + WAVE < deg ? P.adj[(int64_t)s * P.astride + WAVE + lane] : -1;
                // the likely next pop and its row, if requested before (early: a hop ago
                // or more, so it has arrived; the row of a candidate that took the lead
                // in the previous hop was requested at its end and may still be in flight)
                const int32_t rv = S.fcnt > 0 ? key_id(read_lane_u64(S.f, 0)) : -1;
                const bool early = rv >= 0 && (rv == nxt_v || rv == run_v);
                const bool have_row = early || (rv >= 0 && rv == spec_v);
                if (rv >= 0 && rv != run_v) {
                    if (rv == nxt_v) run_nb = nxt_nb;
                    else if (rv == spec_v) run_nb = spec_nb;
                }
                run_v = rv;
                // (its lanes below the degree are read only when the next pop is run_v)
                const int32_t *pf = P.adj + ((run_v >= 0 && lane < deg) ? (int64_t)run_v * P.astride + lane : 0);
                // read ahead the table slots of run_v's neighbours (its first 64) for the
                // next hop's check: issued after this hop's claims, so nothing is
                // inserted between these reads and their use; right away when run_v's
                // row is at hand, else once this hop's last rows are in
                auto spec = [&]() {
                    if (V.spilled && run_v >= 0) {
                        spec_read(V, run_nb, lane < deg && run_nb >= 0 && (int64_t)run_nb < P.n, pa, pb);
                        pv = run_v;
                        pv_tab = V.gtab;
                    } else {
                        pv = -1;
                    }
                };
                n_acc_s = 0;
                n_acc_r = 0;
                bool pushed = false;
                for (int part = 0; part < nparts; ++part) {
                    const bool last = part == nparts - 1;
                    int32_t nbp = part == 0 ? nb : nb2;
                    const bool bad = nbp != -1 && (nbp < 0 || (int64_t)nbp >= P.n);
                    if (bad) nbp = -1;
                    if (ballot(bad) != 0) flags |= DEG_FLAG_BAD_ID;
                    if (!V.spilled && V.count + WAVE > hlimit) {
                        visit_spill(V, P);
                        flags |= DEG_FLAG_HASH_SPILL;
                    } else if (V.spilled && V.count + WAVE > V.limit) {
                        visit_grow(V, P);
                    }
                    bool isnew;
                    if (part == 0 && V.spilled && s == pv && V.gtab == pv_tab) {
                        // the first probe round was read ahead: no table round trip here
                        if (!have_row) run_nb = *pf;
                        int32_t unused = 0;
                        isnew = global_insert<false, true>(V.gtab, (uint32_t)V.Hg - 1u,
                                                           hash_slot(nbp, V.hgshift), nbp, nbp >= 0,
                                                           nullptr, unused, pa, pb);
                    } else if (part > 0 || have_row) {
                        isnew = visit_insert(V, nbp, nbp >= 0);
                    } else {
                        // the next pop's row is requested inside the check, after its table reads
                        isnew = visit_insert<true>(V, nbp, nbp >= 0, pf, run_nb);
                    }
                    if (last && early) spec();
                    if (part == 0) {
                        // the pop after run_v: its row is requested now, for the next hop
                        const int32_t nv = S.fcnt > 1 ? key_id(read_lane_u64(S.f, 1)) : -1;
                        if (nv != nxt_v) {
                            nxt_v = nv;
                            nxt_nb = (nv >= 0 && lane < deg) ? P.adj[(int64_t)nv * P.astride + lane] : -1;
                        }
                    }
                    const uint64_t nm = ballot(isnew);
                    const int cnt = __popcll(nm);
                    V.count += cnt;
                    evals += cnt;
                    if (cnt == 0) {
                        if (last && !early) spec();
                        continue;
                    }
                    const float cd = batch_dist<DT, METRIC, QCH>(P, qv, nbp, nm, nch, mask_tail, xb);
                    if (last && !early) spec();
                    const uint64_t ck = isnew ? make_key(cd, nbp) : KEY_MAX;

                    // R <- top-k of R and the row (Algorithm 1: accepted if delta <= r)
                    const uint64_t old_first = read_lane_u64(R[0], 0);
                    int na;
                    uint64_t rm = ballot(isnew && nbp != vtx);
                    if (nex > 0) rm &= ~excluded_lanes(exl, nex, nbp, rm & ballot(cd <= r));
                    const bool chg = r_merge<RREG>(R, rcnt, total, ovf, kp, ck, rm, mbuf, t10, na);
                    if (chg) last_chg = hops;
                    if (read_lane_u64(R[0], 0) != old_first) last_d1 = hops;
                    const float r_old = r;
                    r = ovf ? key_dist(r_at<RREG>(R, kp - 1)) : __builtin_inff();
                    if (r != r_old) last_r = hops;

                    // S <- S u {n : delta(n,q) <= r (1 + eps)}
                    const float thr = thr_of(r, onep);
                    const bool push = isnew && cd <= thr;
                    const uint64_t pm = ballot(push);
                    const int np = __popcll(pm);
                    n_acc_s += np;
                    n_acc_r += na;
                    if (np > 0) {
                        s_push(S, ck, pm, thr);
                        pushed = true;
                    }
                }
                // the capacity rule once per hop, at the end-of-row threshold (S grows only
                // by pushes)
                if (pushed && s_capacity(S, thr_of(r, onep), P.L)) flags |= DEG_FLAG_QUEUE_OVERFLOW;
                // a new candidate that now leads S is the next pop: its row is requested
                // here (the only read left in flight at the end of a hop, so the next
                // hop's first waits need not include it otherwise)
                if (pushed && S.fcnt > 0) {
                    const int32_t lead = key_id(read_lane_u64(S.f, 0));
                    if (lead != run_v && lead != nxt_v && lead != spec_v) {
                        spec_v = lead;
                        spec_nb = lane < deg ? P.adj[(int64_t)lead * P.astride + lane] : -1;
                    }
                }
            }
        }

        pool_give(V, P);  // a shared visited table goes back at the end of the query

        // ---- trace labels: 1 where the top-10 no longer changes afterwards
        if (FEAT && P.trace != nullptr) {
            for (int i = lane; i < P.trace_rows; i += WAVE) {
                float *row = P.trace + ((int64_t)qi * P.trace_rows + i) * TRACE_W;
                float lab = -1.0f;
                if (i < nrow) lab = (P.trace_interval * (i + 1) > last_chg) ? 1.0f : 0.0f;
                row[16] = lab;
            }
        }

        // ---- exact FP32 rerank of the pool
        if (do_rerank && rcnt > 0) {
            uint64_t NK[RREG];
#pragma unroll
            for (int r2 = 0; r2 < RREG; ++r2) {
                int cntr = rcnt - r2 * WAVE;
                cntr = cntr < 0 ? 0 : (cntr > WAVE ? WAVE : cntr);
                NK[r2] = KEY_MAX;
                if (cntr > 0) {
                    const uint64_t pm2 = cntr == WAVE ? ~0ull : ((1ull << cntr) - 1ull);
                    const int32_t id = lane < cntr ? key_id(R[r2]) : 0;
                    float dd = batch_dist<DT, METRIC, QCH, true>(P, qv, id, pm2, nch, mask_tail, xb);
                    NK[r2] = lane < cntr ? make_key(dd, id) : KEY_MAX;
                }
            }
#pragma unroll
            for (int r2 = 0; r2 < RREG; ++r2) mbuf[r2 * WAVE + lane] = NK[r2];
            wave_sync();
            int rank[RREG];
#pragma unroll
            for (int r2 = 0; r2 < RREG; ++r2) rank[r2] = 0;
            for (int t = 0; t < rcnt; ++t) {
                uint64_t kt = mbuf[t];
#pragma unroll
                for (int r2 = 0; r2 < RREG; ++r2) rank[r2] += (kt < NK[r2]) ? 1 : 0;
            }
#pragma unroll
            for (int r2 = 0; r2 < RREG; ++r2)
                if (r2 * WAVE + lane < rcnt) Sq[rank[r2]] = NK[r2];
            wave_sync();
#pragma unroll
            for (int r2 = 0; r2 < RREG; ++r2) {
                int i = r2 * WAVE + lane;
                R[r2] = i < rcnt ? Sq[i] : KEY_MAX;
            }
            wave_sync();
        }

        // ---- output: R sorted by (distance, id), padded with (-1, +inf)
#pragma unroll
        for (int r2 = 0; r2 < RREG; ++r2) {
            int i = r2 * WAVE + lane;
            if (i < k) {
                bool have = i < rcnt;
                P.out_ids[out_off + i] = have ? key_id(R[r2]) : -1;
                P.out_dists[out_off + i] = have ? key_dist(R[r2]) : __builtin_inff();
            }
        }
        if (hops >= 1024) __builtin_amdgcn_s_setprio(0);
        if (P.out_stats != nullptr && lane == 0) {
            int32_t *st = P.out_stats + (int64_t)qi * 4;
            st[0] = hops;
            st[1] = evals;
            st[2] = flags;
            st[3] = 0;
        }
    }
}

using KernelFn = void (*)(SearchParams);

template <int DT, int METRIC, int QCH>
static KernelFn pick_r(int rreg, int mode) {
    if (mode == 1) {
        switch (rreg) {
            case 1: return search_kernel<DT, METRIC, QCH, 1, 1>;
            case 2: return search_kernel<DT, METRIC, QCH, 2, 1>;
            case 4: return search_kernel<DT, METRIC, QCH, 4, 1>;
            default: return search_kernel<DT, METRIC, QCH, 8, 1>;
        }
    }
    if (mode == 2) {  // rows longer than a wave: k_pool <= 256 and dim <= 512
        if constexpr (QCH <= 4) {
            switch (rreg) {
                case 1: return search_kernel<DT, METRIC, QCH, 1, 2>;
                case 2: return search_kernel<DT, METRIC, QCH, 2, 2>;
                case 4: return search_kernel<DT, METRIC, QCH, 4, 2>;
                default: return nullptr;
            }
        }
        return nullptr;
    }
    switch (rreg) {
        case 1: return search_kernel<DT, METRIC, QCH, 1, 0>;
        case 2: return search_kernel<DT, METRIC, QCH, 2, 0>;
        case 4: return search_kernel<DT, METRIC, QCH, 4, 0>;
        case 8: return search_kernel<DT, METRIC, QCH, 8, 0>;
        default: return search_kernel<DT, METRIC, QCH, 16, 0>;
    }
}
template <int DT, int METRIC>
static KernelFn pick_q(int qch, int rreg, int mode) {
    switch (qch) {
        case 1: return pick_r<DT, METRIC, 1>(rreg, mode);
        case 2: return pick_r<DT, METRIC, 2>(rreg, mode);
        case 4: return pick_r<DT, METRIC, 4>(rreg, mode);
        default: return pick_r<DT, METRIC, 12>(rreg, mode);
    }
}
template <int DT>
static KernelFn pick_m(int metric, int qch, int rreg, int mode) {
    return metric == DEG_METRIC_L2 ? pick_q<DT, DEG_METRIC_L2>(qch, rreg, mode)
                                   : pick_q<DT, DEG_METRIC_IP>(qch, rreg, mode);
}

KernelFn pick_kernel_f32(int metric, int qch, int rreg, int mode);
KernelFn pick_kernel_bf16(int metric, int qch, int rreg, int mode);
KernelFn pick_kernel_fp8(int metric, int qch, int rreg, int mode);

}  // namespace degk
