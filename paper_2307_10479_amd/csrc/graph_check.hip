// MRNG conformity of every edge (Algorithm 2) and the longest edge of every
// vertex: the selection step of the dynamic edge optimisation (Algorithm 5
// optimises the edges of a vertex that fail the check, then its longest edge),
// evaluated for the whole graph at once.
//
// An edge (v1, v2) fails when a common neighbour u of v1 and v2 has both of
// its edges to them shorter than the edge itself: delta(v1, v2) >
// max(w(v1, u), w(v2, u)). The check reads the stored edge weights (the
// distances the construction computed), so it is exact: comparisons only.
//
// One wavefront per vertex v1 (a grid-stride loop over vertices): v1's row
// (ids and weights) goes to LDS; lane j takes the edge to v2 = N(v1)[j], walks
// v2's row from memory and looks each of its entries up in v1's row. Rows of
// up to 64 neighbours take one pass; longer rows (up to 128) a second one.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "deg.h"

namespace {

constexpr int WAVE = 64;
constexpr int MAXD = 128;

__global__ void __launch_bounds__(WAVE) mrng_kernel(const int32_t *adj, int64_t astride,
                                                    const float *w, int64_t wstride, int64_t n,
                                                    int d, uint8_t *ok, unsigned long long *fails,
                                                    int32_t *longest) {
    __shared__ int32_t rid[MAXD];
    __shared__ float rw[MAXD];
    const int lane = (int)threadIdx.x;
    unsigned long long nfail = 0;
    for (int64_t v1 = blockIdx.x; v1 < n; v1 += gridDim.x) {
        for (int j = lane; j < d; j += WAVE) {
            rid[j] = adj[v1 * astride + j];
            rw[j] = w[v1 * wstride + j];
        }
        __syncthreads();
        for (int j = lane; j < d; j += WAVE) {
            const int32_t v2 = rid[j];
            uint8_t res = 255;  // no edge in this slot
            if (v2 >= 0 && v2 < n) {
                const float dv = rw[j];
                bool pass = true;
                const int32_t *r2 = adj + (int64_t)v2 * astride;
                const float *w2 = w + (int64_t)v2 * wstride;
                for (int s = 0; s < d && pass; ++s) {
                    const int32_t u = r2[s];
                    if (u < 0 || u == v1) continue;
                    int t = 0;
                    while (t < d && rid[t] != u) ++t;
                    if (t == d) continue;  // not a common neighbour
                    const float w1u = rw[t], w2u = w2[s];
                    if (dv > (w1u > w2u ? w1u : w2u)) pass = false;
                }
                res = pass ? 1 : 0;
                nfail += pass ? 0 : 1;
            }
            ok[v1 * (int64_t)d + j] = res;
        }
        if (longest != nullptr && lane == 0) {
            // the slot of v1's longest edge (equal weights: the smaller neighbour id)
            int best = -1;
            for (int j = 0; j < d; ++j) {
                const int32_t u = rid[j];
                if (u < 0 || u >= n) continue;
                if (best < 0 || rw[j] > rw[best] || (rw[j] == rw[best] && u < rid[best])) best = j;
            }
            longest[v1] = best;
        }
        __syncthreads();
    }
    // one atomic per lane that saw a failing edge
    if (fails && nfail) atomicAdd(fails, nfail);
}

__global__ void zero_u64(unsigned long long *p) { *p = 0; }

}  // namespace

extern "C" deg_status deg_graph_check_mrng(const deg_graph *g, const float *weights,
                                           int64_t w_stride, uint8_t *out_ok,
                                           int64_t *out_fail_count, int32_t *out_longest,
                                           void *stream) {
    if (!g || !g->adj || !weights || !out_ok || g->n < 1 || g->degree < 1 ||
        g->degree > MAXD || g->row_stride < g->degree || w_stride < g->degree)
        return DEG_ERR_INVALID_ARG;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned long long *fails = reinterpret_cast<unsigned long long *>(out_fail_count);
    if (fails) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, st, fails);
    const int64_t blocks = g->n < 65536 ? g->n : 65536;
    hipLaunchKernelGGL(mrng_kernel, dim3((unsigned)blocks), dim3(WAVE), 0, st, g->adj,
                       (int64_t)g->row_stride, weights, w_stride, g->n, g->degree, out_ok, fails,
                       out_longest);
    return hipGetLastError() == hipSuccess ? DEG_OK : DEG_ERR_HIP;
}
