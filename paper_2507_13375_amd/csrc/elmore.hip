// Elmore RC-tree timing on the layer-assignment trees (Sec. II-C; Fig. rc and
// its d34 example), its exact reverse sweep, and the timing weights that feed
// the DP (Eq. 4, Eq. 5, Sec. III-D look-ahead).
//
// Timing runs in FP32 with compensated (float-float) sums: every downstream
// capacitance, delay, adjoint sum and path sum is a (hi, lo) pair whose error
// stays near FP32 eps^2, so deep trees keep delays within 1e-5 of FP64.
// These kernels are HBM-streaming sweeps over nodes grouped by tree height.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "la_internal.h"

namespace gapla {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int block = kBlock)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 65535 * 16 ? 65535 * 16 : g));
}

// error-free transformations (Knuth TwoSum, FMA TwoProd)
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

struct ff {
    float hi, lo;
};

__device__ __forceinline__ ff ff_add(ff a, float x)
{
    float s, e;
    two_sum(a.hi, x, s, e);
    return {s, a.lo + e};
}

__device__ __forceinline__ ff ff_add(ff a, ff b)
{
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    float h = s + e;
    return {h, e - (h - s)};
}

__device__ __forceinline__ ff ff_norm(ff a)
{
    float h = a.hi + a.lo;
    return {h, a.lo - (h - a.hi)};
}

// x * (a.hi + a.lo), compensated
__device__ __forceinline__ ff ff_mul(float x, ff a)
{
    float p = x * a.hi;
    float e = fmaf(x, a.hi, -p) + x * a.lo;
    float h = p + e;
    return {h, e - (h - p)};
}

__device__ __forceinline__ float ff_val(ff a) { return a.hi + a.lo; }

__device__ __forceinline__ int64_t rvia(const LayerTab &t, int a, int b)
{
    int32_t d = t.pv[a] - t.pv[b];
    return d < 0 ? -d : d;
}

// ---------------------------------------------------------------------------
// RC edges: before assignment, average unit R/C per direction and zero-R pin
// edges (Sec. III-B); after it, lumped via from the parent's entering layer plus
// wire, and the via down to layer 0 at each sink pin.
// ---------------------------------------------------------------------------
__global__ void k_rc(TreeDev T, LayerTab targ, const uint8_t *lay, float *R, float *C)
{
    // per-lane layer lookups read an LDS copy of the table, not the kernel arguments
    __shared__ LayerTab tab;
    {
        const int32_t *s = (const int32_t *)&targ;
        int32_t *d = (int32_t *)&tab;
        for (int i = threadIdx.x; i < (int)(sizeof(LayerTab) / 4); i += blockDim.x) d[i] = s[i];
        __syncthreads();
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < T.nodes + T.sinks;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < T.nodes) {
            const int32_t v = (int32_t)i, p = T.parent[v];
            if (p < 0) {
                R[v] = T.rdrv_k[T.net[v]];
                C[v] = 0.f;
                continue;
            }
            const int d = T.dir[v];
            const int64_t len = T.len[v];
            int64_t r, c;
            if (!lay) {
                r = (int64_t)tab.r_avg[d] * len;
                c = (int64_t)tab.c_avg[d] * len;
            } else {
                const int a = lay[v];
                const int lp = T.parent[p] < 0 ? 0 : lay[p];
                r = rvia(tab, lp, a) + (int64_t)tab.r[a] * len;
                c = (int64_t)tab.c[a] * len;
            }
            R[v] = (float)((double)r * 1e-6);
            C[v] = (float)((double)c * 1e-3);
        } else {
            const int64_t k = i - T.nodes;
            const int32_t v = T.sink_node[k];
            R[i] = lay ? (float)((double)rvia(tab, lay[v], 0) * 1e-6) : 0.f;
            C[i] = 0.f;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward: S(v) = sum over RC children of (C + S), bottom-up by height;
// t(v) = t(parent) + R_v (C_v/2 + S_v), top-down; delay at sink pins.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void elm_up(const TreeDev &T, int32_t v, const float *R, const float *C, float *S,
                                       float *Slo)
{
    ff s{0.f, 0.f};
    const int32_t k = T.sink_id[v];
    if (k >= 0) {
        s = ff_add(s, C[T.nodes + k]);
        s = ff_add(s, T.cpin_ff[v]);
    }
    for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) {
        const int32_t c = T.ch[q];
        s = ff_add(s, C[c]);
        s = ff_add(s, ff{S[c], Slo[c]});
    }
    s = ff_norm(s);
    S[v] = s.hi;
    Slo[v] = s.lo;
}

__device__ __forceinline__ void elm_down(const TreeDev &T, int32_t v, const float *R, const float *C, const float *S,
                                         const float *Slo, float *t, float *tlo, float *delay)
{
    const int32_t p = T.parent[v];
    ff up = p < 0 ? ff{0.f, 0.f} : ff{t[p], tlo[p]};
    ff load = ff_add(ff{S[v], Slo[v]}, 0.5f * C[v]);
    ff tv = ff_norm(ff_add(up, ff_mul(R[v], load)));
    t[v] = tv.hi;
    tlo[v] = tv.lo;
    const int32_t k = T.sink_id[v];
    if (k >= 0) {
        const int64_t e = T.nodes + k;
        ff pl = ff_add(ff{0.5f * C[e], 0.f}, T.cpin_ff[v]);
        delay[k] = ff_val(ff_add(tv, ff_mul(R[e], pl)));
    }
}

// ---------------------------------------------------------------------------
// Reverse sweep for g_k = dJ/d delay_k: G(v) = sum of g below v (bottom-up),
// Sig(v) = Sig(parent) + R_v G(v) (top-down), dR_v = G(v)(C_v/2 + S_v),
// dC_v = R_v G(v)/2 + Sig(parent).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_up(const TreeDev &T, int32_t v, const float *gbar, float *G, float *Glo)
{
    ff g{0.f, 0.f};
    const int32_t k = T.sink_id[v];
    if (k >= 0) g = ff_add(g, gbar[k]);
    for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) {
        const int32_t c = T.ch[q];
        g = ff_add(g, ff{G[c], Glo[c]});
    }
    g = ff_norm(g);
    G[v] = g.hi;
    Glo[v] = g.lo;
}

__device__ __forceinline__ void adj_down(const TreeDev &T, int32_t v, const float *R, const float *C, const float *S,
                                         const float *Slo, const float *G, const float *Glo, const float *gbar,
                                         float *Sig, float *Siglo, float *dR, float *dC)
{
    const int32_t p = T.parent[v];
    const ff up = p < 0 ? ff{0.f, 0.f} : ff{Sig[p], Siglo[p]};
    const ff g{G[v], Glo[v]};
    const ff sv = ff_norm(ff_add(up, ff_mul(R[v], g)));
    Sig[v] = sv.hi;
    Siglo[v] = sv.lo;
    if (dR) dR[v] = ff_val(ff_mul(ff_val(g), ff_add(ff{S[v], Slo[v]}, 0.5f * C[v])));
    if (dC) dC[v] = ff_val(ff_add(up, 0.5f * R[v] * ff_val(g)));
    const int32_t k = T.sink_id[v];
    if (k >= 0) {
        const int64_t e = T.nodes + k;
        const float gk = gbar[k];
        if (dR) dR[e] = gk * (0.5f * C[e] + T.cpin_ff[v]);
        if (dC) dC[e] = ff_val(ff_add(sv, 0.5f * R[e] * gk));
    }
}

// Eq. 5: the edge weight is the largest pin weight in the downstream subtree.
__device__ __forceinline__ void edge_w(const TreeDev &T, int32_t v, const uint16_t *pin_w, uint16_t *seg_w)
{
    uint16_t w = T.sink_id[v] >= 0 ? pin_w[T.sink_id[v]] : 0;
    for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) w = max(w, seg_w[T.ch[q]]);
    seg_w[v] = w;
}

// One launch per dense level (one thread per node), and one single-workgroup launch that
// walks the sparse levels [h0, h1) in sweep order with barriers between levels (the nodes
// of a level read what the previous level wrote).
struct Levels {
    const int32_t *nodes;   // nodes grouped by height
    const int32_t *ptr;     // [levels + 1] group starts
    int32_t h0, h1;
    bool down;              // top-down: from h1 - 1 to h0
};

template <class F>
__device__ __forceinline__ void each_node(const Levels &lv, int32_t cnt, F f)
{
    if (lv.h1 < 0) {   // one level: `nodes` points at it
        const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
        if (i < cnt) f(lv.nodes[i]);
        return;
    }
    for (int32_t q = 0; q < lv.h1 - lv.h0; ++q) {
        const int32_t h = lv.down ? lv.h1 - 1 - q : lv.h0 + q;
        for (int32_t i = lv.ptr[h] + threadIdx.x; i < lv.ptr[h + 1]; i += blockDim.x) f(lv.nodes[i]);
        __syncthreads();
    }
}

__global__ void k_elmore_up(TreeDev T, Levels lv, int32_t cnt, const float *R, const float *C, float *S, float *Slo)
{
    each_node(lv, cnt, [&](int32_t v) { elm_up(T, v, R, C, S, Slo); });
}

__global__ void k_elmore_down(TreeDev T, Levels lv, int32_t cnt, const float *R, const float *C, const float *S,
                              const float *Slo, float *t, float *tlo, float *delay)
{
    each_node(lv, cnt, [&](int32_t v) { elm_down(T, v, R, C, S, Slo, t, tlo, delay); });
}

__global__ void k_adj_up(TreeDev T, Levels lv, int32_t cnt, const float *gbar, float *G, float *Glo)
{
    each_node(lv, cnt, [&](int32_t v) { adj_up(T, v, gbar, G, Glo); });
}

__global__ void k_adj_down(TreeDev T, Levels lv, int32_t cnt, const float *R, const float *C, const float *S,
                           const float *Slo, const float *G, const float *Glo, const float *gbar, float *Sig,
                           float *Siglo, float *dR, float *dC)
{
    each_node(lv, cnt, [&](int32_t v) { adj_down(T, v, R, C, S, Slo, G, Glo, gbar, Sig, Siglo, dR, dC); });
}

__global__ void k_edge_w(TreeDev T, Levels lv, int32_t cnt, const uint16_t *pin_w, uint16_t *seg_w)
{
    each_node(lv, cnt, [&](int32_t v) { edge_w(T, v, pin_w, seg_w); });
}

// ---------------------------------------------------------------------------
// Tiles: a workgroup takes a run of whole nets (at most kETile nodes, heights below kEMaxH),
// orders its nodes by height in LDS and runs both sweeps there, level by level with
// barriers.  Each node does the same operations in the same order as the per-level kernels,
// so the results are the same bits.
// ---------------------------------------------------------------------------
constexpr int kEThreads = 256;

struct TileLevels {
    int16_t ord[kETile];        // tile-local nodes by height
    int32_t start[kEMaxH + 1];  // level h: ord[start[h], start[h + 1])
    int32_t cur[kEMaxH];
    int32_t maxh;
};

// orders the tile's nodes [n0, n0 + nn) by height; returns the highest level
__device__ __forceinline__ int32_t tile_levels(TileLevels &L, const int32_t *height, int32_t n0, int32_t nn)
{
    for (int i = threadIdx.x; i <= kEMaxH; i += blockDim.x) L.start[i] = 0;
    if (threadIdx.x == 0) L.maxh = 0;
    __syncthreads();
    for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) {
        const int32_t h = height[n0 + u];
        atomicAdd(&L.start[h + 1], 1);
        atomicMax(&L.maxh, h);
    }
    __syncthreads();
    const int32_t mh = L.maxh;
    if (threadIdx.x == 0)
        for (int32_t h = 1; h <= mh + 1; ++h) L.start[h] += L.start[h - 1];
    __syncthreads();
    for (int32_t h = threadIdx.x; h <= mh; h += blockDim.x) L.cur[h] = L.start[h];
    __syncthreads();
    for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) L.ord[atomicAdd(&L.cur[height[n0 + u]], 1)] = (int16_t)u;
    __syncthreads();
    return mh;
}

__global__ void __launch_bounds__(kEThreads) k_elmore_tiles(TreeDev T, const int32_t *tiles, int32_t ntiles,
                                                            const int32_t *height, const float *R, const float *C,
                                                            float *S, float *Slo, float *delay)
{
    __shared__ TileLevels L;
    __shared__ float sh[kETile], sl[kETile], th[kETile], tl[kETile];
    for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const int32_t n0 = tiles[2 * ti], nn = tiles[2 * ti + 1] - n0;
        const int32_t mh = tile_levels(L, height, n0, nn);
        // S(v) = sum over RC children of (C + S), bottom-up
        for (int32_t h = 0; h <= mh; ++h) {
            for (int32_t i = L.start[h] + threadIdx.x; i < L.start[h + 1]; i += blockDim.x) {
                const int32_t u = L.ord[i], v = n0 + u;
                ff x{0.f, 0.f};
                const int32_t k = T.sink_id[v];
                if (k >= 0) {
                    x = ff_add(x, C[T.nodes + k]);
                    x = ff_add(x, T.cpin_ff[v]);
                }
                for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) {
                    const int32_t c = T.ch[q], cu = c - n0;
                    x = ff_add(x, C[c]);
                    x = ff_add(x, ff{sh[cu], sl[cu]});
                }
                x = ff_norm(x);
                sh[u] = x.hi;
                sl[u] = x.lo;
            }
            __syncthreads();
        }
        for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) {
            S[n0 + u] = sh[u];
            Slo[n0 + u] = sl[u];
        }
        // t(v) = t(parent) + R_v (C_v/2 + S_v), top-down; delay at sink pins
        for (int32_t h = mh; h >= 0; --h) {
            for (int32_t i = L.start[h] + threadIdx.x; i < L.start[h + 1]; i += blockDim.x) {
                const int32_t u = L.ord[i], v = n0 + u;
                const int32_t p = T.parent[v];
                const ff up = p < 0 ? ff{0.f, 0.f} : ff{th[p - n0], tl[p - n0]};
                const ff load = ff_add(ff{sh[u], sl[u]}, 0.5f * C[v]);
                const ff tv = ff_norm(ff_add(up, ff_mul(R[v], load)));
                th[u] = tv.hi;
                tl[u] = tv.lo;
                const int32_t k = T.sink_id[v];
                if (k >= 0) {
                    const int64_t e = T.nodes + k;
                    const ff pl = ff_add(ff{0.5f * C[e], 0.f}, T.cpin_ff[v]);
                    delay[k] = ff_val(ff_add(tv, ff_mul(R[e], pl)));
                }
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(kEThreads) k_adj_tiles(TreeDev T, const int32_t *tiles, int32_t ntiles,
                                                         const int32_t *height, const float *R, const float *C,
                                                         const float *S, const float *Slo, const float *gbar, float *G,
                                                         float *Glo, float *Sig, float *Siglo, float *dR, float *dC)
{
    __shared__ TileLevels L;
    __shared__ float gh[kETile], gl[kETile], qh[kETile], ql[kETile];
    for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const int32_t n0 = tiles[2 * ti], nn = tiles[2 * ti + 1] - n0;
        const int32_t mh = tile_levels(L, height, n0, nn);
        // G(v) = sum of g below v, bottom-up
        for (int32_t h = 0; h <= mh; ++h) {
            for (int32_t i = L.start[h] + threadIdx.x; i < L.start[h + 1]; i += blockDim.x) {
                const int32_t u = L.ord[i], v = n0 + u;
                ff g{0.f, 0.f};
                const int32_t k = T.sink_id[v];
                if (k >= 0) g = ff_add(g, gbar[k]);
                for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) {
                    const int32_t cu = T.ch[q] - n0;
                    g = ff_add(g, ff{gh[cu], gl[cu]});
                }
                g = ff_norm(g);
                gh[u] = g.hi;
                gl[u] = g.lo;
            }
            __syncthreads();
        }
        // Sig(v) = Sig(parent) + R_v G(v), top-down, and the R / C gradients
        for (int32_t h = mh; h >= 0; --h) {
            for (int32_t i = L.start[h] + threadIdx.x; i < L.start[h + 1]; i += blockDim.x) {
                const int32_t u = L.ord[i], v = n0 + u;
                const int32_t p = T.parent[v];
                const ff up = p < 0 ? ff{0.f, 0.f} : ff{qh[p - n0], ql[p - n0]};
                const ff g{gh[u], gl[u]};
                const ff sv = ff_norm(ff_add(up, ff_mul(R[v], g)));
                qh[u] = sv.hi;
                ql[u] = sv.lo;
                if (dR) dR[v] = ff_val(ff_mul(ff_val(g), ff_add(ff{S[v], Slo[v]}, 0.5f * C[v])));
                if (dC) dC[v] = ff_val(ff_add(up, 0.5f * R[v] * ff_val(g)));
                const int32_t k = T.sink_id[v];
                if (k >= 0) {
                    const int64_t e = T.nodes + k;
                    const float gk = gbar[k];
                    if (dR) dR[e] = gk * (0.5f * C[e] + T.cpin_ff[v]);
                    if (dC) dC[e] = ff_val(ff_add(sv, 0.5f * R[e] * gk));
                }
            }
            __syncthreads();
        }
        for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) {
            G[n0 + u] = gh[u];
            Glo[n0 + u] = gl[u];
            Sig[n0 + u] = qh[u];
            Siglo[n0 + u] = ql[u];
        }
        __syncthreads();
    }
}

// Eq. 5 on the tiles: the largest pin weight below each segment, bottom-up in LDS
__global__ void __launch_bounds__(kEThreads) k_edge_w_tiles(TreeDev T, const int32_t *tiles, int32_t ntiles,
                                                            const int32_t *height, const uint16_t *pin_w,
                                                            uint16_t *seg_w)
{
    __shared__ TileLevels L;
    __shared__ uint16_t wl[kETile];
    for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const int32_t n0 = tiles[2 * ti], nn = tiles[2 * ti + 1] - n0;
        const int32_t mh = tile_levels(L, height, n0, nn);
        for (int32_t h = 0; h <= mh; ++h) {
            for (int32_t i = L.start[h] + threadIdx.x; i < L.start[h + 1]; i += blockDim.x) {
                const int32_t u = L.ord[i], v = n0 + u;
                uint16_t w = T.sink_id[v] >= 0 ? pin_w[T.sink_id[v]] : 0;
                for (int32_t q = T.ch_ptr[v]; q < T.ch_ptr[v + 1]; ++q) w = max(w, wl[T.ch[q] - n0]);
                wl[u] = w;
            }
            __syncthreads();
        }
        for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) seg_w[n0 + u] = wl[u];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Wavefront runs: the nets of at most kWTile nodes, a run of whole nets per one-wavefront
// workgroup.  Lane slot p = lane + 64 j holds the run's node of rank p by height, from one packed
// record read coalesced, so a level's nodes sit in as few slots as possible and a level skips the
// slots that hold none of its heights.  The child list (run-local ids) and the sweep state sit in
// LDS, and each level costs one barrier of a single wavefront.  A wavefront takes runs
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next run's records are read as the current run
// starts and its inputs (which need the records) after the current run's first sweep, so a
// run's loads are in flight during its predecessor's levels.  Per node the operations are those
// of the per-level kernels, in the same order.
// ---------------------------------------------------------------------------
constexpr int kWPer = kWTile / 64;

// One run: its descriptor and, per lane slot, its node's record, run-local id, sink id, pin load
// and one child entry of the run
struct RunIn {
    int32_t n0, nn, maxh, s0max, s1min, nq;
    uint32_t rec[kWPer];   // height | (run-local parent + 1) << 8 | first child entry << 16 | children << 24
    int32_t u[kWPer];      // run-local node id
    int32_t sk[kWPer];     // sink id, -1 if none
    float cp[kWPer];       // pin load (fF)
    uint32_t ch[kWPer];    // run-local node id of the run's child entry lane + 64 j
    __device__ int hgt(int j) const { return (int)(rec[j] & 0xffu); }
    __device__ int par(int j) const { return (int)((rec[j] >> 8) & 0xffu) - 1; }
    __device__ int c0(int j) const { return (int)((rec[j] >> 16) & 0xffu); }
    __device__ int c1(int j) const { return c0(j) + (int)(rec[j] >> 24); }
    // slot j holds a node of height h at all (the same answer in every lane)
    __device__ bool holds(int j, int32_t h) const { return j == 0 ? h <= s0max : h >= s1min; }
};

__device__ __forceinline__ void run_in(const int4 *runs, const int4 *wpos, const uint8_t *wchl, int32_t ri,
                                       RunIn &a)
{
    const int lane = threadIdx.x;
    const int4 d = runs[ri];
    a.n0 = d.x;
    a.nn = d.y & 0xff;
    a.maxh = (d.y >> 8) & 0xff;
    a.s0max = (d.y >> 16) & 0xff;
    a.s1min = (d.y >> 24) & 0xff;
    a.nq = d.w;
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
        const int32_t p = lane + 64 * j;
        a.rec[j] = 0xffu;   // height 255: in no level
        a.u[j] = 0;
        a.sk[j] = -1;
        a.cp[j] = 0.f;
        a.ch[j] = 0;
        if (p < a.nn) {
            const int4 w = wpos[a.n0 + p];
            a.rec[j] = (uint32_t)w.x;
            a.u[j] = w.y;
            a.sk[j] = w.z;
            a.cp[j] = __int_as_float(w.w);
        }
        if (p < a.nq) a.ch[j] = wchl[d.z + p];
    }
}

// the run's child list into LDS
__device__ __forceinline__ void run_children(const RunIn &a, uint8_t *chl)
{
#pragma unroll
    for (int j = 0; j < kWPer; ++j)
        if ((int32_t)threadIdx.x + 64 * j < a.nq) chl[threadIdx.x + 64 * j] = (uint8_t)a.ch[j];
}

// Inputs of the forward sweep per lane slot: the segment's R and C; at a sink pin its pin
// edge's C and R
struct FwdIn {
    float r[kWPer], c[kWPer], ce[kWPer], re[kWPer];
};

__device__ __forceinline__ void fwd_in(const TreeDev &T, const RunIn &a, const float *R, const float *C, FwdIn &f)
{
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
        f.r[j] = f.c[j] = f.ce[j] = f.re[j] = 0.f;
        if ((int32_t)threadIdx.x + 64 * j < a.nn) {
            f.r[j] = R[a.n0 + a.u[j]];
            f.c[j] = C[a.n0 + a.u[j]];
        }
        if (a.sk[j] >= 0) {
            f.ce[j] = C[T.nodes + a.sk[j]];
            f.re[j] = R[T.nodes + a.sk[j]];
        }
    }
}

__global__ void __launch_bounds__(64) k_elmore_wave(TreeDev T, const int4 *runs, const int4 *wpos,
                                                    const uint8_t *wchl, int32_t nruns, const float *R, const float *C,
                                                    float *S, float *Slo, float *delay)
{
    __shared__ float cc[kWTile], sh[kWTile], sl[kWTile], th[kWTile], tl[kWTile], dl[kWTile];
    __shared__ int32_t skl[kWTile];
    __shared__ uint8_t chl[kWTile];
    const int lane = threadIdx.x;
    int32_t ri = blockIdx.x;
    if (ri >= nruns) return;
    RunIn a;
    FwdIn f;
    run_in(runs, wpos, wchl, ri, a);
    fwd_in(T, a, R, C, f);
    for (;;) {
        const int32_t rn = ri + (int32_t)gridDim.x;
        const bool more = rn < nruns;
        RunIn an;
        FwdIn fn;
        if (more) run_in(runs, wpos, wchl, rn, an);
        run_children(a, chl);
#pragma unroll
        for (int j = 0; j < kWPer; ++j)
            if (lane + 64 * j < a.nn) {
                cc[a.u[j]] = f.c[j];
                skl[a.u[j]] = a.sk[j];
            }
        __syncthreads();
        // S(v) = sum over RC children of (C + S), bottom-up
        float xh[kWPer], xl[kWPer];
#pragma unroll
        for (int j = 0; j < kWPer; ++j) xh[j] = xl[j] = 0.f;
        for (int32_t h = 0; h <= a.maxh; ++h) {
#pragma unroll
            for (int j = 0; j < kWPer; ++j) {
                if (!a.holds(j, h) || a.hgt(j) != h) continue;
                const int32_t u = a.u[j];
                ff x{0.f, 0.f};
                if (a.sk[j] >= 0) {
                    x = ff_add(x, f.ce[j]);
                    x = ff_add(x, a.cp[j]);
                }
                for (int32_t q = a.c0(j); q < a.c1(j); ++q) {
                    const int32_t cu = chl[q];
                    x = ff_add(x, cc[cu]);
                    x = ff_add(x, ff{sh[cu], sl[cu]});
                }
                x = ff_norm(x);
                sh[u] = xh[j] = x.hi;
                sl[u] = xl[j] = x.lo;
            }
            __syncthreads();
        }
        // the next run's inputs: its records have arrived during the sweep
        if (more) fwd_in(T, an, R, C, fn);
        // results leave in node order (coalesced), from LDS
#pragma unroll
        for (int j = 0; j < kWPer; ++j) {
            const int32_t p = lane + 64 * j;
            if (p < a.nn) {
                S[a.n0 + p] = sh[p];
                Slo[a.n0 + p] = sl[p];
            }
        }
        // t(v) = t(parent) + R_v (C_v/2 + S_v), top-down; delay at sink pins
        for (int32_t h = a.maxh; h >= 0; --h) {
#pragma unroll
            for (int j = 0; j < kWPer; ++j) {
                if (!a.holds(j, h) || a.hgt(j) != h) continue;
                const int32_t u = a.u[j], p = a.par(j);
                const ff up = p < 0 ? ff{0.f, 0.f} : ff{th[p], tl[p]};
                const ff load = ff_add(ff{xh[j], xl[j]}, 0.5f * f.c[j]);
                const ff tv = ff_norm(ff_add(up, ff_mul(f.r[j], load)));
                th[u] = tv.hi;
                tl[u] = tv.lo;
                if (a.sk[j] >= 0) {
                    const ff pl = ff_add(ff{0.5f * f.ce[j], 0.f}, a.cp[j]);
                    dl[u] = ff_val(ff_add(tv, ff_mul(f.re[j], pl)));
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kWPer; ++j) {
            const int32_t p = lane + 64 * j;
            if (p < a.nn && skl[p] >= 0) delay[skl[p]] = dl[p];
        }
        if (!more) break;
        ri = rn;
        a = an;
        f = fn;
    }
}

// Adjoint-form weights (Q10 segment and pin weights, look-ahead lambda in mOhm) from the
// reverse sweep's G (a segment) and Sigma (its parent), each product and sum rounded as
// written, so every kernel that forms them gets the same bits.
__device__ __forceinline__ uint16_t adj_q10(float g_hi, float g_lo)
{
    const float q = rintf(__fmul_rn(-1024.0f, __fadd_rn(g_hi, g_lo)));
    return (uint16_t)(q < 0.f ? 0.f : (q > 1024.f ? 1024.f : q));
}

__device__ __forceinline__ int32_t adj_lambda(float sig_hi, float sig_lo)
{
    // -Sigma * 1e6 as a float-float product, then rounded
    const float sh = -sig_hi, sl = -sig_lo;
    const float ph = __fmul_rn(sh, 1e6f);
    const float pl = __fadd_rn(__fmaf_rn(sh, 1e6f, -ph), __fmul_rn(sl, 1e6f));
    const float x = rintf(__fadd_rn(ph, pl));
    return x <= 0.f ? 0 : (x >= 2147483520.f ? 2147483647 : (int32_t)x);
}

// Inputs of the reverse sweep per lane slot: the segment's R and the sink's dJ/d delay
struct AdjIn {
    float r[kWPer], gk[kWPer];
};

__device__ __forceinline__ void adj_in(const RunIn &a, const float *R, const float *gbar, AdjIn &x)
{
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
        x.r[j] = (int32_t)threadIdx.x + 64 * j < a.nn ? R[a.n0 + a.u[j]] : 0.f;
        x.gk[j] = a.sk[j] >= 0 ? gbar[a.sk[j]] : 0.f;
    }
}

// GRADS: the R / C gradients are written (la_elmore_backward); without them (the adjoint
// weights) the kernel keeps fewer registers live and runs more waves per SIMD, and, given
// seg_w, writes the weights of its nodes and sinks itself.  As in k_elmore_wave, the next run's
// inputs are read during the current run's sweeps.
template <bool GRADS>
__global__ void __launch_bounds__(64, GRADS ? 1 : 8) k_adj_wave(TreeDev T, const int4 *runs, const int4 *wpos,
                                                 const uint8_t *wchl, int32_t nruns, const float *R, const float *C,
                                                 const float *S, const float *Slo, const float *gbar, float *G,
                                                 float *Glo, float *Sig, float *Siglo, float *dR, float *dC,
                                                 uint16_t *seg_w, uint16_t *pin_w, int32_t *lam)
{
    __shared__ float gh[kWTile], gl[kWTile], qh[kWTile], ql[kWTile];
    __shared__ int32_t skl[kWTile], lml[kWTile];
    __shared__ uint16_t pwl[kWTile];
    __shared__ uint8_t chl[kWTile];
    const int lane = threadIdx.x;
    int32_t ri = blockIdx.x;
    if (ri >= nruns) return;
    RunIn a;
    AdjIn in;
    run_in(runs, wpos, wchl, ri, a);
    adj_in(a, R, gbar, in);
    for (;;) {
        const int32_t rn = ri + (int32_t)gridDim.x;
        const bool more = rn < nruns;
        RunIn an;
        AdjIn inn;
        if (more) run_in(runs, wpos, wchl, rn, an);
        run_children(a, chl);
#pragma unroll
        for (int j = 0; j < kWPer; ++j)
            if (lane + 64 * j < a.nn) skl[a.u[j]] = a.sk[j];
        __syncthreads();
        // G(v) = sum of g below v, bottom-up
        float xh[kWPer], xl[kWPer];
#pragma unroll
        for (int j = 0; j < kWPer; ++j) xh[j] = xl[j] = 0.f;
        for (int32_t h = 0; h <= a.maxh; ++h) {
#pragma unroll
            for (int j = 0; j < kWPer; ++j) {
                if (!a.holds(j, h) || a.hgt(j) != h) continue;
                const int32_t u = a.u[j];
                ff g{0.f, 0.f};
                if (a.sk[j] >= 0) g = ff_add(g, in.gk[j]);
                for (int32_t q = a.c0(j); q < a.c1(j); ++q) {
                    const int32_t cu = chl[q];
                    g = ff_add(g, ff{gh[cu], gl[cu]});
                }
                g = ff_norm(g);
                gh[u] = xh[j] = g.hi;
                gl[u] = xl[j] = g.lo;
            }
            __syncthreads();
        }
        if (more) adj_in(an, R, gbar, inn);
        // results leave in node order (coalesced), from LDS
#pragma unroll
        for (int j = 0; j < kWPer; ++j) {
            const int32_t p = lane + 64 * j;
            if (p < a.nn) {
                G[a.n0 + p] = gh[p];
                Glo[a.n0 + p] = gl[p];
            }
        }
        // Sig(v) = Sig(parent) + R_v G(v), top-down, and the R / C gradients
        for (int32_t h = a.maxh; h >= 0; --h) {
#pragma unroll
            for (int j = 0; j < kWPer; ++j) {
                if (!a.holds(j, h) || a.hgt(j) != h) continue;
                const int32_t u = a.u[j], v = a.n0 + u, p = a.par(j);
                const ff up = p < 0 ? ff{0.f, 0.f} : ff{qh[p], ql[p]};
                const ff g{xh[j], xl[j]};
                const ff sv = ff_norm(ff_add(up, ff_mul(in.r[j], g)));
                qh[u] = sv.hi;
                ql[u] = sv.lo;
                if (!GRADS && seg_w) {
                    lml[u] = p < 0 ? 0 : adj_lambda(up.hi, up.lo);
                    if (a.sk[j] >= 0) pwl[u] = adj_q10(in.gk[j], 0.f);
                }
                if (GRADS) {
                    const float cv = C[v];
                    if (dR) dR[v] = ff_val(ff_mul(ff_val(g), ff_add(ff{S[v], Slo[v]}, 0.5f * cv)));
                    if (dC) dC[v] = ff_val(ff_add(up, 0.5f * in.r[j] * ff_val(g)));
                    const int32_t k = a.sk[j];
                    if (k >= 0) {
                        const int64_t e = T.nodes + k;
                        if (dR) dR[e] = in.gk[j] * (0.5f * C[e] + T.cpin_ff[v]);
                        if (dC) dC[e] = ff_val(ff_add(sv, 0.5f * R[e] * in.gk[j]));
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kWPer; ++j) {
            const int32_t p = lane + 64 * j, v = a.n0 + p;
            if (p < a.nn) {
                Sig[v] = qh[p];
                Siglo[v] = ql[p];
                if (!GRADS && seg_w) {
                    seg_w[v] = adj_q10(gh[p], gl[p]);
                    lam[v] = lml[p];
                    if (skl[p] >= 0) pin_w[skl[p]] = pwl[p];
                }
            }
        }
        if (!more) break;
        ri = rn;
        a = an;
        in = inn;
    }
}

// Eq. 5 on the wavefront runs: the largest pin weight below each segment, bottom-up in LDS
__global__ void __launch_bounds__(64) k_edge_w_wave(TreeDev T, const int4 *runs, const int4 *wpos,
                                                    const uint8_t *wchl, int32_t nruns, const uint16_t *pin_w,
                                                    uint16_t *seg_w)
{
    __shared__ uint16_t wl[kWTile];
    __shared__ uint8_t chl[kWTile];
    const int lane = threadIdx.x;
    for (int32_t ri = blockIdx.x; ri < nruns; ri += gridDim.x) {
        RunIn a;
        run_in(runs, wpos, wchl, ri, a);
        run_children(a, chl);
        uint16_t x[kWPer];
#pragma unroll
        for (int j = 0; j < kWPer; ++j) x[j] = a.sk[j] >= 0 ? pin_w[a.sk[j]] : 0;
        __syncthreads();
        for (int32_t h = 0; h <= a.maxh; ++h) {
#pragma unroll
            for (int j = 0; j < kWPer; ++j) {
                if (!a.holds(j, h) || a.hgt(j) != h) continue;
                uint16_t m = x[j];
                for (int32_t q = a.c0(j); q < a.c1(j); ++q) m = max(m, wl[chl[q]]);
                wl[a.u[j]] = x[j] = m;
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kWPer; ++j)
            if (lane + 64 * j < a.nn) seg_w[a.n0 + a.u[j]] = x[j];
    }
}

constexpr int kTailBlock = 1024;
constexpr int32_t kTailNodes = 1024;   // levels this sparse run in the single-workgroup launch

__global__ void k_neg(const float *x, float *y, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = -x[i];
}

// ---------------------------------------------------------------------------
// Slack, WNS, pin weights (Eq. 4), batches (Alg. 1 slack bins)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f2ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord2f(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

__global__ void k_slack(TreeDev T, const float *delay, float *slack, uint32_t *wns_ord)
{
    __shared__ uint32_t smin;
    if (threadIdx.x == 0) smin = 0xffffffffu;
    __syncthreads();
    uint32_t m = 0xffffffffu;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < T.sinks; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = T.sink_node[k];
        const float s = T.budget_ps[T.net[v]] - delay[k];
        slack[k] = s;
        m = min(m, f2ord(s));
    }
    // one LDS atomic per wavefront, one device atomic per workgroup
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = min(m, (uint32_t)__shfl_down((int)m, d));
    if ((threadIdx.x & 63) == 0) atomicMin(&smin, m);
    __syncthreads();
    if (threadIdx.x == 0) atomicMin(wns_ord, smin);
}

__global__ void k_pin_weights(TreeDev T, const float *slack, const uint32_t *wns_ord, uint16_t *pin_w)
{
    const float wns = ord2f(*wns_ord);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < T.sinks; k += (int64_t)gridDim.x * blockDim.x) {
        uint16_t q = 0;
        if (wns < 0.f) {
            const float rho = slack[k] / wns;
            const float w = 1.0f / (1.0f + expf(-10.0f * (rho - 0.3f)));
            q = (uint16_t)rintf(1024.0f * w);
        }
        pin_w[k] = q;
    }
}

__global__ void k_tiers(TreeDev T, const float *slack, const uint32_t *wns_ord, uint8_t *tier)
{
    const float wns = ord2f(*wns_ord);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < T.nets; i += (int64_t)gridDim.x * blockDim.x) {
        float ns = INFINITY;
        for (int32_t k = T.net_sink_ptr[i]; k < T.net_sink_ptr[i + 1]; ++k) ns = fminf(ns, slack[k]);
        uint8_t tr = (uint8_t)(7 + (i & 3));
        if (wns < 0.f) {
            const float rho = ns / wns;
            if (rho >= 1.0f) tr = 0;
            else if (rho >= 0.99f) tr = 1;
            else if (rho >= 0.96f) tr = 2;
            else if (rho >= 0.91f) tr = 3;
            else if (rho >= 0.84f) tr = 4;
            else if (rho >= 0.75f) tr = 5;
            else if (rho >= 0.7f) tr = 6;
        }
        tier[i] = tr;
    }
}

__global__ void k_lambda_plain(TreeDev T, const uint16_t *seg_w, int32_t *lam)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes; v += (int64_t)gridDim.x * blockDim.x)
        lam[v] = T.parent[v] < 0 ? 0 : (int32_t)(((int64_t)seg_w[v] * T.rest[v]) >> 10);
}

// gbar = dJ/d delay of J = sum over violating sinks of (w/1024) * slack
__global__ void k_adj_seed(TreeDev T, const float *slack, const uint16_t *pin_w, float *gbar)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < T.sinks; k += (int64_t)gridDim.x * blockDim.x)
        gbar[k] = slack[k] < 0.f ? -(float)pin_w[k] * (1.0f / 1024.0f) : 0.f;
}

__global__ void k_adj_weights(TreeDev T, const float *G, const float *Glo, const float *Sig, const float *Siglo,
                              const float *gbar, uint16_t *seg_w, uint16_t *pin_w, int32_t *lam)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes; v += (int64_t)gridDim.x * blockDim.x) {
        seg_w[v] = adj_q10(G[v], Glo[v]);
        const int32_t p = T.parent[v];
        lam[v] = p < 0 ? 0 : adj_lambda(Sig[p], Siglo[p]);
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < T.sinks; k += (int64_t)gridDim.x * blockDim.x)
        pin_w[k] = adj_q10(gbar[k], 0.f);
}

// ---------------------------------------------------------------------------
// TNS / WNS: FP64 block partials, then one block sums them in a fixed order.
// ---------------------------------------------------------------------------
__global__ void k_tns_partial(TreeDev T, const float *delay, double *part)
{
    __shared__ double ssum[kBlock];
    __shared__ double smin[kBlock];
    double s = 0.0, m = INFINITY;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < T.sinks; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = T.sink_node[k];
        const double sl = (double)(T.budget_ps[T.net[v]] - delay[k]);
        if (sl < 0.0) s += sl;
        m = fmin(m, sl);
    }
    ssum[threadIdx.x] = s;
    smin[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ssum[0];
        part[2 * blockIdx.x + 1] = smin[0];
    }
}

__global__ void k_tns_final(const double *part, int nb, double *out)
{
    __shared__ double ssum[kBlock];
    __shared__ double smin[kBlock];
    double s = 0.0, m = INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        s += part[2 * i];
        m = fmin(m, part[2 * i + 1]);
    }
    ssum[threadIdx.x] = s;
    smin[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ssum[0];
        out[1] = smin[0];
    }
}

}  // namespace

TreeDev tree_view(const la_batch *b)
{
    TreeDev t;
    t.nets = b->nets;
    t.nodes = b->nodes;
    t.sinks = b->sinks;
    t.parent = b->parent;
    t.ch_ptr = b->ch_ptr;
    t.ch = b->ch;
    t.net = b->net;
    t.net_ptr = b->net_ptr;
    t.len = b->len;
    t.g0 = b->g0;
    t.dir = b->dir;
    t.flags = b->flags;
    t.cpin = b->cpin;
    t.cpin_ff = b->cpin_ff;
    t.sink_id = b->sink_id;
    t.sink_node = b->sink_node;
    t.net_sink_ptr = b->net_sink_ptr;
    t.rest = b->rest;
    t.budget_fs = b->budget_fs;
    t.rdrv = b->rdrv;
    t.budget_ps = b->budget_ps;
    t.rdrv_k = b->rdrv_k;
    return t;
}

// A forward sweep over the batch-owned R/C describes those arrays as they were; once they are
// rewritten the reverse sweep and the adjoint weights must not reuse that forward's state.
static void forget_forward_on_batch_rc(la_batch *b)
{
    if (b->fwd_R == b->R || b->fwd_C == b->C) b->fwd_done = b->bwd_done = false;
}

la_status launch_rc_pre(la_batch *b)
{
    LA_TIMED(b, "k_rc", b->stream,
             hipLaunchKernelGGL(k_rc, dim3(grid_for(b->nodes + b->sinks)), dim3(kBlock), 0, b->stream, tree_view(b),
                                b->tab, (const uint8_t *)nullptr, b->R, b->C));
    LA_HIP(hipGetLastError());
    b->rc_assigned = false;
    forget_forward_on_batch_rc(b);
    return LA_OK;
}

la_status launch_rc_from_layers(la_batch *b)
{
    LA_TIMED(b, "k_rc", b->stream,
             hipLaunchKernelGGL(k_rc, dim3(grid_for(b->nodes + b->sinks)), dim3(kBlock), 0, b->stream, tree_view(b),
                                b->tab, (const uint8_t *)b->cur_layer, b->R, b->C));
    LA_HIP(hipGetLastError());
    b->rc_assigned = true;
    forget_forward_on_batch_rc(b);
    return LA_OK;
}

// Nodes grouped by height: host copy of the level starts, device nodes and starts.
struct LevelList {
    const std::vector<int32_t> *lp;   // [levels + 1]
    const int32_t *nodes, *dptr;
};

// Start of the run of top levels that each hold at most kTailNodes nodes; those levels go to one
// single-workgroup launch when there are at least two of them.
static int32_t tail_start(const std::vector<int32_t> &lp)
{
    const int32_t levels = (int32_t)lp.size() - 1;
    int32_t h0 = levels;
    while (h0 > 0 && lp[h0] - lp[h0 - 1] <= kTailNodes) --h0;
    return levels - h0 >= 2 ? h0 : levels;
}

// Visits the levels bottom-up (down = false) or top-down.  `launch(lv, grid, block, cnt)` issues
// one kernel over the nodes that `lv` names.
template <class Launch>
static void sweep_levels(const LevelList &ll, bool down, Launch launch)
{
    const auto &lp = *ll.lp;
    const int32_t levels = (int32_t)lp.size() - 1;
    if (levels <= 0 || lp[levels] == 0) return;
    const int32_t h0 = tail_start(lp);
    auto dense = [&](int32_t h) {
        const int32_t cnt = lp[h + 1] - lp[h];
        if (cnt) launch(Levels{ll.nodes + lp[h], nullptr, 0, -1, false}, dim3((cnt + kBlock - 1) / kBlock),
                        dim3(kBlock), cnt);
    };
    auto tail = [&]() {
        if (h0 < levels) launch(Levels{ll.nodes, ll.dptr, h0, levels, down}, dim3(1), dim3(kTailBlock), 0);
    };
    if (!down) {
        for (int32_t h = 0; h < h0; ++h) dense(h);
        tail();
    } else {
        tail();
        for (int32_t h = h0 - 1; h >= 0; --h) dense(h);
    }
}

static LevelList untiled_levels(const la_batch *b) { return LevelList{&b->h_ebig_ptr, b->e_big_nodes, b->e_big_ptr}; }

// workgroups of the tile kernels: 8 per CU of a 256-CU part (the loop over tiles strides by it)
static int tile_grid(const la_batch *b) { return std::max(1, std::min<int>(b->e_ntiles, 2048)); }
// one-wavefront workgroups of the wavefront-run kernels: up to 32 per CU (the loop strides by it)
static int wave_grid(const la_batch *b) { return std::max(1, std::min<int>(b->e_nwtiles, 8192)); }

la_status elmore_forward(la_batch *b, const float *R, const float *C, float *delay)
{
    const TreeDev T = tree_view(b);
    // small nets in wavefront runs, the larger ones in workgroup tiles, the others level by level
    if (b->e_nwtiles > 0)
        LA_TIMED(b, "k_elmore_wave", b->stream,
                 hipLaunchKernelGGL(k_elmore_wave, dim3(wave_grid(b)), dim3(64), 0, b->stream, T,
                                    (const int4 *)b->e_wrun, (const int4 *)b->e_wpos, b->e_wchl, b->e_nwtiles, R, C, b->el_S,
                                    b->el_Slo, delay));
    if (b->e_ntiles > 0)
        LA_TIMED(b, "k_elmore_tiles", b->stream,
                 hipLaunchKernelGGL(k_elmore_tiles, dim3(tile_grid(b)), dim3(kEThreads), 0, b->stream, T, b->e_tile,
                                    b->e_ntiles, b->height, R, C, b->el_S, b->el_Slo, delay));
    const LevelList ll = untiled_levels(b);
    sweep_levels(ll, false, [&](const Levels &lv, dim3 g, dim3 t, int32_t cnt) {
        LA_TIMED(b, "k_elmore_up", b->stream,
                 hipLaunchKernelGGL(k_elmore_up, g, t, 0, b->stream, T, lv, cnt, R, C, b->el_S, b->el_Slo));
    });
    sweep_levels(ll, true, [&](const Levels &lv, dim3 g, dim3 t, int32_t cnt) {
        LA_TIMED(b, "k_elmore_down", b->stream,
                 hipLaunchKernelGGL(k_elmore_down, g, t, 0, b->stream, T, lv, cnt, R, C, b->el_S, b->el_Slo, b->el_t,
                                    b->el_tlo, delay));
    });
    LA_HIP(hipGetLastError());
    b->fwd_R = R;
    b->fwd_C = C;
    b->fwd_done = true;
    return LA_OK;
}

// gbar: dJ/d delay per sink (from_dslack: the array holds dJ/dslack and is negated first)
la_status elmore_backward(la_batch *b, const float *g, bool from_dslack, float *dR, float *dC, uint16_t *seg_w,
                          uint16_t *pin_w, int32_t *lam)
{
    if (!b->fwd_done) return set_error(LA_ERR_STATE, "la_elmore_backward needs a forward on this batch first");
    const TreeDev T = tree_view(b);
    const float *gbar = g;
    if (from_dslack) {
        LA_TIMED(b, "k_neg", b->stream,
                 hipLaunchKernelGGL(k_neg, dim3(grid_for(b->sinks)), dim3(kBlock), 0, b->stream, g, b->scratch_f,
                                    b->sinks));
        gbar = b->scratch_f;
    }
    float *Glo = b->el_Glo, *Siglo = b->el_Siglo;
    if (b->e_nwtiles > 0)
        LA_TIMED(b, "k_adj_wave", b->stream, {
            auto kern = (dR || dC) ? k_adj_wave<true> : k_adj_wave<false>;
            hipLaunchKernelGGL(kern, dim3(wave_grid(b)), dim3(64), 0, b->stream, T, (const int4 *)b->e_wrun,
                               (const int4 *)b->e_wpos, b->e_wchl, b->e_nwtiles, b->fwd_R, b->fwd_C, b->el_S, b->el_Slo, gbar, b->el_G, Glo, b->el_Sig,
                               Siglo, dR, dC, (dR || dC) ? nullptr : seg_w, pin_w, lam);
        });
    if (b->e_ntiles > 0)
        LA_TIMED(b, "k_adj_tiles", b->stream,
                 hipLaunchKernelGGL(k_adj_tiles, dim3(tile_grid(b)), dim3(kEThreads), 0, b->stream, T, b->e_tile,
                                    b->e_ntiles, b->height, b->fwd_R, b->fwd_C, b->el_S, b->el_Slo, gbar, b->el_G,
                                    Glo, b->el_Sig, Siglo, dR, dC));
    const LevelList ll = untiled_levels(b);
    sweep_levels(ll, false, [&](const Levels &lv, dim3 g, dim3 t, int32_t cnt) {
        LA_TIMED(b, "k_adj_up", b->stream,
                 hipLaunchKernelGGL(k_adj_up, g, t, 0, b->stream, T, lv, cnt, gbar, b->el_G, Glo));
    });
    sweep_levels(ll, true, [&](const Levels &lv, dim3 g, dim3 t, int32_t cnt) {
        LA_TIMED(b, "k_adj_down", b->stream,
                 hipLaunchKernelGGL(k_adj_down, g, t, 0, b->stream, T, lv, cnt, b->fwd_R, b->fwd_C, b->el_S,
                                    b->el_Slo, b->el_G, Glo, gbar, b->el_Sig, Siglo, dR, dC));
    });
    LA_HIP(hipGetLastError());
    b->bwd_done = true;
    return LA_OK;
}

la_status timing_weights(la_batch *b, const float *delay, int32_t mode, uint16_t *seg_w, uint16_t *pin_w,
                         int32_t *lam, uint8_t *tier)
{
    const TreeDev T = tree_view(b);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, b->stream, b->wns_bits, 0xffffffffu, 1);
    LA_TIMED(b, "k_slack", b->stream,
             hipLaunchKernelGGL(k_slack, dim3(std::min(grid_for(b->sinks), 2048)), dim3(kBlock), 0, b->stream, T, delay,
                                b->slack, b->wns_bits));
    LA_TIMED(b, "k_pin_weights", b->stream,
             hipLaunchKernelGGL(k_pin_weights, dim3(grid_for(b->sinks)), dim3(kBlock), 0, b->stream, T, b->slack,
                                b->wns_bits, pin_w));
    LA_TIMED(b, "k_tiers", b->stream,
             hipLaunchKernelGGL(k_tiers, dim3(grid_for(b->nets)), dim3(kBlock), 0, b->stream, T, b->slack,
                                b->wns_bits, tier));
    if (mode == LA_WEIGHTS_PLAIN) {
        if (b->e_nwtiles > 0)
            LA_TIMED(b, "k_edge_w_wave", b->stream,
                     hipLaunchKernelGGL(k_edge_w_wave, dim3(wave_grid(b)), dim3(64), 0, b->stream, T,
                                        (const int4 *)b->e_wrun, (const int4 *)b->e_wpos, b->e_wchl, b->e_nwtiles, pin_w, seg_w));
        if (b->e_ntiles > 0)
            LA_TIMED(b, "k_edge_w_tiles", b->stream,
                     hipLaunchKernelGGL(k_edge_w_tiles, dim3(tile_grid(b)), dim3(kEThreads), 0, b->stream, T,
                                        b->e_tile, b->e_ntiles, b->height, pin_w, seg_w));
        sweep_levels(untiled_levels(b), false, [&](const Levels &lv, dim3 g, dim3 t, int32_t cnt) {
            LA_TIMED(b, "k_edge_w", b->stream,
                     hipLaunchKernelGGL(k_edge_w, g, t, 0, b->stream, T, lv, cnt, pin_w, seg_w));
        });
        LA_TIMED(b, "k_lambda_plain", b->stream,
                 hipLaunchKernelGGL(k_lambda_plain, dim3(grid_for(b->nodes)), dim3(kBlock), 0, b->stream, T, seg_w,
                                    lam));
        LA_HIP(hipGetLastError());
        return LA_OK;
    }
    if (!b->fwd_done) return set_error(LA_ERR_STATE, "adjoint weights need la_elmore on this batch first");
    LA_TIMED(b, "k_adj_seed", b->stream,
             hipLaunchKernelGGL(k_adj_seed, dim3(grid_for(b->sinks)), dim3(kBlock), 0, b->stream, T, b->slack, pin_w,
                                b->scratch_f));
    la_status s = elmore_backward(b, b->scratch_f, false, nullptr, nullptr, seg_w, pin_w, lam);
    if (s != LA_OK) return s;
    // the wavefront runs wrote their nets' weights; the other nets' (workgroup tiles, per-level
    // walks) from the stored G and Sigma -- over every node, the runs' ones with the same bits
    const bool others = b->e_ntiles > 0 || (!b->h_ebig_ptr.empty() && b->h_ebig_ptr.back() > 0);
    if (others || b->e_nwtiles == 0)
        LA_TIMED(b, "k_adj_weights", b->stream,
             hipLaunchKernelGGL(k_adj_weights, dim3(grid_for(b->nodes)), dim3(kBlock), 0, b->stream, T, b->el_G,
                                b->el_Glo, b->el_Sig, b->el_Siglo, b->scratch_f, seg_w, pin_w, lam));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

// TNS / WNS into `part` (2 doubles per block for nb blocks, then the 2 results)
static la_status tns_reduce(la_batch *b, const float *delay, double *part, int nb, double *tns, double *wns)
{
    const TreeDev T = tree_view(b);
    hipLaunchKernelGGL(k_tns_partial, dim3(nb), dim3(kBlock), 0, b->stream, T, delay, part);
    hipLaunchKernelGGL(k_tns_final, dim3(1), dim3(kBlock), 0, b->stream, part, nb, part + 2 * nb);
    LA_HIP(hipGetLastError());
    double h[2];
    LA_HIP(hipMemcpyAsync(h, part + 2 * nb, sizeof(h), hipMemcpyDeviceToHost, b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    *tns = h[0];
    *wns = h[1];
    return LA_OK;
}

static int tns_blocks(const la_batch *b, int cap)
{
    return (int)std::min<int64_t>(cap, std::max<int64_t>(1, (b->sinks + kBlock - 1) / kBlock));
}

la_status timing_summary(la_batch *b, const float *delay, double *tns, double *wns)
{
    return tns_reduce(b, delay, b->red, tns_blocks(b, b->red_blocks), tns, wns);
}

// ---------------------------------------------------------------------------
// The same summary without any library-owned allocation: the block partials and the two
// results live in `scratch`, a fixed device array that every GPU holds once for the life of
// the process.  Host code must not pass the array's name to a kernel (on the host it is a
// stand-in symbol, not a device address): it uses the address hipGetSymbolAddress gives on
// each device, kept in g_scratch.  Calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr int kScratchBlocks = 1024;                        // block partials: at most this many
constexpr int kScratchDoubles = 2 * kScratchBlocks + 2;     // (sum, min) per block, then TNS, WNS
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static double *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

la_status scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(LA_ERR_INVALID_ARG, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return LA_OK;
    int cur = -1;
    LA_HIP(hipGetDevice(&cur));
    if (cur != device) LA_HIP(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = (double *)p;
    return LA_OK;
}

la_status timing_summary_noalloc(la_batch *b, const float *delay, double *tns, double *wns)
{
    double *ws = nullptr;
    if (b->device >= 0 && b->device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ws = g_scratch[b->device];
    }
    if (!ws) {
        const la_status s = scratch_setup(b->device);
        if (s != LA_OK) return s;
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ws = g_scratch[b->device];
    }
    // every block strides over the sinks, so any sink count fits kScratchBlocks partials
    const int nb = tns_blocks(b, kScratchBlocks);
    if (2 * nb + 2 > kScratchDoubles)
        return set_error(LA_ERR_RANGE, "la_timing_summary_noalloc: partials exceed the static scratch");
    return tns_reduce(b, delay, ws, nb, tns, wns);
}

}  // namespace gapla
