// Tree dynamic program of Alg. 3 with the look-ahead of Sec. III-D, trace-back of
// Alg. 4, demand commit and history update -- the plain form, in the shape of
// the paper's Alg. 2: for every batch, one launch per tree level bottom-up and
// one per level top-down, DP state in HBM between launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dp_device.h"
#include "la_internal.h"

namespace gapla {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65535 * 8));
}

// one thread per (node of this level and batch, entering-layer index)
template <int NAMAX>
__global__ void __launch_bounds__(kBlock, NAMAX > 6 ? 4 : 5) k_dp_level(DPArgs a, const int32_t *nodes, int32_t cnt)
{
    __shared__ LayerTab tb;
    load_tab(a.tab, tb);
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = tid / a.NA;
    const int j = (int)(tid - i * a.NA);
    if (i >= cnt) return;
    const int32_t n = nodes[i];
    const bool root = a.T.flags[n] & kRoot;
    int l;
    if (root) {
        if (j != 0) return;
        l = 0;
    } else {
        const int d = a.T.dir[n];
        if (j >= tb.nA[d]) return;
        l = tb.lay[d][j];
    }
    GlobalState st(a);
    const int64_t kap = root ? 0 : kappa_seg(a, tb, n, l);
    dp_node<GlobalState, NAMAX>(a, tb, st, n, l, j, root, kap);
}

// Alg. 4: each node takes the layer its parent recorded for the parent's entering layer.
__global__ void k_trace_level(DPArgs a, const int32_t *nodes, int32_t cnt, uint8_t *cur, uint8_t *vlo, uint8_t *vhi,
                              uint8_t *out_layers, int has_prev, int32_t *chg_node, uint8_t *chg_old,
                              uint8_t *chg_new, int32_t *chg_count)
{
    __shared__ LayerTab tb;
    load_tab(a.tab, tb);
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool changed = false;
    uint8_t old_l = 0;
    int ln = 0;
    int32_t n = 0;
    if (i < cnt) {
        n = nodes[i];
        const int32_t p = a.T.parent[n];
        const int jp = (p < 0 || a.T.parent[p] < 0) ? 0 : tb.jidx[cur[p] & (kMaxL - 1)];
        GlobalState st(a);
        trace_node(tb, st, n, n, jp, p < 0, cur, vlo, vhi, out_layers, has_prev, &ln, &changed, &old_l);
    }
    append_change(ChangeList{chg_node, chg_old, chg_new, chg_count}, changed, n, old_l, (uint8_t)ln);
}

// API grid order ((y * X + x) * L + l) <-> the plane layout of grid_index
__global__ void k_grid_perm(LayerTab tab, const int32_t *src, int32_t *dst, int64_t E, int to_planes)
{
    __shared__ LayerTab tb;
    load_tab(tab, tb);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e % tb.L);
        const int32_t cell = (int32_t)(e / tb.L);
        const int32_t i = grid_index(tb, l, plane_pos(tb, tb.dir[l], cell % tb.X, cell / tb.X));
        if (to_planes) dst[i] = src[e];
        else dst[e] = src[i];
    }
}

__global__ void k_zero_i32(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// demand moves of the segments whose layer changed (HBM atomics; integer, so order-free)
// One lane per GCell edge of the changed segments: a wavefront takes 64 changes, scans their
// lengths and walks the concatenated edges, so consecutive lanes move consecutive edges of a
// segment (adjacent records) rather than one lane walking a whole segment.
__global__ void k_commit(TreeDev T, LayerTab tab, const int32_t *chg_node, const uint8_t *chg_old,
                         const uint8_t *chg_new, const int32_t *chg_count, int32_t *D)
{
    const int32_t cnt = *chg_count;
    const int lane = threadIdx.x & 63;
    const int32_t w0 = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), nw = gridDim.x * (blockDim.x >> 6);
    for (int32_t base = w0 * 64; base < cnt; base += nw * 64) {
        const int32_t i = base + lane;
        int32_t q = 0, len = 0, o = 255, nl = 255;
        if (i < cnt) {
            const int32_t n = chg_node[i];
            o = chg_old[i];
            nl = chg_new[i];
            q = T.g0[n];
            len = T.len[n];
        }
        int32_t pre = len;   // inclusive scan of the lengths
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(pre, d);
            if (lane >= d) pre += y;
        }
        const int32_t total = __shfl(pre, 63);
        for (int32_t e0 = 0; e0 < total; e0 += 64) {
            const int32_t e = e0 + lane;
            // the change holding edge e: the first c with pre[c] > e
            int32_t c = 0;
#pragma unroll
            for (int s = 32; s > 0; s >>= 1) {
                const int32_t pc = __shfl(pre, c + s - 1);
                if (pc <= e) c += s;
            }
            const int32_t pc0 = __shfl(pre, c) - __shfl(len, c);   // first edge of change c
            const int32_t qc = __shfl(q, c), oc = __shfl(o, c), nc = __shfl(nl, c);
            if (e < total) {
                const int32_t k = e - pc0;
                if (oc != 255) atomicAdd(&D[grid_index(tab, oc, qc + k)], -1);
                atomicAdd(&D[grid_index(tab, nc, qc + k)], 1);
            }
        }
    }
}

__device__ __forceinline__ int32_t history_step(int32_t d, int32_t cap, int32_t h, int32_t inc)
{
    const int32_t over = d - cap;
    if (over <= 0) return h;
    const int64_t x = (int64_t)h + (int64_t)inc * over;
    return (int32_t)(x > kHistSat ? kHistSat : x);
}

// Four GCell edges per lane (16-byte demand and history, 4-byte capacity accesses), the tail
// one by one.
__global__ void k_history(const int32_t *D, const uint8_t *caps, int32_t *H, int64_t E, int32_t inc)
{
    const int64_t E4 = E / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < E4; g += stride) {
        const int4 d = ((const int4 *)D)[g];
        const uchar4 c = ((const uchar4 *)caps)[g];
        int4 h = ((const int4 *)H)[g];
        const int4 h0 = h;
        h.x = history_step(d.x, c.x, h.x, inc);
        h.y = history_step(d.y, c.y, h.y, inc);
        h.z = history_step(d.z, c.z, h.z, inc);
        h.w = history_step(d.w, c.w, h.w, inc);
        if (h.x != h0.x || h.y != h0.y || h.z != h0.z || h.w != h0.w) ((int4 *)H)[g] = h;
    }
    for (int64_t g = 4 * E4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < E; g += stride)
        H[g] = history_step(D[g], caps[g], H[g], inc);
}

// Counting sort of nodes by (batch, height).  With few buckets each block keeps a
// private histogram in LDS and touches each global counter once, which keeps the
// atomics off a handful of hot addresses.
constexpr int kLdsBuckets = 4096;

// bucket of node v: (batch, height, number of children clipped to 3), so that the nodes of
// one level are grouped by how much DP work they carry
__device__ __forceinline__ int64_t bucket_key(const TreeDev &T, const int32_t *height, int t, int32_t levels, int64_t v)
{
    const int32_t k = T.ch_ptr[v + 1] - T.ch_ptr[v];
    return ((((int64_t)t * levels + height[v]) << 2) | (k < 3 ? k : 3));
}

__global__ void k_bucket_count(TreeDev T, const int32_t *height, const int32_t *tier, int32_t ntier, int32_t levels,
                               int32_t *counts, int32_t *bad)
{
    __shared__ int32_t hist[kLdsBuckets];
    const int64_t nb = (int64_t)ntier * levels * 4;
    const bool local = nb <= kLdsBuckets;
    if (local)
        for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes; v += (int64_t)gridDim.x * blockDim.x) {
        const int t = tier ? tier[T.net[v]] : 0;
        if (t < 0 || t >= ntier) {
            atomicAdd(bad, 1);
            continue;
        }
        const int64_t q = bucket_key(T, height, t, levels, v);
        if (local) atomicAdd(&hist[q], 1);
        else atomicAdd(&counts[q], 1);
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

__global__ void k_bucket_scatter(TreeDev T, const int32_t *height, const int32_t *tier, int32_t ntier, int32_t levels,
                                 int32_t *cursor, int32_t *out)
{
    __shared__ int32_t hist[kLdsBuckets];
    __shared__ int32_t base[kLdsBuckets];
    const int64_t nb = (int64_t)ntier * levels * 4;
    if (nb > kLdsBuckets) {
        for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes;
             v += (int64_t)gridDim.x * blockDim.x) {
            const int t = tier ? tier[T.net[v]] : 0;
            if (t < 0 || t >= ntier) continue;
            out[atomicAdd(&cursor[bucket_key(T, height, t, levels, v)], 1)] = (int32_t)v;
        }
        return;
    }
    // one tile of blockDim nodes at a time: rank inside the tile, then reserve per bucket
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < T.nodes; v0 += (int64_t)gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        const int64_t v = v0 + threadIdx.x;
        int64_t q = -1;
        int32_t r = 0;
        if (v < T.nodes) {
            const int t = tier ? tier[T.net[v]] : 0;
            if (t >= 0 && t < ntier) {
                q = bucket_key(T, height, t, levels, v);
                r = atomicAdd(&hist[q], 1);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            if (hist[i]) base[i] = atomicAdd(&cursor[i], hist[i]);
        __syncthreads();
        if (q >= 0) out[base[q] + r] = (int32_t)v;
        __syncthreads();
    }
}

__global__ void k_interleave(const uint8_t *lo, const uint8_t *hi, uint8_t *out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        out[2 * i] = lo[i];
        out[2 * i + 1] = hi[i];
    }
}

}  // namespace

la_status interleave_vias(la_batch *b, uint8_t *out)
{
    LA_TIMED(b, "k_interleave", b->stream,
             hipLaunchKernelGGL(k_interleave, dim3(grid_for(b->nodes)), dim3(kBlock), 0, b->stream, b->vlo, b->vhi,
                                out, b->nodes));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

DPArgs make_dp_args(la_batch *b, const la_weights *w, const int32_t *H, const int32_t *lut)
{
    DPArgs a;
    a.T = tree_view(b);
    a.tab = b->tab;
    a.w.w_cong = w->w_cong;
    a.w.w_cap = w->w_cap;
    a.w.w_d = w->w_d;
    a.w.w_via = w->w_via;
    a.w.seg_w = w->seg_w_q10;
    a.w.pin_w = w->pin_w_q10;
    a.w.lam = w->lambda_mohm;
    a.w.lut = lut;
    a.w.self_excl = b->has_prev ? 1 : 0;
    a.D = b->D;
    a.caps = b->caps;
    a.H = H;
    a.prev = b->cur_layer;
    a.F = b->F;
    a.S = b->S;
    a.bt = b->bt;
    a.sel = b->sel;
    a.NA = b->NAmax;
    return a;
}

la_status commit_changed(la_batch *b, int32_t *D)
{
    LA_TIMED(b, "k_commit", b->stream,
             hipLaunchKernelGGL(k_commit, dim3(1024), dim3(kBlock), 0, b->stream, tree_view(b), b->tab, b->chg_node,
                                b->chg_old, b->chg_new, b->chg_count, D));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

la_status grid_to_planes(la_batch *b, const int32_t *api, int32_t *planes)
{
    LA_TIMED(b, "k_grid_perm", b->stream,
             hipLaunchKernelGGL(k_grid_perm, dim3(grid_for(b->E)), dim3(kBlock), 0, b->stream, b->tab, api, planes,
                                b->E, 1));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

la_status planes_to_grid(la_batch *b, const int32_t *planes, int32_t *api)
{
    LA_TIMED(b, "k_grid_perm", b->stream,
             hipLaunchKernelGGL(k_grid_perm, dim3(grid_for(b->E)), dim3(kBlock), 0, b->stream, b->tab, planes, api,
                                b->E, 0));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

la_status zero_i32(la_batch *b, int32_t *p, int64_t n)
{
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(n)), dim3(kBlock), 0, b->stream, p, n);
    LA_HIP(hipGetLastError());
    return LA_OK;
}

la_status history_update(la_batch *b, const int32_t *D, int32_t *H, int32_t inc)
{
    LA_TIMED(b, "k_history", b->stream,
             hipLaunchKernelGGL(k_history, dim3(grid_for(b->Eg / 4 + 1)), dim3(kBlock), 0, b->stream, D, b->caps, H,
                                b->Eg, inc));
    LA_HIP(hipGetLastError());
    return LA_OK;
}

// Group nodes by (batch, height, child class); returns the per-bucket counts on the host.
la_status bucket_nodes(la_batch *b, const int32_t *tier, int32_t ntier, std::vector<int32_t> &counts)
{
    const int32_t Hh = b->levels;
    const size_t need = (size_t)ntier * Hh * 4;
    if (need + 1 > b->bucket_cap) {
        if (b->bucket_cnt) (void)hipFree(b->bucket_cnt);
        if (b->bucket_cur) (void)hipFree(b->bucket_cur);
        b->bucket_cnt = b->bucket_cur = nullptr;
        if (hipMalloc((void **)&b->bucket_cnt, (need + 1) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&b->bucket_cur, (need + 1) * sizeof(int32_t)) != hipSuccess)
            return set_error(LA_ERR_OOM, "bucket allocation failed");
        b->bucket_cap = need + 1;
    }
    la_status s = zero_i32(b, b->bucket_cnt, (int64_t)need + 1);
    if (s != LA_OK) return s;
    const TreeDev T = tree_view(b);
    LA_TIMED(b, "k_bucket_count", b->stream,
             hipLaunchKernelGGL(k_bucket_count, dim3(grid_for(b->nodes)), dim3(kBlock), 0, b->stream, T, b->height,
                                tier, ntier, Hh, b->bucket_cnt, b->bucket_cnt + need));
    LA_HIP(hipGetLastError());
    counts.assign(need + 1, 0);
    LA_HIP(hipMemcpyAsync(counts.data(), b->bucket_cnt, (need + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                          b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    if (counts[need] != 0)
        return set_error(LA_ERR_INVALID_ARG, "a net's batch index is outside 0..num_tiers-1");
    counts.pop_back();
    std::vector<int32_t> off(need, 0);
    int64_t acc = 0;
    for (size_t i = 0; i < need; ++i) {
        off[i] = (int32_t)acc;
        acc += counts[i];
    }
    LA_HIP(hipMemcpyAsync(b->bucket_cur, off.data(), need * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    LA_TIMED(b, "k_bucket_scatter", b->stream,
             hipLaunchKernelGGL(k_bucket_scatter, dim3(grid_for(b->nodes)), dim3(kBlock), 0, b->stream, T, b->height,
                                tier, ntier, Hh, b->bucket_cur, b->bucket_nodes));
    LA_HIP(hipGetLastError());
    // the cursor copy must finish before `off` goes out of scope
    LA_HIP(hipStreamSynchronize(b->stream));
    return LA_OK;
}

la_status assign_plain(la_batch *b, const la_weights *w, int32_t *H, const int32_t *lut, uint8_t *out_layers,
                       const int32_t *batch)
{
    const int32_t ntier = batch ? w->num_tiers : 1;
    std::vector<int32_t> counts;
    la_status s = bucket_nodes(b, batch, ntier, counts);
    if (s != LA_OK) return s;
    const int32_t Hh = b->levels;
    std::vector<int64_t> off(counts.size() + 1, 0);
    for (size_t i = 0; i < counts.size(); ++i) off[i + 1] = off[i] + counts[i];
    for (int32_t r = 0; r < w->rounds; ++r) {
        DPArgs a = make_dp_args(b, w, H, lut);
        for (int32_t t = 0; t < ntier; ++t) {
            if (off[((int64_t)t + 1) * Hh * 4] == off[(int64_t)t * Hh * 4]) continue;   // empty batch
            // one level = the four consecutive child-class buckets of (batch, height)
            for (int32_t h = 0; h < Hh; ++h) {
                const int64_t q = ((int64_t)t * Hh + h) * 4;
                const int32_t cnt = (int32_t)(off[q + 4] - off[q]);
                if (!cnt) continue;
                const int64_t threads = (int64_t)cnt * a.NA;
                const dim3 grid((unsigned)((threads + kBlock - 1) / kBlock));
                if (a.NA <= 4)
                    LA_TIMED(b, "k_dp_level", b->stream,
                             hipLaunchKernelGGL(k_dp_level<4>, grid, dim3(kBlock), 0, b->stream, a,
                                                b->bucket_nodes + off[q], cnt));
                else if (a.NA <= 6)
                    LA_TIMED(b, "k_dp_level", b->stream,
                             hipLaunchKernelGGL(k_dp_level<6>, grid, dim3(kBlock), 0, b->stream, a,
                                                b->bucket_nodes + off[q], cnt));
                else
                    LA_TIMED(b, "k_dp_level", b->stream,
                             hipLaunchKernelGGL(k_dp_level<8>, grid, dim3(kBlock), 0, b->stream, a,
                                                b->bucket_nodes + off[q], cnt));
            }
            hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, b->stream, b->chg_count, (int64_t)1);
            for (int32_t h = Hh - 1; h >= 0; --h) {
                const int64_t q = ((int64_t)t * Hh + h) * 4;
                const int32_t cnt = (int32_t)(off[q + 4] - off[q]);
                if (!cnt) continue;
                LA_TIMED(b, "k_trace_level", b->stream,
                         hipLaunchKernelGGL(k_trace_level, dim3((cnt + kBlock - 1) / kBlock), dim3(kBlock), 0,
                                            b->stream, a, b->bucket_nodes + off[q], cnt, b->cur_layer, b->vlo, b->vhi,
                                            out_layers, b->has_prev ? 1 : 0, b->chg_node, b->chg_old, b->chg_new,
                                            b->chg_count));
            }
            s = commit_changed(b, b->D);
            if (s != LA_OK) return s;
        }
        s = history_update(b, b->D, H, w->hist_inc);
        if (s != LA_OK) return s;
        b->has_prev = true;
    }
    LA_HIP(hipGetLastError());
    return LA_OK;
}

}  // namespace gapla
