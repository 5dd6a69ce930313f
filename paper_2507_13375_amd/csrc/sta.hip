// Critical-path net ordering (Sec. III-A, Alg. 1 ordering) on a gate-level graph over the
// nets: static timing with the nets' sink delays, the top-1 critical path of every violating
// primary output, the count of those paths through each net, and the division of the nets into
// ordered subsets (critical by count, semi-critical by slack, the rest).
//
// Each net is driven by one gate; each sink feeds the gate of one net or is a primary output.
// Arrival and required times are single precision, each value rounded once as written and max /
// min exact, so the latest input of each gate (and the bins below) are the same decisions in any
// evaluation order.  The nets are swept level by level of a topological order built on the host
// when the graph is set (one launch per level each way: a level's nets only read the levels
// before it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "la_internal.h"

namespace gapla {

namespace {

constexpr int kSB = 256;

inline int grid_sta(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kSB - 1) / kSB, 8192)); }

__device__ __forceinline__ uint32_t ord_of(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float of_ord(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

struct StaView {
    const int32_t *order;      // nets by level
    const int32_t *fin_ptr;    // [nets + 1] the sinks feeding each net's gate, ascending
    const int32_t *fin;
    const int32_t *next;       // [sinks] net fed, -1 at a primary output
    const float *gd;           // [nets] gate delay, ps
    const int32_t *net_sink_ptr;
    const int32_t *sink_node;
    const int32_t *node_net;
};

// arrival at the drivers of one level's nets and at their sinks; the latest input of each gate
__global__ void k_sta_fwd(StaView v, int32_t lo, int32_t hi, const float *delay, float *AD, float *AS, int32_t *crit_in)
{
    for (int32_t q = lo + blockIdx.x * blockDim.x + threadIdx.x; q < hi; q += gridDim.x * blockDim.x) {
        const int32_t m = v.order[q];
        float in = 0.0f;
        int32_t best = -1;
        for (int32_t j = v.fin_ptr[m]; j < v.fin_ptr[m + 1]; ++j) {
            const int32_t s = v.fin[j];
            const float a = AS[s];
            if (a > in) in = a;
            if (best < 0 || a > AS[best]) best = s;
        }
        const float ad = v.gd[m] + in;
        AD[m] = ad;
        crit_in[m] = best;
        for (int32_t k = v.net_sink_ptr[m]; k < v.net_sink_ptr[m + 1]; ++k) AS[k] = ad + delay[k];
    }
}

// required times of one level's nets (the levels after it are done)
__global__ void k_sta_bwd(StaView v, int32_t lo, int32_t hi, float clock, const float *delay, float *RD, float *RS)
{
    for (int32_t q = lo + blockIdx.x * blockDim.x + threadIdx.x; q < hi; q += gridDim.x * blockDim.x) {
        const int32_t n = v.order[q];
        float rd = INFINITY;
        for (int32_t k = v.net_sink_ptr[n]; k < v.net_sink_ptr[n + 1]; ++k) {
            const int32_t m = v.next[k];
            const float rs = m < 0 ? clock : RD[m] - v.gd[m];
            RS[k] = rs;
            const float r = rs - delay[k];
            if (r < rd) rd = r;
        }
        RD[n] = rd;
    }
}

// slack at every sink; WNS over the primary outputs (ordered-integer minimum, exact)
__global__ void k_sta_slack(StaView v, int64_t sinks, const float *AS, const float *RS, float *slack, uint32_t *wns)
{
    uint32_t m = 0xffffffffu;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sinks; k += (int64_t)gridDim.x * blockDim.x) {
        const float s = RS[k] - AS[k];
        slack[k] = s;
        if (v.next[k] < 0) m = min(m, ord_of(s));
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = min(m, (uint32_t)__shfl_down((int)m, d));
    if ((threadIdx.x & 63) == 0) atomicMin(wns, m);
}

// top-1 critical path of every primary output with slack < 0.7 WNS: back through each gate's
// latest input to a primary input, counting the nets it passes
__global__ void k_sta_paths(StaView v, int64_t sinks, const float *slack, const uint32_t *wns_ord,
                            const int32_t *crit_in, int32_t *crit)
{
    const float wns = of_ord(*wns_ord);
    if (!(wns < 0.0f)) return;
    const float lim = 0.7f * wns;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < sinks; k += (int64_t)gridDim.x * blockDim.x) {
        if (v.next[k] >= 0 || !(slack[k] < lim)) continue;
        int32_t n = v.node_net[v.sink_node[k]];
        for (;;) {
            atomicAdd(&crit[n], 1);
            const int32_t s = crit_in[n];
            if (s < 0) break;
            n = v.node_net[v.sink_node[s]];
        }
    }
}

// C = the largest count above three, and the number of count bins below it
__global__ void k_crit_max(const int32_t *crit, int64_t nets, int32_t *cmax)
{
    int32_t m = 0;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < nets; n += (int64_t)gridDim.x * blockDim.x)
        if (crit[n] > 3) m = max(m, crit[n]);
    for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_down(m, d));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(cmax, m);
}

__device__ __forceinline__ int32_t count_bin(int32_t c, int32_t C)
{
    int32_t k = 0;
    while (((int64_t)c << k) < C) ++k;
    return k;
}

__global__ void k_crit_bins(const int32_t *crit, int64_t nets, const int32_t *cmax, int32_t *kmax)
{
    const int32_t C = *cmax;
    int32_t m = 0;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < nets; n += (int64_t)gridDim.x * blockDim.x)
        if (crit[n] > 3) m = max(m, count_bin(crit[n], C) + 1);
    for (int d = 32; d > 0; d >>= 1) m = max(m, __shfl_down(m, d));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(kmax, m);
}

// the subset of every net: critical bins 0..kc-1, the seven slack bins, then the rest
__global__ void k_alg1_subsets(StaView v, int64_t nets, const float *slack, const int32_t *crit, float wns,
                               const int32_t *cmax, int32_t kc, int32_t *subset)
{
    const int32_t C = *cmax;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < nets; n += (int64_t)gridDim.x * blockDim.x) {
        if (crit[n] > 3) {
            subset[n] = count_bin(crit[n], C);
            continue;
        }
        float ns = INFINITY;
        for (int32_t k = v.net_sink_ptr[n]; k < v.net_sink_ptr[n + 1]; ++k) ns = fminf(ns, slack[k]);
        int32_t b = 7;
        if (wns < 0.0f && ns < 0.7f * wns) {
            const float rho = ns / wns;
            if (rho >= 1.0f) b = 0;
            else if (rho >= 0.99f) b = 1;
            else if (rho >= 0.96f) b = 2;
            else if (rho >= 0.91f) b = 3;
            else if (rho >= 0.84f) b = 4;
            else if (rho >= 0.75f) b = 5;
            else b = 6;
        }
        subset[n] = kc + b;
    }
}

__global__ void k_fill32(int32_t *p, int32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

StaView sta_view(const la_batch *b)
{
    return StaView{b->sta_order, b->sta_fin_ptr, b->sta_fin, b->sta_next, b->sta_gd, b->net_sink_ptr, b->sink_node,
                   b->net};
}

template <typename T>
la_status up(T **dst, const std::vector<T> &src)
{
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    if (hipMalloc((void **)dst, std::max<size_t>(src.size(), 1) * sizeof(T)) != hipSuccess)
        return set_error(LA_ERR_OOM, "la_timing_graph: device arrays");
    if (!src.empty()) LA_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return LA_OK;
}

}  // namespace

la_status timing_graph(la_batch *b, const int32_t *sink_next, const int32_t *gate_fs, int32_t clock_fs)
{
    const int64_t N = b->nets, S = b->sinks;
    // the net of each sink, from the host copy of the net ranges and the device sink map
    std::vector<int32_t> sink_node(S), node_net(b->nodes);
    if (S) LA_HIP(hipMemcpy(sink_node.data(), b->sink_node, S * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (b->nodes) LA_HIP(hipMemcpy(node_net.data(), b->net, b->nodes * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> next(sink_next, sink_next + S), fin_ptr(N + 1, 0), fin(std::max<int64_t>(S, 1));
    for (int64_t k = 0; k < S; ++k) {
        if (next[k] < -1 || next[k] >= N) return set_error(LA_ERR_INVALID_ARG, "la_timing_graph: sink_next out of range");
        if (next[k] >= 0) fin_ptr[next[k] + 1]++;
    }
    for (int64_t m = 0; m < N; ++m) fin_ptr[m + 1] += fin_ptr[m];
    {
        std::vector<int32_t> fill(fin_ptr.begin(), fin_ptr.end() - 1);
        for (int64_t k = 0; k < S; ++k)
            if (next[k] >= 0) fin[fill[next[k]]++] = (int32_t)k;
    }
    // levels of a topological order (Kahn): a net's level is one more than the highest level of
    // the nets whose sinks feed it
    std::vector<int32_t> indeg(N), level(N, 0), queue;
    queue.reserve(N);
    for (int64_t m = 0; m < N; ++m) {
        indeg[m] = fin_ptr[m + 1] - fin_ptr[m];
        if (!indeg[m]) queue.push_back((int32_t)m);
    }
    std::vector<int32_t> nsp(b->h_net_sink_ptr);
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t n = queue[h];
        for (int32_t k = nsp[n]; k < nsp[n + 1]; ++k) {
            const int32_t m = next[k];
            if (m < 0) continue;
            level[m] = std::max(level[m], level[n] + 1);
            if (--indeg[m] == 0) queue.push_back(m);
        }
    }
    if ((int64_t)queue.size() != N) return set_error(LA_ERR_INVALID_ARG, "la_timing_graph: the gate graph has a cycle");
    int32_t nlev = 0;
    for (int64_t m = 0; m < N; ++m) nlev = std::max(nlev, level[m] + 1);
    std::vector<int32_t> lp(nlev + 1, 0), order(N);
    for (int64_t m = 0; m < N; ++m) lp[level[m] + 1]++;
    for (int32_t h = 0; h < nlev; ++h) lp[h + 1] += lp[h];
    {
        std::vector<int32_t> fill(lp.begin(), lp.end() - 1);
        for (int64_t m = 0; m < N; ++m) order[fill[level[m]]++] = (int32_t)m;
    }
    std::vector<float> gd(N);
    for (int64_t m = 0; m < N; ++m) {
        if (gate_fs[m] < 0) return set_error(LA_ERR_INVALID_ARG, "la_timing_graph: negative gate delay");
        gd[m] = (float)((double)gate_fs[m] * 1e-3);
    }
    la_status s = up(&b->sta_next, next);
    if (s == LA_OK) s = up(&b->sta_fin_ptr, fin_ptr);
    if (s == LA_OK) s = up(&b->sta_fin, fin);
    if (s == LA_OK) s = up(&b->sta_order, order);
    if (s == LA_OK) s = up(&b->sta_gd, gd);
    if (s != LA_OK) return s;
    // work arrays: AD, RD per net; AS, RS per sink; latest input per net; reductions
    if (!b->sta_f) {
        if (hipMalloc((void **)&b->sta_f, (size_t)(2 * N + 2 * S + 1) * sizeof(float)) != hipSuccess ||
            hipMalloc((void **)&b->sta_i, (size_t)(N + 8) * sizeof(int32_t)) != hipSuccess)
            return set_error(LA_ERR_OOM, "la_timing_graph: work arrays");
    }
    b->sta_lvl = lp;
    b->sta_clock = (float)((double)clock_fs * 1e-3);
    b->sta_ready = true;
    return LA_OK;
}

la_status sta(la_batch *b, const float *delay, float *slack, int32_t *crit, float *wns_out)
{
    if (!b->sta_ready) return set_error(LA_ERR_STATE, "la_sta needs la_timing_graph first");
    const int64_t N = b->nets, S = b->sinks;
    const hipStream_t s = b->stream;
    const StaView v = sta_view(b);
    float *AD = b->sta_f, *RD = AD + N, *AS = RD + N, *RS = AS + S;
    int32_t *crit_in = b->sta_i;
    uint32_t *wns = (uint32_t *)(b->sta_i + N);
    const int32_t nlev = (int32_t)b->sta_lvl.size() - 1;
    LA_TIMED(b, "k_sta_fwd", s, {
        for (int32_t h = 0; h < nlev; ++h) {
            const int32_t lo = b->sta_lvl[h], hi = b->sta_lvl[h + 1];
            if (hi > lo)
                hipLaunchKernelGGL(k_sta_fwd, dim3(grid_sta(hi - lo)), dim3(kSB), 0, s, v, lo, hi, delay, AD, AS,
                                   crit_in);
        }
    });
    LA_TIMED(b, "k_sta_bwd", s, {
        for (int32_t h = nlev - 1; h >= 0; --h) {
            const int32_t lo = b->sta_lvl[h], hi = b->sta_lvl[h + 1];
            if (hi > lo)
                hipLaunchKernelGGL(k_sta_bwd, dim3(grid_sta(hi - lo)), dim3(kSB), 0, s, v, lo, hi, b->sta_clock, delay,
                                   RD, RS);
        }
    });
    hipLaunchKernelGGL(k_fill32, dim3(1), dim3(64), 0, s, (int32_t *)wns, -1, 1);
    hipLaunchKernelGGL(k_fill32, dim3(grid_sta(N)), dim3(kSB), 0, s, crit, 0, N);
    LA_TIMED(b, "k_sta_slack", s,
             hipLaunchKernelGGL(k_sta_slack, dim3(std::min(grid_sta(S), 2048)), dim3(kSB), 0, s, v, S, AS, RS, slack,
                                wns));
    LA_TIMED(b, "k_sta_paths", s,
             hipLaunchKernelGGL(k_sta_paths, dim3(grid_sta(S)), dim3(kSB), 0, s, v, S, slack, wns, crit_in, crit));
    LA_HIP(hipGetLastError());
    uint32_t w = 0;
    LA_HIP(hipMemcpyAsync(&w, wns, sizeof(w), hipMemcpyDeviceToHost, s));
    LA_HIP(hipStreamSynchronize(s));
    const uint32_t u = (w & 0x80000000u) ? (w & 0x7fffffffu) : ~w;
    float f;
    std::memcpy(&f, &u, sizeof(f));
    *wns_out = S ? f : INFINITY;
    return LA_OK;
}

la_status alg1_subsets(la_batch *b, const float *slack, const int32_t *crit, float wns, int32_t *subset,
                       int32_t *num_subsets)
{
    if (!b->sta_ready) return set_error(LA_ERR_STATE, "la_alg1_subsets needs la_timing_graph first");
    const int64_t N = b->nets;
    const hipStream_t s = b->stream;
    int32_t *cm = b->sta_i + N + 1;   // C, bins
    hipLaunchKernelGGL(k_fill32, dim3(1), dim3(64), 0, s, cm, 0, 2);
    hipLaunchKernelGGL(k_crit_max, dim3(grid_sta(N)), dim3(kSB), 0, s, crit, N, cm);
    hipLaunchKernelGGL(k_crit_bins, dim3(grid_sta(N)), dim3(kSB), 0, s, crit, N, cm, cm + 1);
    LA_HIP(hipGetLastError());
    int32_t kc = 0;
    LA_HIP(hipMemcpyAsync(&kc, cm + 1, sizeof(kc), hipMemcpyDeviceToHost, s));
    LA_HIP(hipStreamSynchronize(s));
    LA_TIMED(b, "k_alg1_subsets", s,
             hipLaunchKernelGGL(k_alg1_subsets, dim3(grid_sta(N)), dim3(kSB), 0, s, sta_view(b), N, slack, crit, wns, cm,
                                kc, subset));
    LA_HIP(hipGetLastError());
    *num_subsets = kc + 8;
    return LA_OK;
}

}  // namespace gapla
