// Quality terms of an assignment (Sec. II): total overflow with the exponential per-edge
// overflow of Eq. 3 and with the clipped difference of Eq. 2, via count, and the wire
// capacitance that stands for power in the weighted score of Eq. 1.  One grid-stride pass
// over the GCell edges, in the library's layout (a lane reads one GCell record, consecutive
// lanes consecutive records), and over the tree nodes; each workgroup leaves its partial
// sums, which the host adds in workgroup order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "dp_device.h"
#include "la_internal.h"

namespace gapla {

namespace {

constexpr int kQThreads = 256;
constexpr int kQBlocks = 2048;   // 8 workgroups per CU of a 256-CU part
constexpr int kQParts = 5;   // tof, overflow sum, overflowed edges, vias, wire capacitance
static_assert(kQBlocks * kQParts == kQPartials, "partials buffer of the batch");

// ofw: [kMaxL] layer weights, then e^{0.5 x} and e^{1.5 x} for x in [-kQSpan, kQSpan]
__global__ void __launch_bounds__(kQThreads) k_quality(LayerTab tab, const int32_t *D, const uint8_t *caps, int64_t,
                                                       const double *ofw, TreeDev T, const uint8_t *layer,
                                                       const uint8_t *vlo, const uint8_t *vhi, double *part)
{
    __shared__ LayerTab tb;
    __shared__ double w[kMaxL];
    __shared__ double ex[2][2 * kQSpan + 1];
    __shared__ double rt[kQThreads / 64];
    __shared__ int64_t ri[4][kQThreads / 64];
    load_tab(tab, tb);
    if (threadIdx.x < (unsigned)tb.L) w[threadIdx.x] = ofw[threadIdx.x];
    for (int i = threadIdx.x; i < 2 * (2 * kQSpan + 1); i += blockDim.x)
        ex[i / (2 * kQSpan + 1)][i % (2 * kQSpan + 1)] = ofw[kMaxL + i];
    __syncthreads();
    double tof = 0.0;
    int64_t osum = 0, oedges = 0, vias = 0, wcap = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto edge = [&](int l, int32_t i) {
        const int32_t c = caps[i];
        const int64_t over = (int64_t)D[i] - c;
        const int z = c > 0 ? 0 : 1;
        tof += w[l] * (over >= -kQSpan && over <= kQSpan ? ex[z][over + kQSpan] : exp((z ? 1.5 : 0.5) * (double)over));
        if (over > 0) {
            osum += over;
            oedges += 1;
        }
    };
    const int32_t P = tb.X * tb.Y;
    // routable layers: one record of a direction's layers per GCell
    for (int d = 0; d < 2; ++d)
        for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < P; q += (int32_t)stride)
            for (int jj = 0; jj < tb.nA[d]; ++jj) edge(tb.lay[d][jj], route_index(tb, d, jj, q));
    // the other layers: one plane each
    for (int l = 0; l < tb.L; ++l)
        if (tb.jidx[l] < 0)
            for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < P; q += (int32_t)stride)
                edge(l, grid_index(tb, l, q));
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes; v += stride) {
        vias += (int64_t)vhi[v] - (int64_t)vlo[v];
        if (T.parent[v] >= 0) wcap += (int64_t)tb.c[layer[v]] * T.len[v];
    }
    // workgroup sums: wavefront shuffles, then the wavefronts in order
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        tof += __shfl_down(tof, d);
        osum += __shfl_down(osum, d);
        oedges += __shfl_down(oedges, d);
        vias += __shfl_down(vias, d);
        wcap += __shfl_down(wcap, d);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        rt[wv] = tof;
        ri[0][wv] = osum;
        ri[1][wv] = oedges;
        ri[2][wv] = vias;
        ri[3][wv] = wcap;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        int64_t s[4] = {0, 0, 0, 0};
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            t += rt[q];
            for (int k = 0; k < 4; ++k) s[k] += ri[k][q];
        }
        double *p = part + (int64_t)blockIdx.x * kQParts;
        p[0] = t;
        for (int k = 0; k < 4; ++k) {
            double bits;
            memcpy(&bits, &s[k], sizeof(bits));
            p[1 + k] = bits;
        }
    }
}

}  // namespace

la_status timing_summary(la_batch *b, const float *delay, double *tns, double *wns);

la_status quality_report(la_batch *b, const double *ofw, const float *delay, const la_score_weights *sw,
                         la_quality *out)
{
    // layer weights, then e^{0.5 x} and e^{1.5 x} for the integer excesses of the table
    double w[kMaxL + 2 * (2 * kQSpan + 1)];
    for (int l = 0; l < kMaxL; ++l) w[l] = (ofw && l < b->tab.L) ? ofw[l] : 1.0;
    for (int z = 0; z < 2; ++z)
        for (int x = -kQSpan; x <= kQSpan; ++x) w[kMaxL + z * (2 * kQSpan + 1) + x + kQSpan] = std::exp((z ? 1.5 : 0.5) * x);
    LA_HIP(hipMemcpyAsync(b->qofw, w, sizeof(w), hipMemcpyHostToDevice, b->stream));

    LA_TIMED(b, "k_quality", b->stream,
             hipLaunchKernelGGL(k_quality, dim3(kQBlocks), dim3(kQThreads), 0, b->stream, b->tab, b->D, b->caps, b->E,
                                b->qofw, tree_view(b), b->cur_layer, b->vlo, b->vhi, b->qpart));
    LA_HIP(hipGetLastError());
    std::vector<double> part((size_t)kQBlocks * kQParts);
    LA_HIP(hipMemcpyAsync(part.data(), b->qpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    la_quality q;
    memset(&q, 0, sizeof(q));
    int64_t s[4] = {0, 0, 0, 0};
    for (int k = 0; k < kQBlocks; ++k) {
        q.tof += part[k * kQParts];
        for (int j = 0; j < 4; ++j) {
            int64_t v;
            memcpy(&v, &part[k * kQParts + 1 + j], sizeof(v));
            s[j] += v;
        }
    }
    q.overflow_sum = s[0];
    q.overflow_edges = s[1];
    q.vias = s[2];
    q.wire_cap_af = s[3];
    if (delay && b->sinks > 0) {
        la_status st = timing_summary(b, delay, &q.tns_ps, &q.wns_ps);
        if (st != LA_OK) return st;
        if (sw)
            q.score = sw->w1 * (q.wns_ps - sw->r1) + sw->w2 * (q.tns_ps - sw->r2) / (double)b->sinks +
                      sw->w3 * ((double)q.wire_cap_af / 1000.0 - sw->r3) + sw->w4 * q.tof;
    }
    *out = q;
    return LA_OK;
}

}  // namespace gapla
