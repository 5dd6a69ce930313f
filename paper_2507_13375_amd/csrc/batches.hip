// Classical batching (Alg. 1, GetBatch: the batching of the routers the paper cites for it).
// A net's box is the GCell rectangle its tree spans.  Within each subset, in increasing net
// order, a net joins the lowest batch in which no net's box shares a GCell with its own, so no
// two nets of a batch share a GCell edge and assigning a batch against one demand snapshot
// equals assigning its nets one after another.  Subsets are batched one after another and never
// share a batch.
//
// The result is the sequential first-fit's, computed in parallel: the nets of a subset are
// taken in chunks in their order; inside a chunk every unplaced net paints its box with a key
// that ranks it by position (a max over keys of one epoch), and a net that holds its own key on
// every GCell of its box has no unplaced earlier net of the chunk overlapping it -- so every
// earlier net overlapping it is placed and its batch is the lowest one free on its box (a bit
// set per GCell and batch, OR-ed over the box).  Nets placed in one epoch overlap no other
// net placed in it.  Repeated until the chunk is placed; one cooperative launch walks every
// subset and chunk with grid-wide barriers.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "la_internal.h"

namespace gapla {

namespace {

namespace cg = cooperative_groups;

constexpr int kBT = 256;            // threads per workgroup
constexpr int kChunk = 8192;        // nets of a subset placed per chunk
constexpr int kBatchWords = 16;     // 64-bit words of batch bits per GCell: at most 1024 batches

// ---- stable order of the nets by (subset, index) ---------------------------------------
// per workgroup of kBT consecutive nets and subset s: cnt[s * nblk + blk]
__global__ void k_sub_count(const int32_t *subset, int64_t nets, int32_t nsub, int32_t nblk, int32_t *cnt)
{
    __shared__ int32_t h[256];
    for (int i = threadIdx.x; i < nsub; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
    if (i < nets) {
        const int32_t s = subset[i];
        if (s >= 0 && s < nsub) atomicAdd(&h[s], 1);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nsub; s += blockDim.x) cnt[(int64_t)s * nblk + blockIdx.x] = h[s];
}

// exclusive prefix of x[0, n) in place, one workgroup (n small: subsets x workgroups)
__global__ void k_excl_scan(int32_t *x, int64_t n, int32_t *total)
{
    __shared__ int32_t part[1024];
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t a = threadIdx.x * per, e = std::min<int64_t>(n, a + per);
    int32_t s = 0;
    for (int64_t i = a; i < e; ++i) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < (int)blockDim.x; ++k) {
            const int32_t v = part[k];
            part[k] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int32_t run = part[threadIdx.x];
    for (int64_t i = a; i < e; ++i) {
        const int32_t v = x[i];
        x[i] = run;
        run += v;
    }
}

// ord[position] = net, by (subset, index); a net's rank among the earlier nets of its workgroup
// with the same subset keeps the order inside the subset
__global__ void k_sub_scatter(const int32_t *subset, int64_t nets, int32_t nsub, int32_t nblk, const int32_t *off,
                              int32_t *ord)
{
    __shared__ int32_t sub[kBT];
    const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
    const int32_t s = i < nets ? subset[i] : -1;
    sub[threadIdx.x] = s;
    __syncthreads();
    if (s < 0 || s >= nsub) return;
    int32_t r = 0;
    for (int k = 0; k < (int)threadIdx.x; ++k) r += sub[k] == s ? 1 : 0;
    ord[off[(int64_t)s * nblk + blockIdx.x] + r] = (int32_t)i;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u64(uint64_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

struct FitState {
    int32_t unres[2];    // unplaced nets counted in an epoch (two slots, alternating)
    int32_t maxb;        // highest batch placed so far
    int32_t overflow;    // a net found no free batch among kBatchWords * 64
};

struct FitArgs {
    const int32_t *ord;        // nets by (subset, index)
    const int32_t *sub_start;  // [nsub + 1] position ranges of the subsets
    int32_t nsub;
    const int16_t *box;        // [nets][4] x min, x max, y min, y max
    int32_t X;
    uint64_t *bits;            // [X * Y][kBatchWords] batches present on each GCell
    uint64_t *stamp;           // [X * Y] epoch << 32 | rank key of the painting nets
    int32_t *batch;            // [nets] out; -1 until placed
    FitState *st;
};

__device__ __forceinline__ uint64_t fit_key(uint64_t epoch, int32_t rank)
{
    return (epoch << 32) | (uint64_t)(0xffffffffu - (uint32_t)rank);
}

__global__ void __launch_bounds__(kBT) k_first_fit(FitArgs a)
{
    cg::grid_group grid = cg::this_grid();
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    uint64_t epoch = 0;
    int32_t base = 0;   // first batch of the current subset
    for (int32_t s = 0; s < a.nsub; ++s) {
        const int32_t p0 = a.sub_start[s], p1 = a.sub_start[s + 1];
        for (int32_t c0 = p0; c0 < p1; c0 += kChunk) {
            const int32_t c1 = min(c0 + kChunk, p1);
            for (;;) {
                ++epoch;
                // the slot this epoch counts into was last read two epochs ago
                if (tid == 0) a.st->unres[epoch & 1] = 0;
                for (int64_t p = c0 + tid; p < c1; p += nthr) {
                    const int32_t net = a.ord[p];
                    if (a.batch[net] >= 0) continue;
                    const int16_t *b = a.box + 4 * (int64_t)net;
                    const uint64_t key = fit_key(epoch, (int32_t)(p - c0));
                    for (int32_t y = b[2]; y <= b[3]; ++y)
                        for (int32_t x = b[0]; x <= b[1]; ++x)
                            atomicMax((unsigned long long *)&a.stamp[(int64_t)y * a.X + x], (unsigned long long)key);
                }
                grid.sync();
                for (int64_t p = c0 + tid; p < c1; p += nthr) {
                    const int32_t net = a.ord[p];
                    if (a.batch[net] >= 0) continue;
                    const int16_t *b = a.box + 4 * (int64_t)net;
                    const uint64_t key = fit_key(epoch, (int32_t)(p - c0));
                    bool mine = true;
                    for (int32_t y = b[2]; y <= b[3] && mine; ++y)
                        for (int32_t x = b[0]; x <= b[1]; ++x)
                            if (a.stamp[(int64_t)y * a.X + x] != key) {
                                mine = false;
                                break;
                            }
                    if (!mine) {
                        atomicAdd(&a.st->unres[epoch & 1], 1);
                        continue;
                    }
                    // the lowest batch >= base free on every GCell of the box
                    int32_t bt = -1;
                    for (int w = base >> 6; w < kBatchWords && bt < 0; ++w) {
                        uint64_t used = w == (base >> 6) ? ((uint64_t(1) << (base & 63)) - 1) : 0;
                        for (int32_t y = b[2]; y <= b[3]; ++y)
                            for (int32_t x = b[0]; x <= b[1]; ++x)
                                used |= a.bits[((int64_t)y * a.X + x) * kBatchWords + w];
                        if (~used) bt = w * 64 + __ffsll((unsigned long long)~used) - 1;
                    }
                    if (bt < 0) {
                        atomicOr(&a.st->overflow, 1);
                        bt = kBatchWords * 64 - 1;
                    }
                    const uint64_t bit = uint64_t(1) << (bt & 63);
                    for (int32_t y = b[2]; y <= b[3]; ++y)
                        for (int32_t x = b[0]; x <= b[1]; ++x)
                            atomicOr((unsigned long long *)&a.bits[((int64_t)y * a.X + x) * kBatchWords + (bt >> 6)],
                                     (unsigned long long)bit);
                    a.batch[net] = bt;
                    atomicMax(&a.st->maxb, bt);
                }
                grid.sync();
                if (a.st->unres[epoch & 1] == 0) break;
            }
        }
        grid.sync();
        base = max(base, a.st->maxb + 1);
    }
}

}  // namespace

la_status get_batches(la_batch *b, const int32_t *subset, int32_t nsub, int32_t *out_batch, int32_t *num_batches)
{
    const int64_t N = b->nets;
    const hipStream_t s = b->stream;
    if (N == 0) {
        *num_batches = 0;
        return LA_OK;
    }
    const int32_t nblk = (int32_t)((N + kBT - 1) / kBT);
    const int64_t cells = (int64_t)b->tab.X * b->tab.Y;
    int32_t *cnt = nullptr, *ord = nullptr, *start = nullptr;
    uint64_t *bits = nullptr, *stamp = nullptr;
    FitState *st = nullptr;
    auto release = [&]() {
        for (void *p : {(void *)cnt, (void *)ord, (void *)start, (void *)bits, (void *)stamp, (void *)st})
            if (p) (void)hipFree(p);
    };
    if (hipMalloc((void **)&cnt, (size_t)nsub * nblk * sizeof(int32_t) + 4) != hipSuccess ||
        hipMalloc((void **)&ord, (size_t)N * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&start, (size_t)(nsub + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&bits, (size_t)cells * kBatchWords * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&stamp, (size_t)cells * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&st, sizeof(FitState)) != hipSuccess) {
        release();
        return set_error(LA_ERR_OOM, "la_get_batches: temporaries");
    }
    auto run = [&]() -> la_status {
        const int g = (int)std::min<int64_t>(4096, (cells * kBatchWords + 255) / 256);
        hipLaunchKernelGGL(k_zero_u64, dim3(g), dim3(256), 0, s, bits, cells * kBatchWords);
        hipLaunchKernelGGL(k_zero_u64, dim3(g), dim3(256), 0, s, stamp, cells);
        hipLaunchKernelGGL(k_fill_i32, dim3((int)std::min<int64_t>(4096, (N + 255) / 256)), dim3(256), 0, s,
                           out_batch, -1, N);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)st, -1, 4);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)st, 0, 2);   // unres slots
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int32_t *)st + 3, 0, 1);   // overflow
        LA_TIMED(b, "k_sub_order", s, {
            hipLaunchKernelGGL(k_sub_count, dim3(nblk), dim3(kBT), 0, s, subset, N, nsub, nblk, cnt);
            hipLaunchKernelGGL(k_excl_scan, dim3(1), dim3(1024), 0, s, cnt, (int64_t)nsub * nblk,
                               cnt + (int64_t)nsub * nblk);
            hipLaunchKernelGGL(k_sub_scatter, dim3(nblk), dim3(kBT), 0, s, subset, N, nsub, nblk, cnt, ord);
        });
        LA_HIP(hipGetLastError());
        // subset starts: the scanned count of each subset's first workgroup, and the total
        std::vector<int32_t> hs(nsub + 1);
        for (int32_t k = 0; k < nsub; ++k)
            LA_HIP(hipMemcpyAsync(&hs[k], cnt + (int64_t)k * nblk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LA_HIP(hipMemcpyAsync(&hs[nsub], cnt + (int64_t)nsub * nblk, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LA_HIP(hipStreamSynchronize(s));
        LA_HIP(hipMemcpyAsync(start, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        // one workgroup per CU slot the kernel can hold at once: a cooperative launch needs the
        // whole grid resident
        int per = 0, cus = 0;
        LA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_first_fit, kBT, 0));
        LA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        const int grid = std::max(1, std::min(per, 2) * cus);
        FitArgs fa{ord, start, nsub, b->bbox, b->tab.X, bits, stamp, out_batch, st};
        void *args[] = {&fa};
        LA_TIMED(b, "k_first_fit", s,
                 LA_HIP(hipLaunchCooperativeKernel((const void *)k_first_fit, dim3(grid), dim3(kBT), args, 0, s)));
        FitState h{};
        LA_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
        LA_HIP(hipStreamSynchronize(s));
        if (h.overflow) return set_error(LA_ERR_RANGE, "la_get_batches: more than 1024 batches");
        *num_batches = h.maxb + 1;
        return LA_OK;
    };
    const la_status r = run();
    (void)hipStreamSynchronize(s);
    release();
    return r;
}

}  // namespace gapla
