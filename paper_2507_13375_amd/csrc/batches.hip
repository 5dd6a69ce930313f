// Classical batching (Alg. 1, GetBatch: the batching of the routers the paper cites for it).
// A net's box is the GCell rectangle its tree spans.  Within each subset, in increasing net
// order, a net joins the lowest batch in which no net's box shares a GCell with its own, so no
// two nets of a batch share a GCell edge and assigning a batch against one demand snapshot
// equals assigning its nets one after another.  Subsets are batched one after another and never
// share a batch.
//
// The result is the sequential first-fit's, computed in parallel: the nets of a subset are
// taken in chunks in their order; inside a chunk every unplaced net paints the bins (squares of
// GCells) of its box with a key that ranks it by position (a max over keys of one epoch), and a
// net that holds its own key on every bin of its box has no unplaced earlier net of the chunk
// overlapping it -- so every earlier net overlapping it is placed and its batch is the lowest
// one free on its box (a bit set per GCell and batch, OR-ed over the box).  Nets placed in one
// epoch share no bin.  Repeated until the chunk is placed; one cooperative launch walks every
// subset and chunk with grid-wide barriers, the bins of a chunk's boxes spread evenly over its
// wavefronts.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "la_internal.h"

namespace gapla {

namespace {

namespace cg = cooperative_groups;

constexpr int kBT = 256;            // threads per workgroup
// The first-fit kernel: a grid-wide barrier costs about 0.1 us per workgroup on this part, so
// few large workgroups
constexpr int kFT = 1024;           // threads per first-fit workgroup
constexpr int kFitGroups = 64;      // first-fit workgroups (fewer where fewer fit at once)
constexpr int kChunk = 8192;        // nets of a subset placed per chunk
constexpr int kBatchWords = 16;     // 64-bit words of batch bits per GCell: at most 1024 batches
static_assert(kBatchWords % 8 == 0, "the batch words are scanned eight at a time");

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
    int32_t unres[2];    // an epoch left a net unplaced (two slots, alternating)
    int32_t maxb;        // highest batch placed so far
    int32_t overflow;    // a net found no free batch among kBatchWords * 64
};

// Blocking is decided on bins of kBin x kBin GCells: two boxes that share a GCell share a bin,
// so a net that holds its key on every bin of its box has no unplaced earlier net overlapping it
// (a shared bin without a shared GCell only delays a net by an epoch: the result is unchanged).
constexpr int kBinShift = 2;

struct FitArgs {
    const int32_t *ord;        // nets by (subset, index)
    const int32_t *sub_start;  // [nsub + 1] position ranges of the subsets
    int32_t nsub;
    const int16_t *box;        // [nets][4] x min, x max, y min, y max (GCells)
    int32_t X, BX;             // GCells and bins per row
    uint64_t *bits;            // [X * Y][kBatchWords] batches present on each GCell
    uint64_t *stamp;           // [bins] epoch << 32 | rank key of the painting nets
    int64_t *ccum;             // [kChunk + 1] bins of the chunk's boxes before each position
    uint64_t *qbox;            // [kChunk] bin box of each position: x0 | y0 << 16 | width << 32
    uint32_t *qstate;          // [kChunk] kPlaced, or the last epoch in which the position waited
    int32_t *batch;            // [nets] out; -1 until placed
    FitState *st;
};

constexpr uint32_t kPlaced = 0xffffffffu;

__device__ __forceinline__ uint64_t fit_key(uint64_t epoch, int32_t rank)
{
    return (epoch << 32) | (uint64_t)(0xffffffffu - (uint32_t)rank);
}

// GCell i (row-major) of a box
__device__ __forceinline__ int64_t box_cell(const int16_t *b, int32_t bw, int32_t X, int32_t i)
{
    return (int64_t)(b[2] + i / bw) * X + (b[0] + i % bw);
}

// bin box of a GCell box: packed corner and width, and the number of bins
__device__ __forceinline__ uint64_t bin_box(const int16_t *b, int32_t &area)
{
    const int32_t x0 = b[0] >> kBinShift, y0 = b[2] >> kBinShift;
    const int32_t w = (b[1] >> kBinShift) - x0 + 1;
    area = w * ((b[3] >> kBinShift) - y0 + 1);
    return (uint64_t)x0 | (uint64_t)y0 << 16 | (uint64_t)w << 32;
}

// The painting and the key checks walk the bins of the chunk's boxes as one flat range (boxes
// in position order, each row-major), split evenly over the wavefronts of the grid, 64
// consecutive bins per wavefront step: box sizes run from one bin to thousands.  A lane starts
// at bin e0 + lane, at position qs (found once per chunk).  `f(q, bin)` visits each bin of the
// box at position q for which `want(state of q)` holds.
template <class W, class F>
__device__ __forceinline__ void walk_bins(const FitArgs &a, int64_t e0, int64_t e1, int32_t qs, int lane, W want,
                                          F f)
{
    if (e0 + lane >= e1) return;
    int32_t q = qs;
    int64_t qbeg = a.ccum[q], qend = a.ccum[q + 1];
    uint64_t bb = a.qbox[q];
    bool on = want(a.qstate[q]);
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        if (e >= qend) {
            do {
                ++q;
                qbeg = qend;
                qend = a.ccum[q + 1];
            } while (e >= qend);
            bb = a.qbox[q];
            on = want(a.qstate[q]);
        }
        if (on) {
            const int32_t i = (int32_t)(e - qbeg), w = (int32_t)(bb >> 32);
            const int32_t x0 = (int32_t)(bb & 0xffff), y0 = (int32_t)((bb >> 16) & 0xffff);
            f(q, (int64_t)(y0 + i / w) * a.BX + (x0 + i % w));
        }
    }
}

// Per chunk: paint (all its nets), then per epoch e: check -> barrier -> the nets that hold
// their key everywhere take their batch while the others paint for epoch e + 1 -> barrier.
__global__ void __launch_bounds__(kFT) k_first_fit(FitArgs a)
{
    cg::grid_group grid = cg::this_grid();
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kFT / 64) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (kFT / 64);
    __shared__ int64_t part[kFT];
    uint64_t epoch = 0;
    int32_t base = 0;     // first batch of the current subset
    int32_t wmax = -1;    // highest batch this wavefront placed in the current subset
    for (int32_t s = 0; s < a.nsub; ++s) {
        const int32_t p0 = a.sub_start[s], p1 = a.sub_start[s + 1];
        wmax = -1;
        for (int32_t c0 = p0; c0 < p1; c0 += kChunk) {
            const int32_t c1 = min(c0 + kChunk, p1), n = c1 - c0;
            // the chunk's bin boxes, bin offsets and states, by the first workgroup
            if (blockIdx.x == 0) {
                const int32_t per = (n + kFT - 1) / kFT, q0 = threadIdx.x * per, q1 = min(n, q0 + per);
                int64_t sum = 0;
                for (int32_t q = q0; q < q1; ++q) {
                    int32_t area;
                    a.qbox[q] = bin_box(a.box + 4 * (int64_t)a.ord[c0 + q], area);
                    a.qstate[q] = 0;
                    sum += area;
                }
                part[threadIdx.x] = sum;
                __syncthreads();
                if (threadIdx.x == 0) {
                    int64_t run = 0;
                    for (int t = 0; t < kFT; ++t) {
                        const int64_t v = part[t];
                        part[t] = run;
                        run += v;
                    }
                    a.ccum[n] = run;
                }
                __syncthreads();
                int64_t run = part[threadIdx.x];
                for (int32_t q = q0; q < q1; ++q) {
                    a.ccum[q] = run;
                    int32_t area;
                    (void)bin_box(a.box + 4 * (int64_t)a.ord[c0 + q], area);
                    run += area;
                }
            }
            grid.sync();
            // this wavefront's share of the chunk's bins and each lane's first position
            const int64_t total = a.ccum[n];
            const int64_t per = ((total + nw - 1) / nw + 63) / 64 * 64;
            const int64_t e0 = min(total, wid * per), e1 = min(total, e0 + per);
            int32_t qs = 0;
            if (e0 + lane < e1) {
                int32_t lo = 0, hi = n - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (a.ccum[mid] <= e0 + lane) lo = mid;
                    else hi = mid - 1;
                }
                qs = lo;
            }
            ++epoch;
            walk_bins(
                a, e0, e1, qs, lane, [&](uint32_t) { return true; },
                [&](int32_t q, int64_t bin) {
                    atomicMax((unsigned long long *)&a.stamp[bin], (unsigned long long)fit_key(epoch, q));
                });
            grid.sync();
            for (;;) {
                // this epoch's slot was last read two barriers ago
                if (wid == 0 && lane == 0) a.st->unres[epoch & 1] = 0;
                // a net that finds a higher key on one of its bins waits: an earlier unplaced net
                // may share a GCell with it
                walk_bins(
                    a, e0, e1, qs, lane, [&](uint32_t st) { return st != kPlaced; },
                    [&](int32_t q, int64_t bin) {
                        if (a.stamp[bin] != fit_key(epoch, q)) a.qstate[q] = (uint32_t)epoch;
                    });
                grid.sync();
                // the waiting nets paint for the next epoch ...
                walk_bins(
                    a, e0, e1, qs, lane, [&](uint32_t st) { return st == (uint32_t)epoch; },
                    [&](int32_t q, int64_t bin) {
                        atomicMax((unsigned long long *)&a.stamp[bin], (unsigned long long)fit_key(epoch + 1, q));
                    });
                // ... and the others take the lowest batch >= base free on every GCell of their box,
                // one wavefront per net.  No two of them share a bin, so none shares a GCell.  The
                // wavefront's positions q = wid + nw * k are read by lane k at once.
                bool waiting = false;
                for (int64_t k0 = 0; wid + nw * k0 < n; k0 += 64) {
                    const int64_t myq = wid + nw * (k0 + lane);
                    uint32_t st = kPlaced;
                    if (myq < n) st = a.qstate[myq];
                    waiting |= __any(st == (uint32_t)epoch) != 0;
                    unsigned long long ready = __ballot(st != kPlaced && st != (uint32_t)epoch);
                    while (ready) {
                        const int k = __ffsll(ready) - 1;
                        ready &= ready - 1;
                        const int32_t q = (int32_t)(wid + nw * (k0 + k));
                        const int32_t net = a.ord[c0 + q];
                        const int16_t *b = a.box + 4 * (int64_t)net;
                        const int32_t bw = b[1] - b[0] + 1, area = bw * (b[3] - b[2] + 1);
                        // eight batch words (64 bytes of a GCell's 128-byte record) per pass over
                        // the box; words below the subset's first batch count as taken
                        int32_t bt = -1;
                        const int wb = base >> 6;
                        for (int w0 = wb & ~7; w0 < kBatchWords && bt < 0; w0 += 8) {
                            unsigned long long u[8];
#pragma unroll
                            for (int k = 0; k < 8; ++k) u[k] = 0ull;
                            for (int32_t i = lane; i < area; i += 64) {
                                const ulonglong2 *p =
                                    (const ulonglong2 *)(a.bits + box_cell(b, bw, a.X, i) * kBatchWords + w0);
#pragma unroll
                                for (int k = 0; k < 4; ++k) {
                                    const ulonglong2 x = p[k];
                                    u[2 * k] |= x.x;
                                    u[2 * k + 1] |= x.y;
                                }
                            }
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                for (int o = 32; o > 0; o >>= 1) u[k] |= __shfl_xor(u[k], o);
                                const int w = w0 + k;
                                if (w < wb) u[k] = ~0ull;
                                else if (w == wb) u[k] |= (1ull << (base & 63)) - 1;
                                if (bt < 0 && ~u[k]) bt = w * 64 + __ffsll(~u[k]) - 1;
                            }
                        }
                        if (bt < 0) {
                            if (lane == 0) a.st->overflow = 1;
                            bt = kBatchWords * 64 - 1;
                        }
                        const unsigned long long bit = 1ull << (bt & 63);
                        for (int32_t i = lane; i < area; i += 64) {
                            uint64_t *wd = &a.bits[box_cell(b, bw, a.X, i) * kBatchWords + (bt >> 6)];
                            *wd |= bit;
                        }
                        if (lane == 0) {
                            a.batch[net] = bt;
                            a.qstate[q] = kPlaced;
                        }
                        wmax = max(wmax, bt);
                    }
                }
                if (waiting && lane == 0) a.st->unres[epoch & 1] = 1;
                grid.sync();
                const bool again = a.st->unres[epoch & 1] != 0;
                ++epoch;
                if (!again) break;
            }
        }
        if (lane == 0 && wmax >= 0) atomicMax(&a.st->maxb, wmax);
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
    const int32_t BX = ((b->tab.X - 1) >> kBinShift) + 1, BY = ((b->tab.Y - 1) >> kBinShift) + 1;
    const int64_t bins = (int64_t)BX * BY;
    int32_t *cnt = nullptr, *ord = nullptr, *start = nullptr;
    uint64_t *bits = nullptr, *stamp = nullptr;
    int64_t *ccum = nullptr;
    uint64_t *qbox = nullptr;
    uint32_t *qstate = nullptr;
    FitState *st = nullptr;
    auto release = [&]() {
        for (void *p : {(void *)cnt, (void *)ord, (void *)start, (void *)bits, (void *)stamp, (void *)ccum,
                        (void *)qbox, (void *)qstate, (void *)st})
            if (p) (void)hipFree(p);
    };
    if (hipMalloc((void **)&cnt, (size_t)nsub * nblk * sizeof(int32_t) + 4) != hipSuccess ||
        hipMalloc((void **)&ord, (size_t)N * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&start, (size_t)(nsub + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&bits, (size_t)cells * kBatchWords * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&stamp, (size_t)bins * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&ccum, (size_t)(kChunk + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void **)&qbox, (size_t)kChunk * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&qstate, (size_t)kChunk * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void **)&st, sizeof(FitState)) != hipSuccess) {
        release();
        return set_error(LA_ERR_OOM, "la_get_batches: temporaries");
    }
    auto run = [&]() -> la_status {
        const int g = (int)std::min<int64_t>(4096, (cells * kBatchWords + 255) / 256);
        hipLaunchKernelGGL(k_zero_u64, dim3(g), dim3(256), 0, s, bits, cells * kBatchWords);
        hipLaunchKernelGGL(k_zero_u64, dim3(g), dim3(256), 0, s, stamp, bins);
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
        LA_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_first_fit, kFT, 0));
        LA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        const int grid = std::max(1, std::min(kFitGroups, per * cus));
        FitArgs fa{ord, start, nsub, b->bbox, b->tab.X, BX, bits, stamp, ccum, qbox, qstate, out_batch, st};
        void *args[] = {&fa};
        LA_TIMED(b, "k_first_fit", s,
                 LA_HIP(hipLaunchCooperativeKernel((const void *)k_first_fit, dim3(grid), dim3(kFT), args, 0, s)));
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
