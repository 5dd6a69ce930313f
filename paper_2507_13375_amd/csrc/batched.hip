// Batched form of the layer-assignment DP: one persistent launch per batch (tier)
// instead of one launch per tree level.  Workgroups pull groups of nets from a
// work queue, stage whole nets in LDS (DP state, congestion costs, children,
// height order), run the bottom-up DP of Alg. 3 and the top-down trace-back of
// Alg. 4 with workgroup barriers between levels, and append changed segments for
// the commit.  Nets larger than one LDS tile keep their DP state in HBM and walk
// their own levels in a workgroup of their own.  All negotiation rounds of a
// la_assign call are captured once as a hipGraph and replayed.
//
// Every net's result depends only on its own inputs and the demand snapshot of its
// batch, so the layers equal the plain form's for any grid size or claim order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "dp_device.h"
#include "la_internal.h"

namespace gapla {

DPArgs make_dp_args(la_batch *b, const la_weights *w, const int32_t *H, const int32_t *lut);
la_status commit_changed(la_batch *b, int32_t *D);
la_status history_update(la_batch *b, const int32_t *D, int32_t *H, int32_t inc);

// tile sizes built for a routable-layer count per direction (every count takes kCap)
bool tile_size_supported(int NA, int cap)
{
    return cap == kCap || (NA > 4 && NA <= 6 && (cap == 128 || cap == 256));
}

namespace {

constexpr int kThreads = 256;
constexpr int kBook = 10 * kClaimNets + 8;  // ints of per-claim bookkeeping
constexpr int kHB = kHeightClasses;   // height classes of small nets per batch
constexpr int kNB = kPartBuckets;     // partition buckets per batch
constexpr int32_t kMergeNets = 64;     // batches of at most this many small nets may share a launch

// DP state and per-node inputs of one LDS tile, indexed by tile-local node id.  ZW: every net
// of the tile has zero segment weights, look-ahead coefficients and pin weights, so the delay
// and look-ahead terms of the cost are zero; reading the weights as the constant 0 lets the
// compiler drop those terms (and the capacitances that only they use) -- the same costs, bit
// for bit, for such a tile.

template <int NAMAX, bool ZW = false>
struct LdsState {
    int64_t *F_;
    int32_t *S_;
    uint8_t *bt_, *sel_;
    const int16_t *chp, *chl;
    const uint4 *rec;     // len, lam, segw | dir << 16 | flags << 24, cpin
    const uint16_t *pinw_;
    __device__ int nch(int32_t s) const { return chp[s + 1] - chp[s]; }
    __device__ int32_t ch_state(int32_t s, int q) const { return chl[chp[s] + q]; }
    __device__ int64_t &F(int32_t s, int j) const { return F_[s * NAMAX + j]; }
    __device__ int32_t &S(int32_t s, int j) const { return S_[s * NAMAX + j]; }
    __device__ uint8_t &bt(int32_t s, int j) const { return bt_[s * NAMAX + j]; }
    __device__ uint8_t &sel(int32_t s, int jp) const { return sel_[s * NAMAX + jp]; }
    __device__ NodeIn in(int32_t s) const
    {
        const uint4 r = rec[s];
        return NodeIn{(int32_t)r.x, ZW ? 0u : r.y, ZW ? 0u : (r.z & 0xffffu), (int)((r.z >> 16) & 1u),
                      (uint8_t)(r.z >> 24), (int32_t)r.w};
    }
    __device__ uint32_t pinw(int32_t s) const { return ZW ? 0u : (uint32_t)pinw_[s]; }
};

// The tile state with the current DP item's node header in registers: its child count and first
// child, and the first child's direction, so that the child's state can be read before its record.
template <class Base>
struct ItemState : Base {
    int32_t cur, c0, k, cdir;
    __device__ ItemState(const Base &b, int32_t u, uint32_t hd)
        : Base(b), cur(u), c0((int32_t)((hd >> 8) & 0xffu)), k((int32_t)((hd >> 16) & 0xffu)),
          cdir((int32_t)((hd >> 26) & 1u))
    {
    }
    __device__ int nch(int32_t s) const { return s == cur ? k : Base::nch(s); }
    __device__ int32_t ch_state(int32_t s, int q) const { return (s == cur && q == 0) ? c0 : Base::ch_state(s, q); }
    __device__ NodeIn in(int32_t s) const
    {
        NodeIn r = Base::in(s);
        if (k > 0 && s == c0) r.dir = cdir;
        return r;
    }
};

// LDS layout of one tile (byte offsets), shared by the host launch and the kernel.  The
// congestion table (L x 2 x 64 int32) follows at LUT; the launch sizes it by L.
template <int NAMAX, int CAP>
struct Tile {
    static constexpr int nkey = 4 * CAP + 4;                       // (height, child class) buckets
    // F holds kappa_n(l) until the DP item (n, l) reads it and overwrites it with f
    static constexpr size_t F = 0;                                  // int64 [CAP][NAMAX]
    static constexpr size_t REC = F + (size_t)CAP * NAMAX * 8;     // uint4 [CAP] per-node inputs
    static constexpr size_t S = REC + (size_t)CAP * 16;            // int32 [CAP][NAMAX]
    static constexpr size_t GID = S + (size_t)CAP * NAMAX * 4;     // int32 [CAP]
    static constexpr size_t LEN = GID + (size_t)CAP * 4;           // int32 [CAP+1] prefix of segment lengths
    static constexpr size_t G0 = LEN + (size_t)(CAP + 1) * 4;      // int32 [CAP] in-plane position of the first edge
    static constexpr size_t KEYS = G0 + (size_t)CAP * 4;           // int32 [nkey] bucket starts
    static constexpr size_t BOOK = KEYS + (size_t)nkey * 4;         // int32 [kBook]
    static constexpr size_t PAR = BOOK + (size_t)kBook * 4;         // int16 [CAP]
    static constexpr size_t CHP = PAR + (size_t)CAP * 2;           // int16 [CAP+2]
    static constexpr size_t CHL = CHP + (size_t)(CAP + 2) * 2;     // int16 [CAP]
    static constexpr size_t ORD = CHL + (size_t)CAP * 2;           // uint32 [CAP] item header by order position
    static constexpr size_t KEY = ORD + (size_t)CAP * 4;           // int16 [CAP] bucket of each node
    static constexpr size_t PINW = KEY + (size_t)CAP * 2;          // uint16 [CAP]
    static constexpr size_t BT = PINW + (size_t)CAP * 2;           // uint8 [CAP][NAMAX] b << 4 | t
    static constexpr size_t SEL = BT + (size_t)CAP * NAMAX;        // uint8 [CAP][NAMAX]
    static constexpr size_t ENT = SEL + (size_t)CAP * NAMAX;       // uint8 [CAP] entering-layer index
    static constexpr size_t FLD = ENT + (size_t)CAP;               // uint8 [CAP] flags | dir << 4
    static constexpr size_t PRV = FLD + (size_t)CAP;               // uint8 [CAP] previous layer (255: none)
    static constexpr size_t NEWL = PRV + (size_t)CAP;              // uint8 [CAP] new layer of a moved segment, else 255
    static constexpr size_t SMAP = NEWL + (size_t)CAP;             // uint8 [CAP * NAMAX] GCell step -> segment
    static constexpr size_t LUT = (SMAP + (size_t)CAP * NAMAX + 15) & ~(size_t)15;
    static size_t bytes(int L) { return LUT + (size_t)L * 2 * kNDelta * 4; }
};

struct BArgs {
    const int32_t *tier_nets;
    const int32_t *tier_off;    // [2*T+1]: bucket starts; batch t spans [off[2t], off[2t+2])
    int32_t tier, tier_hi;      // batches tier..tier_hi run together (tier_hi > tier: merged small batches)
    int32_t *ctr;               // work-queue counter of this (round, batch group)
    const int32_t *cl_start;    // claim starts (positions in tier_nets); batch t's claims from cl_off[t]
    const int32_t *cl_off;
    const int32_t *height;
    const int32_t *net_big, *bn_order, *bn_lvl, *bn_lvl_off, *bn_nlev;
    int4 *bn_rec;               // per bn_order position: the node's record (k_big_records)
    const uint8_t *net_zw;      // per net: all timing weights zero
    const uint4 *nrec;          // static node records (see la_batch::nrec)
    const uint2 *dynrec;        // this call's node weights: look-ahead, segment | pin << 16
    const int4 *cnet;           // per sorted net position: first node, nodes, first child entry, zero flag
    const int32_t *ch;          // child entries (global node ids)
    uint8_t *cur, *vlo, *vhi, *out_layers;
    int has_prev;
    ChangeList cl;
    int32_t *Dw;                // demand moves of the small nets go straight here; NULL: to cl
};

// In-place inclusive prefix sum of x[0, n) by the whole workgroup (wave scans, then the
// wave totals); tmp holds one int per wavefront.  Ends with a barrier.
__device__ __forceinline__ void block_scan(int32_t *x, int32_t n, int32_t *tmp)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t carry = 0;
    for (int32_t c0 = 0; c0 < n; c0 += blockDim.x) {
        const int32_t i = c0 + threadIdx.x;
        int32_t v = i < n ? x[i] : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(v, d);
            if (lane >= d) v += y;
        }
        if (lane == 63) tmp[w] = v;
        __syncthreads();
        int32_t pre = carry, tot = carry;
        for (int q = 0; q < nw; ++q) {
            const int32_t t = tmp[q];
            if (q < w) pre += t;
            tot += t;
        }
        if (i < n) x[i] = v + pre;
        carry = tot;
        __syncthreads();
    }
}

template <int NAMAX, int CAP>
__global__ void __launch_bounds__(kThreads, NAMAX > 6 || CAP > 192 ? 3 : 4) k_batched_dp(DPArgs a, BArgs ba)
{
    using TL = Tile<NAMAX, CAP>;
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ LayerTab tb;
    __shared__ int32_t scan_tmp[kThreads / 64];
    load_tab(a.tab, tb);
    int64_t *F = (int64_t *)(smem + TL::F);
    int64_t *kap = F;   // congestion costs, replaced by f item by item
    int32_t *S = (int32_t *)(smem + TL::S);
    int32_t *gid = (int32_t *)(smem + TL::GID);
    int32_t *lenp = (int32_t *)(smem + TL::LEN);
    int32_t *g0a = (int32_t *)(smem + TL::G0);
    uint4 *rec = (uint4 *)(smem + TL::REC);
    int32_t *kst = (int32_t *)(smem + TL::KEYS);
    int32_t *book = (int32_t *)(smem + TL::BOOK);
    int16_t *par = (int16_t *)(smem + TL::PAR);
    int16_t *chp = (int16_t *)(smem + TL::CHP);
    int16_t *chl = (int16_t *)(smem + TL::CHL);
    uint32_t *hdr = (uint32_t *)(smem + TL::ORD);
    int16_t *key = (int16_t *)(smem + TL::KEY);
    uint16_t *pinw = (uint16_t *)(smem + TL::PINW);
    uint8_t *bt = smem + TL::BT;
    uint8_t *sel = smem + TL::SEL;
    uint8_t *newl = smem + TL::NEWL;
    uint8_t *smap = smem + TL::SMAP;
    uint8_t *ent = smem + TL::ENT;
    uint8_t *fld = smem + TL::FLD;
    uint8_t *prv = smem + TL::PRV;
    int32_t *lut = (int32_t *)(smem + TL::LUT);

    // bookkeeping: [0] claim index, [1] #tiles, [2] max height of the tile; per tile: first
    // and end claim index, node count, all-zero-weight flag; per claimed net: node count, first
    // global node, first global child entry, tile-local node base and child base, zero-weight flag
    constexpr int Q = kClaimNets;
    int32_t *s_base = book, *s_nsub = book + 1, *s_maxlev = book + 2;
    int32_t *s_sub0 = book + 8, *s_sub1 = book + 8 + Q, *s_tn = book + 8 + 2 * Q;
    int32_t *s_nn = book + 8 + 3 * Q, *s_g0 = book + 8 + 4 * Q, *s_c0 = book + 8 + 5 * Q;
    int32_t *s_lb = book + 8 + 6 * Q, *s_cb = book + 8 + 7 * Q;
    int32_t *s_zn = book + 8 + 8 * Q, *s_tz = book + 8 + 9 * Q;
    static_assert(kBook >= 8 + 10 * kClaimNets && kClaimNets <= kThreads, "bookkeeping layout");
    static_assert(kClaimUnitsMax / (1 + kNetUnits) + 1 <= kClaimNets, "nets per claim");

    const int L = tb.L;
    for (int i = threadIdx.x; i < L * 2 * kNDelta; i += blockDim.x) lut[i] = a.w.lut[i];

    LdsState<NAMAX> st{F, S, bt, sel, chp, chl, rec, pinw};
    LdsState<NAMAX, true> stz{F, S, bt, sel, chp, chl, rec, pinw};
    // the claims of the small nets of batches tier..tier_hi (big nets run in k_batched_big);
    // batch t lists n_t claims and an end slot from cl_off[t]
    auto nclaims = [&](int32_t t) { return max(0, ba.cl_off[t + 1] - ba.cl_off[t] - 1); };
    int32_t ncl = 0;
    for (int32_t t = ba.tier; t <= ba.tier_hi; ++t) ncl += nclaims(t);

    for (;;) {
        if (threadIdx.x == 0) *s_base = atomicAdd(ba.ctr, 1);
        __syncthreads();
        int32_t c = *s_base;
        if (c >= ncl) break;
        int32_t t = ba.tier;
        while (c >= nclaims(t)) c -= nclaims(t++);
        const int32_t coff = ba.cl_off[t];
        // at most kClaimNets by construction (each net counts >= 1 + kNetUnits units)
        const int32_t p0 = ba.cl_start[coff + c], nclaim = min(ba.cl_start[coff + c + 1] - p0, kClaimNets);
        if (threadIdx.x < nclaim) {
            const int4 cr = ba.cnet[p0 + threadIdx.x];
            s_g0[threadIdx.x] = cr.x;
            s_nn[threadIdx.x] = cr.y;
            s_c0[threadIdx.x] = cr.z;
            s_zn[threadIdx.x] = (a.w.w_d == 0 || cr.w) ? 1 : 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // split the claimed nets (each of at most CAP nodes) into tiles of at most CAP;
            // a claim can be empty (a net longer than one claim's units spans several)
            int32_t ns = 0, nodes = 0, kids = 0;
            for (int32_t i = 0; i < nclaim; ++i) {
                const int32_t n = s_nn[i];
                if (i == 0 || nodes + n > CAP) {
                    if (i) {
                        s_sub1[ns - 1] = i;
                        s_tn[ns - 1] = nodes;
                    }
                    s_tz[ns] = 1;
                    s_sub0[ns++] = i;
                    nodes = 0;
                    kids = 0;
                }
                s_tz[ns - 1] &= s_zn[i];
                s_lb[i] = nodes;
                s_cb[i] = kids;
                nodes += n;
                kids += n - 1;
            }
            if (ns > 0) {
                s_sub1[ns - 1] = nclaim;
                s_tn[ns - 1] = nodes;
            }
            *s_nsub = ns;
        }
        __syncthreads();
        const int32_t nsub = *s_nsub;
        for (int32_t sb = 0; sb < nsub; ++sb) {
            const int32_t i0 = s_sub0[sb], i1 = s_sub1[sb], nn = s_tn[sb];
            const bool zt = s_tz[sb] != 0;   // every net of the tile has zero timing weights
            // ---- stage the tile: topology, inputs, (height, class) counts ----------------
            for (int32_t i = threadIdx.x; i < TL::nkey; i += blockDim.x) kst[i] = 0;
            if (threadIdx.x == 0) {
                *s_maxlev = 0;
                lenp[0] = 0;
                chp[nn] = (int16_t)(s_cb[i1 - 1] + s_nn[i1 - 1] - 1);
            }
            __syncthreads();
            // one pass over the tile's nodes and its child entries (both contiguous in HBM): a
            // node reads its static record, this call's weights and its previous layer; an
            // entry its child's global id
            const int32_t nent = nn - (i1 - i0);
            for (int32_t u = threadIdx.x; u < max(nn, nent); u += blockDim.x) {
                if (u < nent) {
                    int32_t lo_ = i0, hi_ = i1;   // the net of entry u: last k with s_cb[k] <= u
                    while (hi_ - lo_ > 1) {
                        const int32_t mid = (lo_ + hi_) >> 1;
                        if (s_cb[mid] <= u) lo_ = mid;
                        else hi_ = mid;
                    }
                    chl[u] = (int16_t)(ba.ch[s_c0[lo_] + (u - s_cb[lo_])] - s_g0[lo_] + s_lb[lo_]);
                }
                if (u >= nn) continue;
                int32_t lo_ = i0, hi_ = i1;      // the net of u: last k with s_lb[k] <= u
                while (hi_ - lo_ > 1) {
                    const int32_t mid = (lo_ + hi_) >> 1;
                    if (s_lb[mid] <= u) lo_ = mid;
                    else hi_ = mid;
                }
                const int32_t g0 = s_g0[lo_], lb = s_lb[lo_];
                const int32_t g = g0 + (u - lb);
                gid[u] = g;
                const uint4 nr = ba.nrec[g];
                // a zero-weight tile reads its weights as 0 (LdsState<.., true>) and skips the loads
                const uint2 dw = zt ? make_uint2(0u, 0u) : ba.dynrec[g];
                const int pv = a.w.self_excl ? a.prev[g] : 255;
                const uint32_t po = nr.y >> 16;
                const bool isroot = po == 0xffffu;
                par[u] = (int16_t)(isroot ? -1 : (int32_t)po + lb);
                const int32_t kk = (int32_t)(nr.w & 0xffu);
                chp[u] = (int16_t)(s_cb[lo_] + (int32_t)(nr.w >> 24));
                const int32_t h = (int32_t)((nr.w >> 16) & 0xffu);
                // classes inside a level: 0 leaves, 1 one child, 2 a root with one child (one
                // state), 3 two or more children
                const int32_t bk = 4 * h + (kk >= 2 ? 3 : (kk == 1 && isroot ? 2 : kk));
                key[u] = (int16_t)bk;
                atomicAdd(&kst[bk + 1], 1);
                atomicMax(s_maxlev, h);
                const int32_t len = (int32_t)(nr.y & 0xffffu);
                const uint32_t fd = (nr.w >> 8) & 0xffu;
                const uint32_t fl = fd & 15u, dr = fd >> 4;
                lenp[u + 1] = len;
                g0a[u] = (int32_t)nr.x;
                fld[u] = (uint8_t)fd;
                rec[u] = make_uint4((uint32_t)len, dw.x, (dw.y & 0xffffu) | (dr << 16) | (fl << 24), nr.z);
                pinw[u] = (uint16_t)(dw.y >> 16);
                prv[u] = (uint8_t)pv;
#pragma unroll
                for (int jj = 0; jj < NAMAX; ++jj) kap[u * NAMAX + jj] = 0;
            }
            __syncthreads();
            const int32_t maxlev = *s_maxlev;
            block_scan(kst, 4 * maxlev + 5, scan_tmp);   // bucket starts
            block_scan(lenp, nn + 1, scan_tmp);          // lenp[u]: first GCell step of u
            // (height, class) order; kst[q] ends as the end of bucket q = start of q+1.  The
            // step -> segment map serves the gather and the demand moves.
            const int32_t steps = lenp[nn];
            static_assert(CAP <= 256, "the step map holds tile-local node ids in one byte");
            const bool mapped = steps <= CAP * NAMAX;
            // the segment of GCell step pidx: the last u with lenp[u] <= pidx
            auto seg_of = [&](int32_t pidx) -> int32_t {
                if (mapped) return smap[pidx];
                int32_t lo_ = 0, hi_ = nn;
                while (hi_ - lo_ > 1) {
                    const int32_t mid = (lo_ + hi_) >> 1;
                    if (lenp[mid] <= pidx) lo_ = mid;
                    else hi_ = mid;
                }
                return lo_;
            };
            for (int32_t u = threadIdx.x; u < nn; u += blockDim.x) {
                {
                    // the item header of u at its (height, class) position: node, first child,
                    // child count, root flag, direction, the first child's direction
                    const int32_t kq = chp[u + 1] - chp[u];
                    const int32_t c0 = kq > 0 ? chl[chp[u]] : 0;
                    hdr[atomicAdd(&kst[key[u]], 1)] =
                        (uint32_t)u | (uint32_t)c0 << 8 | (uint32_t)min(kq, 255) << 16 | (par[u] < 0 ? 1u << 24 : 0u) |
                        (uint32_t)(fld[u] >> 4) << 25 | (kq > 0 ? (uint32_t)(fld[c0] >> 4) << 26 : 0u);
                }
                if (mapped)
                    for (int32_t q = lenp[u]; q < lenp[u + 1]; ++q) smap[q] = (uint8_t)u;
            }
            if (mapped) __syncthreads();
            // congestion costs: one thread per GCell edge of the tile's segments, every
            // routable layer of the segment's direction at once
            for (int32_t pidx = threadIdx.x; pidx < steps; pidx += blockDim.x) {
                const int32_t u = seg_of(pidx);
                const int d = fld[u] >> 4;
                const int32_t q = g0a[u] + (pidx - lenp[u]);   // in-plane position of this edge
                const int self = prv[u];
                const int na = tb.nA[d];
                // the edge's record: its routable layers in pairs (8-byte aligned; a record of
                // odd length ends in a padding word)
                const int32_t g = route_index(tb, d, 0, q);
                const int2 *dr = (const int2 *)(a.D + g), *hr = (const int2 *)(a.H + g);
                const uint16_t *cr = (const uint16_t *)(a.caps + g);
#pragma unroll
                for (int jp = 0; jp < NAMAX; jp += 2) {
                    if (jp < na) {
                        const int2 dv = dr[jp / 2], hv = hr[jp / 2];
                        const uint32_t cv = cr[jp / 2];
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2) {
                            const int jj = jp + h2;
                            if (jj < na) {
                                const int l = tb.lay[d][jj];
                                const int32_t cap = (int32_t)((cv >> (8 * h2)) & 0xffu);
                                int32_t dd = (h2 ? dv.y : dv.x) - (self == l ? 1 : 0) - cap;
                                dd = dd < kDeltaMin ? kDeltaMin
                                                    : (dd > kDeltaMin + kNDelta - 1 ? kDeltaMin + kNDelta - 1 : dd);
                                const int64_t v = (int64_t)lut[(l * 2 + (cap > 0 ? 0 : 1)) * kNDelta + dd - kDeltaMin] +
                                                  (int64_t)(h2 ? hv.y : hv.x);
                                atomicAdd((unsigned long long *)&kap[u * NAMAX + jj], (unsigned long long)v);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // ---- DP bottom-up, one height level at a time ----------------------------------
            // A level of at most kThreads / kGroup items (tall trees) is bound by one item's
            // latency: it takes a group of kGroup lanes per item (node, entering layer), items
            // with one to three children lane-parallel, the others on the group's first lane.
            // Larger levels take one lane per item, except that items of nodes with two or more
            // children (the slowest, and few) take a group each; the group items start and end
            // on wavefront boundaries, so no wavefront runs both code paths.
            for (int32_t h = 0; h <= maxlev; ++h) {
                const int32_t lb = h == 0 ? 0 : kst[4 * h - 1], le = kst[4 * h + 3];
                const int32_t items = (le - lb) * NAMAX;
                // one-lane items first: NAMAX per node of classes 0-1, one per root of class 2 (its
                // single state), and NAMAX per node of class 3 when the via weight is zero; padded
                // to a wavefront boundary; then, with a positive via weight, group items of kGroup
                // lanes for class 3 (every item of a short level goes to a group)
                int32_t c2b = lb, nA1 = 0, nR = 0, nA = 0, pA = 0, total = items * kGroup;
                const int32_t c1e = kst[4 * h + 1], c2e = kst[4 * h + 2];
                if (items > kThreads / kGroup) {
                    nA1 = (c1e - lb) * NAMAX;
                    nR = c2e - c1e;
                    c2b = a.w.w_via > 0 ? c2e : le;
                    nA = nA1 + nR + (c2b - c2e) * NAMAX;
                    pA = (nA + 63) & ~63;
                    total = pA + (le - c2b) * NAMAX * kGroup;
                }
                for (int32_t it = threadIdx.x; it < total; it += blockDim.x) {
                    int32_t pos;
                    int j, sub = -1;
                    if (it < pA) {
                        if (it >= nA) continue;
                        if (it < nA1) {
                            pos = lb + it / NAMAX;
                            j = it % NAMAX;
                        } else if (it < nA1 + nR) {
                            pos = c1e + (it - nA1);
                            j = 0;
                        } else {
                            const int32_t r = it - nA1 - nR;
                            pos = c2e + r / NAMAX;
                            j = r % NAMAX;
                        }
                    } else {
                        const int32_t r = it - pA;
                        const int32_t gi = r / kGroup;
                        sub = r % kGroup;
                        pos = c2b + gi / NAMAX;
                        j = gi % NAMAX;
                    }
                    const uint32_t hd = hdr[pos];
                    const int32_t u = (int32_t)(hd & 0xffu);
                    const bool root = (hd >> 24) & 1u;
                    int l;
                    if (root) {
                        if (j != 0) continue;
                        l = 0;
                    } else {
                        const int d = (hd >> 25) & 1u;
                        if (j >= tb.nA[d]) continue;
                        l = tb.lay[d][j];
                    }
                    const int64_t kp = root ? 0 : kap[u * NAMAX + j];
                    const int k = (int)((hd >> 16) & 0xffu);
                    const ItemState<LdsState<NAMAX>> ist(st, u, hd);
                    const ItemState<LdsState<NAMAX, true>> istz(stz, u, hd);
                    // group items with one to three children are lane-parallel; the others run
                    // on one lane (the group's first)
                    if (sub >= 0 && a.w.w_via > 0 && k >= 1 && k <= 3) {
                        if (zt)
                            dp_group<ItemState<LdsState<NAMAX, true>>, NAMAX>(a, tb, istz, u, l, j, root, kp, sub);
                        else
                            dp_group<ItemState<LdsState<NAMAX>>, NAMAX>(a, tb, ist, u, l, j, root, kp, sub);
                    } else if (sub <= 0) {   // no child count 2..3 here while the via weight is positive
                        if (zt)
                            dp_node<ItemState<LdsState<NAMAX, true>>, NAMAX, true, false>(a, tb, istz, u, l, j, root,
                                                                                          kp);
                        else
                            dp_node<ItemState<LdsState<NAMAX>>, NAMAX, true, false>(a, tb, ist, u, l, j, root, kp);
                    }
                }
                __syncthreads();
            }
            // ---- trace-back top-down: entering-layer indices, in LDS -------------------------
            for (int32_t h = maxlev; h >= 0; --h) {
                const int32_t lb = h == 0 ? 0 : kst[4 * h - 1], le = kst[4 * h + 3];
                for (int32_t it = lb + threadIdx.x; it < le; it += blockDim.x) {
                    const int32_t u = (int32_t)(hdr[it] & 0xffu);
                    const int32_t pu = par[u];
                    int ln;
                    ent[u] = (uint8_t)trace_choice(tb, st, u, (pu < 0 || par[pu] < 0) ? 0 : ent[pu], pu < 0, &ln);
                }
                __syncthreads();
            }
            // ---- layers, via spans and demand moves of the tile, in node order --------------
            for (int32_t u0 = 0; u0 < nn; u0 += blockDim.x) {
                const int32_t u = u0 + threadIdx.x;
                bool changed = false;
                uint8_t old_l = 0;
                int ln = 0;
                int32_t n = 0;
                if (u < nn) {
                    n = gid[u];
                    const int32_t pu = par[u];
                    const int j = trace_choice(tb, st, u, (pu < 0 || par[pu] < 0) ? 0 : ent[pu], pu < 0, &ln);
                    // the previous layer was staged (prv) when this round has one
                    trace_write(st, u, n, j, ln, pu < 0, ba.cur, ba.vlo, ba.vhi, ba.out_layers, ba.has_prev, &changed,
                                &old_l, ba.has_prev ? prv[u] : 0);
                }
                if (ba.Dw) {
                    if (u < nn) newl[u] = changed ? (uint8_t)ln : (uint8_t)255;
                } else {
                    append_change(ba.cl, changed, n, old_l, (uint8_t)ln);
                }
            }
            if (ba.Dw) {
                // demand moves, one lane per GCell edge of the moved segments (the DP of this
                // batch reads the other demand buffer); the previous layer is prv, if any
                __syncthreads();
                for (int32_t pidx = threadIdx.x; pidx < steps; pidx += blockDim.x) {
                    const int32_t u = seg_of(pidx);
                    const int nl = newl[u];
                    if (nl == 255) continue;
                    const int32_t q = g0a[u] + (pidx - lenp[u]);
                    const int ol = ba.has_prev ? prv[u] : 255;
                    if (ol != 255) atomicAdd(&ba.Dw[grid_index(tb, ol, q)], -1);
                    atomicAdd(&ba.Dw[grid_index(tb, nl, q)], 1);
                }
            }
            __syncthreads();   // the next tile restages the LDS this pass reads
        }
        __syncthreads();
    }
}

// Per position of a big net's level order, the node's record for the level walk: node id,
// parent, child count | direction << 8 | flags << 16, length; its first three children and pin
// load; this call's look-ahead coefficient and segment weight.  One read then gives a DP item
// its node's inputs and children, which otherwise take three dependent reads per level.
__global__ void __launch_bounds__(256) k_big_records(DPArgs a, BArgs ba)
{
    const int32_t off0 = ba.tier_off[ba.tier * kNB], cnt = ba.tier_off[ba.tier * kNB + 1] - off0;
    for (int32_t i = blockIdx.y; i < cnt; i += gridDim.y) {
        const int32_t q = ba.net_big[ba.tier_nets[off0 + i]];
        const int32_t lo = ba.bn_lvl_off[q];
        const int32_t p0 = ba.bn_lvl[lo], p1 = ba.bn_lvl[lo + ba.bn_nlev[q]];
        for (int32_t p = p0 + blockIdx.x * blockDim.x + threadIdx.x; p < p1; p += gridDim.x * blockDim.x) {
            const int32_t n = ba.bn_order[p];
            const int32_t c0 = a.T.ch_ptr[n], k = a.T.ch_ptr[n + 1] - c0;
            int4 *r = ba.bn_rec + 3 * (int64_t)p;
            r[0] = make_int4(n, a.T.parent[n], k | (int32_t)a.T.dir[n] << 8 | (int32_t)a.T.flags[n] << 16, a.T.len[n]);
            r[1] = make_int4(k > 0 ? a.T.ch[c0] : -1, k > 1 ? a.T.ch[c0 + 1] : -1, k > 2 ? a.T.ch[c0 + 2] : -1,
                             a.T.cpin[n]);
            r[2] = make_int4(a.w.lam[n], (int32_t)a.w.seg_w[n], 0, 0);
        }
    }
}

// HBM state of a big net with the current node's record in registers: its inputs, child count
// and first three children come from the record, everything else from HBM as in GlobalState.
struct BigState : GlobalState {
    int32_t cur;
    int4 r0, r1, r2;
    __device__ BigState(const DPArgs &a_, const int4 *rec) : GlobalState(a_), r0(rec[0]), r1(rec[1]), r2(rec[2])
    {
        cur = r0.x;
    }
    __device__ int nch(int32_t s) const { return s == cur ? (r0.z & 0xff) : GlobalState::nch(s); }
    __device__ int32_t ch_state(int32_t s, int q) const
    {
        if (s == cur && q < 3) return q == 0 ? r1.x : (q == 1 ? r1.y : r1.z);
        return GlobalState::ch_state(s, q);
    }
    __device__ NodeIn in(int32_t s) const
    {
        if (s == cur)
            return NodeIn{r0.w, (uint32_t)r2.x, (uint16_t)r2.y, (uint8_t)((r0.z >> 8) & 0xff),
                          (uint8_t)((r0.z >> 16) & 0xff), r1.w};
        return GlobalState::in(s);
    }
};

// Congestion costs kappa_n(l) of every node and candidate layer of the batch's nets larger
// than one LDS tile, into their slots of the HBM state array F (each DP item of k_batched_big
// reads its slot before it overwrites it with f): the level walk then does no gather.  Workgroup
// row y takes big net y; a wavefront takes a node, its lanes the segment's GCell edges (every
// candidate layer at once: a record holds them side by side), summed across the wavefront.
template <int NAMAX>
__global__ void __launch_bounds__(256) k_kappa_big(DPArgs a, BArgs ba)
{
    __shared__ LayerTab tb;
    load_tab(a.tab, tb);
    const int lane = threadIdx.x & 63;
    const int32_t wv = blockIdx.x * 4 + (threadIdx.x >> 6), nwv = gridDim.x * 4;
    const int32_t off0 = ba.tier_off[ba.tier * kNB], cnt = ba.tier_off[ba.tier * kNB + 1] - off0;
    for (int32_t i = blockIdx.y; i < cnt; i += gridDim.y) {
        const int32_t net = ba.tier_nets[off0 + i];
        const int32_t n0 = a.T.net_ptr[net], n1 = a.T.net_ptr[net + 1];
        for (int32_t n = n0 + wv; n < n1; n += nwv) {
            const int d = a.T.dir[n];
            const int na = tb.nA[d];
            const bool root = a.T.parent[n] < 0;
            const int32_t len = root ? 0 : a.T.len[n];
            const int self = a.w.self_excl ? a.prev[n] : 255;
            const int32_t step = tb.nAp[d];
            const int32_t g0 = route_index(tb, d, 0, a.T.g0[n]);
            int64_t acc[NAMAX];
#pragma unroll
            for (int j = 0; j < NAMAX; ++j) acc[j] = 0;
            for (int32_t k = lane; k < len; k += 64) {
                const int32_t g = g0 + k * step;
#pragma unroll
                for (int j = 0; j < NAMAX; ++j) {
                    if (j < na) {
                        const int l = tb.lay[d][j];
                        const int32_t cap = a.caps[g + j];
                        int32_t dd = a.D[g + j] - (self == l ? 1 : 0) - cap;
                        dd = dd < kDeltaMin ? kDeltaMin : (dd > kDeltaMin + kNDelta - 1 ? kDeltaMin + kNDelta - 1 : dd);
                        acc[j] += a.w.lut[(l * 2 + (cap > 0 ? 0 : 1)) * kNDelta + dd - kDeltaMin] + (int64_t)a.H[g + j];
                    }
                }
            }
            int64_t mine = 0;
#pragma unroll
            for (int j = 0; j < NAMAX; ++j) {
                int64_t v = acc[j];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
                if (lane == j) mine = v;
            }
            if (lane < a.NA) a.F[(int64_t)n * a.NA + lane] = lane < na ? mine : 0;
        }
    }
}

// Nets larger than one LDS tile: one workgroup per net, DP state in HBM, the net's own
// height levels walked with workgroup barriers.
template <int NAMAX>
__global__ void __launch_bounds__(kThreads) k_batched_big(DPArgs a, BArgs ba)
{
    __shared__ LayerTab tb;
    load_tab(a.tab, tb);
    GlobalState gst(a);
    const int32_t off0 = ba.tier_off[ba.tier * kNB], cnt = ba.tier_off[ba.tier * kNB + 1] - off0;
    for (int32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const int32_t net = ba.tier_nets[off0 + i];
        const int32_t q = ba.net_big[net];
        const int32_t lo = ba.bn_lvl_off[q], nl = ba.bn_nlev[q];
        for (int32_t h = 0; h < nl; ++h) {
            const int32_t b0 = ba.bn_lvl[lo + h], c = ba.bn_lvl[lo + h + 1] - b0;
            // most levels of a tall tree hold a few nodes: then each item takes a group of
            // kGroup lanes (one to three children lane-parallel, others on the first lane)
            const bool grp = a.w.w_via > 0 && c * NAMAX <= kThreads / kGroup;
            const int32_t span = grp ? c * NAMAX * kGroup : c * NAMAX;
            for (int32_t it = threadIdx.x; it < span; it += blockDim.x) {
                const int32_t gi = grp ? it / kGroup : it;
                const int sub = grp ? it % kGroup : 0;
                // the node's record (k_big_records): inputs and first children in one read
                const BigState bst(a, ba.bn_rec + 3 * (int64_t)(b0 + gi / NAMAX));
                const int32_t n = bst.cur;
                const int j = gi % NAMAX;
                const bool root = bst.r0.y < 0;
                int l;
                if (root) {
                    if (j != 0) continue;
                    l = 0;
                } else {
                    const int d = (bst.r0.z >> 8) & 0xff;
                    if (j >= tb.nA[d]) continue;
                    l = tb.lay[d][j];
                }
                // the congestion cost, from k_kappa_big
                const int64_t kp = root ? 0 : a.F[(int64_t)n * a.NA + j];
                if (!grp) {
                    dp_node<BigState, NAMAX>(a, tb, bst, n, l, j, root, kp);
                } else {
                    const int k = bst.nch(n);
                    if (k >= 1 && k <= 3)
                        dp_group<BigState, NAMAX>(a, tb, bst, n, l, j, root, kp, sub);
                    else if (sub == 0)
                        dp_node<BigState, NAMAX, false>(a, tb, bst, n, l, j, root, kp);
                }
            }
            __syncthreads();
        }
        for (int32_t h = nl - 1; h >= 0; --h) {
            const int32_t b0 = ba.bn_lvl[lo + h], c = ba.bn_lvl[lo + h + 1] - b0;
            for (int32_t it0 = 0; it0 < c; it0 += blockDim.x) {
                const int32_t it = it0 + threadIdx.x;
                bool changed = false;
                uint8_t old_l = 0;
                int ln = 0;
                int32_t n = 0;
                if (it < c) {
                    const int4 r0 = ba.bn_rec[3 * (int64_t)(b0 + it)];
                    n = r0.x;
                    const int32_t pp = r0.y;
                    const int jp = (pp < 0 || a.T.parent[pp] < 0) ? 0 : tb.jidx[ba.cur[pp] & (kMaxL - 1)];
                    trace_node(tb, gst, n, n, jp, pp < 0, ba.cur, ba.vlo, ba.vhi, ba.out_layers, ba.has_prev, &ln,
                               &changed, &old_l);
                }
                append_change(ba.cl, changed, n, old_l, (uint8_t)ln);
            }
            __syncthreads();
        }
    }
}

// ---- batch (tier) partition -----------------------------------------------------------
// Bucket of a net: its batch's big nets first, then its small nets from the tallest
// tree to the shortest (height classes 0..kHB-1, taller trees share the last class), so
// a workgroup's tile holds trees of similar height and walks few levels, and the work
// queue hands out the long trees first.
__device__ __forceinline__ int32_t net_bucket(int t, bool big, bool zw, int32_t h)
{
    return t * kNB + (big ? 0 : 1 + (zw ? kHB : 0) + (kHB - 1 - (h < kHB - 1 ? h : kHB - 1)));
}

// zw[net] = 1 when the net's segment weights and look-ahead coefficients (below its root) and its
// sinks' pin weights are all zero: the DP of such a net has no delay or look-ahead term
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_net_zero_weights(TreeDev T, const uint16_t *seg_w, const uint16_t *pin_w, const int32_t *lam,
                                   uint8_t *zw, uint2 *dynrec)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < T.nodes; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sid = T.sink_id[v];
        const uint32_t pw = sid >= 0 ? pin_w[sid] : 0u, sw = seg_w[v];
        const int32_t lm = lam[v];
        bool nz = pw != 0;
        if (T.parent[v] >= 0) nz = nz || sw != 0 || lm != 0;
        if (nz) zw[T.net[v]] = 0;
        // the weights a tile stages for this node, in one 8-byte record
        dynrec[v] = make_uint2((uint32_t)lm, sw | (pw << 16));
    }
}

constexpr int kLdsNB = 2048;   // buckets counted in LDS; more go straight to HBM counters
constexpr int kPartGroups = 512;   // workgroups of the partition: each adds its bucket counts to HBM once

__global__ void k_tier_count(const int32_t *tier, int32_t ntier, int64_t nets, int32_t cap,
                             const uint8_t *zw, const int32_t *net_ptr, const int32_t *height, int32_t *cnt,
                             int32_t *bad)
{
    __shared__ int32_t hist[kLdsNB];
    const int32_t nb = ntier * kNB;
    const bool local = nb <= kLdsNB;
    if (local)
        for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nets; i += (int64_t)gridDim.x * blockDim.x) {
        const int t = tier ? tier[i] : 0;
        if (t < 0 || t >= ntier) {
            atomicAdd(bad, 1);
            continue;
        }
        const int32_t q = net_bucket(t, net_ptr[i + 1] - net_ptr[i] > cap, zw[i] != 0, height[net_ptr[i]]);
        atomicAdd(local ? &hist[q] : &cnt[q], 1);
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            if (hist[i]) atomicAdd(&cnt[i], hist[i]);
}

// off[0..nb] = exclusive prefix of cnt, cur = off; the claim counters start at zero
__global__ void k_tier_offsets(const int32_t *cnt, int32_t nb, int32_t *off, int32_t *cur, int32_t *claim,
                               int32_t nclaim)
{
    __shared__ int32_t tmp[1024 / 64];
    for (int32_t i = threadIdx.x; i <= nb; i += blockDim.x) off[i] = i == 0 ? 0 : cnt[i - 1];
    __syncthreads();
    block_scan(off, nb + 1, tmp);
    for (int32_t i = threadIdx.x; i < nb; i += blockDim.x) cur[i] = off[i];
    for (int32_t i = threadIdx.x; i < nclaim; i += blockDim.x) claim[i] = 0;
}

__global__ void k_tier_scatter(const int32_t *tier, int32_t ntier, int64_t nets, int32_t cap,
                               const uint8_t *zw, const int32_t *net_ptr, const int32_t *height, int32_t *cur,
                               int32_t *out)
{
    __shared__ int32_t hist[kLdsNB];
    __shared__ int32_t base[kLdsNB];
    const int32_t nb = ntier * kNB;
    if (nb > kLdsNB) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nets;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int t = tier ? tier[i] : 0;
            if (t < 0 || t >= ntier) continue;
            out[atomicAdd(&cur[net_bucket(t, net_ptr[i + 1] - net_ptr[i] > cap, zw[i] != 0, height[net_ptr[i]])], 1)] =
                (int32_t)i;
        }
        return;
    }
    // a workgroup takes a contiguous range of nets: counts them per bucket, reserves each bucket's
    // span once (one global atomic per bucket and workgroup), then places them, in any order
    // inside a bucket
    const int64_t per = (nets + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < nets ? r0 + per : nets;
    auto bucket = [&](int64_t i) -> int32_t {
        const int t = tier ? tier[i] : 0;
        if (t < 0 || t >= ntier) return -1;
        return net_bucket(t, net_ptr[i + 1] - net_ptr[i] > cap, zw[i] != 0, height[net_ptr[i]]);
    };
    for (int i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const int32_t q = bucket(i);
        if (q >= 0) atomicAdd(&hist[q], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x)
        if (hist[k]) base[k] = atomicAdd(&cur[k], hist[k]);
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const int32_t q = bucket(i);
        if (q >= 0) out[atomicAdd(&base[q], 1)] = (int32_t)i;
    }
}

// ---- claims: slices of each batch's sorted small nets by units (nodes + kNetUnits) -------
// pre[0] = 0, pre[i + 1] = units of the net at sorted position i
// (and the record a claim reads per net position: first node, nodes, first child entry, zero flag)
// (positions at or after *listed, the end of the partitioned net list, hold no net: 0 units)
__global__ void k_claim_units(const int32_t *tier_nets, int64_t nets, const int32_t *listed, const int32_t *net_ptr,
                              const int32_t *ch_ptr, const uint8_t *zw, int32_t *pre, int4 *cnet)
{
    const int64_t n_listed = *listed;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nets; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == 0) pre[0] = 0;
        if (i >= n_listed) {
            pre[i + 1] = 0;
            continue;
        }
        const int32_t net = tier_nets[i];
        const int32_t n0 = net_ptr[net], nn = net_ptr[net + 1] - n0;
        pre[i + 1] = nn + kNetUnits;
        cnet[i] = make_int4(n0, nn, ch_ptr[n0], zw[net]);
        if (i == 0) pre[0] = 0;
    }
}

// inclusive scan of each 1024-element chunk in place; the chunk's total to blk[chunk]
__global__ void k_scan_chunks(int32_t *x, int64_t n, int32_t *blk)
{
    __shared__ int32_t tmp[1024 / 64];
    const int64_t c0 = (int64_t)blockIdx.x * 1024;
    const int32_t m = (int32_t)std::min<int64_t>(1024, n - c0);
    block_scan(x + c0, m, tmp);
    if (threadIdx.x == 0) blk[blockIdx.x] = x[c0 + m - 1];
}

// inclusive scan of the chunk totals (one workgroup)
__global__ void k_scan_totals(int32_t *blk, int32_t nblk)
{
    __shared__ int32_t tmp[1024 / 64];
    block_scan(blk, nblk, tmp);
}

__global__ void k_scan_add(int32_t *x, int64_t n, const int32_t *blk)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t chunk = i / 1024;
        if (chunk > 0) x[i] += blk[chunk - 1];
    }
}

// batch t gets n_t = ceil(its units / units) claims and one end slot, from cl_off[t]
__global__ void k_claim_offsets(const int32_t *tier_off, int32_t ntier, const int32_t *pre, int32_t units,
                                int32_t *cl_off)
{
    __shared__ int32_t tmp[1024 / 64];
    for (int t = threadIdx.x; t < ntier; t += blockDim.x) {
        const int32_t s0 = tier_off[t * kNB + 1], s1 = tier_off[(t + 1) * kNB];
        cl_off[t + 1] = s1 > s0 ? (pre[s1] - pre[s0] + units - 1) / units + 1 : 0;
    }
    if (threadIdx.x == 0) cl_off[0] = 0;
    __syncthreads();
    block_scan(cl_off + 1, ntier, tmp);
}

// claim c of batch t holds the small nets whose unit prefix, counted from the batch's first
// small net, lies in [c, c + 1) * units; slot n_t holds the batch's end
__global__ void k_claim_starts(const int32_t *tier_off, int32_t ntier, int64_t nets, const int32_t *pre,
                               int32_t units, const int32_t *cl_off, int32_t *cl_start)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nets; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = ntier;   // batch of position i: tier_off[t*kNB] <= i < tier_off[(t+1)*kNB]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (tier_off[mid * kNB] <= i) lo = mid;
            else hi = mid;
        }
        const int32_t t = lo;
        const int32_t s0 = tier_off[t * kNB + 1], s1 = tier_off[(t + 1) * kNB];
        if (i < s0 || i >= s1) continue;   // a big net (its own kernel)
        const int32_t base = cl_off[t], nt = cl_off[t + 1] - base - 1;
        const int32_t c = (pre[i] - pre[s0]) / units;
        const int32_t cp = i == s0 ? -1 : (pre[i - 1] - pre[s0]) / units;
        for (int32_t q = cp + 1; q <= c; ++q) cl_start[base + q] = (int32_t)i;
        if (i == s1 - 1)
            for (int32_t q = c + 1; q <= nt; ++q) cl_start[base + q] = s1;
    }
}

// dst = src over n ints, 16 bytes per access (both arrays 256-byte aligned)
__global__ void k_copy_i32(int32_t *__restrict__ dst, const int32_t *__restrict__ src, int64_t n)
{
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride)
        ((int4 *)dst)[i] = ((const int4 *)src)[i];
    for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ void k_zero_counts(int32_t *p, int32_t n)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

inline int grid1d(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

// workgroups of the tile kernel that fit the GPU at once (its LDS tile and registers)
template <int NAMAX, int CAP>
int occupancy_grid(int L)
{
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batched_dp<NAMAX, CAP>, kThreads,
                                                       Tile<NAMAX, CAP>::bytes(L));
    return std::max(1, cus) * std::max(1, per);
}

template <int NAMAX, int CAP>
la_status launch_tiles(la_batch *b, const DPArgs &a, const BArgs &ba, hipStream_t s)
{
    const int full = occupancy_grid<NAMAX, CAP>(b->tab.L);
    const int grid = b->tune.workgroups > 0 ? std::min(b->tune.workgroups, full) : full;
    auto kern = k_batched_dp<NAMAX, CAP>;
    const size_t lds = Tile<NAMAX, CAP>::bytes(b->tab.L);
    LA_TIMED(b, "k_batched_dp", s, hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, a, ba));
    return LA_OK;
}

la_status launch_batched(la_batch *b, const DPArgs &a, const BArgs &ba, int32_t nbig, int32_t nsmall, hipStream_t s)
{
    const int NA = b->NAmax, cap = b->tune.tile_nodes;
    // The big nets (a workgroup each, walking tall trees level by level) run beside the tile
    // kernel on a second stream, joined before the batch's commit: both read the demand map as
    // it was before the batch and append to one change list.
    const bool fork = nbig > 0 && nsmall > 0;
    hipStream_t sb = s;
    if (nbig > 0) {
        // the big nets' congestion costs first, on the whole GPU: launched beside the tile
        // kernel, whose persistent workgroups hold every slot, they would wait for it
        const int kx = (int)std::max<int64_t>(1, std::min<int64_t>((b->max_net_nodes + 3) / 4, 512));
        LA_TIMED(b, "k_big_records", s,
                 hipLaunchKernelGGL(k_big_records, dim3(kx, std::min(nbig, 4096)), dim3(256), 0, s, a, ba));
        auto kbig = NA <= 4 ? k_kappa_big<4> : (NA <= 6 ? k_kappa_big<6> : k_kappa_big<8>);
        LA_TIMED(b, "k_kappa_big", s,
                 hipLaunchKernelGGL(kbig, dim3(kx, std::min(nbig, 4096)), dim3(256), 0, s, a, ba));
    }
    if (fork) {
        LA_HIP(hipEventRecord(b->ev_fork, s));
        LA_HIP(hipStreamWaitEvent(b->side_stream, b->ev_fork, 0));
        sb = b->side_stream;
    }
    if (nbig > 0) {
        auto big = NA <= 4 ? k_batched_big<4> : (NA <= 6 ? k_batched_big<6> : k_batched_big<8>);
        LA_TIMED(b, "k_batched_big", sb,
                 hipLaunchKernelGGL(big, dim3(std::min(nbig, 4096)), dim3(kThreads), 0, sb, a, ba));
    }
    if (nsmall > 0) {
        la_status st = LA_OK;
        if (NA <= 4) st = launch_tiles<4, kCap>(b, a, ba, s);
        else if (NA <= 6)
            st = cap == 128 ? launch_tiles<6, 128>(b, a, ba, s)
                            : (cap == 256 ? launch_tiles<6, 256>(b, a, ba, s) : launch_tiles<6, kCap>(b, a, ba, s));
        else st = launch_tiles<8, kCap>(b, a, ba, s);
        if (st != LA_OK) return st;
    }
    if (fork) {
        LA_HIP(hipEventRecord(b->ev_join, sb));
        LA_HIP(hipStreamWaitEvent(s, b->ev_join, 0));
    }
    LA_HIP(hipGetLastError());
    return LA_OK;
}

// small nets of batch t in the partition counts
int32_t small_nets(const std::vector<int32_t> &cnt, int32_t t)
{
    int32_t n = 0;
    for (int q = 1; q < kNB; ++q) n += cnt[t * kNB + q];
    return n;
}

// R rounds over the batches onto stream s: per batch the persistent DP kernels and the
// commit of the changed segments, then the history update of the round.  A batch with many
// small nets commits them from its DP kernel into a copy of the demand map (its DP reads the
// map as it was before the batch); the copy then becomes the current map.
la_status enqueue_rounds(la_batch *b, const la_weights *w, int32_t *H, const int32_t *lut, uint8_t *out_layers,
                         int32_t ntier, const std::vector<int32_t> &cnt, const std::vector<int32_t> &groups,
                         hipStream_t s)
{
    const int32_t ngroup = (int32_t)groups.size() / 2;
    const int32_t R = w->rounds;
    la_status st = LA_OK;
    bool has_prev = b->has_prev;
    const hipStream_t keep = b->stream;
    b->stream = s;   // commit_changed and history_update launch on the batch's stream
    int32_t *dcur = b->D, *dalt = b->D_alt;
    const int cgrid = (int)std::min<int64_t>(4096, (b->Eg / 4 + 255) / 256 + 1);
    for (int32_t r = 0; r < R && st == LA_OK; ++r) {
        DPArgs a = make_dp_args(b, w, H, lut);
        a.w.self_excl = has_prev ? 1 : 0;
        for (int32_t gi = 0; gi < ngroup && st == LA_OK; ++gi) {
            const int32_t t = groups[2 * gi], t_hi = groups[2 * gi + 1];
            int32_t nbig = 0, nsmall = 0;
            for (int32_t q = t; q <= t_hi; ++q) {
                nbig += cnt[q * kNB];
                nsmall += small_nets(cnt, q);
            }
            if (nbig + nsmall == 0) continue;
            const bool fused = nsmall >= b->tune.fuse_nets;
            // the change list holds the big nets' moves and, unfused, the small nets'
            const bool listed = !fused || nbig > 0;
            a.D = dcur;
            if (fused)
                LA_TIMED(b, "k_copy_i32", s,
                         hipLaunchKernelGGL(k_copy_i32, dim3(cgrid), dim3(256), 0, s, dalt, dcur, b->Eg));
            if (listed) hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, s, b->chg_count, 1);
            BArgs ba;
            ba.tier_nets = b->tier_nets;
            ba.tier_off = b->tier_off;
            ba.tier = t;
            ba.tier_hi = t_hi;
            ba.ctr = b->claim + r * ntier + gi;
            ba.cl_start = b->cl_start;
            ba.cl_off = b->cl_off;
            ba.height = b->height;
            ba.net_big = b->net_big;
            ba.bn_order = b->bn_order;
            ba.bn_lvl = b->bn_lvl;
            ba.bn_lvl_off = b->bn_lvl_off;
            ba.bn_nlev = b->bn_nlev;
            ba.bn_rec = (int4 *)b->bn_rec;
            ba.net_zw = b->net_zw;
            ba.nrec = (const uint4 *)b->nrec;
            ba.dynrec = (const uint2 *)b->dynrec;
            ba.cnet = (const int4 *)b->cnet;
            ba.ch = b->ch;
            ba.cur = b->cur_layer;
            ba.vlo = b->vlo;
            ba.vhi = b->vhi;
            ba.out_layers = out_layers;
            ba.has_prev = has_prev ? 1 : 0;
            ba.cl = ChangeList{b->chg_node, b->chg_old, b->chg_new, b->chg_count};
            ba.Dw = fused ? dalt : nullptr;
            st = launch_batched(b, a, ba, nbig, nsmall, s);
            if (st == LA_OK && listed) st = commit_changed(b, fused ? dalt : dcur);
            if (fused) std::swap(dcur, dalt);
        }
        if (st == LA_OK) st = history_update(b, dcur, H, w->hist_inc);
        has_prev = true;
    }
    if (st == LA_OK && dcur != b->D)
        LA_TIMED(b, "k_copy_i32", s, hipLaunchKernelGGL(k_copy_i32, dim3(cgrid), dim3(256), 0, s, b->D, dcur, b->Eg));
    b->stream = keep;
    return st;
}

}  // namespace

la_status assign_batched(la_batch *b, const la_weights *w, int32_t *H, const int32_t *lut, uint8_t *out_layers,
                         const int32_t *batch, bool direct)
{
    const int32_t ntier = batch ? w->num_tiers : 1;
    const int32_t nb = ntier * kNB;
    const int32_t R = w->rounds;
    if (b->claim_cap < R * ntier) {
        if (b->claim) (void)hipFree(b->claim);
        b->claim = nullptr;
        if (hipMalloc((void **)&b->claim, (size_t)R * ntier * sizeof(int32_t)) != hipSuccess)
            return set_error(LA_ERR_OOM, "claim counters");
        b->claim_cap = R * ntier;
    }
    // partition and claim arrays hold every batch (more than the 256 la_build_batch sized them for
    // when the caller hands over its own batches)
    if (b->part_cap < ntier) {
        for (int32_t **p : {&b->tier_off, &b->tier_cur, &b->tier_cnt, &b->cl_off, &b->cl_start}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        const int64_t starts = (b->nodes + (int64_t)kNetUnits * b->nets) / kClaimUnitsMin + 2 * (int64_t)ntier + 2;
        if (hipMalloc((void **)&b->tier_off, ((size_t)ntier * kNB + 2) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&b->tier_cur, ((size_t)ntier * kNB + 2) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&b->tier_cnt, ((size_t)ntier * kNB + 2) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&b->cl_off, ((size_t)ntier + 2) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void **)&b->cl_start, (size_t)starts * sizeof(int32_t)) != hipSuccess) {
            b->part_cap = 0;
            return set_error(LA_ERR_OOM, "batch partition arrays");
        }
        b->part_cap = ntier;
        b->cl_start_cap = starts;
        for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);   // they hold the old arrays
        b->graphs.clear();
    }
    // partition the nets by batch (big nets first, then nets with timing weights, then those
    // without, each by height) and check the batch indices
    LA_TIMED(b, "k_net_zero_weights", b->stream, {
        hipLaunchKernelGGL(k_fill_u8, dim3(grid1d(b->nets)), dim3(256), 0, b->stream, b->net_zw, (uint8_t)1, b->nets);
        hipLaunchKernelGGL(k_net_zero_weights, dim3(grid1d(b->nodes)), dim3(256), 0, b->stream, tree_view(b),
                           w->seg_w_q10, w->pin_w_q10, w->lambda_mohm, b->net_zw, (uint2 *)b->dynrec);
    });
    hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(1024), 0, b->stream, b->tier_cnt, nb + 1);
    LA_TIMED(b, "k_tier_count", b->stream,
             hipLaunchKernelGGL(k_tier_count, dim3(std::min(grid1d(b->nets), kPartGroups)), dim3(256), 0, b->stream,
                                batch, ntier, b->nets, b->tune.tile_nodes, b->net_zw, b->net_ptr, b->height,
                                b->tier_cnt, b->tier_cnt + nb));
    // the counts (and the count of nets whose batch index is out of range) before anything reads
    // the partition: the net list holds only the nets of valid batches
    LA_HIP(hipGetLastError());
    std::vector<int32_t> cnt(nb + 1);
    LA_HIP(hipMemcpyAsync(cnt.data(), b->tier_cnt, (nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    if (cnt[nb]) return set_error(LA_ERR_INVALID_ARG, "a net's batch index is outside 0..num_tiers-1");
    hipLaunchKernelGGL(k_tier_offsets, dim3(1), dim3(1024), 0, b->stream, b->tier_cnt, nb, b->tier_off, b->tier_cur,
                       b->claim, R * ntier);
    LA_TIMED(b, "k_tier_scatter", b->stream,
             hipLaunchKernelGGL(k_tier_scatter, dim3(std::min(grid1d(b->nets), kPartGroups)), dim3(256), 0,
                                b->stream, batch, ntier, b->nets, b->tune.tile_nodes, b->net_zw, b->net_ptr,
                                b->height, b->tier_cur, b->tier_nets));
    // work-queue claims of each batch's small nets
    {
        const int64_t n = b->nets + 1;
        const int32_t nchunk = (int32_t)((n + 1023) / 1024);
        hipLaunchKernelGGL(k_claim_units, dim3(grid1d(b->nets)), dim3(256), 0, b->stream, b->tier_nets, b->nets,
                           b->tier_off + nb, b->net_ptr, b->ch_ptr, b->net_zw, b->cl_pre, (int4 *)b->cnet);
        hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(256), 0, b->stream, b->cl_pre, n, b->cl_blk);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, b->stream, b->cl_blk, nchunk);
        hipLaunchKernelGGL(k_scan_add, dim3(grid1d(n)), dim3(256), 0, b->stream, b->cl_pre, n, b->cl_blk);
        hipLaunchKernelGGL(k_claim_offsets, dim3(1), dim3(256), 0, b->stream, b->tier_off, ntier, b->cl_pre,
                           b->tune.claim_units, b->cl_off);
        hipLaunchKernelGGL(k_claim_starts, dim3(grid1d(b->nets)), dim3(256), 0, b->stream, b->tier_off, ntier,
                           b->nets, b->cl_pre, b->tune.claim_units, b->cl_off, b->cl_start);
    }
    LA_HIP(hipGetLastError());

    // Consecutive batches of at most kMergeNets small nets whose bounding boxes are pairwise
    // disjoint run as one launch: no net of a later batch reads a GCell edge that an earlier
    // one commits to, so the result equals running the batches one after another.
    std::vector<int32_t> groups;
    {
        std::vector<int64_t> off(nb + 1, 0);
        for (int32_t q = 0; q < nb; ++q) off[q + 1] = off[q] + cnt[q];
        auto mergeable = [&](int32_t t) {
            const int32_t n = small_nets(cnt, t);
            return cnt[t * kNB] == 0 && n >= 1 && n <= kMergeNets;
        };
        std::vector<std::vector<int32_t>> nets_of(ntier);
        int32_t cand = 0;
        for (int32_t t = 0; t < ntier; ++t) cand += mergeable(t) ? 1 : 0;
        if (cand >= 2) {
            for (int32_t t = 0; t < ntier; ++t) {
                if (!mergeable(t)) continue;
                const int64_t p0 = off[t * kNB + 1], n = off[(t + 1) * kNB] - p0;
                nets_of[t].resize(n);
                LA_HIP(hipMemcpyAsync(nets_of[t].data(), b->tier_nets + p0, n * sizeof(int32_t), hipMemcpyDeviceToHost,
                                      b->stream));
            }
            LA_HIP(hipStreamSynchronize(b->stream));
        }
        auto overlap = [&](int32_t a, int32_t c) {
            const int16_t *p = &b->h_bbox[(size_t)4 * a], *q = &b->h_bbox[(size_t)4 * c];
            return p[0] <= q[1] && q[0] <= p[1] && p[2] <= q[3] && q[2] <= p[3];
        };
        int32_t lo = -1, hi = -1;
        bool open = false;                 // the current group still takes batches
        std::vector<int32_t> members;      // nets of the current group
        for (int32_t t = 0; t < ntier; ++t) {
            if (cnt[t * kNB] + small_nets(cnt, t) == 0) continue;
            bool join = open && cand >= 2 && mergeable(t);
            for (size_t i = 0; join && i < nets_of[t].size(); ++i)
                for (size_t k = 0; join && k < members.size(); ++k)
                    if (overlap(nets_of[t][i], members[k])) join = false;
            if (join) {
                hi = t;
                members.insert(members.end(), nets_of[t].begin(), nets_of[t].end());
                continue;
            }
            if (lo >= 0) {
                groups.push_back(lo);
                groups.push_back(hi);
            }
            lo = hi = t;
            open = cand >= 2 && mergeable(t);
            members = nets_of[t];
        }
        if (lo >= 0) {
            groups.push_back(lo);
            groups.push_back(hi);
        }
    }

    if (!b->side_stream) LA_HIP(hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking));
    if (!b->ev_fork) LA_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    if (!b->ev_join) LA_HIP(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    // the rounds, as one graph: per batch the persistent DP, then the commit; history per round.
    // While kernels are being timed the same launches go straight to the batch's stream.
    if (b->prof_on || direct) {
        hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(256), 0, b->stream, b->claim, R * ntier);
        la_status st = enqueue_rounds(b, w, H, lut, out_layers, ntier, cnt, groups, b->stream);
        if (st != LA_OK) return st;
        b->has_prev = true;
        return LA_OK;
    }
    std::vector<int64_t> key = {R, ntier, b->has_prev, w->w_cong, w->w_cap, w->w_d, w->w_via, w->hist_inc,
                                (int64_t)w->seg_w_q10, (int64_t)w->pin_w_q10, (int64_t)w->lambda_mohm,
                                (int64_t)lut, (int64_t)H, (int64_t)out_layers, (int64_t)batch, b->tune.tile_nodes,
                                b->tune.claim_units, b->tune.workgroups, b->tune.fuse_nets};
    for (int32_t t = 0; t < ntier; ++t) {
        key.push_back(cnt[t * kNB]);
        key.push_back(small_nets(cnt, t) > 0);
    }
    key.insert(key.end(), groups.begin(), groups.end());
    // a few graphs stay instantiated (most recently used first): the calls of a schedule
    // alternate between a handful of keys (the first call after a reset has no previous layers)
    auto &cache = b->graphs;
    size_t hit = 0;
    while (hit < cache.size() && cache[hit].first != key) ++hit;
    if (hit == cache.size()) {
        if (!b->cap_stream) LA_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipStream_t s = b->cap_stream;
        LA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const la_status st = enqueue_rounds(b, w, H, lut, out_layers, ntier, cnt, groups, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st != LA_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        if (cache.size() >= kGraphSlots) {
            (void)hipGraphExecDestroy(cache.back().second);
            cache.pop_back();
        }
        cache.insert(cache.begin(), std::make_pair(key, ex));
        b->graph_instantiations += 1;
    } else {
        std::rotate(cache.begin(), cache.begin() + hit, cache.begin() + hit + 1);
        // replay: the work-queue counters start from zero again
        hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(256), 0, b->stream, b->claim, R * ntier);
    }
    LA_HIP(hipGraphLaunch(cache.front().second, b->stream));
    b->has_prev = true;
    return LA_OK;
}

// ---- batch indices --------------------------------------------------------------------
namespace {
__global__ void k_widen_u8(const uint8_t *in, int32_t *out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}
}  // namespace

la_status batch_indices(la_batch *b, const la_weights *w, const int32_t **out)
{
    *out = nullptr;
    if (w->net_batch) {
        *out = w->net_batch;
    } else if (w->net_tier) {
        hipLaunchKernelGGL(k_widen_u8, dim3(grid1d(b->nets)), dim3(256), 0, b->stream, w->net_tier, b->batch_i32,
                           b->nets);
        LA_HIP(hipGetLastError());
        *out = b->batch_i32;
    }
    return LA_OK;
}

// ---- autotuner ------------------------------------------------------------------------
// la_tune times the launch configurations of the batched form on the instance itself: every
// tile size built for its routable-layer count, claim sizes around each tile size, then the
// fused-commit threshold of the fastest.  Each candidate runs one negotiation round of the
// caller's weights and batches from the same saved state (demand, previous layers, via spans,
// history), directly rather than from a graph; a first untimed pass loads every kernel.  The
// state is restored at the end, so la_tune changes nothing but the configuration, which is
// cached per instance shape for later batches of the same shape.  Every candidate gives the
// same layers, bit for bit (each net's result depends only on its own inputs and its batch's
// demand snapshot).
namespace {
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, Tuning> g_tune_cache;

std::vector<int64_t> shape_key(const la_batch *b)
{
    return {b->device, b->nets, b->nodes, b->tab.L, b->tab.X, b->tab.Y, b->NAmax, b->levels, b->max_net_nodes,
            b->gcell_edges};
}

struct Saved {
    int32_t *D = nullptr, *Hi = nullptr;
    uint8_t *cur = nullptr, *vlo = nullptr, *vhi = nullptr;
    ~Saved()
    {
        for (void *p : {(void *)D, (void *)Hi, (void *)cur, (void *)vlo, (void *)vhi})
            if (p) (void)hipFree(p);
    }
};
}  // namespace

la_status tune_batched(la_batch *b, const la_weights *w, const int32_t *history, const int32_t *lut,
                       const int32_t *batch, bool use_cache)
{
    const std::vector<int64_t> key = shape_key(b);
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            b->tune = it->second;
            return LA_OK;
        }
    }
    const int64_t M = std::max<int64_t>(b->nodes, 1);
    Saved sv;
    if (hipMalloc((void **)&sv.D, b->Eg * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&sv.Hi, b->Eg * sizeof(int32_t)) != hipSuccess || hipMalloc((void **)&sv.cur, M) != hipSuccess ||
        hipMalloc((void **)&sv.vlo, M) != hipSuccess || hipMalloc((void **)&sv.vhi, M) != hipSuccess)
        return set_error(LA_ERR_OOM, "la_tune: saved state");
    la_status st = grid_to_planes(b, history, b->Hi);
    if (st != LA_OK) return st;
    const hipStream_t s = b->stream;
    LA_HIP(hipMemcpyAsync(sv.D, b->D, b->Eg * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    LA_HIP(hipMemcpyAsync(sv.Hi, b->Hi, b->Eg * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    LA_HIP(hipMemcpyAsync(sv.cur, b->cur_layer, M, hipMemcpyDeviceToDevice, s));
    LA_HIP(hipMemcpyAsync(sv.vlo, b->vlo, M, hipMemcpyDeviceToDevice, s));
    LA_HIP(hipMemcpyAsync(sv.vhi, b->vhi, M, hipMemcpyDeviceToDevice, s));
    const bool prev0 = b->has_prev;
    auto restore = [&]() -> la_status {
        LA_HIP(hipMemcpyAsync(b->D, sv.D, b->Eg * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        LA_HIP(hipMemcpyAsync(b->Hi, sv.Hi, b->Eg * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        LA_HIP(hipMemcpyAsync(b->cur_layer, sv.cur, M, hipMemcpyDeviceToDevice, s));
        LA_HIP(hipMemcpyAsync(b->vlo, sv.vlo, M, hipMemcpyDeviceToDevice, s));
        LA_HIP(hipMemcpyAsync(b->vhi, sv.vhi, M, hipMemcpyDeviceToDevice, s));
        b->has_prev = prev0;
        return LA_OK;
    };
    la_weights w1 = *w;
    w1.rounds = 1;
    const Tuning keep = b->tune;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LA_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(LA_ERR_HIP, "la_tune: event");
    }
    // one round of candidate t from the saved state: its time (ms), or < 0 on failure
    auto run = [&](const Tuning &t, bool timed) -> double {
        if (restore() != LA_OK) return -1.0;
        b->tune = t;
        if (timed && hipEventRecord(e0, s) != hipSuccess) return -1.0;
        if (assign_batched(b, &w1, b->Hi, lut, nullptr, batch, true) != LA_OK) return -1.0;
        if (timed && hipEventRecord(e1, s) != hipSuccess) return -1.0;
        if (hipStreamSynchronize(s) != hipSuccess) return -1.0;
        float ms = 0.f;
        if (timed && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        return ms;
    };
    std::vector<Tuning> cand;
    for (int cap : kTileCaps) {
        if (!tile_size_supported(b->NAmax, cap)) continue;
        for (double f : {0.85, 1.15, 1.5}) {
            Tuning t = keep;
            t.tile_nodes = cap;
            t.claim_units = std::max(kClaimUnitsMin, std::min(kClaimUnitsMax, (int)(f * cap)));
            t.tuned = 0;
            cand.push_back(t);
        }
    }
    Tuning best = cand.front();
    double best_ms = -1.0;
    for (const Tuning &t : cand) (void)run(t, false);   // loads every kernel variant
    auto consider = [&](const Tuning &t) {
        const double ms = run(t, true);
        if (ms >= 0.0 && (best_ms < 0.0 || ms < best_ms)) {
            best_ms = ms;
            best = t;
        }
    };
    for (const Tuning &t : cand) consider(t);
    const Tuning base = best;
    for (int32_t fuse : {4096, 65536}) {
        Tuning t = base;
        t.fuse_nets = fuse;
        consider(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = restore();
    if (st == LA_OK) LA_HIP(hipStreamSynchronize(s));
    if (st != LA_OK || best_ms < 0.0) {
        b->tune = keep;
        return st != LA_OK ? st : set_error(LA_ERR_HIP, "la_tune: no candidate ran");
    }
    best.tuned = 1;
    b->tune = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    return LA_OK;
}

}  // namespace gapla
