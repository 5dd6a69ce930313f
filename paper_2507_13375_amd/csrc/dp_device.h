// Device routines of the tree DP (Alg. 3 with the Sec. III-D look-ahead) and the
// trace-back (Alg. 4), shared by the plain per-level kernels (state in HBM) and
// the batched kernels (state in LDS) through a small state-accessor type.
//
// For a node n and the layer l its parent segment takes, the DP considers the
// via stacks [b,t] at n that contain l and n's pin layer 0, lets each child take
// its best layer inside [b,t] by the look-ahead key, and keeps the stack of
// lowest look-ahead cost f'; ties keep the lowest b, then t, and a child's
// lowest layer.
//
// Three evaluation orders give that same result:
//  - hull candidates (via weight > 0, at most two children): a stack wider than
//    the hull of l, the pin layer and the chosen child layers costs more than
//    that hull with the same choices, so only hulls can win.  Each tuple of
//    child layers names one hull; it is a candidate when every child's choice is
//    its own key minimum (lowest layer on ties) inside that hull.  Valid tuples
//    are collected in a bit mask first and only those are costed.
//  - self-hull stacks (via weight > 0, three children): each child's keys are
//    computed once; a stack is costed only when it equals the hull of l, the pin layer
//    and the children's key minima inside it (any other stack loses to that hull).
//  - the full enumeration otherwise: every stack, each child's minimum rescanned.
//
// Integer widths: la_build_batch bounds every net so that R < 2^31, C, S < 2^30 and
// via sums < 2^24, hence R*X fits a 32x32-bit product; weights are Q10 (<= 1024);
// la_assign bounds w_d < 2^20 and the whole cost of a net below 2^62.
#pragma once

#include <type_traits>

#include "la_internal.h"

namespace gapla {

struct DPArgs {
    TreeDev T;
    LayerTab tab;      // copied into LDS by each kernel (`tb` below) before per-lane use
    DPWeights w;
    const int32_t *D;
    const uint8_t *caps;
    const int32_t *H;
    const uint8_t *prev;
    int64_t *F;        // [node][NA] f' (cost with the node's look-ahead term) of the chosen candidate
    int32_t *S;        // [node][NA] its X = C + 2S (aF, unsigned)
    uint8_t *bt;       // [node][NA] chosen via stack, b << 4 | t
    uint8_t *sel;      // [node][NA] node's layer for each entering-layer index of its parent
    int32_t NA;
};

// Copies the layer table into LDS: kernels index it with per-lane layer numbers, which
// must not read the kernel-argument block lane by lane.
__device__ __forceinline__ void load_tab(const LayerTab &src, LayerTab &dst)
{
    const int32_t *s = (const int32_t *)&src;
    int32_t *d = (int32_t *)&dst;
    for (int i = threadIdx.x; i < (int)(sizeof(LayerTab) / 4); i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

// Per-node inputs of the DP: segment length (GCells), look-ahead coefficient, Q10 segment
// weight, direction, flags and pin capacitance.
struct NodeIn {
    int32_t len;
    uint32_t lam, segw;
    int dir;
    uint8_t flags;
    int32_t cpin;
};

// DP state in HBM, indexed by global node id (plain form).  Besides the DP state, a state
// type gives the per-node inputs (`in`) and, at sinks, the pin weight.
struct GlobalState {
    const DPArgs &a;
    __device__ GlobalState(const DPArgs &a_) : a(a_) {}
    __device__ int nch(int32_t s) const { return a.T.ch_ptr[s + 1] - a.T.ch_ptr[s]; }
    __device__ int32_t ch_state(int32_t s, int q) const { return a.T.ch[a.T.ch_ptr[s] + q]; }
    __device__ int64_t &F(int32_t s, int j) const { return a.F[(int64_t)s * a.NA + j]; }
    __device__ int32_t &S(int32_t s, int j) const { return a.S[(int64_t)s * a.NA + j]; }
    __device__ uint8_t &bt(int32_t s, int j) const { return a.bt[(int64_t)s * a.NA + j]; }
    __device__ uint8_t &sel(int32_t s, int jp) const { return a.sel[(int64_t)s * a.NA + jp]; }
    __device__ NodeIn in(int32_t s) const
    {
        return NodeIn{a.T.len[s], (uint32_t)a.w.lam[s], a.w.seg_w[s], a.T.dir[s], a.T.flags[s], a.T.cpin[s]};
    }
    __device__ uint32_t pinw(int32_t s) const
    {
        const int32_t sid = a.T.sink_id[s];
        return sid >= 0 ? a.w.pin_w[sid] : 0u;
    }
};

// exact products of operands of known width
__device__ __forceinline__ uint64_t mul_u32(uint32_t a, uint32_t b) { return (uint64_t)a * (uint64_t)b; }
// a * b for a result below 2^64
__device__ __forceinline__ uint64_t mul_u64_u32(uint64_t a, uint32_t b)
{
    return (uint64_t)(uint32_t)a * b + (((uint64_t)(uint32_t)(a >> 32) * b) << 32);
}

// T(w, R, X) = (w * ((R * X) >> 11)) >> 10 for R, X < 2^32 and w <= 1024
__device__ __forceinline__ int64_t Tq(uint32_t w, uint32_t R, uint32_t X)
{
    return (int64_t)(mul_u64_u32(mul_u32(R, X) >> 11, w) >> 10);
}

// multiplication by the delay weight w_d (uniform; 1 by default)
struct Wd {
    uint32_t v;
    __device__ __forceinline__ int64_t operator()(int64_t x) const
    {
        return v == 1 ? x : (int64_t)mul_u64_u32((uint64_t)x, v);
    }
};

__device__ __forceinline__ uint32_t rvia_d(const LayerTab &t, int a, int b)
{
    const int32_t d = t.pv[a] - t.pv[b];
    return (uint32_t)(d < 0 ? -d : d);
}

// congestion cost kappa_n(l): marginal Eq. 3 cost plus history along the GCell edges of segment n;
// with first/stride, the part over GCell steps first, first + stride, ... (integer, so parts
// summed in any order give the same total)
__device__ __forceinline__ int64_t kappa_seg(const DPArgs &a, const LayerTab &tb, int32_t n, int l, int first = 0,
                                             int stride = 1)
{
    const int32_t len = a.T.len[n];
    const int d = a.T.dir[n];
    const int32_t step = tb.nAp[d];
    int32_t g = route_index(tb, d, tb.jidx[l], a.T.g0[n]) + first * step;
    const int32_t self = (a.w.self_excl && a.prev[n] == l) ? 1 : 0;
    const int32_t *lut = a.w.lut + l * 2 * kNDelta;
    int64_t s = 0;
    // unrolled so that several edges' loads are in flight at once
#pragma unroll 4
    for (int32_t k = first; k < len; k += stride, g += stride * step) {
        const int32_t cap = a.caps[g];
        int32_t d = a.D[g] - self - cap;
        d = d < kDeltaMin ? kDeltaMin : (d > kDeltaMin + kNDelta - 1 ? kDeltaMin + kNDelta - 1 : d);
        s += lut[(cap > 0 ? 0 : kNDelta) + d - kDeltaMin] + (int64_t)a.H[g];
    }
    return s;
}

// children per node handled by the hull-candidate order (more: full enumeration)
constexpr int kHullKids = 3;

// Per-child inputs that do not depend on the parent's layer.
struct ChildIn {
    int32_t cs;       // state index
    int32_t len;
    uint32_t w;       // Q10 segment weight
    uint32_t lam;     // look-ahead coefficient
    int dir;
};

template <class St>
__device__ __forceinline__ ChildIn child_in(const St &st, int32_t s, int q)
{
    ChildIn c;
    c.cs = st.ch_state(s, q);
    const NodeIn n = st.in(c.cs);
    c.len = n.len;
    c.w = n.segw;
    c.lam = n.lam;
    c.dir = n.dir;
    return c;
}

// The DP state of a (node, entering layer) keeps f' -- the subtree cost f plus the node's
// look-ahead term (Sec. III-D) -- and X = C + 2S (segment capacitance plus twice the
// downstream capacitance).  A parent entering on l ranks child layer t by
// key = f' + w_d T(w, Rvia(l, t), X).
// (jc: t's index in the child's direction list)
template <class St>
__device__ __forceinline__ int64_t child_key_j(const LayerTab &tb, const St &st, const Wd &wd, const ChildIn &c, int l,
                                               int t, int jc)
{
    return st.F(c.cs, jc) + wd(Tq(c.w, rvia_d(tb, l, t), (uint32_t)st.S(c.cs, jc)));
}

template <class St>
__device__ __forceinline__ int64_t child_key(const LayerTab &tb, const St &st, const Wd &wd, const ChildIn &c, int l,
                                             int t)
{
    return child_key_j(tb, st, wd, c, l, t, tb.jidx[t]);
}

// What a chosen child layer t contributes to its parent: V, the key without the child's
// look-ahead term (it enters the parent's f), and Z = C + S, the capacitance it presents.
struct ChildVZ {
    int64_t V;
    uint32_t Z;
};

template <class St>
__device__ __forceinline__ ChildVZ child_vz_j(const LayerTab &tb, const St &st, const Wd &wd, const ChildIn &c, int l,
                                             int t, int jc)
{
    const uint32_t X = (uint32_t)st.S(c.cs, jc);
    const uint32_t Z = (X + (uint32_t)(tb.c[t] * c.len)) >> 1;   // (C + 2S + C) / 2, exact
    ChildVZ r;
    r.V = st.F(c.cs, jc) - wd((int64_t)(mul_u32(c.lam, 2 * Z) >> 11)) + wd(Tq(c.w, rvia_d(tb, l, t), X));
    r.Z = Z;
    return r;
}

template <class St>
__device__ __forceinline__ ChildVZ child_vz(const LayerTab &tb, const St &st, const Wd &wd, const ChildIn &c, int l,
                                           int t)
{
    return child_vz_j(tb, st, wd, c, l, t, tb.jidx[t]);
}

__device__ __forceinline__ bool child_layer_ok(const LayerTab &tab, int cdir, int t)
{
    return tab.jidx[t] >= 0 && tab.dir[t] == cdir;
}

// Bit jj is set when a child's layer ly[jj] (ascending in jj; n of them) is its lowest-layer
// key minimum inside the hull of [lo, hi] and ly[jj]: no lower layer in that hull has a key
// <= its key and no higher one a smaller key.  Two running minima, O(NAMAX).
template <int NAMAX>
__device__ __forceinline__ uint32_t hull_min_mask(const int64_t (&ky)[NAMAX], const int (&ly)[NAMAX], int n, int lo,
                                                  int hi)
{
    bool low_ok[NAMAX];
    int64_t pm = INT64_MAX;   // minimum over the lower layers at or above lo
#pragma unroll
    for (int jj = 0; jj < NAMAX; ++jj) {
        low_ok[jj] = ly[jj] < lo || ky[jj] < pm;
        if (jj < n && ly[jj] >= lo) pm = min(pm, ky[jj]);
    }
    uint32_t m = 0;
    int64_t sm = INT64_MAX;   // minimum over the higher layers at or below hi
#pragma unroll
    for (int jj = NAMAX - 1; jj >= 0; --jj) {
        if (jj < n) {
            if (low_ok[jj] && (ly[jj] > hi || ky[jj] <= sm)) m |= 1u << jj;
            if (ly[jj] <= hi) sm = min(sm, ky[jj]);
        }
    }
    return m;
}

// For each layer index jj of a child (layers ascending, n of them), 8 bits at bit 8*jj: the
// highest lower layer whose key is <= its key, plus one (0: none), and at bit 8*jj + 4 the
// lowest higher layer whose key is smaller, minus one (15: none).  Layer jj is the child's
// lowest-layer key minimum inside a window [b, t] that holds it exactly when the first field
// is <= b and t <= the second.
template <int NAMAX>
__device__ __forceinline__ uint64_t block_bounds(const int64_t (&ky)[NAMAX], const int (&ly)[NAMAX], int n)
{
    uint64_t p = 0;
#pragma unroll
    for (int jj = 0; jj < NAMAX; ++jj) {
        int lb = 0, ub = 15;
#pragma unroll
        for (int i = 0; i < jj; ++i)
            if (i < n && ky[i] <= ky[jj]) lb = ly[i] + 1;
#pragma unroll
        for (int i = NAMAX - 1; i > jj; --i)
            if (i < n && ky[i] < ky[jj]) ub = ly[i] - 1;
        p |= (uint64_t)(lb | ub << 4) << (8 * jj);
    }
    return p;
}

// Best candidate so far; `better` applies the (f', b, t) order of the full enumeration.
struct Best {
    int64_t fp = INT64_MAX;
    uint32_t X = 0;
    int b = 0, t = 0;
    __device__ bool better(int64_t fp_, int b_, int t_) const
    {
        return fp_ < fp || (fp_ == fp && (b_ < b || (b_ == b && t_ < t)));
    }
};

// DP of node state s for its entering layer l (index j in its direction list; j = 0 and
// l = 0 at the root).  kap is kappa_n(l) (0 at the root).  NAMAX bounds the routable
// layers per direction.  SMALLK = false leaves out the one- and two-child orders (callers
// that run those items with dp_group); HULL23 = false leaves out the two- and three-child
// hull order (callers that run every such item with dp_group when the via weight is positive).
template <class St, int NAMAX, bool SMALLK = true, bool HULL23 = true>
__device__ __forceinline__ void dp_node(const DPArgs &a, const LayerTab &tb, const St &st, int32_t s, int l, int j,
                                        bool root, int64_t kap)
{
    const int L = tb.L;
    const Wd wd{(uint32_t)a.w.w_d};
    const NodeIn me = st.in(s);
    const uint8_t fl = me.flags;
    const bool pin = fl & (kSink | kDriver);
    const int lo = pin ? 0 : l;
    const int hi = l;
    int64_t own_const = 0;
    uint32_t Cs = 0, Rw = 0, segw = 0, lam = 0;
    if (!root) {
        Cs = (uint32_t)(tb.c[l] * me.len);
        Rw = (uint32_t)(tb.r[l] * me.len);
        own_const = a.w.w_cong * kap + a.w.w_cap * (int64_t)Cs;
        segw = me.segw;
        lam = me.lam;
    }
    const int32_t cpin = me.cpin;
    const int64_t pin_term = (fl & kSink) ? wd(Tq(st.pinw(s), rvia_d(tb, l, 0), 2 * (uint32_t)cpin)) : 0;
    const int k = st.nch(s);

    Best best;
    // f' and X of stack [b,t] given the children's summed f-contributions and capacitances
    // (at the root every segment term is zero)
    auto price = [&](int b, int t, int64_t sumV, int64_t sumZ, uint32_t &X) -> int64_t {
        const uint32_t Sn = (uint32_t)(cpin + sumZ);
        X = Cs + 2 * Sn;
        return a.w.w_via * (t - b) + sumV + pin_term + own_const + wd(Tq(segw, Rw, X)) +
               wd((int64_t)(mul_u32(lam, 2 * (Cs + Sn)) >> 11));
    };
    auto eval = [&](int b, int t, int64_t sumV, int64_t sumZ) -> bool {
        uint32_t X;
        const int64_t fp = price(b, t, sumV, sumZ, X);
        if (best.better(fp, b, t)) {
            best.fp = fp;
            best.X = X;
            best.b = b;
            best.t = t;
            return true;
        }
        return false;
    };

    bool done = false;
    if (a.w.w_via > 0 && k == 0) {
        eval(lo, hi, 0, 0);
        done = true;
    } else if (SMALLK && a.w.w_via > 0 && k == 1) {
        // ---- one child: each of its layers names one hull ---------------------------------
        // keys and X stay in registers; a candidate's f-part is its key minus the child's
        // look-ahead term
        const ChildIn c0 = child_in(st, s, 0);
        const int n0 = tb.nA[c0.dir];
        int64_t ky[NAMAX];
        uint32_t xq[NAMAX];
        int ly[NAMAX];
#pragma unroll
        for (int jj = 0; jj < NAMAX; ++jj) {
            ly[jj] = tb.lay[c0.dir][jj < n0 ? jj : 0];
            xq[jj] = jj < n0 ? (uint32_t)st.S(c0.cs, jj) : 0u;
            ky[jj] = jj < n0 ? st.F(c0.cs, jj) + wd(Tq(c0.w, rvia_d(tb, l, ly[jj]), xq[jj])) : 0;
        }
        const uint32_t m = hull_min_mask<NAMAX>(ky, ly, n0, lo, hi);
        // every layer is priced (independent chains, no branches), then the (f', b, t)
        // minimum over the candidates is kept
        int sel0 = 0;
#pragma unroll
        for (int jj = 0; jj < NAMAX; ++jj) {
            const uint32_t Z = (xq[jj] + (uint32_t)(tb.c[ly[jj]] * c0.len)) >> 1;
            const int64_t V = ky[jj] - wd((int64_t)(mul_u32(c0.lam, 2 * Z) >> 11));
            const int b = min(lo, ly[jj]), t = max(hi, ly[jj]);
            uint32_t X;
            const int64_t fp = price(b, t, V, Z, X);
            if (((m >> jj) & 1u) && best.better(fp, b, t)) {
                best.fp = fp;
                best.X = X;
                best.b = b;
                best.t = t;
                sel0 = ly[jj];
            }
        }
        st.sel(c0.cs, j) = (uint8_t)sel0;
        done = true;
    } else if (HULL23 && a.w.w_via > 0 && k >= 2 && k <= kHullKids && (SMALLK || k > 2)) {
        // ---- two or three children: hull candidates ---------------------------------------
        // A winning stack is the hull of lo, hi and the children's choices, each choice being
        // its child's key minimum inside that hull.  Such a choice is also the minimum inside
        // the smaller hull of lo, hi and itself alone, so each child's candidates are its
        // single-child mask; the block bounds then test a combination in O(1) per child.
        // per child: layers 4 bits per index, block bounds 8 bits per index, candidate mask
        uint32_t lyp[kHullKids], cand[kHullKids];
        uint64_t bnd[kHullKids];
        ChildIn cin[kHullKids];
#pragma unroll
        for (int q = 0; q < kHullKids; ++q) {
            lyp[q] = 0;
            bnd[q] = 0;
            cand[q] = 1;   // children beyond k: one pass that tests nothing
            cin[q] = ChildIn{};
            if (q < k) {
                const ChildIn cq = child_in(st, s, q);
                cin[q] = cq;
                const int nq = tb.nA[cq.dir];
                int64_t ky[NAMAX];
                int ly[NAMAX];
#pragma unroll
                for (int jj = 0; jj < NAMAX; ++jj) {
                    ly[jj] = tb.lay[cq.dir][jj < nq ? jj : 0];
                    ky[jj] = jj < nq ? child_key_j(tb, st, wd, cq, l, ly[jj], jj) : 0;
                    lyp[q] |= (uint32_t)ly[jj] << (4 * jj);
                }
                bnd[q] = block_bounds<NAMAX>(ky, ly, nq);
                cand[q] = hull_min_mask<NAMAX>(ky, ly, nq, lo, hi);
            }
        }
        auto lay_of = [&](int q, int jj) { return (int)((lyp[q] >> (4 * jj)) & 15u); };
        // child q's choice jj passes inside [b, t]
        auto inside = [&](int q, int jj, int b, int t) {
            const uint32_t f = (uint32_t)(bnd[q] >> (8 * jj));
            return (int)(f & 15u) <= b && t <= (int)((f >> 4) & 15u);
        };
        // Pairs of the first two children's candidates that pass inside their own hull with
        // lo and hi.  For two children that is the whole test; a third child can only widen
        // the hull, and a minimum inside the wider hull is one inside the narrower, so for
        // three it is a necessary condition, completed per third choice below.
        static_assert(kHullKids == 3 && NAMAX * NAMAX <= 64, "pair mask");
        uint64_t pm = 0;
        for (uint32_t m0 = cand[0]; m0; m0 &= m0 - 1) {
            const int j0 = __ffs(m0) - 1;
            const int L0 = lay_of(0, j0);
#pragma unroll
            for (int j1 = 0; j1 < NAMAX; ++j1) {
                const int L1 = lay_of(1, j1);
                const int b = min(lo, min(L0, L1)), t = max(hi, max(L0, L1));
                const bool ok = ((cand[1] >> j1) & 1u) && inside(0, j0, b, t) && inside(1, j1, b, t);
                pm |= (uint64_t)ok << (j0 * NAMAX + j1);
            }
        }
        uint32_t sel_pack = 0;   // chosen child layers, 4 bits per child
        while (pm) {
            const int p = __ffsll((unsigned long long)pm) - 1;
            pm &= pm - 1;
            const int j0 = p / NAMAX, j1 = p - (p / NAMAX) * NAMAX;
            const int L0 = lay_of(0, j0), L1 = lay_of(1, j1);
            const int b01 = min(lo, min(L0, L1)), t01 = max(hi, max(L0, L1));
            const ChildVZ c0 = child_vz_j(tb, st, wd, cin[0], l, L0, j0);
            const ChildVZ c1 = child_vz_j(tb, st, wd, cin[1], l, L1, j1);
            if (k == 2) {
                if (eval(b01, t01, c0.V + c1.V, (int64_t)c0.Z + c1.Z)) sel_pack = (uint32_t)(L0 | L1 << 4);
                continue;
            }
#pragma unroll
            for (int j2 = 0; j2 < NAMAX; ++j2) {
                const int L2 = lay_of(2, j2);
                const int b = min(b01, L2), t = max(t01, L2);
                if (!((cand[2] >> j2) & 1u) || !inside(0, j0, b, t) || !inside(1, j1, b, t) || !inside(2, j2, b, t))
                    continue;
                const ChildVZ c2 = child_vz_j(tb, st, wd, cin[2], l, L2, j2);
                if (eval(b, t, c0.V + c1.V + c2.V, (int64_t)c0.Z + c1.Z + c2.Z))
                    sel_pack = (uint32_t)(L0 | L1 << 4 | L2 << 8);
            }
        }
#pragma unroll
        for (int q = 0; q < kHullKids; ++q)
            if (q < k) st.sel(st.ch_state(s, q), j) = (uint8_t)((sel_pack >> (4 * q)) & 15u);
        done = true;
    }
    if (!done) {
        // ---- full enumeration: every stack, each child rescanned ------------------------
        for (int b = 0; b <= lo; ++b)
            for (int t = hi; t < L; ++t) {
                bool ok = true;
                int64_t sumV = 0, sumZ = 0;
                for (int q = 0; q < k && ok; ++q) {
                    const ChildIn c = child_in(st, s, q);
                    int bl = -1;
                    int64_t bk = 0;
                    for (int lc = b; lc <= t; ++lc) {
                        if (!child_layer_ok(tb, c.dir, lc)) continue;
                        const int64_t key = child_key(tb, st, wd, c, l, lc);
                        if (bl < 0 || key < bk) {
                            bl = lc;
                            bk = key;
                        }
                    }
                    ok = bl >= 0;
                    if (ok) {
                        const ChildVZ v = child_vz(tb, st, wd, c, l, bl);
                        sumV += v.V;
                        sumZ += v.Z;
                    }
                }
                if (ok) eval(b, t, sumV, sumZ);
            }
        // each child's layer at the chosen stack, by the same rule
        for (int q = 0; q < k; ++q) {
            const ChildIn c = child_in(st, s, q);
            int bl = 0;
            bool have = false;
            int64_t bk = 0;
            for (int lc = best.b; lc <= best.t; ++lc) {
                if (!child_layer_ok(tb, c.dir, lc)) continue;
                const int64_t key = child_key(tb, st, wd, c, l, lc);
                if (!have || key < bk) {
                    have = true;
                    bk = key;
                    bl = lc;
                }
            }
            st.sel(c.cs, j) = (uint8_t)bl;
        }
    }

    st.F(s, j) = best.fp;
    st.S(s, j) = (int32_t)best.X;
    st.bt(s, j) = (uint8_t)(best.b << 4 | best.t);
}

// ---- lane-parallel DP of one item ---------------------------------------------------------
// The 8 lanes of an aligned group (sub = lane & 7) share one item (node state s, entering
// layer l, index j) with one to three children and a positive via weight: lane sub takes the
// children's layer index sub.  Candidate tests use minima across the group (prefix/suffix
// scans, broadcasts) and the best candidate is a group argmin over (f', b, t), so the result
// equals dp_node's.  Every lane of the group must call it; lane 0 writes the state.
constexpr int kGroup = 8;

// Lane exchanges inside an aligned group of 8 lanes (half a DPP row of 16), as DPP moves on
// the VALU instead of general lane shuffles through the LDS crossbar.  A move from a lane
// outside the group (a shift at the group's edge) keeps the lane's own value; callers ignore it.
namespace gx {
constexpr int kRowShl = 0x100, kRowShr = 0x110, kHalfMirror = 0x141;
constexpr int quad(int a, int b, int c, int d) { return a | b << 2 | c << 4 | d << 6; }
template <int CTRL>
__device__ __forceinline__ int32_t mov(int32_t x)
{
    return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint32_t mov(uint32_t x)
{
    return (uint32_t)mov<CTRL>((int32_t)x);
}
template <int CTRL>
__device__ __forceinline__ int64_t mov(int64_t x)
{
    const uint32_t lo = (uint32_t)mov<CTRL>((int32_t)(uint32_t)x), hi = (uint32_t)mov<CTRL>((int32_t)(x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// value of group lane I in every lane of the group (sub = this lane's index in it)
template <int I, class T>
__device__ __forceinline__ T bcast(T x, int sub)
{
    constexpr int qi = I & 3, qj = (7 - I) & 3;
    const T a = mov<quad(qi, qi, qi, qi)>(x);                 // lane I, seen from its own quad
    const T b = mov<quad(qj, qj, qj, qj)>(mov<kHalfMirror>(x)); // lane I, seen from the other quad
    return (sub >> 2) == (I >> 2) ? a : b;
}
template <int I, class F>
__device__ __forceinline__ void each_lane(F &&f)
{
    if constexpr (I < kGroup) {
        f(std::integral_constant<int, I>{});
        each_lane<I + 1>(f);
    }
}
}  // namespace gx

// inclusive prefix minimum over the group's lanes 0..sub
__device__ __forceinline__ int64_t grp_min_up(int64_t x, int sub)
{
    int64_t o = gx::mov<gx::kRowShr + 1>(x);
    if (sub >= 1) x = o < x ? o : x;
    o = gx::mov<gx::kRowShr + 2>(x);
    if (sub >= 2) x = o < x ? o : x;
    o = gx::mov<gx::kRowShr + 4>(x);
    if (sub >= 4) x = o < x ? o : x;
    return x;
}

// inclusive suffix minimum over the group's lanes sub..7
__device__ __forceinline__ int64_t grp_min_down(int64_t x, int sub)
{
    int64_t o = gx::mov<gx::kRowShl + 1>(x);
    if (sub + 1 < kGroup) x = o < x ? o : x;
    o = gx::mov<gx::kRowShl + 2>(x);
    if (sub + 2 < kGroup) x = o < x ? o : x;
    o = gx::mov<gx::kRowShl + 4>(x);
    if (sub + 4 < kGroup) x = o < x ? o : x;
    return x;
}

template <class St, int NAMAX>
__device__ __forceinline__ void dp_group(const DPArgs &a, const LayerTab &tb, const St &st, int32_t s, int l, int j,
                                         bool root, int64_t kap, int sub)
{
    static_assert(NAMAX <= kGroup, "one lane per layer index");
    const Wd wd{(uint32_t)a.w.w_d};
    const NodeIn me = st.in(s);
    const bool pin = me.flags & (kSink | kDriver);
    const int lo = pin ? 0 : l;
    const int hi = l;
    int64_t own_const = 0;
    uint32_t Cs = 0, Rw = 0;
    if (!root) {
        Cs = (uint32_t)(tb.c[l] * me.len);
        Rw = (uint32_t)(tb.r[l] * me.len);
        own_const = a.w.w_cong * kap + a.w.w_cap * (int64_t)Cs;
    }
    const int64_t pin_term =
        (me.flags & kSink) ? wd(Tq(st.pinw(s), rvia_d(tb, l, 0), 2 * (uint32_t)me.cpin)) : 0;
    // f' and X of stack [b,t] for the children's summed f-parts and capacitances
    auto value = [&](int b, int t, int64_t sumV, int64_t sumZ, uint32_t &X) -> int64_t {
        const uint32_t Sn = (uint32_t)(me.cpin + sumZ);
        int64_t fp = a.w.w_via * (t - b) + sumV + pin_term;
        X = 2 * Sn;
        if (!root) {
            X = Cs + 2 * Sn;
            fp += own_const + wd(Tq(me.segw, Rw, X)) + wd((int64_t)(mul_u32(me.lam, 2 * (Cs + Sn)) >> 11));
        }
        return fp;
    };
    const int k = st.nch(s);
    // this lane's candidate: f', stack b << 4 | t, X and the children's layers (4 bits each)
    int64_t fp = INT64_MAX;
    uint32_t bt = 0xff, X = 0, sel = 0;
    const ChildIn c0 = child_in(st, s, 0);
    const int n0 = tb.nA[c0.dir];
    const bool v0 = sub < n0;
    const int l0 = tb.lay[c0.dir][v0 ? sub : 0];
    const int64_t k0 = v0 ? child_key_j(tb, st, wd, c0, l, l0, sub) : INT64_MAX;
    if (k == 1) {
        // layer l0 is a candidate when no lower layer inside its hull has a key <= its key
        // and no higher one a smaller key (exclusive scans over the lanes in layer order)
        const int64_t below = gx::mov<gx::kRowShr + 1>(grp_min_up(v0 && l0 >= lo ? k0 : INT64_MAX, sub));
        const int64_t above = gx::mov<gx::kRowShl + 1>(grp_min_down(v0 && l0 <= hi ? k0 : INT64_MAX, sub));
        const bool ok = v0 && (l0 < lo || sub == 0 || k0 < below) && (l0 > hi || sub == kGroup - 1 || k0 <= above);
        if (ok) {
            const ChildVZ v = child_vz_j(tb, st, wd, c0, l, l0, sub);
            const int b = min(lo, l0), t = max(hi, l0);
            fp = value(b, t, v.V, v.Z, X);
            bt = (uint32_t)(b << 4 | t);
            sel = (uint32_t)l0;
        }
    } else if (k == 2) {
        // two children: a pair is a candidate when each choice is its child's key minimum in
        // the pair's hull; per child and layer, the highest lower layer with a key <= and the
        // lowest higher layer with a smaller key bound the hulls where it stays the minimum
        const ChildIn c1 = child_in(st, s, 1);
        const int n1 = tb.nA[c1.dir];
        const bool v1 = sub < n1;
        const int l1 = tb.lay[c1.dir][v1 ? sub : 0];
        const int64_t k1 = v1 ? child_key_j(tb, st, wd, c1, l, l1, sub) : INT64_MAX;
        int lb0 = -1, ub0 = 16, lb1 = -1, ub1 = 16;
        gx::each_lane<0>([&](auto I_) {
            constexpr int i = decltype(I_)::value;
            const int64_t ki0 = gx::bcast<i>(k0, sub), ki1 = gx::bcast<i>(k1, sub);
            const int li0 = tb.lay[c0.dir][i < kMaxA ? i : 0], li1 = tb.lay[c1.dir][i < kMaxA ? i : 0];
            if (i < n0 && i < sub && ki0 <= k0) lb0 = li0;
            if (i < n1 && i < sub && ki1 <= k1) lb1 = li1;
            if (i < n0 && i > sub && ki0 < k0 && ub0 == 16) ub0 = li0;
            if (i < n1 && i > sub && ki1 < k1 && ub1 == 16) ub1 = li1;
        });
        // child 1's layer, bounds and validity of every index, for the pairs of this lane
        const uint32_t pack1 = (uint32_t)l1 | (uint32_t)(lb1 + 1) << 4 | (uint32_t)(ub1 + 1) << 9 | (v1 ? 1u << 14 : 0u);
        // the pairs of this lane's choice with each of child 1's indices that pass (bit i)
        uint32_t pm = 0;
        gx::each_lane<0>([&](auto I_) {
            constexpr int i = decltype(I_)::value;
            const uint32_t p = gx::bcast<i>(pack1, sub);
            const int L2 = (int)(p & 15u), lb2 = (int)((p >> 4) & 31u) - 1, ub2 = (int)((p >> 9) & 31u) - 1;
            const int b = min(lo, min(l0, L2)), t = max(hi, max(l0, L2));
            if (v0 && ((p >> 14) & 1u) && lb0 < b && t < ub0 && lb2 < b && t < ub2) pm |= 1u << i;
        });
        // each lane's own contributions; child 1's reach the pairs by shuffles inside the group.
        // Only the passing pairs are priced, in ascending i (the order of the tie rule): a pass
        // per pair of the lane with the most, every lane of the branch taking part in each (the
        // shuffles read other lanes), a lane with none left pricing nothing.
        ChildVZ z0{0, 0}, z1o{0, 0};
        if (v0) z0 = child_vz_j(tb, st, wd, c0, l, l0, sub);
        if (v1) z1o = child_vz_j(tb, st, wd, c1, l, l1, sub);
        const int gbase = __lane_id() & ~(kGroup - 1);
        while (__any(pm != 0)) {
            const bool have = pm != 0;
            const int i = have ? __ffs(pm) - 1 : 0;
            pm &= pm - 1;
            const int src = gbase + i;
            const int64_t V1 = __shfl((long long)z1o.V, src);
            const uint32_t Z1 = (uint32_t)__shfl((int)z1o.Z, src);
            const int L2 = (int)((uint32_t)__shfl((int)pack1, src) & 15u);
            if (have) {
                const int b = min(lo, min(l0, L2)), t = max(hi, max(l0, L2));
                uint32_t Xc;
                const int64_t f = value(b, t, z0.V + V1, (int64_t)z0.Z + Z1, Xc);
                const uint32_t btc = (uint32_t)(b << 4 | t);
                if (f < fp || (f == fp && btc < bt)) {
                    fp = f;
                    bt = btc;
                    X = Xc;
                    sel = (uint32_t)l0 | (uint32_t)L2 << 4;
                }
            }
        }
    } else {
        // three children: per child, lane sub finds the block bounds of the child's index sub
        // (from the group's keys, one broadcast at a time) and whether that index is a
        // single-child candidate (prefix / suffix minima across the group, as for one child);
        // the group then shares both, so every lane holds each child's bounds and candidate
        // mask -- the values the serial hull order computes -- and lane sub takes the
        // combinations whose first choice is index sub
        uint32_t lyp[3], cand[3];
        uint64_t bnd[3];
        ChildIn cq[3];
        int nq[3];
        cq[0] = c0;
        const int gbase = __lane_id() & ~(kGroup - 1);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (q > 0) cq[q] = child_in(st, s, q);
            const int dq = cq[q].dir;
            nq[q] = tb.nA[dq];
            const bool vq = sub < nq[q];
            const int lq = tb.lay[dq][vq ? sub : 0];
            const int64_t kq = q == 0 ? k0 : (vq ? child_key_j(tb, st, wd, cq[q], l, lq, sub) : INT64_MAX);
            // the highest lower index with a key <= this one (its layer + 1, else 0) and the lowest
            // higher index with a smaller key (its layer - 1, else 15)
            int lbq = 0, ubq = 15;
            lyp[q] = 0;
            gx::each_lane<0>([&](auto I_) {
                constexpr int i = decltype(I_)::value;
                const int64_t ki = gx::bcast<i>(kq, sub);
                const int li = tb.lay[dq][i < kMaxA ? i : 0];
                if (i < nq[q] && i < sub && ki <= kq) lbq = li + 1;
                if (i < nq[q] && i > sub && ki < kq && ubq == 15) ubq = li - 1;
                if constexpr (i < NAMAX) lyp[q] |= (uint32_t)li << (4 * i);
            });
            const int64_t below = gx::mov<gx::kRowShr + 1>(grp_min_up(vq && lq >= lo ? kq : INT64_MAX, sub));
            const int64_t above = gx::mov<gx::kRowShl + 1>(grp_min_down(vq && lq <= hi ? kq : INT64_MAX, sub));
            const bool okq =
                vq && (lq < lo || sub == 0 || kq < below) && (lq > hi || sub == kGroup - 1 || kq <= above);
            cand[q] = (uint32_t)((__ballot(okq) >> gbase) & 0xffu);
            const uint32_t myb = (uint32_t)(lbq | ubq << 4);
            bnd[q] = 0;
            gx::each_lane<0>([&](auto I_) {
                constexpr int i = decltype(I_)::value;
                if constexpr (i < NAMAX) bnd[q] |= (uint64_t)gx::bcast<i>(myb, sub) << (8 * i);
            });
        }
        auto lay_of = [&](int q, int jj) { return (int)((lyp[q] >> (4 * jj)) & 15u); };
        auto inside = [&](int q, int jj, int b, int t) {
            const uint32_t f = (uint32_t)(bnd[q] >> (8 * jj));
            return (int)(f & 15u) <= b && t <= (int)((f >> 4) & 15u);
        };
        if ((cand[0] >> sub) & 1u) {
            const ChildVZ z0 = child_vz_j(tb, st, wd, cq[0], l, l0, sub);
            for (uint32_t m1 = cand[1]; m1; m1 &= m1 - 1) {
                const int j1 = __ffs(m1) - 1;
                const int L1 = lay_of(1, j1);
                const int b01 = min(lo, min(l0, L1)), t01 = max(hi, max(l0, L1));
                // necessary inside the pair's hull (a third choice can only widen it)
                if (!inside(0, sub, b01, t01) || !inside(1, j1, b01, t01)) continue;
                const ChildVZ z1 = child_vz_j(tb, st, wd, cq[1], l, L1, j1);
                for (uint32_t m2 = cand[2]; m2; m2 &= m2 - 1) {
                    const int j2 = __ffs(m2) - 1;
                    const int L2 = lay_of(2, j2);
                    const int b = min(b01, L2), t = max(t01, L2);
                    if (!inside(0, sub, b, t) || !inside(1, j1, b, t) || !inside(2, j2, b, t)) continue;
                    const ChildVZ z2 = child_vz_j(tb, st, wd, cq[2], l, L2, j2);
                    uint32_t Xc;
                    const int64_t f = value(b, t, z0.V + z1.V + z2.V, (int64_t)z0.Z + z1.Z + z2.Z, Xc);
                    const uint32_t btc = (uint32_t)(b << 4 | t);
                    if (f < fp || (f == fp && btc < bt)) {
                        fp = f;
                        bt = btc;
                        X = Xc;
                        sel = (uint32_t)l0 | (uint32_t)L1 << 4 | (uint32_t)L2 << 8;
                    }
                }
            }
        }
    }
    // group argmin over (f', b, t, lane): a total order, so every lane ends with the same
    // candidate whatever the exchange pattern -- on equal (f', b, t) the lowest lane, i.e. the
    // lowest first-child layer (and each lane already kept the lowest other choices)
    bt |= (uint32_t)sub << 8;
    auto take = [&](int64_t ofp, uint32_t obt, uint32_t oX, uint32_t osel) {
        if (ofp < fp || (ofp == fp && obt < bt)) {
            fp = ofp;
            bt = obt;
            X = oX;
            sel = osel;
        }
    };
    constexpr int kX1 = gx::quad(1, 0, 3, 2), kX2 = gx::quad(2, 3, 0, 1), kX4 = gx::kHalfMirror;
    take(gx::mov<kX1>(fp), gx::mov<kX1>(bt), gx::mov<kX1>(X), gx::mov<kX1>(sel));
    take(gx::mov<kX2>(fp), gx::mov<kX2>(bt), gx::mov<kX2>(X), gx::mov<kX2>(sel));
    take(gx::mov<kX4>(fp), gx::mov<kX4>(bt), gx::mov<kX4>(X), gx::mov<kX4>(sel));
    bt &= 0xffu;
    if (sub == 0) {
        st.F(s, j) = fp;
        st.S(s, j) = (int32_t)X;
        st.bt(s, j) = (uint8_t)bt;
        st.sel(c0.cs, j) = (uint8_t)(sel & 15u);
        if (k >= 2) st.sel(st.ch_state(s, 1), j) = (uint8_t)((sel >> 4) & 15u);
        if (k == 3) st.sel(st.ch_state(s, 2), j) = (uint8_t)((sel >> 8) & 15u);
    }
}

// Commit list of the current batch: segments whose layer changed (old = 255 when the
// segment has no previous layer).
struct ChangeList {
    int32_t *node;
    uint8_t *old_l, *new_l;
    int32_t *count;
};

// Appends one entry per lane with `pred`, one atomic per wavefront.  Every lane of the
// wavefront must call it (uniform control flow).
__device__ __forceinline__ void append_change(const ChangeList &cl, bool pred, int32_t n, uint8_t old_l,
                                              uint8_t new_l)
{
    const uint64_t mask = __ballot(pred);
    if (!mask) return;
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(cl.count, (int32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        const int32_t pos = base + (int32_t)__popcll(mask & __lanemask_lt());
        cl.node[pos] = n;
        cl.old_l[pos] = old_l;
        cl.new_l[pos] = new_l;
    }
}

// Alg. 4 at node state s: its layer is the one its parent recorded for the parent's entering
// layer.  jp: the index of the parent's entering layer in the parent's direction list (0 when
// the parent is the root).  Sets *ln to the layer (0 at the root) and returns s's own
// entering-layer index.
template <class St>
__device__ __forceinline__ int trace_choice(const LayerTab &tb, const St &st, int32_t s, int jp, bool root, int *ln_out)
{
    int ln = 0, j = 0;
    if (!root) {
        // jp < the parent's routable-layer count and the parent's DP recorded a routable
        // layer of s's direction; the clamps only keep every index inside its array
        ln = st.sel(s, (jp >= 0 && jp < kMaxA) ? jp : 0);
        ln = ln < tb.L ? ln : 0;
        j = tb.jidx[ln] < 0 ? 0 : tb.jidx[ln];
    }
    *ln_out = ln;
    return j;
}

// Writes node n's layer ln and the via span recorded for its entering index j.  old: n's
// layer before this pass when the caller has it, else -1 (read from cur).  Sets *changed /
// *old_l for the commit list.
template <class St>
__device__ __forceinline__ void trace_write(const St &st, int32_t s, int32_t n, int j, int ln, bool root, uint8_t *cur,
                                            uint8_t *vlo, uint8_t *vhi, uint8_t *out_layers, int has_prev,
                                            bool *changed, uint8_t *old_l, int old_in = -1)
{
    const uint8_t bt = st.bt(s, j);
    vlo[n] = bt >> 4;
    vhi[n] = bt & 15;
    const uint8_t old = old_in >= 0 ? (uint8_t)old_in : cur[n];
    cur[n] = (uint8_t)ln;
    if (out_layers) out_layers[n] = (uint8_t)ln;
    *changed = !root && (!has_prev || old != ln);
    *old_l = has_prev ? old : (uint8_t)255;
}

// Both steps at node n (state s); returns n's entering-layer index.
template <class St>
__device__ __forceinline__ int trace_node(const LayerTab &tb, const St &st, int32_t s, int32_t n, int jp, bool root,
                                          uint8_t *cur, uint8_t *vlo, uint8_t *vhi, uint8_t *out_layers,
                                          int has_prev, int *ln_out, bool *changed, uint8_t *old_l, int old_in = -1)
{
    const int j = trace_choice(tb, st, s, jp, root, ln_out);
    trace_write(st, s, n, j, *ln_out, root, cur, vlo, vhi, out_layers, has_prev, changed, old_l, old_in);
    return j;
}

}  // namespace gapla
