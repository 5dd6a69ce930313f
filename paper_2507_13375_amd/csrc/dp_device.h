// Device routines of the tree DP (Alg. 3, Sec. III-D look-ahead) and trace-back
// (Alg. 4), shared by the plain per-level kernels and the batched kernels.
//
// For a node n and the layer l its parent segment takes, the DP enumerates the
// via stacks [b,t] at n that contain l and n's pin layer 0 (b ascending, then t
// ascending), lets each child take its best layer inside [b,t] by the
// look-ahead key, and keeps the stack of lowest look-ahead cost f'; ties keep
// the first (lowest b, then t) stack and the lowest child layer.  The children's
// running minima are extended one layer at a time as t grows, so each stack
// costs one key per child whose direction matches layer t.
#pragma once

#include "la_internal.h"

namespace gapla {

struct DPArgs {
    TreeDev T;
    LayerTab tab;
    DPWeights w;
    const int32_t *D;
    const uint8_t *caps;
    const int32_t *H;
    const uint8_t *prev;
    int64_t *F, *KA;   // [node][NA] subtree cost f and f + look-ahead of the node's own segment
    int32_t *S;        // [node][NA] downstream capacitance of the chosen candidate (aF)
    uint8_t *bt;       // [node][NA][2] chosen via stack
    uint8_t *sel;      // [node][kMaxL] node's layer for each entering layer of its parent
    int32_t NA;
};

constexpr int kFastChildren = 4;

// T(w, R, X) = (w * ((R * X) >> 11)) >> 10, operands non-negative
__device__ __forceinline__ int64_t Tq(int64_t w, int64_t R, int64_t X) { return (w * ((R * X) >> 11)) >> 10; }

__device__ __forceinline__ int64_t rvia_d(const LayerTab &t, int a, int b)
{
    const int32_t d = t.pv[a] - t.pv[b];
    return d < 0 ? -d : d;
}

// congestion cost kappa_n(l): marginal Eq. 3 cost plus history along the GCell edges of segment n
__device__ __forceinline__ int64_t kappa_seg(const DPArgs &a, int32_t n, int l)
{
    const int32_t len = a.T.len[n];
    const int32_t step = a.T.dir[n] == 0 ? a.tab.L : a.tab.X * a.tab.L;
    int32_t g = a.T.g0[n] + l;
    const int32_t self = (a.w.self_excl && a.prev[n] == l) ? 1 : 0;
    const int32_t *lut = a.w.lut + l * 2 * kNDelta;
    int64_t s = 0;
    for (int32_t k = 0; k < len; ++k, g += step) {
        const int32_t cap = a.caps[g];
        int32_t d = a.D[g] - self - cap;
        d = d < kDeltaMin ? kDeltaMin : (d > kDeltaMin + kNDelta - 1 ? kDeltaMin + kNDelta - 1 : d);
        s += lut[(cap > 0 ? 0 : kNDelta) + d - kDeltaMin] + (int64_t)a.H[g];
    }
    return s;
}

struct ChildKey {
    int64_t key, V;
    int32_t Z;
};

// key, f-contribution and downstream capacitance of child c on layer t under parent layer l
__device__ __forceinline__ ChildKey child_key(const DPArgs &a, int32_t c, int32_t clen, int64_t cw, int l, int t)
{
    const int64_t idx = (int64_t)c * a.NA + a.tab.jidx[t];
    const int32_t Cc = a.tab.c[t] * clen;
    const int32_t Sc = a.S[idx];
    const int64_t X = (int64_t)Cc + 2 * (int64_t)Sc;
    const int64_t tv = a.w.w_d * Tq(cw, rvia_d(a.tab, l, t), X);
    ChildKey r;
    r.V = a.F[idx] + tv;
    r.key = a.KA[idx] + tv;
    r.Z = Cc + Sc;
    return r;
}

__device__ __forceinline__ bool child_layer_ok(const LayerTab &tab, int cdir, int t)
{
    return tab.jidx[t] >= 0 && tab.dir[t] == cdir;
}

// DP of node n for the entering layer l (index j in its direction list; j = 0, l = 0 at the root).
__device__ void dp_node_layer(const DPArgs &a, int32_t n, int l, int j, bool root)
{
    const int L = a.tab.L;
    const uint8_t fl = a.T.flags[n];
    const bool pin = fl & (kSink | kDriver);
    const int lo = pin ? 0 : l;
    const int hi = l;
    int64_t own_const = 0, Cs = 0, Rw = 0, segw = 0, lam = 0;
    if (!root) {
        const int32_t len = a.T.len[n];
        Cs = (int64_t)a.tab.c[l] * len;
        Rw = (int64_t)a.tab.r[l] * len;
        own_const = a.w.w_cong * kappa_seg(a, n, l) + a.w.w_cap * Cs;
        segw = a.w.seg_w[n];
        lam = a.w.lam[n];
    }
    const int32_t cpin = a.T.cpin[n];
    const int32_t sid = a.T.sink_id[n];
    const int64_t pin_term = sid >= 0 ? a.w.w_d * Tq(a.w.pin_w[sid], rvia_d(a.tab, l, 0), 2 * (int64_t)cpin) : 0;
    const int32_t c0 = a.T.ch_ptr[n], k = a.T.ch_ptr[n + 1] - c0;

    int64_t best_fp = INT64_MAX, best_f = 0, best_S = 0;
    int best_b = 0, best_t = 0;
    uint8_t best_sel[kFastChildren] = {0, 0, 0, 0};

    auto eval = [&](int b, int t, int64_t sumV, int64_t sumZ) -> bool {
        const int64_t Sn = cpin + sumZ;
        int64_t f = a.w.w_via * (t - b) + sumV + pin_term;
        int64_t fp = f;
        if (!root) {
            f += own_const + a.w.w_d * Tq(segw, Rw, Cs + 2 * Sn);
            fp = f + a.w.w_d * ((lam * 2 * (Cs + Sn)) >> 11);
        }
        if (fp < best_fp) {
            best_fp = fp;
            best_f = f;
            best_S = Sn;
            best_b = b;
            best_t = t;
            return true;
        }
        return false;
    };

    if (k <= kFastChildren) {
        int32_t cid[kFastChildren], clen[kFastChildren];
        int cdir[kFastChildren];
        int64_t cw[kFastChildren];
#pragma unroll
        for (int q = 0; q < kFastChildren; ++q) {
            if (q < k) {
                cid[q] = a.T.ch[c0 + q];
                cdir[q] = a.T.dir[cid[q]];
                clen[q] = a.T.len[cid[q]];
                cw[q] = a.w.seg_w[cid[q]];
            } else {
                cid[q] = 0;
                cdir[q] = -1;
                clen[q] = 0;
                cw[q] = 0;
            }
        }
        for (int b = 0; b <= lo; ++b) {
            bool have[kFastChildren];
            int64_t bk[kFastChildren], bV[kFastChildren];
            int32_t bZ[kFastChildren];
            uint8_t bl[kFastChildren];
#pragma unroll
            for (int q = 0; q < kFastChildren; ++q) {
                have[q] = q >= k;   // absent children never block a stack
                bk[q] = 0;
                bV[q] = 0;
                bZ[q] = 0;
                bl[q] = 0;
            }
            for (int t = b; t < L; ++t) {
#pragma unroll
                for (int q = 0; q < kFastChildren; ++q) {
                    if (q < k && child_layer_ok(a.tab, cdir[q], t)) {
                        const ChildKey ck = child_key(a, cid[q], clen[q], cw[q], l, t);
                        if (!have[q] || ck.key < bk[q]) {
                            have[q] = true;
                            bk[q] = ck.key;
                            bV[q] = ck.V;
                            bZ[q] = ck.Z;
                            bl[q] = (uint8_t)t;
                        }
                    }
                }
                if (t < hi) continue;
                bool ok = true;
                int64_t sumV = 0, sumZ = 0;
#pragma unroll
                for (int q = 0; q < kFastChildren; ++q) {
                    ok = ok && have[q];
                    sumV += bV[q];
                    sumZ += bZ[q];
                }
                if (!ok) continue;
                if (eval(b, t, sumV, sumZ)) {
#pragma unroll
                    for (int q = 0; q < kFastChildren; ++q) best_sel[q] = bl[q];
                }
            }
        }
    } else {
        // many children: each stack rescans every child (the definition, written out)
        for (int b = 0; b <= lo; ++b)
            for (int t = hi; t < L; ++t) {
                bool ok = true;
                int64_t sumV = 0, sumZ = 0;
                for (int q = 0; q < k && ok; ++q) {
                    const int32_t c = a.T.ch[c0 + q];
                    const int cd = a.T.dir[c];
                    const int32_t cl = a.T.len[c];
                    const int64_t w = a.w.seg_w[c];
                    bool have = false;
                    ChildKey best{0, 0, 0};
                    for (int lc = b; lc <= t; ++lc) {
                        if (!child_layer_ok(a.tab, cd, lc)) continue;
                        const ChildKey ck = child_key(a, c, cl, w, l, lc);
                        if (!have || ck.key < best.key) {
                            have = true;
                            best = ck;
                        }
                    }
                    ok = have;
                    sumV += best.V;
                    sumZ += best.Z;
                }
                if (ok) eval(b, t, sumV, sumZ);
            }
    }

    const int64_t idx = (int64_t)n * a.NA + j;
    a.F[idx] = best_f;
    a.S[idx] = (int32_t)best_S;
    if (!root) a.KA[idx] = best_f + a.w.w_d * ((lam * 2 * (Cs + best_S)) >> 11);
    a.bt[2 * idx] = (uint8_t)best_b;
    a.bt[2 * idx + 1] = (uint8_t)best_t;
    if (k <= kFastChildren) {
        for (int q = 0; q < k; ++q) a.sel[(int64_t)a.T.ch[c0 + q] * kMaxL + l] = best_sel[q];
    } else {
        for (int q = 0; q < k; ++q) {
            const int32_t c = a.T.ch[c0 + q];
            const int cd = a.T.dir[c];
            const int32_t cl = a.T.len[c];
            const int64_t w = a.w.seg_w[c];
            bool have = false;
            int64_t bk = 0;
            int bl = 0;
            for (int lc = best_b; lc <= best_t; ++lc) {
                if (!child_layer_ok(a.tab, cd, lc)) continue;
                const ChildKey ck = child_key(a, c, cl, w, l, lc);
                if (!have || ck.key < bk) {
                    have = true;
                    bk = ck.key;
                    bl = lc;
                }
            }
            a.sel[(int64_t)c * kMaxL + l] = (uint8_t)bl;
        }
    }
}

// Alg. 4 at node n: its layer is the one its parent recorded for the parent's entering
// layer; its via span is the stack recorded for its own entering layer.  Segments
// whose layer changed go to the commit list (old = 255 when there is no previous layer).
__device__ __forceinline__ void trace_node(const DPArgs &a, int32_t n, uint8_t *cur, uint8_t *vlo, uint8_t *vhi,
                                           uint8_t *out_layers, int has_prev, int32_t *chg_node, uint8_t *chg_old,
                                           uint8_t *chg_new, int32_t *chg_count)
{
    const int32_t p = a.T.parent[n];
    int ln = 0, j = 0;
    if (p >= 0) {
        const int lp = a.T.parent[p] < 0 ? 0 : (cur[p] & (kMaxL - 1));
        ln = a.sel[(int64_t)n * kMaxL + lp];
        // the parent's DP recorded a routable layer of n's direction; the masks only keep
        // every index inside its array
        ln = ln < a.tab.L ? ln : 0;
        j = a.tab.jidx[ln] < 0 ? 0 : a.tab.jidx[ln];
    }
    const int64_t idx = (int64_t)n * a.NA + j;
    vlo[n] = a.bt[2 * idx];
    vhi[n] = a.bt[2 * idx + 1];
    const uint8_t old = cur[n];
    cur[n] = (uint8_t)ln;
    if (out_layers) out_layers[n] = (uint8_t)ln;
    if (p >= 0 && (!has_prev || old != ln)) {
        const int32_t pos = atomicAdd(chg_count, 1);
        chg_node[pos] = n;
        chg_old[pos] = has_prev ? old : (uint8_t)255;
        chg_new[pos] = (uint8_t)ln;
    }
}

}  // namespace gapla
