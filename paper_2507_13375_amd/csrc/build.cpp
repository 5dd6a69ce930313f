// la_build_batch: validation, layer-assignment tree construction (a node at every
// bend, Sec. III-B), height levels, per-node attributes and upload.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "la_internal.h"

namespace gapla {

namespace {

struct Pt {
    int32_t x, y;
};

inline int sgn(int32_t v) { return (v > 0) - (v < 0); }

// Turns the polyline of one input edge into its corner points (endpoints
// included).  Returns false for a diagonal piece, a piece that doubles back, or
// an edge of zero length.
bool corners(const std::vector<Pt> &pts, std::vector<Pt> &out)
{
    out.clear();
    int dx = 0, dy = 0;   // direction of the piece that ends at out.back()
    for (const Pt &p : pts) {
        if (!out.empty() && p.x == out.back().x && p.y == out.back().y) continue;
        if (out.empty()) {
            out.push_back(p);
            continue;
        }
        const Pt &q = out.back();
        if (p.x != q.x && p.y != q.y) return false;
        int ndx = sgn(p.x - q.x), ndy = sgn(p.y - q.y);
        if (out.size() >= 2 && ndx == dx && ndy == dy) {
            out.back() = p;           // keeps going straight: no corner at q
            continue;
        }
        if (out.size() >= 2 && ndx == -dx && ndy == -dy) return false;
        out.push_back(p);
        dx = ndx;
        dy = ndy;
    }
    return out.size() >= 2;
}

template <typename T>
la_status upload(T **dst, const std::vector<T> &src)
{
    size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return set_error(LA_ERR_OOM, "hipMalloc failed in la_build_batch");
    if (!src.empty()) LA_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return LA_OK;
}

template <typename T>
la_status alloc(T **dst, size_t n)
{
    hipError_t e = hipMalloc((void **)dst, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return set_error(LA_ERR_OOM, "hipMalloc failed");
    return LA_OK;
}

}  // namespace

la_status build_tab(const la_grid *g, const la_layer_rc *rc, LayerTab &t)
{
    if (!g || !rc || !g->layer_dir || !rc->r_mohm || !rc->c_af || (g->L > 1 && !rc->via_r_mohm))
        return set_error(LA_ERR_INVALID_ARG, "null grid or layer table");
    if (g->L < 1 || g->L > kMaxL || g->X < 1 || g->Y < 1 || g->X > 32767 || g->Y > 32767 || g->min_layer < 0 ||
        g->min_layer >= g->L)
        return set_error(LA_ERR_INVALID_ARG, "grid size or layer count out of range (L <= 16, X, Y <= 32767)");
    if ((int64_t)g->X * g->Y * g->L >= (int64_t(1) << 31))
        return set_error(LA_ERR_RANGE, "grid index X*Y*L must stay below 2^31");
    memset(&t, 0, sizeof(t));
    t.L = g->L;
    t.min_layer = g->min_layer;
    t.X = g->X;
    t.Y = g->Y;
    int64_t vsum = 0;
    t.pv[0] = 0;
    for (int l = 0; l < g->L; ++l) {
        if (g->layer_dir[l] > 1) return set_error(LA_ERR_INVALID_ARG, "layer_dir must be 0 or 1");
        if (rc->r_mohm[l] < 0 || rc->c_af[l] < 0) return set_error(LA_ERR_INVALID_ARG, "negative unit R or C");
        t.dir[l] = g->layer_dir[l];
        t.r[l] = rc->r_mohm[l];
        t.c[l] = rc->c_af[l];
        t.jidx[l] = -1;
        if (l + 1 < g->L) {
            if (rc->via_r_mohm[l] < 0) return set_error(LA_ERR_INVALID_ARG, "negative via R");
            vsum += rc->via_r_mohm[l];
        }
        t.pv[l + 1] = (int32_t)std::min<int64_t>(vsum, INT32_MAX);
    }
    if (vsum >= (int64_t(1) << 24)) return set_error(LA_ERR_RANGE, "total via resistance must stay below 2^24 mOhm");
    for (int l = g->min_layer; l < g->L; ++l) {
        int d = t.dir[l];
        if (t.nA[d] >= kMaxA) return set_error(LA_ERR_INVALID_ARG, "more than 8 routable layers in one direction");
        t.jidx[l] = (int8_t)t.nA[d];
        t.lay[d][t.nA[d]++] = (int8_t)l;
    }
    for (int d = 0; d < 2; ++d) {
        int64_t sr = 0, sc = 0;
        for (int j = 0; j < t.nA[d]; ++j) {
            sr += t.r[t.lay[d][j]];
            sc += t.c[t.lay[d][j]];
        }
        t.r_avg[d] = t.nA[d] ? (int32_t)(sr / t.nA[d]) : 0;
        t.c_avg[d] = t.nA[d] ? (int32_t)(sc / t.nA[d]) : 0;
    }
    const int64_t P = (int64_t)t.X * t.Y;
    int nr = 0;
    for (int l = 0; l < g->L; ++l) t.nrk[l] = (int8_t)(t.jidx[l] < 0 ? nr++ : 0);
    for (int d = 0; d < 2; ++d) t.nAp[d] = (t.nA[d] + 1) & ~1;
    if ((int64_t)(t.nAp[0] + t.nAp[1] + nr) * P >= (int64_t(1) << 31))
        return set_error(LA_ERR_INVALID_ARG, "grid too large for 32-bit edge indices");
    t.goff[0] = 0;
    t.goff[1] = (int32_t)(t.nAp[0] * P);
    t.goff[2] = (int32_t)((t.nAp[0] + t.nAp[1]) * P);
    return LA_OK;
}

la_status build_batch(const la_nets *nets, const la_grid *grid, const la_layer_rc *layer_rc, const uint8_t *edge_caps,
                      void *stream, la_batch **out)
{
    if (!out) return set_error(LA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!nets || !edge_caps) return set_error(LA_ERR_INVALID_ARG, "nets or edge_caps is NULL");
    LayerTab tab;
    la_status st = build_tab(grid, layer_rc, tab);
    if (st != LA_OK) return st;
    const int32_t N = nets->num_nets, NN = nets->num_nodes;
    if (N < 0 || NN < 0 || nets->num_waypoints < 0) return set_error(LA_ERR_INVALID_ARG, "negative size");
    if (N > 0 && (!nets->net_node_ptr || !nets->node_parent || !nets->node_x || !nets->node_y || !nets->node_flags ||
                  !nets->node_cpin_af || !nets->edge_wp_ptr || !nets->net_budget_fs || !nets->net_rdrv_mohm ||
                  (nets->num_waypoints > 0 && (!nets->wp_x || !nets->wp_y))))
        return set_error(LA_ERR_INVALID_ARG, "a la_nets array is NULL");
    const int32_t X = tab.X, Y = tab.Y, L = tab.L;
    if (N > 0 && (nets->net_node_ptr[0] != 0 || nets->net_node_ptr[N] != NN))
        return set_error(LA_ERR_INVALID_ARG, "net_node_ptr must run from 0 to num_nodes");
    if (NN > 0 && (nets->edge_wp_ptr[0] != 0 || nets->edge_wp_ptr[NN] != nets->num_waypoints))
        return set_error(LA_ERR_INVALID_ARG, "edge_wp_ptr must run from 0 to num_waypoints");

    // ---- pass 1: validate every net and count its layer-assignment nodes -------
    std::vector<int64_t> la_count(N + 1, 0);
    std::vector<Pt> pts, cor;
    std::vector<int32_t> stack, seen;
    auto bad = [&](int32_t net, const char *why) {
        return set_error(LA_ERR_BAD_TREE, "net " + std::to_string(net) + ": " + why);
    };
    int64_t total = 0;
    for (int32_t i = 0; i < N; ++i) {
        const int32_t b0 = nets->net_node_ptr[i], n = nets->net_node_ptr[i + 1] - b0;
        if (n < 1) return bad(i, "net has no node");
        int64_t bends = 0;
        for (int32_t k = 0; k < n; ++k) {
            const int32_t v = b0 + k;
            const int x = nets->node_x[v], y = nets->node_y[v];
            if (x < 0 || x >= X || y < 0 || y >= Y) return bad(i, "node outside the grid");
            const uint8_t f = nets->node_flags[v];
            const bool drv = f & 2, snk = f & 1;
            if (drv && snk) return bad(i, "node is both driver and sink");
            if (k == 0) {
                if (nets->node_parent[v] != -1 || !drv) return bad(i, "node 0 must be the driver, with parent -1");
                continue;
            }
            if (drv) return bad(i, "more than one driver");
            const int32_t p = nets->node_parent[v];
            if (p < 0 || p >= n || p == k) return bad(i, "parent index out of range");
            const int32_t w0 = nets->edge_wp_ptr[v], w1 = nets->edge_wp_ptr[v + 1];
            if (w1 < w0) return bad(i, "edge_wp_ptr decreases");
            pts.clear();
            pts.push_back({nets->node_x[b0 + p], nets->node_y[b0 + p]});
            for (int32_t w = w0; w < w1; ++w) {
                if (nets->wp_x[w] < 0 || nets->wp_x[w] >= X || nets->wp_y[w] < 0 || nets->wp_y[w] >= Y)
                    return bad(i, "waypoint outside the grid");
                pts.push_back({nets->wp_x[w], nets->wp_y[w]});
            }
            pts.push_back({x, y});
            if (!corners(pts, cor)) return bad(i, "edge is diagonal, doubles back or has zero length");
            bends += (int64_t)cor.size() - 2;
        }
        // every node must hang below the driver: walk children from node 0
        seen.assign(n, 0);
        std::vector<int32_t> first(n, -1), nxt(n, -1);
        for (int32_t k = n - 1; k >= 1; --k) {
            int32_t p = nets->node_parent[b0 + k];
            nxt[k] = first[p];
            first[p] = k;
        }
        stack.assign(1, 0);
        int32_t reached = 0;
        while (!stack.empty()) {
            int32_t u = stack.back();
            stack.pop_back();
            if (seen[u]) return bad(i, "cycle");
            seen[u] = 1;
            ++reached;
            for (int32_t c = first[u]; c >= 0; c = nxt[c]) stack.push_back(c);
        }
        if (reached != n) return bad(i, "node not connected to the driver (cycle)");
        la_count[i] = n + bends;
        total += n + bends;
    }
    if (total >= INT32_MAX / 2) return set_error(LA_ERR_RANGE, "too many layer-assignment nodes for int32 indices");

    // ---- pass 2: emit nodes in canonical order ----------------------------------
    const int64_t M = total;
    std::vector<int32_t> parent(M), xs(M), ys(M), len(M, 0), netof(M), cpin(M, 0), net_ptr(N + 1);
    std::vector<uint8_t> dir(M, 0), flags(M, 0);
    int64_t pos = 0;
    for (int32_t i = 0; i < N; ++i) {
        const int32_t b0 = nets->net_node_ptr[i], n = nets->net_node_ptr[i + 1] - b0;
        const int64_t base = pos;
        net_ptr[i] = (int32_t)base;
        int64_t bend = base + n;
        for (int32_t k = 0; k < n; ++k) {
            const int32_t v = b0 + k;
            const int64_t g = base + k;
            xs[g] = nets->node_x[v];
            ys[g] = nets->node_y[v];
            netof[g] = i;
            const uint8_t f = nets->node_flags[v];
            flags[g] = (uint8_t)((f & 1 ? kSink : 0) | (f & 2 ? kDriver | kRoot : 0));
            cpin[g] = (f & 1) ? nets->node_cpin_af[v] : 0;
            parent[g] = -1;
        }
        for (int32_t k = 1; k < n; ++k) {
            const int32_t v = b0 + k, p = nets->node_parent[v];
            pts.clear();
            pts.push_back({nets->node_x[b0 + p], nets->node_y[b0 + p]});
            for (int32_t w = nets->edge_wp_ptr[v]; w < nets->edge_wp_ptr[v + 1]; ++w)
                pts.push_back({nets->wp_x[w], nets->wp_y[w]});
            pts.push_back({nets->node_x[v], nets->node_y[v]});
            corners(pts, cor);
            int64_t up = base + p;
            for (size_t j = 1; j < cor.size(); ++j) {
                const bool last = j + 1 == cor.size();
                const int64_t g = last ? base + k : bend++;
                if (!last) {
                    xs[g] = cor[j].x;
                    ys[g] = cor[j].y;
                    netof[g] = i;
                }
                parent[g] = (int32_t)up;
                len[g] = std::abs(cor[j].x - cor[j - 1].x) + std::abs(cor[j].y - cor[j - 1].y);
                dir[g] = cor[j].y == cor[j - 1].y ? 0 : 1;
                up = g;
            }
        }
        pos = base + la_count[i];
    }
    net_ptr[N] = (int32_t)M;

    // a direction with segments needs at least one routable layer
    for (int64_t v = 0; v < M; ++v)
        if (parent[v] >= 0 && tab.nA[dir[v]] == 0)
            return set_error(LA_ERR_BAD_TREE, "a segment's direction has no routable layer");

    // ---- children, sinks, heights, r_est, grid offsets ------------------------------
    std::vector<int32_t> ch_ptr(M + 1, 0), chl(std::max<int64_t>(M, 1)), sink_id(M, -1), sink_node;
    std::vector<int32_t> net_sink_ptr(N + 1, 0), height(M, 0), rest(M, 0), g0(M, 0);
    for (int64_t v = 0; v < M; ++v)
        if (parent[v] >= 0) ch_ptr[parent[v] + 1]++;
    for (int64_t v = 0; v < M; ++v) ch_ptr[v + 1] += ch_ptr[v];
    {
        std::vector<int32_t> fill(ch_ptr.begin(), ch_ptr.end() - 1);
        for (int64_t v = 0; v < M; ++v)
            if (parent[v] >= 0) chl[fill[parent[v]]++] = (int32_t)v;
    }
    sink_node.reserve(M / 2 + 1);
    for (int32_t i = 0; i < N; ++i) {
        net_sink_ptr[i] = (int32_t)sink_node.size();
        for (int32_t v = net_ptr[i]; v < net_ptr[i + 1]; ++v)
            if (flags[v] & kSink) {
                sink_id[v] = (int32_t)sink_node.size();
                sink_node.push_back(v);
            }
    }
    net_sink_ptr[N] = (int32_t)sink_node.size();
    const int64_t S = (int64_t)sink_node.size();

    int32_t max_h = 0, max_net = 0;
    int64_t gcell = 0;
    double bc = 0, bcap = 0, bvia = 0, bd = 0;
    int32_t cmax = 0, rmax = 0;
    for (int l = 0; l < L; ++l) {
        cmax = std::max(cmax, tab.c[l]);
        rmax = std::max(rmax, tab.r[l]);
    }
    std::vector<int32_t> order;
    for (int32_t i = 0; i < N; ++i) {
        const int32_t b0 = net_ptr[i], n = net_ptr[i + 1] - b0;
        max_net = std::max(max_net, n);
        // pre-order from the root (parents before children)
        order.clear();
        stack.assign(1, b0);
        while (!stack.empty()) {
            int32_t u = stack.back();
            stack.pop_back();
            order.push_back(u);
            for (int32_t j = ch_ptr[u]; j < ch_ptr[u + 1]; ++j) stack.push_back(chl[j]);
        }
        int64_t sum_len = 0, max_len = 0, sum_cpin = 0;
        for (int32_t u : order) {
            const int32_t p = parent[u];
            if (p >= 0) {
                rest[u] = (int32_t)std::min<int64_t>(
                    INT32_MAX, (int64_t)rest[p] + (parent[p] >= 0 ? (int64_t)tab.r_avg[dir[p]] * len[p] : 0));
                sum_len += len[u];
                max_len = std::max<int64_t>(max_len, len[u]);
                const int32_t xl = dir[u] == 0 ? std::min(xs[p], xs[u]) : xs[u];
                const int32_t yl = dir[u] == 0 ? ys[u] : std::min(ys[p], ys[u]);
                g0[u] = plane_pos(tab, dir[u], xl, yl);
            }
            sum_cpin += cpin[u];
        }
        for (size_t j = order.size(); j-- > 0;) {
            const int32_t u = order[j];
            int32_t h = 0;
            for (int32_t q = ch_ptr[u]; q < ch_ptr[u + 1]; ++q) h = std::max(h, height[chl[q]] + 1);
            height[u] = h;
            max_h = std::max(max_h, h);
        }
        gcell += sum_len;
        // worst cases of the fixed-point terms of this net
        const double Smax = (double)sum_cpin + (double)cmax * (double)sum_len;
        const double Xmax = (double)cmax * (double)max_len + 2.0 * Smax;
        const double Rmax = (double)rmax * (double)max_len + (double)tab.pv[L - 1 < 0 ? 0 : L - 1];
        int64_t max_rest = 0;
        for (int32_t u : order) max_rest = std::max<int64_t>(max_rest, rest[u]);
        if (Smax >= 1073741824.0 || Rmax >= 2147483648.0 || max_rest >= INT32_MAX)
            return set_error(LA_ERR_RANGE, "net " + std::to_string(i) + ": wire too long for 32-bit R or C sums");
        const double Tmax = Rmax * Xmax / 2048.0;
        const double LAmax = 2147483647.0 * 2.0 * Smax / 2048.0;
        bc = std::max(bc, (double)n * (double)max_len * (double)(kLutSat + kHistSat));
        bcap = std::max(bcap, (double)cmax * (double)sum_len);
        bvia = std::max(bvia, (double)n * L);
        bd = std::max(bd, (double)n * (3.0 * Tmax + 2.0 * LAmax));
    }

    // ---- nodes grouped by height (stable in canonical order) ---------------------
    std::vector<int32_t> level_ptr(max_h + 2, 0), level_nodes(std::max<int64_t>(M, 1));
    for (int64_t v = 0; v < M; ++v) level_ptr[height[v] + 1]++;
    for (int h = 0; h <= max_h; ++h) level_ptr[h + 1] += level_ptr[h];
    {
        std::vector<int32_t> fill(level_ptr.begin(), level_ptr.end() - 1);
        for (int64_t v = 0; v < M; ++v) level_nodes[fill[height[v]]++] = (int32_t)v;
    }

    // ---- Elmore tiles: runs of whole nets in canonical order -- one wavefront's run of at
    // most kWTile nodes for nets of at most kWTile nodes, one workgroup's run of at most kETile
    // nodes (heights below kEMaxH) for the larger ones; the other nets' nodes grouped by height
    std::vector<int32_t> etile, wtile, ebig_ptr(max_h + 2, 0), ebig_nodes;
    {
        std::vector<char> ebig(std::max<int32_t>(N, 1), 0);
        int32_t t0 = -1, tn = 0, w0 = -1, wn = 0;
        for (int32_t i = 0; i < N; ++i) {
            const int32_t b0 = net_ptr[i], n = net_ptr[i + 1] - b0;
            int32_t hm = 0;
            for (int32_t v = b0; v < b0 + n; ++v) hm = std::max(hm, height[v]);
            // a run is a contiguous node range: a net of the other class closes it
            if (n <= kWTile) {
                if (t0 >= 0) {
                    etile.push_back(t0);
                    etile.push_back(t0 + tn);
                    t0 = -1;
                    tn = 0;
                }
                if (w0 >= 0 && wn + n > kWTile) {
                    wtile.push_back(w0);
                    wtile.push_back(w0 + wn);
                    w0 = -1;
                    wn = 0;
                }
                if (w0 < 0) w0 = b0;
                wn += n;
                continue;
            }
            if (w0 >= 0) {
                wtile.push_back(w0);
                wtile.push_back(w0 + wn);
                w0 = -1;
                wn = 0;
            }
            const bool big = n > kETile || hm >= kEMaxH;
            if (t0 >= 0 && (big || tn + n > kETile)) {
                etile.push_back(t0);
                etile.push_back(t0 + tn);
                t0 = -1;
                tn = 0;
            }
            if (big) {
                ebig[i] = 1;
                for (int32_t v = b0; v < b0 + n; ++v) ebig_ptr[height[v] + 1]++;
                continue;
            }
            if (t0 < 0) t0 = b0;
            tn += n;
        }
        if (t0 >= 0) {
            etile.push_back(t0);
            etile.push_back(t0 + tn);
        }
        if (w0 >= 0) {
            wtile.push_back(w0);
            wtile.push_back(w0 + wn);
        }
        for (int h = 0; h <= max_h; ++h) ebig_ptr[h + 1] += ebig_ptr[h];
        ebig_nodes.resize(std::max<int32_t>(ebig_ptr[max_h + 1], 1));
        std::vector<int32_t> fill(ebig_ptr.begin(), ebig_ptr.end() - 1);
        for (int32_t i = 0; i < N; ++i)
            if (ebig[i])
                for (int32_t v = net_ptr[i]; v < net_ptr[i + 1]; ++v) ebig_nodes[fill[height[v]]++] = v;
    }

    // ---- batched form: nets with more nodes than one LDS tile, nodes grouped by height ---
    std::vector<int32_t> net_big(std::max<int32_t>(N, 1), -1), bn_order, bn_lvl, bn_lvl_off, bn_nlev;
    for (int32_t i = 0; i < N; ++i) {
        const int32_t b0 = net_ptr[i], n = net_ptr[i + 1] - b0;
        if (n <= kBigMin) continue;
        net_big[i] = (int32_t)bn_nlev.size();
        int32_t hmax = 0;
        for (int32_t v = b0; v < b0 + n; ++v) hmax = std::max(hmax, height[v]);
        std::vector<int32_t> cnt(hmax + 2, 0);
        for (int32_t v = b0; v < b0 + n; ++v) cnt[height[v] + 1]++;
        for (int32_t h = 0; h <= hmax; ++h) cnt[h + 1] += cnt[h];
        const int32_t base = (int32_t)bn_order.size();
        bn_order.resize(base + n);
        bn_lvl_off.push_back((int32_t)bn_lvl.size());
        bn_nlev.push_back(hmax + 1);
        for (int32_t h = 0; h <= hmax + 1; ++h) bn_lvl.push_back(base + cnt[h]);
        for (int32_t v = b0; v < b0 + n; ++v) bn_order[base + cnt[height[v]]++] = v;
    }

    // ---- algorithmic work of one DP round and of the Elmore sweeps -------------------
    // Enumeration (Alg. 3): an entering layer l of node v takes the stacks [b, t] holding l
    // (and the pin layer 0 at pins); each stack folds every child's best layer (an int64
    // add and compare/select, 6 VALU ops) and prices the stack (10 ops).  Bytes: node
    // inputs, congestion gathers (demand 4 B, capacity 1 B, history 4 B per GCell edge and
    // routable layer, Eq. 3) and the chosen layer and via span.
    double dp_ops = 0, dp_bytes = 0, dp_ops_above[3] = {0, 0, 0};
    for (int32_t i = 0; i < N; ++i) {
        double ops = 0;
        for (int64_t v = net_ptr[i]; v < net_ptr[i + 1]; ++v) {
            const int k = ch_ptr[v + 1] - ch_ptr[v];
            const bool pin = (flags[v] & (kSink | kDriver)) != 0;
            const double per_stack = 6.0 * k + 10.0;
            if (parent[v] < 0) {
                ops += (double)L * per_stack;
            } else {
                const int d = dir[v];
                for (int j = 0; j < tab.nA[d]; ++j) {
                    const int l = tab.lay[d][j];
                    const int lo = pin ? 0 : l;
                    ops += (double)(lo + 1) * (double)(L - l) * per_stack;
                }
                dp_bytes += 9.0 * (double)len[v] * (double)tab.nA[d];
            }
            dp_bytes += 25.0 + 3.0 + ((flags[v] & kSink) ? 6.0 : 0.0);
        }
        dp_ops += ops;
        for (int c = 0; c < 3; ++c)
            if (net_ptr[i + 1] - net_ptr[i] > kTileCaps[c]) dp_ops_above[c] += ops;
    }
    dp_bytes += 9.0 * (double)N;

    // ---- allocate and upload --------------------------------------------------------
    la_batch *b = new la_batch();
    b->dp_ops = dp_ops;
    b->dp_bytes = dp_bytes;
    for (int c = 0; c < 3; ++c) b->dp_ops_above[c] = dp_ops_above[c];
    b->el_fwd_bytes = 28.0 * (double)(M + S);
    b->el_bwd_bytes = 40.0 * (double)(M + S);
    b->stream = (hipStream_t)stream;
    {
        const hipError_t e = hipGetDevice(&b->device);
        if (e != hipSuccess) {
            delete b;
            return hip_fail(e, "hipGetDevice");
        }
    }
    b->tab = tab;
    b->nets = N;
    b->nodes = M;
    b->sinks = S;
    b->E = (int64_t)X * Y * L;
    b->Eg = tab.goff[2] + (int64_t)(L - tab.nA[0] - tab.nA[1]) * X * Y;
    b->levels = max_h + 1;
    b->max_net_nodes = max_net;
    b->gcell_edges = gcell;
    b->NAmax = std::max(1, std::max(tab.nA[0], tab.nA[1]));
    b->bnd_cong = bc;
    b->bnd_cap = bcap;
    b->bnd_via = bvia;
    b->bnd_d = bd;
    b->h_level_ptr = level_ptr;
    b->h_ebig_ptr = ebig_ptr;
    b->e_ntiles = (int32_t)(etile.size() / 2);
    b->e_nwtiles = (int32_t)(wtile.size() / 2);
    b->h_net_ptr = net_ptr;
    b->h_bbox.resize((size_t)4 * N);
    for (int32_t i = 0; i < N; ++i) {
        int32_t x0 = INT32_MAX, x1 = -1, y0 = INT32_MAX, y1 = -1;
        for (int32_t v = net_ptr[i]; v < net_ptr[i + 1]; ++v) {
            x0 = std::min(x0, xs[v]);
            x1 = std::max(x1, xs[v]);
            y0 = std::min(y0, ys[v]);
            y1 = std::max(y1, ys[v]);
        }
        int16_t *bb = &b->h_bbox[(size_t)4 * i];
        bb[0] = (int16_t)x0;
        bb[1] = (int16_t)x1;
        bb[2] = (int16_t)y0;
        bb[3] = (int16_t)y1;
    }
    std::vector<int32_t> budget(nets->net_budget_fs, nets->net_budget_fs + N);
    std::vector<int32_t> rdrv(nets->net_rdrv_mohm, nets->net_rdrv_mohm + N);
    // capacities in the plane layout
    std::vector<uint8_t> caps(b->Eg, 0);
    for (int32_t y = 0; y < Y; ++y)
        for (int32_t x = 0; x < X; ++x)
            for (int l = 0; l < L; ++l)
                caps[grid_index(tab, l, plane_pos(tab, tab.dir[l], x, y))] = edge_caps[((int64_t)y * X + x) * L + l];
    la_status s = LA_OK;
    auto chk = [&](la_status r) {
        if (s == LA_OK && r != LA_OK) s = r;
    };
    chk(upload(&b->parent, parent));
    chk(upload(&b->ch_ptr, ch_ptr));
    chk(upload(&b->ch, chl));
    chk(upload(&b->net, netof));
    chk(upload(&b->net_ptr, net_ptr));
    chk(upload(&b->len, len));
    chk(upload(&b->g0, g0));
    chk(upload(&b->cpin, cpin));
    chk(upload(&b->sink_id, sink_id));
    chk(upload(&b->sink_node, sink_node));
    chk(upload(&b->net_sink_ptr, net_sink_ptr));
    b->h_net_sink_ptr = net_sink_ptr;
    chk(upload(&b->rest, rest));
    chk(upload(&b->budget_fs, budget));
    chk(upload(&b->rdrv, rdrv));
    {
        // the budgets (ps) and driver resistances (kOhm) in single precision, each rounded once
        std::vector<float> bp(std::max<int32_t>(N, 1), 0.f), rk(std::max<int32_t>(N, 1), 0.f);
        for (int32_t i = 0; i < N; ++i) {
            bp[i] = (float)((double)budget[i] * 1e-3);
            rk[i] = (float)((double)rdrv[i] * 1e-6);
        }
        chk(upload(&b->budget_ps, bp));
        chk(upload(&b->rdrv_k, rk));
    }
    chk(upload(&b->dir, dir));
    chk(upload(&b->flags, flags));
    chk(upload(&b->level_nodes, level_nodes));
    chk(upload(&b->level_ptr, level_ptr));
    chk(upload(&b->e_tile, etile));
    {
        // wavefront runs: lane slot p of a run (p = lane + 64 j) takes the run's node of rank p by
        // height (ties in node order), so each level's nodes fill as few slots as possible
        const size_t nr = wtile.size() / 2;
        std::vector<int32_t> wrun(std::max<size_t>(nr, 1) * 4, 0);
        std::vector<int32_t> wpos((size_t)std::max<int64_t>(M, 1) * 4, 0);
        std::vector<uint8_t> wchl((size_t)std::max<int64_t>(M, 1), 0);
        std::vector<int32_t> rank;
        for (size_t r = 0; r < nr; ++r) {
            const int32_t n0 = wtile[2 * r], n1 = wtile[2 * r + 1], q0 = ch_ptr[n0], q1 = ch_ptr[n1];
            const int32_t nn = n1 - n0;
            rank.resize(nn);
            for (int32_t u = 0; u < nn; ++u) rank[u] = u;
            std::stable_sort(rank.begin(), rank.end(),
                             [&](int32_t x, int32_t y) { return height[n0 + x] < height[n0 + y]; });
            for (int32_t p = 0; p < nn; ++p) {
                const int32_t v = n0 + rank[p];
                const uint32_t pl = parent[v] < 0 ? 0u : (uint32_t)(parent[v] - n0 + 1);
                int32_t *w = &wpos[(size_t)4 * (n0 + p)];
                w[0] = (int32_t)((uint32_t)height[v] | pl << 8 | (uint32_t)(ch_ptr[v] - q0) << 16 |
                                 (uint32_t)(ch_ptr[v + 1] - ch_ptr[v]) << 24);
                w[1] = rank[p];
                w[2] = sink_id[v];
                const float cp = (float)((double)cpin[v] * 1e-3);
                std::memcpy(&w[3], &cp, 4);
            }
            for (int32_t q = q0; q < q1; ++q) wchl[q] = (uint8_t)(chl[q] - n0);
            const int32_t mh = height[n0 + rank[nn - 1]];
            const int32_t s0max = height[n0 + rank[std::min(nn, 64) - 1]];
            const int32_t s1min = nn > 64 ? height[n0 + rank[64]] : 255;
            wrun[4 * r] = n0;
            wrun[4 * r + 1] =
                (int32_t)((uint32_t)nn | (uint32_t)mh << 8 | (uint32_t)s0max << 16 | (uint32_t)s1min << 24);
            wrun[4 * r + 2] = q0;
            wrun[4 * r + 3] = q1 - q0;
        }
        static_assert(kWTile <= 128, "run-local ids, heights and child offsets fit a byte");
        chk(upload(&b->e_wrun, wrun));
        chk(upload(&b->e_wpos, wpos));
        chk(upload(&b->e_wchl, wchl));
    }
    {
        // pin loads in fF as single precision, rounded once from the exact product
        std::vector<float> cf(std::max<int64_t>(M, 1), 0.f);
        for (int64_t v = 0; v < M; ++v) cf[v] = (float)((double)cpin[v] * 1e-3);
        chk(upload(&b->cpin_ff, cf));
    }
    chk(upload(&b->e_big_nodes, ebig_nodes));
    chk(upload(&b->e_big_ptr, ebig_ptr));
    chk(upload(&b->height, height));
    {
        // one 16-byte record per node for the batched form's tiles (fields hold for nets of at
        // most 256 nodes, the only ones a tile stages): in-plane first GCell edge; length and
        // parent offset inside the net; pin load; child count, flags | direction << 4, height
        // and the offset of the node's first child entry inside the net's entries
        std::vector<uint32_t> rec((size_t)std::max<int64_t>(M, 1) * 4, 0);
        for (int32_t i = 0; i < N; ++i) {
            const int32_t n0 = net_ptr[i], c0 = ch_ptr[n0];
            for (int32_t v = n0; v < net_ptr[i + 1]; ++v) {
                uint32_t *r = &rec[(size_t)4 * v];
                const int32_t po = parent[v] < 0 ? 0xffff : ((parent[v] - n0) & 0xffff);
                r[0] = (uint32_t)g0[v];
                r[1] = ((uint32_t)len[v] & 0xffffu) | ((uint32_t)po << 16);
                r[2] = (uint32_t)cpin[v];
                r[3] = (uint32_t)std::min(ch_ptr[v + 1] - ch_ptr[v], 255) | ((uint32_t)(flags[v] | dir[v] << 4) << 8) |
                       ((uint32_t)std::min(height[v], 255) << 16) | ((uint32_t)std::min(ch_ptr[v] - c0, 255) << 24);
            }
        }
        chk(upload(&b->nrec, rec));
    chk(upload(&b->bbox, b->h_bbox));
    chk(alloc(&b->batch_i32, std::max<int64_t>(N, 1)));
    }
    chk(alloc(&b->dynrec, (size_t)std::max<int64_t>(M, 1) * 2));
    chk(alloc(&b->cnet, (size_t)std::max<int64_t>(N, 1) * 4));
    chk(alloc(&b->bucket_nodes, M));
    b->n_big = (int32_t)bn_nlev.size();
    chk(upload(&b->net_big, net_big));
    chk(upload(&b->bn_order, bn_order));
    chk(alloc(&b->bn_rec, 12 * std::max<size_t>(bn_order.size(), 1)));
    chk(upload(&b->bn_lvl, bn_lvl));
    chk(upload(&b->bn_lvl_off, bn_lvl_off));
    chk(upload(&b->bn_nlev, bn_nlev));
    chk(alloc(&b->tier_nets, std::max<int64_t>(N, 1)));
    chk(alloc(&b->net_zw, std::max<int64_t>(N, 1)));
    // batch partition of the batched form: up to 256 batches x kPartBuckets buckets (+ error counter)
    chk(alloc(&b->tier_off, 256 * kPartBuckets + 2));
    chk(alloc(&b->tier_cur, 256 * kPartBuckets + 2));
    chk(alloc(&b->tier_cnt, 256 * kPartBuckets + 2));
    // claims: every claim but the last of a batch covers kClaimUnits units
    chk(alloc(&b->cl_pre, (size_t)N + 1));
    chk(alloc(&b->cl_blk, (size_t)N / 1024 + 2));
    b->cl_start_cap = (M + (int64_t)kNetUnits * N) / kClaimUnitsMin + 2 * 256 + 2;
    chk(alloc(&b->cl_start, (size_t)b->cl_start_cap));
    chk(alloc(&b->cl_off, 256 + 2));
    chk(upload(&b->caps, caps));
    chk(alloc(&b->D, b->Eg));
    chk(alloc(&b->D_alt, b->Eg));
    chk(alloc(&b->Hi, b->Eg));
    chk(alloc(&b->cur_layer, M));
    chk(alloc(&b->vlo, M));
    chk(alloc(&b->vhi, M));
    chk(alloc(&b->F, M * b->NAmax));
    chk(alloc(&b->S, M * b->NAmax));
    chk(alloc(&b->bt, M * b->NAmax));
    chk(alloc(&b->sel, M * b->NAmax + kMaxA));   // rows of NAmax, padded for the clamped index
    chk(alloc(&b->chg_node, M));
    chk(alloc(&b->chg_old, M));
    chk(alloc(&b->chg_new, M));
    chk(alloc(&b->chg_count, 4));
    chk(alloc(&b->lut, (size_t)L * 2 * kNDelta));
    chk(alloc(&b->R, M + S));
    chk(alloc(&b->C, M + S));
    chk(alloc(&b->el_S, M));
    chk(alloc(&b->el_Slo, M));
    chk(alloc(&b->el_t, M));
    chk(alloc(&b->el_tlo, M));
    chk(alloc(&b->el_G, M));
    chk(alloc(&b->el_Glo, M));
    chk(alloc(&b->el_Siglo, M));
    chk(alloc(&b->el_Sig, M));
    chk(alloc(&b->slack, S));
    chk(alloc(&b->scratch_f, S));
    chk(alloc(&b->wns_bits, 4));
    b->red_blocks = 1024;
    chk(alloc(&b->red, (size_t)b->red_blocks * 4));
    chk(alloc(&b->qofw, (size_t)kMaxL + 2 * (2 * kQSpan + 1)));
    chk(alloc(&b->qpart, (size_t)kQPartials));
    if (s != LA_OK) {
        la_free_batch(b);
        return s;
    }
    // initial contents; any failure from here on frees the whole batch
    auto init = [&]() -> la_status {
        std::vector<int32_t> lut((size_t)L * 2 * kNDelta);
        la_default_cong_lut(L, nullptr, lut.data());
        LA_HIP(hipMemcpy(b->lut, lut.data(), lut.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        LA_HIP(hipMemsetAsync(b->F, 0, M * b->NAmax * sizeof(int64_t), b->stream));
        LA_HIP(hipMemsetAsync(b->S, 0, M * b->NAmax * sizeof(int32_t), b->stream));
        LA_HIP(hipMemsetAsync(b->bt, 0, M * b->NAmax, b->stream));
        LA_HIP(hipMemsetAsync(b->sel, 0, M * b->NAmax + kMaxA, b->stream));
        LA_HIP(hipMemsetAsync(b->D, 0, b->Eg * sizeof(int32_t), b->stream));
        LA_HIP(hipMemsetAsync(b->Hi, 0, b->Eg * sizeof(int32_t), b->stream));   // record padding stays 0
        LA_HIP(hipMemsetAsync(b->cur_layer, 0, M, b->stream));
        LA_HIP(hipMemsetAsync(b->vlo, 0, M, b->stream));
        LA_HIP(hipMemsetAsync(b->vhi, 0, M, b->stream));
        // address of the static scratch on this device (la_timing_summary_noalloc)
        const la_status ss = scratch_setup(b->device);
        if (ss != LA_OK) return ss;
        return launch_rc_pre(b);
    };
    const la_status r = init();
    if (r != LA_OK) {
        la_free_batch(b);
        return r;
    }
    *out = b;
    return LA_OK;
}

}  // namespace gapla
