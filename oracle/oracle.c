/*
 * ORACLE -- test infrastructure only.  A plain, slow, obviously-correct CPU
 * statement of the GAP-LA layer-assignment hot path (Zhao, Guo, Zhang, Lin,
 * "GAP-LA: GPU-Accelerated Performance-Driven Layer Assignment").  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.  It shares no code with the HIP library.
 *
 * What it computes, with the passage each part follows:
 *   - the layer-assignment directed tree: a node at every bend so that no
 *     tree edge bends and layers change only at nodes (Sec. III-B, Fig. graph_b);
 *   - the Elmore delay of the RC tree of a net in FP64, pi-model wire
 *     segments, the driver as a resistor at the root, pins hung on
 *     zero-capacitance edges (Sec. II-C, Sec. III-B, Fig. rc; the d34 example);
 *   - the reverse (adjoint) sweep of that Elmore pass (not in the paper: the
 *     exact derivative of a weighted TNS with respect to each R and C);
 *   - pin weights as a logistic of slack/WNS with k = 10, b = 0.3 (Eq. 4,
 *     read as the logistic the text and Fig. cost describe) and edge weights
 *     as the maximum over the sinks of the downstream subtree (Eq. 5);
 *   - the integer congestion cost built from the marginal of the exponential
 *     overflow of Eq. 3;
 *   - the tree dynamic program of Alg. 2-3 with the look-ahead cost of
 *     Sec. III-D (f' = f + w_d r_est c) and the trace-back of Alg. 4;
 *   - the batch schedule of Alg. 2: batches in order, each batch assigned
 *     against one demand snapshot and then committed, and negotiation rounds
 *     with a history cost (prior art the paper cites in Sec. I);
 *   - the objective J(a) of a complete assignment and a brute-force minimum
 *     over every layer combination of a small net;
 *   - the quality terms of a routing solution: total overflow with the
 *     exponential per-edge overflow of Eq. 3 and with the clipped difference of
 *     Eq. 2, the via count and the wire capacitance that stands for power in
 *     the weighted score of Eq. 1 (Sec. II).
 *
 * Fixed-point conventions: R in mOhm, C in aF, via R in mOhm, all int32;
 * costs in int64.  T(w, R, X) = (w * ((R * X) >> 11)) >> 10 with w in Q10 and
 * X = 2 x capacitance (so the pi-model half stays an integer).  Timing in FP64
 * with R in kOhm and C in fF, so delays come out in ps.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <limits.h>
#include <omp.h>

#define O_OK 0
#define O_ERR_INVALID_ARG -1
#define O_ERR_BAD_TREE -2
#define O_ERR_RANGE -3
#define O_ERR_OOM -4

#define OMAXL 16
#define NDELTA 64
#define DELTA_MIN (-32)
#define LUT_SAT (1 << 20)
#define HIST_SAT (1 << 24)

/* ------------------------------------------------------------------------- */
/* The layer-assignment tree of every net, nodes in canonical order:          */
/* per net, the input nodes in input order, then the bend nodes in the order  */
/* of the input edge they split (edge parent(v)->v in order of v), each edge's */
/* bends from the parent end to the child end.                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nets, nodes, sinks;
    int64_t *net_ptr;      /* [nets+1] */
    int64_t *parent;       /* global index, -1 at the driver */
    int32_t *x, *y;
    int32_t *len;          /* length of segment parent->node in GCells (0 at the root) */
    int8_t *dir;           /* 0 horizontal, 1 vertical, -1 at the root */
    uint8_t *is_sink, *is_driver;
    int32_t *cpin;         /* sink load, aF */
    int64_t *sink_of;      /* node -> sink index, -1 otherwise */
    int64_t *sink_node;    /* [sinks] */
    int64_t *net_of;       /* node -> net */
    int64_t *ch_ptr, *ch;  /* children, ascending canonical index */
    int32_t *budget_fs, *rdrv_mohm;  /* per net */
} otree;

void oracle_tree_free(otree *t)
{
    if (!t) return;
    free(t->net_ptr); free(t->parent); free(t->x); free(t->y); free(t->len); free(t->dir);
    free(t->is_sink); free(t->is_driver); free(t->cpin); free(t->sink_of); free(t->sink_node);
    free(t->net_of); free(t->ch_ptr); free(t->ch); free(t->budget_fs); free(t->rdrv_mohm);
    free(t);
}

typedef struct { int32_t x, y; } pt;

/* Simplify the polyline pts[0..n) (drop repeated points, merge collinear runs).
 * Returns the number of corner points kept in out (endpoints included), or -1 if
 * a piece is diagonal, reverses, or the whole edge has zero length. */
static int simplify(const pt *pts, int n, pt *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (m > 0 && pts[i].x == out[m - 1].x && pts[i].y == out[m - 1].y) continue;
        if (m > 0 && pts[i].x != out[m - 1].x && pts[i].y != out[m - 1].y) return -1;
        if (m >= 2) {
            /* direction of last piece and of the new one */
            int dx0 = (out[m - 1].x > out[m - 2].x) - (out[m - 1].x < out[m - 2].x);
            int dy0 = (out[m - 1].y > out[m - 2].y) - (out[m - 1].y < out[m - 2].y);
            int dx1 = (pts[i].x > out[m - 1].x) - (pts[i].x < out[m - 1].x);
            int dy1 = (pts[i].y > out[m - 1].y) - (pts[i].y < out[m - 1].y);
            if (dx0 == dx1 && dy0 == dy1) { out[m - 1] = pts[i]; continue; }   /* straight on */
            if (dx0 == -dx1 && dy0 == -dy1) return -1;                          /* doubles back */
        }
        out[m++] = pts[i];
    }
    return m >= 2 ? m : -1;
}

/* Build the layer-assignment trees.  Returns O_OK or an error; *bad_net names
 * the first net that failed validation. */
int oracle_tree_build(int64_t nets, const int32_t *net_node_ptr, const int32_t *node_parent,
                      const int16_t *node_x, const int16_t *node_y, const uint8_t *node_flags,
                      const int32_t *node_cpin, const int32_t *edge_wp_ptr, const int16_t *wp_x,
                      const int16_t *wp_y, const int32_t *budget_fs, const int32_t *rdrv_mohm,
                      int32_t X, int32_t Y, otree **out, int64_t *bad_net)
{
    *out = NULL;
    *bad_net = -1;
    if (nets < 0) return O_ERR_INVALID_ARG;
    /* pass 1: validate and count nodes after bend insertion */
    int64_t total = 0, sinks = 0;
    int64_t *cnt = (int64_t *)calloc((size_t)nets + 1, sizeof(int64_t));
    if (!cnt) return O_ERR_OOM;
    pt *buf = NULL, *simp = NULL; int bufcap = 0;
    int rc = O_OK;
    for (int64_t i = 0; i < nets && rc == O_OK; ++i) {
        int64_t b0 = net_node_ptr[i], b1 = net_node_ptr[i + 1], n = b1 - b0;
        if (n < 1) { rc = O_ERR_BAD_TREE; *bad_net = i; break; }
        int64_t extra = 0;
        for (int64_t k = 0; k < n; ++k) {
            int64_t v = b0 + k;
            if (node_x[v] < 0 || node_x[v] >= X || node_y[v] < 0 || node_y[v] >= Y) { rc = O_ERR_BAD_TREE; break; }
            int drv = (node_flags[v] >> 1) & 1, snk = node_flags[v] & 1;
            if (drv && snk) { rc = O_ERR_BAD_TREE; break; }
            if ((k == 0) != (node_parent[v] == -1) || (k == 0) != (drv == 1)) { rc = O_ERR_BAD_TREE; break; }
            if (snk) ++sinks;
            if (k == 0) continue;
            if (node_parent[v] < 0 || node_parent[v] >= n || node_parent[v] == k) { rc = O_ERR_BAD_TREE; break; }
            int nw = edge_wp_ptr[v + 1] - edge_wp_ptr[v];
            if (nw < 0) { rc = O_ERR_BAD_TREE; break; }
            if (nw + 2 > bufcap) {
                bufcap = nw + 2;
                buf = (pt *)realloc(buf, sizeof(pt) * (size_t)bufcap);
                simp = (pt *)realloc(simp, sizeof(pt) * (size_t)bufcap);
                if (!buf || !simp) { rc = O_ERR_OOM; break; }
            }
            int64_t u = b0 + node_parent[v];
            buf[0].x = node_x[u]; buf[0].y = node_y[u];
            for (int j = 0; j < nw; ++j) {
                int32_t wx = wp_x[edge_wp_ptr[v] + j], wy = wp_y[edge_wp_ptr[v] + j];
                if (wx < 0 || wx >= X || wy < 0 || wy >= Y) { rc = O_ERR_BAD_TREE; break; }
                buf[1 + j].x = wx; buf[1 + j].y = wy;
            }
            if (rc) break;
            buf[nw + 1].x = node_x[v]; buf[nw + 1].y = node_y[v];
            int m = simplify(buf, nw + 2, simp);
            if (m < 0) { rc = O_ERR_BAD_TREE; break; }
            extra += m - 2;
        }
        if (rc == O_OK) {
            /* every node must reach the driver without a cycle */
            for (int64_t k = 1; k < n; ++k) {
                int64_t u = k, steps = 0;
                while (u != 0 && steps <= n) { u = node_parent[b0 + u]; ++steps; }
                if (u != 0) { rc = O_ERR_BAD_TREE; break; }
            }
        }
        if (rc != O_OK) { if (rc == O_ERR_BAD_TREE) *bad_net = i; break; }
        cnt[i] = n + extra;
        total += n + extra;
    }
    if (rc != O_OK) { free(cnt); free(buf); free(simp); return rc; }

    otree *t = (otree *)calloc(1, sizeof(otree));
    if (!t) { free(cnt); free(buf); free(simp); return O_ERR_OOM; }
    t->nets = nets; t->nodes = total; t->sinks = sinks;
    t->net_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nets + 1));
    t->parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total + 1));
    t->x = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    t->y = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    t->len = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total + 1));
    t->dir = (int8_t *)malloc((size_t)(total + 1));
    t->is_sink = (uint8_t *)calloc((size_t)(total + 1), 1);
    t->is_driver = (uint8_t *)calloc((size_t)(total + 1), 1);
    t->cpin = (int32_t *)calloc((size_t)(total + 1), sizeof(int32_t));
    t->sink_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total + 1));
    t->sink_node = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sinks + 1));
    t->net_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total + 1));
    t->ch_ptr = (int64_t *)calloc((size_t)(total + 2), sizeof(int64_t));
    t->ch = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total + 1));
    t->budget_fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nets + 1));
    t->rdrv_mohm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nets + 1));
    if (!t->net_ptr || !t->parent || !t->x || !t->y || !t->len || !t->dir || !t->is_sink || !t->is_driver ||
        !t->cpin || !t->sink_of || !t->sink_node || !t->net_of || !t->ch_ptr || !t->ch || !t->budget_fs ||
        !t->rdrv_mohm) {
        oracle_tree_free(t); free(cnt); free(buf); free(simp); return O_ERR_OOM;
    }
    /* pass 2: emit nodes */
    int64_t pos = 0;
    for (int64_t i = 0; i < nets; ++i) {
        int64_t b0 = net_node_ptr[i], n = net_node_ptr[i + 1] - b0;
        int64_t base = pos, next_bend = base + n;
        t->net_ptr[i] = base;
        t->budget_fs[i] = budget_fs[i];
        t->rdrv_mohm[i] = rdrv_mohm[i];
        for (int64_t k = 0; k < n; ++k) {
            int64_t v = b0 + k, g = base + k;
            t->x[g] = node_x[v]; t->y[g] = node_y[v];
            t->is_sink[g] = node_flags[v] & 1;
            t->is_driver[g] = (node_flags[v] >> 1) & 1;
            t->cpin[g] = t->is_sink[g] ? node_cpin[v] : 0;
            t->net_of[g] = i;
            t->parent[g] = -1; t->len[g] = 0; t->dir[g] = -1;
        }
        for (int64_t k = 1; k < n; ++k) {
            int64_t v = b0 + k, u = b0 + node_parent[v];
            int nw = edge_wp_ptr[v + 1] - edge_wp_ptr[v];
            buf[0].x = node_x[u]; buf[0].y = node_y[u];
            for (int j = 0; j < nw; ++j) { buf[1 + j].x = wp_x[edge_wp_ptr[v] + j]; buf[1 + j].y = wp_y[edge_wp_ptr[v] + j]; }
            buf[nw + 1].x = node_x[v]; buf[nw + 1].y = node_y[v];
            int m = simplify(buf, nw + 2, simp);
            int64_t prev = base + node_parent[v];
            for (int j = 1; j < m; ++j) {
                int64_t g = (j == m - 1) ? base + k : next_bend++;
                if (j < m - 1) {
                    t->x[g] = simp[j].x; t->y[g] = simp[j].y;
                    t->is_sink[g] = 0; t->is_driver[g] = 0; t->cpin[g] = 0; t->net_of[g] = i;
                }
                t->parent[g] = prev;
                t->len[g] = abs(simp[j].x - simp[j - 1].x) + abs(simp[j].y - simp[j - 1].y);
                t->dir[g] = simp[j].y == simp[j - 1].y ? 0 : 1;
                prev = g;
            }
        }
        pos = base + cnt[i];
    }
    t->net_ptr[nets] = pos;
    free(cnt); free(buf); free(simp);
    /* sinks and children in canonical order */
    int64_t s = 0;
    for (int64_t v = 0; v < total; ++v) {
        t->sink_of[v] = t->is_sink[v] ? s : -1;
        if (t->is_sink[v]) t->sink_node[s++] = v;
        if (t->parent[v] >= 0) t->ch_ptr[t->parent[v] + 1]++;
    }
    for (int64_t v = 0; v < total; ++v) t->ch_ptr[v + 1] += t->ch_ptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total + 1));
    if (!fill) { oracle_tree_free(t); return O_ERR_OOM; }
    memcpy(fill, t->ch_ptr, sizeof(int64_t) * (size_t)total);
    for (int64_t v = 0; v < total; ++v)
        if (t->parent[v] >= 0) t->ch[fill[t->parent[v]]++] = v;
    free(fill);
    *out = t;
    return O_OK;
}

void oracle_tree_sizes(const otree *t, int64_t *nets, int64_t *nodes, int64_t *sinks)
{
    *nets = t->nets; *nodes = t->nodes; *sinks = t->sinks;
}

void oracle_tree_export(const otree *t, int64_t *net_ptr, int64_t *parent, int32_t *x, int32_t *y, int32_t *len,
                        int8_t *dir, uint8_t *is_sink, int64_t *sink_node)
{
    memcpy(net_ptr, t->net_ptr, sizeof(int64_t) * (size_t)(t->nets + 1));
    memcpy(parent, t->parent, sizeof(int64_t) * (size_t)t->nodes);
    memcpy(x, t->x, sizeof(int32_t) * (size_t)t->nodes);
    memcpy(y, t->y, sizeof(int32_t) * (size_t)t->nodes);
    memcpy(len, t->len, sizeof(int32_t) * (size_t)t->nodes);
    memcpy(dir, t->dir, (size_t)t->nodes);
    memcpy(is_sink, t->is_sink, (size_t)t->nodes);
    memcpy(sink_node, t->sink_node, sizeof(int64_t) * (size_t)t->sinks);
}

/* ------------------------------------------------------------------------- */
/* Technology and weights                                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t X, Y, L, min_layer;
    const uint8_t *layer_dir;         /* [L] */
    const int32_t *r, *c, *vr;        /* [L], [L], [L-1] : mOhm/GCell, aF/GCell, mOhm per via */
    int64_t w_cong, w_cap, w_d, w_via;
    const uint16_t *seg_w;            /* [nodes] Q10 edge weight of the segment parent->node */
    const uint16_t *pin_w;            /* [sinks] Q10 */
    const int32_t *lambda;            /* [nodes] look-ahead coefficient, weighted mOhm */
    const int32_t *lut;               /* [L][2][64] congestion marginal cost */
} oparams;

/* via resistance between layers a and b: sum of the upper-via R of the layers crossed */
static int64_t rvia(const oparams *P, int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    int64_t s = 0;
    for (int k = lo; k < hi; ++k) s += P->vr[k];
    return s;
}

/* allowed layers of a segment of direction d */
static int allowed(const oparams *P, int d, int l) { return l >= P->min_layer && P->layer_dir[l] == d; }

/* T(w, R, X): the weighted delay term, floors as written (operands are non-negative) */
static int64_t Tq(int64_t w, int64_t R, int64_t X) { return (w * ((R * X) >> 11)) >> 10; }

/* Congestion marginal cost of Eq. 3: K ofw (e^{s(d+1)} - e^{s d}) for d = D - Cap clamped
 * to [-32, 31]; s = 0.5 if Cap > 0 and 1.5 if Cap = 0; K = 1024; saturates at 2^20. */
void oracle_cong_lut(int32_t L, const double *ofw, int32_t *lut)
{
    for (int32_t l = 0; l < L; ++l)
        for (int z = 0; z < 2; ++z) {
            double s = z == 0 ? 0.5 : 1.5;
            for (int i = 0; i < NDELTA; ++i) {
                double d = (double)(i + DELTA_MIN);
                double v = 1024.0 * ofw[l] * (exp(s * (d + 1.0)) - exp(s * d));
                lut[(l * 2 + z) * NDELTA + i] = v >= (double)LUT_SAT ? LUT_SAT : (int32_t)nearbyint(v);
            }
        }
}

/* grid index of the k-th GCell edge covered by the segment parent->v on layer l */
static int64_t seg_edge(const oparams *P, const otree *T, int64_t v, int64_t k, int l)
{
    int64_t p = T->parent[v];
    int32_t x, y;
    if (T->dir[v] == 0) { x = (T->x[p] < T->x[v] ? T->x[p] : T->x[v]) + (int32_t)k; y = T->y[v]; }
    else { x = T->x[v]; y = (T->y[p] < T->y[v] ? T->y[p] : T->y[v]) + (int32_t)k; }
    return ((int64_t)y * P->X + x) * P->L + l;
}

/* kappa_v(l): congestion cost of putting segment parent->v on layer l against demand D,
 * without the segment's own previous demand when `self_layer` == l. */
static int64_t kappa(const oparams *P, const otree *T, int64_t v, int l, const int32_t *D, const uint8_t *cap,
                     const int32_t *H, int self_layer)
{
    int64_t s = 0;
    for (int64_t k = 0; k < T->len[v]; ++k) {
        int64_t g = seg_edge(P, T, v, k, l);
        int64_t d = (int64_t)D[g] - (self_layer == l ? 1 : 0) - cap[g];
        if (d < DELTA_MIN) d = DELTA_MIN;
        if (d > DELTA_MIN + NDELTA - 1) d = DELTA_MIN + NDELTA - 1;
        int z = cap[g] > 0 ? 0 : 1;
        s += P->lut[(l * 2 + z) * NDELTA + (d - DELTA_MIN)] + (int64_t)H[g];
    }
    return s;
}

int64_t oracle_kappa(const otree *T, const oparams *P, int64_t v, int32_t l, const int32_t *D, const uint8_t *cap,
                     const int32_t *H, int32_t self_layer)
{
    return kappa(P, T, v, l, D, cap, H, self_layer);
}

/* ------------------------------------------------------------------------- */
/* Tree dynamic program of one net (Alg. 3 and Alg. 4).                       */
/* For every node n and every layer l the segment parent->n may take, it      */
/* enumerates the via stacks [b,t] at n that contain l and n's pin layer,     */
/* lets every child c take its best layer inside [b,t] by the look-ahead key, */
/* and keeps the stack with the lowest look-ahead cost f'.                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t F[OMAXL], S[OMAXL];
    int8_t b[OMAXL], t[OMAXL];
    int8_t sel[OMAXL];      /* this node's layer, indexed by its parent's entering layer */
} dpnode;

/* post-order of the subtree at root r (children before parents) */
static int64_t postorder(const otree *T, int64_t r, int64_t *order, int64_t *stack)
{
    int64_t sp = 0, m = 0;
    stack[sp++] = r;
    while (sp) {
        int64_t v = stack[--sp];
        order[m++] = v;
        for (int64_t j = T->ch_ptr[v]; j < T->ch_ptr[v + 1]; ++j) stack[sp++] = T->ch[j];
    }
    /* order holds a pre-order with children reversed; reversing gives a valid post-order */
    for (int64_t i = 0; i < m / 2; ++i) { int64_t tmp = order[i]; order[i] = order[m - 1 - i]; order[m - 1 - i] = tmp; }
    return m;
}

static int dp_net(const otree *T, const oparams *P, int64_t net, const int32_t *D, const uint8_t *cap,
                  const int32_t *H, const uint8_t *prev, uint8_t *lay, uint8_t *vlo, uint8_t *vhi, int64_t *froot)
{
    const int L = P->L;
    int64_t b0 = T->net_ptr[net], n = T->net_ptr[net + 1] - b0;
    dpnode *st = (dpnode *)calloc((size_t)n, sizeof(dpnode));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *kap = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * OMAXL);
    int8_t *cur = (int8_t *)malloc((size_t)n);
    if (!st || !order || !stack || !kap || !cur) { free(st); free(order); free(stack); free(kap); free(cur); return O_ERR_OOM; }
    postorder(T, b0, order, stack);
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        if (T->parent[v] < 0) continue;
        for (int l = 0; l < L; ++l)
            if (allowed(P, T->dir[v], l))
                kap[(v - b0) * OMAXL + l] = kappa(P, T, v, l, D, cap, H, prev ? prev[v] : -1);
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i], lv = v - b0;
        int root = T->parent[v] < 0;
        int pin = T->is_sink[v] || T->is_driver[v];
        for (int l = 0; l < L; ++l) {
            if (root ? l != 0 : !allowed(P, T->dir[v], l)) continue;
            int lo = l, hi = l;
            if (pin) { if (0 < lo) lo = 0; if (0 > hi) hi = 0; }
            int64_t best_fp = INT64_MAX, best_f = 0, best_S = 0;
            int best_b = -1, best_t = -1;
            for (int b = 0; b <= lo; ++b)
                for (int t = hi; t < L; ++t) {
                    int64_t sumV = 0, Sn = T->cpin[v];
                    int ok = 1;
                    for (int64_t j = T->ch_ptr[v]; j < T->ch_ptr[v + 1] && ok; ++j) {
                        int64_t c = T->ch[j], lc_ = c - b0;
                        int bl = -1; int64_t bkey = 0;
                        for (int lc = b; lc <= t; ++lc) {
                            if (!allowed(P, T->dir[c], lc)) continue;
                            int64_t Z = (int64_t)P->c[lc] * T->len[c] + st[lc_].S[lc];
                            int64_t Xc = (int64_t)P->c[lc] * T->len[c] + 2 * st[lc_].S[lc];
                            int64_t key = st[lc_].F[lc] + P->w_d * Tq(P->seg_w[c], rvia(P, l, lc), Xc) +
                                          P->w_d * (((int64_t)P->lambda[c] * 2 * Z) >> 11);
                            if (bl < 0 || key < bkey) { bl = lc; bkey = key; }
                        }
                        if (bl < 0) { ok = 0; break; }
                        int64_t Xc = (int64_t)P->c[bl] * T->len[c] + 2 * st[lc_].S[bl];
                        sumV += st[lc_].F[bl] + P->w_d * Tq(P->seg_w[c], rvia(P, l, bl), Xc);
                        Sn += (int64_t)P->c[bl] * T->len[c] + st[lc_].S[bl];
                    }
                    if (!ok) continue;
                    int64_t f = P->w_via * (t - b) + sumV;
                    if (T->is_sink[v])
                        f += P->w_d * Tq(P->pin_w[T->sink_of[v]], rvia(P, l, 0), 2 * (int64_t)T->cpin[v]);
                    int64_t fp = f;
                    if (!root) {
                        int64_t Cs = (int64_t)P->c[l] * T->len[v];
                        f += P->w_cong * kap[lv * OMAXL + l] + P->w_cap * Cs +
                             P->w_d * Tq(P->seg_w[v], (int64_t)P->r[l] * T->len[v], Cs + 2 * Sn);
                        fp = f + P->w_d * (((int64_t)P->lambda[v] * 2 * (Cs + Sn)) >> 11);
                    }
                    if (fp < best_fp) { best_fp = fp; best_f = f; best_S = Sn; best_b = b; best_t = t; }
                }
            if (best_b < 0) { free(st); free(order); free(stack); free(kap); free(cur); return O_ERR_BAD_TREE; }
            st[lv].F[l] = best_f; st[lv].S[l] = best_S; st[lv].b[l] = (int8_t)best_b; st[lv].t[l] = (int8_t)best_t;
            /* record each child's layer at the chosen stack (same rule as above) */
            for (int64_t j = T->ch_ptr[v]; j < T->ch_ptr[v + 1]; ++j) {
                int64_t c = T->ch[j], lc_ = c - b0;
                int bl = -1; int64_t bkey = 0;
                for (int lc = best_b; lc <= best_t; ++lc) {
                    if (!allowed(P, T->dir[c], lc)) continue;
                    int64_t Z = (int64_t)P->c[lc] * T->len[c] + st[lc_].S[lc];
                    int64_t Xc = (int64_t)P->c[lc] * T->len[c] + 2 * st[lc_].S[lc];
                    int64_t key = st[lc_].F[lc] + P->w_d * Tq(P->seg_w[c], rvia(P, l, lc), Xc) +
                                  P->w_d * (((int64_t)P->lambda[c] * 2 * Z) >> 11);
                    if (bl < 0 || key < bkey) { bl = lc; bkey = key; }
                }
                st[lc_].sel[l] = (int8_t)bl;
            }
        }
    }
    /* trace-back (Alg. 4): the driver enters on its pin layer 0; every child takes the
     * layer recorded for its parent's entering layer; pre-order = reversed post-order */
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t v = order[i], lv = v - b0;
        int lin;
        if (T->parent[v] < 0) lin = 0;
        else lin = st[lv].sel[cur[T->parent[v] - b0]];
        cur[lv] = (int8_t)lin;
        lay[v] = (uint8_t)lin;
        vlo[v] = (uint8_t)st[lv].b[lin];
        vhi[v] = (uint8_t)st[lv].t[lin];
        if (T->parent[v] < 0) *froot = st[lv].F[0];
    }
    free(st); free(order); free(stack); free(kap); free(cur);
    return O_OK;
}

/* Demand of a segment on a layer: +1 on every GCell edge it covers */
static void add_seg(const oparams *P, const otree *T, int64_t v, int l, int32_t *D, int delta)
{
    for (int64_t k = 0; k < T->len[v]; ++k) D[seg_edge(P, T, v, k, l)] += delta;
}

/*
 * The batch schedule.  For r in rounds: for each tier k in order, every net of
 * the tier runs the DP against the same demand D, then their segments are
 * committed (moved from their previous layer when they have one).  After each
 * round: H += hist_inc * max(0, D - Cap), saturating at 2^24.
 *
 * prev/has_prev carry the previous assignment between calls; with has_prev set
 * the DP excludes each segment's own previous demand and commits move demand.
 */
int oracle_assign(const otree *T, const oparams *P, const uint8_t *cap, int32_t *D, int32_t *H, uint8_t *prev,
                  int32_t *has_prev, const int32_t *net_tier, int32_t rounds, int32_t hist_inc, uint8_t *out_layer,
                  uint8_t *out_vlo, uint8_t *out_vhi, int64_t *out_froot)
{
    /* the nets of each batch, in net order (batches are 0..ntier-1) */
    int32_t ntier = 1;
    if (net_tier)
        for (int64_t i = 0; i < T->nets; ++i) {
            if (net_tier[i] < 0) return O_ERR_INVALID_ARG;
            if (net_tier[i] + 1 > ntier) ntier = net_tier[i] + 1;
        }
    int64_t *bstart = (int64_t *)calloc((size_t)ntier + 1, sizeof(int64_t));
    int64_t *bnets = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T->nets > 0 ? T->nets : 1));
    if (!bstart || !bnets) { free(bstart); free(bnets); return O_ERR_OOM; }
    for (int64_t i = 0; i < T->nets; ++i) bstart[(net_tier ? net_tier[i] : 0) + 1]++;
    for (int32_t k = 0; k < ntier; ++k) bstart[k + 1] += bstart[k];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ntier);
        if (!fill) { free(bstart); free(bnets); return O_ERR_OOM; }
        for (int32_t k = 0; k < ntier; ++k) fill[k] = bstart[k];
        for (int64_t i = 0; i < T->nets; ++i) bnets[fill[net_tier ? net_tier[i] : 0]++] = i;
        free(fill);
    }
    int64_t E = (int64_t)P->X * P->Y * P->L;
    for (int32_t r = 0; r < rounds; ++r) {
        for (int32_t k = 0; k < ntier; ++k) {
            int err = O_OK;
            #pragma omp parallel for schedule(dynamic, 64)
            for (int64_t q = bstart[k]; q < bstart[k + 1]; ++q) {
                const int64_t i = bnets[q];
                int e = dp_net(T, P, i, D, cap, H, *has_prev ? prev : NULL, out_layer, out_vlo, out_vhi, &out_froot[i]);
                if (e != O_OK) {
                    #pragma omp critical
                    err = e;
                }
            }
            if (err != O_OK) { free(bstart); free(bnets); return err; }
            for (int64_t q = bstart[k]; q < bstart[k + 1]; ++q) {
                const int64_t i = bnets[q];
                for (int64_t v = T->net_ptr[i]; v < T->net_ptr[i + 1]; ++v) {
                    if (T->parent[v] < 0) continue;
                    if (*has_prev) {
                        if (prev[v] == out_layer[v]) continue;
                        add_seg(P, T, v, prev[v], D, -1);
                    }
                    add_seg(P, T, v, out_layer[v], D, +1);
                }
            }
        }
        for (int64_t v = 0; v < T->nodes; ++v) prev[v] = out_layer[v];
        *has_prev = 1;
        for (int64_t g = 0; g < E; ++g) {
            int64_t over = (int64_t)D[g] - cap[g];
            if (over > 0) {
                int64_t h = (int64_t)H[g] + (int64_t)hist_inc * over;
                H[g] = (int32_t)(h > HIST_SAT ? HIST_SAT : h);
            }
        }
    }
    free(bstart);
    free(bnets);
    return O_OK;
}

/* ------------------------------------------------------------------------- */
/* Objective of a complete assignment, and brute force over small nets        */
/* ------------------------------------------------------------------------- */

/* J of net `net` under assignment lay[] (root entry ignored). */
static int64_t objective(const otree *T, const oparams *P, int64_t net, const uint8_t *lay, const int32_t *D,
                         const uint8_t *cap, const int32_t *H, const uint8_t *prev, int64_t *order, int64_t *stack,
                         int64_t *S)
{
    int64_t b0 = T->net_ptr[net], n = T->net_ptr[net + 1] - b0;
    postorder(T, b0, order, stack);
    int64_t J = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        int64_t s = T->cpin[v];
        for (int64_t j = T->ch_ptr[v]; j < T->ch_ptr[v + 1]; ++j) {
            int64_t c = T->ch[j];
            s += (int64_t)P->c[lay[c]] * T->len[c] + S[c - b0];
        }
        S[v - b0] = s;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        int root = T->parent[v] < 0;
        int lin = root ? 0 : lay[v];
        if (!root) {
            int64_t Cs = (int64_t)P->c[lin] * T->len[v];
            int64_t Xs = Cs + 2 * S[v - b0];
            int64_t p = T->parent[v];
            int lpar = T->parent[p] < 0 ? 0 : lay[p];
            J += P->w_cong * kappa(P, T, v, lin, D, cap, H, prev ? prev[v] : -1) + P->w_cap * Cs;
            J += P->w_d * (Tq(P->seg_w[v], (int64_t)P->r[lin] * T->len[v], Xs) +
                           Tq(P->seg_w[v], rvia(P, lpar, lin), Xs));
        }
        if (T->is_sink[v]) J += P->w_d * Tq(P->pin_w[T->sink_of[v]], rvia(P, lin, 0), 2 * (int64_t)T->cpin[v]);
        int mn = lin, mx = lin;
        if (T->is_sink[v] || T->is_driver[v]) { if (0 < mn) mn = 0; if (0 > mx) mx = 0; }
        for (int64_t j = T->ch_ptr[v]; j < T->ch_ptr[v + 1]; ++j) {
            int a = lay[T->ch[j]];
            if (a < mn) mn = a;
            if (a > mx) mx = a;
        }
        J += P->w_via * (mx - mn);
    }
    return J;
}

int oracle_objective(const otree *T, const oparams *P, const uint8_t *lay, const int32_t *D, const uint8_t *cap,
                     const int32_t *H, const uint8_t *prev, int64_t *out_J)
{
    int err = O_OK;
    #pragma omp parallel
    {
        int64_t mx = 1;
        for (int64_t i = 0; i < T->nets; ++i) { int64_t n = T->net_ptr[i + 1] - T->net_ptr[i]; if (n > mx) mx = n; }
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        if (!order || !stack || !S) {
            #pragma omp critical
            err = O_ERR_OOM;
        } else {
            #pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < T->nets; ++i) out_J[i] = objective(T, P, i, lay, D, cap, H, prev, order, stack, S);
        }
        free(order); free(stack); free(S);
    }
    return err;
}

/* Minimum of J over every layer combination of net `net` (at most `max_segs` segments).
 * Returns the minimum in *jmin, one minimiser in best_lay (root entry 0), and the
 * number of minimisers in *n_min. */
int oracle_bruteforce(const otree *T, const oparams *P, int64_t net, int32_t max_segs, const int32_t *D,
                      const uint8_t *cap, const int32_t *H, const uint8_t *prev, int64_t *jmin, uint8_t *best_lay,
                      int64_t *n_min)
{
    int64_t b0 = T->net_ptr[net], n = T->net_ptr[net + 1] - b0;
    if (n - 1 > max_segs || n > 64) return O_ERR_RANGE;
    uint8_t *lay = (uint8_t *)calloc((size_t)T->nodes, 1);
    int64_t order[64], stack[64], S[64];
    int opts[64][OMAXL], nopt[64], idx[64];
    if (!lay) return O_ERR_OOM;
    for (int64_t k = 0; k < n; ++k) {
        int64_t v = b0 + k;
        nopt[k] = 0; idx[k] = 0;
        if (T->parent[v] < 0) { opts[k][nopt[k]++] = 0; continue; }
        for (int l = 0; l < P->L; ++l) if (allowed(P, T->dir[v], l)) opts[k][nopt[k]++] = l;
        if (nopt[k] == 0) { free(lay); return O_ERR_BAD_TREE; }
    }
    *jmin = INT64_MAX; *n_min = 0;
    for (;;) {
        for (int64_t k = 0; k < n; ++k) lay[b0 + k] = (uint8_t)opts[k][idx[k]];
        int64_t J = objective(T, P, net, lay, D, cap, H, prev, order, stack, S);
        if (J < *jmin) {
            *jmin = J; *n_min = 1;
            for (int64_t k = 0; k < n; ++k) best_lay[k] = lay[b0 + k];
        } else if (J == *jmin) {
            ++*n_min;
        }
        int64_t k = 0;
        while (k < n && ++idx[k] == nopt[k]) { idx[k] = 0; ++k; }
        if (k == n) break;
    }
    free(lay);
    return O_OK;
}

/* ------------------------------------------------------------------------- */
/* Elmore delay in FP64 (Sec. II-C; Fig. rc and its d34 example)               */
/* RC index space: [0, nodes) is the segment parent->node (the driver          */
/* resistance at the root), [nodes, nodes+sinks) is the pin edge of sink k.   */
/* ------------------------------------------------------------------------- */

/* integer average over the routable layers of direction d */
static int64_t avg_dir(const oparams *P, const int32_t *v, int d)
{
    int64_t s = 0, m = 0;
    for (int l = 0; l < P->L; ++l) if (allowed(P, d, l)) { s += v[l]; ++m; }
    return m ? s / m : 0;
}

/* R (kOhm) and C (fF) of every RC edge.  lay == NULL: before assignment, the
 * average per-direction unit R and C and zero-resistance pin edges (Sec. III-B).
 * Otherwise a tree segment is the lumped via from the parent's entering layer
 * to the segment layer plus the wire; a pin edge is the via down to layer 0. */
void oracle_rc(const otree *T, const oparams *P, const uint8_t *lay, double *R, double *C)
{
    int64_t ravg[2] = {avg_dir(P, P->r, 0), avg_dir(P, P->r, 1)};
    int64_t cavg[2] = {avg_dir(P, P->c, 0), avg_dir(P, P->c, 1)};
    for (int64_t v = 0; v < T->nodes; ++v) {
        int64_t p = T->parent[v];
        if (p < 0) { R[v] = T->rdrv_mohm[T->net_of[v]] * 1e-6; C[v] = 0.0; continue; }
        if (!lay) {
            R[v] = (double)(ravg[T->dir[v]] * T->len[v]) * 1e-6;
            C[v] = (double)(cavg[T->dir[v]] * T->len[v]) * 1e-3;
        } else {
            int a = lay[v], lp = T->parent[p] < 0 ? 0 : lay[p];
            R[v] = (double)(rvia(P, lp, a) + (int64_t)P->r[a] * T->len[v]) * 1e-6;
            C[v] = (double)((int64_t)P->c[a] * T->len[v]) * 1e-3;
        }
    }
    for (int64_t k = 0; k < T->sinks; ++k) {
        int64_t v = T->sink_node[k];
        R[T->nodes + k] = lay ? (double)rvia(P, lay[v], 0) * 1e-6 : 0.0;
        C[T->nodes + k] = 0.0;
    }
}

/* Forward Elmore: S = downstream capacitance, t = delay at every node, delay at every sink pin. */
void oracle_elmore(const otree *T, const double *R, const double *C, double *S, double *t, double *delay)
{
    #pragma omp parallel
    {
        int64_t mx = 1;
        for (int64_t i = 0; i < T->nets; ++i) { int64_t n = T->net_ptr[i + 1] - T->net_ptr[i]; if (n > mx) mx = n; }
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < T->nets; ++i) {
            int64_t n = postorder(T, T->net_ptr[i], order, stack);
            for (int64_t j = 0; j < n; ++j) {
                int64_t v = order[j];
                double s = 0.0;
                if (T->is_sink[v]) s += C[T->nodes + T->sink_of[v]] + T->cpin[v] * 1e-3;
                for (int64_t q = T->ch_ptr[v]; q < T->ch_ptr[v + 1]; ++q) s += C[T->ch[q]] + S[T->ch[q]];
                S[v] = s;
            }
            for (int64_t j = n - 1; j >= 0; --j) {
                int64_t v = order[j], p = T->parent[v];
                t[v] = (p < 0 ? 0.0 : t[p]) + R[v] * (0.5 * C[v] + S[v]);
                if (T->is_sink[v]) {
                    int64_t k = T->sink_of[v];
                    delay[k] = t[v] + R[T->nodes + k] * (0.5 * C[T->nodes + k] + T->cpin[v] * 1e-3);
                }
            }
        }
        free(order); free(stack);
    }
}

/* Reverse sweep: given gbar[k] = dJ/d delay_k, G = sum of gbar below each edge,
 * Sig = sum over the path from the driver of R*G, and dJ/dR, dJ/dC per RC edge. */
void oracle_elmore_adjoint(const otree *T, const double *R, const double *C, const double *S, const double *gbar,
                           double *G, double *Sig, double *dR, double *dC)
{
    #pragma omp parallel
    {
        int64_t mx = 1;
        for (int64_t i = 0; i < T->nets; ++i) { int64_t n = T->net_ptr[i + 1] - T->net_ptr[i]; if (n > mx) mx = n; }
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)mx);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < T->nets; ++i) {
            int64_t n = postorder(T, T->net_ptr[i], order, stack);
            for (int64_t j = 0; j < n; ++j) {
                int64_t v = order[j];
                double g = 0.0;
                if (T->is_sink[v]) g += gbar[T->sink_of[v]];
                for (int64_t q = T->ch_ptr[v]; q < T->ch_ptr[v + 1]; ++q) g += G[T->ch[q]];
                G[v] = g;
            }
            for (int64_t j = n - 1; j >= 0; --j) {
                int64_t v = order[j], p = T->parent[v];
                double up = p < 0 ? 0.0 : Sig[p];
                Sig[v] = up + R[v] * G[v];
                dR[v] = G[v] * (0.5 * C[v] + S[v]);
                dC[v] = 0.5 * R[v] * G[v] + up;
                if (T->is_sink[v]) {
                    int64_t k = T->sink_of[v], e = T->nodes + k;
                    double load = T->cpin[v] * 1e-3;
                    dR[e] = gbar[k] * (0.5 * C[e] + load);
                    dC[e] = 0.5 * R[e] * gbar[k] + Sig[v];
                }
            }
        }
        free(order); free(stack);
    }
}

/* ------------------------------------------------------------------------- */
/* Timing weights and batches                                                 */
/* ------------------------------------------------------------------------- */

/* Eq. 4 read as a logistic: w = 1 / (1 + exp(-k (slack/WNS - b))), k = 10, b = 0.3,
 * quantised to Q10 with round-half-even; all zero when WNS >= 0. */
static uint16_t pin_weight_q10(double slack, double wns)
{
    if (!(wns < 0.0)) return 0;
    double rho = slack / wns;
    double w = 1.0 / (1.0 + exp(-10.0 * (rho - 0.3)));
    return (uint16_t)nearbyint(1024.0 * w);
}

/* Batch of a net from its slack (the smallest slack of its sinks) relative to WNS:
 * 0 for the worst net, then bins [0.99,1), [0.96,0.99), [0.91,0.96), [0.84,0.91),
 * [0.75,0.84), [0.7,0.75); nets better than 0.7 WNS go to 4 trailing batches by net id. */
static uint8_t tier_of(double nslack, double wns, int64_t net)
{
    if (wns < 0.0) {
        double rho = nslack / wns;
        if (rho >= 1.0) return 0;
        for (int k = 1; k <= 5; ++k) {
            double lo = 1.0 - (k / 10.0) * (k / 10.0);
            if (rho >= lo) return (uint8_t)k;
        }
        if (rho >= 0.7) return 6;
    }
    return (uint8_t)(7 + (net & 3));
}

/* slacks (ps), WNS, per-sink Q10 pin weights and per-net batches from sink delays */
void oracle_slack(const otree *T, const double *delay, double *slack, double *wns_out, uint16_t *pin_w,
                  uint8_t *tier)
{
    double wns = INFINITY;
    for (int64_t k = 0; k < T->sinks; ++k) {
        slack[k] = T->budget_fs[T->net_of[T->sink_node[k]]] * 1e-3 - delay[k];
        if (slack[k] < wns) wns = slack[k];
    }
    *wns_out = wns;
    for (int64_t k = 0; k < T->sinks; ++k) pin_w[k] = pin_weight_q10(slack[k], wns);
    for (int64_t i = 0; i < T->nets; ++i) {
        double ns = INFINITY;
        for (int64_t v = T->net_ptr[i]; v < T->net_ptr[i + 1]; ++v)
            if (T->is_sink[v] && slack[T->sink_of[v]] < ns) ns = slack[T->sink_of[v]];
        tier[i] = tier_of(ns, wns, i);
    }
}

/* Eq. 5: edge weight = largest pin weight in the downstream subtree (a sink at the
 * node itself included); look-ahead coefficient lambda = (w * r_est) >> 10 with r_est
 * the average-R estimate of the wire between the driver and the segment's upper end. */
void oracle_edge_weights(const otree *T, const oparams *P, const uint16_t *pin_w, uint16_t *seg_w, int32_t *lambda)
{
    int64_t ravg[2] = {avg_dir(P, P->r, 0), avg_dir(P, P->r, 1)};
    for (int64_t i = 0; i < T->nets; ++i) {
        int64_t b0 = T->net_ptr[i], n = T->net_ptr[i + 1] - b0;
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        int64_t *rest = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        postorder(T, b0, order, stack);
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = order[j];
            uint16_t w = T->is_sink[v] ? pin_w[T->sink_of[v]] : 0;
            for (int64_t q = T->ch_ptr[v]; q < T->ch_ptr[v + 1]; ++q) if (seg_w[T->ch[q]] > w) w = seg_w[T->ch[q]];
            seg_w[v] = w;
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            int64_t v = order[j], p = T->parent[v];
            /* rest[v] = estimated R from the driver to the lower end of segment v */
            int64_t up = p < 0 ? 0 : rest[p - b0];
            rest[v - b0] = up + (p < 0 ? 0 : ravg[T->dir[v]] * T->len[v]);
            lambda[v] = p < 0 ? 0 : (int32_t)(((int64_t)seg_w[v] * up) >> 10);
        }
        free(order); free(stack); free(rest);
    }
}

/* Adjoint-derived weights: from G (sum of dJ/d delay below each edge, <= 0) and Sig,
 * seg_w = min(1024, rne(-1024 G)), pin_w = min(1024, rne(-1024 gbar)) and
 * lambda = rne(-Sig(parent) * 1e6) in weighted mOhm, clamped to [0, 2^31-1]. */
void oracle_adjoint_weights(const otree *T, const double *G, const double *Sig, const double *gbar, uint16_t *seg_w,
                            uint16_t *pin_w, int32_t *lambda)
{
    for (int64_t v = 0; v < T->nodes; ++v) {
        double q = nearbyint(-1024.0 * G[v]);
        seg_w[v] = (uint16_t)(q < 0 ? 0 : (q > 1024 ? 1024 : q));
        int64_t p = T->parent[v];
        double lam = p < 0 ? 0.0 : nearbyint(-Sig[p] * 1e6);
        lambda[v] = (int32_t)(lam < 0 ? 0 : (lam > 2147483647.0 ? 2147483647.0 : lam));
    }
    for (int64_t k = 0; k < T->sinks; ++k) {
        double q = nearbyint(-1024.0 * gbar[k]);
        pin_w[k] = (uint16_t)(q < 0 ? 0 : (q > 1024 ? 1024 : q));
    }
}

/* Classical batching (Alg. 1, GetBatch: the batching of the routers the paper cites for it).
 * A net's box is the GCell rectangle its nodes span.  Within each subset, in increasing net
 * order, a net joins the lowest-numbered batch in which no net's box shares a GCell with its
 * own (then no two nets of a batch share a GCell edge).  Subsets are batched one after another
 * and never share a batch: the batches of subset s follow those of subsets 0..s-1.  A net with
 * subset < 0 (or >= nsub) gets batch -1.  One X x Y occupancy grid per open batch.  Returns the
 * number of batches, or -1 when memory runs out. */
int64_t oracle_get_batches(const otree *T, int32_t X, int32_t Y, const int32_t *subset, int32_t nsub, int32_t *batch)
{
    const int64_t N = T->nets;
    int32_t *box = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(N > 0 ? N : 1));
    if (!box) return -1;
    for (int64_t i = 0; i < N; ++i) {
        int32_t x0 = INT32_MAX, x1 = -1, y0 = INT32_MAX, y1 = -1;
        for (int64_t v = T->net_ptr[i]; v < T->net_ptr[i + 1]; ++v) {
            if (T->x[v] < x0) x0 = T->x[v];
            if (T->x[v] > x1) x1 = T->x[v];
            if (T->y[v] < y0) y0 = T->y[v];
            if (T->y[v] > y1) y1 = T->y[v];
        }
        box[4 * i] = x0; box[4 * i + 1] = x1; box[4 * i + 2] = y0; box[4 * i + 3] = y1;
        batch[i] = -1;
    }
    int64_t base = 0, ok = 1;
    for (int32_t s = 0; s < nsub && ok; ++s) {
        uint8_t **grid = NULL;   /* occupancy of each open batch of this subset */
        int64_t nb = 0;
        for (int64_t i = 0; i < N && ok; ++i) {
            if (subset[i] != s) continue;
            const int32_t *b = &box[4 * i];
            for (int64_t k = 0;; ++k) {
                if (k == nb) {
                    uint8_t **g2 = (uint8_t **)realloc(grid, sizeof(uint8_t *) * (size_t)(nb + 1));
                    if (!g2) { ok = 0; break; }
                    grid = g2;
                    grid[nb] = (uint8_t *)calloc((size_t)X * Y, 1);
                    if (!grid[nb]) { ok = 0; break; }
                    ++nb;
                }
                int free_here = 1;
                for (int32_t y = b[2]; y <= b[3] && free_here; ++y)
                    for (int32_t x = b[0]; x <= b[1]; ++x)
                        if (grid[k][(int64_t)y * X + x]) { free_here = 0; break; }
                if (!free_here) continue;
                for (int32_t y = b[2]; y <= b[3]; ++y)
                    for (int32_t x = b[0]; x <= b[1]; ++x) grid[k][(int64_t)y * X + x] = 1;
                batch[i] = (int32_t)(base + k);
                break;
            }
        }
        for (int64_t k = 0; k < nb; ++k) free(grid[k]);
        free(grid);
        base += nb;
    }
    free(box);
    return ok ? base : -1;
}

/*
 * Static timing of a gate-level graph over the nets (Alg. 1, its first step) and the
 * critical-path count that follows it.  Each net is driven by one gate (delay gate_fs); each sink feeds the gate of
 * net sink_next (or is a primary output, -1).  Single precision, each value rounded once as
 * written (max and min are exact), so decisions taken from it (a gate's latest input, the bins
 * of Alg. 1) come out the same in any evaluation order:
 *   arrival at the driver of net m:  AD[m] = gd[m] + (max over sinks s feeding m of AS[s]; 0 if none)
 *   arrival at sink s of net n:     AS[s] = AD[n] + delay[s]
 *   required at sink s:             RS[s] = clock (primary output) or RD[next[s]] - gd[next[s]]
 *   required at the driver of n:    RD[n] = min over n's sinks s of (RS[s] - delay[s])
 *   slack[s] = RS[s] - AS[s];  WNS = min over primary outputs of their slack.
 * gd and clock in ps, each (float)(fs * 1e-3).  The top-1 critical path of every primary output
 * with slack < 0.7 WNS (only when WNS < 0): its net, then back through each gate's latest input
 * (the lowest sink on equal arrival) to a primary input; crit[n] counts the paths through net n.
 * Returns O_ERR_INVALID_ARG for a cycle or a sink_next outside the nets.
 */
int oracle_sta(const otree *T, const int32_t *sink_next, const int32_t *gate_fs, int32_t clock_fs,
               const float *delay, float *slack, int32_t *crit, float *wns_out)
{
    const int64_t N = T->nets, S = T->sinks;
    int64_t *indeg = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *fin_ptr = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *fin = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    int64_t *topo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    float *AD = (float *)malloc(sizeof(float) * (size_t)(N > 0 ? N : 1));
    float *RD = (float *)malloc(sizeof(float) * (size_t)(N > 0 ? N : 1));
    float *AS = (float *)malloc(sizeof(float) * (size_t)(S > 0 ? S : 1));
    float *RS = (float *)malloc(sizeof(float) * (size_t)(S > 0 ? S : 1));
    int rc = O_OK;
    if (!indeg || !fin_ptr || !fin || !topo || !AD || !RD || !AS || !RS) { rc = O_ERR_OOM; goto done; }
    /* fan-in of each net's gate: the sinks that feed it, ascending */
    for (int64_t k = 0; k < S; ++k) {
        if (sink_next[k] >= N || sink_next[k] < -1) { rc = O_ERR_INVALID_ARG; goto done; }
        if (sink_next[k] >= 0) fin_ptr[sink_next[k] + 1]++;
    }
    for (int64_t m = 0; m < N; ++m) fin_ptr[m + 1] += fin_ptr[m];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
        if (!fill) { rc = O_ERR_OOM; goto done; }
        for (int64_t m = 0; m < N; ++m) fill[m] = fin_ptr[m];
        for (int64_t k = 0; k < S; ++k)
            if (sink_next[k] >= 0) fin[fill[sink_next[k]]++] = k;
        free(fill);
    }
    /* topological order of the nets (Kahn): a net after every net whose sink feeds its gate */
    for (int64_t m = 0; m < N; ++m) indeg[m] = fin_ptr[m + 1] - fin_ptr[m];
    {
        int64_t head = 0, tail = 0;
        for (int64_t m = 0; m < N; ++m) if (indeg[m] == 0) topo[tail++] = m;
        while (head < tail) {
            const int64_t n = topo[head++];
            for (int64_t v = T->net_ptr[n]; v < T->net_ptr[n + 1]; ++v) {
                const int64_t k = T->sink_of[v];
                if (k < 0 || sink_next[k] < 0) continue;
                if (--indeg[sink_next[k]] == 0) topo[tail++] = sink_next[k];
            }
        }
        if (tail != N) { rc = O_ERR_INVALID_ARG; goto done; }
    }
    /* arrival times in topological order */
    for (int64_t q = 0; q < N; ++q) {
        const int64_t m = topo[q];
        float in = 0.0f;
        for (int64_t j = fin_ptr[m]; j < fin_ptr[m + 1]; ++j) if (AS[fin[j]] > in) in = AS[fin[j]];
        AD[m] = (float)((double)gate_fs[m] * 1e-3) + in;
        for (int64_t v = T->net_ptr[m]; v < T->net_ptr[m + 1]; ++v)
            if (T->sink_of[v] >= 0) AS[T->sink_of[v]] = AD[m] + delay[T->sink_of[v]];
    }
    /* required times in reverse topological order */
    const float clock = (float)((double)clock_fs * 1e-3);
    for (int64_t q = N - 1; q >= 0; --q) {
        const int64_t n = topo[q];
        float rd = INFINITY;
        for (int64_t v = T->net_ptr[n]; v < T->net_ptr[n + 1]; ++v) {
            const int64_t k = T->sink_of[v];
            if (k < 0) continue;
            const int32_t m = sink_next[k];
            RS[k] = m < 0 ? clock : RD[m] - (float)((double)gate_fs[m] * 1e-3);
            const float r = RS[k] - delay[k];
            if (r < rd) rd = r;
        }
        RD[n] = rd;
    }
    float wns = INFINITY;
    for (int64_t k = 0; k < S; ++k) {
        slack[k] = RS[k] - AS[k];
        if (sink_next[k] < 0 && slack[k] < wns) wns = slack[k];
    }
    *wns_out = wns;
    for (int64_t n = 0; n < N; ++n) crit[n] = 0;
    if (wns < 0.0f) {
        const float lim = 0.7f * wns;
        for (int64_t k = 0; k < S; ++k) {
            if (sink_next[k] >= 0 || !(slack[k] < lim)) continue;
            int64_t n = T->net_of[T->sink_node[k]];
            for (;;) {
                crit[n] += 1;
                int64_t best = -1;
                for (int64_t j = fin_ptr[n]; j < fin_ptr[n + 1]; ++j)
                    if (best < 0 || AS[fin[j]] > AS[best]) best = fin[j];   /* fin is ascending */
                if (best < 0) break;
                n = T->net_of[T->sink_node[best]];
            }
        }
    }
done:
    free(indeg); free(fin_ptr); free(fin); free(topo); free(AD); free(RD); free(AS); free(RS);
    return rc;
}

/*
 * Alg. 1 division and partition: divide the nets and partition the timing-critical ones into ordered
 * subsets.  Net slack = the minimum slack over the net's sinks.  Critical nets (N_c): more than
 * three counted critical paths; with C the largest count, subset k holds the counts c with
 * C / 2^k <= c < C / 2^(k-1) (subset 0: c = C).  Semi-critical nets (N_s): the other nets whose
 * net slack is below 0.7 WNS, by rho = slack / WNS: 1, [0.99, 1), [0.96, 0.99), [0.91, 0.96),
 * [0.84, 0.91), [0.75, 0.84), [0.7, 0.75) (single precision, as the bins of the weights).  The
 * rest (N_n) form one subset.  Subsets: the critical ones 0..kc-1, the seven slack bins, then
 * the non-critical one; returns their number (kc + 8).
 */
int32_t oracle_alg1_subsets(const otree *T, const float *slack, const int32_t *crit, float wns, int32_t *subset)
{
    const int64_t N = T->nets;
    int32_t C = 0;
    for (int64_t n = 0; n < N; ++n) if (crit[n] > 3 && crit[n] > C) C = crit[n];
    int32_t kc = 0;
    for (int64_t n = 0; n < N; ++n) {
        if (crit[n] <= 3) continue;
        int32_t k = 0;
        while (((int64_t)crit[n] << k) < C) ++k;
        if (k + 1 > kc) kc = k + 1;
    }
    static const float lo[7] = {1.0f, 0.99f, 0.96f, 0.91f, 0.84f, 0.75f, 0.7f};
    for (int64_t n = 0; n < N; ++n) {
        if (crit[n] > 3) {
            int32_t k = 0;
            while (((int64_t)crit[n] << k) < C) ++k;
            subset[n] = k;
            continue;
        }
        float ns = INFINITY;
        for (int64_t v = T->net_ptr[n]; v < T->net_ptr[n + 1]; ++v)
            if (T->sink_of[v] >= 0 && slack[T->sink_of[v]] < ns) ns = slack[T->sink_of[v]];
        int32_t b = 7;   /* non-critical */
        if (wns < 0.0f && ns < 0.7f * wns) {
            const float rho = ns / wns;
            b = 6;
            for (int j = 0; j < 7; ++j) if (rho >= lo[j]) { b = j; break; }
        }
        subset[n] = kc + b;
    }
    return kc + 8;
}

/* Threads the OpenMP loops above use (for reporting timings), and a way to change it (the
 * results do not depend on it: per-net work is independent and commits are integer). */
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* Quality terms (Sec. II).  Over every GCell edge g on every layer l, with demand d and
 * capacity c: Eq. 3 overflow ofw(l) e^{s (d - c)}, s = 0.5 when c > 0 and 1.5 when c = 0,
 * summed in FP64 in grid order ((y X + x) L + l); Eq. 2 overflow max(0, d - c) summed, and the
 * number of edges with d > c.  Vias: the via span t - b of every node (Alg. 4's stack).  Wire
 * capacitance: c(layer) * len over every tree segment (aF). */
void oracle_quality(const otree *T, int32_t X, int32_t Y, int32_t L, const int32_t *c_af, const uint8_t *lay,
                    const uint8_t *vlo, const uint8_t *vhi, const int32_t *D, const uint8_t *cap,
                    const double *ofw, double *tof, int64_t *ov_sum, int64_t *ov_edges, int64_t *vias,
                    int64_t *wire_cap)
{
    double t = 0.0;
    int64_t s2 = 0, n2 = 0;
    for (int64_t g = 0; g < (int64_t)X * Y; ++g)
        for (int l = 0; l < L; ++l) {
            const int64_t e = g * L + l;
            const int64_t over = (int64_t)D[e] - (int64_t)cap[e];
            const double s = cap[e] > 0 ? 0.5 : 1.5;
            t += (ofw ? ofw[l] : 1.0) * exp(s * (double)over);
            if (over > 0) {
                s2 += over;
                n2 += 1;
            }
        }
    int64_t nv = 0, wc = 0;
    for (int64_t v = 0; v < T->nodes; ++v) {
        nv += (int64_t)vhi[v] - (int64_t)vlo[v];
        if (T->parent[v] >= 0) wc += (int64_t)c_af[lay[v]] * T->len[v];
    }
    *tof = t;
    *ov_sum = s2;
    *ov_edges = n2;
    *vias = nv;
    *wire_cap = wc;
}
