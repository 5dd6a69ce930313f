/*
 * Seeded synthetic instance generator for performance-driven layer assignment.
 *
 * It builds the inputs the layer-assignment problem takes (Sec. II-B, II-D of
 * the GAP-LA paper): a GCell grid with per-(edge, layer) capacities, per-layer
 * unit R/C and via R (shaped like the paper's modified Nangate45 table, whose
 * R and via R fall on upper layers), and one 2D Steiner-tree routing solution
 * per net.  Each net's tree is a rectilinear minimum spanning tree over its
 * pins (Prim on Manhattan distance) with every tree edge embedded as an L whose
 * orientation comes from one random bit.
 *
 * This module holds none of the layer-assignment arithmetic: no costs, no
 * trees turned into layer-assignment trees, no timing.  Both the CPU oracle and
 * the HIP library consume what it writes.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  Only IEEE-exact double operations
 * (+, -, *, /, sqrt, floor) are used on random values so that output bits do
 * not depend on the libm build.  Normal variates use the Irwin-Hall sum of 12
 * uniforms minus 6.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GEN_OK 0
#define GEN_ERR_ARG -1
#define GEN_ERR_OOM -4

typedef struct {
    int64_t num_nets;
    int32_t X, Y, L;
    int32_t pin_law;       /* 0: uniform {pin_min..pin_max}; 1: heavy-tailed law up to pin_max */
    int32_t pin_min, pin_max;
    int32_t placement;     /* 0 uniform; 1 hotspot; 2 net-local; 3 mixed hotspot/uniform centres */
    int32_t n_hot;         /* hotspot count */
    double hot_sigma;      /* placement 1: pin sigma around hotspot; 3: centre sigma around hotspot */
    double hot_frac;       /* placement 3: fraction of centres drawn near hotspots */
    int32_t cap_min, cap_max;
    int64_t fanout_every;  /* every net id divisible by this (if > 0) is a high-fanout net */
    int32_t fanout_min, fanout_max;
    int32_t budget_min_fs, budget_max_fs;
    int32_t cpin_af, rdrv_mohm;
    double r0_mohm, c0_af, via0_mohm, rc_decay;   /* per-layer-pair geometric RC law */
    uint64_t seed;
} gen_params;

typedef struct {
    gen_params p;
    int64_t num_nets, num_nodes, num_wp;
    int32_t *net_node_ptr;   /* int64 would be safer; node counts stay < 2^31 for every config */
    int32_t *node_parent;
    int16_t *node_x, *node_y;
    uint8_t *node_flags;
    int32_t *node_cpin_af;
    int32_t *edge_wp_ptr;
    int16_t *wp_x, *wp_y;
    int32_t *net_budget_fs, *net_rdrv_mohm;
    uint8_t *caps;           /* [Y][X][L] */
    int32_t *r_mohm, *c_af, *via_r_mohm;   /* [L], [L], [L-1] */
    uint8_t *layer_dir;      /* [L] 0 = horizontal, 1 = vertical */
} gen_instance;

static inline uint64_t sm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Counter-based form: output number i (0-based) of the splitmix64 sequence started at `seed`. */
static inline uint64_t sm64_at(uint64_t seed, uint64_t i)
{
    uint64_t s = seed + i * 0x9E3779B97F4A7C15ull;
    return sm64(&s);
}

static inline double u01(uint64_t *s) { return (double)(sm64(s) >> 11) * (1.0 / 9007199254740992.0); }

static inline int64_t uint_range(uint64_t *s, int64_t lo, int64_t hi)
{
    uint64_t span = (uint64_t)(hi - lo + 1);
    uint64_t r = sm64(s) >> 32;
    return lo + (int64_t)((r * span) >> 32);
}

static inline double normal01(uint64_t *s)
{
    double acc = 0.0;
    for (int i = 0; i < 12; ++i) acc += u01(s);
    return acc - 6.0;
}

static inline int32_t clampi(int64_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : (int32_t)v); }

static inline int32_t round_clip(double v, int32_t hi) { return clampi((int64_t)floor(v + 0.5), 0, hi); }

static int32_t draw_pins(const gen_params *p, uint64_t *s, int64_t net)
{
    if (p->fanout_every > 0 && net % p->fanout_every == 0 && net > 0)
        return (int32_t)uint_range(s, p->fanout_min, p->fanout_max);
    if (p->pin_law == 0) return (int32_t)uint_range(s, p->pin_min, p->pin_max);
    /* P(2)=.55, P(3)=P(4)=.15, remaining .15 geometric (ratio .8) over 5..pin_max */
    double u = u01(s);
    if (u < 0.55 || p->pin_max < 3) return 2;
    if (u < 0.70 || p->pin_max < 4) return 3;
    if (u < 0.85 || p->pin_max < 5) return 4;
    double v = (u - 0.85) / 0.15;
    int32_t K = p->pin_max - 4;             /* tail values 5..pin_max */
    double rK = 1.0;
    for (int32_t i = 0; i < K; ++i) rK *= 0.8;
    double denom = 1.0 - rK, rk = 1.0;
    for (int32_t k = 0; k < K; ++k) {
        rk *= 0.8;                          /* 0.8^(k+1) */
        if ((1.0 - rk) / denom > v) return 5 + k;
    }
    return p->pin_max;
}

/* open-addressing set of occupied GCells for one net */
typedef struct { uint64_t *keys; int64_t cap; } cellset;

static int cellset_init(cellset *cs, int64_t n)
{
    int64_t c = 16;
    while (c < 4 * n) c <<= 1;
    cs->keys = (uint64_t *)malloc((size_t)c * sizeof(uint64_t));
    if (!cs->keys) return -1;
    memset(cs->keys, 0xff, (size_t)c * sizeof(uint64_t));
    cs->cap = c;
    return 0;
}

/* returns 1 if inserted, 0 if already present */
static int cellset_insert(cellset *cs, uint64_t key)
{
    uint64_t h = sm64_at(key, 7) & (uint64_t)(cs->cap - 1);
    while (cs->keys[h] != ~0ull) {
        if (cs->keys[h] == key) return 0;
        h = (h + 1) & (uint64_t)(cs->cap - 1);
    }
    cs->keys[h] = key;
    return 1;
}

static void place_pin(const gen_params *p, uint64_t *s, double cx, double cy, double sigma, int32_t *x, int32_t *y)
{
    if (p->placement == 0) {
        *x = (int32_t)uint_range(s, 0, p->X - 1);
        *y = (int32_t)uint_range(s, 0, p->Y - 1);
    } else {
        double zx = normal01(s), zy = normal01(s);
        *x = round_clip(cx + sigma * zx, p->X - 1);
        *y = round_clip(cy + sigma * zy, p->Y - 1);
    }
}

void gen_free(gen_instance *g)
{
    if (!g) return;
    free(g->net_node_ptr); free(g->node_parent); free(g->node_x); free(g->node_y);
    free(g->node_flags); free(g->node_cpin_af); free(g->edge_wp_ptr); free(g->wp_x); free(g->wp_y);
    free(g->net_budget_fs); free(g->net_rdrv_mohm); free(g->caps);
    free(g->r_mohm); free(g->c_af); free(g->via_r_mohm); free(g->layer_dir);
    free(g);
}

static int grow(void **ptr, int64_t *cap, int64_t need, size_t elt)
{
    if (need <= *cap) return 0;
    int64_t nc = *cap ? *cap : 1024;
    while (nc < need) nc *= 2;
    void *np = realloc(*ptr, (size_t)nc * elt);
    if (!np) return -1;
    *ptr = np;
    *cap = nc;
    return 0;
}

static inline int64_t rne_pos(double v) { return (int64_t)nearbyint(v); }

int gen_create(const gen_params *pin, gen_instance **out)
{
    *out = NULL;
    const gen_params *p = pin;
    if (p->num_nets <= 0 || p->X < 2 || p->Y < 2 || p->X > 32767 || p->Y > 32767 || p->L < 2 || p->L > 16 ||
        p->pin_min < 2 || p->pin_max < p->pin_min || p->cap_min < 0 || p->cap_max > 255 || p->cap_max < p->cap_min ||
        (p->placement != 0 && p->placement != 1 && p->placement != 2 && p->placement != 3) ||
        ((p->placement == 1 || p->placement == 3) && p->n_hot <= 0))
        return GEN_ERR_ARG;
    gen_instance *g = (gen_instance *)calloc(1, sizeof(gen_instance));
    if (!g) return GEN_ERR_OOM;
    g->p = *p;
    const int32_t L = p->L;
    g->r_mohm = (int32_t *)malloc(sizeof(int32_t) * L);
    g->c_af = (int32_t *)malloc(sizeof(int32_t) * L);
    g->via_r_mohm = (int32_t *)malloc(sizeof(int32_t) * L);
    g->layer_dir = (uint8_t *)malloc((size_t)L);
    if (!g->r_mohm || !g->c_af || !g->via_r_mohm || !g->layer_dir) { gen_free(g); return GEN_ERR_OOM; }
    for (int32_t l = 0; l < L; ++l) {
        double f = 1.0;
        for (int32_t k = 0; k < l / 2; ++k) f *= p->rc_decay;
        g->r_mohm[l] = (int32_t)rne_pos(p->r0_mohm * f);
        g->c_af[l] = (int32_t)rne_pos(p->c0_af * f);
        g->via_r_mohm[l] = (int32_t)rne_pos(p->via0_mohm * f);
        g->layer_dir[l] = (uint8_t)(l & 1);
    }

    const int64_t N = p->num_nets;
    g->num_nets = N;
    g->net_node_ptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N + 1));
    g->net_budget_fs = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    g->net_rdrv_mohm = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!g->net_node_ptr || !g->net_budget_fs || !g->net_rdrv_mohm) { gen_free(g); return GEN_ERR_OOM; }

    uint64_t st = p->seed;
    double hx[256], hy[256];
    int32_t nh = p->n_hot > 256 ? 256 : p->n_hot;
    for (int32_t h = 0; h < nh; ++h) { hx[h] = u01(&st) * p->X; hy[h] = u01(&st) * p->Y; }

    int64_t nn = 0, nw = 0;
    int32_t *par = NULL; int16_t *nx = NULL, *ny = NULL; uint8_t *fl = NULL; int32_t *cp = NULL, *wpp = NULL;
    int16_t *wx = NULL, *wy = NULL;
    int64_t parc = 0, nxc = 0, nyc = 0, flc = 0, cpc = 0, wppc = 0, wxc = 0, wyc = 0;
    /* per-net scratch */
    int32_t scap = 0; int32_t *px = NULL, *py = NULL, *mpar = NULL; int64_t *dist = NULL; uint8_t *intree = NULL;
    int rc = GEN_OK;

    for (int64_t i = 0; i < N; ++i) {
        int32_t np = draw_pins(p, &st, i);
        if (np > scap) {
            scap = np;
            px = (int32_t *)realloc(px, sizeof(int32_t) * np); py = (int32_t *)realloc(py, sizeof(int32_t) * np);
            mpar = (int32_t *)realloc(mpar, sizeof(int32_t) * np); dist = (int64_t *)realloc(dist, sizeof(int64_t) * np);
            intree = (uint8_t *)realloc(intree, (size_t)np);
            if (!px || !py || !mpar || !dist || !intree) { rc = GEN_ERR_OOM; break; }
        }
        double cx = 0, cy = 0, sigma = 0;
        if (p->placement == 1) {
            int32_t h = (int32_t)uint_range(&st, 0, nh - 1);
            cx = hx[h]; cy = hy[h]; sigma = p->hot_sigma;
        } else if (p->placement == 2 || p->placement == 3) {
            if (p->placement == 3 && u01(&st) < p->hot_frac) {
                int32_t h = (int32_t)uint_range(&st, 0, nh - 1);
                cx = hx[h] + p->hot_sigma * normal01(&st);
                cy = hy[h] + p->hot_sigma * normal01(&st);
                cx = cx < 0 ? 0 : (cx > p->X - 1 ? p->X - 1 : cx);
                cy = cy < 0 ? 0 : (cy > p->Y - 1 ? p->Y - 1 : cy);
            } else {
                cx = u01(&st) * p->X; cy = u01(&st) * p->Y;
            }
            sigma = 3.0 * sqrt((double)np);
        }
        /* distinct pins: resample duplicates, then fall back to a deterministic scan */
        cellset cs;
        if (cellset_init(&cs, np)) { rc = GEN_ERR_OOM; break; }
        for (int32_t k = 0; k < np; ++k) {
            int32_t x = 0, y = 0, ok = 0;
            for (int att = 0; att < 4096 && !ok; ++att) {
                place_pin(p, &st, cx, cy, sigma, &x, &y);
                ok = cellset_insert(&cs, (uint64_t)y * (uint64_t)p->X + (uint64_t)x);
            }
            if (!ok) {
                int64_t tot = (int64_t)p->X * p->Y, c0 = (int64_t)y * p->X + x;
                for (int64_t d = 1; d < tot && !ok; ++d) {
                    int64_t c = (c0 + d) % tot;
                    if (cellset_insert(&cs, (uint64_t)c)) { ok = 1; x = (int32_t)(c % p->X); y = (int32_t)(c / p->X); }
                }
                if (!ok) { free(cs.keys); rc = GEN_ERR_ARG; goto done; }
            }
            px[k] = x; py[k] = y;
        }
        free(cs.keys);
        /* Prim's rectilinear MST rooted at pin 0 (the driver); ties go to the lowest index */
        for (int32_t k = 0; k < np; ++k) { intree[k] = 0; dist[k] = INT64_MAX; mpar[k] = -1; }
        intree[0] = 1;
        for (int32_t k = 1; k < np; ++k) { dist[k] = llabs((int64_t)px[k] - px[0]) + llabs((int64_t)py[k] - py[0]); mpar[k] = 0; }
        for (int32_t it = 1; it < np; ++it) {
            int32_t best = -1;
            for (int32_t k = 1; k < np; ++k)
                if (!intree[k] && (best < 0 || dist[k] < dist[best])) best = k;
            intree[best] = 1;
            for (int32_t k = 1; k < np; ++k) {
                if (intree[k]) continue;
                int64_t d = llabs((int64_t)px[k] - px[best]) + llabs((int64_t)py[k] - py[best]);
                if (d < dist[k]) { dist[k] = d; mpar[k] = best; }
            }
        }
        if (grow((void **)&par, &parc, nn + np, sizeof(int32_t)) || grow((void **)&nx, &nxc, nn + np, sizeof(int16_t)) ||
            grow((void **)&ny, &nyc, nn + np, sizeof(int16_t)) || grow((void **)&fl, &flc, nn + np, 1) ||
            grow((void **)&cp, &cpc, nn + np, sizeof(int32_t)) || grow((void **)&wpp, &wppc, nn + np + 1, sizeof(int32_t)) ||
            grow((void **)&wx, &wxc, nw + np, sizeof(int16_t)) || grow((void **)&wy, &wyc, nw + np, sizeof(int16_t))) {
            rc = GEN_ERR_OOM; break;
        }
        g->net_node_ptr[i] = (int32_t)nn;
        for (int32_t k = 0; k < np; ++k) {
            int64_t v = nn + k;
            par[v] = mpar[k];
            nx[v] = (int16_t)px[k]; ny[v] = (int16_t)py[k];
            fl[v] = k == 0 ? 2 : 1;
            cp[v] = k == 0 ? 0 : p->cpin_af;
            wpp[v] = (int32_t)nw;
            if (k > 0) {
                int32_t u = mpar[k];
                if (px[u] != px[k] && py[u] != py[k]) {
                    int bit = (int)(sm64(&st) & 1);
                    wx[nw] = (int16_t)(bit ? px[u] : px[k]);
                    wy[nw] = (int16_t)(bit ? py[k] : py[u]);
                    ++nw;
                }
            }
        }
        nn += np;
        g->net_budget_fs[i] = (int32_t)uint_range(&st, p->budget_min_fs, p->budget_max_fs);
        g->net_rdrv_mohm[i] = p->rdrv_mohm;
        if (nn > INT32_MAX - 8192) { rc = GEN_ERR_ARG; break; }
    }
done:
    free(px); free(py); free(mpar); free(dist); free(intree);
    if (rc != GEN_OK) {
        free(par); free(nx); free(ny); free(fl); free(cp); free(wpp); free(wx); free(wy);
        gen_free(g);
        return rc;
    }
    g->net_node_ptr[N] = (int32_t)nn;
    if (grow((void **)&wpp, &wppc, nn + 1, sizeof(int32_t))) { gen_free(g); return GEN_ERR_OOM; }
    wpp[nn] = (int32_t)nw;
    g->num_nodes = nn; g->num_wp = nw;
    g->node_parent = par; g->node_x = nx; g->node_y = ny; g->node_flags = fl; g->node_cpin_af = cp;
    g->edge_wp_ptr = wpp; g->wp_x = wx; g->wp_y = wy;

    /* capacities: i.i.d. per (edge, layer); the missing edge past the last column (H layers) or row (V) gets 0 */
    int64_t E = (int64_t)p->X * p->Y * L;
    g->caps = (uint8_t *)malloc((size_t)E);
    if (!g->caps) { gen_free(g); return GEN_ERR_OOM; }
    uint64_t cseed = p->seed ^ 0xC0FFEE1234567ull;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        int32_t l = (int32_t)(e % L);
        int64_t xy = e / L;
        int32_t x = (int32_t)(xy % p->X), y = (int32_t)(xy / p->X);
        int edge_exists = g->layer_dir[l] == 0 ? (x < p->X - 1) : (y < p->Y - 1);
        uint64_t r = sm64_at(cseed, (uint64_t)e) >> 32;
        uint64_t span = (uint64_t)(p->cap_max - p->cap_min + 1);
        g->caps[e] = edge_exists ? (uint8_t)(p->cap_min + (int32_t)((r * span) >> 32)) : 0;
    }
    *out = g;
    return GEN_OK;
}

void gen_sizes(const gen_instance *g, int64_t *nets, int64_t *nodes, int64_t *wps)
{
    *nets = g->num_nets; *nodes = g->num_nodes; *wps = g->num_wp;
}

/* copies everything into caller buffers sized from gen_sizes() */
void gen_export(const gen_instance *g, int32_t *net_node_ptr, int32_t *node_parent, int16_t *node_x, int16_t *node_y,
                uint8_t *node_flags, int32_t *node_cpin_af, int32_t *edge_wp_ptr, int16_t *wp_x, int16_t *wp_y,
                int32_t *net_budget_fs, int32_t *net_rdrv_mohm, uint8_t *caps, int32_t *r_mohm, int32_t *c_af,
                int32_t *via_r_mohm, uint8_t *layer_dir)
{
    const int64_t N = g->num_nets, n = g->num_nodes, w = g->num_wp, L = g->p.L;
    memcpy(net_node_ptr, g->net_node_ptr, sizeof(int32_t) * (size_t)(N + 1));
    memcpy(node_parent, g->node_parent, sizeof(int32_t) * (size_t)n);
    memcpy(node_x, g->node_x, sizeof(int16_t) * (size_t)n);
    memcpy(node_y, g->node_y, sizeof(int16_t) * (size_t)n);
    memcpy(node_flags, g->node_flags, (size_t)n);
    memcpy(node_cpin_af, g->node_cpin_af, sizeof(int32_t) * (size_t)n);
    memcpy(edge_wp_ptr, g->edge_wp_ptr, sizeof(int32_t) * (size_t)(n + 1));
    if (w) { memcpy(wp_x, g->wp_x, sizeof(int16_t) * (size_t)w); memcpy(wp_y, g->wp_y, sizeof(int16_t) * (size_t)w); }
    memcpy(net_budget_fs, g->net_budget_fs, sizeof(int32_t) * (size_t)N);
    memcpy(net_rdrv_mohm, g->net_rdrv_mohm, sizeof(int32_t) * (size_t)N);
    memcpy(caps, g->caps, (size_t)((int64_t)g->p.X * g->p.Y * L));
    memcpy(r_mohm, g->r_mohm, sizeof(int32_t) * (size_t)L);
    memcpy(c_af, g->c_af, sizeof(int32_t) * (size_t)L);
    memcpy(via_r_mohm, g->via_r_mohm, sizeof(int32_t) * (size_t)(L - 1));
    memcpy(layer_dir, g->layer_dir, (size_t)L);
}

/* out[i] = output number (start + i) of the splitmix64 sequence started at `seed`. */
void gen_counter_u64(uint64_t seed, int64_t start, int64_t n, uint64_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = sm64_at(seed, (uint64_t)(start + i));
}

/*
 * Synthetic gate-level timing graph over the nets, for the critical-path net ordering of
 * Alg. 1: every net is driven by one gate whose delay is uniform in {dmin..dmax} fs; every
 * net gets a logic level uniform in {0..levels-1}; every sink of a net at level h feeds the
 * gate of a net drawn uniformly from the nets at level h + 1 (sink_next = that net), unless
 * the net is at the last level or, with probability po_frac, the sink is a primary output
 * (sink_next = -1).  Sinks are numbered in node order (the sink-flagged input nodes in net and
 * node order).  Structure only: no delay or timing arithmetic.
 */
int gen_timing_graph(int64_t nets, const int32_t *net_node_ptr, const uint8_t *node_flags, int32_t levels,
                     double po_frac, int32_t dmin_fs, int32_t dmax_fs, uint64_t seed, int32_t *net_level,
                     int32_t *sink_next, int32_t *gate_delay_fs)
{
    if (nets < 0 || levels < 1 || dmin_fs < 0 || dmax_fs < dmin_fs || !(po_frac >= 0.0 && po_frac <= 1.0))
        return GEN_ERR_ARG;
    uint64_t s = seed ^ 0x74696d696e674441ull;   /* a stream of its own */
    int64_t *cnt = (int64_t *)calloc((size_t)levels + 1, sizeof(int64_t));
    int64_t *by_level = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nets > 0 ? nets : 1));
    if (!cnt || !by_level) {
        free(cnt);
        free(by_level);
        return GEN_ERR_OOM;
    }
    for (int64_t i = 0; i < nets; ++i) {
        net_level[i] = (int32_t)uint_range(&s, 0, levels - 1);
        gate_delay_fs[i] = (int32_t)uint_range(&s, dmin_fs, dmax_fs);
        cnt[net_level[i] + 1]++;
    }
    for (int32_t h = 0; h < levels; ++h) cnt[h + 1] += cnt[h];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)levels);
        if (!fill) {
            free(cnt);
            free(by_level);
            return GEN_ERR_OOM;
        }
        for (int32_t h = 0; h < levels; ++h) fill[h] = cnt[h];
        for (int64_t i = 0; i < nets; ++i) by_level[fill[net_level[i]]++] = i;
        free(fill);
    }
    int64_t k = 0;
    for (int64_t i = 0; i < nets; ++i) {
        const int32_t h = net_level[i];
        const int64_t n_next = h + 1 < levels ? cnt[h + 2] - cnt[h + 1] : 0;
        for (int32_t v = net_node_ptr[i]; v < net_node_ptr[i + 1]; ++v) {
            if (!(node_flags[v] & 1)) continue;
            const double u = u01(&s);
            if (n_next == 0 || u < po_frac) {
                sink_next[k++] = -1;
            } else {
                sink_next[k++] = (int32_t)by_level[cnt[h + 1] + uint_range(&s, 0, n_next - 1)];
            }
        }
    }
    free(cnt);
    free(by_level);
    return GEN_OK;
}
