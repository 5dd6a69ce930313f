/*
 * gapla.h -- C ABI of the MI355X (gfx950) layer-assignment library.
 *
 * The library lifts the 2D routing tree of every net onto metal layers so that
 * its planar projection is unchanged (problem formulation, Sec. II-D of the
 * GAP-LA paper), minimising via count, GCell-edge congestion and
 * Elmore-delay / capacitance cost with the tree dynamic program of Alg. 2-4
 * and its look-ahead (Sec. III-D), and it evaluates the Elmore RC-tree timing
 * that weights that program (Sec. II-C, Fig. rc) together with the exact
 * reverse sweep of that timing.
 *
 * Conventions shared by every call:
 *  - Units: R in mOhm, C in aF, via R in mOhm (int32) on input; timing outputs
 *    and R/C views are float with R in kOhm and C in fF, so delays are in ps.
 *  - Memory: la_build_batch copies its HOST inputs.  Every other pointer
 *    argument is a DEVICE pointer on the batch's device, owned by the caller,
 *    unless stated otherwise.  The batch owns its own tree, DP scratch,
 *    demand map and R/C views; they live until la_free_batch.
 *  - Node order: the library numbers the nodes of the layer-assignment tree
 *    canonically -- per net, the input nodes in input order followed by one
 *    node per bend, in the order of the input edge it splits (edge parent(v)->v
 *    in order of v) and, within an edge, from the parent end.  Every per-node
 *    array (weights in, layers out, R/C, gradients) uses this order.  Sinks are
 *    numbered in node order.  RC-edge index space [0, nodes) is the segment
 *    parent(n)->n (the driver resistance at a net's root); [nodes, nodes+sinks)
 *    is the pin edge of sink k.
 *  - Streams: every call enqueues on the stream given to la_build_batch and
 *    returns without waiting, except where stated.  A batch must not be used
 *    from two host threads at once.
 *  - Errors: no exception crosses this ABI.  Argument and tree validation
 *    happen on the host before any device work and return the status at once;
 *    device faults surface as LA_ERR_HIP at the next call that synchronises.
 *    la_last_error() gives a per-thread message for the last failure.
 */
#ifndef GAPLA_H
#define GAPLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LA_OK = 0,
    LA_ERR_INVALID_ARG = -1, /* null pointer, bad size, bad enum                            */
    LA_ERR_BAD_TREE = -2,    /* malformed 2D tree: cycle, diagonal or zero-length edge, ...   */
    LA_ERR_RANGE = -3,       /* a fixed-point product could leave its integer range          */
    LA_ERR_OOM = -4,         /* device or host allocation failed                              */
    LA_ERR_HIP = -5,         /* a HIP runtime call failed                                     */
    LA_ERR_STATE = -6        /* call out of order (e.g. backward before forward)             */
} la_status;

typedef struct la_batch la_batch;

/* The 2D global-routing solution of every net (Sec. II-B): one rooted tree per
 * net whose edges are axis-aligned polylines on the GCell grid.  HOST pointers,
 * copied by la_build_batch. */
typedef struct {
    int32_t num_nets, num_nodes, num_waypoints;
    const int32_t *net_node_ptr;  /* [num_nets+1] nodes of net i: [ptr[i], ptr[i+1]); node 0 = driver     */
    const int32_t *node_parent;   /* [num_nodes] net-local parent index, -1 exactly at the driver          */
    const int16_t *node_x;        /* [num_nodes] GCell column, 0 <= x < X                                   */
    const int16_t *node_y;        /* [num_nodes] GCell row,    0 <= y < Y                                   */
    const uint8_t *node_flags;    /* [num_nodes] bit0 sink pin, bit1 driver pin; pins sit on layer 0        */
    const int32_t *node_cpin_af;  /* [num_nodes] sink pin load (aF); ignored for non-sinks                  */
    const int32_t *edge_wp_ptr;   /* [num_nodes+1] bend waypoints of edge parent(v)->v, parent end first    */
    const int16_t *wp_x, *wp_y;   /* [num_waypoints]                                                        */
    const int32_t *net_budget_fs; /* [num_nets] required time at every sink of the net (fs)                 */
    const int32_t *net_rdrv_mohm; /* [num_nets] driver resistance (mOhm)                                    */
} la_nets;

/* GCell grid: X columns, Y rows, L layers; layer_dir[l] = 0 horizontal, 1 vertical (HOST). */
typedef struct {
    int32_t X, Y, L, min_layer;   /* layers below min_layer carry no wire (pins still sit on layer 0) */
    const uint8_t *layer_dir;
} la_grid;

/* Per-layer unit wire R and C per GCell and the resistance of the via from layer k to k+1
 * (the paper's "R of Upper Via" column, Table Nangate45) (HOST). */
typedef struct {
    const int32_t *r_mohm;        /* [L] */
    const int32_t *c_af;          /* [L] */
    const int32_t *via_r_mohm;    /* [L-1] */
} la_layer_rc;

/*
 * la_build_batch -- validate the nets, insert a node at every bend so that no
 * tree edge bends and layers change only at nodes (Sec. III-B, Fig. graph_b),
 * levelise the trees by height, and upload everything.
 *  edge_caps: HOST [Y][X][L] capacity of the GCell edge leaving (x, y) towards
 *             +x on horizontal layers and +y on vertical layers.
 *  stream:    hipStream_t (NULL = default stream) used by every later call.
 *  out:       receives a new batch; the caller frees it with la_free_batch.
 * Returns LA_ERR_BAD_TREE for malformed trees (the failing net is named in
 * la_last_error), LA_ERR_RANGE when a net's worst-case cost terms could leave
 * int64 or the grid index leaves int32, LA_ERR_INVALID_ARG for bad sizes.
 */
la_status la_build_batch(const la_nets *nets, const la_grid *grid, const la_layer_rc *layer_rc,
                         const uint8_t *edge_caps, void *stream, la_batch **out);

/* Launch configuration of the batched form (see la_tune). */
typedef struct {
    int32_t tile_nodes;   /* nodes of one workgroup's LDS tile: 192, or 128 / 256 at 5-6 routable
                             layers per direction; nets with more nodes run in the big-net kernel */
    int32_t claim_units;  /* work-queue claim size, sum over its nets of (nodes + 3): 96..316   */
    int32_t workgroups;   /* persistent workgroups per launch, 0 = as many as fit the GPU        */
    int32_t fuse_nets;    /* a batch with at least this many small nets moves its demand from
                             its DP kernel (otherwise through a changed-segment list)            */
    int32_t tuned;        /* output: 1 when la_tune chose the values                            */
} la_tuning;

typedef struct {
    int64_t nets, nodes, sinks, rc_edges, grid_edges;
    int32_t levels;               /* tree height + 1 over all nets                          */
    int32_t max_net_nodes;
    int64_t gcell_edges;          /* total wire length (GCells) over all segments            */
    const int32_t *node_parent;   /* device [nodes] global parent index, -1 at roots (batch-owned) */
    const int32_t *node_net;      /* device [nodes] */
    const int32_t *sink_node;     /* device [sinks] */
    /* Algorithmic work of one DP round over every net (Alg. 3 as written): integer lane-ops of
     * the stack enumeration, sum over nodes n and entering layers l of (lo+1)(L-hi) stacks x
     * (6 per child + 10), and the compulsory bytes (node inputs, congestion gathers of 9 B per
     * GCell edge and routable layer, outputs).  Elmore: compulsory bytes of one forward and one
     * reverse sweep.  dp_ops_big_per_round: the part of dp_ops_per_round from nets of more than
     * tuning.tile_nodes nodes, which the batched form runs in its own kernel with the DP state
     * in HBM. */
    double dp_ops_per_round, dp_bytes_per_round, elmore_fwd_bytes, elmore_bwd_bytes;
    double dp_ops_big_per_round;
    int64_t graph_instantiations; /* round graphs the batched form has instantiated so far       */
    la_tuning tuning;             /* the batched form's current launch configuration            */
} la_info;
la_status la_batch_info(const la_batch *b, la_info *out);

/* Integer DP inputs (fixed point, see la_assign). */
typedef struct {
    int64_t w_cong, w_cap, w_d, w_via; /* global cost weights, each >= 0                        */
    const uint16_t *seg_w_q10;    /* device [nodes] Q10 edge weight of segment parent(n)->n (Eq. 5), <= 1024 */
    const uint16_t *pin_w_q10;    /* device [sinks] Q10 pin weight (Eq. 4), <= 1024          */
    const int32_t *lambda_mohm;   /* device [nodes] look-ahead coefficient >= 0 (0 turns it off)      */
    const uint8_t *net_tier;      /* device [nets] batch of each net (Alg. 1 order); NULL = one batch */
    const int32_t *cong_lut;      /* device [L][2][64] marginal congestion cost; NULL = built-in table */
    int32_t rounds;               /* negotiation rounds, >= 1                                */
    int32_t hist_inc;             /* history increment per unit of overflow, >= 0            */
    int32_t form;                 /* LA_FORM_PLAIN or LA_FORM_BATCHED (same results)          */
    int32_t num_tiers;            /* batches are 0..num_tiers-1 (ignored when net_tier and
                                     net_batch are NULL); up to 256 for net_tier, 65536 for net_batch */
    const int32_t *net_batch;     /* dev [nets] int32 batch of each net (e.g. from la_get_batches);
                                     when given it replaces net_tier                              */
} la_weights;

#define LA_FORM_PLAIN 0    /* the paper's Alg. 2 shape: one launch per tree level per batch     */
#define LA_FORM_BATCHED 1  /* persistent per-batch launches, whole nets on chip, hipGraph rounds */

/*
 * la_assign -- layer assignment of every net (Alg. 2): for each round, for each
 * batch in order, the DP of Alg. 3 with the look-ahead of Sec. III-D runs for
 * every net of the batch against one snapshot of the demand map, Alg. 4 traces
 * the choice back, and the batch's segments are committed to the demand map;
 * after each round history += hist_inc * max(0, demand - capacity), saturating
 * at 2^24.  From the second round on (and on any later call) a segment's own
 * previous demand is excluded from its congestion cost and commits move demand.
 *
 * Cost of a complete assignment a (every term integer, T(w,R,X) =
 * (w*((R*X)>>11))>>10, X = C + 2*S the doubled pi-model load):
 *   w_cong*sum kappa_s(a_s) + w_cap*sum C_s + w_via*sum_n (max-min of the layers at n)
 *   + w_d*[ sum_s T(w_s, r(a_s)*len_s, X_s) + T(w_s, Rvia(l_parent, a_s), X_s)
 *           + sum_sinks T(wpin, Rvia(a_n, 0), 2*Cpin) ]
 * with kappa from cong_lut (Eq. 3 marginal, indexed by demand - capacity).
 * The DP keeps, per node and entering layer, the via stack [b,t] with the lowest
 * look-ahead cost; ties go to the lowest b, then t, and a child's lowest layer.
 *
 *  history:    device [Y*X*L] int32 congestion history, read and updated.
 *  out_layers: device [nodes] layer of segment parent(n)->n; 0 at roots.
 * Returns LA_ERR_RANGE when the weights could overflow a net's int64 cost.
 * Layers are bit-identical for both forms and any launch configuration.
 */
la_status la_assign(la_batch *b, const la_weights *w, int32_t *history, uint8_t *out_layers);

/*
 * la_tune -- the autotuner of the batched form (Alg. 2's batch loop as one persistent launch
 * per batch): times, on this instance, one negotiation round of the given weights, batches and
 * history (host order, device [Y*X*L], read only) for each tile size built for the batch's
 * routable-layer count and three claim sizes around it, then two fused-commit thresholds for
 * the fastest, and keeps the fastest configuration for the batch's later la_assign calls.
 * Every configuration gives the same layers, bit for bit.  The demand map, previous layers,
 * via spans and round flag are restored afterwards, so la_tune changes no result.  The choice
 * is cached per instance shape (nets, nodes, grid, layers, levels, wire length) in the process:
 * a later batch of the same shape takes it without timing.  Synchronises.  Allocates
 * temporaries for the saved state.  `out` (HOST, may be NULL) receives the choice.
 */
la_status la_tune(la_batch *b, const la_weights *w, const int32_t *history, la_tuning *out);
/* Sets the batched form's configuration explicitly (tuned = 0); LA_ERR_INVALID_ARG for a tile
 * size not built for this batch's layer count or values out of range. */
la_status la_set_tuning(la_batch *b, const la_tuning *t);
la_status la_get_tuning(const la_batch *b, la_tuning *out);

/*
 * la_get_batches -- classical batching (Alg. 1, GetBatch: the batching of the
 * routers the paper cites for it).  A net's box is the GCell rectangle its tree spans.  Within
 * each subset, in increasing net order, a net joins the lowest batch in which no net's box
 * shares a GCell with its own (so the nets of a batch share no GCell edge); subsets are batched
 * one after another and never share a batch: subset s's batches follow those of subsets
 * 0..s-1.  The result is that of the sequential first-fit, bit for bit.
 *  net_subset:  device [nets] int32 subset of each net (0..num_subsets-1; any other value leaves
 *               the net out, batch -1)
 *  out_batch:   device [nets] int32 batch of each net, for la_weights.net_batch
 *  num_batches: HOST, receives the number of batches.
 * At most 1024 batches in all (LA_ERR_RANGE beyond).  num_subsets in 1..256.  Allocates
 * temporaries (the GCell grid's batch bits, 136 B per GCell), synchronises.
 */
la_status la_get_batches(la_batch *b, const int32_t *net_subset, int32_t num_subsets, int32_t *out_batch,
                         int32_t *num_batches);

/*
 * Critical-path net ordering (Sec. III-A; Alg. 1 ordering) on a gate-level graph over the nets.
 * la_timing_graph sets the graph: each net is driven by one gate (gate_delay_fs: HOST [nets]);
 * sink k (node order) feeds the gate of net sink_next[k] (HOST [sinks]), or is a primary output
 * (-1) whose required time is clock_fs.  Copied; ordered topologically on the host.
 * LA_ERR_INVALID_ARG for an index out of range, a negative delay or a cycle.
 */
la_status la_timing_graph(la_batch *b, const int32_t *sink_next, const int32_t *gate_delay_fs, int32_t clock_fs);
/*
 * la_sta -- static timing with the given sink delays (DEVICE [sinks] ps, e.g. from la_elmore) in
 * single precision, each value rounded once as written: arrival at a net's driver = gate delay +
 * the latest arrival among the sinks feeding the gate (0 if none); at a sink = its driver's +
 * its delay; required at an output = clock, at a sink feeding net m = required at m's driver -
 * m's gate delay, at a driver = min over its sinks of (required - delay).
 *  out_slack: DEVICE [sinks] required - arrival;  *wns: HOST, the least output slack.
 *  out_crit:  DEVICE [nets] int32, the number of top-1 critical paths through each net: one per
 *             primary output with slack < 0.7 WNS (when WNS < 0), from its net back through
 *             each gate's latest input (the lowest sink on equal arrival) to a primary input.
 * Synchronises.  LA_ERR_STATE without la_timing_graph.
 */
la_status la_sta(la_batch *b, const float *sink_delay, float *out_slack, int32_t *out_crit, float *wns);
/*
 * la_alg1_subsets -- Alg. 1 division and partition: critical nets (more than three counted paths) by count
 * against the largest, C: subset k holds C / 2^k <= count < C / 2^(k-1); the other nets whose
 * net slack (least over its sinks) is below 0.7 WNS by rho = slack / WNS in the bins 1,
 * [0.99, 1), [0.96, 0.99), [0.91, 0.96), [0.84, 0.91), [0.75, 0.84), [0.7, 0.75); then the rest.
 * Subsets: critical 0..kc-1, the seven slack bins, the rest; *num_subsets = kc + 8 (HOST).
 * out_subset: DEVICE [nets] int32, for la_get_batches.  Synchronises.
 */
la_status la_alg1_subsets(la_batch *b, const float *slack, const int32_t *crit, float wns, int32_t *out_subset,
                          int32_t *num_subsets);

/* Via span (lowest, highest layer) at every node of the last assignment: device [nodes][2]. */
la_status la_vias(la_batch *b, uint8_t *out_lo_hi);

/* Copy of the demand map: device [Y*X*L] int32. */
la_status la_demand(la_batch *b, int32_t *out_demand);

/* Forget the previous assignment: demand back to zero, next la_assign starts at round 0. */
la_status la_reset(la_batch *b);

/*
 * la_batch_rc -- batch-owned device views (float [nodes+sinks]) of the RC edges
 * of the current solution: before any assignment the average per-direction unit
 * R and C with zero-resistance pin edges (Sec. III-B); after one, a segment is
 * the lumped via from its parent's entering layer plus the wire, and a pin edge
 * the via down to layer 0.  The driver resistance sits at each root.
 */
la_status la_batch_rc(la_batch *b, float **R, float **C);

/*
 * la_elmore -- Elmore delay (Sec. II-C; d34 example of Fig. rc) of every sink on
 * the batch's current RC: S = downstream capacitance bottom-up, then
 * t(v) = t(parent) + R_v*(C_v/2 + S_v) top-down, compensated FP32 sums.
 *  out_delay: device [sinks] float, ps.
 */
la_status la_elmore(la_batch *b, float *out_delay);

/* Same on caller-given R, C (device float [nodes+sinks]); they must stay unchanged
 * until la_elmore_backward has run for this forward. */
la_status la_elmore_rc(la_batch *b, const float *R, const float *C, float *out_delay);

/*
 * la_elmore_backward -- exact reverse sweep of the last forward for
 * slack_k = budget_k - delay_k: with g_k = -dSlack_k, G(v) = sum of g below v,
 * Sig(v) = Sig(parent) + R_v*G(v); dR_v = G(v)*(C_v/2 + S_v),
 * dC_v = R_v*G(v)/2 + Sig(parent).
 *  dSlack: device [sinks] dJ/dslack; out_dR, out_dC: device [nodes+sinks] (either may be NULL).
 * LA_ERR_STATE if no forward ran on this batch, or if the last forward read the batch-owned
 * R/C views (la_elmore) and a later la_assign, la_reset or la_load_state rewrote them.
 */
la_status la_elmore_backward(la_batch *b, const float *dSlack, float *out_dR, float *out_dC);

/* FP64 TNS (sum of negative slacks) and WNS (smallest slack) of delays [sinks]; synchronises
 * the stream and writes the HOST doubles. */
la_status la_timing_summary(la_batch *b, const float *delay, double *tns, double *wns);

/* la_timing_summary_noalloc -- the same TNS / WNS, bit for bit, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid it).  It calls no
 * allocator: its workgroup partials (at most 1024 workgroups, each striding over the sinks, so
 * any sink count fits) and its two results live in a fixed 16 KB device array that each GPU
 * holds once until the process ends; la_build_batch looks up that array's address on its
 * device.  Every call on one GPU shares the array: calls that overlap on one GPU (two host
 * threads, or two streams) race and must be serialised by the caller.  Synchronises the
 * batch's stream and writes the HOST doubles.  LA_ERR_INVALID_ARG for NULL arguments;
 * LA_ERR_RANGE if the partials would not fit the array. */
la_status la_timing_summary_noalloc(la_batch *b, const float *delay, double *tns, double *wns);

/*
 * la_quality_report -- quality terms of the current assignment (Sec. II, Eq. 1-3).
 * Over every GCell edge of every layer l, with demand d and capacity c: tof, the sum of the
 * Eq. 3 overflow ofw(l) e^{s (d - c)} (s = 0.5 if c > 0, 1.5 if c = 0; FP64, summed per
 * workgroup and then in workgroup order, so within rounding of any other order);
 * overflow_sum, the sum of the Eq. 2 overflow max(0, d - c), and overflow_edges, the number
 * of edges with d > c.  vias: the sum over tree nodes of the via span (via_hi - via_lo) of
 * the last la_assign.  wire_cap_af: the sum over tree segments of c(layer) * length, the
 * capacitance that stands for power.  The integer sums are exact.  With delays (DEVICE
 * [sinks], ps; NULL skips timing) it also reports WNS and TNS as la_timing_summary does and
 * the Eq. 1 score w1 (WNS - r1) + w2 (TNS - r2) / N_end + w3 (pow - r3) + w4 tof, with
 * N_end = sinks and pow = wire_cap_af / 1000 (fF); without delays or weights score = 0.
 * ofw: HOST [L] overflow weight per layer (NULL = all 1).  Synchronises the batch's stream
 * and writes the HOST struct `out`.  LA_ERR_INVALID_ARG for NULL b or out.
 */
typedef struct {
    double w1, w2, w3, w4;   /* weights of WNS, TNS / N_end, power and total overflow */
    double r1, r2, r3;       /* reference WNS, TNS, power */
} la_score_weights;
typedef struct {
    double tof;              /* Eq. 3 total overflow */
    int64_t overflow_sum;    /* Eq. 2 total overflow */
    int64_t overflow_edges;
    int64_t vias;
    int64_t wire_cap_af;
    double wns_ps, tns_ps;   /* 0 without delays */
    double score;
} la_quality;
la_status la_quality_report(la_batch *b, const double *ofw, const float *delay, const la_score_weights *sw,
                            la_quality *out);

#define LA_WEIGHTS_PLAIN 0    /* Eq. 4 pin weights, Eq. 5 edge weights, lambda = (w*r_est)>>10 */
#define LA_WEIGHTS_ADJOINT 1  /* weights and lambda from the reverse sweep of weighted TNS     */

/*
 * la_timing_weights -- DP inputs from sink delays (device [sinks], ps) on the
 * batch's current RC.  slack = budget - delay, WNS = min slack, pin weight
 * w = rne(1024/(1+exp(-10(slack/WNS - 0.3)))) (Eq. 4 as a logistic; 0 if WNS >= 0),
 * batch of a net from its worst slack relative to WNS (Alg. 1 bins: 1, [0.99,1),
 * [0.96,.99), [0.91,.96), [0.84,.91), [0.75,.84), [0.7,.75), then 4 batches by net id).
 *  PLAIN: seg_w = max pin weight downstream (Eq. 5); lambda = (seg_w*r_est)>>10, r_est the
 *         average-R estimate from the driver to the segment's upper end (Sec. III-D).
 *  ADJOINT: J = sum over violating sinks of (w/1024)*slack; its reverse sweep gives
 *         seg_w = min(1024, rne(-1024 G)), pin_w = rne(-1024 g), lambda = rne(-Sig(parent)*1e6).
 *         Needs the forward sweep that produced `delay` to be the batch's last one and still
 *         current (LA_ERR_STATE otherwise, as for la_elmore_backward).
 * Outputs are device arrays sized [nodes], [sinks], [nodes], [nets].
 */
la_status la_timing_weights(la_batch *b, const float *delay, int32_t mode, uint16_t *seg_w_q10,
                            uint16_t *pin_w_q10, int32_t *lambda_mohm, uint8_t *net_tier);

/* Built-in congestion table: K=1024, out[l][z][i] = rne(1024*ofw[l]*(e^{s(d+1)}-e^{s d})),
 * d = i-32, s = 0.5 (z=0, capacity > 0) or 1.5 (z=1, capacity 0), saturating at 2^20.
 * ofw: HOST [L] (NULL = all 1); out: HOST [L*2*64]. */
la_status la_default_cong_lut(int32_t L, const double *ofw, int32_t *out);

/* Checkpoint of the negotiation state (demand, previous layers, round flag): with
 * host_buf NULL, *bytes receives the size; otherwise the state is copied out
 * (synchronises).  la_load_state restores it; history is the caller's own array. */
la_status la_save_state(la_batch *b, void *host_buf, size_t *bytes);
la_status la_load_state(la_batch *b, const void *host_buf, size_t bytes);

/* Wait for all work the batch enqueued. */
la_status la_sync(la_batch *b);

/* Kernel timing for roofline reports.  Between la_profile_begin and la_profile_end every
 * launch of the library's hot kernels is bracketed by hipEvents on the batch's stream, and
 * the batched form launches its kernels directly instead of replaying its hipGraph.
 * la_profile_end synchronises and writes, for up to `cap` kernels, the kernel name, the
 * number of launches and the summed launch durations (ms) into `out`, and the count to *n. */
typedef struct {
    char name[32];
    int32_t launches;
    double total_ms;
} la_kernel_stat;
la_status la_profile_begin(la_batch *b);
la_status la_profile_end(la_batch *b, la_kernel_stat *out, int32_t cap, int32_t *n);

void la_free_batch(la_batch *b);
const char *la_status_str(la_status s);
const char *la_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GAPLA_H */
