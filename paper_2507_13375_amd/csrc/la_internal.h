// Internal state of a layer-assignment batch and helpers shared by the HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gapla.h"

namespace gapla {

constexpr int kMaxL = 16;          // layers supported (4-bit layer ids)
constexpr int kQPartials = 2048 * 5;   // quality report: workgroups x partial sums
constexpr int kQSpan = 64;             // quality report: e^{s x} tabulated for integer x in [-kQSpan, kQSpan]
constexpr int kETile = 1024;        // nodes of one Elmore tile (whole nets, swept in one workgroup)
constexpr int kEMaxH = 128;         // tree heights an Elmore tile handles
constexpr int kWTile = 128;         // nodes of one wavefront's Elmore run (nets of at most that many nodes)
constexpr int kCap = 192;          // default nodes of one batched-form workgroup's LDS tile
constexpr int kTileCaps[3] = {128, 192, 256};   // tile sizes the batched form is built for
constexpr int kBigMin = 128;       // smallest tile: nets above it get their own level lists
constexpr int kClaimUnits = 220;   // default work-queue claim size: sum over its nets of (nodes + kNetUnits)
constexpr int kNetUnits = 3;
constexpr int kClaimUnitsMin = 96, kClaimUnitsMax = 316;   // claim sizes the autotuner may pick
constexpr int kClaimNets = 80;     // bound on the nets of one claim (kClaimUnitsMax / (1 + kNetUnits) + 1)
constexpr int32_t kFuseDefault = 16384;   // batches with this many small nets commit from their DP kernel
constexpr size_t kGraphSlots = 4;         // round graphs kept instantiated per batch
constexpr int32_t kMaxBatches = 65536;    // batches of one la_assign call given as int32 indices

// Launch configuration of the batched form (la_tune picks it per instance shape).
struct Tuning {
    int32_t tile_nodes = kCap;        // LDS tile capacity; nets above it run in the big-net kernel
    int32_t claim_units = kClaimUnits;
    int32_t workgroups = 0;           // persistent workgroups per launch; 0 = as many as fit the GPU
    int32_t fuse_nets = kFuseDefault;
    int32_t tuned = 0;                // 1 once la_tune chose it
};
constexpr int kMaxA = 8;           // routable layers per direction
constexpr int kHeightClasses = 32;   // batched work queue: height classes of small nets per batch
// partition buckets per batch: its big nets, then its small nets with a non-zero timing weight,
// then those whose weights are all zero, each by height class
constexpr int kPartBuckets = 1 + 2 * kHeightClasses;
constexpr int kNDelta = 64;        // congestion table entries per (layer, zero-capacity flag)
constexpr int kDeltaMin = -32;
constexpr int32_t kLutSat = 1 << 20;
constexpr int32_t kHistSat = 1 << 24;

// node flag bits
constexpr uint8_t kSink = 1, kDriver = 2, kRoot = 4;

// Layer table handed to kernels by value.
struct LayerTab {
    int32_t L, min_layer, X, Y;
    int32_t nA[2];                  // routable layers per direction
    int8_t lay[2][kMaxA];           // routable layers of each direction, ascending
    int8_t jidx[kMaxL];             // index of a layer inside its direction list, -1 if not routable
    uint8_t dir[kMaxL];
    int32_t r[kMaxL], c[kMaxL];     // mOhm / aF per GCell
    int32_t pv[kMaxL + 1];          // prefix sums of via R: Rvia(a,b) = |pv[a]-pv[b]|
    int32_t r_avg[2], c_avg[2];     // integer averages over routable layers per direction
    int32_t nAp[2];                 // record length per direction: nA rounded up to even (8-byte records)
    int32_t goff[3];                // grid-array regions: routable layers of direction 0, of 1, the rest
    int8_t nrk[kMaxL];              // rank of a layer among the non-routable ones
};

// Grid arrays inside the library are stored by direction: for each direction one record per
// GCell holding its routable layers of that direction (ascending; padded to an even count so
// that records are 8-byte aligned), records ordered along the
// direction -- horizontal row by row (x fastest), vertical column by column (y fastest) -- so
// a segment's GCell edges on all its candidate layers are consecutive words.  Non-routable
// layers follow, one plane each.  The API's arrays use (y * X + x) * L + l; la_assign and
// la_demand convert.
// position of GCell (x, y) along direction d
__host__ __device__ inline int32_t plane_pos(const LayerTab &t, int d, int32_t x, int32_t y)
{
    return d == 0 ? y * t.X + x : x * t.Y + y;
}
// index of the edge at position q of routable layer index jj of direction d
__host__ __device__ inline int32_t route_index(const LayerTab &t, int d, int jj, int32_t q)
{
    return t.goff[d] + q * t.nAp[d] + jj;
}
// index of the edge at position q (along layer l's direction) of any layer l
__host__ __device__ inline int32_t grid_index(const LayerTab &t, int l, int32_t q)
{
    return t.jidx[l] >= 0 ? route_index(t, t.dir[l], t.jidx[l], q) : t.goff[2] + t.nrk[l] * t.X * t.Y + q;
}

// Integer weights handed to the DP kernels.
struct DPWeights {
    int64_t w_cong, w_cap, w_d, w_via;
    const uint16_t *seg_w;
    const uint16_t *pin_w;
    const int32_t *lam;
    const int32_t *lut;
    int32_t self_excl;              // exclude each segment's previous demand
};

// Device view of the layer-assignment tree (canonical node order).
struct TreeDev {
    int64_t nets, nodes, sinks;
    const int32_t *parent;          // global parent, -1 at roots
    const int32_t *ch_ptr, *ch;     // children, ascending canonical index
    const int32_t *net;             // node -> net
    const int32_t *net_ptr;         // [nets+1]
    const int32_t *len;             // segment length (GCells), 0 at roots
    const int32_t *g0;              // in-plane index of the first GCell edge covered: the edge at
                                    // step k on layer l is grid_index(l, g0 + k)
    const uint8_t *dir;             // 0 H, 1 V (root: 0)
    const uint8_t *flags;
    const int32_t *cpin;            // aF, sinks only
    const float *cpin_ff;           // the same in fF, single precision (rounded once)
    const int32_t *sink_id;         // node -> sink or -1
    const int32_t *sink_node;       // [sinks]
    const int32_t *net_sink_ptr;    // [nets+1] sinks of a net are contiguous
    const int32_t *rest;            // average-R estimate (mOhm) from the driver to the segment's upper end
    const int32_t *budget_fs;       // per net
    const int32_t *rdrv;            // per net, mOhm
    const float *budget_ps;         // per net, ps (single precision, rounded once)
    const float *rdrv_k;            // per net, kOhm (single precision, rounded once)
};

}  // namespace gapla

struct la_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    gapla::LayerTab tab{};
    int64_t nets = 0, nodes = 0, sinks = 0, E = 0;
    int64_t Eg = 0;   // length of the library's grid arrays (E plus record padding)
    int32_t levels = 0, max_net_nodes = 0;
    int64_t gcell_edges = 0;
    int32_t NAmax = 0;              // stride of per-(node, layer index) DP arrays

    // per-net worst-case unit bounds for the range check (max over nets)
    double bnd_cong = 0, bnd_cap = 0, bnd_via = 0, bnd_d = 0;

    // host copies
    std::vector<int32_t> h_level_ptr;   // [levels+1]
    // Elmore: tiles of whole nets ([start, end) node pairs) and, grouped by height, the nodes of
    // the nets no tile takes
    int32_t *e_tile = nullptr, *e_big_nodes = nullptr, *e_big_ptr = nullptr;
    int32_t e_ntiles = 0;
    // wavefront runs of the nets of <= kWTile nodes: per run {first node, node count | max height
    // << 8 | the highest height in lane slots 0-63 << 16 | the lowest in slots 64-127 << 24, first
    // child entry, child entries}; per lane slot of a run (index first node + slot) {height |
    // (run-local parent + 1) << 8 | first child entry inside the run's entries << 16 | child
    // count << 24, run-local node id, sink id or -1, pin load in fF as float bits}; per child entry
    // of a run its run-local node id
    int32_t *e_wrun = nullptr;
    int32_t *e_wpos = nullptr;
    uint8_t *e_wchl = nullptr;
    int32_t e_nwtiles = 0;
    float *cpin_ff = nullptr;           // [nodes] pin load in fF (float)
    float *budget_ps = nullptr, *rdrv_k = nullptr;   // [nets] budget in ps, driver resistance in kOhm (float)
    std::vector<int32_t> h_ebig_ptr;    // [levels+1]
    std::vector<int32_t> h_net_ptr;
    std::vector<int16_t> h_bbox;        // [nets][4] x min, x max, y min, y max of the net's nodes
    int16_t *bbox = nullptr;            // the same on the device

    // device tree
    int32_t *parent = nullptr, *ch_ptr = nullptr, *ch = nullptr, *net = nullptr, *net_ptr = nullptr;
    int32_t *len = nullptr, *g0 = nullptr, *cpin = nullptr, *sink_id = nullptr, *sink_node = nullptr;
    int32_t *net_sink_ptr = nullptr, *rest = nullptr, *budget_fs = nullptr, *rdrv = nullptr;
    uint8_t *dir = nullptr, *flags = nullptr;
    int32_t *level_nodes = nullptr, *level_ptr = nullptr, *height = nullptr;
    uint8_t *caps = nullptr;

    // negotiation state; D_alt receives a batch's demand moves while its DP reads D (batched form).
    // caps, D, D_alt and Hi (the history during la_assign) use the plane layout of grid_index.
    int32_t *D = nullptr, *D_alt = nullptr, *Hi = nullptr;
    uint8_t *cur_layer = nullptr, *vlo = nullptr, *vhi = nullptr;
    bool has_prev = false;

    // plain-form DP state
    int64_t *F = nullptr;
    int32_t *S = nullptr;
    uint8_t *bt = nullptr, *sel = nullptr;
    int32_t *bucket_nodes = nullptr, *bucket_cnt = nullptr, *bucket_cur = nullptr;
    size_t bucket_cap = 0;

    // changed-segment list of the current batch (tier)
    int32_t *chg_node = nullptr, *chg_count = nullptr;
    uint8_t *chg_old = nullptr, *chg_new = nullptr;

    // default congestion table (device)
    int32_t *lut = nullptr;

    // batched form: nets too large for one workgroup's LDS keep their DP state in HBM and
    // walk their own height levels (bn_order: node ids per net by height; bn_lvl: level
    // starts into bn_order; bn_lvl_off/bn_nlev: each big net's first level and level count)
    int32_t *net_big = nullptr;
    uint8_t *net_zw = nullptr;      // per net: 1 when every timing weight the DP reads is zero
    // tile staging: a static 16-byte record per node (built at la_build_batch), the weights of
    // the current la_assign call per node (look-ahead coefficient, segment | pin weight << 16),
    // and per position of the batch-sorted net list its first node, node count, first child
    // entry and zero-weight flag
    uint32_t *nrec = nullptr, *dynrec = nullptr;
    int32_t *cnet = nullptr;
    int32_t *bn_order = nullptr, *bn_lvl = nullptr, *bn_lvl_off = nullptr, *bn_nlev = nullptr;
    int32_t *bn_rec = nullptr;      // [bn_order positions][12]: the node's record for the level walk (per call)
    int32_t n_big = 0;
    int32_t *tier_nets = nullptr, *tier_off = nullptr, *tier_cur = nullptr, *tier_cnt = nullptr;
    int32_t *claim = nullptr;
    int32_t claim_cap = 0;
    // claims of the batched work queue: prefix of (nodes + kNetUnits) over the batch-sorted nets,
    // per-block partial sums of that scan, claim starts (positions in tier_nets) and per-batch
    // claim offsets
    int32_t *cl_pre = nullptr, *cl_blk = nullptr, *cl_start = nullptr, *cl_off = nullptr;
    int64_t cl_start_cap = 0;
    int32_t part_cap = 256;         // batches the partition and claim arrays hold
    int32_t *batch_i32 = nullptr;   // [nets] u8 batch indices widened for the kernels

    // gate-level timing graph of Alg. 1 (la_timing_graph): per sink the net it feeds, the fan-in
    // sinks of each net's gate, the nets in topological order (level starts on the host), gate
    // delays (ps); work arrays of the timing (AD, RD per net, AS, RS per sink; latest input)
    int32_t *sta_next = nullptr, *sta_fin_ptr = nullptr, *sta_fin = nullptr, *sta_order = nullptr;
    float *sta_gd = nullptr, *sta_f = nullptr;
    int32_t *sta_i = nullptr;
    std::vector<int32_t> sta_lvl;
    float sta_clock = 0.f;
    bool sta_ready = false;
    std::vector<int32_t> h_net_sink_ptr;   // [nets+1] host copy
    hipStream_t cap_stream = nullptr;
    // the big nets' DP kernel runs on its own stream beside the tile kernel, forked and joined by events
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // instantiated round graphs of the batched form by call key, most recently used first
    std::vector<std::pair<std::vector<int64_t>, hipGraphExec_t>> graphs;
    int64_t graph_instantiations = 0;

    // RC and Elmore state
    float *R = nullptr, *C = nullptr;   // batch RC views [nodes+sinks]
    bool rc_assigned = false;
    float *el_S = nullptr, *el_Slo = nullptr, *el_t = nullptr, *el_tlo = nullptr;
    float *el_G = nullptr, *el_Glo = nullptr, *el_Sig = nullptr, *el_Siglo = nullptr;
    const float *fwd_R = nullptr, *fwd_C = nullptr;
    bool fwd_done = false, bwd_done = false;
    float *slack = nullptr;
    float *scratch_f = nullptr;         // [sinks] temporaries
    uint32_t *wns_bits = nullptr;       // ordered-int encoding of the WNS float
    double *red = nullptr;              // reduction partials
    double *qofw = nullptr;             // overflow weights and exponential table of the quality report
    double *qpart = nullptr;            // [kQPartials] its workgroup partial sums
    int32_t red_blocks = 0;

    // algorithmic work per DP round and per Elmore sweep (computed at build); the part of the
    // DP work in nets above each tile size of kTileCaps
    double dp_ops = 0, dp_bytes = 0, el_fwd_bytes = 0, el_bwd_bytes = 0;
    double dp_ops_above[3] = {0, 0, 0};
    gapla::Tuning tune;

    // kernel timing (la_profile_begin/end): an event pair per bracketed launch
    bool prof_on = false;
    std::vector<const char *> prof_name;
    std::vector<hipEvent_t> prof_ev;    // 2 per record, reused across sessions
    size_t prof_used = 0;
};

namespace gapla {

// errors ---------------------------------------------------------------------
la_status set_error(la_status s, const std::string &msg);
la_status hip_fail(hipError_t e, const char *what);

#define LA_HIP(call)                                                \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return gapla::hip_fail(e_, #call);    \
    } while (0)

TreeDev tree_view(const la_batch *b);

// Brackets the launches made in its scope with events on `s` while profiling is on.
class KernelTimer {
public:
    KernelTimer(la_batch *b, const char *name, hipStream_t s);
    ~KernelTimer();
    KernelTimer(const KernelTimer &) = delete;
    KernelTimer &operator=(const KernelTimer &) = delete;

private:
    la_batch *b_;
    hipStream_t s_;
    size_t rec_ = SIZE_MAX;
};

#define LA_TIMED(b, name, s, ...)                         \
    do {                                                  \
        gapla::KernelTimer kt_((b), (name), (s));         \
        __VA_ARGS__;                                      \
    } while (0)

// kernels launched from more than one source file
la_status launch_rc_from_layers(la_batch *b);
la_status launch_rc_pre(la_batch *b);
la_status elmore_forward(la_batch *b, const float *R, const float *C, float *delay);
// with seg_w (and no dR, dC) the wavefront runs also write the adjoint-form weights of their nodes
la_status elmore_backward(la_batch *b, const float *gbar_neg_dslack, bool from_dslack, float *dR, float *dC,
                          uint16_t *seg_w = nullptr, uint16_t *pin_w = nullptr, int32_t *lam = nullptr);
la_status commit_changed(la_batch *b, int32_t *D);
// conversions between the API's grid order (E int32) and the library's layout (Eg int32)
la_status grid_to_planes(la_batch *b, const int32_t *api, int32_t *planes);
la_status planes_to_grid(la_batch *b, const int32_t *planes, int32_t *api);
la_status history_update(la_batch *b, const int32_t *D, int32_t *H, int32_t hist_inc);
la_status assign_plain(la_batch *b, const la_weights *w, int32_t *H, const int32_t *lut, uint8_t *out_layers,
                       const int32_t *batch);
// batch: device [nets] int32 batch of each net (NULL: one batch)
la_status assign_batched(la_batch *b, const la_weights *w, int32_t *H, const int32_t *lut, uint8_t *out_layers,
                         const int32_t *batch, bool direct = false);
bool tile_size_supported(int NA, int cap);
// classical batching (Alg. 1 GetBatch) of the nets by subset; synchronises
la_status get_batches(la_batch *b, const int32_t *subset, int32_t nsub, int32_t *out_batch, int32_t *num_batches);
// picks b->tune on the instance (or from the cache of instance shapes); state is unchanged
la_status tune_batched(la_batch *b, const la_weights *w, const int32_t *history, const int32_t *lut,
                       const int32_t *batch, bool use_cache);
// the batch indices the forms read: the caller's int32 array, a widened copy of its u8 tiers, or NULL
la_status batch_indices(la_batch *b, const la_weights *w, const int32_t **out);
// Alg. 1's ordering on a gate graph over the nets (sta.hip)
la_status timing_graph(la_batch *b, const int32_t *sink_next, const int32_t *gate_fs, int32_t clock_fs);
la_status sta(la_batch *b, const float *delay, float *slack, int32_t *crit, float *wns_out);
la_status alg1_subsets(la_batch *b, const float *slack, const int32_t *crit, float wns, int32_t *subset,
                       int32_t *num_subsets);
// the static scratch of the allocation-free entry point: its address on `device` (once per device)
la_status scratch_setup(int device);
la_status timing_summary_noalloc(la_batch *b, const float *delay, double *tns, double *wns);

}  // namespace gapla
