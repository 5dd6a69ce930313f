// C ABI entry points (include/gapla.h): argument checks, dispatch, state handling.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "la_internal.h"

namespace gapla {

static thread_local std::string g_last_error;

la_status set_error(la_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

la_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? LA_ERR_OOM : LA_ERR_HIP;
}

la_status build_batch(const la_nets *, const la_grid *, const la_layer_rc *, const uint8_t *, void *, la_batch **);
la_status timing_weights(la_batch *b, const float *delay, int32_t mode, uint16_t *seg_w, uint16_t *pin_w,
                         int32_t *lam, uint8_t *tier);
la_status timing_summary(la_batch *b, const float *delay, double *tns, double *wns);
la_status quality_report(la_batch *b, const double *ofw, const float *delay, const la_score_weights *sw,
                         la_quality *out);
la_status zero_i32(la_batch *b, int32_t *p, int64_t n);
la_status interleave_vias(la_batch *b, uint8_t *out);

KernelTimer::KernelTimer(la_batch *b, const char *name, hipStream_t s) : b_(b), s_(s)
{
    if (!b->prof_on) return;
    const size_t need = 2 * (b->prof_used + 1);
    while (b->prof_ev.size() < need) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;   // the launch then goes untimed
        b->prof_ev.push_back(e);
    }
    rec_ = b->prof_used;
    if (hipEventRecord(b->prof_ev[2 * rec_], s) != hipSuccess) {
        rec_ = SIZE_MAX;
        return;
    }
    if (b->prof_name.size() <= rec_) b->prof_name.resize(rec_ + 1);
    b->prof_name[rec_] = name;
    b->prof_used = rec_ + 1;
}

KernelTimer::~KernelTimer()
{
    if (rec_ == SIZE_MAX) return;
    (void)hipEventRecord(b_->prof_ev[2 * rec_ + 1], s_);
}

static void fill_tuning(const Tuning &t, la_tuning *o)
{
    o->tile_nodes = t.tile_nodes;
    o->claim_units = t.claim_units;
    o->workgroups = t.workgroups;
    o->fuse_nets = t.fuse_nets;
    o->tuned = t.tuned;
}

static la_status set_device(const la_batch *b)
{
    int cur = -1;
    LA_HIP(hipGetDevice(&cur));
    if (cur != b->device) LA_HIP(hipSetDevice(b->device));
    return LA_OK;
}

}  // namespace gapla

using namespace gapla;

extern "C" {

const char *la_status_str(la_status s)
{
    switch (s) {
    case LA_OK: return "LA_OK";
    case LA_ERR_INVALID_ARG: return "LA_ERR_INVALID_ARG";
    case LA_ERR_BAD_TREE: return "LA_ERR_BAD_TREE";
    case LA_ERR_RANGE: return "LA_ERR_RANGE";
    case LA_ERR_OOM: return "LA_ERR_OOM";
    case LA_ERR_HIP: return "LA_ERR_HIP";
    case LA_ERR_STATE: return "LA_ERR_STATE";
    }
    return "LA_ERR_UNKNOWN";
}

const char *la_last_error(void) { return g_last_error.c_str(); }

la_status la_default_cong_lut(int32_t L, const double *ofw, int32_t *out)
{
    if (L < 1 || L > kMaxL || !out) return set_error(LA_ERR_INVALID_ARG, "la_default_cong_lut: bad L or out");
    for (int l = 0; l < L; ++l) {
        const double w = ofw ? ofw[l] : 1.0;
        for (int z = 0; z < 2; ++z) {
            const double s = z == 0 ? 0.5 : 1.5;
            for (int i = 0; i < kNDelta; ++i) {
                const double d = (double)(i + kDeltaMin);
                const double v = 1024.0 * w * (std::exp(s * (d + 1.0)) - std::exp(s * d));
                out[(l * 2 + z) * kNDelta + i] = v >= (double)kLutSat ? kLutSat : (int32_t)std::nearbyint(v);
            }
        }
    }
    return LA_OK;
}

la_status la_build_batch(const la_nets *nets, const la_grid *grid, const la_layer_rc *layer_rc,
                         const uint8_t *edge_caps, void *stream, la_batch **out)
{
    return build_batch(nets, grid, layer_rc, edge_caps, stream, out);
}

la_status la_batch_info(const la_batch *b, la_info *o)
{
    if (!b || !o) return set_error(LA_ERR_INVALID_ARG, "la_batch_info: NULL argument");
    o->nets = b->nets;
    o->nodes = b->nodes;
    o->sinks = b->sinks;
    o->rc_edges = b->nodes + b->sinks;
    o->grid_edges = b->E;
    o->levels = b->levels;
    o->max_net_nodes = b->max_net_nodes;
    o->gcell_edges = b->gcell_edges;
    o->node_parent = b->parent;
    o->node_net = b->net;
    o->sink_node = b->sink_node;
    o->dp_ops_per_round = b->dp_ops;
    o->dp_bytes_per_round = b->dp_bytes;
    o->elmore_fwd_bytes = b->el_fwd_bytes;
    o->elmore_bwd_bytes = b->el_bwd_bytes;
    int ci = 0;
    while (ci < 2 && kTileCaps[ci] != b->tune.tile_nodes) ++ci;
    o->dp_ops_big_per_round = b->dp_ops_above[ci];
    o->graph_instantiations = b->graph_instantiations;
    fill_tuning(b->tune, &o->tuning);
    return LA_OK;
}

static la_status check_weights(const la_batch *b, const la_weights *w, const int32_t *history, const char *who)
{
    const std::string n(who);
    if (!b || !w || !history) return set_error(LA_ERR_INVALID_ARG, n + ": NULL batch, weights or history");
    if (!w->seg_w_q10 || !w->lambda_mohm || (b->sinks > 0 && !w->pin_w_q10))
        return set_error(LA_ERR_INVALID_ARG, n + ": weight arrays must be given");
    if (w->w_cong < 0 || w->w_cap < 0 || w->w_d < 0 || w->w_via < 0 || w->rounds < 1 || w->hist_inc < 0)
        return set_error(LA_ERR_INVALID_ARG, n + ": weights must be >= 0 and rounds >= 1");
    if (w->form != LA_FORM_PLAIN && w->form != LA_FORM_BATCHED)
        return set_error(LA_ERR_INVALID_ARG, n + ": unknown form");
    if (w->net_batch && (w->num_tiers < 1 || w->num_tiers > kMaxBatches))
        return set_error(LA_ERR_INVALID_ARG, n + ": num_tiers must be in 1..65536 with net_batch");
    if (!w->net_batch && w->net_tier && (w->num_tiers < 1 || w->num_tiers > 256))
        return set_error(LA_ERR_INVALID_ARG, n + ": num_tiers must be in 1..256");
    const double bound = (double)w->w_cong * b->bnd_cong + (double)w->w_cap * b->bnd_cap +
                         (double)w->w_via * b->bnd_via + (double)w->w_d * b->bnd_d;
    if (!(bound < 4.0e18) || w->w_d >= (int64_t(1) << 20))
        return set_error(LA_ERR_RANGE, n + ": weights could overflow a net's int64 cost");
    return LA_OK;
}

la_status la_tune(la_batch *b, const la_weights *w, const int32_t *history, la_tuning *out)
{
    la_status s = check_weights(b, w, history, "la_tune");
    if (s != LA_OK) return s;
    s = set_device(b);
    if (s != LA_OK) return s;
    if (b->nodes > 0) {
        const int32_t *batch = nullptr;
        s = batch_indices(b, w, &batch);
        if (s != LA_OK) return s;
        s = tune_batched(b, w, history, w->cong_lut ? w->cong_lut : b->lut, batch, true);
        if (s != LA_OK) return s;
    }
    if (out) fill_tuning(b->tune, out);
    return LA_OK;
}

la_status la_set_tuning(la_batch *b, const la_tuning *t)
{
    if (!b || !t) return set_error(LA_ERR_INVALID_ARG, "la_set_tuning: NULL argument");
    if (!tile_size_supported(b->NAmax, t->tile_nodes))
        return set_error(LA_ERR_INVALID_ARG, "la_set_tuning: tile size not built for this layer count");
    if (t->claim_units < kClaimUnitsMin || t->claim_units > kClaimUnitsMax || t->workgroups < 0 || t->fuse_nets < 1)
        return set_error(LA_ERR_INVALID_ARG, "la_set_tuning: claim units, workgroups or fuse threshold out of range");
    b->tune.tile_nodes = t->tile_nodes;
    b->tune.claim_units = t->claim_units;
    b->tune.workgroups = t->workgroups;
    b->tune.fuse_nets = t->fuse_nets;
    b->tune.tuned = 0;
    return LA_OK;
}

la_status la_get_batches(la_batch *b, const int32_t *net_subset, int32_t num_subsets, int32_t *out_batch,
                         int32_t *num_batches)
{
    if (!b || !num_batches || (b->nets > 0 && (!net_subset || !out_batch)))
        return set_error(LA_ERR_INVALID_ARG, "la_get_batches: NULL argument");
    if (num_subsets < 1 || num_subsets > 256)
        return set_error(LA_ERR_INVALID_ARG, "la_get_batches: num_subsets must be in 1..256");
    const la_status s = set_device(b);
    if (s != LA_OK) return s;
    return get_batches(b, net_subset, num_subsets, out_batch, num_batches);
}

la_status la_timing_graph(la_batch *b, const int32_t *sink_next, const int32_t *gate_delay_fs, int32_t clock_fs)
{
    if (!b || (b->sinks > 0 && !sink_next) || (b->nets > 0 && !gate_delay_fs))
        return set_error(LA_ERR_INVALID_ARG, "la_timing_graph: NULL argument");
    const la_status s = set_device(b);
    if (s != LA_OK) return s;
    return timing_graph(b, sink_next, gate_delay_fs, clock_fs);
}

la_status la_sta(la_batch *b, const float *sink_delay, float *out_slack, int32_t *out_crit, float *wns)
{
    if (!b || !wns || (b->sinks > 0 && (!sink_delay || !out_slack)) || (b->nets > 0 && !out_crit))
        return set_error(LA_ERR_INVALID_ARG, "la_sta: NULL argument");
    const la_status s = set_device(b);
    if (s != LA_OK) return s;
    return sta(b, sink_delay, out_slack, out_crit, wns);
}

la_status la_alg1_subsets(la_batch *b, const float *slack, const int32_t *crit, float wns, int32_t *out_subset,
                          int32_t *num_subsets)
{
    if (!b || !num_subsets || (b->nets > 0 && (!slack || !crit || !out_subset)))
        return set_error(LA_ERR_INVALID_ARG, "la_alg1_subsets: NULL argument");
    const la_status s = set_device(b);
    if (s != LA_OK) return s;
    return alg1_subsets(b, slack, crit, wns, out_subset, num_subsets);
}

la_status la_get_tuning(const la_batch *b, la_tuning *out)
{
    if (!b || !out) return set_error(LA_ERR_INVALID_ARG, "la_get_tuning: NULL argument");
    fill_tuning(b->tune, out);
    return LA_OK;
}

la_status la_assign(la_batch *b, const la_weights *w, int32_t *history, uint8_t *out_layers)
{
    la_status s = check_weights(b, w, history, "la_assign");
    if (s != LA_OK) return s;
    s = set_device(b);
    if (s != LA_OK) return s;
    const int32_t *lut = w->cong_lut ? w->cong_lut : b->lut;
    if (b->nodes == 0) return LA_OK;
    // the kernels read and update the history in the plane layout
    s = grid_to_planes(b, history, b->Hi);
    if (s != LA_OK) return s;
    const int32_t *batch = nullptr;
    s = batch_indices(b, w, &batch);
    if (s != LA_OK) return s;
    s = (w->form == LA_FORM_PLAIN) ? assign_plain(b, w, b->Hi, lut, out_layers, batch)
                                   : assign_batched(b, w, b->Hi, lut, out_layers, batch);
    if (s != LA_OK) return s;
    s = planes_to_grid(b, b->Hi, history);
    if (s != LA_OK) return s;
    return launch_rc_from_layers(b);
}

la_status la_vias(la_batch *b, uint8_t *out)
{
    if (!b || !out) return set_error(LA_ERR_INVALID_ARG, "la_vias: NULL argument");
    return interleave_vias(b, out);
}

la_status la_demand(la_batch *b, int32_t *out)
{
    if (!b || !out) return set_error(LA_ERR_INVALID_ARG, "la_demand: NULL argument");
    return planes_to_grid(b, b->D, out);
}

la_status la_reset(la_batch *b)
{
    if (!b) return set_error(LA_ERR_INVALID_ARG, "la_reset: NULL batch");
    la_status s = zero_i32(b, b->D, b->Eg);
    if (s != LA_OK) return s;
    LA_HIP(hipMemsetAsync(b->cur_layer, 0, b->nodes, b->stream));
    b->has_prev = false;
    b->fwd_done = b->bwd_done = false;
    return launch_rc_pre(b);
}

la_status la_batch_rc(la_batch *b, float **R, float **C)
{
    if (!b || !R || !C) return set_error(LA_ERR_INVALID_ARG, "la_batch_rc: NULL argument");
    *R = b->R;
    *C = b->C;
    return LA_OK;
}

la_status la_elmore(la_batch *b, float *out_delay)
{
    if (!b || (!out_delay && b->sinks)) return set_error(LA_ERR_INVALID_ARG, "la_elmore: NULL argument");
    return elmore_forward(b, b->R, b->C, out_delay);
}

la_status la_elmore_rc(la_batch *b, const float *R, const float *C, float *out_delay)
{
    if (!b || !R || !C || (!out_delay && b->sinks)) return set_error(LA_ERR_INVALID_ARG, "la_elmore_rc: NULL argument");
    return elmore_forward(b, R, C, out_delay);
}

la_status la_elmore_backward(la_batch *b, const float *dSlack, float *out_dR, float *out_dC)
{
    if (!b || (!dSlack && b->sinks)) return set_error(LA_ERR_INVALID_ARG, "la_elmore_backward: NULL argument");
    return elmore_backward(b, dSlack, true, out_dR, out_dC);
}

la_status la_quality_report(la_batch *b, const double *ofw, const float *delay, const la_score_weights *sw,
                            la_quality *out)
{
    if (!b || !out) return set_error(LA_ERR_INVALID_ARG, "la_quality_report: NULL batch or out");
    la_status s = set_device(b);
    if (s != LA_OK) return s;
    return quality_report(b, ofw, delay, sw, out);
}

la_status la_timing_summary(la_batch *b, const float *delay, double *tns, double *wns)
{
    if (!b || !tns || !wns || (!delay && b->sinks)) return set_error(LA_ERR_INVALID_ARG, "la_timing_summary: NULL");
    return timing_summary(b, delay, tns, wns);
}

la_status la_timing_summary_noalloc(la_batch *b, const float *delay, double *tns, double *wns)
{
    if (!b || !tns || !wns || (!delay && b->sinks))
        return set_error(LA_ERR_INVALID_ARG, "la_timing_summary_noalloc: NULL");
    const la_status s = set_device(b);
    if (s != LA_OK) return s;
    return timing_summary_noalloc(b, delay, tns, wns);
}

la_status la_timing_weights(la_batch *b, const float *delay, int32_t mode, uint16_t *seg_w, uint16_t *pin_w,
                            int32_t *lam, uint8_t *tier)
{
    if (!b || !seg_w || !lam || !tier || (b->sinks && (!delay || !pin_w)))
        return set_error(LA_ERR_INVALID_ARG, "la_timing_weights: NULL argument");
    if (mode != LA_WEIGHTS_PLAIN && mode != LA_WEIGHTS_ADJOINT)
        return set_error(LA_ERR_INVALID_ARG, "la_timing_weights: unknown mode");
    return timing_weights(b, delay, mode, seg_w, pin_w, lam, tier);
}

static const uint32_t kStateMagic = 0x4c415354u;   // "LAST"

la_status la_save_state(la_batch *b, void *host_buf, size_t *bytes)
{
    if (!b || !bytes) return set_error(LA_ERR_INVALID_ARG, "la_save_state: NULL argument");
    const size_t need = 16 + (size_t)b->Eg * sizeof(int32_t) + (size_t)b->nodes;
    if (!host_buf) {
        *bytes = need;
        return LA_OK;
    }
    if (*bytes < need) return set_error(LA_ERR_INVALID_ARG, "la_save_state: buffer too small");
    uint8_t *p = (uint8_t *)host_buf;
    uint32_t hdr[4] = {kStateMagic, (uint32_t)b->has_prev, (uint32_t)b->Eg, (uint32_t)b->nodes};
    memcpy(p, hdr, 16);
    LA_HIP(hipMemcpyAsync(p + 16, b->D, b->Eg * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    LA_HIP(hipMemcpyAsync(p + 16 + b->Eg * sizeof(int32_t), b->cur_layer, b->nodes, hipMemcpyDeviceToHost, b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    *bytes = need;
    return LA_OK;
}

la_status la_load_state(la_batch *b, const void *host_buf, size_t bytes)
{
    if (!b || !host_buf) return set_error(LA_ERR_INVALID_ARG, "la_load_state: NULL argument");
    const size_t need = 16 + (size_t)b->Eg * sizeof(int32_t) + (size_t)b->nodes;
    const uint8_t *p = (const uint8_t *)host_buf;
    uint32_t hdr[4];
    if (bytes < need) return set_error(LA_ERR_INVALID_ARG, "la_load_state: buffer too small");
    memcpy(hdr, p, 16);
    if (hdr[0] != kStateMagic || hdr[2] != (uint32_t)b->Eg || hdr[3] != (uint32_t)b->nodes)
        return set_error(LA_ERR_INVALID_ARG, "la_load_state: state of a different batch");
    LA_HIP(hipMemcpyAsync(b->D, p + 16, b->Eg * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    LA_HIP(hipMemcpyAsync(b->cur_layer, p + 16 + b->Eg * sizeof(int32_t), b->nodes, hipMemcpyHostToDevice, b->stream));
    LA_HIP(hipStreamSynchronize(b->stream));
    b->has_prev = hdr[1] != 0;
    return b->has_prev ? launch_rc_from_layers(b) : launch_rc_pre(b);
}

la_status la_sync(la_batch *b)
{
    if (!b) return set_error(LA_ERR_INVALID_ARG, "la_sync: NULL batch");
    LA_HIP(hipStreamSynchronize(b->stream));
    return LA_OK;
}

la_status la_profile_begin(la_batch *b)
{
    if (!b) return set_error(LA_ERR_INVALID_ARG, "la_profile_begin: NULL batch");
    if (b->prof_on) return set_error(LA_ERR_STATE, "la_profile_begin: profiling already on");
    b->prof_used = 0;
    b->prof_on = true;
    return LA_OK;
}

la_status la_profile_end(la_batch *b, la_kernel_stat *out, int32_t cap, int32_t *n)
{
    if (!b || !n || cap < 0 || (cap > 0 && !out)) return set_error(LA_ERR_INVALID_ARG, "la_profile_end: bad argument");
    if (!b->prof_on) return set_error(LA_ERR_STATE, "la_profile_end: profiling is not on");
    b->prof_on = false;
    const la_status sd = set_device(b);
    if (sd != LA_OK) return sd;
    LA_HIP(hipStreamSynchronize(b->stream));
    std::vector<la_kernel_stat> acc;
    for (size_t i = 0; i < b->prof_used; ++i) {
        float ms = 0.f;
        LA_HIP(hipEventElapsedTime(&ms, b->prof_ev[2 * i], b->prof_ev[2 * i + 1]));
        size_t k = 0;
        while (k < acc.size() && std::strncmp(acc[k].name, b->prof_name[i], sizeof(acc[k].name)) != 0) ++k;
        if (k == acc.size()) {
            la_kernel_stat z{};
            std::strncpy(z.name, b->prof_name[i], sizeof(z.name) - 1);
            acc.push_back(z);
        }
        acc[k].launches += 1;
        acc[k].total_ms += ms;
    }
    b->prof_used = 0;
    *n = (int32_t)acc.size();
    for (size_t k = 0; k < acc.size() && (int32_t)k < cap; ++k) out[k] = acc[k];
    return LA_OK;
}

void la_free_batch(la_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    void *ptrs[] = {b->parent, b->ch_ptr, b->ch, b->net, b->net_ptr, b->len, b->g0, b->cpin, b->sink_id,
                    b->sink_node, b->net_sink_ptr, b->rest, b->budget_fs, b->rdrv, b->dir, b->flags,
                    b->level_nodes, b->level_ptr, b->height, b->caps, b->D, b->cur_layer, b->vlo, b->vhi,
                    b->F, b->S, b->bt, b->sel, b->bucket_nodes, b->bucket_cnt, b->bucket_cur,
                    b->chg_node, b->chg_count, b->chg_old, b->chg_new, b->lut, b->R, b->C, b->el_S,
                    b->el_Slo, b->el_t, b->el_tlo, b->el_G, b->el_Glo, b->el_Sig, b->el_Siglo, b->slack,
                    b->scratch_f, b->wns_bits, b->red, b->net_big, b->net_zw, b->nrec, b->dynrec, b->cnet, b->bbox, b->batch_i32, b->sta_next, b->sta_fin_ptr, b->sta_fin,
                    b->sta_order, b->sta_gd, b->sta_f, b->sta_i, b->bn_order, b->bn_rec, b->bn_lvl, b->bn_lvl_off,
                    b->bn_nlev, b->tier_nets, b->tier_off, b->tier_cur, b->tier_cnt, b->claim,
                    b->cl_pre, b->cl_blk, b->cl_start, b->cl_off, b->D_alt, b->Hi,
                    b->e_tile, b->e_wrun, b->e_wpos, b->e_wchl, b->cpin_ff, b->budget_ps, b->rdrv_k, b->e_big_nodes, b->e_big_ptr, b->qofw, b->qpart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    delete b;
}

}  // extern "C"
