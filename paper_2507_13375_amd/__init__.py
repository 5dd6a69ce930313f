"""Python binding of libgapla.so (include/gapla.h): GAP-LA layer assignment and
Elmore timing on MI355X.

Every function here only marshals arguments: torch tensors on the GPU supply
device memory and the current HIP stream; all work runs in the library's HIP
kernels.  There is no CPU fallback: importing a function without the built
library raises at once.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgapla.so")
_lib = None

LA_OK, LA_ERR_INVALID_ARG, LA_ERR_BAD_TREE, LA_ERR_RANGE, LA_ERR_OOM, LA_ERR_HIP, LA_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
LA_FORM_PLAIN, LA_FORM_BATCHED = 0, 1
LA_WEIGHTS_PLAIN, LA_WEIGHTS_ADJOINT = 0, 1
W_CONG, W_CAP, W_D, W_VIA, HIST_INC = 1000, 100, 1, 100000, 64

EXPORTS = ["la_build_batch", "la_batch_info", "la_assign", "la_vias", "la_demand", "la_reset", "la_batch_rc",
           "la_elmore", "la_elmore_rc", "la_elmore_backward", "la_timing_summary", "la_timing_summary_noalloc",
           "la_quality_report",
           "la_timing_weights",
           "la_default_cong_lut", "la_save_state", "la_load_state", "la_sync", "la_profile_begin", "la_profile_end",
           "la_tune", "la_set_tuning", "la_get_tuning", "la_get_batches", "la_timing_graph", "la_sta",
           "la_alg1_subsets",
           "la_free_batch", "la_status_str", "la_last_error"]

V, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64


class la_nets(ctypes.Structure):
    _fields_ = [("num_nets", I32), ("num_nodes", I32), ("num_waypoints", I32), ("net_node_ptr", V),
                ("node_parent", V), ("node_x", V), ("node_y", V), ("node_flags", V), ("node_cpin_af", V),
                ("edge_wp_ptr", V), ("wp_x", V), ("wp_y", V), ("net_budget_fs", V), ("net_rdrv_mohm", V)]


class la_grid(ctypes.Structure):
    _fields_ = [("X", I32), ("Y", I32), ("L", I32), ("min_layer", I32), ("layer_dir", V)]


class la_layer_rc(ctypes.Structure):
    _fields_ = [("r_mohm", V), ("c_af", V), ("via_r_mohm", V)]


class la_tuning(ctypes.Structure):
    _fields_ = [("tile_nodes", I32), ("claim_units", I32), ("workgroups", I32), ("fuse_nets", I32), ("tuned", I32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class la_info(ctypes.Structure):
    _fields_ = [("nets", I64), ("nodes", I64), ("sinks", I64), ("rc_edges", I64), ("grid_edges", I64),
                ("levels", I32), ("max_net_nodes", I32), ("gcell_edges", I64), ("node_parent", V),
                ("node_net", V), ("sink_node", V), ("dp_ops_per_round", ctypes.c_double),
                ("dp_bytes_per_round", ctypes.c_double), ("elmore_fwd_bytes", ctypes.c_double),
                ("elmore_bwd_bytes", ctypes.c_double), ("dp_ops_big_per_round", ctypes.c_double),
                ("graph_instantiations", I64), ("tuning", la_tuning)]


class la_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", I32), ("total_ms", ctypes.c_double)]


class la_score_weights(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("w1", "w2", "w3", "w4", "r1", "r2", "r3")]


class la_quality(ctypes.Structure):
    _fields_ = [("tof", ctypes.c_double), ("overflow_sum", I64), ("overflow_edges", I64), ("vias", I64),
                ("wire_cap_af", I64), ("wns_ps", ctypes.c_double), ("tns_ps", ctypes.c_double),
                ("score", ctypes.c_double)]


class la_weights(ctypes.Structure):
    _fields_ = [("w_cong", I64), ("w_cap", I64), ("w_d", I64), ("w_via", I64), ("seg_w_q10", V),
                ("pin_w_q10", V), ("lambda_mohm", V), ("net_tier", V), ("cong_lut", V), ("rounds", I32),
                ("hist_inc", I32), ("form", I32), ("num_tiers", I32), ("net_batch", V)]


class LAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_status_name(code), msg))
        self.code = code


def _status_name(code):
    try:
        return _load().la_status_str(code).decode()
    except Exception:
        return str(code)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgapla.so is not built (run __graft_entry__.build()); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        lib.la_status_str.restype = ctypes.c_char_p
        lib.la_status_str.argtypes = [ctypes.c_int]
        lib.la_last_error.restype = ctypes.c_char_p
        lib.la_build_batch.argtypes = [ctypes.POINTER(la_nets), ctypes.POINTER(la_grid), ctypes.POINTER(la_layer_rc),
                                       V, V, ctypes.POINTER(V)]
        lib.la_batch_info.argtypes = [V, ctypes.POINTER(la_info)]
        lib.la_assign.argtypes = [V, ctypes.POINTER(la_weights), V, V]
        lib.la_vias.argtypes = [V, V]
        lib.la_demand.argtypes = [V, V]
        lib.la_reset.argtypes = [V]
        lib.la_batch_rc.argtypes = [V, ctypes.POINTER(V), ctypes.POINTER(V)]
        lib.la_elmore.argtypes = [V, V]
        lib.la_elmore_rc.argtypes = [V, V, V, V]
        lib.la_elmore_backward.argtypes = [V, V, V, V]
        lib.la_timing_summary.argtypes = [V, V, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.la_timing_summary_noalloc.argtypes = [V, V, ctypes.POINTER(ctypes.c_double),
                                                  ctypes.POINTER(ctypes.c_double)]
        lib.la_quality_report.argtypes = [V, V, V, ctypes.POINTER(la_score_weights), ctypes.POINTER(la_quality)]
        lib.la_timing_weights.argtypes = [V, V, I32, V, V, V, V]
        lib.la_default_cong_lut.argtypes = [I32, V, V]
        lib.la_save_state.argtypes = [V, V, ctypes.POINTER(ctypes.c_size_t)]
        lib.la_load_state.argtypes = [V, V, ctypes.c_size_t]
        lib.la_tune.argtypes = [V, ctypes.POINTER(la_weights), V, ctypes.POINTER(la_tuning)]
        lib.la_set_tuning.argtypes = [V, ctypes.POINTER(la_tuning)]
        lib.la_get_tuning.argtypes = [V, ctypes.POINTER(la_tuning)]
        lib.la_get_batches.argtypes = [V, V, I32, V, ctypes.POINTER(I32)]
        lib.la_timing_graph.argtypes = [V, V, V, I32]
        lib.la_sta.argtypes = [V, V, V, V, ctypes.POINTER(ctypes.c_float)]
        lib.la_alg1_subsets.argtypes = [V, V, V, ctypes.c_float, V, ctypes.POINTER(I32)]
        lib.la_sync.argtypes = [V]
        lib.la_profile_begin.argtypes = [V]
        lib.la_profile_end.argtypes = [V, ctypes.POINTER(la_kernel_stat), I32, ctypes.POINTER(I32)]
        lib.la_free_batch.argtypes = [V]
        lib.la_free_batch.restype = None
        for name in EXPORTS:
            if name not in ("la_status_str", "la_last_error", "la_free_batch"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _chk(code, what):
    if code != LA_OK:
        raise LAError(code, "%s: %s" % (what, _load().la_last_error().decode()))


def _np(a):
    return None if a is None else np.ascontiguousarray(a).ctypes.data_as(V)


def _dev(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return V(t.data_ptr())


def _stream():
    import torch
    return V(torch.cuda.current_stream().cuda_stream)


def _on(b):
    """The batch's handle, after checking that torch's current stream is the batch's stream.

    The library enqueues every call on the stream the batch was built with, while torch
    allocates and frees the tensors it is handed on its current stream; with two different
    streams torch could reuse a buffer the library still reads, or read an output early."""
    import torch
    cur = torch.cuda.current_stream().cuda_stream or 0
    if cur != b.stream:
        raise ValueError("batch built on stream %#x but torch's current stream is %#x; call it under "
                         "torch.cuda.stream() of the batch's stream" % (b.stream, cur))
    return b.h


class Batch:
    """Owns one la_batch handle and its sizes."""

    def __init__(self, handle, inst, stream=0):
        self.h = handle
        self.stream = int(stream or 0)
        info = la_info()
        _chk(_load().la_batch_info(self.h, ctypes.byref(info)), "la_batch_info")
        self.nets, self.nodes, self.sinks = info.nets, info.nodes, info.sinks
        self.rc_edges, self.grid_edges, self.levels = info.rc_edges, info.grid_edges, info.levels
        self.max_net_nodes, self.gcell_edges = info.max_net_nodes, info.gcell_edges
        self.dp_ops_per_round, self.dp_bytes_per_round = info.dp_ops_per_round, info.dp_bytes_per_round
        self.elmore_fwd_bytes, self.elmore_bwd_bytes = info.elmore_fwd_bytes, info.elmore_bwd_bytes
        self.dp_ops_big_per_round = info.dp_ops_big_per_round
        self.X, self.Y, self.L = inst.X, inst.Y, inst.L
        self._info = info

    def free(self):
        if self.h is not None and _lib is not None:
            _lib.la_free_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def la_build_batch(inst, min_layer: int = 0, stream=None) -> Batch:
    """Build a batch from an instance (any object with the la_nets / grid / RC arrays as attributes)."""
    lib = _load()
    keep = dict(
        net_node_ptr=np.ascontiguousarray(inst.net_node_ptr, np.int32),
        node_parent=np.ascontiguousarray(inst.node_parent, np.int32),
        node_x=np.ascontiguousarray(inst.node_x, np.int16), node_y=np.ascontiguousarray(inst.node_y, np.int16),
        node_flags=np.ascontiguousarray(inst.node_flags, np.uint8),
        node_cpin_af=np.ascontiguousarray(inst.node_cpin_af, np.int32),
        edge_wp_ptr=np.ascontiguousarray(inst.edge_wp_ptr, np.int32),
        wp_x=np.ascontiguousarray(inst.wp_x, np.int16), wp_y=np.ascontiguousarray(inst.wp_y, np.int16),
        net_budget_fs=np.ascontiguousarray(inst.net_budget_fs, np.int32),
        net_rdrv_mohm=np.ascontiguousarray(inst.net_rdrv_mohm, np.int32),
        layer_dir=np.ascontiguousarray(inst.layer_dir, np.uint8), r=np.ascontiguousarray(inst.r_mohm, np.int32),
        c=np.ascontiguousarray(inst.c_af, np.int32), vr=np.ascontiguousarray(inst.via_r_mohm, np.int32),
        caps=np.ascontiguousarray(inst.caps, np.uint8))
    k = keep
    nets = la_nets(len(k["net_node_ptr"]) - 1, len(k["node_parent"]), len(k["wp_x"]), _np(k["net_node_ptr"]),
                   _np(k["node_parent"]), _np(k["node_x"]), _np(k["node_y"]), _np(k["node_flags"]),
                   _np(k["node_cpin_af"]), _np(k["edge_wp_ptr"]), _np(k["wp_x"]), _np(k["wp_y"]),
                   _np(k["net_budget_fs"]), _np(k["net_rdrv_mohm"]))
    grid = la_grid(inst.X, inst.Y, inst.L, min_layer, _np(k["layer_dir"]))
    rc = la_layer_rc(_np(k["r"]), _np(k["c"]), _np(k["vr"]))
    h = V()
    s = stream if stream is not None else _stream()
    s = s.value if isinstance(s, V) else s
    _chk(lib.la_build_batch(ctypes.byref(nets), ctypes.byref(grid), ctypes.byref(rc), _np(k["caps"]), V(s),
                            ctypes.byref(h)), "la_build_batch")
    return Batch(h, inst, s)


def la_free_batch(b: Batch):
    b.free()


def la_assign(b: Batch, seg_w_q10, pin_w_q10, lambda_mohm, history, out_layers, net_tier=None, num_tiers=1,
              w_cong=W_CONG, w_cap=W_CAP, w_d=W_D, w_via=W_VIA, rounds=1, hist_inc=HIST_INC, form=LA_FORM_PLAIN,
              cong_lut=None, net_batch=None):
    """net_tier: u8 batch per net (<= 256 batches); net_batch: int32 batch per net (replaces it)."""
    w = la_weights(w_cong, w_cap, w_d, w_via, _dev(seg_w_q10), _dev(pin_w_q10), _dev(lambda_mohm), _dev(net_tier),
                   _dev(cong_lut), rounds, hist_inc, form, num_tiers, _dev(net_batch))
    _chk(_load().la_assign(_on(b), ctypes.byref(w), _dev(history), _dev(out_layers)), "la_assign")


def la_tune(b: Batch, seg_w_q10, pin_w_q10, lambda_mohm, history, net_tier=None, num_tiers=1, w_cong=W_CONG,
            w_cap=W_CAP, w_d=W_D, w_via=W_VIA, hist_inc=HIST_INC, cong_lut=None, net_batch=None) -> dict:
    """Autotune the batched form on this instance (one round per candidate, state restored)."""
    w = la_weights(w_cong, w_cap, w_d, w_via, _dev(seg_w_q10), _dev(pin_w_q10), _dev(lambda_mohm), _dev(net_tier),
                   _dev(cong_lut), 1, hist_inc, LA_FORM_BATCHED, num_tiers, _dev(net_batch))
    t = la_tuning()
    _chk(_load().la_tune(_on(b), ctypes.byref(w), _dev(history), ctypes.byref(t)), "la_tune")
    return t.as_dict()


def la_set_tuning(b: Batch, tile_nodes=192, claim_units=220, workgroups=0, fuse_nets=16384):
    t = la_tuning(tile_nodes, claim_units, workgroups, fuse_nets, 0)
    _chk(_load().la_set_tuning(b.h, ctypes.byref(t)), "la_set_tuning")


def la_get_tuning(b: Batch) -> dict:
    t = la_tuning()
    _chk(_load().la_get_tuning(b.h, ctypes.byref(t)), "la_get_tuning")
    return t.as_dict()


def la_batch_info(b: Batch) -> dict:
    """The batch's sizes, work figures, graph count and launch configuration."""
    info = la_info()
    _chk(_load().la_batch_info(b.h, ctypes.byref(info)), "la_batch_info")
    out = {k: getattr(info, k) for k, _ in la_info._fields_ if k not in ("node_parent", "node_net", "sink_node", "tuning")}
    out["tuning"] = info.tuning.as_dict()
    return out


def la_get_batches(b: Batch, net_subset, num_subsets, out_batch) -> int:
    """Classical batching (Alg. 1 GetBatch) of the nets by subset; returns the batch count."""
    n = I32()
    _chk(_load().la_get_batches(_on(b), _dev(net_subset), int(num_subsets), _dev(out_batch), ctypes.byref(n)),
         "la_get_batches")
    return n.value


def la_timing_graph(b: Batch, sink_next, gate_delay_fs, clock_fs: int):
    """Gate graph over the nets for Alg. 1 (host arrays: net fed by each sink or -1; gate delays, fs)."""
    nxt = np.ascontiguousarray(sink_next, np.int32)
    gd = np.ascontiguousarray(gate_delay_fs, np.int32)
    _chk(_load().la_timing_graph(b.h, V(nxt.ctypes.data), V(gd.ctypes.data), int(clock_fs)), "la_timing_graph")


def la_sta(b: Batch, sink_delay, out_slack, out_crit) -> float:
    """Static timing of the gate graph and critical-path counts (Alg. 1: static timing and critical-path counts); returns WNS."""
    w = ctypes.c_float()
    _chk(_load().la_sta(_on(b), _dev(sink_delay), _dev(out_slack), _dev(out_crit), ctypes.byref(w)), "la_sta")
    return w.value


def la_alg1_subsets(b: Batch, slack, crit, wns: float, out_subset) -> int:
    """Alg. 1 division and partition: ordered subsets of the nets; returns their number."""
    n = I32()
    _chk(_load().la_alg1_subsets(_on(b), _dev(slack), _dev(crit), ctypes.c_float(wns), _dev(out_subset),
                                 ctypes.byref(n)), "la_alg1_subsets")
    return n.value


def la_vias(b: Batch, out_lo_hi):
    _chk(_load().la_vias(_on(b), _dev(out_lo_hi)), "la_vias")


def la_demand(b: Batch, out):
    _chk(_load().la_demand(_on(b), _dev(out)), "la_demand")


def la_reset(b: Batch):
    _chk(_load().la_reset(_on(b)), "la_reset")


def la_batch_rc(b: Batch):
    """(R, C) device pointers of the batch-owned float views [rc_edges]."""
    R, C = V(), V()
    _chk(_load().la_batch_rc(b.h, ctypes.byref(R), ctypes.byref(C)), "la_batch_rc")
    return R.value, C.value


def la_elmore(b: Batch, out_delay):
    _chk(_load().la_elmore(_on(b), _dev(out_delay)), "la_elmore")


def la_elmore_rc(b: Batch, R, C, out_delay):
    _chk(_load().la_elmore_rc(_on(b), _dev(R), _dev(C), _dev(out_delay)), "la_elmore_rc")


def la_elmore_backward(b: Batch, dSlack, out_dR, out_dC):
    _chk(_load().la_elmore_backward(_on(b), _dev(dSlack), _dev(out_dR), _dev(out_dC)), "la_elmore_backward")


def la_timing_summary(b: Batch, delay):
    tns, wns = ctypes.c_double(), ctypes.c_double()
    _chk(_load().la_timing_summary(_on(b), _dev(delay), ctypes.byref(tns), ctypes.byref(wns)), "la_timing_summary")
    return tns.value, wns.value


def la_timing_summary_noalloc(b: Batch, delay):
    """la_timing_summary without any allocation (its partials sit in the library's static
    device scratch); calls on one GPU must not overlap."""
    tns, wns = ctypes.c_double(), ctypes.c_double()
    _chk(_load().la_timing_summary_noalloc(_on(b), _dev(delay), ctypes.byref(tns), ctypes.byref(wns)),
         "la_timing_summary_noalloc")
    return tns.value, wns.value


def la_quality_report(b: Batch, ofw=None, delay=None, weights=None) -> dict:
    """Quality terms of the current assignment: Eq. 3 and Eq. 2 total overflow, overflowed
    edges, vias, wire capacitance (aF); WNS, TNS and the Eq. 1 score when delays are given.
    weights: dict of w1..w4, r1..r3 (missing keys 0)."""
    w = None
    if ofw is not None:
        w = np.ascontiguousarray(ofw, np.float64)
    sw = None
    if weights is not None:
        sw = la_score_weights(*[float(weights.get(k, 0.0)) for k in ("w1", "w2", "w3", "w4", "r1", "r2", "r3")])
    q = la_quality()
    _chk(_load().la_quality_report(_on(b), None if w is None else w.ctypes.data, _dev(delay),
                                   None if sw is None else ctypes.byref(sw), ctypes.byref(q)), "la_quality_report")
    return {k: getattr(q, k) for k, _ in la_quality._fields_}


def la_timing_weights(b: Batch, delay, mode, seg_w_q10, pin_w_q10, lambda_mohm, net_tier):
    _chk(_load().la_timing_weights(_on(b), _dev(delay), mode, _dev(seg_w_q10), _dev(pin_w_q10), _dev(lambda_mohm),
                                   _dev(net_tier)), "la_timing_weights")


def la_default_cong_lut(L: int, ofw=None) -> np.ndarray:
    out = np.empty((L, 2, 64), np.int32)
    _chk(_load().la_default_cong_lut(L, _np(None if ofw is None else np.asarray(ofw, np.float64)), _np(out)),
         "la_default_cong_lut")
    return out


def la_save_state(b: Batch) -> bytes:
    n = ctypes.c_size_t()
    _chk(_load().la_save_state(_on(b), None, ctypes.byref(n)), "la_save_state")
    buf = ctypes.create_string_buffer(n.value)
    _chk(_load().la_save_state(_on(b), buf, ctypes.byref(n)), "la_save_state")
    return buf.raw


def la_load_state(b: Batch, state: bytes):
    buf = ctypes.create_string_buffer(state, len(state))
    _chk(_load().la_load_state(_on(b), buf, len(state)), "la_load_state")


def la_sync(b: Batch):
    _chk(_load().la_sync(_on(b)), "la_sync")


def la_profile_begin(b: Batch):
    _chk(_load().la_profile_begin(b.h), "la_profile_begin")


def la_profile_end(b: Batch) -> dict:
    """{kernel name: (launches, summed launch time in ms)} of the launches since la_profile_begin."""
    cap = 64
    out = (la_kernel_stat * cap)()
    n = I32(0)
    _chk(_load().la_profile_end(b.h, out, cap, ctypes.byref(n)), "la_profile_end")
    return {out[i].name.decode(): (out[i].launches, out[i].total_ms) for i in range(min(n.value, cap))}


def la_status_str(code: int) -> str:
    return _load().la_status_str(code).decode()


def la_last_error() -> str:
    return _load().la_last_error().decode()


def _elmore_fn():
    import torch

    class ElmoreFn(torch.autograd.Function):
        """delay = Elmore(R, C) on a batch's trees; backward is the library's reverse sweep."""

        @staticmethod
        def forward(ctx, R, C, batch):
            delay = torch.empty(batch.sinks, dtype=torch.float32, device=R.device)
            R, C = R.contiguous(), C.contiguous()
            la_elmore_rc(batch, R, C, delay)
            ctx.batch = batch
            ctx.save_for_backward(R, C)
            return delay

        @staticmethod
        def backward(ctx, g):
            R, C = ctx.saved_tensors
            b = ctx.batch
            scratch = torch.empty(b.sinks, dtype=torch.float32, device=R.device)
            la_elmore_rc(b, R, C, scratch)          # the reverse sweep reads the forward's state
            dR = torch.empty_like(R)
            dC = torch.empty_like(C)
            la_elmore_backward(b, (-g).contiguous(), dR, dC)   # dJ/dslack = -dJ/ddelay
            return dR, dC, None

    return ElmoreFn


_ELMORE = None


def elmore(R, C, batch):
    """Differentiable Elmore delay (torch.autograd.Function over la_elmore_rc / la_elmore_backward)."""
    global _ELMORE
    if _ELMORE is None:
        _ELMORE = _elmore_fn()
    return _ELMORE.apply(R, C, batch)
