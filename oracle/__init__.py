"""ORACLE -- test infrastructure only.

A plain CPU statement (C, FP64 timing, int64 costs) of the GAP-LA layer
assignment hot path: layer-assignment tree (Sec. III-B), Elmore delay (Sec.
II-C, Fig. rc), pin and edge weights (Eq. 4, Eq. 5), congestion cost from
Eq. 3, the tree DP with look-ahead and its trace-back (Alg. 2-4, Sec. III-D),
the batch schedule with negotiation rounds, the objective J and a brute
force.  See oracle.c for every definition.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
import this package.  It shares no code with paper_2507_13375_amd.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("GAPLA_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_INVALID_ARG, ERR_BAD_TREE, ERR_RANGE, ERR_OOM = 0, -1, -2, -3, -4

# default integer cost weights (fixed-point units: see oracle.c)
W_CONG, W_CAP, W_D, W_VIA = 1000, 100, 1, 100000
HIST_INC = 64


class OracleError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("oracle error %d %s" % (code, what))
        self.code = code


def build(force: bool = False) -> str:
    """Compile oracle/oracle.c into oracle/liboracle.so (gcc -O2, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _OParams(ctypes.Structure):
    _fields_ = [("X", ctypes.c_int32), ("Y", ctypes.c_int32), ("L", ctypes.c_int32), ("min_layer", ctypes.c_int32),
                ("layer_dir", ctypes.c_void_p), ("r", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("vr", ctypes.c_void_p), ("w_cong", ctypes.c_int64), ("w_cap", ctypes.c_int64),
                ("w_d", ctypes.c_int64), ("w_via", ctypes.c_int64), ("seg_w", ctypes.c_void_p),
                ("pin_w", ctypes.c_void_p), ("lam", ctypes.c_void_p), ("lut", ctypes.c_void_p)]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        V, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.oracle_tree_build.argtypes = [I64] + [V] * 11 + [I32, I32, ctypes.POINTER(V), ctypes.POINTER(I64)]
        lib.oracle_tree_build.restype = ctypes.c_int
        lib.oracle_tree_free.argtypes = [V]
        lib.oracle_tree_sizes.argtypes = [V] + [ctypes.POINTER(I64)] * 3
        lib.oracle_tree_export.argtypes = [V] * 9
        lib.oracle_cong_lut.argtypes = [I32, V, V]
        lib.oracle_kappa.argtypes = [V, ctypes.POINTER(_OParams), I64, I32, V, V, V, I32]
        lib.oracle_kappa.restype = I64
        lib.oracle_assign.argtypes = [V, ctypes.POINTER(_OParams), V, V, V, V, ctypes.POINTER(I32), V, I32, I32,
                                      V, V, V, V]
        lib.oracle_assign.restype = ctypes.c_int
        lib.oracle_objective.argtypes = [V, ctypes.POINTER(_OParams), V, V, V, V, V, V]
        lib.oracle_objective.restype = ctypes.c_int
        lib.oracle_bruteforce.argtypes = [V, ctypes.POINTER(_OParams), I64, I32, V, V, V, V,
                                          ctypes.POINTER(I64), V, ctypes.POINTER(I64)]
        lib.oracle_bruteforce.restype = ctypes.c_int
        lib.oracle_rc.argtypes = [V, ctypes.POINTER(_OParams), V, V, V]
        lib.oracle_elmore.argtypes = [V] * 6
        lib.oracle_elmore_adjoint.argtypes = [V] * 9
        lib.oracle_slack.argtypes = [V, V, V, ctypes.POINTER(ctypes.c_double), V, V]
        lib.oracle_edge_weights.argtypes = [V, ctypes.POINTER(_OParams), V, V, V]
        lib.oracle_adjoint_weights.argtypes = [V] * 7
        lib.oracle_set_num_threads.argtypes = [I32]
        lib.oracle_get_batches.argtypes = [V, I32, I32, V, I32, V]
        lib.oracle_get_batches.restype = I64
        lib.oracle_sta.argtypes = [V, V, V, I32, V, V, V, ctypes.POINTER(ctypes.c_float)]
        lib.oracle_alg1_subsets.argtypes = [V, V, V, ctypes.c_float, V]
        lib.oracle_alg1_subsets.restype = I32
        lib.oracle_quality.argtypes = [V, I32, I32, I32] + [V] * 7 + [ctypes.POINTER(ctypes.c_double)] + \
            [ctypes.POINTER(I64)] * 4
        lib.oracle_quality.restype = None
        _lib = lib
    return _lib


class Tree:
    """Layer-assignment directed trees of an instance, canonical node order."""

    def __init__(self, inst):
        lib = _load()
        self.inst = inst
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        a = inst
        rc = lib.oracle_tree_build(a.num_nets, _p(a.net_node_ptr), _p(a.node_parent), _p(a.node_x), _p(a.node_y),
                                   _p(a.node_flags), _p(a.node_cpin_af), _p(a.edge_wp_ptr),
                                   _p(a.wp_x if a.wp_x.size else np.zeros(1, np.int16)),
                                   _p(a.wp_y if a.wp_y.size else np.zeros(1, np.int16)),
                                   _p(a.net_budget_fs), _p(a.net_rdrv_mohm), a.X, a.Y, ctypes.byref(h),
                                   ctypes.byref(bad))
        if rc != OK:
            raise OracleError(rc, "tree build (net %d)" % bad.value)
        self._h = h
        nn, no, ns = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib.oracle_tree_sizes(h, ctypes.byref(nn), ctypes.byref(no), ctypes.byref(ns))
        self.nets, self.nodes, self.sinks = nn.value, no.value, ns.value
        self.net_ptr = np.empty(self.nets + 1, np.int64)
        self.parent = np.empty(self.nodes, np.int64)
        self.x = np.empty(self.nodes, np.int32)
        self.y = np.empty(self.nodes, np.int32)
        self.len = np.empty(self.nodes, np.int32)
        self.dir = np.empty(self.nodes, np.int8)
        self.is_sink = np.empty(self.nodes, np.uint8)
        self.sink_node = np.empty(max(self.sinks, 1), np.int64)[:self.sinks]
        lib.oracle_tree_export(h, _p(self.net_ptr), _p(self.parent), _p(self.x), _p(self.y), _p(self.len),
                               _p(self.dir), _p(self.is_sink), _p(self.sink_node) if self.sinks else None)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.oracle_tree_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def num_edges(self) -> int:
        i = self.inst
        return i.X * i.Y * i.L


def cong_lut(L: int, ofw=None) -> np.ndarray:
    """Integer marginal congestion cost [L][2][64] from Eq. 3 (see oracle_cong_lut)."""
    lib = _load()
    ofw = np.ones(L, np.float64) if ofw is None else np.asarray(ofw, np.float64)
    out = np.empty((L, 2, 64), np.int32)
    lib.oracle_cong_lut(L, _p(ofw), _p(out))
    return out


class Params:
    """Technology, weights and the per-segment / per-sink integer DP inputs."""

    def __init__(self, tree: Tree, seg_w=None, pin_w=None, lam=None, w_cong=W_CONG, w_cap=W_CAP, w_d=W_D,
                 w_via=W_VIA, min_layer=0, lut=None):
        i = tree.inst
        self.tree = tree
        self.seg_w = np.ascontiguousarray(seg_w if seg_w is not None else np.full(tree.nodes, 1024, np.uint16),
                                          np.uint16)
        self.pin_w = np.ascontiguousarray(pin_w if pin_w is not None else np.full(max(tree.sinks, 1), 1024, np.uint16),
                                          np.uint16)
        if self.pin_w.size == 0:
            self.pin_w = np.zeros(1, np.uint16)
        self.lam = np.ascontiguousarray(lam if lam is not None else np.zeros(tree.nodes, np.int32), np.int32)
        self.lut = np.ascontiguousarray(lut if lut is not None else cong_lut(i.L), np.int32)
        self.layer_dir = np.ascontiguousarray(i.layer_dir, np.uint8)
        self.r = np.ascontiguousarray(i.r_mohm, np.int32)
        self.c = np.ascontiguousarray(i.c_af, np.int32)
        self.vr = np.ascontiguousarray(i.via_r_mohm, np.int32)
        self.s = _OParams(i.X, i.Y, i.L, min_layer, _p(self.layer_dir), _p(self.r), _p(self.c), _p(self.vr),
                          w_cong, w_cap, w_d, w_via, _p(self.seg_w), _p(self.pin_w), _p(self.lam), _p(self.lut))


class State:
    """Negotiation state: demand D, history H, previous layers."""

    def __init__(self, tree: Tree, H=None):
        i = tree.inst
        self.D = np.zeros(i.X * i.Y * i.L, np.int32)
        self.H = np.zeros(i.X * i.Y * i.L, np.int32) if H is None else np.array(H, np.int32).reshape(-1)
        self.prev = np.zeros(tree.nodes, np.uint8)
        self.has_prev = 0


def assign(tree: Tree, P: Params, state: State, net_tier=None, rounds: int = 1, hist_inc: int = HIST_INC):
    """Run `rounds` negotiation rounds of the batch schedule; returns (layers, via_lo, via_hi, F_root)."""
    lib = _load()
    caps = np.ascontiguousarray(tree.inst.caps).reshape(-1)
    lay = np.zeros(tree.nodes, np.uint8)
    vlo = np.zeros(tree.nodes, np.uint8)
    vhi = np.zeros(tree.nodes, np.uint8)
    froot = np.zeros(tree.nets, np.int64)
    hp = ctypes.c_int32(state.has_prev)
    tier = None if net_tier is None else np.ascontiguousarray(net_tier, np.int32)
    rc = lib.oracle_assign(tree.handle, ctypes.byref(P.s), _p(caps), _p(state.D), _p(state.H), _p(state.prev),
                           ctypes.byref(hp), _p(tier), rounds, hist_inc, _p(lay), _p(vlo), _p(vhi), _p(froot))
    if rc != OK:
        raise OracleError(rc, "assign")
    state.has_prev = hp.value
    return lay, vlo, vhi, froot


def objective(tree: Tree, P: Params, layers, D, H=None, prev=None) -> np.ndarray:
    """J of every net under `layers` against demand D (self-exclusion when prev is given)."""
    lib = _load()
    caps = np.ascontiguousarray(tree.inst.caps).reshape(-1)
    H = np.zeros_like(D) if H is None else H
    out = np.zeros(tree.nets, np.int64)
    rc = lib.oracle_objective(tree.handle, ctypes.byref(P.s), _p(np.ascontiguousarray(layers, np.uint8)),
                              _p(np.ascontiguousarray(D, np.int32)), _p(caps), _p(np.ascontiguousarray(H, np.int32)),
                              _p(None if prev is None else np.ascontiguousarray(prev, np.uint8)), _p(out))
    if rc != OK:
        raise OracleError(rc, "objective")
    return out


def bruteforce(tree: Tree, P: Params, net: int, D, H=None, prev=None, max_segs: int = 6):
    """(J_min, one minimiser as net-local layers, number of minimisers)."""
    lib = _load()
    caps = np.ascontiguousarray(tree.inst.caps).reshape(-1)
    H = np.zeros_like(D) if H is None else H
    n = int(tree.net_ptr[net + 1] - tree.net_ptr[net])
    best = np.zeros(max(n, 1), np.uint8)
    jmin, nmin = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.oracle_bruteforce(tree.handle, ctypes.byref(P.s), net, max_segs, _p(np.ascontiguousarray(D, np.int32)),
                               _p(caps), _p(np.ascontiguousarray(H, np.int32)),
                               _p(None if prev is None else np.ascontiguousarray(prev, np.uint8)),
                               ctypes.byref(jmin), _p(best), ctypes.byref(nmin))
    if rc != OK:
        raise OracleError(rc, "bruteforce")
    return jmin.value, best[:n], nmin.value


def kappa(tree: Tree, P: Params, node: int, layer: int, D, H=None, self_layer: int = -1) -> int:
    lib = _load()
    caps = np.ascontiguousarray(tree.inst.caps).reshape(-1)
    H = np.zeros_like(D) if H is None else H
    return lib.oracle_kappa(tree.handle, ctypes.byref(P.s), node, layer, _p(np.ascontiguousarray(D, np.int32)),
                            _p(caps), _p(np.ascontiguousarray(H, np.int32)), self_layer)


def quality(tree: Tree, layers, vlo, vhi, D, ofw=None) -> dict:
    """Quality terms of an assignment (Sec. II): Eq. 3 total overflow (FP64), Eq. 2 total
    overflow and overflowed edges, via count, wire capacitance in aF."""
    lib = _load()
    inst = tree.inst
    caps = np.ascontiguousarray(inst.caps, np.uint8).reshape(-1)
    c_af = np.ascontiguousarray(inst.c_af, np.int32)
    tof = ctypes.c_double()
    o2, n2, nv, wc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lib.oracle_quality(tree.handle, inst.X, inst.Y, inst.L, _p(c_af), _p(np.ascontiguousarray(layers, np.uint8)),
                       _p(np.ascontiguousarray(vlo, np.uint8)), _p(np.ascontiguousarray(vhi, np.uint8)),
                       _p(np.ascontiguousarray(D, np.int32).reshape(-1)), _p(caps),
                       _p(None if ofw is None else np.ascontiguousarray(ofw, np.float64)), ctypes.byref(tof),
                       ctypes.byref(o2), ctypes.byref(n2), ctypes.byref(nv), ctypes.byref(wc))
    return {"tof": tof.value, "overflow_sum": o2.value, "overflow_edges": n2.value, "vias": nv.value,
            "wire_cap_af": wc.value}


def get_batches(tree: Tree, X: int, Y: int, subset, nsub: int):
    """Classical batching (Alg. 1, GetBatch): per subset, in net order, a net joins the lowest
    batch whose nets' boxes share no GCell with its own.  Returns (batch per net, count)."""
    sub = np.ascontiguousarray(subset, np.int32)
    out = np.empty(max(tree.nets, 1), np.int32)
    n = int(_load().oracle_get_batches(tree.handle, int(X), int(Y), _p(sub), int(nsub), _p(out)))
    if n < 0:
        raise MemoryError("oracle_get_batches")
    return out[:tree.nets], n


def sta(tree: Tree, sink_next, gate_delay_fs, clock_fs: int, delay):
    """Static timing of the gate graph over the nets (Alg. 1, its first step) in single precision, and
    the critical-path counts that follow it.  delay: per-sink Elmore delay (ps, float32).  Returns
    (slack per sink, critical paths per net, WNS)."""
    sl = np.empty(max(tree.sinks, 1), np.float32)
    cr = np.empty(max(tree.nets, 1), np.int32)
    w = ctypes.c_float()
    rc = _load().oracle_sta(tree.handle, _p(np.ascontiguousarray(sink_next, np.int32)),
                            _p(np.ascontiguousarray(gate_delay_fs, np.int32)), int(clock_fs),
                            _p(np.ascontiguousarray(delay, np.float32)), _p(sl), _p(cr), ctypes.byref(w))
    if rc != OK:
        raise OracleError(rc, "sta")
    return sl[:tree.sinks], cr[:tree.nets], w.value


def alg1_subsets(tree: Tree, slack, crit, wns: float):
    """Alg. 1 division and partition: the ordered subsets (critical by path count, semi-critical by slack,
    then the rest).  Returns (subset per net, number of subsets)."""
    out = np.empty(max(tree.nets, 1), np.int32)
    n = _load().oracle_alg1_subsets(tree.handle, _p(np.ascontiguousarray(slack, np.float32)),
                                    _p(np.ascontiguousarray(crit, np.int32)), ctypes.c_float(wns), _p(out))
    return out[:tree.nets], int(n)


def num_threads() -> int:
    """Threads the oracle's OpenMP loops run on."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only; results do not change)."""
    _load().oracle_set_num_threads(int(n))


def rc(tree: Tree, P: Params, layers=None):
    """R (kOhm) and C (fF) of every RC edge [nodes + sinks]; layers=None gives the pre-assignment RC."""
    lib = _load()
    R = np.empty(tree.nodes + tree.sinks, np.float64)
    C = np.empty(tree.nodes + tree.sinks, np.float64)
    lib.oracle_rc(tree.handle, ctypes.byref(P.s), _p(None if layers is None else np.ascontiguousarray(layers, np.uint8)),
                  _p(R), _p(C))
    return R, C


def elmore(tree: Tree, R, C):
    """(S, t, delay): downstream C and delay per node, delay per sink (ps)."""
    lib = _load()
    S = np.empty(tree.nodes, np.float64)
    t = np.empty(tree.nodes, np.float64)
    d = np.empty(max(tree.sinks, 1), np.float64)
    lib.oracle_elmore(tree.handle, _p(np.ascontiguousarray(R, np.float64)), _p(np.ascontiguousarray(C, np.float64)),
                      _p(S), _p(t), _p(d))
    return S, t, d[:tree.sinks]


def elmore_adjoint(tree: Tree, R, C, S, gbar):
    """(G, Sig, dR, dC) for upstream gradient gbar = dJ/d delay per sink."""
    lib = _load()
    G = np.empty(tree.nodes, np.float64)
    Sig = np.empty(tree.nodes, np.float64)
    dR = np.empty(tree.nodes + tree.sinks, np.float64)
    dC = np.empty(tree.nodes + tree.sinks, np.float64)
    lib.oracle_elmore_adjoint(tree.handle, _p(np.ascontiguousarray(R, np.float64)),
                              _p(np.ascontiguousarray(C, np.float64)), _p(np.ascontiguousarray(S, np.float64)),
                              _p(np.ascontiguousarray(gbar, np.float64)), _p(G), _p(Sig), _p(dR), _p(dC))
    return G, Sig, dR, dC


def slack(tree: Tree, delay):
    """(slack per sink, WNS, Q10 pin weights (Eq. 4), batch per net)."""
    lib = _load()
    s = np.empty(max(tree.sinks, 1), np.float64)
    w = np.empty(max(tree.sinks, 1), np.uint16)
    tier = np.empty(tree.nets, np.uint8)
    wns = ctypes.c_double()
    lib.oracle_slack(tree.handle, _p(np.ascontiguousarray(delay, np.float64)), _p(s), ctypes.byref(wns), _p(w),
                     _p(tier))
    return s[:tree.sinks], wns.value, w[:tree.sinks], tier


def edge_weights(tree: Tree, P: Params, pin_w):
    """(seg_w Q10 per node (Eq. 5), lambda per node (look-ahead coefficient))."""
    lib = _load()
    sw = np.zeros(tree.nodes, np.uint16)
    lam = np.zeros(tree.nodes, np.int32)
    pw = np.ascontiguousarray(pin_w, np.uint16)
    lib.oracle_edge_weights(tree.handle, ctypes.byref(P.s), _p(pw if pw.size else np.zeros(1, np.uint16)), _p(sw),
                            _p(lam))
    return sw, lam


def adjoint_weights(tree: Tree, G, Sig, gbar):
    """(seg_w, pin_w, lambda) from the adjoint sums G and Sig."""
    lib = _load()
    sw = np.zeros(tree.nodes, np.uint16)
    pw = np.zeros(max(tree.sinks, 1), np.uint16)
    lam = np.zeros(tree.nodes, np.int32)
    lib.oracle_adjoint_weights(tree.handle, _p(np.ascontiguousarray(G, np.float64)),
                               _p(np.ascontiguousarray(Sig, np.float64)),
                               _p(np.ascontiguousarray(gbar, np.float64) if len(gbar) else np.zeros(1)), _p(sw),
                               _p(pw), _p(lam))
    return sw, pw[:tree.sinks], lam


def plain_weights(tree: Tree, P: Params, layers=None):
    """Timing weights of the plain form: Elmore on the current RC, slack, Eq. 4 pin weights,
    Eq. 5 edge weights, look-ahead coefficients and batches."""
    R, C = rc(tree, P, layers)
    S, t, d = elmore(tree, R, C)
    sl, wns, pw, tier = slack(tree, d)
    sw, lam = edge_weights(tree, P, pw)
    return dict(seg_w=sw, pin_w=pw, lam=lam, tier=tier, delay=d, slack=sl, wns=wns)


def adjoint_form_weights(tree: Tree, P: Params, layers=None):
    """Timing weights of the differentiation form: Elmore, slack, omega = Eq. 4 weight of each
    violating sink, gbar = dJ/d delay of J = sum omega min(0, slack), reverse sweep, then
    seg_w = -G, pin_w = -gbar, lambda = -Sig(parent) (quantised)."""
    R, C = rc(tree, P, layers)
    S, t, d = elmore(tree, R, C)
    sl, wns, pw, tier = slack(tree, d)
    gbar = -(pw.astype(np.float64) / 1024.0) * (sl < 0)
    G, Sig, dR, dC = elmore_adjoint(tree, R, C, S, gbar)
    sw, pw2, lam = adjoint_weights(tree, G, Sig, gbar)
    return dict(seg_w=sw, pin_w=pw2, lam=lam, tier=tier, delay=d, slack=sl, wns=wns, dR=dR, dC=dC, G=G, Sig=Sig)
