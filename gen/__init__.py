"""Seeded synthetic layer-assignment instances (inputs only; no method arithmetic).

The five workload presets stand in for the ISPD 2025 designs the paper
evaluates on (Table "Benchmark details"): grids of GCells with 8-12
alternating H/V layers, per-(edge, layer) integer capacities, per-layer unit
R/C and via R that fall geometrically on upper layer pairs (the shape of the
paper's modified Nangate45 table), and one 2D rectilinear Steiner tree per
net (an L-embedded rectilinear MST over distinct pins; pin 0 drives).

    c1  1,000 nets      64x64 x 8   pins U{2..8}, uniform placement, cap U{4..12}
    c2  200,000 nets    512^2 x 10  heavy-tailed pins (<=64), 16 hotspots sigma 40, cap U{6..16}
    c3  2,000,000 nets  1024^2 x 12 heavy-tailed pins (<=256), net-local sigma 3*sqrt(p), cap U{6..16}
    c4  the c3 instance (used with the adjoint-weighted schedule)
    c5  12,000,000 nets 2048^2 x 12 heavy-tailed pins (<=256) + 120 nets of U{1000..4000} pins,
        centres 75% near 16 hotspots (sigma 80) / 25% uniform, cap U{6..16}

Randomness is splitmix64 with seed 2507133750 + config number.  The library
that the oracle and the HIP path both consume is ``gen/libgen.so`` (C).
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None

SEED_BASE = 2507133750


class _Params(ctypes.Structure):
    _fields_ = [
        ("num_nets", ctypes.c_int64), ("X", ctypes.c_int32), ("Y", ctypes.c_int32), ("L", ctypes.c_int32),
        ("pin_law", ctypes.c_int32), ("pin_min", ctypes.c_int32), ("pin_max", ctypes.c_int32),
        ("placement", ctypes.c_int32), ("n_hot", ctypes.c_int32), ("hot_sigma", ctypes.c_double),
        ("hot_frac", ctypes.c_double), ("cap_min", ctypes.c_int32), ("cap_max", ctypes.c_int32),
        ("fanout_every", ctypes.c_int64), ("fanout_min", ctypes.c_int32), ("fanout_max", ctypes.c_int32),
        ("budget_min_fs", ctypes.c_int32), ("budget_max_fs", ctypes.c_int32),
        ("cpin_af", ctypes.c_int32), ("rdrv_mohm", ctypes.c_int32),
        ("r0_mohm", ctypes.c_double), ("c0_af", ctypes.c_double), ("via0_mohm", ctypes.c_double),
        ("rc_decay", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


def build(force: bool = False) -> str:
    """Compile gen/gen.c into gen/libgen.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gen_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        lib.gen_create.restype = ctypes.c_int
        lib.gen_free.argtypes = [ctypes.c_void_p]
        lib.gen_sizes.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3
        lib.gen_export.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 16
        lib.gen_counter_u64.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
        lib.gen_timing_graph.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Instance:
    """One layer-assignment input: grid, layer RC table and the 2D trees of all nets."""
    name: str
    X: int
    Y: int
    L: int
    net_node_ptr: np.ndarray   # int32 [nets+1]; node 0 of each net is its driver pin
    node_parent: np.ndarray    # int32 [nodes] net-local parent, -1 for the driver
    node_x: np.ndarray         # int16
    node_y: np.ndarray         # int16
    node_flags: np.ndarray     # uint8 bit0 sink pin, bit1 driver pin
    node_cpin_af: np.ndarray   # int32 sink load (aF)
    edge_wp_ptr: np.ndarray    # int32 [nodes+1] bend waypoints of edge parent->node
    wp_x: np.ndarray           # int16
    wp_y: np.ndarray           # int16
    net_budget_fs: np.ndarray  # int32 required-time budget per net (fs)
    net_rdrv_mohm: np.ndarray  # int32 driver resistance (mOhm)
    caps: np.ndarray           # uint8 [Y][X][L]
    r_mohm: np.ndarray         # int32 [L]   unit wire R per GCell
    c_af: np.ndarray           # int32 [L]   unit wire C per GCell
    via_r_mohm: np.ndarray     # int32 [L-1] via from layer k to k+1
    layer_dir: np.ndarray      # uint8 [L]   0 = H, 1 = V
    params: dict = field(default_factory=dict)

    @property
    def num_nets(self) -> int:
        return int(self.net_node_ptr.shape[0] - 1)

    @property
    def num_nodes(self) -> int:
        return int(self.node_parent.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.net_node_ptr, self.node_parent, self.node_x, self.node_y, self.node_flags,
                  self.node_cpin_af, self.edge_wp_ptr, self.wp_x, self.wp_y, self.net_budget_fs,
                  self.net_rdrv_mohm, self.caps, self.r_mohm, self.c_af, self.via_r_mohm, self.layer_dir):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


_DEFAULTS = dict(pin_law=0, pin_min=2, pin_max=8, placement=0, n_hot=16, hot_sigma=40.0, hot_frac=0.0,
                 cap_min=4, cap_max=12, fanout_every=0, fanout_min=1000, fanout_max=4000,
                 budget_min_fs=-50000, budget_max_fs=200000, cpin_af=1000, rdrv_mohm=1000000,
                 r0_mohm=20000.0, c0_af=200.0, via0_mohm=5000.0, rc_decay=0.7)

CONFIGS = {
    1: dict(num_nets=1000, X=64, Y=64, L=8, pin_law=0, pin_min=2, pin_max=8, placement=0, cap_min=4, cap_max=12),
    2: dict(num_nets=200000, X=512, Y=512, L=10, pin_law=1, pin_max=64, placement=1, n_hot=16, hot_sigma=40.0,
            cap_min=6, cap_max=16),
    3: dict(num_nets=2000000, X=1024, Y=1024, L=12, pin_law=1, pin_max=256, placement=2, cap_min=6, cap_max=16),
    5: dict(num_nets=12000000, X=2048, Y=2048, L=12, pin_law=1, pin_max=256, placement=3, n_hot=16,
            hot_sigma=80.0, hot_frac=0.75, cap_min=6, cap_max=16, fanout_every=99999, fanout_min=1000,
            fanout_max=4000),
}
CONFIGS[4] = dict(CONFIGS[3])
CONFIG_SEED = {1: SEED_BASE + 1, 2: SEED_BASE + 2, 3: SEED_BASE + 3, 4: SEED_BASE + 3, 5: SEED_BASE + 5}


def generate(num_nets: int, X: int, Y: int, L: int, seed: int, name: str = "custom", **kw) -> Instance:
    """Generate an instance from explicit parameters (see _DEFAULTS for the rest)."""
    lib = _load()
    p = dict(_DEFAULTS)
    p.update(kw)
    p.update(num_nets=num_nets, X=X, Y=Y, L=L, seed=seed)
    cp = _Params(**p)
    h = ctypes.c_void_p()
    rc = lib.gen_create(ctypes.byref(cp), ctypes.byref(h))
    if rc != 0:
        raise ValueError("gen_create failed with code %d for %s" % (rc, p))
    try:
        nn, no, nw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib.gen_sizes(h, ctypes.byref(nn), ctypes.byref(no), ctypes.byref(nw))
        N, n, w = nn.value, no.value, nw.value
        a = dict(
            net_node_ptr=np.empty(N + 1, np.int32), node_parent=np.empty(n, np.int32),
            node_x=np.empty(n, np.int16), node_y=np.empty(n, np.int16), node_flags=np.empty(n, np.uint8),
            node_cpin_af=np.empty(n, np.int32), edge_wp_ptr=np.empty(n + 1, np.int32),
            wp_x=np.empty(max(w, 1), np.int16), wp_y=np.empty(max(w, 1), np.int16),
            net_budget_fs=np.empty(N, np.int32), net_rdrv_mohm=np.empty(N, np.int32),
            caps=np.empty((Y, X, L), np.uint8), r_mohm=np.empty(L, np.int32), c_af=np.empty(L, np.int32),
            via_r_mohm=np.empty(L - 1, np.int32), layer_dir=np.empty(L, np.uint8))
        order = ["net_node_ptr", "node_parent", "node_x", "node_y", "node_flags", "node_cpin_af", "edge_wp_ptr",
                 "wp_x", "wp_y", "net_budget_fs", "net_rdrv_mohm", "caps", "r_mohm", "c_af", "via_r_mohm",
                 "layer_dir"]
        lib.gen_export(h, *[a[k].ctypes.data_as(ctypes.c_void_p) for k in order])
        a["wp_x"] = a["wp_x"][:w]
        a["wp_y"] = a["wp_y"][:w]
    finally:
        lib.gen_free(h)
    return Instance(name=name, X=X, Y=Y, L=L, params=p, **a)


def config(c: int, num_nets: int | None = None) -> Instance:
    """Instance of workload preset `c` (1..5); `num_nets` truncates it to a smaller net count."""
    p = dict(CONFIGS[c])
    if num_nets is not None:
        p["num_nets"] = num_nets
    n = p.pop("num_nets")
    X, Y, L = p.pop("X"), p.pop("Y"), p.pop("L")
    return generate(n, X, Y, L, CONFIG_SEED[c], name="c%d" % c, **p)


def timing_graph(inst: Instance, levels: int = 24, po_frac: float = 0.2, dmin_fs: int = 8000, dmax_fs: int = 25000,
                 seed: int = 2507133750 + 100, clock_fs: int = 1000000) -> dict:
    """Synthetic gate-level timing graph over the nets of `inst` (for Alg. 1's critical-path
    ordering): per net a logic level and the delay of its driving gate (fs); per sink (node
    order) the net whose gate it feeds, or -1 for a primary output; the clock period (required
    time at every primary output).  1 ns leaves about a quarter of the outputs violating on the
    2M-net workload before assignment."""
    lib = _load()
    nptr = np.ascontiguousarray(inst.net_node_ptr, np.int32)
    flags = np.ascontiguousarray(inst.node_flags, np.uint8)
    n = int(inst.num_nets)
    sinks = int(np.count_nonzero(flags & 1))
    lvl = np.empty(max(n, 1), np.int32)
    nxt = np.empty(max(sinks, 1), np.int32)
    gd = np.empty(max(n, 1), np.int32)
    sd = seed
    rc = lib.gen_timing_graph(n, nptr.ctypes.data_as(ctypes.c_void_p), flags.ctypes.data_as(ctypes.c_void_p),
                              int(levels), float(po_frac), int(dmin_fs), int(dmax_fs), ctypes.c_uint64(sd & (2**64 - 1)),
                              lvl.ctypes.data_as(ctypes.c_void_p), nxt.ctypes.data_as(ctypes.c_void_p),
                              gd.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("gen_timing_graph failed (%d)" % rc)
    return dict(net_level=lvl[:n], sink_next=nxt[:sinks], gate_delay_fs=gd[:n], levels=levels, clock_fs=int(clock_fs))


def counter_u64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Counter-based splitmix64 outputs start..start+n-1 of the sequence seeded with `seed`."""
    lib = _load()
    out = np.empty(n, np.uint64)
    if n:
        lib.gen_counter_u64(ctypes.c_uint64(seed & (2**64 - 1)), start, n, out.ctypes.data_as(ctypes.c_void_p))
    return out


def synthetic_weights(num_nodes: int, num_sinks: int, num_nets: int, seed: int, n_tiers: int = 11,
                      lambda_max: int = 2000000, w_max: int = 1024) -> dict:
    """Seeded integer DP inputs of the right shapes (segment / pin weights, look-ahead
    coefficients and tiers), used where a test needs identical integer inputs on both sides."""
    r = counter_u64(seed, 3 * num_nodes + num_sinks + num_nets)
    seg_w = (r[:num_nodes] % np.uint64(w_max + 1)).astype(np.uint16)
    lam = (r[num_nodes:2 * num_nodes] % np.uint64(lambda_max + 1)).astype(np.int32)
    pin_w = (r[3 * num_nodes:3 * num_nodes + num_sinks] % np.uint64(w_max + 1)).astype(np.uint16)
    tier = (r[3 * num_nodes + num_sinks:] % np.uint64(max(n_tiers, 1))).astype(np.uint8)
    return dict(seg_w_q10=seg_w, lambda_mohm=lam, pin_w_q10=pin_w, net_tier=tier)
