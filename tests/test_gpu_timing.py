"""GPU parity of the timing path against the FP64 oracle: RC edges, Elmore delay, reverse
sweep, torch autograd wrapper, TNS/WNS and the DP timing weights (Eq. 4, Eq. 5, adjoint)."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, dev, host, say, tier_flips_at_bin_edges, torch
from helpers import make_instance

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def c1():
    return gen.config(1)


def _rel_close(gpu, ref, rel=REL, what=""):
    gpu = np.asarray(gpu, np.float64)
    err = np.abs(gpu - ref)
    bad = np.nonzero(err > rel * np.abs(ref) + 1e-30)[0]
    assert bad.size == 0, "%s: %d of %d outside %.0e, worst %g at %d (gpu %r ref %r)" % (
        what, bad.size, ref.size, rel, (err / np.maximum(np.abs(ref), 1e-30)).max(), bad[0], gpu[bad[0]], ref[bad[0]])


@pytest.mark.parametrize("cfg,n", [(1, None), (2, 20000)])
def test_elmore_before_assignment(cfg, n):
    inst = gen.config(cfg, num_nets=n)
    say("elmore pre-LA c%d nets=%d" % (cfg, inst.num_nets))
    g = DeviceRun(inst)
    T = oracle.Tree(inst)
    P = oracle.Params(T)
    R, C = oracle.rc(T, P, None)
    Rg, Cg = g.rc()
    _rel_close(host(Rg), R, 1e-7, "R")
    _rel_close(host(Cg), C, 1e-7, "C")
    S, t, d = oracle.elmore(T, R, C)
    _rel_close(host(g.elmore())[:T.sinks], d, REL, "delay")


def _oracle_weights(inst):
    T = oracle.Tree(inst)
    w = oracle.plain_weights(T, oracle.Params(T))
    return T, w


def test_elmore_after_assignment_and_summary(c1):
    T, w = _oracle_weights(c1)
    o = oracle.Params(T, seg_w=w["seg_w"], pin_w=w["pin_w"], lam=w["lam"])
    st = oracle.State(T)
    lay, _, _, _ = oracle.assign(T, o, st, w["tier"], rounds=2)
    g = DeviceRun(c1)
    g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=2)
    R, C = oracle.rc(T, o, lay)
    Rg, Cg = g.rc()
    _rel_close(host(Rg), R, 1e-7, "R")
    _rel_close(host(Cg), C, 1e-7, "C")
    S, t, d = oracle.elmore(T, R, C)
    dg = g.elmore()
    _rel_close(host(dg)[:T.sinks], d, REL, "delay")
    tns, wns = la.la_timing_summary(g.b, dg)
    sl = c1.net_budget_fs[np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1] * 1e-3 - d
    assert tns == pytest.approx(sl[sl < 0].sum(), rel=REL)
    assert wns == pytest.approx(sl.min(), rel=REL, abs=1e-3)


def _adjoint_tol(gpu, ref, net_of):
    # relative to max(|g|, 1e-3 * largest |g| of the same net)
    scale = np.abs(ref)
    mx = np.zeros(net_of.max() + 1)
    np.maximum.at(mx, net_of, np.abs(ref))
    floor = 1e-3 * mx[net_of]
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    return err <= REL * np.maximum(scale, floor) + 1e-30


@pytest.mark.parametrize("signs", ["tns", "mixed"])
def test_elmore_backward_matches_oracle_adjoint(c1, signs):
    inst = c1
    T = oracle.Tree(inst)
    P = oracle.Params(T)
    R, C = oracle.rc(T, P, None)
    S, t, d = oracle.elmore(T, R, C)
    rng = np.random.default_rng(7)
    # the same FP32 values go to both sides
    if signs == "tns":
        # dJ/dslack of a weighted TNS: w >= 0 on violating sinks, 0 elsewhere
        dslack = (rng.uniform(0, 1, T.sinks) * (rng.uniform(0, 1, T.sinks) < 0.6)).astype(np.float32)
    else:
        dslack = rng.uniform(-1, 1, T.sinks).astype(np.float32)
    gbar = -dslack.astype(np.float64)
    G, Sig, dR, dC = oracle.elmore_adjoint(T, R, C, S, gbar)
    # the same sweep on |g| bounds every partial sum, hence the rounding of mixed-sign sums
    _, _, dRa, dCa = oracle.elmore_adjoint(T, R, C, S, np.abs(gbar))
    g = DeviceRun(inst)
    g.elmore()
    t_ = torch()
    dRg = t_.empty(T.nodes + T.sinks, dtype=t_.float32, device="cuda")
    dCg = t_.empty_like(dRg)
    la.la_elmore_backward(g.b, dev(dslack), dRg, dCg)
    node_net = np.searchsorted(T.net_ptr, np.arange(T.nodes), side="right") - 1
    sink_net = node_net[T.sink_node]
    net_of = np.concatenate([node_net, sink_net])
    for name, gpu, ref, refabs in (("dR", host(dRg), dR, dRa), ("dC", host(dCg), dC, dCa)):
        if signs == "tns":
            ok = _adjoint_tol(gpu, ref, net_of)
        else:
            ok = np.abs(gpu.astype(np.float64) - ref) <= REL * np.abs(refabs) + 1e-30
        assert ok.all(), "%s: %d bad, first %d gpu %r ref %r" % (name, (~ok).sum(), np.nonzero(~ok)[0][0],
                                                               gpu[~ok][0], ref[~ok][0])


def test_backward_before_forward_is_state_error(c1):
    g = DeviceRun(c1)
    t_ = torch()
    z = t_.zeros(g.b.sinks, dtype=t_.float32, device="cuda")
    with pytest.raises(la.LAError) as e:
        la.la_elmore_backward(g.b, z, None, None)
    assert e.value.code == la.LA_ERR_STATE


def test_autograd_function(c1):
    t_ = torch()
    g = DeviceRun(c1)
    R0, C0 = g.rc()
    R = R0.clone().requires_grad_(True)
    C = C0.clone().requires_grad_(True)
    d = la.elmore(R, C, g.b)
    wts = t_.linspace(0.05, 1, d.numel(), device="cuda")
    (d * wts).sum().backward()
    T = oracle.Tree(c1)
    Rr, Cr = oracle.rc(T, oracle.Params(T), None)
    S, _, _ = oracle.elmore(T, Rr, Cr)
    _, _, dR, dC = oracle.elmore_adjoint(T, Rr, Cr, S, host(wts).astype(np.float64))
    node_net = np.searchsorted(T.net_ptr, np.arange(T.nodes), side="right") - 1
    net_of = np.concatenate([node_net, node_net[T.sink_node]])
    assert _adjoint_tol(host(R.grad), dR, net_of).all()
    assert _adjoint_tol(host(C.grad), dC, net_of).all()


@pytest.mark.parametrize("cfg,n", [(1, None), (2, 40000)])
def test_plain_weights(cfg, n):
    inst = gen.config(cfg, num_nets=n)
    say("plain weights c%d" % cfg)
    T, w = _oracle_weights(inst)
    g = DeviceRun(inst)
    t_ = torch()
    d = g.elmore()
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(max(T.sinks, 1), dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    la.la_timing_weights(g.b, d, la.LA_WEIGHTS_PLAIN, sw, pw, lam, tier)
    pwg, swg, lg, tg = host(pw)[:T.sinks].astype(np.int64), host(sw).astype(np.int64), host(lam), host(tier)
    assert np.abs(pwg - w["pin_w"]).max() <= 1
    assert np.abs(swg - w["seg_w"]).max() <= 1
    same = swg == w["seg_w"]
    assert (lg[same] == w["lam"][same]).all()
    sl = w["slack"]
    ns = np.full(T.nets, np.inf)
    sink_net = np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1
    np.minimum.at(ns, sink_net, sl)
    flips = tier_flips_at_bin_edges(tg, w["tier"], ns / w["wns"])
    say("pin weight LSB diffs %d, tier flips %d" % (int((pwg != w["pin_w"]).sum()), flips))


def test_adjoint_weights(c1):
    T = oracle.Tree(c1)
    w = oracle.adjoint_form_weights(T, oracle.Params(T), None)
    g = DeviceRun(c1)
    t_ = torch()
    d = g.elmore()
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(max(T.sinks, 1), dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    la.la_timing_weights(g.b, d, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
    swg, pwg, lg = host(sw).astype(np.int64), host(pw)[:T.sinks].astype(np.int64), host(lam).astype(np.int64)
    assert np.abs(pwg - w["pin_w"]).max() <= 1
    assert np.abs(swg - w["seg_w"]).max() <= 1
    assert (np.abs(lg - w["lam"]) <= 1 + 1e-5 * np.abs(w["lam"])).all()


def _net_of(T):
    node_net = np.searchsorted(T.net_ptr, np.arange(T.nodes), side="right") - 1
    return np.concatenate([node_net, node_net[T.sink_node]])


def _heights(T):
    h = np.zeros(T.nodes, np.int64)
    changed = True
    par = T.parent
    while changed:                               # relax: h(parent) >= h(child) + 1
        nonroot = par >= 0
        cand = np.zeros(T.nodes, np.int64)
        np.maximum.at(cand, par[nonroot], h[nonroot] + 1)
        changed = bool((cand > h).any())
        h = np.maximum(h, cand)
    return h


@pytest.mark.parametrize("kind", ["untiled", "tiles"])
def test_large_nets_elmore_adjoint_and_eq5(kind):
    # Nets of at most 128 layer-assignment nodes take the one-wavefront runs; nets of up to 1024
    # nodes and height below 128 the workgroup tiles; the others (more than 1024 nodes or height
    # 128 or more) the per-level kernels (one launch per dense level, one workgroup over the sparse
    # top levels).  Each instance mixes wavefront-run nets with nets of one of the other two
    # classes.  Forward, reverse sweep and Eq. 5 weights against the FP64 oracle.
    fan = dict(untiled=dict(fanout_every=40, fanout_min=1000, fanout_max=1600),
               tiles=dict(fanout_every=12, fanout_min=120, fanout_max=400))[kind]
    inst = gen.generate(240, 256, 256, 10, 23, pin_law=1, pin_max=16, placement=2, cap_min=4, cap_max=10,
                        budget_min_fs=-400000, budget_max_fs=-100000, **fan)
    T = oracle.Tree(inst)
    sizes = np.diff(T.net_ptr)
    h = _heights(T)
    net_h = np.zeros(T.nets, np.int64)
    np.maximum.at(net_h, np.searchsorted(T.net_ptr, np.arange(T.nodes), side="right") - 1, h)
    untiled = (sizes > 1024) | (net_h >= 128)
    tiled = ~untiled & (sizes > 128)
    say("%s: %d untiled, %d tile, %d wavefront-run nets (largest %d nodes, tallest %d levels)" % (
        kind, untiled.sum(), tiled.sum(), T.nets - untiled.sum() - tiled.sum(), sizes.max(), net_h.max() + 1))
    assert (untiled if kind == "untiled" else tiled).sum() >= 3 and (sizes <= 128).sum() >= 100
    P = oracle.Params(T)
    R, C = oracle.rc(T, P, None)
    S, t, d = oracle.elmore(T, R, C)
    g = DeviceRun(inst)
    dg = g.elmore()
    _rel_close(host(dg)[:T.sinks], d, REL, "delay")
    # reverse sweep for a weighted TNS
    rng = np.random.default_rng(29)
    dslack = rng.uniform(0, 1, T.sinks).astype(np.float32)
    G, Sig, dR, dC = oracle.elmore_adjoint(T, R, C, S, -dslack.astype(np.float64))
    t_ = torch()
    dRg = t_.empty(T.nodes + T.sinks, dtype=t_.float32, device="cuda")
    dCg = t_.empty_like(dRg)
    la.la_elmore_backward(g.b, dev(dslack), dRg, dCg)
    net_of = _net_of(T)
    for name, gpu, ref in (("dR", host(dRg), dR), ("dC", host(dCg), dC)):
        ok = _adjoint_tol(gpu, ref, net_of)
        assert ok.all(), "%s: %d bad (%d in untiled nets, %d in tile nets)" % (
            name, (~ok).sum(), (~ok & untiled[net_of]).sum(), (~ok & tiled[net_of]).sum())
    # plain weights: Eq. 5 over the untiled nets' levels
    w = oracle.plain_weights(T, P)
    d2 = g.elmore()
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(max(T.sinks, 1), dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    la.la_timing_weights(g.b, d2, la.LA_WEIGHTS_PLAIN, sw, pw, lam, tier)
    swg, pwg, lg = host(sw).astype(np.int64), host(pw)[:T.sinks].astype(np.int64), host(lam)
    assert np.abs(pwg - w["pin_w"]).max() <= 1
    assert np.abs(swg - w["seg_w"]).max() <= 1
    same = swg == w["seg_w"]
    assert (lg[same] == w["lam"][same]).all()
    # where the pin weights agree over a whole net, Eq. 5 (an integer max) must agree exactly
    sink_net = net_of[T.nodes:]
    bad_net = np.zeros(T.nets, bool)
    bad_net[sink_net[pwg != w["pin_w"]]] = True
    exact = ~bad_net[net_of[:T.nodes]]
    assert (swg[exact] == w["seg_w"][exact]).all() and (lg[exact] == w["lam"][exact]).all()
    say("%s Eq. 5: %d of %d nodes in nets with identical pin weights" % (kind, exact.sum(), T.nodes))


def test_wavefront_run_limits():
    # chains of 128 nodes (heights 0-127: one full run, both lane slots), 65 and 64 nodes and two
    # small nets: runs of 128, 65 and 69 nodes, at the largest height a run holds and at the
    # boundary of its two lane slots; forward, reverse sweep and adjoint-form weights
    nets = []
    for i, n in enumerate((128, 65, 64, 2, 3)):
        nodes = [(0, 2 * i, -1, "driver")] + [(k, 2 * i, k - 1, "sink") for k in range(1, n)]
        nets.append((nodes, None))
    inst = make_instance(nets, X=160, Y=16, L=8, budget_fs=[-20000] * len(nets))
    T = oracle.Tree(inst)
    assert np.diff(T.net_ptr).tolist() == [128, 65, 64, 2, 3] and _heights(T).max() == 127
    P = oracle.Params(T)
    R, C = oracle.rc(T, P, None)
    S, t, d = oracle.elmore(T, R, C)
    g = DeviceRun(inst)
    dg = g.elmore()
    _rel_close(host(dg)[:T.sinks], d, REL, "delay")
    rng = np.random.default_rng(31)
    dslack = rng.uniform(0, 1, T.sinks).astype(np.float32)
    G, Sig, dR, dC = oracle.elmore_adjoint(T, R, C, S, -dslack.astype(np.float64))
    t_ = torch()
    dRg = t_.empty(T.nodes + T.sinks, dtype=t_.float32, device="cuda")
    dCg = t_.empty_like(dRg)
    la.la_elmore_backward(g.b, dev(dslack), dRg, dCg)
    net_of = _net_of(T)
    for name, gpu, ref in (("dR", host(dRg), dR), ("dC", host(dCg), dC)):
        assert _adjoint_tol(gpu, ref, net_of).all(), name
    w = oracle.adjoint_form_weights(T, P, None)
    d2 = g.elmore()
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(T.sinks, dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    la.la_timing_weights(g.b, d2, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
    swg, pwg, lg = host(sw).astype(np.int64), host(pw).astype(np.int64), host(lam).astype(np.int64)
    assert np.abs(pwg - w["pin_w"]).max() <= 1
    assert np.abs(swg - w["seg_w"]).max() <= 1
    assert (np.abs(lg - w["lam"]) <= 1 + 1e-5 * np.abs(w["lam"])).all()
    say("run limits: %d nodes, %d sinks, %d nonzero segment weights" % (T.nodes, T.sinks, (swg > 0).sum()))


def test_backward_after_reassignment_is_state_error(c1):
    # la_elmore reads the batch-owned R/C; la_assign then rewrites them from the new layers, so
    # that forward no longer describes them and the reverse sweep must refuse to reuse it
    T = oracle.Tree(c1)
    g = DeviceRun(c1)
    g.elmore()
    g.assign(np.full(T.nodes, 512), np.full(T.sinks, 512), np.zeros(T.nodes), None, rounds=1)
    t_ = torch()
    z = t_.zeros(g.b.sinks, dtype=t_.float32, device="cuda")
    with pytest.raises(la.LAError) as e:
        la.la_elmore_backward(g.b, z, None, None)
    assert e.value.code == la.LA_ERR_STATE
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(T.sinks, dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    with pytest.raises(la.LAError) as e:
        la.la_timing_weights(g.b, z, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
    assert e.value.code == la.LA_ERR_STATE
    # a fresh forward makes both legal again
    d = g.elmore()
    la.la_elmore_backward(g.b, z, None, None)
    la.la_timing_weights(g.b, d, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
    torch().cuda.synchronize()


def test_call_on_another_stream_is_refused(c1):
    t_ = torch()
    g = DeviceRun(c1)
    d = t_.empty(g.b.sinks, dtype=t_.float32, device="cuda")
    s = t_.cuda.Stream()
    with t_.cuda.stream(s):
        with pytest.raises(ValueError):
            la.la_elmore(g.b, d)
    la.la_elmore(g.b, d)


def test_central_differences_on_sampled_2m_nets():
    # The differentiation form's gradient at its full size: the 2,000,000-net batch on an assigned
    # RC (vias included; a seeded assignment), J = sum over violating sinks of w * slack with w the
    # Eq. 4 weight.  On 1,000 seeded nets: central differences of each net's own J_net (h = 1e-3
    # relative, FP64) against the FP64 reverse sweep (1e-8), and the GPU's FP32 reverse sweep
    # against both (1e-5 of max(|g|, 1e-3 x the net's largest |g|)).  J is linear in each single R
    # and C away from slack = 0, so the differences are exact up to rounding; edges whose
    # perturbation flips a sink of the net across slack = 0 are skipped.
    from test_gpu_assign import _subset
    inst = gen.config(4)
    T = oracle.Tree(inst)
    P = oracle.Params(T)
    rng = np.random.default_rng(4)
    lay = np.zeros(T.nodes, np.uint8)
    nonroot = T.parent >= 0
    for d in (0, 1):
        opts = np.nonzero(inst.layer_dir == d)[0]
        m = nonroot & (T.dir == d)
        lay[m] = opts[rng.integers(0, len(opts), int(m.sum()))]
    R, C = oracle.rc(T, P, lay)
    R32, C32 = R.astype(np.float32), C.astype(np.float32)
    R64, C64 = R32.astype(np.float64), C32.astype(np.float64)
    S, t, d = oracle.elmore(T, R64, C64)
    sl, wns, pw, tier = oracle.slack(T, d)
    omega = np.where(sl < 0, pw / 1024.0, 0.0)
    say("c4 gradient: %d nets, %d violating sinks" % (T.nets, int((sl < 0).sum())))
    # GPU: forward on the same float R/C, then the reverse sweep of J
    run = DeviceRun(inst)
    t_ = torch()
    Rg, Cg = dev(R32), dev(C32)
    delay = t_.empty(T.sinks, dtype=t_.float32, device="cuda")
    la.la_elmore_rc(run.b, Rg, Cg, delay)
    dRg = t_.empty(T.nodes + T.sinks, dtype=t_.float32, device="cuda")
    dCg = t_.empty_like(dRg)
    la.la_elmore_backward(run.b, dev(omega.astype(np.float32)), dRg, dCg)
    dRg, dCg = host(dRg).astype(np.float64), host(dCg).astype(np.float64)
    # the sample: 1,000 seeded nets among those with a violating sink (the others have J_net = 0)
    sink_net_full = np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1
    nets = np.sort(rng.choice(np.unique(sink_net_full[sl < 0]), 1000, replace=False))
    sub = _subset(inst, nets)
    Ts = oracle.Tree(sub)
    nidx = np.concatenate([np.arange(T.net_ptr[i], T.net_ptr[i + 1]) for i in nets])
    sidx = np.nonzero(np.isin(T.sink_node, nidx))[0]
    ridx = np.concatenate([nidx, T.nodes + sidx])       # the sample's RC edges in the full index space
    Rs, Cs = R64[ridx].copy(), C64[ridx].copy()
    om_s = omega[sidx]
    bud = sub.net_budget_fs[np.searchsorted(Ts.net_ptr, Ts.sink_node, side="right") - 1] * 1e-3
    s_net = np.searchsorted(Ts.net_ptr, Ts.sink_node, side="right") - 1
    n_of = _net_of(Ts)
    Ss, _, ds = oracle.elmore(Ts, Rs, Cs)
    G, Sig, dR_o, dC_o = oracle.elmore_adjoint(Ts, Rs, Cs, Ss, -om_s)
    viol0 = bud - ds < 0

    def jnet(delays):
        j = np.zeros(Ts.nets)
        np.add.at(j, s_net, om_s * np.minimum(0.0, bud - delays))
        return j, (bud - delays) < 0

    # the RC edges of every sampled net, position by position
    members = [[] for _ in range(Ts.nets)]
    for e in range(Ts.nodes + Ts.sinks):
        members[n_of[e]].append(e)
    depth = max(len(m) for m in members)
    fd = {"R": np.full(len(n_of), np.nan), "C": np.full(len(n_of), np.nan)}
    floor = {"R": np.zeros(len(n_of)), "C": np.zeros(len(n_of))}
    h = 1e-3
    for q in range(depth):
        es = np.array([m[q] for m in members if len(m) > q])
        for name, arr in (("R", Rs), ("C", Cs)):
            x0 = arr[es].copy()
            step = h * np.where(x0 != 0, np.abs(x0), 1.0)
            arr[es] = x0 + step
            jp, vp = jnet(oracle.elmore(Ts, Rs, Cs)[2])
            arr[es] = x0 - step
            jm, vm = jnet(oracle.elmore(Ts, Rs, Cs)[2])
            arr[es] = x0
            ok_sign = np.ones(Ts.nets, bool)
            flip = (vp != viol0) | (vm != viol0)
            ok_sign[s_net[flip]] = False
            nn = n_of[es]
            keep = ok_sign[nn]
            fd[name][es[keep]] = (jp[nn] - jm[nn])[keep] / (2 * step[keep])
            floor[name][es] = 16 * np.finfo(np.float64).eps * (np.abs(jp[nn]) + np.abs(jm[nn])) / (2 * step)
    checked = 0
    for name, ref, gpu in (("R", dR_o, dRg[ridx]), ("C", dC_o, dCg[ridx])):
        m = ~np.isnan(fd[name])
        checked += int(m.sum())
        err_fd = np.abs(fd[name][m] - ref[m])
        assert (err_fd <= 1e-8 * np.abs(ref[m]) + floor[name][m]).all(), "FD vs FP64 adjoint (%s)" % name
        ok = _adjoint_tol(gpu, ref, n_of)
        assert ok.all(), "GPU d%s vs FP64 adjoint: %d bad" % (name, (~ok).sum())
        ok_fd = _adjoint_tol(gpu[m], fd[name][m], n_of[m])
        assert ok_fd.all(), "GPU d%s vs central differences: %d bad" % (name, (~ok_fd).sum())
    say("central differences: %d RC-edge partials on %d nets" % (checked, Ts.nets))
    assert checked > 10000
