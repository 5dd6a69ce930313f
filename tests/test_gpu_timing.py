"""GPU parity of the timing path against the FP64 oracle: RC edges, Elmore delay, reverse
sweep, torch autograd wrapper, TNS/WNS and the DP timing weights (Eq. 4, Eq. 5, adjoint)."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, dev, host, say, torch

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


def _tier_boundary_ok(gt, ot, rho):
    """Batches may differ only where the FP64 rho lies within 1e-5 of the bin edge between them."""
    edges = np.array([1.0, 0.99, 0.96, 0.91, 0.84, 0.75, 0.7])
    diff = np.nonzero(gt != ot)[0]
    for i in diff:
        a, b = sorted((int(gt[i]), int(ot[i])))
        if b > 7 or a > 6:
            e = 0.7
        else:
            e = edges[b] if b < len(edges) else 0.7
        assert abs(rho[i] - e) < 1e-5 * max(1.0, abs(e)), (i, gt[i], ot[i], rho[i])
    return diff.size


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
    flips = _tier_boundary_ok(tg, w["tier"], ns / w["wns"])
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
