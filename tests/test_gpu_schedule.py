"""GPU parity of whole negotiation schedules (Alg. 2 batch loop with rounds and history) against
the oracle, element by element: layers, via spans, demand and history after every call.

- c2 in full (200,000 nets) with 5 rounds over the 11 Alg. 1 batches, both forms: the four
  non-critical batches hold about 50,000 nets each, so from the second round on the batched form
  moves their demand (-1 on the old layer, +1 on the new) from inside its DP kernel.
- c4 in full (2,000,000 nets): the differentiation schedule of 3 outer iterations of 5 rounds.
  Each iteration's integer weights come from the oracle's adjoint form on the oracle's own
  layers and go to both sides; the GPU's own adjoint weights are checked beside them (+-1 LSB).
- the look-ahead off (lambda = 0) on both forms, at a size where batches take the fused commit.
- a tie between a child's layers inside its parent's stack (lowest layer wins) on both forms."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, assert_assign_equal, dev, host, oracle_assign, say, tier_flips_at_bin_edges, torch
from helpers import make_instance

pytestmark = pytest.mark.gpu

FORMS = [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED]


def _plain_weights(inst):
    T = oracle.Tree(inst)
    return oracle.plain_weights(T, oracle.Params(T))


@pytest.mark.parametrize("form", FORMS)
def test_config2_full_five_rounds(form):
    inst = gen.config(2)
    w = _plain_weights(inst)
    counts = np.bincount(w["tier"], minlength=11)
    say("c2 R=5 form=%d batches %s" % (form, counts.tolist()))
    assert counts[7:].min() >= 16384        # these batches take the fused commit in the batched form
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], w["tier"], rounds=5)
    g = DeviceRun(inst).assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=5, form=form)
    assert_assign_equal(g, o, "c2 R=5")


def _adjoint_weights_gpu(run, T):
    t_ = torch()
    d = run.elmore()
    sw = t_.empty(T.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(max(T.sinks, 1), dtype=t_.uint16, device="cuda")
    lam = t_.empty(T.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(T.nets, dtype=t_.uint8, device="cuda")
    la.la_timing_weights(run.b, d, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
    return dict(seg_w=host(sw).astype(np.int64), pin_w=host(pw)[:T.sinks].astype(np.int64),
                lam=host(lam).astype(np.int64), tier=host(tier))


def test_config4_full_adjoint_schedule():
    # the headline schedule at its full size: R = 5 rounds x I = 3 iterations, batched form
    R_ROUNDS, I_ITERS = 5, 3
    inst = gen.config(4)
    T = oracle.Tree(inst)
    P0 = oracle.Params(T)
    st = oracle.State(T)
    run = DeviceRun(inst)
    say("c4: %d nets, %d LA nodes" % (T.nets, T.nodes))
    lay = None
    sink_net = np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1
    for it in range(I_ITERS):
        w = oracle.adjoint_form_weights(T, P0, lay)
        # the GPU's own weights from its own timing of the same layers
        gw = _adjoint_weights_gpu(run, T)
        assert np.abs(gw["seg_w"] - w["seg_w"]).max() <= 1
        assert np.abs(gw["pin_w"] - w["pin_w"]).max() <= 1
        # lambda = -Sig(parent) * 1e6 sums omega * (upstream R) over the sinks below; a sink
        # whose quantised omega differs by one LSB on the two sides (FP32 against FP64 slack)
        # moves it by at most |d omega| * (the net's summed R) * 1e6, so that is added to the
        # rounding and FP32 allowance, net by net
        R, _ = oracle.rc(T, P0, lay)
        node_net = np.searchsorted(T.net_ptr, np.arange(T.nodes), side="right") - 1
        rsum = np.bincount(np.concatenate([node_net, sink_net]), weights=R, minlength=T.nets)
        dom = np.bincount(sink_net, weights=np.abs(gw["pin_w"] - w["pin_w"]) / 1024.0, minlength=T.nets)
        slackq = 1e6 * dom * rsum * (1 + 1e-6)
        dl = np.abs(gw["lam"] - w["lam"])
        tight = dom[node_net] == 0
        say("iteration %d: lambda max diff %d on nets with equal omegas (%d nodes), %d on the others (%d nodes)" % (
            it, int(dl[tight].max(initial=0)), int(tight.sum()), int(dl[~tight].max(initial=0)), int((~tight).sum())))
        assert (dl <= 1 + 1e-5 * np.abs(w["lam"]) + slackq[node_net]).all()
        ns = np.full(T.nets, np.inf)
        np.minimum.at(ns, sink_net, w["slack"])
        flips = tier_flips_at_bin_edges(gw["tier"], w["tier"], ns / w["wns"])
        say("iteration %d: weight LSB diffs seg %d pin %d, batch flips %d" % (
            it, int((gw["seg_w"] != w["seg_w"]).sum()), int((gw["pin_w"] != w["pin_w"]).sum()), flips))
        # identical integer inputs on both sides
        P = oracle.Params(T, seg_w=w["seg_w"], pin_w=w["pin_w"], lam=w["lam"])
        lay, vlo, vhi, _ = oracle.assign(T, P, st, w["tier"], rounds=R_ROUNDS)
        g = run.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=R_ROUNDS,
                       form=la.LA_FORM_BATCHED)
        assert_assign_equal(g, dict(layers=lay, vlo=vlo, vhi=vhi, D=st.D, H=st.H, tree=T), "c4 iteration %d" % it)
        say("iteration %d: layers, via spans, demand and history equal the oracle's" % it)


@pytest.mark.parametrize("form", FORMS)
def test_lookahead_off(form):
    # lambda = 0 turns the look-ahead off (the paper's "w/o look-ahead" ablation); 80,000 nets so
    # the non-critical batches take the fused commit of the batched form
    inst = gen.config(2, num_nets=80000)
    w = _plain_weights(inst)
    lam0 = np.zeros_like(w["lam"])
    say("lambda=0 form=%d" % form)
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], lam0, w["tier"], rounds=3)
    g = DeviceRun(inst).assign(w["seg_w"], w["pin_w"], lam0, w["tier"], num_tiers=11, rounds=3, form=form)
    assert_assign_equal(g, o, "lambda=0")


@pytest.mark.parametrize("form", FORMS)
def test_child_tie_takes_the_lowest_layer(form):
    # driver -H-> sink A -H-> sink B with history that ties B's costs on layers 0, 2 and 4 and
    # sends A to layer 4 (the oracle pins this case in closed form): B must take layer 0
    V = 1000
    nets = [([(0, 0, -1, "driver"), (5, 0, 0, "sink"), (9, 0, 1, "sink")], [[], [], []])]
    inst = make_instance(nets, X=12, Y=3, L=8)
    T = oracle.Tree(inst)
    L = inst.L
    H = np.zeros(inst.X * inst.Y * L, np.int32)
    for x in range(5, 9):
        H[x * L + 0], H[x * L + 2] = V, V // 2
    for x in range(0, 5):
        for l in (0, 2, 6):
            H[x * L + l] = 1 << 20
    sw = np.zeros(T.nodes, np.uint16)
    sw[1] = 1024
    pw = np.zeros(T.sinks, np.uint16)
    lam = np.zeros(T.nodes, np.int32)
    kw = dict(w_cong=1, w_cap=0, w_d=1, w_via=V)
    o = oracle_assign(inst, sw, pw, lam, None, rounds=1, H0=H, **kw)
    assert o["layers"][1] == 4 and o["layers"][2] == 0
    run = DeviceRun(inst)
    run.H.copy_(dev(H))
    g = run.assign(sw, pw, lam, None, rounds=1, form=form, **kw)
    assert_assign_equal(g, o, "tie")
