"""GPU parity of layer assignment (Alg. 2-4 with look-ahead, commit, history) against the
oracle: bit-exact layers, via spans, demand and history on identical integer inputs."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, assert_assign_equal, oracle_assign, say
from helpers import make_instance

pytestmark = pytest.mark.gpu

FORMS = [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED]


def _weights_from_oracle(inst):
    T = oracle.Tree(inst)
    return oracle.plain_weights(T, oracle.Params(T))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("rounds,tiered", [(1, False), (1, True), (5, True)])
def test_config1(form, rounds, tiered):
    inst = gen.config(1)
    w = _weights_from_oracle(inst)
    tiers = w["tier"] if tiered else None
    say("c1 form=%d rounds=%d tiered=%s" % (form, rounds, tiered))
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], tiers, rounds=rounds)
    g = DeviceRun(inst).assign(w["seg_w"], w["pin_w"], w["lam"], tiers, num_tiers=11, rounds=rounds, form=form)
    assert_assign_equal(g, o, "c1")


@pytest.mark.parametrize("form", FORMS)
def test_synthetic_weights_many_tiers(form):
    inst = gen.generate(3000, 96, 80, 10, 99, pin_law=1, pin_max=40, placement=1, n_hot=6, hot_sigma=12.0,
                        cap_min=0, cap_max=6)
    T = oracle.Tree(inst)
    sw = gen.synthetic_weights(T.nodes, T.sinks, T.nets, seed=5, n_tiers=7)
    say("synthetic form=%d nodes=%d" % (form, T.nodes))
    o = oracle_assign(inst, sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], rounds=3,
                      w_d=3, w_via=7000)
    g = DeviceRun(inst).assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], num_tiers=7,
                            rounds=3, form=form, w_d=3, w_via=7000)
    assert_assign_equal(g, o, "synthetic")


def _star(k, L=8):
    # a Steiner node with k sink branches (a node with more than four children)
    nodes = [(10, 10, -1, "driver"), (14, 10, 0, "steiner")]
    wps = [[], []]
    dirs = [(1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1), (3, 2)]
    for q in range(k):
        dx, dy = dirs[q % len(dirs)]
        x, y = 14 + dx * (1 + q // len(dirs)), 10 + dy * (3 + q // len(dirs))
        nodes.append((x, y, 1, "sink"))
        wps.append([(x, 10)] if dx and dy else [])
    return nodes, wps


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("case", ["star6", "star8_sink_centre", "l16", "l2", "min_layer", "driver_only",
                                  "zero_weights"])
def test_edge_cases(case, form):
    L, min_layer, kw = 8, 0, {}
    if case == "star6":
        nets = [_star(6), _star(3)]
    elif case == "star8_sink_centre":
        n, w = _star(8)
        n[1] = (n[1][0], n[1][1], 0, "sink")
        nets = [(n, w)]
    elif case == "l16":
        nets = [_star(4)]
        L = 16
    elif case == "l2":
        nets = [_star(2)]
        L = 2
    elif case == "min_layer":
        nets = [_star(5)]
        min_layer = 2
    elif case == "driver_only":
        nets = [([(3, 3, -1, "driver")], [[]]), _star(2)]
    else:
        nets = [_star(5), _star(2)]
        kw = dict(w_cong=0, w_cap=0, w_d=0, w_via=0)
    rc = None
    if L != 8:
        r = [20000 - 900 * i for i in range(L)]
        c = [200 - 9 * i for i in range(L)]
        rc = (r, c, [5000] * (L - 1))
    inst = make_instance(nets, X=24, Y=24, L=L, layer_rc=rc,
                         caps=np.random.default_rng(1).integers(0, 3, (24, 24, L)).astype(np.uint8))
    T = oracle.Tree(inst)
    rng = np.random.default_rng(3)
    sw = rng.integers(0, 1025, T.nodes)
    pw = rng.integers(0, 1025, max(T.sinks, 1))
    lam = rng.integers(0, 500000, T.nodes)
    o = oracle_assign(inst, sw, pw, lam, None, rounds=2, min_layer=min_layer, **kw)
    g = DeviceRun(inst, min_layer=min_layer).assign(sw, pw, lam, None, rounds=2, form=form, **kw)
    assert_assign_equal(g, o, case)


def test_empty_batch():
    inst = make_instance([], X=4, Y=4)
    g = DeviceRun(inst)
    assert g.b.nets == 0 and g.b.nodes == 0
    g.assign(np.zeros(1), np.zeros(1), np.zeros(1))


@pytest.mark.parametrize("form", FORMS)
def test_config2_full(form):
    inst = gen.config(2)
    w = _weights_from_oracle(inst)
    say("c2 full form=%d" % form)
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], w["tier"], rounds=1)
    g = DeviceRun(inst).assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=1, form=form)
    assert_assign_equal(g, o, "c2")


def _subset(inst, nets):
    """The instance restricted to the given nets (same grid and capacities)."""
    ptr = inst.net_node_ptr
    parts = [np.arange(ptr[i], ptr[i + 1]) for i in nets]
    idx = np.concatenate(parts)
    counts = np.array([len(p) for p in parts])
    wp_counts = np.diff(inst.edge_wp_ptr)[idx]
    wp_idx = np.concatenate([np.arange(inst.edge_wp_ptr[v], inst.edge_wp_ptr[v + 1]) for v in idx])
    return gen.Instance(
        name="subset", X=inst.X, Y=inst.Y, L=inst.L,
        net_node_ptr=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32),
        node_parent=inst.node_parent[idx], node_x=inst.node_x[idx], node_y=inst.node_y[idx],
        node_flags=inst.node_flags[idx], node_cpin_af=inst.node_cpin_af[idx],
        edge_wp_ptr=np.concatenate([[0], np.cumsum(wp_counts)]).astype(np.int32),
        wp_x=inst.wp_x[wp_idx.astype(np.int64)] if wp_idx.size else inst.wp_x[:0],
        wp_y=inst.wp_y[wp_idx.astype(np.int64)] if wp_idx.size else inst.wp_y[:0],
        net_budget_fs=inst.net_budget_fs[nets], net_rdrv_mohm=inst.net_rdrv_mohm[nets], caps=inst.caps,
        r_mohm=inst.r_mohm, c_af=inst.c_af, via_r_mohm=inst.via_r_mohm, layer_dir=inst.layer_dir)


@pytest.mark.parametrize("form", FORMS)
def test_config3_full_size_sampled(form):
    # one round, one batch: every net meets the empty demand map, so each sampled net's
    # result is fixed by the net alone and the oracle checks it one by one
    inst = gen.config(3)
    say("c3 full sampled form=%d" % form)
    g = DeviceRun(inst)
    n = g.b.nodes
    sw = gen.synthetic_weights(n, g.b.sinks, g.b.nets, seed=11)
    res = g.assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], None, rounds=1, form=form)
    rng = np.random.default_rng(3)
    nets = np.sort(rng.choice(inst.num_nets, 3000, replace=False))
    sub = _subset(inst, nets)
    T = oracle.Tree(inst)
    la_ptr = T.net_ptr
    nidx = np.concatenate([np.arange(la_ptr[i], la_ptr[i + 1]) for i in nets])
    sidx = np.nonzero(np.isin(T.sink_node, nidx))[0]
    o = oracle_assign(sub, sw["seg_w_q10"][nidx], sw["pin_w_q10"][sidx], sw["lambda_mohm"][nidx], None, rounds=1)
    for k in ("layers", "vlo", "vhi"):
        gv = res[k][nidx]
        ov = o[k]
        if k == "layers":
            gv = np.where(o["tree"].parent >= 0, gv, 0)
            ov = np.where(o["tree"].parent >= 0, ov, 0)
        assert np.array_equal(gv, ov), k
    # demand is a recount of the layers on the full grid
    nonroot = T.parent >= 0
    per_layer = np.bincount(res["layers"][nonroot], weights=T.len[nonroot], minlength=inst.L)
    assert np.array_equal(res["D"].reshape(-1, inst.L).sum(0), per_layer.astype(np.int64))


@pytest.mark.parametrize("form", FORMS)
def test_nets_larger_than_a_tile(form):
    # high-fanout nets (hundreds of layer-assignment nodes) take the HBM-state path
    inst = gen.generate(400, 160, 160, 8, 17, pin_law=1, pin_max=12, placement=2, fanout_every=37, fanout_min=150,
                        fanout_max=320, cap_min=2, cap_max=8)
    T = oracle.Tree(inst)
    sizes = np.diff(T.net_ptr)
    assert (sizes > 256).sum() >= 5
    sw = gen.synthetic_weights(T.nodes, T.sinks, T.nets, seed=8, n_tiers=3)
    say("big nets form=%d max nodes %d" % (form, sizes.max()))
    o = oracle_assign(inst, sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], rounds=2)
    g = DeviceRun(inst).assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], num_tiers=3,
                            rounds=2, form=form)
    assert_assign_equal(g, o, "big")


@pytest.mark.parametrize("form", FORMS)
def test_huge_nets_with_four_children(form):
    # nets of 1,000-1,600 pins (up to thousands of layer-assignment nodes, one node with four
    # children): the big-net walk reads a node's first three children from its record and the
    # fourth from the child list
    inst = gen.generate(240, 256, 256, 10, 23, pin_law=1, pin_max=16, placement=2, fanout_every=40,
                        fanout_min=1000, fanout_max=1600, cap_min=4, cap_max=10)
    T = oracle.Tree(inst)
    par = np.asarray(T.parent)
    kids = np.bincount(par[par >= 0], minlength=T.nodes)
    sizes = np.diff(T.net_ptr)
    big = sizes[np.repeat(np.arange(T.nets), sizes)] > 256
    assert (kids[big] >= 4).any()
    sw = gen.synthetic_weights(T.nodes, T.sinks, T.nets, seed=11, n_tiers=2)
    o = oracle_assign(inst, sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], rounds=2)
    g = DeviceRun(inst).assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], sw["net_tier"], num_tiers=2,
                               rounds=2, form=form)
    say("huge nets form=%d: %d big-net nodes, %d with four or more children" % (
        form, big.sum(), (kids[big] >= 4).sum()))
    assert_assign_equal(g, o, "huge")


def test_graph_replays_match_eager_plain_form():
    # the batched rounds run as a captured hipGraph; every replay, with eager work and
    # synchronisation in between, must give the plain (eager) form's result
    inst = gen.config(2, num_nets=30000)
    w = _weights_from_oracle(inst)
    ref = DeviceRun(inst).assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=3)
    g = DeviceRun(inst)
    for rep in range(4):
        la.la_reset(g.b)
        g.H.zero_()
        res = g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=3, form=la.LA_FORM_BATCHED)
        for k in ("layers", "vlo", "vhi", "D", "H"):
            assert np.array_equal(res[k], ref[k]), (rep, k)
        say("replay %d ok" % rep)


def test_checkpoint_resume_on_gpu():
    inst = gen.config(1)
    w = _weights_from_oracle(inst)
    g = DeviceRun(inst)
    g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=2, form=la.LA_FORM_BATCHED)
    state = la.la_save_state(g.b)
    H_saved = g.H.clone()
    nxt = g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=1, form=la.LA_FORM_BATCHED)
    g2 = DeviceRun(inst)
    la.la_load_state(g2.b, state)
    g2.H.copy_(H_saved)
    again = g2.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=1, form=la.LA_FORM_PLAIN)
    for k in ("layers", "vlo", "vhi", "D", "H"):
        assert np.array_equal(nxt[k], again[k]), k


def test_out_of_range_batch_index_is_rejected():
    inst = gen.config(1)
    g = DeviceRun(inst)
    n = g.b.nodes
    for form in FORMS:
        with pytest.raises(la.LAError) as e:
            g.assign(np.zeros(n), np.zeros(g.b.sinks), np.zeros(n), np.full(g.b.nets, 5), num_tiers=3, form=form)
        assert e.value.code == la.LA_ERR_INVALID_ARG


def test_merged_single_net_batches():
    # forty batches of one net each, then one large batch: disjoint tiny batches share a
    # launch, and the result still equals the oracle's one-batch-after-another schedule
    inst = gen.config(3, num_nets=6000)
    T = oracle.Tree(inst)
    sw = gen.synthetic_weights(T.nodes, T.sinks, T.nets, seed=21)
    tiers = np.full(T.nets, 40, np.uint8)
    tiers[:40] = np.arange(40)
    say("merged batches: %d nets" % T.nets)
    o = oracle_assign(inst, sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], tiers, rounds=2)
    run = DeviceRun(inst)
    la.la_profile_begin(run.b)
    g = run.assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], tiers, num_tiers=41, rounds=2,
                   form=la.LA_FORM_BATCHED)
    stats = la.la_profile_end(run.b)
    assert_assign_equal(g, o, "merged")
    launches = stats["k_batched_dp"][0]
    say("k_batched_dp launches: %d for 2 rounds of 41 batches" % launches)
    assert launches < 2 * 41
