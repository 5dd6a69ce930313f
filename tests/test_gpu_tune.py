"""The batched form's launch configurations and its autotuner (the persistent per-batch launch
of Alg. 2's batch loop): every configuration gives the oracle's layers, via spans, demand and
history bit for bit; la_tune picks one on the instance and leaves the state as it was; the
round graphs are not instantiated again in a steady-state schedule."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, assert_assign_equal, dev, host, oracle_assign, say, torch

pytestmark = pytest.mark.gpu

# (tile nodes, claim units, workgroups, fused-commit threshold): every tile size, the claim
# size bounds, a small persistent grid, and fused commits for every batch / for none
CONFIGS = [(128, 96, 0, 1), (192, 220, 0, 16384), (256, 316, 0, 1 << 30), (192, 150, 64, 4096),
           (128, 300, 200, 1 << 30), (256, 96, 0, 1)]


@pytest.fixture(scope="module")
def c2_case():
    inst = gen.config(2, num_nets=60000)
    T = oracle.Tree(inst)
    w = oracle.plain_weights(T, oracle.Params(T))
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], w["tier"], rounds=3)
    return inst, w, o


@pytest.mark.parametrize("cfg", CONFIGS)
def test_every_configuration_matches_the_oracle(c2_case, cfg):
    inst, w, o = c2_case
    run = DeviceRun(inst)
    la.la_set_tuning(run.b, *cfg)
    assert la.la_get_tuning(run.b) == dict(tile_nodes=cfg[0], claim_units=cfg[1], workgroups=cfg[2],
                                           fuse_nets=cfg[3], tuned=0)
    say("tuning %s" % (cfg,))
    g = run.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=3, form=la.LA_FORM_BATCHED)
    assert_assign_equal(g, o, "tuning %s" % (cfg,))


def test_tune_keeps_state_and_results(c2_case):
    inst, w, o = c2_case
    run = DeviceRun(inst)
    # one call first, so the tuner starts from a state with previous layers and history
    first = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], w["tier"], rounds=1)
    g1 = run.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=1, form=la.LA_FORM_BATCHED)
    assert_assign_equal(g1, first, "before tuning")
    t = la.la_tune(run.b, dev(w["seg_w"], np.uint16), dev(w["pin_w"], np.uint16), dev(w["lam"], np.int32), run.H,
                   net_tier=dev(w["tier"], np.uint8), num_tiers=11)
    say("la_tune chose %s" % t)
    assert t["tuned"] == 1 and t["tile_nodes"] in (128, 192, 256) and 96 <= t["claim_units"] <= 316
    assert la.la_batch_info(run.b)["tuning"] == t
    # nothing moved: demand, layers and via spans are those of the first call
    D = torch().empty(run.E, dtype=torch().int32, device="cuda")
    la.la_demand(run.b, D)
    assert np.array_equal(host(D), first["D"])
    assert np.array_equal(host(run.H), first["H"])
    # the next two rounds continue from there, as on the oracle
    st = first["state"]
    lay, vlo, vhi, _ = oracle.assign(first["tree"], first["params"], st, w["tier"], rounds=2)
    g2 = run.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=2, form=la.LA_FORM_BATCHED)
    assert_assign_equal(g2, dict(layers=lay, vlo=vlo, vhi=vhi, D=st.D, H=st.H, tree=first["tree"]), "after tuning")
    # a second batch of the same shape takes the cached choice without timing
    run2 = DeviceRun(inst)
    t2 = la.la_tune(run2.b, dev(w["seg_w"], np.uint16), dev(w["pin_w"], np.uint16), dev(w["lam"], np.int32),
                    run2.H, net_tier=dev(w["tier"], np.uint8), num_tiers=11)
    assert t2 == t


def test_set_tuning_rejects_bad_values(c2_case):
    inst, _, _ = c2_case
    run = DeviceRun(gen.config(1, num_nets=50))
    for bad in [(100, 220, 0, 1), (192, 50, 0, 1), (192, 400, 0, 1), (192, 220, -1, 1), (192, 220, 0, 0)]:
        with pytest.raises(la.LAError) as e:
            la.la_set_tuning(run.b, *bad)
        assert e.value.code == la.LA_ERR_INVALID_ARG
    # eight layers: four routable layers per direction, built for the default tile size only
    with pytest.raises(la.LAError):
        la.la_set_tuning(run.b, 128, 220, 0, 1)


def test_steady_state_schedule_instantiates_no_graph():
    inst = gen.config(2, num_nets=20000)
    run = DeviceRun(inst)
    t_ = torch()
    d = t_.empty(run.b.sinks, dtype=t_.float32, device="cuda")
    sw = t_.empty(run.b.nodes, dtype=t_.uint16, device="cuda")
    pw = t_.empty(run.b.sinks, dtype=t_.uint16, device="cuda")
    lam = t_.empty(run.b.nodes, dtype=t_.int32, device="cuda")
    tier = t_.empty(run.b.nets, dtype=t_.uint8, device="cuda")

    def step():
        la.la_reset(run.b)
        run.H.zero_()
        for _ in range(3):
            la.la_elmore(run.b, d)
            la.la_timing_weights(run.b, d, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
            la.la_assign(run.b, sw, pw, lam, run.H, run.layers, net_tier=tier, num_tiers=11, rounds=2,
                         form=la.LA_FORM_BATCHED)
        t_.cuda.synchronize()
        return host(run.layers).copy(), host(run.H).copy()

    a = step()
    n1 = la.la_batch_info(run.b)["graph_instantiations"]
    b = step()
    n2 = la.la_batch_info(run.b)["graph_instantiations"]
    say("graph instantiations: %d after the first step, %d after the second" % (n1, n2))
    assert n1 >= 1 and n2 == n1
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
