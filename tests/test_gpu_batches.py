"""GPU classical batching (Alg. 1, GetBatch) against the oracle's sequential first-fit, and the
layer assignment run on those batches (int32 batch indices) against the oracle's schedule on
the same batches: batch indices and counts bit for bit; layers, via spans, demand and history
element by element on both forms."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, assert_assign_equal, dev, host, oracle_assign, say, torch

pytestmark = pytest.mark.gpu


def _gpu_batches(run, subset, nsub):
    t_ = torch()
    out = t_.empty(max(run.b.nets, 1), dtype=t_.int32, device="cuda")
    n = la.la_get_batches(run.b, dev(subset, np.int32), nsub, out)
    return host(out)[:run.b.nets], n


@pytest.mark.parametrize("nets,nsub", [(2000, 1), (60000, 3), (500000, 11)])
def test_batches_equal_the_oracle(nets, nsub):
    inst = gen.config(4, num_nets=nets)
    T = oracle.Tree(inst)
    rng = np.random.default_rng(nets)
    # subsets in random order with some nets left out (-1) and some beyond the range (nsub)
    subset = rng.integers(-1, nsub + 1, T.nets).astype(np.int32)
    ob, on = oracle.get_batches(T, inst.X, inst.Y, subset, nsub)
    run = DeviceRun(inst)
    gb, gn = _gpu_batches(run, subset, nsub)
    say("%d nets, %d subsets: %d batches (oracle %d)" % (nets, nsub, gn, on))
    assert gn == on
    bad = np.nonzero(gb != ob)[0]
    assert bad.size == 0, (bad[:5], gb[bad[:5]], ob[bad[:5]])


def test_grid_not_a_multiple_of_the_bin_size():
    # 37 x 29 GCells: the blocking bins (4 x 4 GCells) of the last row and column are partial
    inst = gen.generate(3000, 37, 29, 8, 4242, pin_law=1, pin_max=24, placement=1, n_hot=4, hot_sigma=6.0)
    T = oracle.Tree(inst)
    rng = np.random.default_rng(37)
    subset = rng.integers(0, 3, T.nets).astype(np.int32)
    ob, on = oracle.get_batches(T, inst.X, inst.Y, subset, 3)
    gb, gn = _gpu_batches(DeviceRun(inst), subset, 3)
    say("37x29 grid, 3000 nets: %d batches (oracle %d)" % (gn, on))
    assert gn == on and np.array_equal(gb, ob)


def test_single_net_and_identical_boxes():
    # every net of c1 in one subset, then the same nets twice over (identical boxes stack up)
    inst = gen.config(1, num_nets=300)
    T = oracle.Tree(inst)
    sub = np.zeros(T.nets, np.int32)
    ob, on = oracle.get_batches(T, inst.X, inst.Y, sub, 1)
    gb, gn = _gpu_batches(DeviceRun(inst), sub, 1)
    assert gn == on and np.array_equal(gb, ob)


@pytest.mark.parametrize("form", [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED])
def test_assignment_on_classical_batches(form):
    # Alg. 1 flow on a 40,000-net sample: the 11 slack-bin batches as subsets, each split into
    # bounding-box-disjoint batches; two negotiation rounds over them
    inst = gen.config(4, num_nets=40000)
    T = oracle.Tree(inst)
    w = oracle.plain_weights(T, oracle.Params(T))
    ob, on = oracle.get_batches(T, inst.X, inst.Y, w["tier"].astype(np.int32), 11)
    run = DeviceRun(inst)
    gb, gn = _gpu_batches(run, w["tier"].astype(np.int32), 11)
    assert gn == on and np.array_equal(gb, ob)
    say("form %d: %d classical batches" % (form, gn))
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], ob, rounds=2)
    sw, pw, lm = dev(w["seg_w"], np.uint16), dev(w["pin_w"], np.uint16), dev(w["lam"], np.int32)
    la.la_assign(run.b, sw, pw, lm, run.H, run.layers, num_tiers=gn, rounds=2, form=form,
                 net_batch=dev(gb, np.int32))
    t_ = torch()
    vias = t_.empty(2 * run.b.nodes, dtype=t_.uint8, device="cuda")
    la.la_vias(run.b, vias)
    D = t_.empty(run.E, dtype=t_.int32, device="cuda")
    la.la_demand(run.b, D)
    v = host(vias).reshape(-1, 2)
    g = dict(layers=host(run.layers)[:run.b.nodes], vlo=v[:, 0], vhi=v[:, 1], D=host(D), H=host(run.H))
    assert_assign_equal(g, o, "classical batches")


def test_batch_index_out_of_range_is_refused():
    inst = gen.config(1, num_nets=100)
    run = DeviceRun(inst)
    n = run.b.nodes
    for form in (la.LA_FORM_PLAIN, la.LA_FORM_BATCHED):
        with pytest.raises(la.LAError) as e:
            la.la_assign(run.b, dev(np.zeros(n), np.uint16), dev(np.zeros(run.b.sinks), np.uint16),
                         dev(np.zeros(n), np.int32), run.H, run.layers, num_tiers=3, form=form,
                         net_batch=dev(np.full(run.b.nets, 3), np.int32))
        assert e.value.code == la.LA_ERR_INVALID_ARG
