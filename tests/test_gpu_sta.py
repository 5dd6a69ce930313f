"""GPU critical-path net ordering (Sec. III-A; Alg. 1 ordering) against the oracle: static
timing of the synthetic gate graph, top-1 critical-path counts and the ordered subsets, bit for
bit (single precision, each value rounded once, on identical sink delays: the oracle's FP64
Elmore delays rounded to single precision feed both sides); then the whole Alg. 1 flow --
subsets, classical batches, layer assignment -- element by element."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, assert_assign_equal, dev, host, say, torch

pytestmark = pytest.mark.gpu


def _setup(nets, clock_fs=1000000):
    inst = gen.config(4, num_nets=nets)
    T = oracle.Tree(inst)
    tg = gen.timing_graph(inst, clock_fs=clock_fs)
    R, C = oracle.rc(T, oracle.Params(T), None)
    _, _, d = oracle.elmore(T, R, C)
    d32 = d.astype(np.float32)
    run = DeviceRun(inst)
    la.la_timing_graph(run.b, tg["sink_next"], tg["gate_delay_fs"], tg["clock_fs"])
    return inst, T, tg, d32, run


def _gpu_sta(run, d32):
    t_ = torch()
    sl = t_.empty(max(run.b.sinks, 1), dtype=t_.float32, device="cuda")
    cr = t_.empty(max(run.b.nets, 1), dtype=t_.int32, device="cuda")
    wns = la.la_sta(run.b, dev(d32), sl, cr)
    return sl, cr, wns


@pytest.mark.parametrize("nets", [20000, 2000000])
def test_sta_counts_and_subsets_equal_the_oracle(nets):
    inst, T, tg, d32, run = _setup(nets)
    osl, ocr, ownz = oracle.sta(T, tg["sink_next"], tg["gate_delay_fs"], tg["clock_fs"], d32)
    sl, cr, wns = _gpu_sta(run, d32)
    say("%d nets: WNS %.3f ps (oracle %.3f), %d nets on critical paths, %d critical" % (
        nets, wns, ownz, int((ocr > 0).sum()), int((ocr > 3).sum())))
    assert np.float32(wns) == np.float32(ownz)
    gs = host(sl)[:T.sinks]
    bad = np.nonzero(gs != osl)[0]
    assert bad.size == 0, (bad[:5], gs[bad[:5]], osl[bad[:5]])
    assert np.array_equal(host(cr)[:T.nets], ocr)
    t_ = torch()
    sub = t_.empty(max(run.b.nets, 1), dtype=t_.int32, device="cuda")
    n = la.la_alg1_subsets(run.b, sl, cr, wns, sub)
    osub, on = oracle.alg1_subsets(T, osl, ocr, ownz)
    say("subsets %d (oracle %d): %s" % (n, on, np.bincount(osub, minlength=on).tolist()))
    assert n == on and np.array_equal(host(sub)[:T.nets], osub)


def test_alg1_flow_assignment():
    # Alg. 1's ordering and GetBatch, then the layer assignment (two rounds, batched form) on their batches
    inst, T, tg, d32, run = _setup(40000, clock_fs=800000)
    sl, cr, wns = _gpu_sta(run, d32)
    t_ = torch()
    sub = t_.empty(run.b.nets, dtype=t_.int32, device="cuda")
    nsub = la.la_alg1_subsets(run.b, sl, cr, wns, sub)
    bat = t_.empty(run.b.nets, dtype=t_.int32, device="cuda")
    nb = la.la_get_batches(run.b, sub, nsub, bat)
    osl, ocr, ownz = oracle.sta(T, tg["sink_next"], tg["gate_delay_fs"], tg["clock_fs"], d32)
    osub, on = oracle.alg1_subsets(T, osl, ocr, ownz)
    ob, onb = oracle.get_batches(T, inst.X, inst.Y, osub, on)
    assert nb == onb and np.array_equal(host(bat)[:T.nets], ob)
    say("Alg. 1 flow: %d subsets, %d batches" % (nsub, nb))
    w = oracle.plain_weights(T, oracle.Params(T))
    P = oracle.Params(T, seg_w=w["seg_w"], pin_w=w["pin_w"], lam=w["lam"])
    st = oracle.State(T)
    lay, vlo, vhi, _ = oracle.assign(T, P, st, ob, rounds=2)
    la.la_assign(run.b, dev(w["seg_w"], np.uint16), dev(w["pin_w"], np.uint16), dev(w["lam"], np.int32), run.H,
                 run.layers, num_tiers=nb, rounds=2, form=la.LA_FORM_BATCHED, net_batch=bat)
    vias = t_.empty(2 * run.b.nodes, dtype=t_.uint8, device="cuda")
    la.la_vias(run.b, vias)
    D = t_.empty(run.E, dtype=t_.int32, device="cuda")
    la.la_demand(run.b, D)
    v = host(vias).reshape(-1, 2)
    g = dict(layers=host(run.layers)[:run.b.nodes], vlo=v[:, 0], vhi=v[:, 1], D=host(D), H=host(run.H))
    assert_assign_equal(g, dict(layers=lay, vlo=vlo, vhi=vhi, D=st.D, H=st.H, tree=T), "Alg. 1 flow")


def test_graph_errors():
    inst = gen.config(1, num_nets=50)
    run = DeviceRun(inst)
    t_ = torch()
    sl = t_.empty(run.b.sinks, dtype=t_.float32, device="cuda")
    cr = t_.empty(run.b.nets, dtype=t_.int32, device="cuda")
    with pytest.raises(la.LAError) as e:
        la.la_sta(run.b, t_.zeros(run.b.sinks, dtype=t_.float32, device="cuda"), sl, cr)
    assert e.value.code == la.LA_ERR_STATE
    tg = gen.timing_graph(inst)
    nxt = tg["sink_next"].copy()
    # net 0's first sink feeds net 1 and net 1's first sink feeds net 0: a cycle
    sink_net = np.repeat(np.arange(inst.num_nets), np.diff(inst.net_node_ptr))[(inst.node_flags & 1) != 0]
    nxt[np.nonzero(sink_net == 0)[0][0]] = 1
    nxt[np.nonzero(sink_net == 1)[0][0]] = 0
    with pytest.raises(la.LAError) as e:
        la.la_timing_graph(run.b, nxt, tg["gate_delay_fs"], tg["clock_fs"])
    assert e.value.code == la.LA_ERR_INVALID_ARG
    nxt = tg["sink_next"].copy()
    nxt[0] = inst.num_nets
    with pytest.raises(la.LAError) as e:
        la.la_timing_graph(run.b, nxt, tg["gate_delay_fs"], tg["clock_fs"])
    assert e.value.code == la.LA_ERR_INVALID_ARG
