"""The largest workload at full size: 12,000,000 nets on 2048x2048 GCells x 12 layers plus 120
nets of 1,000-4,000 pins (which take the big-net path of the batched form).  Pre-assignment
Elmore delays of sampled nets against the oracle; one batched round from the empty demand map,
checked net by net on a sample holding every huge net; the demand and history maps against a
recount of the assigned layers."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, host, oracle_assign, say
from test_gpu_assign import _subset

pytestmark = pytest.mark.gpu

REL = 1e-5


def test_config5_full_size_sampled():
    inst = gen.config(5)
    sizes = np.diff(inst.net_node_ptr)
    huge = np.nonzero(sizes > 1000)[0]
    say("c5: %d nets, %d input nodes, %d nets of more than 1000 pins" % (inst.num_nets, inst.num_nodes, huge.size))
    assert huge.size == 120
    T = oracle.Tree(inst)
    g = DeviceRun(inst)
    assert g.b.nodes == T.nodes and g.b.sinks == T.sinks
    say("c5 batch: %d LA nodes, %d sinks, %d levels" % (g.b.nodes, g.b.sinks, g.b.levels))

    rng = np.random.default_rng(5)
    nets = np.unique(np.concatenate([huge, rng.choice(inst.num_nets, 1500, replace=False)]))
    sub = _subset(inst, nets)
    nidx = np.concatenate([np.arange(T.net_ptr[i], T.net_ptr[i + 1]) for i in nets])
    sidx = np.nonzero(np.isin(T.sink_node, nidx))[0]

    # Elmore with the average per-direction R and C (before any assignment)
    Ts = oracle.Tree(sub)
    R, C = oracle.rc(Ts, oracle.Params(Ts), None)
    _, _, d_o = oracle.elmore(Ts, R, C)
    d_g = host(g.elmore())[:T.sinks][sidx].astype(np.float64)
    err = np.abs(d_g - d_o)
    assert np.all(err <= REL * np.abs(d_o) + 1e-30), "delay: worst rel %g" % (err / np.abs(d_o)).max()

    # one round in one batch: every net meets the empty map, so each sampled net stands alone
    sw = gen.synthetic_weights(T.nodes, T.sinks, T.nets, seed=13)
    res = g.assign(sw["seg_w_q10"], sw["pin_w_q10"], sw["lambda_mohm"], None, rounds=1, form=la.LA_FORM_BATCHED)
    o = oracle_assign(sub, sw["seg_w_q10"][nidx], sw["pin_w_q10"][sidx], sw["lambda_mohm"][nidx], None, rounds=1)
    nonroot_s = o["tree"].parent >= 0
    for k in ("layers", "vlo", "vhi"):
        gv, ov = res[k][nidx], o[k]
        if k == "layers":
            gv, ov = np.where(nonroot_s, gv, 0), np.where(nonroot_s, ov, 0)
        bad = np.nonzero(gv != ov)[0]
        assert bad.size == 0, "%s differs at %d sampled nodes" % (k, bad.size)

    # demand: per layer, the assigned wire length; history after the round: 64 per overflow unit
    nonroot = T.parent >= 0
    per_layer = np.bincount(res["layers"][nonroot], weights=T.len[nonroot], minlength=inst.L)
    D = res["D"].astype(np.int64)
    assert np.array_equal(D.reshape(-1, inst.L).sum(0), per_layer.astype(np.int64))
    over = np.maximum(D - inst.caps.reshape(-1).astype(np.int64), 0)
    assert np.array_equal(res["H"].astype(np.int64), np.minimum(64 * over, 1 << 24))
