"""Quality report (Sec. II, Eq. 1-3) of the HIP path against the oracle: the same assignment
problem is solved on both sides (bit-exact, checked elsewhere), then each side evaluates its
own result -- Eq. 3 and Eq. 2 totals, vias, wire capacitance, WNS, TNS and the Eq. 1 score."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, oracle_assign, say

pytestmark = pytest.mark.gpu

REL_T = 1e-5     # FP32 compensated timing against FP64
REL_TOF = 1e-12  # FP64 sums in different orders


def _check(inst, rounds, form, ofw, timing):
    T = oracle.Tree(inst)
    w = oracle.plain_weights(T, oracle.Params(T))
    g = DeviceRun(inst)
    g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=11, rounds=rounds, form=form)
    o = oracle_assign(inst, w["seg_w"], w["pin_w"], w["lam"], w["tier"], rounds=rounds)
    sw = {"w1": -3.0, "w2": -5.0, "w3": 0.25, "w4": 2.0, "r1": -1.0, "r2": -100.0, "r3": 10.0}
    dg = g.elmore() if timing else None
    q = la.la_quality_report(g.b, ofw=ofw, delay=dg, weights=sw if timing else None)
    qo = oracle.quality(T, o["layers"], o["vlo"], o["vhi"], o["D"], ofw)
    say("%s: gpu %s" % (inst.name, q))
    say("%s: oracle %s" % (inst.name, qo))
    for k in ("overflow_sum", "overflow_edges", "vias", "wire_cap_af"):
        assert q[k] == qo[k], k
    assert q["tof"] == pytest.approx(qo["tof"], rel=REL_TOF)
    if not timing:
        assert q["score"] == 0.0 and q["wns_ps"] == 0.0 and q["tns_ps"] == 0.0
        return
    R, C = oracle.rc(T, o["params"], o["layers"])
    _, _, d = oracle.elmore(T, R, C)
    sl = inst.net_budget_fs[np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1] * 1e-3 - d
    tns, wns = sl[sl < 0].sum(), sl.min()
    assert q["tns_ps"] == pytest.approx(tns, rel=REL_T)
    assert q["wns_ps"] == pytest.approx(wns, rel=REL_T, abs=1e-3)
    score = (sw["w1"] * (wns - sw["r1"]) + sw["w2"] * (tns - sw["r2"]) / T.sinks +
             sw["w3"] * (qo["wire_cap_af"] / 1000.0 - sw["r3"]) + sw["w4"] * qo["tof"])
    assert q["score"] == pytest.approx(score, rel=REL_T)


@pytest.mark.parametrize("form", [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED])
def test_quality_c1(form):
    inst = gen.config(1)
    _check(inst, 3, form, np.linspace(0.5, 3.0, inst.L), True)


def test_quality_c2_no_timing():
    _check(gen.config(2), 2, la.LA_FORM_BATCHED, None, False)


def test_quality_empty_demand():
    # before any assignment: zero demand, so every edge gives ofw e^{-s c}
    inst = gen.config(1, num_nets=40)
    g = DeviceRun(inst)
    q = la.la_quality_report(g.b)
    T = oracle.Tree(inst)
    z = np.zeros(T.nodes, np.uint8)
    qo = oracle.quality(T, z, z, z, np.zeros(inst.X * inst.Y * inst.L, np.int32))
    assert q["tof"] == pytest.approx(qo["tof"], rel=REL_TOF)
    assert q["overflow_sum"] == 0 and q["vias"] == 0 and q["wire_cap_af"] == qo["wire_cap_af"]


def test_quality_min_layer():
    # layers below min_layer are not routable: their edges sit in planes of their own
    from helpers import make_instance
    from test_gpu_assign import _star
    inst = make_instance([_star(5), _star(3)], X=24, Y=24, L=8,
                         caps=np.random.default_rng(2).integers(0, 3, (24, 24, 8)).astype(np.uint8))
    T = oracle.Tree(inst)
    rng = np.random.default_rng(5)
    sw = rng.integers(0, 1025, T.nodes)
    pw = rng.integers(0, 1025, max(T.sinks, 1))
    lam = rng.integers(0, 500000, T.nodes)
    o = oracle_assign(inst, sw, pw, lam, None, rounds=2, min_layer=2)
    g = DeviceRun(inst, min_layer=2)
    g.assign(sw, pw, lam, None, rounds=2, form=la.LA_FORM_BATCHED)
    ofw = np.linspace(1.0, 2.0, inst.L)
    q = la.la_quality_report(g.b, ofw=ofw)
    qo = oracle.quality(T, o["layers"], o["vlo"], o["vhi"], o["D"], ofw)
    for k in ("overflow_sum", "overflow_edges", "vias", "wire_cap_af"):
        assert q[k] == qo[k], k
    assert q["tof"] == pytest.approx(qo["tof"], rel=REL_TOF)


@pytest.mark.parametrize("form", [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED])
def test_quality_large_excess(form):
    # excesses far outside the tabulated [-64, 64]: 200 two-pin nets stacked on one row whose only
    # horizontal layer has capacity 5 (over = 195, factor 0.5), 150 on a row of capacity 0
    # (over = 150, factor 1.5); both sides evaluate e^{s x} directly there
    from helpers import make_instance
    X, Y, L = 24, 12, 2
    caps = np.full((Y, X, L), 40, np.uint8)
    caps[5, :, 0] = 5
    caps[7, :, 0] = 0
    nets = [([(2, 5, -1, "driver"), (20, 5, 0, "sink")], None)] * 200 + \
           [([(3, 7, -1, "driver"), (18, 7, 0, "sink")], None)] * 150
    inst = make_instance(nets, X=X, Y=Y, L=L, caps=caps)
    _check(inst, 2, form, None, False)
