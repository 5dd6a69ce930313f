"""Oracle: Eq. 4 pin weights, Eq. 5 edge weights, look-ahead coefficients, Alg. 1 slack bins."""
import numpy as np
import pytest

import gen
import oracle
from helpers import golden, make_instance


def _two_sink_net(budget_fs):
    nodes = [(0, 4, -1, "driver"), (4, 4, 0, "steiner"), (4, 8, 1, "sink"), (8, 4, 1, "sink")]
    return make_instance([(nodes, [[]] * 4)], X=12, Y=12, budget_fs=[budget_fs])


def test_eq4_logistic_values():
    fx = golden("eq4_logistic.json")
    T = oracle.Tree(_two_sink_net(0))
    for v in fx["values"]:
        # WNS = -100 ps (sink 1), sink 0 at rho * WNS
        delay = np.array([100.0 * v["rho"], 100.0])
        sl, wns, pw, tier = oracle.slack(T, delay)
        assert wns == pytest.approx(-100.0)
        assert int(pw[0]) == v["q10"]


def test_paper_weighting_example_and_eq5():
    fx = golden("eq4_logistic.json")["weighting_example"]
    T = oracle.Tree(_two_sink_net(0))
    delay = -np.array(fx["slack_ps"])
    sl, wns, pw, tier = oracle.slack(T, delay)
    assert pw.tolist() == fx["q10"] and pw[1] > pw[0]
    P = oracle.Params(T)
    sw, lam = oracle.edge_weights(T, P, pw)
    # edge into the Steiner node carries the worse sink; each sink edge its own weight
    assert sw[1] == max(fx["q10"]) and sw[2] == fx["q10"][0] and sw[3] == fx["q10"][1]
    assert lam[1] == 0   # nothing upstream of the driver's own segment


def test_no_violation_means_zero_weights():
    T = oracle.Tree(_two_sink_net(10**6))
    sl, wns, pw, tier = oracle.slack(T, np.array([1.0, 2.0]))
    assert wns > 0 and (pw == 0).all() and tier[0] == 7


def test_eq5_max_over_downstream_sinks_and_lambda():
    I = gen.generate(200, 40, 40, 8, 31, pin_max=8)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    rng = np.random.default_rng(1)
    pw = rng.integers(0, 1025, T.sinks).astype(np.uint16)
    sw, lam = oracle.edge_weights(T, P, pw)
    sink_of = {int(v): k for k, v in enumerate(T.sink_node)}
    ch = [[] for _ in range(T.nodes)]
    for v in range(T.nodes):
        if T.parent[v] >= 0:
            ch[T.parent[v]].append(v)
    ravg = [sum(I.r_mohm[0::2]) // 4, sum(I.r_mohm[1::2]) // 4]
    for v in range(T.nodes):
        stack, best = [v], 0
        while stack:
            u = stack.pop()
            if u in sink_of:
                best = max(best, int(pw[sink_of[u]]))
            stack.extend(ch[u])
        assert sw[v] == best
        # r_est: average-R wire from the driver down to the segment's upper end
        rest, u = 0, int(T.parent[v])
        while u >= 0 and T.parent[u] >= 0:
            rest += ravg[T.dir[u]] * int(T.len[u])
            u = int(T.parent[u])
        assert lam[v] == ((int(sw[v]) * rest) >> 10 if T.parent[v] >= 0 else 0)


def test_alg1_slack_bins():
    fx = golden("alg1_slack_bins.json")
    cases = fx["cases"]
    nets = []
    for c in cases:
        nets.append(([(0, 0, -1, "driver"), (2, 0, 0, "sink")], [[], []]))
    budgets = [int(round(c["net_slack_ps"] * 1000)) for c in cases]
    T = oracle.Tree(make_instance(nets, X=4, Y=4, budget_fs=budgets))
    sl, wns, pw, tier = oracle.slack(T, np.zeros(T.sinks))
    assert wns == pytest.approx(fx["wns_ps"])
    assert tier.tolist() == [c["tier"] for c in cases]


def test_adjoint_weights_bound_eq5():
    # -G(s) sums the weights of the violating sinks below s, so it is at least their maximum
    I = gen.generate(150, 40, 40, 8, 41, pin_max=8, budget_min_fs=-60000, budget_max_fs=20000)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    w = oracle.adjoint_form_weights(T, P, None)
    viol = w["slack"] < 0
    omega = np.where(viol, w["pin_w"], 0)
    ch = [[] for _ in range(T.nodes)]
    for v in range(T.nodes):
        if T.parent[v] >= 0:
            ch[T.parent[v]].append(v)
    sink_of = {int(v): k for k, v in enumerate(T.sink_node)}
    for v in range(T.nodes):
        stack, mx = [v], 0
        while stack:
            u = stack.pop()
            if u in sink_of:
                mx = max(mx, int(omega[sink_of[u]]))
            stack.extend(ch[u])
        assert w["seg_w"][v] >= mx - 1
    assert (w["lam"] >= 0).all()


def _chain_net(budget_fs):
    # driver -H(4)-> A -V(5)-> B -H(5)-> sink: one sink, so every edge above it carries its weight
    nodes = [(0, 0, -1, "driver"), (4, 0, 0, "steiner"), (4, 5, 1, "steiner"), (9, 5, 2, "sink")]
    return make_instance([(nodes, [[]] * 4)], X=12, Y=8, L=8, budget_fs=[budget_fs])


@pytest.mark.parametrize("assigned", [False, True])
def test_adjoint_weights_closed_form_on_a_chain(assigned):
    # One violating sink of weight w (its Eq. 4 weight, slack = WNS so rho = 1).  With
    # J = w min(0, slack): dJ/d delay = -w, G = -w on every edge above the sink, and
    # Sig(v) = -w * (resistance from the driver down to v, R_drv included).  The adjoint form
    # quantises seg_w = pin_w = rne(1024 w) (= the Q10 weight itself) and
    # lambda_s = rne(1e6 w R_up(parent(s))) with R_up in kOhm, i.e. weighted mOhm.
    I = _chain_net(-400000)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    L = I.L
    lay = np.array([0, 2, 3, 4], np.uint8) if assigned else None
    out = oracle.adjoint_form_weights(T, P, lay)
    assert out["slack"][0] < 0
    q = int(golden("eq4_logistic.json")["values"][0]["q10"])   # rho = 1
    w = q / 1024.0
    assert out["pin_w"].tolist() == [q]
    assert out["seg_w"].tolist() == [q, q, q, q]
    # resistance of each RC edge, recomputed from the layer table (mOhm)
    r, vr = [int(v) for v in I.r_mohm], [int(v) for v in I.via_r_mohm]
    lens = [0, 4, 5, 5]
    if assigned:
        lays = [0, 2, 3, 4]
        ent = [0, 0, 2, 3]                     # entering layer of each segment's upper node
        Rm = [1000000] + [sum(vr[min(ent[v], lays[v]):max(ent[v], lays[v])]) + r[lays[v]] * lens[v]
                          for v in range(1, 4)]
    else:
        ravg = [sum(r[0::2]) // (L // 2), sum(r[1::2]) // (L // 2)]
        Rm = [1000000, ravg[0] * 4, ravg[1] * 5, ravg[0] * 5]
    up = np.cumsum(Rm)                          # R from the driver through edge v (mOhm)
    want = [0] + [int(np.rint(1e6 * w * up[v - 1] * 1e-6)) for v in range(1, 4)]
    assert out["lam"].tolist() == want
    # and G, Sig themselves
    assert np.allclose(out["G"], -w, rtol=0, atol=1e-15)
    assert np.allclose(out["Sig"], -w * up * 1e-6, rtol=1e-13)


def test_adjoint_weights_quantisation_rounds_half_even_and_clamps():
    # seg_w and pin_w clamp at 1024 and round half to even; lambda clamps at 0 and 2^31 - 1
    I = _chain_net(-400000)
    T = oracle.Tree(I)
    G = np.array([-1.5, -(700.5 / 1024), -(701.5 / 1024), 0.25])
    Sig = np.array([-3000.0, -(12.5e-6), -(13.5e-6), 5.0])
    gbar = np.array([-(11.5 / 1024)])
    sw, pw, lam = oracle.adjoint_weights(T, G, Sig, gbar)
    assert sw.tolist() == [1024, 700, 702, 0]
    assert pw.tolist() == [12]
    assert lam.tolist() == [0, 2147483647, 12, 14]
