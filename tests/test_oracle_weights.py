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
