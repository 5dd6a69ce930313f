"""Oracle: Elmore delay (Sec. II-C, Fig. rc) and its reverse sweep."""
import numpy as np
import pytest

import gen
import oracle
from helpers import golden, make_instance


def _chain(N, cpin_af):
    nodes = [(0, 0, -1, "driver")] + [(k, 0, k - 1, "steiner") for k in range(1, N)] + [(N, 0, N - 1, "sink")]
    return make_instance([(nodes, [[]] * (N + 1))], X=N + 2, Y=2, cpin_af=cpin_af)


@pytest.mark.parametrize("N,R,C,CL", [(7, 2.0, 3.0, 5.0), (1, 1.5, 0.25, 2.0), (40, 0.03, 0.2, 1.0)])
def test_rc_chain_closed_form(N, R, C, CL):
    # uniform chain of N pi-segments (R, C each) with load CL: t_end = N R CL + R C N^2 / 2
    T = oracle.Tree(_chain(N, int(round(CL * 1000))))
    Rv = np.full(T.nodes + T.sinks, R)
    Cv = np.full(T.nodes + T.sinks, C)
    Rv[0], Cv[0] = 0.0, 0.0           # no driver resistance in the textbook chain
    Rv[T.nodes:], Cv[T.nodes:] = 0.0, 0.0
    S, t, d = oracle.elmore(T, Rv, Cv)
    want = N * R * CL + R * C * N * N / 2
    assert d[0] == pytest.approx(want, rel=1e-13)
    if (N, R, C, CL) == (7, 2.0, 3.0, 5.0):
        assert d[0] == pytest.approx(217.0, rel=1e-13)


def test_paper_d34_relation():
    fx = golden("fig_rc_d34.json")
    par = fx["parent"]
    # nodes 3,4,5,6,7 laid out as 3->4 (H), 4->5 (V), 4->6 (H), 6->7 (V)
    nodes = [(0, 4, -1, "driver"), (3, 4, 0, "steiner"), (3, 7, 1, "sink"), (6, 4, 1, "steiner"), (6, 1, 3, "sink")]
    assert [n[2] for n in nodes] == par
    T = oracle.Tree(make_instance([(nodes, [[]] * 5)], X=8, Y=8, cpin_af=700))
    rng = np.random.default_rng(3)
    R = rng.uniform(0.1, 2.0, T.nodes + T.sinks)
    C = rng.uniform(0.1, 2.0, T.nodes + T.sinks)
    R[0] = 0.0
    C[0] = 0.0
    C[T.nodes:] = 0.0
    S, t, d = oracle.elmore(T, R, C)
    # pi-model node capacitances: half of every incident edge plus the pin load
    load = {2: 0.7, 4: 0.7}
    Cn = np.zeros(5)
    for v in range(1, 5):
        Cn[v] += C[v] / 2
        Cn[par[v]] += C[v] / 2
    for v, c in load.items():
        Cn[v] += c
    d34 = t[1] - t[0]
    assert d34 == pytest.approx(R[1] * (Cn[1] + Cn[2] + Cn[3] + Cn[4]), rel=1e-13)


def _path_sum_elmore(T, R, C, cpin):
    """Textbook Elmore: delay(k) = sum over RC edges e on the path to k of R_e * (C_e/2 + C below e)."""
    nodes = T.nodes
    ch = [[] for _ in range(nodes)]
    for v in range(nodes):
        if T.parent[v] >= 0:
            ch[T.parent[v]].append(v)
    sink_of = {int(v): k for k, v in enumerate(T.sink_node)}

    def below(v):  # all capacitance strictly below node v (edges and loads), by explicit enumeration
        tot, stack = 0.0, list(ch[v])
        if v in sink_of:
            tot += C[nodes + sink_of[v]] + cpin[v]
        while stack:
            u = stack.pop()
            tot += C[u]
            if u in sink_of:
                tot += C[nodes + sink_of[u]] + cpin[u]
            stack.extend(ch[u])
        return tot

    out = []
    for k, v in enumerate(T.sink_node):
        e = nodes + k
        dl = R[e] * (C[e] / 2 + cpin[v])
        u = int(v)
        while u >= 0:
            dl += R[u] * (C[u] / 2 + below(u))
            u = int(T.parent[u])
        out.append(dl)
    return np.array(out)


def test_elmore_equals_path_sum_definition():
    I = gen.generate(40, 32, 32, 8, 11, pin_max=7)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    lay = np.array([np.nonzero(I.layer_dir == max(d, 0))[0][-1] for d in T.dir], np.uint8)
    for layers in (None, lay):
        R, C = oracle.rc(T, P, layers)
        S, t, d = oracle.elmore(T, R, C)
        cpin = np.zeros(T.nodes)
        cpin[T.sink_node] = 1.0
        assert np.allclose(d, _path_sum_elmore(T, R, C, cpin), rtol=1e-12, atol=0)


def test_rc_of_assignment_follows_layer_table():
    # segment R = via from the parent's entering layer + wire; pin edge = via down to layer 0
    nodes = [(0, 0, -1, "driver"), (5, 0, 0, "steiner"), (5, 3, 1, "sink")]
    I = make_instance([(nodes, [[]] * 3)], X=8, Y=8, L=8)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    r, c, vr = I.r_mohm, I.c_af, I.via_r_mohm
    lay = np.array([0, 4, 3], np.uint8)
    R, C = oracle.rc(T, P, lay)
    assert R[1] == pytest.approx((vr[0] + vr[1] + vr[2] + vr[3] + 5 * r[4]) * 1e-6, rel=1e-15)
    assert R[2] == pytest.approx((vr[3] + 3 * r[3]) * 1e-6, rel=1e-15)
    assert R[T.nodes] == pytest.approx((vr[0] + vr[1] + vr[2]) * 1e-6, rel=1e-15)
    assert C[1] == pytest.approx(5 * c[4] * 1e-3) and C[2] == pytest.approx(3 * c[3] * 1e-3)
    assert R[0] == pytest.approx(1.0) and C[0] == 0.0
    # before assignment: average unit R/C per direction, zero-resistance pin edges
    R0, C0 = oracle.rc(T, P, None)
    assert R0[1] == pytest.approx(5 * (sum(r[0::2]) // 4) * 1e-6) and R0[T.nodes] == 0.0
    assert C0[2] == pytest.approx(3 * (sum(c[1::2]) // 4) * 1e-3)


def test_adjoint_matches_central_differences():
    I = gen.generate(60, 40, 40, 8, 21, pin_max=8, budget_min_fs=-40000, budget_max_fs=5000)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    lay = np.array([np.nonzero(I.layer_dir == max(d, 0))[0][min(1, 0)] for d in T.dir], np.uint8)
    R, C = oracle.rc(T, P, lay)
    S, t, d = oracle.elmore(T, R, C)
    rng = np.random.default_rng(5)
    gbar = -rng.uniform(0.0, 1.0, T.sinks)
    G, Sig, dR, dC = oracle.elmore_adjoint(T, R, C, S, gbar)
    sink_net = np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1
    h = 1e-3
    checked = 0
    for net in range(0, T.nets, 3):
        mine = np.nonzero(sink_net == net)[0]
        rc_idx = list(range(T.net_ptr[net], T.net_ptr[net + 1])) + [T.nodes + k for k in mine]
        for e in rc_idx:
            for arr, grad in ((R, dR), (C, dC)):
                x0 = arr[e]
                step = h * (abs(x0) if x0 != 0 else 1.0)
                arr[e] = x0 + step
                jp = float(gbar[mine] @ oracle.elmore(T, R, C)[2][mine])
                arr[e] = x0 - step
                jm = float(gbar[mine] @ oracle.elmore(T, R, C)[2][mine])
                arr[e] = x0
                fd = (jp - jm) / (2 * step)
                # J is linear in each single R and C, so the difference quotient is exact up to
                # the FP64 rounding of jp and jm
                floor = 16 * np.finfo(np.float64).eps * (abs(jp) + abs(jm)) / (2 * step)
                assert abs(fd - grad[e]) <= 1e-8 * abs(grad[e]) + floor
                checked += 1
    assert checked > 200
