"""Oracle: the layer-assignment directed tree (Sec. III-B)."""
import numpy as np
import pytest

import gen
import oracle
from helpers import fixture_nets, golden, make_instance


def test_fig_graph_node_counts():
    fx = golden("fig_graph_tree.json")
    I = make_instance(fixture_nets(fx), X=fx["grid"][0], Y=fx["grid"][1])
    T = oracle.Tree(I)
    assert np.diff(T.net_ptr).tolist() == [n["expected_nodes"] for n in fx["nets"]]
    # the added node sits at the bend and splits 4->7 into two straight segments
    b = T.net_ptr[1]
    bend = T.net_ptr[2] - 1
    assert (T.x[bend], T.y[bend]) == (10, 8)
    assert T.parent[bend] == b + 1 and T.parent[b + 3] == bend


def _polyline_edges(pts):
    s = set()
    for (x0, y0), (x1, y1) in zip(pts[:-1], pts[1:]):
        if y0 == y1:
            for x in range(min(x0, x1), max(x0, x1)):
                s.add((0, x, y0))
        else:
            for y in range(min(y0, y1), max(y0, y1)):
                s.add((1, x0, y))
    return s


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_segments_straight_and_projection_kept(seed):
    I = gen.generate(300, 48, 40, 8, seed, pin_max=9)
    T = oracle.Tree(I)
    assert T.nets == I.num_nets
    nonroot = T.parent >= 0
    p = T.parent[nonroot]
    x, y, px, py = T.x[nonroot], T.y[nonroot], T.x[p], T.y[p]
    assert ((x == px) | (y == py)).all()
    assert (T.len[nonroot] == np.abs(x - px) + np.abs(y - py)).all() and (T.len[nonroot] >= 1).all()
    assert (T.dir[nonroot] == np.where(y == py, 0, 1)).all()
    # per net: the GCell edges covered by the LA segments equal those of the input polylines
    for i in range(0, I.num_nets, 7):
        b0, b1 = I.net_node_ptr[i], I.net_node_ptr[i + 1]
        want = set()
        for v in range(b0 + 1, b1):
            u = b0 + I.node_parent[v]
            pts = [(int(I.node_x[u]), int(I.node_y[u]))]
            pts += list(zip(I.wp_x[I.edge_wp_ptr[v]:I.edge_wp_ptr[v + 1]].tolist(),
                            I.wp_y[I.edge_wp_ptr[v]:I.edge_wp_ptr[v + 1]].tolist()))
            pts.append((int(I.node_x[v]), int(I.node_y[v])))
            want |= _polyline_edges(pts)
        got = set()
        for v in range(T.net_ptr[i], T.net_ptr[i + 1]):
            if T.parent[v] >= 0:
                got |= _polyline_edges([(int(T.x[T.parent[v]]), int(T.y[T.parent[v]])), (int(T.x[v]), int(T.y[v]))])
        assert got == want
    # one node per bend of the input
    assert T.nodes == I.num_nodes + len(I.wp_x)


def _one(nodes, wps, X=8, Y=8):
    return make_instance([(nodes, wps)], X=X, Y=Y)


@pytest.mark.parametrize("case", ["diagonal", "zero_length", "cycle", "two_drivers", "off_grid", "reversal",
                                  "driver_not_first"])
def test_bad_trees_rejected(case):
    if case == "diagonal":
        I = _one([(0, 0, -1, "driver"), (3, 2, 0, "sink")], [[], []])
    elif case == "zero_length":
        I = _one([(1, 1, -1, "driver"), (1, 1, 0, "sink")], [[], []])
    elif case == "cycle":
        I = _one([(0, 0, -1, "driver"), (2, 0, 2, "steiner"), (4, 0, 1, "sink")], [[], [], []])
    elif case == "two_drivers":
        I = _one([(0, 0, -1, "driver"), (2, 0, 0, "driver")], [[], []])
    elif case == "off_grid":
        I = _one([(0, 0, -1, "driver"), (9, 0, 0, "sink")], [[], []])
    elif case == "reversal":
        I = _one([(0, 0, -1, "driver"), (2, 0, 0, "sink")], [[], [(5, 0)]])
    else:
        I = _one([(2, 0, 1, "sink"), (0, 0, -1, "driver")], [[], []])
    with pytest.raises(oracle.OracleError) as e:
        oracle.Tree(I)
    assert e.value.code == oracle.ERR_BAD_TREE


def test_collinear_waypoints_merge_and_node_order():
    # waypoints on a straight run add no node; a corner adds exactly one
    I = _one([(0, 0, -1, "driver"), (6, 3, 0, "sink")], [[], [(2, 0), (4, 0), (6, 0), (6, 1)]], X=8, Y=8)
    T = oracle.Tree(I)
    assert T.nodes == 3
    assert (T.x[2], T.y[2]) == (6, 0) and T.len.tolist() == [0, 3, 6]
