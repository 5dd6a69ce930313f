"""Pins of the oracle's quality terms (Sec. II, Eq. 1-3): closed forms of the Eq. 3 and Eq. 2
totals on constructed demand maps, and the via count and wire capacitance of an assignment
against two other derivations (the objective's via and capacitance terms, and the RC model)."""
import math

import numpy as np
import pytest

import gen
import oracle


@pytest.fixture(scope="module")
def small():
    inst = gen.config(1, num_nets=60)
    return inst, oracle.Tree(inst)


def _layers(T):
    z = np.zeros(T.nodes, np.uint8)
    return z, z, z


def test_eq3_at_capacity_is_the_weight_sum(small):
    inst, T = small
    ofw = np.linspace(0.5, 2.0, inst.L)
    D = inst.caps.astype(np.int32)
    q = oracle.quality(T, *_layers(T), D, ofw)
    # e^0 on every edge: X * Y edges per layer, each weighted by its layer's ofw
    assert q["tof"] == pytest.approx(inst.X * inst.Y * ofw.sum(), rel=1e-12)
    assert q["overflow_sum"] == 0 and q["overflow_edges"] == 0


def test_eq3_slope_depends_on_zero_capacity(small):
    inst, T = small
    caps = inst.caps.astype(np.int64)
    for k in (2, -3):
        D = (caps + k).astype(np.int32)
        q = oracle.quality(T, *_layers(T), D)
        zero = (caps == 0).reshape(-1, inst.L)
        n_zero, n_pos = int(zero.sum()), int((~zero).sum())
        # s = 1.5 on edges without capacity, 0.5 elsewhere
        want = n_pos * math.exp(0.5 * k) + n_zero * math.exp(1.5 * k)
        assert q["tof"] == pytest.approx(want, rel=1e-12)
        if k > 0:
            assert q["overflow_sum"] == k * caps.size and q["overflow_edges"] == caps.size
        else:
            assert q["overflow_sum"] == 0 and q["overflow_edges"] == 0


def test_eq2_counts_only_the_excess():
    inst = gen.config(1, num_nets=10)
    T = oracle.Tree(inst)
    caps = inst.caps.astype(np.int64).reshape(-1)
    rng = np.random.default_rng(4)
    D = caps + rng.integers(-4, 5, caps.size)
    D = np.maximum(D, 0).astype(np.int32)
    q = oracle.quality(T, *_layers(T), D)
    excess = [int(d) - int(c) for d, c in zip(D.tolist(), caps.tolist()) if d > c]
    assert q["overflow_sum"] == sum(excess) and q["overflow_edges"] == len(excess)


def test_vias_and_capacitance_of_an_assignment(small):
    inst, T = small
    P = oracle.Params(T)
    st = oracle.State(T)
    lay, vlo, vhi, _ = oracle.assign(T, P, st, rounds=2)
    q = oracle.quality(T, lay, vlo, vhi, st.D)
    # the objective with only the via weight counts the span of each node's layers
    Pv = oracle.Params(T, w_cong=0, w_cap=0, w_d=0, w_via=1)
    assert q["vias"] == int(oracle.objective(T, Pv, lay, st.D).sum())
    # the objective with only the capacitance weight sums c(layer) * len
    Pc = oracle.Params(T, w_cong=0, w_cap=1, w_d=0, w_via=0)
    assert q["wire_cap_af"] == int(oracle.objective(T, Pc, lay, st.D).sum())
    # the RC model's tree-segment capacitances (fF) add up to the same total
    R, C = oracle.rc(T, P, lay)
    nonroot = T.parent >= 0
    assert float(np.asarray(C)[:T.nodes][nonroot].sum()) * 1000.0 == pytest.approx(q["wire_cap_af"], rel=1e-9)
    # demand after the rounds: every GCell edge a segment covers holds one unit per segment
    lens = np.asarray(T.len)[nonroot]
    assert int(st.D.sum()) == int(lens.sum())


def test_eq3_far_outside_the_tabulated_range():
    # one edge 195 over a capacity of 5 (slope 0.5) and one 150 over a capacity of 0 (slope 1.5),
    # every other edge empty at capacity 40: closed form of the Eq. 3 total
    from helpers import make_instance
    X, Y, L = 6, 5, 2
    caps = np.full((Y, X, L), 40, np.uint8)
    caps[1, 2, 0] = 5
    caps[3, 4, 1] = 0
    inst = make_instance([([(0, 0, -1, "driver"), (3, 0, 0, "sink")], None)], X=X, Y=Y, L=L, caps=caps)
    T = oracle.Tree(inst)
    D = np.zeros((Y, X, L), np.int32)
    D[1, 2, 0] = 200
    D[3, 4, 1] = 150
    q = oracle.quality(T, *_layers(T), D.reshape(-1))
    want = (X * Y * L - 2) * math.exp(-20.0) + math.exp(0.5 * 195) + math.exp(1.5 * 150)
    assert q["tof"] == pytest.approx(want, rel=1e-12)
    assert q["overflow_sum"] == 195 + 150 and q["overflow_edges"] == 2
