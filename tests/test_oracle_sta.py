"""Pins of the oracle's static timing of the gate graph, critical-path counts and Alg. 1
division (Sec. III-A; Alg. 1 ordering), and of the synthetic timing graph.

- closed forms on hand-built chains and fan-ins (delays exact in single precision): arrival,
  required time and slack along the path, the latest input on a gate, the lowest sink on a tie;
- a pure-Python enumeration of every path on small random graphs (integer-valued delays, so the
  single-precision sums are exact): the latest arrival at every output, the slack at every sink
  (the least over the paths through it) and the nets of each output's top-1 critical path;
- the division and partition rules on hand-made counts and slacks;
- the generator's graph: every edge goes one level up, sinks in node order, outputs at the top."""
import numpy as np

import gen
import oracle
from helpers import make_instance


def _chain_instance(n_nets, sinks_per_net=1, X=64, Y=8):
    # net i: driver at (4 i, 0), sinks at (4 i + 1 + j, 0)
    nets = []
    for i in range(n_nets):
        nodes = [(4 * i, 0, -1, "driver")] + [(4 * i + 1 + j, 0, j, "sink") for j in range(sinks_per_net)]
        nets.append((nodes, [[] for _ in nodes]))
    return make_instance(nets, X=X, Y=Y)


def test_chain_closed_form():
    inst = _chain_instance(3)
    T = oracle.Tree(inst)
    # net 0 -> net 1 -> net 2 -> output; gate delays 10, 12.5, 20 ps; wire delays 1.5, 2.25, 3.75 ps
    nxt = np.array([1, 2, -1], np.int32)
    gd = np.array([10000, 12500, 20000], np.int32)
    d = np.array([1.5, 2.25, 3.75], np.float32)
    arr = 10 + 1.5 + 12.5 + 2.25 + 20 + 3.75
    for clock, crit in ((60000, [0, 0, 0]), (40000, [1, 1, 1])):
        sl, cr, wns = oracle.sta(T, nxt, gd, clock, d)
        assert wns == clock / 1000.0 - arr
        assert np.all(sl == np.float32(wns))          # slack is the same along the one path
        assert cr.tolist() == crit


def test_latest_input_and_tie():
    # nets 0 and 1 feed net 2's gate; net 2's sink is the output
    inst = _chain_instance(3)
    T = oracle.Tree(inst)
    nxt = np.array([2, 2, -1], np.int32)
    gd = np.array([10000, 10000, 5000], np.int32)
    for d0, d1, path in ((4.0, 2.0, [1, 0, 1]), (2.0, 4.0, [0, 1, 1]), (3.0, 3.0, [1, 0, 1])):
        d = np.array([d0, d1, 1.0], np.float32)
        sl, cr, wns = oracle.sta(T, nxt, gd, 1000, d)
        assert wns == 1.0 - (10.0 + max(d0, d1) + 5.0 + 1.0)
        assert cr.tolist() == path                    # on a tie the lower sink (net 0's) is taken
        # the other input's slack is its margin: later by |d0 - d1|
        assert sl[0] == np.float32(wns + (max(d0, d1) - d0))
        assert sl[1] == np.float32(wns + (max(d0, d1) - d1))


def _brute(T, nxt, gd_fs, clock_fs, d):
    # every path of gates: (sinks in order) from a net with no fan-in to an output sink
    nets = T.nets
    sink_net = np.searchsorted(T.net_ptr, T.sink_node, side="right") - 1
    sinks_of = [[] for _ in range(nets)]
    for k in range(T.sinks):
        sinks_of[sink_net[k]].append(k)
    fanin = [[] for _ in range(nets)]
    for k in range(T.sinks):
        if nxt[k] >= 0:
            fanin[nxt[k]].append(k)
    gd = [g / 1000.0 for g in gd_fs]
    paths = []   # (net list, sink list)

    def walk(n, nl, sl):
        for k in sinks_of[n]:
            if nxt[k] < 0:
                paths.append((nl + [n], sl + [k]))
            else:
                walk(int(nxt[k]), nl + [n], sl + [k])
    for n in range(nets):
        if not fanin[n]:
            walk(n, [], [])
    clock = clock_fs / 1000.0
    arr_out = {}
    best_path = {}
    slack = [np.inf] * T.sinks
    for nl, sl in paths:
        t = 0.0
        at_sink = []
        for n, k in zip(nl, sl):
            t += gd[n] + float(d[k])
            at_sink.append(t)
        e = sl[-1]
        if e not in arr_out or t > arr_out[e]:
            arr_out[e] = t
        # slack at each sink on the path: required along this path minus arrival along it is
        # clock - total; the sink's slack is the least over the paths through it ... of
        # (required - latest arrival); with exact sums: clock - (longest path through the sink)
    # longest path through each sink = latest arrival at it + longest tail after it
    longest_to = {}
    for nl, sl in paths:
        t = 0.0
        for n, k in zip(nl, sl):
            t += gd[n] + float(d[k])
            longest_to[k] = max(longest_to.get(k, -np.inf), t)
    tail = {}
    for nl, sl in paths:
        tot = sum(gd[n] + float(d[k]) for n, k in zip(nl, sl))
        t = 0.0
        for n, k in zip(nl, sl):
            t += gd[n] + float(d[k])
            tail[k] = max(tail.get(k, -np.inf), tot - t)
    for k in longest_to:
        slack[k] = clock - (longest_to[k] + tail[k])
    return arr_out, slack, sink_net, fanin, sinks_of, longest_to


def test_paths_enumerated_on_small_random_graphs():
    for seed in range(5):
        inst = gen.generate(120, 40, 40, 8, 300 + seed)
        tg = gen.timing_graph(inst, levels=5, po_frac=0.3, seed=seed)
        T = oracle.Tree(inst)
        rng = np.random.default_rng(seed)
        d = rng.integers(1, 64, T.sinks).astype(np.float32) / 8.0     # exact in single precision
        gd = (rng.integers(8, 24, T.nets) * 1000).astype(np.int32)
        nxt = tg["sink_next"]
        arr_out, slack_bf, sink_net, fanin, sinks_of, longest_to = _brute(T, nxt, gd, 60000, d)
        sl, cr, wns = oracle.sta(T, nxt, gd, 60000, d)
        outs = np.nonzero(nxt < 0)[0]
        assert wns == min(60.0 - arr_out[e] for e in outs)
        for k in range(T.sinks):
            assert sl[k] == np.float32(slack_bf[k]), (seed, k)
        # top-1 critical path of every violating output below 0.7 WNS: follow the latest input
        # (lowest sink on ties) from the brute-force arrivals
        exp = np.zeros(T.nets, np.int64)
        if wns < 0:
            for e in outs:
                if not sl[e] < np.float32(0.7) * np.float32(wns):
                    continue
                n = sink_net[e]
                while True:
                    exp[n] += 1
                    if not fanin[n]:
                        break
                    best = max(fanin[n], key=lambda k: (longest_to[k], -k))
                    n = sink_net[best]
        assert np.array_equal(cr, exp), seed


def test_division_and_partition():
    # 8 nets, one sink each; counts and slacks set by hand, WNS = -100
    inst = _chain_instance(8)
    T = oracle.Tree(inst)
    crit = np.array([40, 20, 19, 10, 4, 3, 0, 0], np.int32)
    slack = np.array([-100, -100, -100, -100, -100, -100, -75, -60], np.float32)
    sub, n = oracle.alg1_subsets(T, slack, crit, -100.0)
    # critical (count > 3): C = 40 -> [40] 0, [20, 40) 1, [10, 20) 2, [5, 10) 3, [2.5, 5) 4: kc = 5
    assert n == 5 + 8
    assert sub[:5].tolist() == [0, 1, 2, 2, 4]
    # semi-critical: net 5 (3 paths, slack = WNS: rho 1 -> first bin), net 6 (rho 0.75 -> bin 5)
    assert sub[5] == 5 + 0 and sub[6] == 5 + 5
    # net 7 (slack -60, rho 0.6) is above 0.7 WNS: the non-critical subset, last
    assert sub[7] == 5 + 7
    # no violation: no critical or semi-critical subset is used
    sub, n = oracle.alg1_subsets(T, np.full(8, 5.0, np.float32), np.zeros(8, np.int32), 5.0)
    assert n == 8 and np.all(sub == 7)


def test_generated_graph_structure():
    inst = gen.config(4, num_nets=20000)
    tg = gen.timing_graph(inst)
    lvl, nxt = tg["net_level"], tg["sink_next"]
    flags = inst.node_flags
    sink_net = np.repeat(np.arange(inst.num_nets), np.diff(inst.net_node_ptr))[(flags & 1) != 0]
    assert len(nxt) == int(np.count_nonzero(flags & 1))
    fed = nxt >= 0
    assert np.all(lvl[nxt[fed]] == lvl[sink_net[fed]] + 1)             # one level up: acyclic
    assert np.all(nxt[lvl[sink_net] == tg["levels"] - 1] == -1)         # the top level only outputs
    assert 0.15 < np.mean(~fed) < 0.3
    assert tg["gate_delay_fs"].min() >= 8000 and tg["gate_delay_fs"].max() <= 25000
