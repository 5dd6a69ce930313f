"""Oracle: congestion cost (Eq. 3), tree DP with look-ahead and trace-back (Alg. 2-4), batch schedule.

The DP is pinned against a brute-force minimum over every layer combination
where the method is exact (W_d = 0, or one unit C on every layer), against its
own objective J for any weights, and J itself is pinned term by term against
quantities computed independently (Elmore RC, Eq. 3 overflow, via hulls and
wire capacitance recounted from the assignment)."""
import math

import numpy as np
import pytest

import gen
import oracle
from helpers import golden, make_instance, recount_demand


def test_eq3_marginal_cost_table():
    fx = golden("eq3_lut.json")
    lut = oracle.cong_lut(8)
    for v in fx["values"]:
        assert lut[3, 1 if v["cap_zero"] else 0, v["delta"] + 32] == v["cost"]
    assert (np.diff(lut[:, 0, :], axis=1) >= 0).all() and (np.diff(lut[:, 1, :], axis=1) >= 0).all()


def _small(seed, L=8, pin_max=4, X=24, Y=24, nets=40):
    I = gen.generate(nets, X, Y, L, seed, pin_max=pin_max)
    rng = np.random.default_rng(seed)
    I.caps = rng.integers(0, 6, I.caps.shape).astype(np.uint8)
    return I, rng


def _rand_params(T, rng, w_cong=1000, w_cap=100, w_d=1, w_via=100000, lam=True):
    sw = rng.integers(0, 1025, T.nodes).astype(np.uint16)
    pw = rng.integers(0, 1025, max(T.sinks, 1)).astype(np.uint16)
    la = rng.integers(0, 3_000_000, T.nodes).astype(np.int32) if lam else np.zeros(T.nodes, np.int32)
    return oracle.Params(T, seg_w=sw, pin_w=pw, lam=la, w_cong=w_cong, w_cap=w_cap, w_d=w_d, w_via=w_via)


def _run_dp(T, P, D=None, H=None):
    st = oracle.State(T, H)
    if D is not None:
        st.D[:] = D
    lay, vlo, vhi, froot = oracle.assign(T, P, st, None, rounds=1)
    return lay, vlo, vhi, froot


def _check_against_bruteforce(T, P, D, H, exact):
    lay, vlo, vhi, froot = _run_dp(T, P, D, H)
    J = oracle.objective(T, P, lay, D, H)
    assert (froot == J).all(), "F_root must equal J of the traced assignment"
    n_checked = 0
    for net in range(T.nets):
        if T.net_ptr[net + 1] - T.net_ptr[net] - 1 > 6:
            continue
        jmin, best, nmin = oracle.bruteforce(T, P, net, D, H)
        assert froot[net] >= jmin
        if exact:
            assert froot[net] == jmin
            if nmin == 1:
                b0 = T.net_ptr[net]
                got = lay[b0:T.net_ptr[net + 1]].copy()
                got[0] = 0
                assert got.tolist() == best.tolist()
        n_checked += 1
    assert n_checked >= 10


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_dp_exact_without_delay_weight(seed):
    I, rng = _small(seed)
    T = oracle.Tree(I)
    P = _rand_params(T, rng, w_d=0, w_via=int(rng.integers(1, 200000)))
    D = rng.integers(0, 9, T.num_edges).astype(np.int32)
    H = rng.integers(0, 5000, T.num_edges).astype(np.int32)
    _check_against_bruteforce(T, P, D, H, exact=True)


@pytest.mark.parametrize("seed", [5, 6])
def test_dp_exact_with_uniform_unit_capacitance(seed):
    I, rng = _small(seed)
    I.c_af = np.full(I.L, 120, np.int32)
    T = oracle.Tree(I)
    P = _rand_params(T, rng, w_d=int(rng.integers(1, 4)))
    D = rng.integers(0, 9, T.num_edges).astype(np.int32)
    _check_against_bruteforce(T, P, D, None, exact=True)


@pytest.mark.parametrize("seed", [7, 8])
def test_dp_exact_at_twelve_layers(seed):
    I, rng = _small(seed, L=12, pin_max=3, nets=16)
    T = oracle.Tree(I)
    P = _rand_params(T, rng, w_d=0)
    D = rng.integers(0, 9, T.num_edges).astype(np.int32)
    _check_against_bruteforce(T, P, D, None, exact=True)


@pytest.mark.parametrize("seed,lam", [(9, True), (10, False), (11, True)])
def test_dp_consistent_for_any_weights(seed, lam):
    I, rng = _small(seed)
    T = oracle.Tree(I)
    P = _rand_params(T, rng, w_d=int(rng.integers(1, 50)), lam=lam)
    D = rng.integers(0, 9, T.num_edges).astype(np.int32)
    _check_against_bruteforce(T, P, D, None, exact=False)


def _hulls(T, lay):
    lo = np.zeros(T.nodes, np.int64)
    hi = np.zeros(T.nodes, np.int64)
    for v in range(T.nodes):
        a = 0 if T.parent[v] < 0 else int(lay[v])
        s = {a}
        if T.is_sink[v] or T.parent[v] < 0:
            s.add(0)
        lo[v], hi[v] = min(s), max(s)
    for v in range(T.nodes):
        p = T.parent[v]
        if p >= 0:
            lo[p] = min(lo[p], lay[v])
            hi[p] = max(hi[p], lay[v])
    return lo, hi


def test_invariants_on_config1(c1_instance):
    I = c1_instance
    T = oracle.Tree(I)
    P0 = oracle.Params(T)
    w = oracle.plain_weights(T, P0)
    P = oracle.Params(T, seg_w=w["seg_w"], pin_w=w["pin_w"], lam=w["lam"])
    st = oracle.State(T)
    lay, vlo, vhi, froot = oracle.assign(T, P, st, w["tier"], rounds=1)
    nonroot = T.parent >= 0
    # every segment on a layer of its own direction (the 3D result projects onto the 2D tree)
    assert (I.layer_dir[lay[nonroot]] == T.dir[nonroot]).all()
    # via span at every node is the hull of its entering layer, child layers and pin layer
    lo, hi = _hulls(T, lay)
    assert (vlo == lo).all() and (vhi == hi).all()
    # demand equals an independent recount, and is conserved per layer
    Dr = recount_demand(T, lay, I.X, I.Y, I.L)
    assert (st.D == Dr).all()
    per_layer = np.bincount(lay[nonroot], weights=T.len[nonroot], minlength=I.L)
    assert np.array_equal(st.D.reshape(-1, I.L).sum(0), per_layer.astype(np.int64))


def test_objective_terms_pinned_independently(c1_instance):
    I = c1_instance
    T = oracle.Tree(I)
    rng = np.random.default_rng(2)
    lay = np.zeros(T.nodes, np.uint8)
    for v in range(T.nodes):
        if T.parent[v] >= 0:
            opts = np.nonzero(I.layer_dir == T.dir[v])[0]
            lay[v] = opts[rng.integers(0, len(opts))]
    D = rng.integers(0, 14, T.num_edges).astype(np.int32)
    Z = np.zeros(T.num_edges, np.int32)

    def J(**kw):
        base = dict(w_cong=0, w_cap=0, w_d=0, w_via=0)
        base.update(kw)
        return int(oracle.objective(T, oracle.Params(T, **base), lay, D).sum())

    # capacitance: sum of wire C of the assignment (aF) = Elmore RC model C (fF) * 1000
    R, C = oracle.rc(T, oracle.Params(T), lay)
    assert J(w_cap=1) == round(C[:T.nodes].sum() * 1000)
    # vias: hull spans recounted from the layers
    lo, hi = _hulls(T, lay)
    assert J(w_via=1) == int((hi - lo).sum())
    # delay with unit weights: sum over RC edges of R (C/2 + S) from the FP64 Elmore pass,
    # in mOhm*aF/1024, each term floored once
    S, t, d = oracle.elmore(T, R, C)
    Sfull = np.concatenate([S, np.full(T.sinks, 1.0)])
    mask = np.ones(T.nodes + T.sinks, bool)
    mask[np.nonzero(T.parent < 0)[0]] = False            # the driver resistance is not a DP term
    ref = (R[mask] * (C[mask] / 2 + Sfull[mask])).sum() * 1e9 / 1024
    nterms = 2 * int((T.parent >= 0).sum()) + T.sinks
    got = J(w_d=1)
    assert ref - nterms <= got <= ref + 1e-6 * ref
    # congestion: with H = 0, each segment's cost is 1024 x the rise of the Eq. 3 total
    # overflow (s = 0.5 for c > 0, 1.5 for c = 0) when it joins demand D, up to rounding
    caps = I.caps.reshape(-1).astype(np.float64)
    s = np.where(caps > 0, 0.5, 1.5)
    P = oracle.Params(T)
    for v in np.nonzero(T.parent >= 0)[0][:300]:
        k = oracle.kappa(T, P, int(v), int(lay[v]), D)
        Dv = np.zeros(T.num_edges, np.int64)
        one = np.zeros(T.nodes, np.uint8)
        one[:] = lay
        Dv += recount_demand_single(T, int(v), int(lay[v]), I)
        dd = np.clip(D - caps, -32, 31)
        rise = (np.exp(s * (dd + Dv)) - np.exp(s * dd))[Dv > 0].sum() * 1024
        assert abs(k - rise) <= 0.5 * T.len[v] + 1e-9 * rise or k == int(T.len[v]) * (1 << 20)
    assert J(w_cong=1) == sum(oracle.kappa(T, P, int(v), int(lay[v]), D) for v in np.nonzero(T.parent >= 0)[0])
    del Z


def recount_demand_single(T, v, l, I):
    D = np.zeros((I.Y, I.X, I.L), np.int64)
    p = T.parent[v]
    if T.dir[v] == 0:
        x0, x1 = sorted((int(T.x[p]), int(T.x[v])))
        D[int(T.y[v]), x0:x1, l] += 1
    else:
        y0, y1 = sorted((int(T.y[p]), int(T.y[v])))
        D[y0:y1, int(T.x[v]), l] += 1
    return D.reshape(-1)


def test_self_exclusion_and_history():
    I, rng = _small(12, nets=60)
    T = oracle.Tree(I)
    P = _rand_params(T, rng)
    st = oracle.State(T)
    lay0, _, _, _ = oracle.assign(T, P, st, None, rounds=1)
    # history after one round: 64 x overflow, saturating at 2^24
    over = np.maximum(st.D.astype(np.int64) - I.caps.reshape(-1), 0)
    assert (st.H == np.minimum(64 * over, 1 << 24)).all()
    # round 2: the objective seen by the DP excludes each segment's own previous demand
    D1, H1 = st.D.copy(), st.H.copy()
    lay1, _, _, froot1 = oracle.assign(T, P, st, None, rounds=1)
    J = oracle.objective(T, P, lay1, D1, H1, prev=lay0)
    assert (froot1 == J).all()
    # demand after the move equals a recount
    assert (st.D == recount_demand(T, lay1, I.X, I.Y, I.L)).all()


def test_resume_reproduces_next_round():
    I, rng = _small(13, nets=80)
    T = oracle.Tree(I)
    P = _rand_params(T, rng)
    tiers = rng.integers(0, 4, T.nets).astype(np.uint8)
    a = oracle.State(T)
    la, va, ha, fa = oracle.assign(T, P, a, tiers, rounds=3)
    b = oracle.State(T)
    oracle.assign(T, P, b, tiers, rounds=2)
    saved = (b.D.copy(), b.H.copy(), b.prev.copy(), b.has_prev)
    c = oracle.State(T)
    c.D[:], c.H[:], c.prev[:], c.has_prev = saved
    lc, vc, hc, fc = oracle.assign(T, P, c, tiers, rounds=1)
    assert (la == lc).all() and (a.D == c.D).all() and (a.H == c.H).all() and (fa == fc).all()


def test_single_segment_net_closed_form():
    # a straight 2-pin net: the driver stack and the sink stack both span 0..a
    I = make_instance([([(1, 2, -1, "driver"), (7, 2, 0, "sink")], [[], []])], X=10, Y=4, L=8)
    T = oracle.Tree(I)
    rng = np.random.default_rng(4)
    D = rng.integers(0, 12, T.num_edges).astype(np.int32)
    P = oracle.Params(T, w_d=1, lam=np.zeros(T.nodes, np.int32))
    lay, vlo, vhi, froot = _run_dp(T, P, D)
    r, c, vr, L = I.r_mohm, I.c_af, I.via_r_mohm, I.L
    lut = oracle.cong_lut(L)
    caps = I.caps.reshape(-1)

    def cost(a):
        k = 0
        for x in range(1, 7):
            g = ((2 * I.X) + x) * L + a
            k += int(lut[a, 0 if caps[g] else 1, min(max(int(D[g]) - int(caps[g]), -32), 31) + 32])
        C = int(c[a]) * 6
        X = C + 2 * 1000
        rv = int(sum(vr[:a]))
        T_ = lambda R, XX: (1024 * ((R * XX) >> 11)) >> 10
        return 1000 * k + 100 * C + 2 * 100000 * a + T_(int(r[a]) * 6, X) + T_(rv, X) + T_(rv, 2000)

    costs = {a: cost(a) for a in range(0, L, 2)}
    best = min(costs, key=lambda a: (costs[a], a))
    assert lay[1] == best and froot[0] == costs[best]


def _forced_upstream_case(seed):
    """driver -H-> A1 -H-> A2, with sinks hanging from A2 on V segments.  One H layer and three
    V layers: the upstream wire is fixed, so r_est (average R of the one H layer) is the true
    upstream resistance.  Resistances are multiples of 2048 mOhm so every floor is exact."""
    rng = np.random.default_rng(seed)
    x1 = int(rng.integers(2, 6))
    x2 = x1 + int(rng.integers(2, 6))
    ns = int(rng.integers(1, 3))
    nodes = [(0, 6, -1, "driver"), (x1, 6, 0, "steiner"), (x2, 6, 1, "steiner")]
    for k in range(ns):
        nodes.append((x2, 6 + (1 if k == 0 else -1) * int(rng.integers(1, 7)), 2, "sink"))
    r = (2048 * rng.integers(1, 24, 4)).tolist()
    c = rng.integers(20, 600, 4).tolist()
    vr = (2048 * rng.integers(0, 8, 3)).tolist()
    I = make_instance([(nodes, [[]] * len(nodes))], X=x2 + 2, Y=13, L=4, layer_rc=(r, c, vr),
                      layer_dir=[0, 1, 1, 1], cpin_af=int(rng.integers(200, 2000)))
    return I, rng


def test_lookahead_exact_when_upstream_is_fixed():
    # Sec. III-D: f'_u = f_u + w_d r_est_u c_u charges a subtree's capacitance to the upstream
    # resistance.  With the upstream wire fixed, r_est is exact and the DP with look-ahead finds
    # the true minimum of J; without it the DP ignores the after-effect.
    misses_without = 0
    for seed in range(80):
        I, rng = _forced_upstream_case(seed)
        T = oracle.Tree(I)
        base = oracle.Params(T)
        sw, lam = oracle.edge_weights(T, base, np.full(T.sinks, 1024, np.uint16))
        assert (lam[T.parent >= 0] % 2048 == 0).all()
        w_via = int(rng.integers(0, 3)) * 1000
        D = np.zeros(T.num_edges, np.int32)
        P = oracle.Params(T, seg_w=sw, lam=lam, w_cong=0, w_cap=0, w_via=w_via, w_d=1)
        lay, _, _, froot = _run_dp(T, P, D)
        jmin, best, nmin = oracle.bruteforce(T, P, 0, D)
        assert froot[0] == jmin, seed
        P0 = oracle.Params(T, seg_w=sw, lam=np.zeros(T.nodes, np.int32), w_cong=0, w_cap=0, w_via=w_via, w_d=1)
        lay0, _, _, froot0 = _run_dp(T, P0, D)
        assert froot0[0] >= jmin
        misses_without += int(froot0[0] > jmin)
    assert misses_without >= 5


def test_ties_go_to_lowest_layers():
    # with every weight zero all stacks tie: the rule is smallest b, then smallest t, and each
    # child takes its lowest allowed layer inside the stack
    I = gen.generate(60, 20, 20, 8, 77, pin_max=6)
    T = oracle.Tree(I)
    P = oracle.Params(T, w_cong=0, w_cap=0, w_d=0, w_via=0)
    lay, vlo, vhi, froot = _run_dp(T, P)
    nonroot = T.parent >= 0
    assert (lay[nonroot] == T.dir[nonroot]).all()       # layer 0 for H, layer 1 for V
    assert (froot == 0).all() and (vlo == 0).all()
    for v in range(T.nodes):
        need = [0 if T.parent[v] < 0 else int(lay[v])] + [int(lay[c]) for c in np.nonzero(T.parent == v)[0]]
        assert vhi[v] == max(need)


def test_rip_up_sees_only_other_nets():
    # a net alone on a roomy grid: in round 2 its own previous demand is excluded, so it meets
    # exactly the empty grid of round 1 again and repeats its choice and cost
    nets = []
    for k in range(6):
        y = 2 + 3 * k
        nets.append(([(1, y, -1, "driver"), (9, y, 0, "steiner"), (9, y + 2, 1, "sink"), (14, y, 1, "sink")],
                     [[], [], [], []]))
    I = make_instance(nets, X=18, Y=22, L=8, caps=np.full((22, 18, 8), 2, np.uint8))
    T = oracle.Tree(I)
    P = oracle.Params(T, seg_w=np.full(T.nodes, 700, np.uint16), lam=np.full(T.nodes, 90000, np.int32))
    st = oracle.State(T)
    lay1, _, _, f1 = oracle.assign(T, P, st, None, rounds=1)
    assert (st.H == 0).all()
    lay2, _, _, f2 = oracle.assign(T, P, st, None, rounds=1)
    assert (lay1 == lay2).all() and (f1 == f2).all()


def test_history_saturates():
    I, rng = _small(14, nets=60)
    I.caps[:] = 0
    T = oracle.Tree(I)
    P = _rand_params(T, rng)
    st = oracle.State(T)
    oracle.assign(T, P, st, None, rounds=2, hist_inc=1 << 23)
    D = st.D.astype(np.int64)
    assert st.H.max() == 1 << 24 and (st.H[D >= 2] == 1 << 24).all()


# ---- the history term of the congestion cost (Eq. 3 marginal plus history H) --------------

def _seg_edges(T, v, I, l):
    """API grid indices of the GCell edges segment parent->v covers on layer l (recounted
    from the coordinates)."""
    p = int(T.parent[v])
    if T.dir[v] == 0:
        x0, x1 = sorted((int(T.x[p]), int(T.x[v])))
        return [((int(T.y[v]) * I.X) + x) * I.L + l for x in range(x0, x1)]
    y0, y1 = sorted((int(T.y[p]), int(T.y[v])))
    return [((y * I.X) + int(T.x[v])) * I.L + l for y in range(y0, y1)]


def test_kappa_rises_by_the_history_along_the_segment():
    # kappa_s(l) = sum over the segment's GCell edges of [LUT(D - Cap) + H]: with the demand held,
    # adding a history map raises it by exactly the history summed over those edges on layer l
    I, rng = _small(15, nets=50)
    T = oracle.Tree(I)
    P = oracle.Params(T)
    D = rng.integers(0, 9, T.num_edges).astype(np.int32)
    H = np.zeros(T.num_edges, np.int32)
    H[rng.random(T.num_edges) < 0.4] = rng.integers(1, 1 << 20, 1)[0]
    H += rng.integers(0, 3000, T.num_edges).astype(np.int32)
    checked = 0
    for v in np.nonzero(T.parent >= 0)[0][:200]:
        for l in np.nonzero(I.layer_dir == T.dir[v])[0]:
            rise = oracle.kappa(T, P, int(v), int(l), D, H) - oracle.kappa(T, P, int(v), int(l), D)
            assert rise == int(H[_seg_edges(T, int(v), I, int(l))].astype(np.int64).sum())
            checked += 1
    assert checked > 300


def test_objective_history_term_is_history_under_the_recounted_demand():
    # W_cong * sum_s kappa_s(a_s): the history part is H summed over every GCell edge the
    # assignment occupies, i.e. the dot product of H with the recounted demand
    I = gen.generate(80, 24, 24, 8, 16, pin_max=6)
    T = oracle.Tree(I)
    rng = np.random.default_rng(16)
    lay = np.zeros(T.nodes, np.uint8)
    for v in range(T.nodes):
        if T.parent[v] >= 0:
            opts = np.nonzero(I.layer_dir == T.dir[v])[0]
            lay[v] = opts[rng.integers(0, len(opts))]
    D = rng.integers(0, 10, T.num_edges).astype(np.int32)
    H = rng.integers(0, 50000, T.num_edges).astype(np.int32)
    P = oracle.Params(T, w_cong=7, w_cap=0, w_d=0, w_via=0)
    dj = int(oracle.objective(T, P, lay, D, H).sum() - oracle.objective(T, P, lay, D).sum())
    occ = recount_demand(T, lay, I.X, I.Y, I.L)
    assert dj == 7 * int(occ @ H.astype(np.int64))


def test_history_alone_moves_a_single_segment():
    # a straight 2-pin net with a closed-form cost per layer: history on the layer that wins
    # without it moves the net, and F_root is the closed form with the history included
    I = make_instance([([(1, 2, -1, "driver"), (7, 2, 0, "sink")], [[], []])], X=10, Y=4, L=8)
    T = oracle.Tree(I)
    rng = np.random.default_rng(17)
    D = rng.integers(0, 12, T.num_edges).astype(np.int32)
    P = oracle.Params(T, w_d=1, lam=np.zeros(T.nodes, np.int32))
    r, c, vr, L = I.r_mohm, I.c_af, I.via_r_mohm, I.L
    lut = oracle.cong_lut(L)
    caps = I.caps.reshape(-1)

    def cost(a, H):
        k = 0
        for x in range(1, 7):
            g = ((2 * I.X) + x) * L + a
            k += int(lut[a, 0 if caps[g] else 1, min(max(int(D[g]) - int(caps[g]), -32), 31) + 32]) + int(H[g])
        C = int(c[a]) * 6
        X = C + 2 * 1000
        rv = int(sum(vr[:a]))
        T_ = lambda R, XX: (1024 * ((R * XX) >> 11)) >> 10
        return 1000 * k + 100 * C + 2 * 100000 * a + T_(int(r[a]) * 6, X) + T_(rv, X) + T_(rv, 2000)

    H0 = np.zeros(T.num_edges, np.int32)
    c0 = {a: cost(a, H0) for a in range(0, L, 2)}
    a0 = min(c0, key=lambda a: (c0[a], a))
    H = H0.copy()
    for x in range(1, 7):
        H[((2 * I.X) + x) * L + a0] = 5000 + 13 * x
    c1 = {a: cost(a, H) for a in range(0, L, 2)}
    a1 = min(c1, key=lambda a: (c1[a], a))
    assert a1 != a0
    lay, vlo, vhi, froot = _run_dp(T, P, D, H)
    assert lay[1] == a1 and froot[0] == c1[a1]
    jmin, best, nmin = oracle.bruteforce(T, P, 0, D, H)
    assert jmin == c1[a1] and nmin == 1 and best[1] == a1


# ---- tie between a child's layers: the lowest layer, and its capacitance upstream ---------

def test_child_tie_takes_the_lowest_layer_and_its_capacitance():
    # driver -H-> sink A -H-> sink B.  History on B's edges makes B's cost equal on layers 0, 2
    # and 4 (the via stack [0, l] costs W_via l, the history the rest), and B carries no delay
    # weight, so B's keys tie whatever A's layer.  A's history sends A to layer 4, whose stack
    # [0, 4] holds all three tied layers: B must take the lowest, 0, and the capacitance of B on
    # layer 0 (not 2 or 4) must reach A's downstream load, which A's delay term prices.
    V = 1000
    I = make_instance([([(0, 0, -1, "driver"), (5, 0, 0, "sink"), (9, 0, 1, "sink")], [[], [], []])],
                      X=12, Y=3, L=8)
    T = oracle.Tree(I)
    L = I.L
    H = np.zeros(T.num_edges, np.int32)
    for x in range(5, 9):                      # B's edges: 4 of them
        H[x * L + 0] = V                       # 0 * V + 4 V = 4 V
        H[x * L + 2] = V // 2                  # 2 V + 2 V
        H[x * L + 4] = 0                       # 4 V
        H[x * L + 6] = 0                       # 6 V: dearer
    for x in range(0, 5):                      # A's edges: only layer 4 is cheap
        for l in (0, 2, 6):
            H[x * L + l] = 1 << 20
    sw = np.zeros(T.nodes, np.uint16)
    sw[1] = 1024                               # A's segment prices its downstream capacitance
    P = oracle.Params(T, seg_w=sw, pin_w=np.zeros(T.sinks, np.uint16), lam=np.zeros(T.nodes, np.int32),
                      w_cong=1, w_cap=0, w_d=1, w_via=V)
    D = np.zeros(T.num_edges, np.int32)
    lay, vlo, vhi, froot = _run_dp(T, P, D, H)
    assert lay[1] == 4 and lay[2] == 0
    assert (vlo[1], vhi[1]) == (0, 4)
    # F_root is J of the traced assignment, whose downstream load at A has B on layer 0
    assert froot[0] == oracle.objective(T, P, lay, D, H)[0]
    c, vr = I.c_af, I.via_r_mohm
    S_A = 1000 + int(c[0]) * 4 + 1000
    X_A = int(c[4]) * 5 + 2 * S_A
    T_ = lambda w, R, XX: (w * ((R * XX) >> 11)) >> 10
    lut = oracle.cong_lut(L)
    base = int(lut[0, 0, 0 - 8 + 32])          # D = 0, cap = 8 on every edge and layer
    F_B = 4 * base + 4 * V
    F_A = 4 * V + F_B + 5 * base + T_(1024, int(I.r_mohm[4]) * 5, X_A)
    root = 4 * V + F_A + T_(1024, int(sum(vr[:4])), X_A)
    assert froot[0] == root
