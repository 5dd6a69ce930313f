"""Pins of the oracle's classical batching (Alg. 1, GetBatch; the batching of the routers the
paper cites for it): within a subset, in net order, a net joins the lowest batch whose nets'
boxes share no GCell with its own; subsets are batched one after another.

- closed forms on hand-built nets (identical boxes, disjoint boxes, a chain, boxes that touch
  at one GCell, subsets that never share a batch, nets left out);
- a pure-Python pairwise brute force on small random instances;
- on a larger sample, properties that define first-fit: no two nets of a batch share a GCell,
  and a net in batch k overlaps an earlier net of its subset in every batch below k."""
import numpy as np

import gen
import oracle
from helpers import make_instance


def _two_pin(x0, y0, x1, y1):
    # driver at (x0, y0), sink at (x1, y1), one bend at (x1, y0)
    wps = [[], [(x1, y0)]] if (x0 != x1 and y0 != y1) else [[], []]
    return ([(x0, y0, -1, "driver"), (x1, y1, 0, "sink")], wps)


def _batches(nets, subset=None, X=32, Y=32):
    inst = make_instance(nets, X=X, Y=Y)
    T = oracle.Tree(inst)
    sub = np.zeros(T.nets, np.int32) if subset is None else np.asarray(subset, np.int32)
    ns = 1 if subset is None else max(int(sub.max()) + 1, 1)
    return oracle.get_batches(T, X, Y, sub, ns)


def test_identical_boxes_take_one_batch_each():
    b, n = _batches([_two_pin(2, 2, 8, 6)] * 5)
    assert n == 5 and b.tolist() == [0, 1, 2, 3, 4]


def test_disjoint_boxes_share_batch_zero():
    b, n = _batches([_two_pin(1, 1, 4, 4), _two_pin(6, 1, 9, 4), _two_pin(1, 6, 4, 9), _two_pin(6, 6, 9, 9)])
    assert n == 1 and b.tolist() == [0, 0, 0, 0]


def test_chain_alternates():
    # A overlaps B, B overlaps C, A and C are apart: A, C in batch 0, B in batch 1
    b, n = _batches([_two_pin(0, 0, 5, 3), _two_pin(5, 0, 10, 3), _two_pin(10, 0, 15, 3)])
    assert b.tolist() == [0, 1, 0] and n == 2


def test_boxes_touching_at_one_gcell_conflict_and_adjacent_ones_do_not():
    # sharing the corner GCell (5, 5) is a conflict; boxes on neighbouring GCells are not
    b, _ = _batches([_two_pin(0, 0, 5, 5), _two_pin(5, 5, 9, 9), _two_pin(6, 0, 9, 4)])
    assert b.tolist() == [0, 1, 0]


def test_first_fit_takes_the_lowest_free_batch():
    # nets 0 and 1 share row 2 (batches 0, 1); net 2 overlaps only net 0, so it takes batch 1
    b, _ = _batches([_two_pin(0, 0, 6, 2), _two_pin(0, 2, 6, 6), _two_pin(1, 0, 3, 1)])
    assert b.tolist() == [0, 1, 1]
    # a net overlapping both goes above them; one overlapping neither stays in batch 0
    b, _ = _batches([_two_pin(0, 0, 6, 2), _two_pin(0, 2, 6, 6), _two_pin(1, 1, 3, 5), _two_pin(8, 0, 9, 9)])
    assert b.tolist() == [0, 1, 2, 0]


def test_subsets_keep_their_order_and_never_share_a_batch():
    nets = [_two_pin(0, 0, 3, 3), _two_pin(10, 10, 13, 13), _two_pin(20, 20, 23, 23), _two_pin(0, 0, 3, 3)]
    # subset 1 holds nets 0 and 3 (same box), subset 0 nets 1 and 2 (apart); net 2 is left out below
    b, n = _batches(nets, subset=[1, 0, 0, 1])
    assert b.tolist() == [1, 0, 0, 2] and n == 3
    b, n = _batches(nets, subset=[1, 0, -1, 1])
    assert b.tolist() == [1, 0, -1, 2] and n == 3


def _boxes(T):
    out = []
    for i in range(T.nets):
        s = slice(int(T.net_ptr[i]), int(T.net_ptr[i + 1]))
        out.append((int(T.x[s].min()), int(T.x[s].max()), int(T.y[s].min()), int(T.y[s].max())))
    return out


def _overlap(a, b):
    return a[0] <= b[1] and b[0] <= a[1] and a[2] <= b[3] and b[2] <= a[3]


def _brute(T, subset, nsub):
    # pairwise first-fit, written from the definition (small inputs only)
    bx = _boxes(T)
    out = [-1] * T.nets
    base = 0
    for s in range(nsub):
        members = []
        nb = 0
        for i in range(T.nets):
            if subset[i] != s:
                continue
            k = 0
            while any(out[j] == base + k and _overlap(bx[i], bx[j]) for j in members):
                k += 1
            out[i] = base + k
            nb = max(nb, k + 1)
            members.append(i)
        base += nb
    return out, base


def test_brute_force_on_small_random_instances():
    rng = np.random.default_rng(2507)
    for seed in range(6):
        inst = gen.generate(300, 48, 48, 8, seed + 11)
        T = oracle.Tree(inst)
        nsub = 3
        subset = rng.integers(-1, nsub, T.nets).astype(np.int32)
        b, n = oracle.get_batches(T, inst.X, inst.Y, subset, nsub)
        bb, nn = _brute(T, subset, nsub)
        assert n == nn and b.tolist() == bb


def test_first_fit_properties_on_a_sample():
    inst = gen.config(4, num_nets=20000)
    T = oracle.Tree(inst)
    sub = (np.arange(T.nets) % 3 == 0).astype(np.int32)   # two subsets
    b, n = oracle.get_batches(T, inst.X, inst.Y, sub, 2)
    assert b.min() == 0 and b.max() == n - 1
    # the two subsets' batches are disjoint ranges, subset 0 first
    assert b[sub == 0].max() < b[sub == 1].min()
    bx = np.array(_boxes(T))
    X, Y = inst.X, inst.Y
    # no two nets of a batch share a GCell: the per-batch coverage counts never exceed 1
    for k in range(n):
        cov = np.zeros((Y + 1, X + 1), np.int32)
        for i in np.nonzero(b == k)[0]:
            x0, x1, y0, y1 = bx[i]
            cov[y0, x0] += 1
            cov[y0, x1 + 1] -= 1
            cov[y1 + 1, x0] -= 1
            cov[y1 + 1, x1 + 1] += 1
        assert np.cumsum(np.cumsum(cov, 0), 1).max() <= 1, k
    # a net in batch k > base of its subset overlaps an earlier net of its subset in each lower batch
    base = {0: 0, 1: int(b[sub == 1].min())}
    rng = np.random.default_rng(7)
    for i in rng.choice(np.nonzero(b > 0)[0], 300, replace=False):
        s = sub[i]
        earlier = np.nonzero((sub == s) & (np.arange(T.nets) < i))[0]
        ov = earlier[(bx[earlier, 0] <= bx[i, 1]) & (bx[i, 0] <= bx[earlier, 1]) &
                     (bx[earlier, 2] <= bx[i, 3]) & (bx[i, 2] <= bx[earlier, 3])]
        assert set(range(base[s], int(b[i]))) <= set(b[ov].tolist()), i
