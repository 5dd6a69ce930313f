"""Kernel timing mode and the per-round work figures used for roofline reports: timed runs give
the same assignment as untimed (graph) runs, launch counts follow the schedule, and the work
figures match a count made from the oracle's trees."""
import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, say

pytestmark = pytest.mark.gpu


def _enumeration_count(inst, T):
    """Stacks x (6 per child + 10) summed over nodes and entering layers, and the congestion
    gather bytes (9 per GCell edge and routable layer), from the oracle's trees."""
    L = inst.L
    dirs = np.asarray(inst.layer_dir)
    routable = [[l for l in range(L) if dirs[l] == d] for d in (0, 1)]
    nch = np.bincount(T.parent[T.parent >= 0], minlength=T.nodes)
    ops, gather = 0.0, 0.0
    for v in range(T.nodes):
        per = 6.0 * nch[v] + 10.0
        if T.parent[v] < 0:
            ops += L * per
            continue
        pin = bool(T.is_sink[v])
        for l in routable[int(T.dir[v])]:
            ops += ((0 if pin else l) + 1) * (L - l) * per
        gather += 9.0 * T.len[v] * len(routable[int(T.dir[v])])
    return ops, gather


def test_work_figures():
    inst = gen.config(1)
    T = oracle.Tree(inst)
    b = la.la_build_batch(inst)
    ops, gather = _enumeration_count(inst, T)
    say("c1 dp ops %.0f (lib %.0f)" % (ops, b.dp_ops_per_round))
    assert b.dp_ops_per_round == ops
    fixed = 28.0 * T.nodes + 6.0 * T.sinks + 9.0 * T.nets
    assert b.dp_bytes_per_round == gather + fixed
    assert b.elmore_fwd_bytes == 28.0 * (T.nodes + T.sinks)
    assert b.elmore_bwd_bytes == 40.0 * (T.nodes + T.sinks)


@pytest.mark.parametrize("form", [la.LA_FORM_PLAIN, la.LA_FORM_BATCHED])
def test_timed_run_matches_untimed(form):
    inst = gen.config(1)
    T = oracle.Tree(inst)
    w = oracle.plain_weights(T, oracle.Params(T))
    rounds, ntier = 3, 11
    used_tiers = len(np.unique(w["tier"]))
    runs = []
    for timed in (False, True):
        g = DeviceRun(inst)
        if timed:
            la.la_profile_begin(g.b)
        r = g.assign(w["seg_w"], w["pin_w"], w["lam"], w["tier"], num_tiers=ntier, rounds=rounds, form=form)
        if timed:
            stats = la.la_profile_end(g.b)
            say("form %d timed kernels: %s" % (form, sorted(stats)))
            for name, (n, ms) in stats.items():
                assert n > 0 and ms >= 0.0, name
            assert stats["k_history"][0] == rounds
            assert stats["k_commit"][0] == rounds * used_tiers
            if form == la.LA_FORM_BATCHED:
                # config 1 nets all fit one tile: one persistent launch per used batch and round
                assert stats["k_batched_dp"][0] == rounds * used_tiers
                assert "k_batched_big" not in stats
            else:
                assert stats["k_dp_level"][0] >= rounds * used_tiers
                assert "k_batched_dp" not in stats
        runs.append(r)
    for k in ("layers", "vlo", "vhi", "D", "H"):
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_profile_state_errors():
    inst = gen.config(1, num_nets=50)
    b = la.la_build_batch(inst)
    with pytest.raises(la.LAError):
        la.la_profile_end(b)
    la.la_profile_begin(b)
    with pytest.raises(la.LAError):
        la.la_profile_begin(b)
    assert la.la_profile_end(b) == {}
