"""The allocation-free TNS / WNS entry point against la_timing_summary, through the C ABI: two
calls in a row on one GPU, the second on a smaller batch, then the first batch again (the
static scratch keeps the last call's partials; nothing may leak into the next call)."""
import numpy as np
import pytest

import gen
import paper_2507_13375_amd as la
from gpu_util import DeviceRun, say, torch

pytestmark = pytest.mark.gpu


def _summaries(run):
    d = run.elmore()
    ref = la.la_timing_summary(run.b, d)
    got = la.la_timing_summary_noalloc(run.b, d)
    return ref, got


def test_noalloc_summary_matches_two_calls_shrinking():
    big = DeviceRun(gen.config(2, num_nets=60000))
    small = DeviceRun(gen.config(1, num_nets=200))
    say("noalloc: %d sinks, then %d sinks" % (big.b.sinks, small.b.sinks))
    assert small.b.sinks < big.b.sinks
    for run in (big, small, big):
        ref, got = _summaries(run)
        say("  sinks %d: ref %r got %r" % (run.b.sinks, ref, got))
        assert got == ref          # same kernels and block count: the same bits
        assert ref[0] < 0 and ref[1] < 0
    torch().cuda.synchronize()


def test_noalloc_summary_rejects_null():
    run = DeviceRun(gen.config(1, num_nets=50))
    with pytest.raises(la.LAError) as e:
        la.la_timing_summary_noalloc(run.b, None)
    assert e.value.code == la.LA_ERR_INVALID_ARG
