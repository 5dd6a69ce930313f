"""C ABI: the library loads, exports every symbol include/gapla.h declares, and its host-side
validation returns the documented status before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import gen
import oracle
import paper_2507_13375_amd as la
from helpers import make_instance

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gapla.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:la_status|void|const char \*)\s*(la_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18
    lib = ctypes.CDLL(la.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert sorted(la.EXPORTS) == names


def test_status_names():
    assert la.la_status_str(0) == "LA_OK"
    assert la.la_status_str(-2) == "LA_ERR_BAD_TREE"
    assert la.la_status_str(-6) == "LA_ERR_STATE"


def test_default_congestion_table_is_eq3():
    # both sides build the Eq. 3 marginal table from its definition in FP64
    for L in (2, 8, 12, 16):
        assert np.array_equal(la.la_default_cong_lut(L), oracle.cong_lut(L))
    ofw = np.linspace(0.5, 2.0, 10)
    assert np.array_equal(la.la_default_cong_lut(10, ofw), oracle.cong_lut(10, ofw))


def _expect(inst, code, **kw):
    with pytest.raises(la.LAError) as e:
        la.la_build_batch(inst, stream=la.V(0), **kw)
    assert e.value.code == code, str(e.value)
    return str(e.value)


@pytest.mark.parametrize("case", ["diagonal", "zero_length", "cycle", "two_drivers", "off_grid", "reversal",
                                  "driver_not_first"])
def test_bad_trees_rejected_on_host(case):
    nets = {
        "diagonal": [(0, 0, -1, "driver"), (3, 2, 0, "sink")],
        "zero_length": [(1, 1, -1, "driver"), (1, 1, 0, "sink")],
        "cycle": [(0, 0, -1, "driver"), (2, 0, 2, "steiner"), (4, 0, 1, "sink")],
        "two_drivers": [(0, 0, -1, "driver"), (2, 0, 0, "driver")],
        "off_grid": [(0, 0, -1, "driver"), (9, 0, 0, "sink")],
        "reversal": [(0, 0, -1, "driver"), (2, 0, 0, "sink")],
        "driver_not_first": [(2, 0, 1, "sink"), (0, 0, -1, "driver")],
    }[case]
    wps = [[], [(5, 0)]] if case == "reversal" else [[]] * len(nets)
    good = ([(0, 0, -1, "driver"), (3, 0, 0, "sink")], [[], []])
    inst = make_instance([good, (nets, wps)], X=8, Y=8)
    msg = _expect(inst, la.LA_ERR_BAD_TREE)
    assert "net 1" in msg


def test_invalid_arguments_on_host():
    I = gen.generate(4, 8, 8, 8, 3)
    I.L = 17
    _expect(I, la.LA_ERR_INVALID_ARG)
    I = gen.generate(4, 8, 8, 8, 3)
    _expect(I, la.LA_ERR_INVALID_ARG, min_layer=8)
    I = gen.generate(4, 8, 8, 8, 3)
    I.net_node_ptr = I.net_node_ptr.copy()
    I.net_node_ptr[-1] += 1
    _expect(I, la.LA_ERR_INVALID_ARG)


def test_range_checks_on_host():
    I = gen.generate(2, 16, 16, 8, 3)
    I.via_r_mohm = np.full(7, 3_000_000, np.int32)        # total via R beyond 2^24 mOhm
    _expect(I, la.LA_ERR_RANGE)
    big = make_instance([([(0, 0, -1, "driver"), (2, 0, 0, "sink")], [[], []])], X=16000, Y=16000, L=16,
                        caps=np.zeros((1, 1, 16), np.uint8))
    _expect(big, la.LA_ERR_RANGE)


def test_python_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    monkeypatch.setattr(la, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(la, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        la.la_status_str(0)


def test_quality_report_rejects_null_arguments_on_host():
    lib = la._load()
    q = la.la_quality()
    assert lib.la_quality_report(None, None, None, None, ctypes.byref(q)) == la.LA_ERR_INVALID_ARG
