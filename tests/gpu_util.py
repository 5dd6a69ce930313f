"""Runs the HIP path (through the C ABI) and the oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle
import paper_2507_13375_amd as la


def torch():
    import torch as t
    return t


def dev(a, dtype=None):
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype)))
    return x.cuda()


def host(x):
    torch().cuda.synchronize()
    return x.cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class DeviceRun:
    """One batch on the GPU plus helpers to run assignment and timing through the C ABI."""

    def __init__(self, inst, min_layer=0):
        t = torch()
        self.inst = inst
        self.b = la.la_build_batch(inst, min_layer=min_layer)
        self.E = inst.X * inst.Y * inst.L
        self.H = t.zeros(self.E, dtype=t.int32, device="cuda")
        self.layers = t.zeros(max(self.b.nodes, 1), dtype=t.uint8, device="cuda")

    def assign(self, seg_w, pin_w, lam, tiers=None, num_tiers=1, rounds=1, form=la.LA_FORM_PLAIN, **kw):
        t = torch()
        sw = dev(seg_w, np.uint16)
        pw = dev(pin_w if len(pin_w) else np.zeros(1), np.uint16)
        lm = dev(lam, np.int32)
        tr = None if tiers is None else dev(tiers, np.uint8)
        la.la_assign(self.b, sw, pw, lm, self.H, self.layers, net_tier=tr, num_tiers=num_tiers, rounds=rounds,
                     form=form, **kw)
        vias = t.empty(2 * max(self.b.nodes, 1), dtype=t.uint8, device="cuda")
        la.la_vias(self.b, vias)
        D = t.empty(self.E, dtype=t.int32, device="cuda")
        la.la_demand(self.b, D)
        v = host(vias).reshape(-1, 2)
        return dict(layers=host(self.layers)[:self.b.nodes], vlo=v[:self.b.nodes, 0], vhi=v[:self.b.nodes, 1],
                    D=host(D), H=host(self.H))

    def rc(self):
        """Copies of the batch-owned R, C views (float [rc_edges])."""
        R, C = la.la_batch_rc(self.b)
        n = self.b.rc_edges
        return _wrap(R, n).clone(), _wrap(C, n).clone()

    def elmore(self):
        t = torch()
        d = t.empty(max(self.b.sinks, 1), dtype=t.float32, device="cuda")
        la.la_elmore(self.b, d)
        return d


def _wrap(ptr, n):
    """float32 tensor aliasing n floats of device memory owned by the library."""
    t = torch()

    class _A:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<f4", "data": (ptr, False), "version": 3,
                                    "strides": None}

    return t.as_tensor(_A(), device="cuda")


def oracle_assign(inst, seg_w, pin_w, lam, tiers=None, rounds=1, H0=None, min_layer=0, **kw):
    T = oracle.Tree(inst)
    P = oracle.Params(T, seg_w=seg_w, pin_w=pin_w, lam=lam, min_layer=min_layer, **kw)
    st = oracle.State(T, H0)
    lay, vlo, vhi, fr = oracle.assign(T, P, st, tiers, rounds=rounds)
    return dict(layers=lay, vlo=vlo, vhi=vhi, D=st.D, H=st.H, froot=fr, tree=T, params=P, state=st)


def assert_assign_equal(g, o, what=""):
    nonroot = o["tree"].parent >= 0
    for k in ("vlo", "vhi"):
        bad = np.nonzero(g[k] != o[k])[0]
        assert bad.size == 0, "%s %s differ at %d nodes, first %s: gpu %s oracle %s" % (
            what, k, bad.size, bad[:5], g[k][bad[:5]], o[k][bad[:5]])
    bad = np.nonzero((g["layers"] != o["layers"]) & nonroot)[0]
    assert bad.size == 0, "%s layers differ at %d nodes, first %s: gpu %s oracle %s" % (
        what, bad.size, bad[:5], g["layers"][bad[:5]], o["layers"][bad[:5]])
    assert np.array_equal(g["D"], o["D"]), what + " demand differs"
    assert np.array_equal(g["H"], o["H"]), what + " history differs"


# lower bound of each critical batch's slack/WNS bin (Alg. 1 slack bins): batch 0 is rho = 1,
# batch k in 1..6 is [LOW[k], LOW[k-1]); batches 7..10 hold the non-critical nets (rho < 0.7)
BIN_LOW = [1.0, 0.99, 0.96, 0.91, 0.84, 0.75, 0.7]


def tier_flips_at_bin_edges(gt, ot, rho):
    """Number of nets whose batch differs; every difference must be between two neighbouring
    bins with the FP64 rho within 1e-5 of the edge between them (FP32 slack on the GPU)."""
    diff = np.nonzero(gt != ot)[0]
    for i in diff:
        a, b = sorted((int(gt[i]), int(ot[i])))
        assert a <= 6 and (b == a + 1 or (a == 6 and b >= 7)), (i, gt[i], ot[i], rho[i])
        e = BIN_LOW[a]
        assert abs(rho[i] - e) < 1e-5, (i, gt[i], ot[i], rho[i])
    return diff.size
