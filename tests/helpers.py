"""Small hand-built instances for tests (inputs only)."""
import json
import os

import numpy as np

import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def make_instance(nets, X=16, Y=16, L=8, caps=None, budget_fs=None, cpin_af=1000, rdrv_mohm=1000000, layer_rc=None,
                  name="hand", layer_dir=None):
    """nets: list of (nodes, waypoints) where nodes = [(x, y, parent, kind)], kind in driver/sink/steiner,
    waypoints[k] = list of (x, y) bends on the edge parent(k) -> k."""
    ptr, par, xs, ys, fl, cp, wpp, wx, wy = [0], [], [], [], [], [], [0], [], []
    for nodes, wps in nets:
        for k, (x, y, p, kind) in enumerate(nodes):
            par.append(p)
            xs.append(x)
            ys.append(y)
            fl.append({"driver": 2, "sink": 1, "steiner": 0}[kind])
            cp.append(cpin_af if kind == "sink" else 0)
            for (a, b) in (wps[k] if wps else []):
                wx.append(a)
                wy.append(b)
            wpp.append(len(wx))
        ptr.append(len(par))
    N = len(nets)
    if layer_rc is None:
        ref = gen.generate(1, 4, 4, L, 1)
        r, c, vr = ref.r_mohm, ref.c_af, ref.via_r_mohm
    else:
        r, c, vr = (np.asarray(a, np.int32) for a in layer_rc)
    if caps is None:
        caps = np.full((Y, X, L), 8, np.uint8)
    return gen.Instance(
        name=name, X=X, Y=Y, L=L, net_node_ptr=np.array(ptr, np.int32), node_parent=np.array(par, np.int32),
        node_x=np.array(xs, np.int16), node_y=np.array(ys, np.int16), node_flags=np.array(fl, np.uint8),
        node_cpin_af=np.array(cp, np.int32), edge_wp_ptr=np.array(wpp, np.int32), wp_x=np.array(wx, np.int16),
        wp_y=np.array(wy, np.int16),
        net_budget_fs=np.array(budget_fs if budget_fs is not None else [0] * N, np.int32),
        net_rdrv_mohm=np.full(N, rdrv_mohm, np.int32), caps=np.asarray(caps, np.uint8),
        r_mohm=np.asarray(r, np.int32), c_af=np.asarray(c, np.int32), via_r_mohm=np.asarray(vr, np.int32),
        layer_dir=(np.arange(L) & 1).astype(np.uint8) if layer_dir is None else np.asarray(layer_dir, np.uint8))


def fixture_nets(fx):
    out = []
    for n in fx["nets"]:
        nodes = [(a[0], a[1], a[2], a[3]) for a in n["nodes"]]
        out.append((nodes, [[tuple(p) for p in w] for w in n["waypoints"]]))
    return out


def recount_demand(tree, layers, X, Y, L):
    """Independent recount of per-(edge, layer) demand from an assignment (numpy)."""
    D = np.zeros((Y, X, L), np.int64)
    par = tree.parent
    for v in np.nonzero(par >= 0)[0]:
        p = par[v]
        l = int(layers[v])
        if tree.dir[v] == 0:
            x0, x1 = sorted((int(tree.x[p]), int(tree.x[v])))
            D[int(tree.y[v]), x0:x1, l] += 1
        else:
            y0, y1 = sorted((int(tree.y[p]), int(tree.y[v])))
            D[y0:y1, int(tree.x[v]), l] += 1
    return D.reshape(-1)
