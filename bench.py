"""Throughput of the GAP-LA hot path on one MI355X: nets layer-assigned per second.

One step = the whole path over the 2,000,000-net workload (1024x1024 GCells, 12
layers): I outer iterations of [Elmore forward -> timing weights -> la_assign
with R negotiation rounds], then the Elmore timing of the final assignment.
nets/s = nets x R x I / step time.  Inputs are resident in HBM before timing.

The batched+adjoint form (persistent per-batch DP kernels in a hipGraph,
weights from the Elmore reverse sweep) is the reported value; the plain
per-level-launch form with Eq. 4/5 weights runs the same schedule beside it,
and so does the batched form with the plain form's weights (the batching gain
alone).  The CPU oracle is timed on a bounded sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

R_ROUNDS, I_ITERS = 5, 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--nets", type=int, default=None, help="truncate the workload (testing only)")
    ap.add_argument("--forms", default="batched,plain,batched_plainw",
                    help="batched (adjoint weights), plain (Eq. 4/5 weights), batched_plainw (batched, Eq. 4/5 weights)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--ablations", action="store_true",
                    help="also run the batched+adjoint schedule without look-ahead and with other w_d / w_cap, "
                         "and report the quality terms of each (one step each)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device-to-device copy of this many bytes (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2507_13375_amd as la

    torch.cuda.set_device(0)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    inst = gen.config(args.config, num_nets=args.nets)
    log("generated c%d: %d nets %d input nodes in %.1fs" % (args.config, inst.num_nets, inst.num_nodes,
                                                            time.time() - t0))
    t0 = time.time()
    b = la.la_build_batch(inst)
    torch.cuda.synchronize()
    log("la_build_batch: %d LA nodes, %d sinks, %d levels, %.1fs" % (b.nodes, b.sinks, b.levels, time.time() - t0))

    dev = "cuda"
    E = inst.X * inst.Y * inst.L
    H = torch.zeros(E, dtype=torch.int32, device=dev)
    layers = torch.zeros(b.nodes, dtype=torch.uint8, device=dev)
    delay = torch.zeros(b.sinks, dtype=torch.float32, device=dev)
    sw = torch.zeros(b.nodes, dtype=torch.uint16, device=dev)
    pw = torch.zeros(b.sinks, dtype=torch.uint16, device=dev)
    lam = torch.zeros(b.nodes, dtype=torch.int32, device=dev)
    tier = torch.zeros(b.nets, dtype=torch.uint8, device=dev)

    def step(form, mode, lookahead=True, **weights):
        la.la_reset(b)
        H.zero_()
        for _ in range(I_ITERS):
            la.la_elmore(b, delay)
            la.la_timing_weights(b, delay, mode, sw, pw, lam, tier)
            if not lookahead:
                lam.zero_()
            la.la_assign(b, sw, pw, lam, H, layers, net_tier=tier, num_tiers=11, rounds=R_ROUNDS, form=form,
                         **weights)
        la.la_elmore(b, delay)

    # the batched form's launch configuration, tuned once on this instance (outside the timed
    # steps) with the first iteration's adjoint weights
    tuning = None
    if any(n.startswith("batched") for n in args.forms.split(",")):
        t0 = time.time()
        la.la_reset(b)
        H.zero_()
        la.la_elmore(b, delay)
        la.la_timing_weights(b, delay, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
        tuning = la.la_tune(b, sw, pw, lam, H, net_tier=tier, num_tiers=11)
        b.dp_ops_big_per_round = la.la_batch_info(b)["dp_ops_big_per_round"]
        log("la_tune: %s in %.2fs" % (tuning, time.time() - t0))

    results = {}
    for name in args.forms.split(","):
        form = la.LA_FORM_PLAIN if name == "plain" else la.LA_FORM_BATCHED
        mode = la.LA_WEIGHTS_ADJOINT if name == "batched" else la.LA_WEIGHTS_PLAIN
        try:
            for _ in range(args.warmup):
                step(form, mode)
            torch.cuda.synchronize()
        except la.LAError as e:
            log("form %s unavailable: %s" % (name, e))
            continue
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        g0 = la.la_batch_info(b)["graph_instantiations"]
        ev0.record()
        for _ in range(args.steps):
            step(form, mode)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        graphs_timed = la.la_batch_info(b)["graph_instantiations"] - g0
        tns, wns = la.la_timing_summary(b, delay)
        results[name] = dict(ms=ms, nets_per_s=inst.num_nets * R_ROUNDS * I_ITERS / (ms * 1e-3), tns=tns, wns=wns,
                             graphs_timed=graphs_timed)
        log("form %s: %.2f ms/step, %.3e nets/s, TNS %.1f ps, WNS %.2f ps" % (name, ms, results[name]["nets_per_s"],
                                                                          tns, wns))
        # one more step on the same stream with every hot launch bracketed by HIP events
        # (the batched form then launches its kernels directly instead of replaying its graph)
        la.la_profile_begin(b)
        step(form, mode)
        results[name]["kernels"] = la.la_profile_end(b)
        for k, (n, t) in sorted(results[name]["kernels"].items(), key=lambda kv: -kv[1][1]):
            log("  %-16s %6d launches %10.3f ms/step %9.2f us/launch" % (k, n, t, 1e3 * t / n))
        if name == "batched":
            # quality terms of the final assignment (not part of the timed step); the first call
            # loads the kernel, the second is timed
            la.la_quality_report(b, delay=delay, weights=SCORE_WEIGHTS)
            la.la_profile_begin(b)
            q = la.la_quality_report(b, delay=delay, weights=SCORE_WEIGHTS)
            results[name]["quality"] = quality_rate(b, inst, q, la.la_profile_end(b))
            log("  quality: %s" % results[name]["quality"])

    ablations = None
    if args.ablations:
        # Sec. IV ablations on synthetic data: look-ahead off, and the delay and capacitance weights
        # scaled (from the defaults W_D = 1, W_CAP = 100)
        ablations = {}
        variants = [("default", {}), ("no_lookahead", {"lookahead": False}),
                    ("w_d_x0", {"w_d": 0}), ("w_d_x4", {"w_d": 4 * la.W_D}),
                    ("w_cap_x0", {"w_cap": 0}), ("w_cap_x10", {"w_cap": 10 * la.W_CAP})]
        for vname, kw in variants:
            t0 = time.time()
            step(la.LA_FORM_BATCHED, la.LA_WEIGHTS_ADJOINT, **kw)
            q = la.la_quality_report(b, delay=delay, weights=SCORE_WEIGHTS)
            torch.cuda.synchronize()
            ablations[vname] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()}
            ablations[vname]["wall_s"] = round(time.time() - t0, 3)
            log("ablation %-12s %s" % (vname, ablations[vname]))
        ablations["alg1_order"] = alg1_step(la, b, inst, delay, sw, pw, lam, tier, H, layers)
        log("ablation alg1_order   %s" % ablations["alg1_order"])

    main_form = "batched" if "batched" in results else "plain"
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst, main_form)

    r = results[main_form]
    digest = inst.digest()
    roof = {k: roofline(b, k, v["kernels"], digest) for k, v in results.items()}
    out = {
        "metric": "nets layer-assigned/sec (DP+Elmore) at 2M nets; batched vs plain, same GPU",
        "value": r["nets_per_s"],
        "unit": "nets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+fp32",
        "data": "synthetic",
        "config": {"workload": "c%d: %d nets, %dx%d GCells x %d layers, %s form, R=%d rounds x I=%d iterations"
                               % (args.config, inst.num_nets, inst.X, inst.Y, inst.L,
                                  "batched+adjoint" if main_form == "batched" else "plain", R_ROUNDS, I_ITERS),
                   "nets": inst.num_nets, "la_nodes": b.nodes, "rounds": R_ROUNDS, "iterations": I_ITERS,
                   "form": main_form, "tuning": tuning},
        "forms": {k: {"nets_per_s": v["nets_per_s"], "ms_per_step": v["ms"], "tns_ps": v["tns"], "wns_ps": v["wns"],
                      "roofline": roof[k], "elmore": elmore_rate(b, v["kernels"], digest),
                      "graph_instantiations_in_timed_steps": v["graphs_timed"],
                      "kernel_ms_per_step": {n: round(t, 4) for n, (c, t) in v["kernels"].items()}}
                  for k, v in results.items()},
        "roofline": roof[main_form],
        "cpu_baseline": cpu,
    }
    if "quality" in results.get("batched", {}):
        out["quality"] = results["batched"]["quality"]
    if ablations is not None:
        out["ablations"] = ablations
    if "batched" in results and "plain" in results:
        out["batched_over_plain"] = results["batched"]["nets_per_s"] / results["plain"]["nets_per_s"]
    if "batched_plainw" in results and "plain" in results:
        # same weights as the plain form: the gain of the batched orchestration alone
        out["batched_over_plain_same_weights"] = (results["batched_plainw"]["nets_per_s"] /
                                                  results["plain"]["nets_per_s"])
    print(json.dumps(out), flush=True)


def alg1_step(la, b, inst, delay, sw, pw, lam, tier, H, layers):
    """The paper's whole ordering flow (Alg. 1) in place of the slack bins and net-id batches:
    per iteration, static timing of a synthetic gate graph over the nets with the current sink
    delays, top-1 critical-path counts, the ordered subsets and their classical batches, then
    R rounds on those batches (adjoint-form weights); quality terms of the result and the time
    of the ordering calls (STA + subsets + batching) beside the whole step."""
    import gen
    import torch

    tg = gen.timing_graph(inst)
    la.la_timing_graph(b, tg["sink_next"], tg["gate_delay_fs"], tg["clock_fs"])
    slack = torch.empty(b.sinks, dtype=torch.float32, device="cuda")
    crit = torch.empty(b.nets, dtype=torch.int32, device="cuda")
    sub = torch.empty(b.nets, dtype=torch.int32, device="cuda")
    bat = torch.empty(b.nets, dtype=torch.int32, device="cuda")
    t0 = time.time()
    t_order = 0.0
    batches = []
    la.la_reset(b)
    H.zero_()
    for _ in range(I_ITERS):
        la.la_elmore(b, delay)
        la.la_timing_weights(b, delay, la.LA_WEIGHTS_ADJOINT, sw, pw, lam, tier)
        torch.cuda.synchronize()
        t1 = time.time()
        wns = la.la_sta(b, delay, slack, crit)
        nsub = la.la_alg1_subsets(b, slack, crit, wns, sub)
        nb = la.la_get_batches(b, sub, nsub, bat)
        torch.cuda.synchronize()
        t_order += time.time() - t1
        batches.append(nb)
        la.la_assign(b, sw, pw, lam, H, layers, num_tiers=nb, rounds=R_ROUNDS, form=la.LA_FORM_BATCHED,
                     net_batch=bat)
    la.la_elmore(b, delay)
    q = la.la_quality_report(b, delay=delay, weights=SCORE_WEIGHTS)
    torch.cuda.synchronize()
    out = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()}
    out.update(wall_s=round(time.time() - t0, 3), ordering_s=round(t_order, 3), batches=batches,
               critical_nets=int((crit > 3).sum().item()))
    return out


# the sources each measured kernel is built from (its traffic figure holds for these only)
KERNEL_SOURCES = {   # the kernel's code and the host code that lays out the records it reads
    "k_batched_dp": ("batched.hip", "dp_device.h", "la_internal.h", "build.cpp"),
    "k_elmore_wave": ("elmore.hip", "la_internal.h", "build.cpp"),
    "k_adj_wave": ("elmore.hip", "la_internal.h", "build.cpp"),
}


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", "%s_c4_2M_traffic.md" % kernel)


def kernel_sources_sha256(kernel="k_batched_dp"):
    """Hash of the sources of a kernel (the traffic figures hold for these only)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2507_13375_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_digest, kernel="k_batched_dp"):
    """HBM bytes per launch of `kernel` from its committed FETCH_SIZE/WRITE_SIZE summary, or None
    when it is missing, was taken on other kernel sources, or on another workload (the figure is
    per launch of one instance: its digest must match)."""
    try:
        vals = {}
        with open(traffic_file(kernel)) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("|", "#", "`")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel_sources_sha256") != kernel_sources_sha256(kernel):
            return None
        if vals.get("workload_digest") != workload_digest:
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes, one int32 op per lane per clock at 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def roofline(b, form, kernels, workload_digest):
    """The DP enumeration kernel against the vector-ALU peak.  Algorithmic work = stacks x
    (6 ops per child + 10) over every node and entering layer (la_info.dp_ops_per_round),
    times the rounds the step runs; divided by that kernel's summed launch time."""
    batched = form.startswith("batched")
    name = "k_batched_dp" if batched else "k_dp_level"
    if name not in kernels:
        return None
    n, ms = kernels[name]
    ops_round = b.dp_ops_per_round - (b.dp_ops_big_per_round if batched else 0.0)
    ops = ops_round * R_ROUNDS * I_ITERS
    achieved = ops / (ms * 1e-3) / 1e12
    # the same launches against HBM: the algorithmic bytes (per node and per GCell edge and
    # layer of its segment) over the launch time
    alg_bytes = b.dp_bytes_per_round * R_ROUNDS * I_ITERS / n
    hbm_gbs = alg_bytes / (ms / n * 1e-3) / 1e9
    return {"bound": "alu", "kernel": name, "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / ALU_PEAK_TOPS, "traffic": measured_traffic(workload_digest) if form == "batched" else None,
            "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": alg_bytes,
            "hbm": {"achieved": hbm_gbs, "peak": 8000.0, "unit": "GB/s", "frac": hbm_gbs / 8000.0},
            "launches": n, "avg_launch_us": 1e3 * ms / n, "ops_per_launch": ops / n}


# Eq. 1 weights for the reported score: illustrative (the paper's are per design), r = 0
SCORE_WEIGHTS = {"w1": -1.0, "w2": -1.0, "w3": 1.0, "w4": 1.0}


def quality_rate(b, inst, q, kernels):
    """Quality terms and the evaluator kernel's algorithmic HBM rate: demand (4 B) and capacity
    (1 B) per GCell edge, layer, via span, parent and length (11 B) per tree node."""
    out = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in q.items()}
    if "k_quality" in kernels:
        n, ms = kernels["k_quality"]
        gbs = (inst.X * inst.Y * inst.L * 5.0 + b.nodes * 11.0) / (ms / n * 1e-3) / 1e9
        out.update({"bound": "hbm", "kernel_us": 1e3 * ms / n, "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                    "frac": gbs / 8000.0})
    return out


def elmore_rate(b, kernels, workload_digest=None):
    """Algorithmic HBM rate of the Elmore forward sweeps (28 B per RC edge per sweep) and of the
    reverse sweeps of the adjoint weights (40 B per RC edge), with the measured traffic of the
    wavefront-run kernels that take the small nets, where a summary for these sources exists."""
    names = ("k_elmore_wave", "k_elmore_tiles", "k_elmore_up", "k_elmore_down")   # runs, tiles, untiled nets
    if not any(k in kernels for k in names):
        return None
    sweeps = I_ITERS + 1
    ms = sum(kernels[k][1] for k in names if k in kernels)
    gbs = b.elmore_fwd_bytes * sweeps / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
           "ms_per_sweep": ms / sweeps,
           "traffic_k_elmore_wave": measured_traffic(workload_digest, "k_elmore_wave") if workload_digest else None}
    back = ("k_adj_wave", "k_adj_tiles", "k_adj_up", "k_adj_down")
    nb = kernels["k_adj_wave"][0] if "k_adj_wave" in kernels else 0
    if nb:
        bms = sum(kernels[k][1] for k in back if k in kernels)
        bgbs = b.elmore_bwd_bytes * nb / (bms * 1e-3) / 1e9
        out["reverse"] = {"achieved": bgbs, "frac": bgbs / 8000.0, "ms_per_sweep": bms / nb,
                          "traffic_k_adj_wave": (measured_traffic(workload_digest, "k_adj_wave")
                                                 if workload_digest else None)}
    return out


def _oracle_schedule(T, adjoint):
    """The step's schedule on the oracle: I iterations of [FP64 Elmore -> weights -> R rounds],
    then the Elmore timing of the final assignment (the same work as one timed GPU step)."""
    import oracle

    P0 = oracle.Params(T)
    st = oracle.State(T)
    lay = None
    for _ in range(I_ITERS):
        w = (oracle.adjoint_form_weights if adjoint else oracle.plain_weights)(T, P0, lay)
        P = oracle.Params(T, seg_w=w["seg_w"], pin_w=w["pin_w"], lam=w["lam"])
        lay, _, _, _ = oracle.assign(T, P, st, w["tier"], rounds=R_ROUNDS)
    R, C = oracle.rc(T, P0, lay)
    oracle.elmore(T, R, C)
    return lay


def cpu_baseline(inst, form, single_nets=20000):
    """The oracle (as it stands) on the host cores: the whole workload with the reported form's
    schedule (batched+adjoint: adjoint-form weights; plain: Eq. 4/5 weights) on every host
    thread, then the first `single_nets` nets of the same generator on one thread."""
    import gen
    import oracle

    adjoint = form == "batched"
    T = oracle.Tree(inst)
    cores = oracle.num_threads()
    t0 = time.time()
    _oracle_schedule(T, adjoint)
    dt = time.time() - t0
    del T
    log("cpu oracle: %d nets, %d rounds x %d iterations in %.1fs on %d threads" % (
        inst.num_nets, R_ROUNDS, I_ITERS, dt, cores))
    single = None
    if inst.name in ("c3", "c4") and single_nets:
        sub = gen.config(4, num_nets=min(single_nets, inst.num_nets))
        Ts = oracle.Tree(sub)
        oracle.set_num_threads(1)
        try:
            t1 = time.time()
            _oracle_schedule(Ts, adjoint)
            ds = time.time() - t1
        finally:
            oracle.set_num_threads(cores)
        single = {"value": sub.num_nets * R_ROUNDS * I_ITERS / ds, "unit": "nets/s", "cores": 1,
                  "sample": "first %d nets of the workload, same schedule" % sub.num_nets}
        log("cpu oracle single thread: %d nets in %.1fs" % (sub.num_nets, ds))
    return {"value": inst.num_nets * R_ROUNDS * I_ITERS / dt, "unit": "nets/s", "cores": cores, "kind": "oracle",
            "sample": "the whole workload (%d nets), %s schedule: %d iterations x %d rounds, then Elmore" % (
                inst.num_nets, "adjoint-form" if adjoint else "plain-form", I_ITERS, R_ROUNDS),
            "single_thread": single}


if __name__ == "__main__":
    main()
