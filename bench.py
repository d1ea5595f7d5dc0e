"""Benchmark: levelized STA of the 1M-pin design on one MI355X.

A step is one pass of the whole timing path over the resident design: RC delay
calculation (FP64 moments), forward propagation of the late and early views, and the
backward required-time/slack pass with WNS/TNS.  The graph build (levelization and
layout, host code, once per design) and the upload are outside the timed region and
reported separately.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pin-updates/s at 1M pins (bit-exact) + %HBM roofline; surrogate vs exact speedup"
HBM_PEAK_GBS = 8000.0


def fwd_bytes_per_pass(G, A, n_views):
    """Algorithmic bytes of the forward pass: per gate 17 B for the first view (arc
    pointer 4, load 4, arrival+slew out 8, argmax 1: it is stored as one byte) and 9 B for
    each further view; per arc 34 B for the first view (driver id, gathered arrival+slew,
    net delay+spread, table id, input-pin arrival+slew, arc delay) and 20 B for each
    further view."""
    return (17 + 9 * (n_views - 1)) * G + (34 + 20 * (n_views - 1)) * A


def bwd_bytes_per_pass(D, A, n_views):
    """Per sink arc: its id 4, gathered RAT of the gate output 4, arc delay 4, net delay 4,
    input-pin arrival 4, required time and slack out 8 (28 B), and 20 B for each further
    view (all but the id and the net delay); per driver: arrival 4, required time and slack
    out 8, sink pointer 4 (16 B), and 12 B for each further view."""
    return (28 + 20 * (n_views - 1)) * A + (16 + 12 * (n_views - 1)) * D


def dc_bytes(D, A, M):
    """Per driver: node pointer, sink pointer, load (12 B); per node R, C, parent (10 B);
    per sink: arc id, tap, pin cap, net delay, spread (17 B)."""
    return 12 * D + 10 * M + 17 * A


def cpu_model():
    """Model name of the host processor (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the event-bracketed pass (for counter-collection runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="first run one plain device copy of MB megabytes (a known-size reference "
                         "dispatch for HBM byte counters)")
    ap.add_argument("--schedule", choices=["auto", "span", "level", "level_plain", "view"], default="auto",
                    help="auto: the library's choice (fused spans for wide levels); level: one launch per "
                         "level; level_plain: the same without hipGraph replay")
    ap.add_argument("--surrogate-nets", type=int, default=1_000_000,
                    help="RC-tree nets of the learned-surrogate comparison (0: skip it)")
    ap.add_argument("--surrogate-train-steps", type=int, default=3000)
    ap.add_argument("--batch-designs", type=int, default=64,
                    help="designs of the batched-corners comparison (0: skip it)")
    ap.add_argument("--only", choices=["surrogate", "batched"], default=None,
                    help="run one side comparison alone and print its JSON object")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (one design on one GPU); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_08395_amd import gen, sta

    if args.only:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        if args.only == "surrogate":
            print(json.dumps(surrogate_bench(dev, args.surrogate_nets, args.surrogate_train_steps)), flush=True)
        else:
            print(json.dumps(batch_bench(dev, args.batch_designs)), flush=True)
        return

    name = args.workload
    cfg = gen.CONFIGS[name]
    t0 = time.perf_counter()
    d = gen.make_design(**cfg)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, cfg["n_levels"], **gen.RAT_PARAMS[name])
    t_gen = time.perf_counter() - t0

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    g = sta.Graph(d, n_tables=lib.n_tables)
    t_build = time.perf_counter() - t0
    if args.schedule != "auto":
        g.set_schedule(1 << 30 if args.schedule == "view" else 0, args.schedule != "level_plain")
        g.set_level_fusion(args.schedule == "span")
    t0 = time.perf_counter()
    g.upload(dev)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t0
    s = g.sizes
    D, A, G, M, E, L = (s[k] for k in ("n_drivers", "n_arcs", "n_gates", "n_nodes", "n_endpoints", "n_levels"))
    modes = [sta.STA_LATE, sta.STA_EARLY]
    V = len(modes)
    L_lib = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).to(dev))
    views = sta.make_views(modes)
    pi = np.zeros((d.n_pi, V, 2), np.float32)
    pi[:, :, 0] = pa[:, None]
    pi[:, :, 1] = ps[:, None]
    pi_t = torch.from_numpy(pi).to(dev)
    rat = np.stack([late, early], axis=1).astype(np.float32)
    rat_t = torch.from_numpy(rat).to(dev)
    nd = sta.alloc_net(g)
    tm = sta.alloc_timing(g, V)
    sl = sta.alloc_slack(g, V)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        sta.delay_calc(g, sta.STA_DC_FP64, out=nd)
        sta.propagate(g, L_lib, views, pi_t, nd, out=tm)
        sta.slack(g, views, nd, tm, rat_t, out=sl)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: wall clock over K steps, and HIP events on the same stream around
    # each library call of every step (per-call device time)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        e = ev[k]
        e[0].record()
        sta.delay_calc(g, sta.STA_DC_FP64, out=nd)
        e[1].record()
        sta.propagate(g, L_lib, views, pi_t, nd, out=tm)
        e[2].record()
        sta.slack(g, views, nd, tm, rat_t, out=sl)
        e[3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    call_ms = {name: float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(args.steps)]))
               for i, name in enumerate(("delay_calc", "propagate", "slack"))}
    if args.no_profile:
        print(json.dumps({"ms_per_step": ms_step, "call_ms": call_ms, "note": "counter run"}), flush=True)
        return

    # which kernels each call launches and their durations (library instrumentation:
    # HIP events around every launch, eager launches; three extra untimed steps, averaged)
    launches = {}
    n_prof = 3
    for _ in range(n_prof):
        for call, fn in (("delay_calc", lambda: sta.delay_calc(g, sta.STA_DC_FP64, out=nd)),
                         ("propagate", lambda: sta.propagate(g, L_lib, views, pi_t, nd, out=tm)),
                         ("slack", lambda: sta.slack(g, views, nd, tm, rat_t, out=sl))):
            sta.profile_begin()
            fn()
            for k, (n, ms) in sta.profile_end().items():
                n0, ms0 = launches.setdefault(call, {}).get(k, (0, 0.0))
                launches[call][k] = (n0 + n / n_prof, ms0 + ms / n_prof)
    torch.cuda.synchronize()

    updates = (s["n_pins"] - d.n_pi) * V
    value = updates / (ms_step * 1e-3)
    # algorithmic bytes of one step by pass, and of each timing kernel: the fused-span
    # kernels cover the gates/arcs (drivers/sink arcs) of the fused spans, each counted
    # once; the level kernels the rest.  A kernel's device time per step is its call's
    # time in the timed region (HIP events on the library's stream), apportioned among the
    # call's kernels by the HIP events the library records around each launch in the
    # instrumented steps; its average launch duration is that time over its launches.
    fam_bytes = {"forward": fwd_bytes_per_pass(G, A, V), "backward": bwd_bytes_per_pass(D, A, V),
                 "delay_calc": dc_bytes(D, A, M)}
    kstats = {k: v for d_ in launches.values() for k, v in d_.items()}
    sp = g.spans
    b_fs = fwd_bytes_per_pass(sp["fwd_span_gates"], sp["fwd_span_arcs"], V) if "k_forward_span" in kstats else 0
    b_bs = (bwd_bytes_per_pass(sp["bwd_span_drivers"], sp["bwd_span_arcs"], V)
            if "k_backward_span" in kstats else 0)
    kbytes = {"k_delay_calc": fam_bytes["delay_calc"],
              "k_forward_span": b_fs, "k_forward": fam_bytes["forward"] - b_fs,
              "k_forward_view": fam_bytes["forward"],
              "k_backward_span": b_bs, "k_backward": fam_bytes["backward"] - b_bs}
    kernels = {}
    for call, ks in launches.items():
        ev_total = sum(ms for _, ms in ks.values())
        for kname, (n, ev_ms) in ks.items():
            n = int(round(n))
            if kname not in kbytes or n == 0:
                continue
            ms = call_ms[call] * ev_ms / ev_total
            kernels[kname] = {"launches_per_step": n, "avg_us": 1e3 * ms / n, "ms_per_step": ms,
                              "instrumented_avg_us": 1e3 * ev_ms / n,
                              "bytes_per_launch": kbytes[kname] / n,
                              "GB_s": kbytes[kname] / (ms * 1e-3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    dk = kernels[dom]
    achieved = dk["GB_s"]
    traffic = measured_traffic(dom)
    ms_prop = call_ms["propagate"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: seeded levelized DAG, {s['n_pins']} pins, {L} levels, "
                               f"geometric fanin (mean 2.5, max 16), 16 fanout-64 nets, RC chains 2-8 nodes, "
                               f"128 NLDM 7x7 table pairs, late+early views; FP32 propagation, FP64 RC moments",
                   "pins": s["n_pins"], "primary_inputs": d.n_pi, "gates": G, "arcs": A, "rc_nodes": M,
                   "levels": L, "endpoints": E, "views": ["late", "early"],
                   "step": "delay_calc + propagate(late,early) + slack(late,early)"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": dk["bytes_per_launch"], "avg_launch_us": dk["avg_us"],
                     "launches_per_step": dk["launches_per_step"]},
        "propagate_ms": ms_prop,
        "call_ms": call_ms,
        "propagate_pin_updates_per_s": updates / (ms_prop * 1e-3),
        "kernels": kernels,
        "fusion_plan": sp,
        "algorithmic_bytes_per_step": fam_bytes,
        "pass_GB_s": sum(fam_bytes.values()) / (ms_step * 1e-3) / 1e9,
        "schedule": ("view" if "k_forward_view" in kstats else "span" if "k_forward_span" in kstats else "level")
                    + ("" if args.schedule == "auto" else f" (forced {args.schedule})"),
        "host": {"generate_s": t_gen, "build_graph_s": t_build, "upload_s": t_upload,
                 "graph_bytes": s["graph_bytes"], "nproc": os.cpu_count(), "cpu_model": cpu_model()},
    }

    # cold caches: a 1 GiB write between steps evicts L2 and the 256 MB Infinity Cache;
    # and a plain 1 GiB device copy as the achievable-bandwidth reference
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(3):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    dst = torch.empty_like(flush)
    ms_copy = _time_ms(lambda: dst.copy_(flush), reps=5)
    out["cold_ms_per_step"] = float(np.median(cold))
    out["copy_GB_s"] = 2 * flush.numel() * 4 / (ms_copy * 1e-3) / 1e9
    del flush, dst
    # analyses on the same timed design: TNS adjoint (both views) and the 64 worst paths
    adj = sta.alloc_adjoint(g, V)
    out["adjoint"] = {"ms": _time_ms(lambda: sta.tns_adjoint(g, L_lib, views, nd, tm, sl, out=adj)),
                      "what": "dTNS/d(arc delay, net delay, AT, load) for late and early"}
    out["critical_paths"] = {"ms": _time_ms(lambda: sta.critical_paths(g, views, 0, 64, tm, sl)),
                             "what": "64 worst late endpoints and their argmax paths"}
    if args.batch_designs > 0:
        out["batched"] = batch_bench(dev, args.batch_designs)
    if args.surrogate_nets > 0:
        out["surrogate"] = surrogate_bench(dev, args.surrogate_nets, args.surrogate_train_steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, lib, pa, ps, late, early, updates, args.cpu_seconds, g, nd, tm, sl)
    print(json.dumps(out), flush=True)


def _time_ms(fn, reps=5, warm=2):
    import torch
    for _ in range(warm):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_bench(dev, n_designs, reps=5):
    """Uneven designs x 4 corners, the whole timing pass (RC delay calculation, forward
    propagation, required times and slack): the single-design calls looped over the
    designs vs the batch (span steps for the designs the autotuner plans there, the
    persistent unit queue for the rest, every design built with its size class's tuned
    span length), each replayed from captured launch sequences."""
    import torch
    from paper_2203_08395_amd import autotune, gen, sta
    specs = gen.c3_designs(n_designs)
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    L_lib = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).to(dev))
    V = len(gen.CORNER_KAPPAS)
    views = sta.make_views([sta.STA_LATE] * V, list(range(V)))
    t0 = time.perf_counter()
    designs, loop_e = [], []
    pins = updates = nbytes = 0
    for sp in specs:
        d = gen.make_design(**sp)
        g = sta.Graph(d, n_tables=lib.tab.shape[1]).upload(dev)
        pa, ps = gen.make_pi(d)
        pi = np.zeros((max(d.n_pi, 1), V, 2), np.float32)
        pi[:d.n_pi, :, 0] = pa[:, None]
        pi[:d.n_pi, :, 1] = ps[:, None]
        E = g.sizes["n_endpoints"]
        nd, tm, sl = sta.alloc_net(g), sta.alloc_timing(g, V), sta.alloc_slack(g, V)
        pi_t = torch.from_numpy(pi).to(dev)
        # required time: the 90th percentile of the endpoint arrivals of each corner
        sta.delay_calc(g, out=nd)
        sta.propagate(g, L_lib, views, pi_t, nd, out=tm)
        at_ep = tm["drv_ts"][torch.from_numpy(g.ep_driver.astype(np.int64)).to(dev), :, 0]
        rat = torch.zeros((max(E, 1), V), dtype=torch.float32, device=dev)
        if E:
            rat[:E] = torch.quantile(at_ep, 0.9, dim=0)[None, :]
        designs.append(d)
        loop_e.append((g, pi_t, nd, tm, sl, rat))
        pins += d.n_pins
        updates += (d.n_pins - d.n_pi) * V
        s = g.sizes
        nbytes += dc_bytes(s["n_drivers"], s["n_arcs"], s["n_nodes"]) + \
            fwd_bytes_per_pass(s["n_gates"], s["n_arcs"], V) + bwd_bytes_per_pass(s["n_drivers"], s["n_arcs"], V)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0

    def loop():
        for g, pi, nd, tm, sl, rat in loop_e:
            sta.delay_calc(g, out=nd)
            sta.propagate(g, L_lib, views, pi, nd, out=tm)
            sta.slack(g, views, nd, tm, rat, out=sl)

    ms_loop = _time_ms(loop, reps=reps)
    ref = [(e[3]["drv_ts"].clone(), e[3]["arc_ts"].clone(), e[4]["drv_slack"].clone(), e[4]["arc_slack"].clone(),
            e[4]["tns"].clone(), e[4]["wns"].clone(), e[2]["net_delay"].clone()) for e in loop_e]
    # autotuning: span length per size class, then the forward schedule per design
    tuner = autotune.Tuner()
    t0 = time.perf_counter()
    recs = [tuner.tune(e[0], d, L_lib, views, e[1], e[5]) for d, e in zip(designs, loop_e)]
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    _, est = autotune.Tuner.plan([r["span_ms"] for r in recs], [r["unit_ms"] for r in recs], V, n_cu)
    graphs = []
    for d, e, r in zip(designs, loop_e, recs):
        caps = tuple(r["spans"])
        g = e[0] if caps == tuple(e[0].span_levels) else sta.Graph(d, n_tables=lib.tab.shape[1], span_levels=caps).upload(dev)
        graphs.append((g, e[1], sta.alloc_net(g), sta.alloc_timing(g, V), e[5], sta.alloc_slack(g, V)))
    for g, pi, nd, *_ in graphs:
        sta.delay_calc(g, out=nd)

    def make_batch(sched_):
        return sta.Batch([(x[0], x[1], x[2], x[3], sc, x[4], x[5]) for x, sc in zip(graphs, sched_)], L_lib, views)
    classes = [autotune.size_class(e[0].sizes["n_pins"], e[0].sizes["n_levels"], V) for e in loop_e]
    sched, fwd_nw, bwd_nw, plan_ms = tuner.pick_plan(classes, [r["unit_ms"] for r in recs], make_batch, V)
    t_tune = time.perf_counter() - t0
    try:
        tuner.save()
    except OSError:
        pass
    entries = [(x[0], x[1], x[2], x[3], sc, x[4], x[5]) for x, sc in zip(graphs, sched)]
    b = sta.Batch(entries, L_lib, views).set_tiling(fwd_nw, bwd_nw)

    def batched():
        b.delay_calc()
        b.propagate()
        b.slack()

    ms_batch = _time_ms(batched, reps=reps)
    ms_dc = _time_ms(b.delay_calc, reps=reps)
    ms_fwd = _time_ms(b.propagate, reps=reps)
    ms_bwd = _time_ms(b.slack, reps=reps)
    same = all(torch.equal(r[0], e[3]["drv_ts"]) and torch.equal(r[1], e[3]["arc_ts"]) and
               torch.equal(r[2], e[6]["drv_slack"]) and torch.equal(r[3], e[6]["arc_slack"]) and
               torch.equal(r[4], e[6]["tns"]) and torch.equal(r[5], e[6]["wns"]) and
               torch.equal(r[6], e[2]["net_delay"]) for r, e in zip(ref, entries))
    info = b.info()
    # the previous batched design for reference: every design's forward pass as persistent
    # units (each (design, corner) walked by one workgroup)
    bp = sta.Batch([(e[0], e[1], e[2], e[3], sta.BATCH_PERSISTENT) for e in entries], L_lib, views)
    ms_fwd_pers = _time_ms(bp.propagate, reps=reps)
    caps_used = {}
    for r in recs:
        k = f"{r['spans'][0]}x{r['spans'][1]}"
        caps_used[k] = caps_used.get(k, 0) + 1
    achieved = nbytes / (ms_batch * 1e-3) / 1e9
    return {
        "workload": f"{len(specs)} seeded designs, pins log-uniform 5k-500k (sum {pins}), levels 30*sqrt(P/5k), "
                    f"x {V} corners (tables scaled {list(gen.CORNER_KAPPAS)}), late; delay calc + propagate + "
                    f"slack per step, FP32 timing, FP64 moments",
        "pins": pins, "pin_updates": updates,
        "loop_ms": ms_loop, "batched_ms": ms_batch, "speedup_vs_loop": ms_loop / ms_batch,
        "batched_split_ms": {"delay_calc": ms_dc, "propagate": ms_fwd, "slack": ms_bwd},
        "propagate_all_persistent_ms": ms_fwd_pers,
        "loop_pin_updates_per_s": updates / (ms_loop * 1e-3),
        "batched_pin_updates_per_s": updates / (ms_batch * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "bytes_per_step": nbytes},
        "plan": info,
        "autotune": {"measured": tuner.measured, "seconds": t_tune, "span_lengths": caps_used,
                     "views_per_wavefront": {"forward": fwd_nw, "backward": bwd_nw},
                     "candidates_ms": plan_ms,
                     "latency_model_forward_ms": est, "cache": tuner.path},
        "bitwise_equal_to_loop": bool(same),
        "setup_s": t_setup,
    }


def surrogate_bench(dev, n_nets, train_steps, tol_ps=1.0):
    """Exact RC-tree moments vs the learned surrogate on n_nets random RC trees (2-64 nodes):
    the network is trained on the GPU on the sinks of the first 80% of the nets, calibrated
    on the next 10% and judged on the last 10%; speeds are for all nets."""
    import torch
    from paper_2203_08395_amd import gen, surrogate as sur
    t0 = time.perf_counter()
    T = gen.make_rc_trees(n_nets, seed=4)
    tr = sur.Trees(T, dev)
    t_gen = time.perf_counter() - t0
    N, S, M = T.n_nets, T.n_sinks, T.n_nodes
    data = sur.dataset(tr)
    torch.cuda.synchronize()
    tr.check_status()
    n_tr, n_cal = int(0.8 * N), int(0.9 * N)
    s_tr, s_cal = int(T.sink_ptr[n_tr]), int(T.sink_ptr[n_cal])
    feat, target = data["feat"], data["target"]
    norm = sur.norm_stats(feat[:s_tr])
    model = sur.Model(sur.init_params(0), norm, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = sur.train(model, feat, target, np.arange(s_tr), steps=train_steps, batch=8192, lr=3e-3, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    y = sur.predict(model, feat)
    sur.calibrate(model, feat[s_tr:s_cal], target[s_tr:s_cal], y[s_tr:s_cal], quantile=0.999, min_count=256)
    buf = sur.EvalBuffers(tr)
    d_ex = torch.empty(S, dtype=torch.float32, device=dev)
    s_ex = torch.empty(S, dtype=torch.float32, device=dev)
    ms_exact = _time_ms(lambda: sur.exact(tr, d_ex, s_ex))
    ms_sur = _time_ms(lambda: sur.evaluate(tr, model, feat, tol_ps, buf))
    ms_net = _time_ms(lambda: sur.predict(model, feat, y))
    feat2 = torch.empty_like(feat)
    ms_feat = _time_ms(lambda: sur.features(tr, feat2))
    same_feat = bool(torch.equal(feat2, feat))

    def end_to_end():
        sur.features(tr, feat2)
        sur.evaluate(tr, model, feat2, tol_ps, buf)
    ms_e2e = _time_ms(end_to_end)
    torch.cuda.synchronize()
    tr.check_status()
    served = 1.0 - int(buf.count.item()) / N
    # errors on the held-out test nets
    f = feat[s_cal:].cpu().numpy()
    yt = y[s_cal:].cpu().numpy()
    exd, exs = data["delay"][s_cal:].cpu().numpy(), data["slew"][s_cal:].cpu().numpy()
    L, U = f[:, 0] * f[:, 2] * 1e-3, f[:, 0] * f[:, 1] * 1e-3
    e_net = np.abs(L + np.clip(yt[:, 0], 0, 1) * (U - L) - exd)
    e_mid = np.abs(0.5 * (L + U) - exd)
    flag = buf.flag.cpu().numpy()
    sink_net = np.repeat(np.arange(N), np.diff(T.sink_ptr))
    trusted = ~flag[sink_net[s_cal:]].astype(bool)
    ed = np.abs(buf.delay[s_cal:].cpu().numpy() - exd)[trusted]
    es = np.abs(buf.slew[s_cal:].cpu().numpy() - exs)[trusted]
    exact_bytes = 12 * M + 16 * S + 12 * N
    net_bytes = 56 * S
    net_flops = 9984 * S
    feat_bytes = 12 * M + 8 * S + 52 * S + 12 * N    # node R/C/parent, sink node/cap, 48 B out, net data
    net_hbm = net_bytes / (ms_net * 1e-3) / 1e9
    net_mfma = net_flops / (ms_net * 1e-3) / 1e12
    return {
        "workload": f"{N} random recursive RC trees, 2-64 nodes (R 10-500 ohm, C 0.1-5 fF), {S} sinks "
                    f"(leaves), 12 features per sink -> MLP 12-64-64-2, BF16 operands / FP32 accumulate",
        "nets": N, "sinks": S, "rc_nodes": M, "tol_ps": tol_ps,
        "exact_ms": ms_exact,
        "end_to_end_ms": ms_e2e, "end_to_end_speedup_vs_exact": ms_exact / ms_e2e,
        "end_to_end": "features (k_tree_features, no moment sweeps) + network, decode, error bound and "
                      "exact fallback of the untrusted nets (sta_surrogate_eval)",
        "features_ms": ms_feat, "features_bitwise_equal_to_dataset": same_feat,
        "surrogate_on_resident_features_ms": ms_sur, "speedup_vs_exact_on_resident_features": ms_exact / ms_sur,
        "nets_served_by_network": served,
        "network_only_ms": ms_net, "network_only_speedup_vs_exact": ms_exact / ms_net,
        "exact_GB_s": exact_bytes / (ms_exact * 1e-3) / 1e9,
        "features_GB_s": feat_bytes / (ms_feat * 1e-3) / 1e9,
        "network_GB_s": net_hbm, "network_TFLOP_s": net_mfma,
        "network_roofline": {"bytes_per_sink": 56, "flops_per_sink": 9984,
                             "hbm_frac": net_hbm / HBM_PEAK_GBS, "mfma_bf16_frac": net_mfma / 2500.0,
                             "bound": "hbm" if net_bytes / 8e12 > net_flops / 2.5e15 else "mfma"},
        "test_delay_rms_ps": {"network": float(np.sqrt(np.mean(e_net ** 2))),
                              "elmore_bound_midpoint": float(np.sqrt(np.mean(e_mid ** 2)))},
        "test_sinks_within_tol": {"network": float(np.mean(e_net <= tol_ps)),
                                  "elmore_bound_midpoint": float(np.mean(e_mid <= tol_ps))},
        "test_trusted_sinks": int(trusted.sum()),
        "test_trusted_max_err_ps": {"delay": float(ed.max()) if ed.size else 0.0,
                                    "slew": float(es.max()) if es.size else 0.0},
        "train": {"steps": train_steps, "batch": 8192, "seconds": t_train, "loss_first": float(losses[0]),
                  "loss_last": float(np.mean(losses[-50:]))},
        "generate_s": t_gen,
    }


def kernel_source_sha256():
    """sha256 over the span and delay-calculation kernels' source and the header that holds
    their tiling constants, in that order."""
    import hashlib
    h = hashlib.sha256()
    for f in ("sta_kernels.hip", "sta_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2203_08395_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs (FETCH_SIZE and
    WRITE_SIZE scaled by a known-size copy), or None when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_c2.json")
    try:
        rec = json.load(open(path))
        if kernel_source_sha256() != rec["source_sha256"]:
            return None
        return rec["kernels"][kernel]["bytes_per_dispatch"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(d, lib, pa, ps, late, early, updates, budget_s, g, nd, tm, sl):
    """The oracle as it stands over whole passes of the same workload, timed twice: the
    OpenMP build on the host's cores (level by level, each level's gates in parallel; the
    reported value) and the serial build on one core.  Each leg gets half the budget; the
    last results of both are compared bit for bit with the GPU's."""
    import oracle

    def leg(par, seconds):
        t_pass, res = [], None
        t_all = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            res = oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY), par=par)
            t_pass.append(time.perf_counter() - t0)
            if time.perf_counter() - t_all > seconds or len(t_pass) >= 200:
                break
        return float(np.median(t_pass)), len(t_pass), res

    cores = oracle.threads()
    sec_par, n_par, res_par = leg(True, 0.5 * budget_s)
    sec_1, n_1, res_1 = leg(False, 0.5 * budget_s)
    D, A = d.n_drivers, d.n_arcs
    h = {k: v.cpu().numpy() for k, v in list(nd.items()) + list(tm.items()) + list(sl.items()) if k != "scratch"}

    def same_as_gpu(res):
        chk = [(g.drv_to_input(h["load"][:D]), res["load"]), (g.arc_to_input(h["net_delay"][:A]), res["net_delay"])]
        for v, m in enumerate(("late", "early")):
            r = res[m]
            chk += [(g.drv_to_input(h["drv_ts"][:D, v, 0]), r["at_drv"]), (g.drv_to_input(h["drv_ts"][:D, v, 1]), r["slew_drv"]),
                    (g.arc_to_input(h["arc_ts"][:A, v, 0]), r["at_in"]), (g.arc_to_input(h["arc_delay"][:A, v]), r["arc_delay"]),
                    (g.drv_to_input(h["drv_slack"][:D, v]), r["slack_drv"]), (g.arc_to_input(h["arc_slack"][:A, v]), r["slack_in"]),
                    (np.array([h["tns"][v]]), np.array([r["tns"]]))]
        return all(np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))
                   for a, b in chk)

    return {"value": updates / sec_par, "unit": "pin-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_par} whole passes of the same workload (delay calc + late/early propagate + slack), "
                      f"median {sec_par * 1e3:.1f} ms per pass, the oracle's OpenMP build (gcc -O2 -fopenmp) on "
                      f"{cores} threads, level by level",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_core": {"value": updates / sec_1, "unit": "pin-updates/s", "cores": 1,
                            "sample": f"{n_1} whole passes, median {sec_1 * 1e3:.1f} ms per pass, serial build"},
            "gpu_bitwise_equal": bool(same_as_gpu(res_par) and same_as_gpu(res_1))}


if __name__ == "__main__":
    main()
