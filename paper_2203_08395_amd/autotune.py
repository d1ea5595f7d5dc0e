"""Tiling and schedule autotuner for batched timing.

Per design size class (pins and levels at half-octave resolution, and the view count) it
measures on the GPU, with the class's first design as the sample:

  * the level-tile size: the longest fused span (gate levels forward, driver levels
    backward; the graph rebuilt with ``sta_build_graph_spans`` for each candidate) that
    gives the shortest forward + backward pass of that design through the fused spans
    (the forward time of the chosen length is what the plan below compares);
  * the persistent schedule's unit time: one workgroup walking every level of one view
    (the standalone view-schedule time of the design).

The measurements are cached per class in a JSON file.  For a batch, ``pick_plan`` times a
family of candidate plans on the batch itself (the designs with the shortest persistent
units sent to the persistent launch, which runs beside the span steps, in growing
fractions) and keeps the fastest, cached per batch composition; when many designs share
the span steps those launches are bound by throughput, not by the longest design, which
the following latency model (``plan``, an estimate reported beside the measurement)
does not capture.  The model picks each design's forward schedule by minimizing

    T_spans + T_persistent,
    T_spans      = the longest span pass among the span designs (the batch's span steps
                   run every span design side by side, so the longest one sets the time),
    T_persistent = max(longest unit, total unit time x views / workgroups),

over the designs sorted by unit time (the shortest units are the candidates for the
persistent launch).
"""
from __future__ import annotations

import json
import math
import os

from . import sta

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sta_tile_tune.json")
SPAN_CANDIDATES = ((4, 4), (6, 6), (8, 8))


def size_class(pins, levels, views):
    h = lambda x: round(2 * math.log2(max(int(x), 1))) / 2  # noqa: E731
    return f"P{h(pins)}_L{h(levels)}_V{int(views)}"


class Tuner:
    def __init__(self, path=None, reps=3, candidates=SPAN_CANDIDATES):
        self.path = path or os.environ.get("STA_TUNE_CACHE", DEFAULT_CACHE)
        self.reps = reps
        self.candidates = tuple(tuple(c) for c in candidates)
        self.cache = {}
        self.measured = 0
        try:
            with open(self.path) as f:
                self.cache = json.load(f)
        except (OSError, ValueError):
            self.cache = {}

    def save(self):
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def _time(self, fn):
        import torch
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(self.reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / self.reps

    def tune(self, g0, design, lib, views, pi_ts, ep_rat):
        """The class record of a design ({"spans": [f, b], "span_ms": forward ms,
        "slack_ms": ..., "unit_ms": ..., "by_caps": {"fxb": [forward ms, slack ms]}}): measured on first sight of its size class, then cached.  g0: the
        design's graph with the default span lengths, uploaded; the other candidates are
        built from ``design`` with ``sta_build_graph_spans``."""
        s = g0.sizes
        key = size_class(s["n_pins"], s["n_levels"], views.n_views)
        if key in self.cache:
            return self.cache[key]

        def span_ms(g):
            """(propagate ms, slack ms) through the fused spans, and the buffers"""
            nd = sta.delay_calc(g)
            tm = sta.alloc_timing(g, views.n_views)
            sl = sta.alloc_slack(g, views.n_views)
            t_f = self._time(lambda: sta.propagate(g, lib, views, pi_ts, nd, out=tm))
            t_b = self._time(lambda: sta.slack(g, views, nd, tm, ep_rat, out=sl))
            return (t_f, t_b), nd, tm

        by_caps = {}
        for caps in self.candidates:
            g = g0 if tuple(caps) == tuple(g0.span_levels) else \
                sta.Graph(design, n_tables=lib.n_tables, span_levels=caps).upload(pi_ts.device)
            by_caps[f"{caps[0]}x{caps[1]}"] = list(span_ms(g)[0])
        _, nd, tm = span_ms(g0)
        g0.set_schedule(1 << 30, True)             # the view walk: one workgroup per view
        unit = self._time(lambda: sta.propagate(g0, lib, views, pi_ts, nd, out=tm))
        g0.set_schedule(-1, True)
        best = min(by_caps, key=lambda k: sum(by_caps[k]))      # the whole pass decides
        rec = {"spans": [int(x) for x in best.split("x")], "span_ms": by_caps[best][0],
               "slack_ms": by_caps[best][1], "unit_ms": unit, "by_caps": by_caps}
        self.cache[key] = rec
        self.measured += 1
        return rec

    def pick_plan(self, classes, unit_ms, make_batch, n_views,
                  fractions=(0.0, 0.25, 0.5, 0.75, 0.875, 1.0), views_per_wave=(1, 2, 4)):
        """Measures candidate plans of a batch; returns (schedules, fwd views per wavefront,
        bwd views per wavefront, the measured times).

        Forward candidate (f, w) sends the round(f * n) designs with the shortest persistent
        units to the persistent launch (beside the span steps) and the others to the span
        steps, w views per span wavefront; backward candidate w is the views per wavefront
        of the backward span steps.  make_batch(schedules) builds the batch.  The measured
        times are cached under the batch's signature (its sorted size classes)."""
        import hashlib
        sig = "plan_" + hashlib.sha1("|".join(sorted(classes)).encode()).hexdigest()[:16]
        n = len(unit_ms)
        order = sorted(range(n), key=lambda i: unit_ms[i])
        ws = [w for w in views_per_wave if w <= n_views and n_views % w == 0]

        def sched_of(f):
            k = int(round(f * n))
            sc = [sta.BATCH_SPANS] * n
            for i in order[:k]:
                sc[i] = sta.BATCH_PERSISTENT
            return sc
        if sig not in self.cache:
            fwd, bwd = {}, {}
            for f in fractions:
                b = make_batch(sched_of(f))
                for w in ws:
                    b.set_tiling(w, min(2, n_views))
                    fwd[f"{f:g}/{w}"] = self._time(lambda: b.propagate(use_graph=True))
                if f == fractions[0]:
                    for w in ws:
                        b.set_tiling(1, w)
                        bwd[str(w)] = self._time(lambda: b.slack(use_graph=True))
                del b
            self.cache[sig] = {"forward_ms": fwd, "slack_ms": bwd}
            self.measured += 1
        rec = self.cache[sig]
        bf = min(rec["forward_ms"], key=rec["forward_ms"].get)
        bb = min(rec["slack_ms"], key=rec["slack_ms"].get)
        f, w = bf.split("/")
        return sched_of(float(f)), int(w), int(bb), rec

    @staticmethod
    def plan(span_ms, unit_ms, n_views, workgroups):
        """Forward schedule per design (sta.BATCH_SPANS or sta.BATCH_PERSISTENT) and the
        estimated makespan in ms."""
        n = len(span_ms)
        order = sorted(range(n), key=lambda i: unit_ms[i])
        best, best_k = None, 0
        for k in range(n + 1):
            pers, rest = order[:k], order[k:]
            t_p = 0.0
            if pers:
                t_p = max(max(unit_ms[i] for i in pers), sum(unit_ms[i] for i in pers) * n_views / workgroups)
            t = t_p + (max(span_ms[i] for i in rest) if rest else 0.0)
            if best is None or t < best - 1e-12:
                best, best_k = t, k
        sched = [sta.BATCH_SPANS] * n
        for i in order[:best_k]:
            sched[i] = sta.BATCH_PERSISTENT
        return sched, best
