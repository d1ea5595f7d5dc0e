"""Schedule autotuner for batched propagation.

For a design size class (pins, levels, views, rounded to half octaves) it measures on the
GPU the two ways the library can propagate one design: the persistent schedule (one
workgroup walks every level of one view; the standalone view-schedule time is the time
of one such unit) and the level schedule (one launch per level for all views).  The
measurements are cached per class in a JSON file.  For a batch it then picks the set of
designs that go to the one persistent launch by minimizing the estimated makespan

    max(longest persistent unit, total persistent unit time / workgroups)
        + sum of the level-schedule times of the other designs

over the thresholds of the persistent designs sorted by unit time.
"""
from __future__ import annotations

import json
import math
import os

from . import sta

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sta_schedule_tune.json")


def size_class(pins, levels, views):
    h = lambda x: round(2 * math.log2(max(int(x), 1))) / 2  # noqa: E731
    return f"P{h(pins)}_L{h(levels)}_V{int(views)}"


class Tuner:
    def __init__(self, path=None, reps=3):
        self.path = path or os.environ.get("STA_TUNE_CACHE", DEFAULT_CACHE)
        self.reps = reps
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

    def timings(self, g, lib, views, pi_ts, nd, tm):
        """(persistent unit ms, level-schedule ms) of one design, measured or cached."""
        s = g.sizes
        key = size_class(s["n_pins"], s["n_levels"], views.n_views)
        if key not in self.cache:
            g.set_schedule(1 << 30, True)
            t_view = self._time(lambda: sta.propagate(g, lib, views, pi_ts, nd, out=tm))
            g.set_schedule(0, True)
            t_level = self._time(lambda: sta.propagate(g, lib, views, pi_ts, nd, out=tm))
            g.set_schedule(-1, True)
            self.cache[key] = {"unit_ms": t_view, "level_ms": t_level}
            self.measured += 1
        c = self.cache[key]
        return c["unit_ms"], c["level_ms"]

    @staticmethod
    def plan(unit_ms, level_ms, n_views, workgroups):
        """Schedules (sta.BATCH_PERSISTENT / sta.BATCH_LEVELS) per design and the
        estimated makespan in ms."""
        n = len(unit_ms)
        order = sorted(range(n), key=lambda i: unit_ms[i])
        best, best_k = None, 0
        for k in range(n + 1):
            pers = order[:k]
            rest = order[k:]
            t_p = 0.0
            if pers:
                t_p = max(max(unit_ms[i] for i in pers), sum(unit_ms[i] for i in pers) * n_views / workgroups)
            t = t_p + sum(level_ms[i] for i in rest)
            if best is None or t < best:
                best, best_k = t, k
        sched = [sta.BATCH_LEVELS] * n
        for i in order[:best_k]:
            sched[i] = sta.BATCH_PERSISTENT
        return sched, best
