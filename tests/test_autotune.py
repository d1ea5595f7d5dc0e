"""Host logic of the batch autotuner: size classes, the makespan plan, the cache."""
import itertools
import json

from paper_2203_08395_amd import autotune, sta


def test_size_classes_round_to_half_octaves():
    assert autotune.size_class(5000, 30, 4) == autotune.size_class(5200, 31, 4)
    assert autotune.size_class(5000, 30, 4) != autotune.size_class(9000, 30, 4)
    assert autotune.size_class(5000, 30, 4) != autotune.size_class(5000, 30, 8)


def _brute(span, unit, nv, wg):
    """The estimated makespan minimized over every subset sent to the persistent launch."""
    n = len(span)
    best = None
    for r in range(n + 1):
        for S in itertools.combinations(range(n), r):
            rest = [i for i in range(n) if i not in S]
            t_p = max(max(unit[i] for i in S), sum(unit[i] for i in S) * nv / wg) if S else 0.0
            t = t_p + (max(span[i] for i in rest) if rest else 0.0)
            best = t if best is None else min(best, t)
    return best


def test_plan_minimizes_estimated_makespan():
    # one long design sets the span time; the small ones ride along for free
    span = [0.05, 0.06, 0.05, 0.30]
    unit = [0.10, 0.20, 0.15, 5.0]
    sched, t = autotune.Tuner.plan(span, unit, n_views=4, workgroups=256)
    assert sched == [sta.BATCH_SPANS] * 4
    assert abs(t - 0.30) < 1e-12
    # the longest span design has a short unit: it leaves the span steps
    span = [0.05, 0.06, 0.05, 0.30]
    unit = [1.0, 1.0, 1.0, 0.10]
    sched, t = autotune.Tuner.plan(span, unit, n_views=4, workgroups=256)
    assert sched == [sta.BATCH_SPANS] * 3 + [sta.BATCH_PERSISTENT]
    assert abs(t - (0.10 + 0.06)) < 1e-12
    # the planner's threshold family reaches the subset optimum on these cases
    for span, unit, nv, wg in (([0.1, 0.2, 0.3, 0.4], [0.4, 0.3, 0.2, 0.1], 4, 256),
                               ([0.2] * 6, [0.05] * 6, 4, 4), ([1.0, 0.1], [0.05, 2.0], 8, 16)):
        _, t = autotune.Tuner.plan(span, unit, nv, wg)
        assert t <= _brute(span, unit, nv, wg) + 1e-12


def test_cache_round_trip(tmp_path):
    p = tmp_path / "tune.json"
    t = autotune.Tuner(str(p))
    t.cache["P10.0_L5.0_V4"] = {"spans": [6, 6], "span_ms": 0.5, "unit_ms": 0.7, "by_caps": {"6x6": 0.5}}
    t.save()
    assert json.loads(p.read_text())["P10.0_L5.0_V4"]["spans"] == [6, 6]
    assert autotune.Tuner(str(p)).cache == t.cache
