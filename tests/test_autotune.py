"""Host logic of the batch-schedule autotuner: size classes, the makespan plan, the cache."""
import json

from paper_2203_08395_amd import autotune, sta


def test_size_classes_round_to_half_octaves():
    assert autotune.size_class(5000, 30, 4) == autotune.size_class(5200, 31, 4)
    assert autotune.size_class(5000, 30, 4) != autotune.size_class(9000, 30, 4)
    assert autotune.size_class(5000, 30, 4) != autotune.size_class(5000, 30, 8)


def test_plan_minimizes_estimated_makespan():
    # small designs: cheap as persistent units; the big one: better by levels
    unit = [0.1, 0.2, 0.15, 5.0]
    level = [0.5, 0.6, 0.55, 1.0]
    sched, t = autotune.Tuner.plan(unit, level, n_views=4, workgroups=256)
    assert sched == [sta.BATCH_PERSISTENT] * 3 + [sta.BATCH_LEVELS]
    assert abs(t - (0.2 + 1.0)) < 1e-12
    # exhaustive check over all subsets against the planner's threshold family
    import itertools
    best = min(
        (max([unit[i] for i in S] + [0.0]) if len(S) * 4 <= 256 else 0.0) + sum(level[i] for i in range(4) if i not in S)
        for r in range(5) for S in itertools.combinations(range(4), r))
    assert t <= best + 1e-12
    # many units on few workgroups: the total work term dominates
    sched, t = autotune.Tuner.plan([1.0] * 8, [3.0] * 8, n_views=4, workgroups=4)
    assert t == min(max(1.0, k * 4 / 4) + 3.0 * (8 - k) for k in range(9))


def test_cache_round_trip(tmp_path):
    p = tmp_path / "tune.json"
    t = autotune.Tuner(str(p))
    t.cache["P10.0_L5.0_V4"] = {"unit_ms": 0.5, "level_ms": 0.7}
    t.save()
    assert json.loads(p.read_text())["P10.0_L5.0_V4"]["level_ms"] == 0.7
    assert autotune.Tuner(str(p)).cache == t.cache
