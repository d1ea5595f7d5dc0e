"""Parity of the HIP path (through the C ABI) with the CPU oracle, bit for bit: RC delay
calculation (FP64 mode), forward arrival/slew/arc delay/argmax, backward required times,
slacks, WNS and TNS, in every view."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests import tiny
from tests.gpu_common import EARLY, LATE, assert_bitwise, compare_all, gpu_run, say, workload

pytestmark = pytest.mark.gpu

SCHED = pytest.mark.parametrize("schedule", ["span", "level", "level_plain", "view"])


@SCHED
def test_c1_late_and_early(schedule):
    d, lib, pa, ps, late, early = workload("c1")
    compare_all(d, lib, pa, ps, [late, early], [LATE, EARLY], label="c1 10k pins", schedule=schedule)


@SCHED
@pytest.mark.parametrize("seed", range(12))
def test_random_tiny_designs(seed, schedule):
    from tests.test_oracle_graph import _random_tiny
    d, lib, pa, ps = _random_tiny(seed)
    ep = oracle.endpoints(d)
    rng = np.random.default_rng(seed)
    rat = [rng.uniform(0, 2000, ep.size).astype(np.float32) for _ in range(2)]
    compare_all(d, lib, pa, ps, rat, [LATE, EARLY], label=f"tiny seed {seed}", schedule=schedule)


@SCHED
@pytest.mark.parametrize("nv", [1, 2, 4, 8])
def test_view_counts_and_corners(nv, schedule):
    d = gen.make_design(n_pins=30000, n_levels=40, fanin="geom", seed=21, n_fanout64=2)
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    pa, ps = gen.make_pi(d, seed=5)
    late, early = gen.make_rat(d, 40, late_per_level=70.0, hold=120.0)
    modes = [LATE if v % 2 == 0 else EARLY for v in range(nv)]
    # two views on two corners: two distinct table sets in one launch
    sets = [1, 3] if nv == 2 else [(v // 2) % 4 for v in range(nv)]
    rats = [late if m == LATE else early for m in modes]
    compare_all(d, lib, pa, ps, rats, modes, sets, label=f"{nv} views over corners", schedule=schedule)


@SCHED
def test_ragged_tiles_and_extremes(schedule):
    # fanin 64 (a full wavefront), a 200-sink net (a backward tile of several passes),
    # a 256-node RC tree and a one-gate level between wide ones
    rng = np.random.default_rng(3)
    n_pi = 70
    gates = [list(range(64))]                                   # gate 0: fanin 64
    gates += [[int(x)] for x in rng.integers(0, n_pi, 200)]     # gates 1..200
    gates += [[0] + [n_pi + 1 + i for i in range(3)]]           # one deeper gate
    gates += [[n_pi] * 1 for _ in range(200)]                   # 200 sinks on gate 0's output
    nets = []
    for u in range(n_pi + len(gates)):
        m = 256 if u == 5 else int(rng.integers(2, 9))
        parent = [-1] + [int(rng.integers(0, k)) for k in range(1, m)]
        nets.append((parent, [0.0] + list(rng.uniform(10, 500, m - 1)), list(rng.uniform(0.1, 5, m))))
    A = sum(len(x) for x in gates)
    taps = []
    sizes = [len(n[0]) for n in nets]
    for ins in gates:
        for u in ins:
            taps.append(int(rng.integers(0, sizes[u])))
    d = tiny.design(n_pi, gates, nets, pincaps=list(rng.uniform(1, 4, A)), tables=list(rng.integers(0, 128, A)),
                    taps=taps)
    lib = gen.make_library()
    pa = rng.uniform(0, 50, n_pi).astype(np.float32)
    ps = rng.uniform(5, 50, n_pi).astype(np.float32)
    ep = oracle.endpoints(d)
    rat = [rng.uniform(100, 900, ep.size).astype(np.float32) for _ in range(2)]
    compare_all(d, lib, pa, ps, rat, [LATE, EARLY], label="ragged tiles and extremes", schedule=schedule)


@SCHED
@pytest.mark.parametrize("seed,n_tables", [(5, 128), (6, 129)])
def test_drivers_wider_than_a_tile(seed, n_tables, schedule):
    # two drivers with 100+ sinks: their backward levels cannot be tiled and run as level
    # launches between fused spans; an odd table count (sets not a whole number of 16-byte
    # pieces) keeps the forward span's table reads in global memory
    d = tiny.wide_fanout_design(seed)
    lib = gen.make_library(n_tables=n_tables)
    rng = np.random.default_rng(seed)
    pa = rng.uniform(0, 50, d.n_pi).astype(np.float32)
    ps = rng.uniform(5, 50, d.n_pi).astype(np.float32)
    ep = oracle.endpoints(d)
    rat = [rng.uniform(200, 1500, ep.size).astype(np.float32) for _ in range(2)]
    compare_all(d, lib, pa, ps, rat, [LATE, EARLY], label=f"wide drivers seed {seed}", schedule=schedule)


def test_delay_calc_crowded_wavefront():
    # nets of at most 8 nodes: a lane per net of up to 16 sinks, a wavefront per wider net.
    # The first 64 drivers (one wavefront of the lane path) include 20 nets of 60 sinks, so
    # the wavefront's sink range is longer than the lane path stages in LDS and its narrow
    # nets read their sinks from memory; nets of exactly 16 and 17 sinks sit on either side
    # of the lane path's limit, and a later wavefront with nets of 9..16 sinks is staged.
    rng = np.random.default_rng(17)
    n_pi = 200
    fo = np.zeros(n_pi, np.int64)
    fo[:20] = 60
    fo[20:40] = rng.integers(9, 17, 20)
    fo[40], fo[41] = 16, 17
    fo[42:64] = rng.integers(0, 4, 22)
    fo[64:128] = rng.integers(9, 17, 64)
    fo[128:] = rng.integers(0, 5, n_pi - 128)
    pins = np.repeat(np.arange(n_pi), fo)
    rng.shuffle(pins)
    gates = [list(map(int, pins[i:i + 8])) for i in range(0, pins.size, 8)]
    D = n_pi + len(gates)
    nets, sizes = [], []
    for u in range(D):
        m = int(rng.integers(1, 9))
        parent = [-1] + [int(rng.integers(0, k)) if rng.random() < 0.5 else k - 1 for k in range(1, m)]
        nets.append((parent, [0.0] + list(rng.uniform(10, 400, m - 1)), list(rng.uniform(0.1, 4, m))))
        sizes.append(m)
    A = sum(len(x) for x in gates)
    taps = [int(rng.integers(0, sizes[u])) for ins in gates for u in ins]
    d = tiny.design(n_pi, gates, nets, pincaps=list(rng.uniform(0.5, 4, A)), tables=list(rng.integers(0, 128, A)),
                    taps=taps)
    lib = gen.make_library()
    pa = rng.uniform(0, 50, n_pi).astype(np.float32)
    ps = rng.uniform(5, 50, n_pi).astype(np.float32)
    ep = oracle.endpoints(d)
    rat = [rng.uniform(100, 900, ep.size).astype(np.float32) for _ in range(2)]
    compare_all(d, lib, pa, ps, rat, [LATE, EARLY], label="crowded delay-calculation wavefront")


@SCHED
def test_ties_on_gpu(schedule):
    same = tiny.chain_net([100.0, 50.0], [0.5, 0.5, 0.5])
    one = ([-1], [0.0], [0.4])
    # every primary input drives one sink through the same net: all candidates are equal
    d = tiny.design(8, [[4, 3, 2, 1, 0], [5, 6, 7]], [same] * 8 + [one, one],
                    pincaps=[2.0] * 8, tables=[1] * 8)
    lib = gen.make_library(n_tables=2, seed=3)
    g, h = compare_all(d, lib, np.full(8, 20.0, np.float32), np.full(8, 30.0, np.float32),
                       [np.full(2, 500.0, np.float32)] * 2, [LATE, EARLY], label="equal candidates",
                       schedule=schedule)
    assert np.all(h["argmax"][:2] == 0)


def _sqrt_threshold(p):
    """The least float32 a whose float32 square root reaches p (p > 0 finite), by a walk
    over neighbouring floats from p * p."""
    f32 = np.float32
    p = f32(p)
    t = f32(np.float64(p) * np.float64(p))
    while t > 0 and np.sqrt(np.nextafter(t, f32(0))) >= p:
        t = np.nextafter(t, f32(0))
    while not (np.sqrt(t) >= p):
        t = np.nextafter(t, f32(np.inf))
    return t


@SCHED
def test_slews_at_the_axis_square_roots(schedule):
    """Input slews whose radicand S_u^2 + imp2 lies at, just below and just above the least
    value whose FP32 square root reaches each inner slew axis point, and input slews at and
    next to the axis points: the segment taken, hence every output, is the oracle's, bit for
    bit (the span kernel finds the segment from the radicand before taking the root)."""
    import torch
    from tests.gpu_common import SCHEDULES
    f32 = np.float32
    lib = gen.make_library(n_tables=2, seed=5)
    ni_l1, s_pi = [], []
    for p in lib.x[1:6]:
        T = _sqrt_threshold(p)
        assert np.sqrt(T) >= p and np.sqrt(np.nextafter(T, f32(0))) < p
        for a in (T, np.nextafter(T, f32(0)), np.nextafter(T, f32(np.inf)), f32(p) * f32(p)):
            ni_l1.append(a)
            s_pi.append(f32(0))
        for sv in (f32(p), np.nextafter(f32(p), f32(0)), np.nextafter(f32(p), f32(np.inf))):
            ni_l1.append(f32(0))
            s_pi.append(sv)
    for a in (0.0, 1e-41, 1e-30, 1e12):
        ni_l1.append(f32(a))
        s_pi.append(f32(0))
    rng = np.random.default_rng(17)
    for _ in range(64):
        ni_l1.append(f32(rng.uniform(0, float(lib.x[6]) ** 2)))
        s_pi.append(f32(rng.uniform(0, 1.2 * float(lib.x[6]))))
    n = len(ni_l1)
    # one single-arc gate per primary input, then two-input gates over pairs of them
    gates = [[i] for i in range(n)] + [[n + 2 * k, n + 2 * k + 1] for k in range(n // 2)]
    nets = [tiny.chain_net([40.0], [0.3, 0.4])] * (n + len(gates))
    A = n + 2 * (n // 2)
    d = tiny.design(n, gates, nets, tables=[i % 2 for i in range(A)])
    load, nd_o, ni_o = oracle.delay_calc(d)
    ni_in = ni_o.copy()
    ni_in[:n] = np.array(ni_l1, np.float32)
    pa = rng.uniform(0, 50, n).astype(np.float32)
    ps = np.array(s_pi, np.float32)
    say(f"[gpu case] radicands at the axis thresholds: {n} primary inputs, schedule={schedule}")
    g = sta.Graph(d, n_tables=2).upload("cuda")
    thr, graphs, fuse = SCHEDULES[schedule]
    g.set_schedule(thr, graphs)
    g.set_level_fusion(fuse)
    nd = sta.delay_calc(g)
    nd["net_imp2"][:A].copy_(torch.from_numpy(ni_in[g.arc_input]))
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(np.ascontiguousarray(lib.tab)).to("cuda"))
    modes = [LATE, EARLY]
    pi = np.zeros((n, 2, 2), np.float32)
    pi[:, :, 0] = pa[:, None]
    pi[:, :, 1] = ps[:, None]
    t = sta.propagate(g, L, sta.make_views(modes), torch.from_numpy(pi).to("cuda"), nd)
    h = {k: v.cpu().numpy() for k, v in t.items()}
    D, G = d.n_drivers, d.n_gates
    for v, m in enumerate(modes):
        o = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd_o, ni_in, pa, ps, m)
        tag = f"view{v}"
        assert_bitwise(tag + " slew_in", g.arc_to_input(h["arc_ts"][:A, v, 1]), o["slew_in"])
        assert_bitwise(tag + " arc_delay", g.arc_to_input(h["arc_delay"][:A, v]), o["arc_delay"])
        assert_bitwise(tag + " at_drv", g.drv_to_input(h["drv_ts"][:D, v, 0]), o["at_drv"])
        assert_bitwise(tag + " slew_drv", g.drv_to_input(h["drv_ts"][:D, v, 1]), o["slew_drv"])
        assert_bitwise(tag + " argmax", g.gate_to_input(h["argmax"][:G, v].astype(np.int32)), o["argmax"])


@SCHED
def test_pi_only_and_empty_designs(schedule):
    d = tiny.design(3, [], [tiny.chain_net([5.0], [1.0, 1.0])] * 3)
    lib = gen.make_library(n_tables=1, seed=1)
    compare_all(d, lib, np.array([1, 2, 3], np.float32), np.array([5, 6, 7], np.float32),
                [np.array([10, -1, 2.5], np.float32)] * 2, [LATE, EARLY], label="primary inputs only",
                schedule=schedule)
    say("[gpu case] empty design")
    d = tiny.design(0, [], [])
    g, h = gpu_run(d, lib, np.zeros(0, np.float32), np.zeros(0, np.float32), [np.zeros(0, np.float32)],
                   [LATE], schedule=schedule)
    assert h["tns"][0] == 0.0 and np.isinf(h["wns"][0])


@pytest.mark.parametrize("m_range", [(2, 8), (2, 16), (9, 32), (33, 64), (65, 128), (129, 200)])
def test_rc_tree_nets_every_size_class(m_range):
    # random recursive RC trees instead of chains, in each node-count class the delay
    # calculation dispatches on; the whole pipeline bit for bit
    d = gen.make_design(n_pins=3000, n_levels=12, fanin="geom", seed=31, m_range=m_range, tree=True)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d, seed=5)
    late, early = gen.make_rat(d, 12, late_per_level=70.0, hold=120.0)
    compare_all(d, lib, pa, ps, [late, early], [LATE, EARLY], label=f"RC trees {m_range}")


@pytest.mark.parametrize("nets", ["c1 chains", "RC trees"])
def test_fp32_delay_calc_within_1e5(nets):
    if nets == "RC trees":
        d = gen.make_design(n_pins=3000, n_levels=12, fanin="geom", seed=33, m_range=(2, 8), tree=True)
    else:
        d, lib, pa, ps, late, early = workload("c1")
    say(f"[gpu case] fp32 delay calc, {nets}")
    import torch
    g = sta.Graph(d, n_tables=128).upload("cuda")
    nd = sta.delay_calc(g, sta.STA_DC_FP32)
    torch.cuda.synchronize()
    load, m1, imp2 = oracle.delay_calc(d)
    gl = g.drv_to_input(nd["load"].cpu().numpy()[: d.n_drivers])
    gm = g.arc_to_input(nd["net_delay"].cpu().numpy()[: d.n_arcs])
    gi = g.arc_to_input(nd["net_imp2"].cpu().numpy()[: d.n_arcs])
    assert np.all(np.abs(gl - load) <= 1e-5 * load)
    assert np.all(np.abs(gm - m1) <= 1e-5 * m1)
    scale = np.maximum(imp2, m1.astype(np.float64) ** 2)
    assert np.all(np.abs(gi.astype(np.float64) - imp2) <= 1e-5 * scale)


@SCHED
def test_deterministic_reruns(schedule):
    d, lib, pa, ps, late, early = workload("c1")
    say(f"[gpu case] determinism c1 {schedule}")
    _, h1 = gpu_run(d, lib, pa, ps, [late, early], [LATE, EARLY], schedule=schedule)
    _, h2 = gpu_run(d, lib, pa, ps, [late, early], [LATE, EARLY], schedule=schedule)
    for k in h1:
        assert_bitwise("rerun " + k, h1[k].reshape(-1), h2[k].reshape(-1))


@pytest.mark.parametrize("schedule", [None, "level", "view"])
def test_c2_full_size_bitwise(schedule):
    # the 1M-pin workload; schedule None is the library's own choice, which the
    # benchmark times
    d, lib, pa, ps, late, early = workload("c2")
    compare_all(d, lib, pa, ps, [late, early], [LATE, EARLY], label="c2 1M pins", schedule=schedule)


def test_c5_two_million_pins_bitwise():
    # the largest design of the test set (2M pins, 400 levels, 32 fanout-64 nets) through
    # the library's default schedule
    d, lib, pa, ps, late, early = workload("c5")
    compare_all(d, lib, pa, ps, [late, early], [LATE, EARLY], label="c5 2M pins", schedule=None)


def test_c2_four_views_two_corners_bitwise():
    # the 1M-pin workload with late and early views on two corners (four views per launch)
    # through the library's default schedule
    d, _, pa, ps, late, early = workload("c2")
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    compare_all(d, lib, pa, ps, [late, early, late, early], [LATE, EARLY, LATE, EARLY], [1, 1, 3, 3],
                label="c2 1M pins, four views", schedule=None)


def test_graph_replays_match_plain_launches():
    # the level schedule replays a captured hipGraph; replay it several times with torch's
    # own work (zeroing every output) and synchronizations in between, and compare every
    # replay with a plain-launch run
    import torch
    d, lib, pa, ps, late, early = workload("c1")
    say("[gpu case] graph replays c1")
    _, ref = gpu_run(d, lib, pa, ps, [late, early], [LATE, EARLY], schedule="level_plain")
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    g.set_schedule(0, True)
    Lb = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    views = sta.make_views([LATE, EARLY])
    pi = np.zeros((d.n_pi, 2, 2), np.float32)
    pi[:, :, 0] = pa[:, None]
    pi[:, :, 1] = ps[:, None]
    pit = torch.from_numpy(pi).cuda()
    rat = torch.from_numpy(np.stack([late, early], 1).astype(np.float32)).cuda()
    nd = sta.delay_calc(g)
    tm = sta.alloc_timing(g, 2)
    sl = sta.alloc_slack(g, 2)
    for rep in range(4):
        for tsr in list(tm.values()) + [v for k, v in sl.items() if k != "scratch"]:
            tsr.zero_()
        torch.cuda.synchronize()
        sta.propagate(g, Lb, views, pit, nd, out=tm)
        sta.slack(g, views, nd, tm, rat, out=sl)
        torch.cuda.synchronize()
        for k, v in list(tm.items()) + list(sl.items()):
            if k == "scratch":
                continue
            assert_bitwise(f"replay {rep} {k}", v.cpu().numpy().reshape(-1), ref[k].reshape(-1))


def test_default_schedule_choice():
    # left to the library: fused spans for every view count at any size; an explicit
    # threshold selects the view schedule, a negative one restores the library's choice
    import torch
    d, lib, pa, ps, late, early = workload("c1")
    say("[gpu case] default schedule choice c1")
    for modes, want in (([LATE], "k_forward_span"), ([LATE, EARLY], "k_forward_span"),
                        ([LATE, EARLY, LATE, EARLY], "k_forward_span")):
        g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
        L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
        views = sta.make_views(modes)
        nd = sta.delay_calc(g)
        pi = np.zeros((d.n_pi, len(modes), 2), np.float32)
        pi[:, :, 0] = pa[:, None]
        pi[:, :, 1] = ps[:, None]
        pit = torch.from_numpy(pi).cuda()
        sta.profile_begin()
        sta.propagate(g, L, views, pit, nd)
        ran = sta.profile_end()
        torch.cuda.synchronize()
        assert want in ran, (modes, ran)
        g.set_schedule(1 << 30, True)
        sta.profile_begin()
        sta.propagate(g, L, views, pit, nd)
        ran = sta.profile_end()
        torch.cuda.synchronize()
        assert "k_forward_view" in ran, (modes, ran)
        g.set_schedule(-1, True)
        sta.profile_begin()
        sta.propagate(g, L, views, pit, nd)
        ran = sta.profile_end()
        torch.cuda.synchronize()
        assert want in ran, (modes, ran)
