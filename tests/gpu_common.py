"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare in input numbering."""
import sys

import numpy as np

import oracle
from paper_2203_08395_amd import gen, sta

LATE, EARLY = sta.STA_LATE, sta.STA_EARLY


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(x):
    x = np.ascontiguousarray(x)
    if x.dtype == np.float32:
        return x.view(np.uint32)
    if x.dtype == np.float64:
        return x.view(np.uint64)
    return x


def assert_bitwise(name, got, want):
    got, want = np.asarray(got), np.asarray(want)
    assert got.shape == want.shape, (name, got.shape, want.shape)
    bad = np.nonzero(bits(got) != bits(want))[0]
    if bad.size:
        i = bad[0]
        raise AssertionError(f"{name}: {bad.size} of {got.size} differ; first at {i}: got {got[i]!r} want {want[i]!r}")


# name: (view-schedule threshold in arcs per level, replay from hipGraphs, level fusion)
SCHEDULES = {"span": (0, True, True), "level": (0, True, False), "level_plain": (0, False, False),
             "view": (1 << 30, True, True)}


def gpu_run(d, lib, pi_at, pi_slew, ep_rats, modes, table_sets=None, precision=sta.STA_DC_FP64, device="cuda",
            schedule=None):
    """ep_rats[v]: endpoint required times of view v (rank order); schedule: None (the
    library's choice), "level" or "view"."""
    import torch
    V = len(modes)
    g = sta.Graph(d, n_tables=lib.tab.shape[-4]).upload(device)
    if schedule is not None:
        thr, graphs, fuse = SCHEDULES[schedule]
        g.set_schedule(thr, graphs)
        g.set_level_fusion(fuse)
    tables = torch.from_numpy(np.ascontiguousarray(lib.tab)).to(device)
    L = sta.make_library(lib.x, lib.y, tables)
    views = sta.make_views(modes, table_sets)
    nd = sta.delay_calc(g, precision)
    pi = np.zeros((max(d.n_pi, 1), V, 2), np.float32)
    for v in range(V):
        pi[: d.n_pi, v, 0] = pi_at
        pi[: d.n_pi, v, 1] = pi_slew
    pi_t = torch.from_numpy(pi).to(device)
    E = g.sizes["n_endpoints"]
    rat = np.zeros((max(E, 1), V), np.float32)
    for v in range(V):
        rat[:E, v] = ep_rats[v]
    rat_t = torch.from_numpy(rat).to(device)
    torch.cuda.synchronize()
    sta.profile_begin()
    t = sta.propagate(g, L, views, pi_t, nd)
    s = sta.slack(g, views, nd, t, rat_t)
    ran = sta.profile_end()
    torch.cuda.synchronize()
    if schedule == "view" and g.sizes["n_levels"] > 0:
        # wide levels may not fit a workgroup's LDS: then that pass runs per level
        assert "k_forward_view" in ran or "k_backward_view" in ran, ran
    if schedule in ("level", "level_plain") and g.sizes["n_levels"] > 0:
        assert "k_forward" in ran and "k_backward" in ran and "k_forward_span" not in ran, ran
    if schedule == "span" and g.sizes["n_levels"] > 0:
        assert "k_forward_span" in ran or "k_forward" in ran, ran
    host = {k: v.cpu().numpy() for k, v in list(nd.items()) + list(t.items()) + list(s.items()) if k != "scratch"}
    return g, host


def compare_all(d, lib, pi_at, pi_slew, ep_rats, modes, table_sets=None, label="", schedule=None):
    """HIP path vs oracle, bit for bit, every output of every view."""
    say(f"[gpu case] {label}: pins={d.n_pins} views={list(modes)} sets={table_sets} schedule={schedule}")
    g, h = gpu_run(d, lib, pi_at, pi_slew, ep_rats, modes, table_sets, schedule=schedule)
    D, A, G = d.n_drivers, d.n_arcs, d.n_gates
    load, nd, ni = oracle.delay_calc(d)
    assert_bitwise("load", g.drv_to_input(h["load"][:D]), load)
    assert_bitwise("net_delay", g.arc_to_input(h["net_delay"][:A]), nd)
    assert_bitwise("net_imp2", g.arc_to_input(h["net_imp2"][:A]), ni)
    gate_of = np.repeat(np.arange(G), np.diff(d.gate_arc_ptr))
    assert_bitwise("arc_load", g.arc_to_input(h["arc_load"][:A]), load[d.n_pi + gate_of])
    ep = oracle.endpoints(d)
    for v, m in enumerate(modes):
        tab = lib.tab if lib.tab.ndim == 4 else lib.tab[table_sets[v] if table_sets else 0]
        p = oracle.propagate(d, lib.x, lib.y, tab, load, nd, ni, pi_at, pi_slew, m)
        s = oracle.slack(d, nd, p["arc_delay"], p["at_drv"], p["at_in"], ep_rats[v], m)
        tag = f"view{v}/{'late' if m == LATE else 'early'}"
        assert_bitwise(tag + " at_drv", g.drv_to_input(h["drv_ts"][:D, v, 0]), p["at_drv"])
        assert_bitwise(tag + " slew_drv", g.drv_to_input(h["drv_ts"][:D, v, 1]), p["slew_drv"])
        assert_bitwise(tag + " at_in", g.arc_to_input(h["arc_ts"][:A, v, 0]), p["at_in"])
        assert_bitwise(tag + " slew_in", g.arc_to_input(h["arc_ts"][:A, v, 1]), p["slew_in"])
        assert_bitwise(tag + " arc_delay", g.arc_to_input(h["arc_delay"][:A, v]), p["arc_delay"])
        assert_bitwise(tag + " argmax", g.gate_to_input(h["argmax"][:G, v].astype(np.int32)), p["argmax"])
        assert_bitwise(tag + " rat_drv", g.drv_to_input(h["drv_rat"][:D, v]), s["rat_drv"])
        assert_bitwise(tag + " rat_in", g.arc_to_input(h["arc_rat"][:A, v]), s["rat_in"])
        assert_bitwise(tag + " slack_drv", g.drv_to_input(h["drv_slack"][:D, v]), s["slack_drv"])
        assert_bitwise(tag + " slack_in", g.arc_to_input(h["arc_slack"][:A, v]), s["slack_in"])
        want_wns = s["wns"] if ep.size else np.float32(np.inf)
        assert_bitwise(tag + " wns", np.array([h["wns"][v]], np.float32), np.array([want_wns], np.float32))
        assert_bitwise(tag + " tns", np.array([h["tns"][v]]), np.array([s["tns"]], np.float64))
    return g, h


def workload(name):
    cfg = gen.CONFIGS[name]
    d = gen.make_design(**cfg)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, cfg["n_levels"], **gen.RAT_PARAMS[name])
    return d, lib, pa, ps, late, early
