"""Batched delay calculation, propagation and slack (many designs x corners: span steps,
the persistent unit queue and per-design level sequences, replayed from hipGraphs) against
the oracle, bit for bit, per design and view."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests import tiny
from tests.gpu_common import assert_bitwise, say

pytestmark = pytest.mark.gpu

LATE, EARLY = sta.STA_LATE, sta.STA_EARLY
MODES = [LATE, LATE, EARLY, LATE]
SETS = [0, 1, 2, 3]
SP, PE, LV = sta.BATCH_SPANS, sta.BATCH_PERSISTENT, sta.BATCH_LEVELS


def _wide_gate_design(seed):
    """A gate of fanin 64 (a whole wavefront, the widest a gate may be) among ordinary
    gates."""
    rng = np.random.default_rng(seed)
    n_pi = 90
    gates = [[int(x) for x in rng.choice(n_pi, size=int(rng.integers(1, 4)), replace=False)] for _ in range(60)]
    gates += [list(range(64))]                                           # the wide gate
    gates += [[n_pi + int(rng.integers(0, 61)), n_pi + 60] for _ in range(30)]
    nets = []
    for _ in range(n_pi + len(gates)):
        m = int(rng.integers(2, 8))
        nets.append(tiny.chain_net(rng.uniform(10, 500, m - 1).tolist(), rng.uniform(0.1, 5, m).tolist()))
    A = sum(len(x) for x in gates)
    return tiny.design(n_pi, gates, nets, pincaps=list(rng.uniform(1, 4, A)),
                       tables=list(rng.integers(0, 128, A)))


def _designs():
    """(design, schedule, span lengths) of the batch."""
    specs = [(3000, 20, SP, None), (12000, 45, PE, None), (40000, 80, SP, (4, 6)), (5000, 15, LV, None),
             (60000, 110, SP, None), (800, 6, PE, None), (20000, 40, SP, (2, 3))]
    out = []
    for i, (p, l, sched, caps) in enumerate(specs):
        d = gen.make_design(n_pins=p, n_levels=l, fanin="geom", seed=300 + i, n_fanout64=1 if p > 20000 else 0)
        out.append((d, sched, caps))
    out.append((_wide_gate_design(7), SP, None))
    out.append((tiny.wide_fanout_design(8), SP, None))      # backward spans that do not fuse
    # RC trees (not chains): the batched delay calculation then takes its select form for
    # every design of the node-count class
    out.append((gen.make_design(n_pins=4000, n_levels=16, fanin="geom", seed=309, m_range=(2, 8), tree=True),
                SP, None))
    return out


def _rats(d, rng):
    ep = oracle.endpoints(d)
    return [rng.uniform(100, 900, ep.size).astype(np.float32) for _ in MODES]


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    tables = torch.from_numpy(lib.tab).cuda()
    L = sta.make_library(lib.x, lib.y, tables)
    views = sta.make_views(MODES, SETS)
    rng = np.random.default_rng(11)
    entries, keep = [], []
    for d, sched, caps in _designs():
        g = sta.Graph(d, n_tables=lib.tab.shape[1], span_levels=caps).upload("cuda")
        nd = sta.alloc_net(g)
        pa, ps = gen.make_pi(d)
        pi = np.zeros((max(d.n_pi, 1), len(MODES), 2), np.float32)
        pi[:d.n_pi, :, 0] = pa[:, None]
        pi[:d.n_pi, :, 1] = ps[:, None]
        pi_t = torch.from_numpy(pi).cuda()
        tm = sta.alloc_timing(g, len(MODES))
        rats = _rats(d, rng)
        E = g.sizes["n_endpoints"]
        rat = np.zeros((max(E, 1), len(MODES)), np.float32)
        for v in range(len(MODES)):
            rat[:E, v] = rats[v]
        sl = sta.alloc_slack(g, len(MODES))
        entries.append((g, pi_t, nd, tm, sched, torch.from_numpy(rat).cuda(), sl))
        keep.append((d, pa, ps, rats))
    return lib, L, views, entries, keep


def _check_design(lib, d, pa, ps, rats, g, nd, tm, sl, label):
    h = {k: v.cpu().numpy() for k, v in list(nd.items()) + list(tm.items()) + list(sl.items()) if k != "scratch"}
    D, A, G = d.n_drivers, d.n_arcs, d.n_gates
    load, nd_, ni_ = oracle.delay_calc(d)
    assert_bitwise(f"{label} load", g.drv_to_input(h["load"][:D]), load)
    assert_bitwise(f"{label} net_delay", g.arc_to_input(h["net_delay"][:A]), nd_)
    assert_bitwise(f"{label} net_imp2", g.arc_to_input(h["net_imp2"][:A]), ni_)
    gate_of = np.repeat(np.arange(G), np.diff(d.gate_arc_ptr))
    assert_bitwise(f"{label} arc_load", g.arc_to_input(h["arc_load"][:A]), load[d.n_pi + gate_of])
    ep = oracle.endpoints(d)
    for v, (m, st) in enumerate(zip(MODES, SETS)):
        r = oracle.propagate(d, lib.x, lib.y, lib.tab[st], load, nd_, ni_, pa, ps, m)
        s = oracle.slack(d, nd_, r["arc_delay"], r["at_drv"], r["at_in"], rats[v], m)
        tag = f"{label} v{v}"
        assert_bitwise(f"{tag} at", g.drv_to_input(h["drv_ts"][:D, v, 0]), r["at_drv"])
        assert_bitwise(f"{tag} slew", g.drv_to_input(h["drv_ts"][:D, v, 1]), r["slew_drv"])
        assert_bitwise(f"{tag} at_in", g.arc_to_input(h["arc_ts"][:A, v, 0]), r["at_in"])
        assert_bitwise(f"{tag} slew_in", g.arc_to_input(h["arc_ts"][:A, v, 1]), r["slew_in"])
        assert_bitwise(f"{tag} delay", g.arc_to_input(h["arc_delay"][:A, v]), r["arc_delay"])
        if G:
            assert_bitwise(f"{tag} argmax", g.gate_to_input(h["argmax"][:G, v].astype(np.int32)), r["argmax"])
        assert_bitwise(f"{tag} rat_drv", g.drv_to_input(h["drv_rat"][:D, v]), s["rat_drv"])
        assert_bitwise(f"{tag} rat_in", g.arc_to_input(h["arc_rat"][:A, v]), s["rat_in"])
        assert_bitwise(f"{tag} slack_drv", g.drv_to_input(h["drv_slack"][:D, v]), s["slack_drv"])
        assert_bitwise(f"{tag} slack_in", g.arc_to_input(h["arc_slack"][:A, v]), s["slack_in"])
        want_wns = s["wns"] if ep.size else np.float32(np.inf)
        assert_bitwise(f"{tag} wns", np.array([h["wns"][v]], np.float32), np.array([want_wns], np.float32))
        assert_bitwise(f"{tag} tns", np.array([h["tns"][v]]), np.array([s["tns"]], np.float64))


@pytest.mark.parametrize("use_graph,blocks,tiling", [(True, 0, (1, 2)), (False, 0, (4, 4)), (True, 3, (2, 1)),
                                                      (True, 0, (4, 1))])
def test_batch_matches_oracle(batch_setup, use_graph, blocks, tiling):
    import torch
    lib, L, views, entries, keep = batch_setup
    b = sta.Batch(entries, L, views).set_tiling(*tiling)
    info = b.info()
    say(f"[gpu case] batch graph={use_graph} blocks={blocks} views per wavefront {tiling} {info}")
    assert info["persistent_units"] == len(MODES) * sum(1 for e in entries if e[4] == PE)
    assert info["span_designs"] == sum(1 for e in entries if e[4] == SP)
    assert info["slack_designs"] == len(entries)
    assert info["fwd_steps"] >= max(len(e[0].span_list()[0]) for e in entries if e[4] == SP)
    for e in entries:
        for dct in (e[2], e[3], e[6]):
            for t in dct.values():
                t.fill_(7)
    for _ in range(3 if use_graph else 1):
        b.delay_calc(use_graph=use_graph)
        b.propagate(use_graph=use_graph, blocks=blocks)
        b.slack(use_graph=use_graph)
        torch.cuda.synchronize()
    for i, ((d, pa, ps, rats), e) in enumerate(zip(keep, entries)):
        _check_design(lib, d, pa, ps, rats, e[0], e[2], e[3], e[6], f"design {i}")


def test_batch_without_slack_buffers(batch_setup):
    """Designs given without slack buffers take no part in the batched slack pass."""
    import torch
    lib, L, views, entries, keep = batch_setup
    part = [e[:5] for e in entries[:3]] + [entries[4]]
    b = sta.Batch(part, L, views)
    assert b.info()["slack_designs"] == 1
    entries[4][6]["tns"].fill_(7)
    b.delay_calc()
    b.propagate()
    b.slack()
    torch.cuda.synchronize()
    d, pa, ps, rats = keep[4]
    e = entries[4]
    _check_design(lib, d, pa, ps, rats, e[0], e[2], e[3], e[6], "design 4 alone")


def test_batch_argument_errors(batch_setup):
    lib, L, views, entries, keep = batch_setup
    g, pi, nd, tm, _, rat, sl = entries[0]
    with pytest.raises(sta.StaError):
        sta.Batch([(g, pi, nd, tm, 7)], L, views)
    bad = sta.make_views([LATE], [9])
    with pytest.raises(sta.StaError):
        sta.Batch([(g, pi, nd, tm, SP)], L, bad)
    with pytest.raises(sta.StaError):
        sta.Batch([(g, pi, nd, tm, SP, rat, None)], L, views)
    b = sta.Batch([(g, pi, nd, tm, SP)], L, views)
    for bad_tiling in ((3, 1), (1, 8), (0, 2)):
        with pytest.raises(sta.StaError):
            b.set_tiling(*bad_tiling)


def test_c3_batch_bitwise():
    """The full batched workload (64 designs, pins log-uniform 5k-500k, four corners) through
    the batch with a mixed plan (every fourth design on the persistent launch, the rest in
    span steps, four views per span wavefront), every design and corner against the oracle."""
    import torch
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    V = len(gen.CORNER_KAPPAS)
    modes = [LATE] * V
    views = sta.make_views(modes, list(range(V)))
    rng = np.random.default_rng(33)
    entries, keep = [], []
    for i, sp in enumerate(gen.c3_designs(64)):
        d = gen.make_design(**sp)
        g = sta.Graph(d, n_tables=lib.tab.shape[1]).upload("cuda")
        pa, ps = gen.make_pi(d)
        pi = np.zeros((max(d.n_pi, 1), V, 2), np.float32)
        pi[:d.n_pi, :, 0] = pa[:, None]
        pi[:d.n_pi, :, 1] = ps[:, None]
        E = g.sizes["n_endpoints"]
        rats = [rng.uniform(50.0 * sp["n_levels"], 80.0 * sp["n_levels"], E).astype(np.float32) for _ in modes]
        rat = np.zeros((max(E, 1), V), np.float32)
        for v in range(V):
            rat[:E, v] = rats[v]
        entries.append((g, torch.from_numpy(pi).cuda(), sta.alloc_net(g), sta.alloc_timing(g, V),
                        PE if i % 4 == 3 else SP, torch.from_numpy(rat).cuda(), sta.alloc_slack(g, V)))
        keep.append((d, pa, ps, rats))
    b = sta.Batch(entries, L, views).set_tiling(4, 4)
    say(f"[gpu case] c3 batch {b.info()}")
    for _ in range(2):
        b.delay_calc()
        b.propagate()
        b.slack()
    torch.cuda.synchronize()
    for i, ((d, pa, ps, rats), e) in enumerate(zip(keep, entries)):
        h = {k: v.cpu().numpy() for k, v in list(e[2].items()) + list(e[3].items()) + list(e[6].items())
             if k != "scratch"}
        D, A = d.n_drivers, d.n_arcs
        load, nd_, ni_ = oracle.delay_calc(d)
        assert_bitwise(f"c3 design {i} net_delay", e[0].arc_to_input(h["net_delay"][:A]), nd_)
        for v in range(V):
            r = oracle.propagate(d, lib.x, lib.y, lib.tab[v], load, nd_, ni_, pa, ps, LATE)
            s = oracle.slack(d, nd_, r["arc_delay"], r["at_drv"], r["at_in"], rats[v], LATE)
            tag = f"c3 design {i} corner {v}"
            assert_bitwise(f"{tag} at", e[0].drv_to_input(h["drv_ts"][:D, v, 0]), r["at_drv"])
            assert_bitwise(f"{tag} slew", e[0].drv_to_input(h["drv_ts"][:D, v, 1]), r["slew_drv"])
            assert_bitwise(f"{tag} slack", e[0].drv_to_input(h["drv_slack"][:D, v]), s["slack_drv"])
            assert_bitwise(f"{tag} tns", np.array([h["tns"][v]]), np.array([s["tns"]], np.float64))
