"""Batched propagation (many designs x corners in one persistent launch plus per-level
launches, replayed from a hipGraph) against the oracle, bit for bit, per design and view."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests.gpu_common import assert_bitwise, say

pytestmark = pytest.mark.gpu

LATE, EARLY = sta.STA_LATE, sta.STA_EARLY
MODES = [LATE, LATE, EARLY, LATE]
SETS = [0, 1, 2, 3]


def _designs():
    specs = [(3000, 20, 0), (12000, 45, 1), (40000, 80, 0), (5000, 15, 1), (60000, 110, 0), (800, 6, 0)]
    out = []
    for i, (p, l, sched) in enumerate(specs):
        d = gen.make_design(n_pins=p, n_levels=l, fanin="geom", seed=300 + i, n_fanout64=1 if p > 20000 else 0)
        out.append((d, sched))
    return out


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    lib = gen.make_library(kappas=gen.CORNER_KAPPAS)
    tables = torch.from_numpy(lib.tab).cuda()
    L = sta.make_library(lib.x, lib.y, tables)
    views = sta.make_views(MODES, SETS)
    entries, keep = [], []
    for d, sched in _designs():
        g = sta.Graph(d, n_tables=lib.tab.shape[1]).upload("cuda")
        nd = sta.delay_calc(g)
        pa, ps = gen.make_pi(d)
        pi = np.zeros((max(d.n_pi, 1), len(MODES), 2), np.float32)
        pi[:d.n_pi, :, 0] = pa[:, None]
        pi[:d.n_pi, :, 1] = ps[:, None]
        pi_t = torch.from_numpy(pi).cuda()
        tm = sta.alloc_timing(g, len(MODES))
        entries.append((g, pi_t, nd, tm, sched))
        keep.append((d, pa, ps))
    return lib, L, views, entries, keep


def _check_design(lib, d, pa, ps, g, tm, label):
    h = {k: v.cpu().numpy() for k, v in tm.items()}
    D, A, G = d.n_drivers, d.n_arcs, d.n_gates
    for v, (m, st) in enumerate(zip(MODES, SETS)):
        one = gen.Library(x=lib.x, y=lib.y, tab=lib.tab[st])
        load, nd_, ni_ = oracle.delay_calc(d)
        r = oracle.propagate(d, one.x, one.y, one.tab, load, nd_, ni_, pa, ps, m)
        assert_bitwise(f"{label} v{v} at", g.drv_to_input(h["drv_ts"][:D, v, 0]), r["at_drv"])
        assert_bitwise(f"{label} v{v} slew", g.drv_to_input(h["drv_ts"][:D, v, 1]), r["slew_drv"])
        assert_bitwise(f"{label} v{v} at_in", g.arc_to_input(h["arc_ts"][:A, v, 0]), r["at_in"])
        assert_bitwise(f"{label} v{v} delay", g.arc_to_input(h["arc_delay"][:A, v]), r["arc_delay"])
        if G:
            am = g.gate_to_input(h["argmax"][:G, v].astype(np.int32))
            np.testing.assert_array_equal(am, r["argmax"])


@pytest.mark.parametrize("use_graph,blocks", [(True, 0), (False, 0), (True, 3)])
def test_batch_matches_oracle(batch_setup, use_graph, blocks):
    import torch
    lib, L, views, entries, keep = batch_setup
    b = sta.Batch(entries, L, views)
    info = b.info()
    say(f"[gpu case] batch graph={use_graph} blocks={blocks} {info}")
    assert info["persistent_units"] == len(MODES) * sum(1 for e in entries if e[4] == 0)
    for _, _, _, tm, _ in entries:
        for t in tm.values():
            t.zero_()
    for _ in range(3 if use_graph else 1):
        b.propagate(use_graph=use_graph, blocks=blocks)
        torch.cuda.synchronize()
    for i, ((d, pa, ps), (g, _, _, tm, _)) in enumerate(zip(keep, entries)):
        _check_design(lib, d, pa, ps, g, tm, f"design {i}")


def test_batch_argument_errors(batch_setup):
    lib, L, views, entries, keep = batch_setup
    g, pi, nd, tm, _ = entries[0]
    with pytest.raises(sta.StaError):
        sta.Batch([(g, pi, nd, tm, 7)], L, views)
    bad = sta.make_views([LATE], [9])
    with pytest.raises(sta.StaError):
        sta.Batch([(g, pi, nd, tm, 0)], L, bad)
