"""GPU checks of the captured launch sequences: a graph uploaded again into another buffer
(the old one overwritten) and one graph driven from two streams with distinct outputs
both give the oracle's results bit for bit."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests.gpu_common import EARLY, LATE, assert_bitwise, say

pytestmark = pytest.mark.gpu


def _design(seed):
    d = gen.make_design(n_pins=9000, n_levels=30, fanin="geom", seed=seed, n_fanout64=1)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, 30, late_per_level=70.0, hold=120.0)
    return d, lib, pa, ps, late, early


def _inputs(g, d, pa, ps, late, early):
    import torch
    pi = np.zeros((max(d.n_pi, 1), 2, 2), np.float32)
    pi[:d.n_pi, :, 0] = pa[:, None]
    pi[:d.n_pi, :, 1] = ps[:, None]
    E = g.sizes["n_endpoints"]
    rat = np.stack([late, early], axis=1).astype(np.float32)[:E]
    return torch.from_numpy(pi).cuda(), torch.from_numpy(rat).cuda()


def _check(g, d, lib, pa, ps, late, early, tm, sl, tag):
    """Arrivals, slacks and TNS of both views against the oracle."""
    res = oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY))
    D, A = d.n_drivers, d.n_arcs
    for v, key in enumerate(("late", "early")):
        r = res[key]
        assert_bitwise(f"{tag} {key} at_drv", g.drv_to_input(tm["drv_ts"][:D, v, 0].cpu().numpy()), r["at_drv"])
        assert_bitwise(f"{tag} {key} at_in", g.arc_to_input(tm["arc_ts"][:A, v, 0].cpu().numpy()), r["at_in"])
        assert_bitwise(f"{tag} {key} slack_drv", g.drv_to_input(sl["drv_slack"][:D, v].cpu().numpy()), r["slack_drv"])
        assert float(sl["tns"][v]) == r["tns"], (tag, key)


def test_reupload_replays_against_the_new_buffer():
    import torch
    d, lib, pa, ps, late, early = _design(61)
    say(f"[gpu case] re-upload: pins={d.n_pins}")
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    views = sta.make_views([LATE, EARLY])
    pi_t, rat_t = _inputs(g, d, pa, ps, late, early)
    nd = sta.delay_calc(g)
    tm = sta.alloc_timing(g, 2)
    sl = sta.alloc_slack(g, 2)
    for _ in range(2):                      # capture, then replay
        sta.propagate(g, L, views, pi_t, nd, out=tm)
        sta.slack(g, views, nd, tm, rat_t, out=sl)
    torch.cuda.synchronize()
    _check(g, d, lib, pa, ps, late, early, tm, sl, "first buffer")
    old = g.dev
    g.upload("cuda")                        # a new buffer; the old one stays allocated here
    torch.cuda.synchronize()
    assert g.dev.data_ptr() != old.data_ptr()
    # Overwrite the old buffer with the image of a design that differs only in its table
    # ids (same structure, so the same layout and every index still in range): a replay
    # still reading the old buffer would look up other tables and give other results.
    d2 = dataclasses.replace(d, arc_tbl=((d.arc_tbl + 1) % lib.n_tables).astype(np.int32))
    g2 = sta.Graph(d2, n_tables=lib.n_tables)
    assert g2.sizes == g.sizes
    sta._check(sta.load_library().sta_graph_upload(g2.handle, sta._P(old.data_ptr()), old.numel(),
                                                   sta._stream(torch, old.device)), "sta_graph_upload")
    torch.cuda.synchronize()
    for t in list(tm.values()) + [v for k, v in sl.items() if k != "scratch"]:
        t.zero_()
    for _ in range(2):                      # the same output pointers: only the graph buffer moved
        sta.propagate(g, L, views, pi_t, nd, out=tm)
        sta.slack(g, views, nd, tm, rat_t, out=sl)
    torch.cuda.synchronize()
    _check(g, d, lib, pa, ps, late, early, tm, sl, "second buffer")
    del old


def test_two_streams_distinct_outputs():
    import torch
    d, lib, pa, ps, late, early = _design(62)
    say(f"[gpu case] two streams: pins={d.n_pins}")
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    views = sta.make_views([LATE, EARLY])
    nd = sta.delay_calc(g)
    # two argument sets: different primary-input arrivals and slews, separate outputs
    cases = []
    for k, (a, s_) in enumerate(((pa, ps), (pa + np.float32(7.5), ps * np.float32(1.25)))):
        pi_t, rat_t = _inputs(g, d, a, s_, late, early)
        cases.append(dict(pa=a, ps=s_, pi=pi_t, rat=rat_t, tm=sta.alloc_timing(g, 2), sl=sta.alloc_slack(g, 2),
                          stream=torch.cuda.Stream()))
    torch.cuda.synchronize()
    for _ in range(4):                      # alternate: each set keeps its own captured sequence
        for c in cases:
            with torch.cuda.stream(c["stream"]):
                sta.propagate(g, L, views, c["pi"], nd, out=c["tm"])
                sta.slack(g, views, nd, c["tm"], c["rat"], out=c["sl"])
    torch.cuda.synchronize()
    for k, c in enumerate(cases):
        _check(g, d, lib, c["pa"], c["ps"], late, early, c["tm"], c["sl"], f"stream {k}")


def test_more_argument_sets_than_cached():
    """Six output sets in rotation on one stream (the cache keeps four): every call's
    results are still the oracle's."""
    import torch
    d, lib, pa, ps, late, early = _design(63)
    say(f"[gpu case] cache eviction: pins={d.n_pins}")
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    views = sta.make_views([LATE, EARLY])
    nd = sta.delay_calc(g)
    pi_t, rat_t = _inputs(g, d, pa, ps, late, early)
    outs = [(sta.alloc_timing(g, 2), sta.alloc_slack(g, 2)) for _ in range(6)]
    for _ in range(2):
        for tm, sl in outs:
            sta.propagate(g, L, views, pi_t, nd, out=tm)
            sta.slack(g, views, nd, tm, rat_t, out=sl)
    torch.cuda.synchronize()
    for k, (tm, sl) in enumerate(outs):
        _check(g, d, lib, pa, ps, late, early, tm, sl, f"set {k}")
