"""GPU check of sta_slack_noalloc (the entry point that allocates nothing: its scratch is
the library's static device array) against sta_slack on the same inputs, bit for bit:
two calls in a row on the shared array, the second on a smaller design, and a four-view
call on the view schedule."""
import numpy as np
import pytest

from paper_2203_08395_amd import gen, sta
from tests.gpu_common import EARLY, LATE, assert_bitwise, say

pytestmark = pytest.mark.gpu

KEYS = ("drv_rat", "arc_rat", "drv_slack", "arc_slack", "tns", "wns")


def _timed(n_pins, n_levels, seed, modes, schedule_thr=None):
    """Forward pass of a seeded design on the GPU, plus sta_slack's outputs."""
    import torch
    d = gen.make_design(n_pins=n_pins, n_levels=n_levels, fanin="geom", seed=seed, n_fanout64=1)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, n_levels, late_per_level=70.0, hold=120.0)
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    if schedule_thr is not None:
        g.set_schedule(schedule_thr, True)
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    V = len(modes)
    views = sta.make_views(modes)
    pi = np.zeros((max(d.n_pi, 1), V, 2), np.float32)
    pi[:d.n_pi, :, 0] = pa[:, None]
    pi[:d.n_pi, :, 1] = ps[:, None]
    E = g.sizes["n_endpoints"]
    rat = np.zeros((max(E, 1), V), np.float32)
    for v, m in enumerate(modes):
        rat[:E, v] = (late if m == LATE else early)[:E]
    pi_t, rat_t = torch.from_numpy(pi).cuda(), torch.from_numpy(rat).cuda()
    nd = sta.delay_calc(g)
    tm = sta.propagate(g, L, views, pi_t, nd)
    ref = sta.slack(g, views, nd, tm, rat_t)
    torch.cuda.synchronize()
    return g, views, nd, tm, rat_t, {k: ref[k].cpu().numpy() for k in KEYS}


def _fresh_out(g, n_views):
    """Outputs filled with a NaN pattern, so that a value left unwritten cannot pass."""
    out = sta.alloc_slack(g, n_views)
    del out["scratch"]
    for k in KEYS:
        out[k].fill_(float("nan"))
    return out


def _compare(tag, got, ref):
    for k in KEYS:
        assert_bitwise(f"{tag} {k}", got[k].cpu().numpy().reshape(-1), ref[k].reshape(-1))


def test_noalloc_slack_equals_slack_twice_then_smaller():
    import torch
    big = _timed(20000, 40, 71, [LATE, EARLY])
    small = _timed(2500, 12, 72, [LATE, EARLY])
    for tag, (g, views, nd, tm, rat_t, ref) in (("first call, 20k pins", big), ("second call, 2.5k pins", small)):
        say(f"[gpu case] sta_slack_noalloc {tag}")
        out = _fresh_out(g, views.n_views)
        sta.slack_noalloc(g, views, nd, tm, rat_t, out)
        torch.cuda.synchronize()
        _compare(tag, out, ref)
    # the larger design again, after the smaller one left its partials in the array
    g, views, nd, tm, rat_t, ref = big
    say("[gpu case] sta_slack_noalloc third call, 20k pins again")
    out = _fresh_out(g, views.n_views)
    sta.slack_noalloc(g, views, nd, tm, rat_t, out)
    torch.cuda.synchronize()
    _compare("third call", out, ref)


def test_noalloc_slack_view_schedule_four_views():
    import torch
    g, views, nd, tm, rat_t, ref = _timed(4000, 16, 73, [LATE, EARLY, LATE, EARLY], schedule_thr=1 << 30)
    say("[gpu case] sta_slack_noalloc four views, view schedule")
    out = _fresh_out(g, views.n_views)
    sta.slack_noalloc(g, views, nd, tm, rat_t, out)
    torch.cuda.synchronize()
    _compare("view schedule", out, ref)


def test_noalloc_slack_rejects_bad_arguments():
    g, views, nd, tm, rat_t, _ = _timed(2500, 12, 74, [LATE])
    out = _fresh_out(g, 1)
    out["tns"] = None
    with pytest.raises(sta.StaError):
        sta.slack_noalloc(g, views, nd, tm, rat_t, out)
