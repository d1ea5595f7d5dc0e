"""GPU checks of the TNS adjoint (against the oracle's chain rule and FP64 finite
differences), its torch.autograd wrapper, and the critical-path report."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

LATE, EARLY = sta.STA_LATE, sta.STA_EARLY


def _setup(cfg_name=None, seed=None, n_pins=None, n_levels=None, modes=(LATE, EARLY)):
    if cfg_name:
        cfg = gen.CONFIGS[cfg_name]
        rp = gen.RAT_PARAMS[cfg_name]
    else:
        cfg = dict(n_pins=n_pins, n_levels=n_levels, fanin="geom", seed=seed, n_fanout64=1)
        rp = dict(late_per_level=70.0, hold=120.0)
    d = gen.make_design(**cfg)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, cfg["n_levels"], **rp)
    return d, lib, pa, ps, late, early, modes


def _gpu(d, lib, pa, ps, late, early, modes, fusion=True):
    import torch
    g = sta.Graph(d, n_tables=lib.n_tables).upload("cuda")
    g.set_level_fusion(fusion)
    L = sta.make_library(lib.x, lib.y, torch.from_numpy(lib.tab).cuda())
    views = sta.make_views(modes)
    V = len(modes)
    nd = sta.delay_calc(g)
    pi = np.zeros((max(d.n_pi, 1), V, 2), np.float32)
    pi[:d.n_pi, :, 0] = pa[:, None]
    pi[:d.n_pi, :, 1] = ps[:, None]
    E = g.sizes["n_endpoints"]
    rat = np.stack([late if m == LATE else early for m in modes], axis=1).astype(np.float32)
    pi_t, rat_t = torch.from_numpy(pi).cuda(), torch.from_numpy(rat[:E]).cuda()
    t = sta.propagate(g, L, views, pi_t, nd)
    s = sta.slack(g, views, nd, t, rat_t)
    return dict(g=g, L=L, views=views, nd=nd, t=t, s=s, pi=pi_t, rat=rat_t)


def _oracle(d, lib, pa, ps, late, early):
    return oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY))


@pytest.mark.parametrize("fusion", [True, False], ids=["spans", "levels"])
@pytest.mark.parametrize("case", ["c1", "geom_a", "geom_b", "late_only", "wide"])
def test_adjoint_matches_oracle(case, fusion):
    import torch
    if case == "c1":
        args = _setup("c1")
    elif case == "late_only":
        args = _setup(seed=44, n_pins=6000, n_levels=40, modes=(LATE,))
    elif case == "wide":
        from tests import tiny
        d = tiny.wide_fanout_design(7)
        pa, ps = gen.make_pi(d)
        late, early = gen.make_rat(d, 25, late_per_level=55.0, hold=120.0)
        args = (d, gen.make_library(), pa, ps, late, early, (LATE, EARLY))
    else:
        args = _setup(seed={"geom_a": 41, "geom_b": 42}[case], n_pins=20000, n_levels=70)
    d, lib, pa, ps, late, early, modes = args
    say(f"[gpu case] adjoint {case} fusion={fusion}: pins={d.n_pins} views={list(modes)}")
    r = _gpu(*args, fusion=fusion)
    g = r["g"]
    adj = sta.tns_adjoint(g, r["L"], r["views"], r["nd"], r["t"], r["s"])
    torch.cuda.synchronize()
    sta.profile_begin()
    sta.tns_adjoint(g, r["L"], r["views"], r["nd"], r["t"], r["s"])
    kinds = sta.profile_end()
    assert ("k_adjoint_span" in kinds) == fusion, kinds
    h = {k: v.cpu().numpy() for k, v in adj.items()}
    res = _oracle(d, lib, pa, ps, late, early)
    D, A = d.n_drivers, d.n_arcs
    for v, m in enumerate(modes):
        key = "late" if m == LATE else "early"
        g_at, g_arc = oracle.tns_adjoint(d, res[key], m)
        np.testing.assert_array_equal(g.drv_to_input(h["g_drv_at"][:D, v]), g_at.astype(np.float32))
        np.testing.assert_array_equal(g.arc_to_input(h["g_arc_delay"][:A, v]), g_arc.astype(np.float32))
        np.testing.assert_array_equal(g.arc_to_input(h["g_net_delay"][:A, v]), g_arc.astype(np.float32))
        gl = np.zeros(D)
        gl[d.n_pi:] = g_at[d.n_pi:] * oracle.load_slope(d, lib, res[key], res["load"])
        got = g.drv_to_input(h["g_load"][:D, v])
        np.testing.assert_allclose(got, gl, rtol=2e-5, atol=2e-5 * max(1.0, np.abs(gl).max()))
        assert np.count_nonzero(g_arc) > 0 or res[key]["tns"] == 0.0


def test_adjoint_finite_differences_2m_pins():
    """The 2M-pin, 400-level design: GPU gradients against FP64 central differences
    (h = 1e-3 ps, 1e-3 fF) on 1000 sampled arcs and 200 sampled gate loads."""
    import torch
    d, lib, pa, ps, late, early, modes = _setup("c5", modes=(LATE,))
    say(f"[gpu case] adjoint FD c5: pins={d.n_pins}")
    r = _gpu(d, lib, pa, ps, late, early, modes)
    g = r["g"]
    adj = sta.tns_adjoint(g, r["L"], r["views"], r["nd"], r["t"], r["s"])
    torch.cuda.synchronize()
    D, A = d.n_drivers, d.n_arcs
    g_arc = g.arc_to_input(adj["g_arc_delay"][:A, 0].cpu().numpy())
    g_load = g.drv_to_input(adj["g_load"][:D, 0].cpu().numpy())
    res = oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE,))
    rr = res["late"]
    rat = oracle.ep_rat_by_driver(d, late)
    rng = np.random.default_rng(5)
    nz = np.nonzero(g_arc)[0]
    arcs = np.concatenate([rng.choice(nz, 500, replace=False), rng.choice(A, 500, replace=False)])
    fd, clean = oracle.fd_arc_delay(d, rr["arc_delay"].astype(np.float64), res["net_delay"].astype(np.float64),
                                    pa.astype(np.float64), rat, oracle.LATE, arcs, h=1e-3)
    say(f"arc FD: {clean.sum()} of {arcs.size} clean, {np.count_nonzero(g_arc[arcs])} nonzero gradients")
    assert clean.mean() >= 0.98
    np.testing.assert_allclose(g_arc[arcs][clean], fd[clean], atol=1e-6)
    gnz = np.nonzero(g_load[d.n_pi:])[0]
    gates = np.concatenate([rng.choice(gnz, 150, replace=False), rng.choice(d.n_gates, 50, replace=False)])
    fdl, cl = oracle.fd_load(d, lib, rr, res["load"], res["net_delay"].astype(np.float64), pa.astype(np.float64),
                             rat, oracle.LATE, gates, h=1e-3)
    say(f"load FD: {cl.sum()} of {gates.size} clean")
    assert cl.mean() >= 0.98
    got = g_load[d.n_pi + gates]
    np.testing.assert_allclose(got[cl], fdl[cl], rtol=1e-4, atol=1e-4)


def test_autograd_tns_gradients():
    import torch
    from paper_2203_08395_amd import adjoint
    d, lib, pa, ps, late, early, modes = _setup(seed=45, n_pins=15000, n_levels=60)
    say(f"[gpu case] autograd TNS: pins={d.n_pins}")
    r = _gpu(d, lib, pa, ps, late, early, modes)
    g = r["g"]
    td = adjoint.TimedDesign(g, r["L"], r["views"], r["pi"], r["rat"], r["nd"]["net_imp2"])
    A, D = d.n_arcs, d.n_drivers
    nd = r["nd"]["net_delay"][:A].clone().requires_grad_(True)
    ld = r["nd"]["load"][:D].clone().requires_grad_(True)
    tns = adjoint.tns(nd, ld, td)
    w = torch.tensor([2.0, -0.5], dtype=torch.float64, device="cuda")
    (tns * w).sum().backward()
    res = _oracle(d, lib, pa, ps, late, early)
    assert float(tns[0]) == res["late"]["tns"] and float(tns[1]) == res["early"]["tns"]
    want_nd = np.zeros(A)
    want_ld = np.zeros(D)
    for v, key in enumerate(("late", "early")):
        g_at, g_arc = oracle.tns_adjoint(d, res[key], LATE if key == "late" else EARLY)
        want_nd += float(w[v]) * g_arc
        want_ld[d.n_pi:] += float(w[v]) * g_at[d.n_pi:] * oracle.load_slope(d, lib, res[key], res["load"])
    np.testing.assert_array_equal(g.arc_to_input(nd.grad.cpu().numpy()), want_nd.astype(np.float32))
    np.testing.assert_allclose(g.drv_to_input(ld.grad.cpu().numpy()), want_ld, rtol=2e-5,
                               atol=2e-5 * max(1.0, np.abs(want_ld).max()))
    # gradients accumulate across calls like any autograd leaf
    tns_b = adjoint.tns(nd, ld, td)
    tns_b.sum().backward()
    g1 = want_nd + sum(oracle.tns_adjoint(d, res[k], m)[1] for k, m in (("late", LATE), ("early", EARLY)))
    np.testing.assert_array_equal(g.arc_to_input(nd.grad.cpu().numpy()), g1.astype(np.float32))


def test_autograd_tns_two_forwards_then_backward():
    """Two forward evaluations at different net delays, then backward of the first only:
    the gradients are those of the first point (the shared buffers hold the second)."""
    import torch
    from paper_2203_08395_amd import adjoint
    d, lib, pa, ps, late, early, modes = _setup(seed=47, n_pins=12000, n_levels=50)
    say(f"[gpu case] autograd TNS, two forwards: pins={d.n_pins}")
    r = _gpu(d, lib, pa, ps, late, early, modes)
    g = r["g"]
    td = adjoint.TimedDesign(g, r["L"], r["views"], r["pi"], r["rat"], r["nd"]["net_imp2"])
    A, D = d.n_arcs, d.n_drivers
    base_nd = r["nd"]["net_delay"][:A].clone()
    ld = r["nd"]["load"][:D].clone()
    x1 = base_nd.clone().requires_grad_(True)
    # the second point: every net delay 25 ps later, which moves slacks and argmaxes
    x2 = (base_nd + 25.0).requires_grad_(True)
    t1 = adjoint.tns(x1, ld, td)
    t2 = adjoint.tns(x2, ld, td)
    t1.sum().backward()
    res = _oracle(d, lib, pa, ps, late, early)
    assert float(t1[0]) == res["late"]["tns"] and float(t1[1]) == res["early"]["tns"]
    want = sum(oracle.tns_adjoint(d, res[k], m)[1] for k, m in (("late", LATE), ("early", EARLY)))
    np.testing.assert_array_equal(g.arc_to_input(x1.grad.cpu().numpy()), want.astype(np.float32))
    assert x2.grad is None
    # the second point's gradient is its own (not the first's)
    t2.sum().backward()
    assert not torch.equal(x2.grad, x1.grad)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_critical_paths_match_oracle(cfg):
    import torch
    d, lib, pa, ps, late, early, modes = _setup(cfg)
    say(f"[gpu case] critical paths {cfg}: pins={d.n_pins}")
    r = _gpu(d, lib, pa, ps, late, early, modes)
    g = r["g"]
    res = _oracle(d, lib, pa, ps, late, early)
    for v, key in enumerate(("late", "early")):
        for k in (1, 17, 64):
            out = sta.critical_paths(g, r["views"], v, k, r["t"], r["s"])
            torch.cuda.synchronize()
            h = {n: x.cpu().numpy() for n, x in out.items()}
            want = oracle.critical_paths(d, res[key], k)
            assert list(h["ep_rank"]) == [p[0] for p in want]
            np.testing.assert_array_equal(h["slack"], np.array([p[1] for p in want], np.float32))
            for i, (_, _, drv, arcs) in enumerate(want):
                n = int(h["len"][i])
                assert n == len(drv)
                assert list(g.drv_input[h["drv"][i, :n]]) == drv
                assert list(g.arc_input[h["arc"][i, :n - 1]]) == arcs


def test_analysis_argument_errors():
    import torch
    d, lib, pa, ps, late, early, modes = _setup(seed=46, n_pins=3000, n_levels=20)
    r = _gpu(d, lib, pa, ps, late, early, modes)
    g = r["g"]
    with pytest.raises(sta.StaError):
        sta.critical_paths(g, r["views"], 0, 0, r["t"], r["s"])
    with pytest.raises(sta.StaError):
        sta.critical_paths(g, r["views"], 0, 65, r["t"], r["s"])
    with pytest.raises(sta.StaError):
        sta.critical_paths(g, r["views"], 2, 4, r["t"], r["s"])
    with pytest.raises(sta.StaError):
        sta.tns_adjoint(g, None, r["views"], r["nd"], r["t"], r["s"])   # g_load needs the library
    out = sta.alloc_adjoint(g, 2, arcs=False, load=False)
    sta.tns_adjoint(g, None, r["views"], r["nd"], r["t"], r["s"], out=out)
    torch.cuda.synchronize()
