"""Pins of the TNS adjoint and critical-path reference (CPU only).

The FP64 perturbation engine is checked against a from-scratch longest-path recomputation;
the chain-rule adjoint is checked against central finite differences of that engine and
against an independent count of failing endpoints per arc by explicit backtrace; the
load gradient against finite differences of the FP64 table lookup."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen


def _small(seed, n_pins=1500, n_levels=25):
    d = gen.make_design(n_pins=n_pins, n_levels=n_levels, fanin="uniform4", seed=seed)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d, seed=seed)
    late, early = gen.make_rat(d, n_levels, 60.0, 92)
    res = oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY))
    return d, lib, pa, late, early, res


def _tns_brute(d, arc_delay, net_delay, pi_at, rat_drv, mode):
    """Longest (shortest, early) path by repeated relaxation until nothing changes, then
    TNS with math.fsum; independent of any level order."""
    import math
    D = d.n_pi + d.n_gates
    at = np.full(D, np.nan)
    at[:d.n_pi] = pi_at
    ptr = d.gate_arc_ptr
    changed = True
    while changed:
        changed = False
        for g in range(d.n_gates):
            a = np.arange(ptr[g], ptr[g + 1])
            src = at[d.arc_drv[a]]
            if np.any(np.isnan(src)):
                continue
            c = src + net_delay[a] + arc_delay[a]
            v = c.max() if mode == oracle.LATE else c.min()
            if at[d.n_pi + g] != v:
                at[d.n_pi + g] = v
                changed = True
    ep = oracle.endpoints(d)
    s = (rat_drv[ep] - at[ep]) if mode == oracle.LATE else (at[ep] - rat_drv[ep])
    return math.fsum(np.minimum(s, 0.0).tolist())


@pytest.mark.parametrize("mode", [oracle.LATE, oracle.EARLY])
def test_tns_delta_matches_full_recomputation(mode):
    d, lib, pa, late, early, res = _small(31, n_pins=400, n_levels=12)
    key = "late" if mode == oracle.LATE else "early"
    r = res[key]
    ad = r["arc_delay"].astype(np.float64)
    nd = res["net_delay"].astype(np.float64)
    rat = oracle.ep_rat_by_driver(d, late if mode == oracle.LATE else early)
    rng = np.random.default_rng(1)
    gates = rng.choice(d.n_gates, 12, replace=False)
    pg, po, pd = [], [0], []
    for g in gates:
        a = np.arange(d.gate_arc_ptr[g], d.gate_arc_ptr[g + 1])
        pg.append(int(g))
        pd.extend((ad[a] + rng.uniform(-20, 20, a.size)).tolist())
        po.append(len(pd))
    base, delta = oracle.tns_delta(d, ad, nd, pa.astype(np.float64), rat, mode, pg, po, pd)
    assert base == pytest.approx(_tns_brute(d, ad, nd, pa, rat, mode), abs=1e-9)
    for i, g in enumerate(gates):
        ad2 = ad.copy()
        ad2[d.gate_arc_ptr[g]:d.gate_arc_ptr[g + 1]] = pd[po[i]:po[i + 1]]
        want = _tns_brute(d, ad2, nd, pa, rat, mode) - _tns_brute(d, ad, nd, pa, rat, mode)
        assert delta[i] == pytest.approx(want, abs=1e-7)


@pytest.mark.parametrize("mode", [oracle.LATE, oracle.EARLY])
def test_adjoint_matches_finite_differences(mode):
    d, lib, pa, late, early, res = _small(32)
    key = "late" if mode == oracle.LATE else "early"
    r = res[key]
    g_at, g_arc = oracle.tns_adjoint(d, r, mode)
    rat = oracle.ep_rat_by_driver(d, late if mode == oracle.LATE else early)
    rng = np.random.default_rng(2)
    nz = np.nonzero(g_arc)[0]
    assert nz.size > 5
    arcs = np.concatenate([rng.choice(nz, min(nz.size, 100), replace=False),
                           rng.choice(d.arc_drv.shape[0], 100, replace=False)])
    fd, clean = oracle.fd_arc_delay(d, r["arc_delay"].astype(np.float64), res["net_delay"].astype(np.float64),
                                    pa.astype(np.float64), rat, mode, arcs)
    assert clean.mean() > 0.95
    np.testing.assert_allclose(fd[clean], g_arc[arcs][clean], atol=1e-6)
    gates = np.unique(np.concatenate([np.nonzero(g_at[d.n_pi:])[0][:60], rng.choice(d.n_gates, 40)]))
    fdl, cl = oracle.fd_load(d, lib, r, res["load"], res["net_delay"].astype(np.float64), pa.astype(np.float64),
                             rat, mode, gates)
    gl = g_at[d.n_pi + gates] * oracle.load_slope(d, lib, r, res["load"])[gates]
    assert cl.mean() > 0.95 and np.count_nonzero(gl) > 0
    np.testing.assert_allclose(fdl[cl], gl[cl], rtol=1e-6, atol=1e-6)


def test_adjoint_counts_failing_paths_through_each_arc():
    d, lib, pa, late, early, res = _small(33)
    r = res["late"]
    g_at, g_arc = oracle.tns_adjoint(d, r, oracle.LATE)
    count = np.zeros(d.arc_drv.shape[0])
    ep = oracle.endpoints(d)
    for e in ep[r["slack_drv"][ep] < 0]:
        u = int(e)
        while u >= d.n_pi:
            g = u - d.n_pi
            a = int(d.gate_arc_ptr[g] + r["argmax"][g])
            count[a] += 1
            u = int(d.arc_drv[a])
    np.testing.assert_array_equal(g_arc, -count)
    # dTNS/dAT of a primary input = minus the failing paths that start there
    starts = np.zeros(d.n_pi)
    for e in ep[r["slack_drv"][ep] < 0]:
        u = int(e)
        while u >= d.n_pi:
            g = u - d.n_pi
            u = int(d.arc_drv[int(d.gate_arc_ptr[g] + r["argmax"][g])])
        starts[u] += 1
    np.testing.assert_array_equal(g_at[:d.n_pi], -starts)


def test_critical_paths_are_consistent_argmax_chains():
    d, lib, pa, late, early, res = _small(34)
    r = res["late"]
    paths = oracle.critical_paths(d, r, 10)
    ep = oracle.endpoints(d)
    worst = np.sort(r["slack_drv"][ep])[:10]
    np.testing.assert_array_equal([p[1] for p in paths], worst.astype(np.float32))
    for rank, s, drv, arcs in paths:
        assert drv[0] == ep[rank] and drv[-1] < d.n_pi and len(drv) == len(arcs) + 1
        for i, a in enumerate(arcs):
            # the arc leads from drv[i+1] into drv[i], and its arrival is the gate's
            o = drv[i]
            assert d.arc_drv[a] == drv[i + 1]
            assert r["at_in"][a] + r["arc_delay"][a] == r["at_drv"][o]
