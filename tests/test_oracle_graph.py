"""Pins of the oracle's levelization, propagation and slack (steps 1, 4-6) by brute
force on tiny DAGs, a closed-form chain and invariants.  CPU only."""
import functools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen
from tests import tiny

f32 = np.float32


def _levels_dfs(d):
    """Longest path in hops from any primary input, by memoised recursion."""
    gp, drv = d.gate_arc_ptr, d.arc_drv

    @functools.lru_cache(maxsize=None)
    def lev(u):
        if u < d.n_pi:
            return 0
        g = u - d.n_pi
        return 1 + max(lev(int(drv[a])) for a in range(gp[g], gp[g + 1]))

    import sys
    sys.setrecursionlimit(100000)
    return np.array([lev(u) for u in range(d.n_drivers)])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_levels_match_dfs(seed):
    d = gen.make_design(n_pins=4000, n_levels=30, fanin="geom", seed=seed, n_fanout64=2)
    lv, topo = oracle.levelize(d)
    assert np.array_equal(lv, _levels_dfs(d))
    assert lv.max() == 30
    # topo is a topological order of the gates
    pos = np.empty(d.n_gates, np.int64)
    pos[topo] = np.arange(d.n_gates)
    for g in range(d.n_gates):
        for a in range(d.gate_arc_ptr[g], d.gate_arc_ptr[g + 1]):
            u = d.arc_drv[a]
            if u >= d.n_pi:
                assert pos[u - d.n_pi] < pos[g]


def test_cycle_rejected():
    d = tiny.design(1, [[0, 2], [1]], [tiny.chain_net([100.0], [1.0, 1.0])] * 3)
    with pytest.raises(oracle.OracleError, match="CYCLE"):
        oracle.levelize(d)


def _random_tiny(seed, n_gates=None):
    rng = np.random.default_rng(seed)
    n_pi = int(rng.integers(1, 4))
    G = int(n_gates or rng.integers(2, 13))
    gates = []
    for g in range(G):
        avail = n_pi + g
        k = int(rng.integers(1, min(3, avail) + 1))
        gates.append([int(x) for x in rng.choice(avail, size=k, replace=False)])
    order = rng.permutation(G)           # relabel so that ids are not a topological order
    inv = np.argsort(order)
    relabel = lambda u: u if u < n_pi else n_pi + int(inv[u - n_pi])
    gates2 = [None] * G
    for g in range(G):
        gates2[inv[g]] = [relabel(u) for u in gates[g]]
    nets = []
    for _ in range(n_pi + G):
        m = int(rng.integers(2, 5))
        nets.append(tiny.chain_net(list(rng.uniform(10, 500, m - 1)), list(rng.uniform(0.1, 5, m))))
    A = sum(len(x) for x in gates2)
    caps = list(rng.uniform(1, 4, A))
    tbl = list(rng.integers(0, 4, A))
    d = tiny.design(n_pi, gates2, nets, pincaps=caps, tables=tbl)
    lib = gen.make_library(n_tables=4, seed=seed)
    at = rng.uniform(0, 50, n_pi).astype(f32)
    sl = rng.uniform(5, 50, n_pi).astype(f32)
    return d, lib, at, sl


def _paths_forward(d, nd, dl, pi_at, better):
    """AT of every pin = best over all PI->pin paths of the left-folded FP32 sum."""
    gp, drv = d.gate_arc_ptr, d.arc_drv
    memo = {}

    def sums(u):                      # every path sum ending at driver u
        if u in memo:
            return memo[u]
        if u < d.n_pi:
            out = [f32(pi_at[u])]
        else:
            g = u - d.n_pi
            out = []
            for a in range(gp[g], gp[g + 1]):
                for x in sums(int(drv[a])):
                    out.append(f32(f32(x + nd[a]) + dl[a]))
        memo[u] = out
        return out

    at_drv = np.array([better(sums(u)) for u in range(d.n_drivers)], f32)
    at_in = np.array([better([f32(x + nd[a]) for x in sums(int(drv[a]))]) for a in range(len(drv))], f32)
    return at_drv, at_in


def _paths_backward(d, nd, dl, ep_rat, better):
    """RAT of every pin = best over all pin->endpoint paths of the backward FP32 fold."""
    gp, drv = d.gate_arc_ptr, d.arc_drv
    gate_of = np.repeat(np.arange(d.n_gates), np.diff(gp))
    fo = [[] for _ in range(d.n_drivers)]
    for a, u in enumerate(drv):
        fo[int(u)].append(a)
    ep = oracle.endpoints(d)
    rank = {int(u): i for i, u in enumerate(ep)}
    memo = {}

    def rin(a):                       # every required-time fold at input pin a
        o = d.n_pi + int(gate_of[a])
        return [f32(r - dl[a]) for r in rdrv(o)]

    def rdrv(u):
        if u in memo:
            return memo[u]
        if u in rank:
            out = [f32(ep_rat[rank[u]])]
        else:
            out = [f32(r - nd[a]) for a in fo[u] for r in rin(a)]
        memo[u] = out
        return out

    rat_drv = np.array([better(rdrv(u)) for u in range(d.n_drivers)], f32)
    rat_in = np.array([better(rin(a)) for a in range(len(drv))], f32)
    return rat_drv, rat_in


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("mode", [oracle.LATE, oracle.EARLY])
def test_brute_force_paths_bitwise(seed, mode):
    d, lib, at, sl = _random_tiny(seed)
    load, nd, ni = oracle.delay_calc(d)
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, at, sl, mode)
    fwd_best = max if mode == oracle.LATE else min
    at_drv, at_in = _paths_forward(d, nd, p["arc_delay"], at, fwd_best)
    assert np.array_equal(at_drv.view(np.uint32), p["at_drv"].view(np.uint32))
    assert np.array_equal(at_in.view(np.uint32), p["at_in"].view(np.uint32))
    ep = oracle.endpoints(d)
    rng = np.random.default_rng(seed)
    rat = rng.uniform(0, 2000, ep.size).astype(f32)
    s = oracle.slack(d, nd, p["arc_delay"], p["at_drv"], p["at_in"], rat, mode)
    bwd_best = min if mode == oracle.LATE else max
    rat_drv, rat_in = _paths_backward(d, nd, p["arc_delay"], rat, bwd_best)
    assert np.array_equal(rat_drv.view(np.uint32), s["rat_drv"].view(np.uint32))
    assert np.array_equal(rat_in.view(np.uint32), s["rat_in"].view(np.uint32))
    sign = 1 if mode == oracle.LATE else -1
    assert np.array_equal(s["slack_drv"], f32(sign) * (s["rat_drv"] - p["at_drv"]))
    assert np.array_equal(s["slack_in"], f32(sign) * (s["rat_in"] - p["at_in"]))


def test_three_gate_chain_closed_form():
    # PI -> g1 -> g2 -> g3, single-input gates, exactly bilinear tables (no sqrt term):
    # every stage follows d = a + b S + c L, s = a' + b' S + c' L with S = sqrt(S_u^2 + imp2)
    nets = [tiny.chain_net([120.0, 80.0], [0.3, 0.6, 0.9]) for _ in range(4)]
    d = tiny.design(1, [[0], [1], [2]], nets, pincaps=[2.0, 1.5, 3.0], tables=[0, 0, 0])
    lib = gen.make_library(n_tables=1, seed=5, bilinear=True)
    load, nd, ni, m1, m2, cd = oracle.delay_calc(d, moments=True)
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, np.array([7.0], f32), np.array([12.0], f32))
    # the generator's bilinear tables: recover a, b, c from three exact corner samples
    T, S = lib.tab[0, 0].astype(np.float64), lib.tab[0, 1].astype(np.float64)
    x, y = lib.x.astype(np.float64), lib.y.astype(np.float64)

    def coef(Tb):
        b = (Tb[1, 0] - Tb[0, 0]) / (x[1] - x[0])
        c = (Tb[0, 1] - Tb[0, 0]) / (y[1] - y[0])
        return Tb[0, 0] - b * x[0] - c * y[0], b, c

    (a, b, c), (a2, b2, c2) = coef(T), coef(S)
    at, slew = 7.0, 12.0
    for g in range(3):
        k = d.net_node_ptr[g] + d.arc_tap[g]
        imp2 = 2 * m2[k] - m1[k] ** 2
        at_in = at + m1[k]
        s_in = math.sqrt(slew * slew + imp2)
        L = cd[d.net_node_ptr[g + 1]]
        at = at_in + a + b * s_in + c * L
        slew = a2 + b2 * s_in + c2 * L
        assert abs(p["at_in"][g] - at_in) <= 2e-6 * at_in
        assert abs(p["at_drv"][g + 1] - at) <= 2e-6 * at
        assert abs(p["slew_drv"][g + 1] - slew) <= 2e-6 * slew


def test_invariants_on_c1():
    d = gen.make_design(**gen.CONFIGS["c1"])
    lib = gen.make_library()
    at, sl = gen.make_pi(d)
    load, nd, ni = oracle.delay_calc(d)
    for mode in (oracle.LATE, oracle.EARLY):
        p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, at, sl, mode)
        cand = p["at_in"] + p["arc_delay"]
        gate_of = np.repeat(np.arange(d.n_gates), np.diff(d.gate_arc_ptr))
        out = p["at_drv"][d.n_pi + gate_of]
        if mode == oracle.LATE:
            assert np.all(out >= cand)
        else:
            assert np.all(out <= cand)
        win = d.gate_arc_ptr[:-1] + p["argmax"]
        assert np.array_equal(out[win], cand[win])
        # the winner is the first arc reaching the extreme
        for g in range(0, d.n_gates, 7):
            seg = cand[d.gate_arc_ptr[g]:d.gate_arc_ptr[g + 1]]
            best = seg.max() if mode == oracle.LATE else seg.min()
            assert p["argmax"][g] == int(np.nonzero(seg == best)[0][0])
        # AT grows along every net arc and every cell arc (delays are positive here)
        assert np.all(p["at_in"] >= p["at_drv"][d.arc_drv])
        assert np.all(p["arc_delay"] > 0)


def test_tns_is_exact_sum():
    rng = np.random.default_rng(4)
    s = (rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000)).astype(f32)
    t = oracle.tns(s)
    exact = sum((Fraction(float(v)) for v in s if v < 0), Fraction(0))
    assert t == float(exact)
    seq = 0.0
    for v in s:
        if v < 0:
            seq += float(v)
    assert abs(seq - t) <= len(s) * 2.0 ** -53 * float(np.abs(s[s < 0].astype(np.float64)).sum())
    assert oracle.tns(np.array([1.0, 2.0], f32)) == 0.0


def test_wns_tns_on_c1():
    d = gen.make_design(**gen.CONFIGS["c1"])
    lib = gen.make_library()
    at, sl = gen.make_pi(d)
    late, early = gen.make_rat(d, 50, **gen.RAT_PARAMS["c1"])
    r = oracle.run(d, lib, at, sl, late, early, modes=(oracle.LATE, oracle.EARLY))
    ep = oracle.endpoints(d)
    for m in ("late", "early"):
        s = r[m]["slack_drv"][ep]
        assert r[m]["wns"] == s.min()
        assert 0.0 < (s < 0).mean() < 0.2
        assert r[m]["tns"] < 0


def test_ties_pick_first_arc():
    # identical drivers, nets, pin caps and tables make every candidate equal
    same = tiny.chain_net([100.0, 50.0], [0.5, 0.5, 0.5])
    one = ([-1], [0.0], [0.4])
    for n_in in (2, 3, 5):
        d = tiny.design(n_in, [list(range(n_in))[::-1]], [same] * n_in + [one],
                        pincaps=[2.0] * n_in, tables=[1] * n_in)
        lib = gen.make_library(n_tables=2, seed=3)
        load, nd, ni = oracle.delay_calc(d)
        for mode in (oracle.LATE, oracle.EARLY):
            p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni,
                                 np.full(n_in, 20.0, f32), np.full(n_in, 30.0, f32), mode)
            assert p["argmax"][0] == 0
    # arcs 1 and 2 tie above arc 0 (late) / below arc 0 (early)
    d = tiny.design(3, [[0, 1, 2]], [same] * 3 + [one], pincaps=[2.0] * 3, tables=[1] * 3)
    load, nd, ni = oracle.delay_calc(d)
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, np.array([5, 20, 20], f32),
                         np.full(3, 30.0, f32), oracle.LATE)
    assert p["argmax"][0] == 1
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, np.array([25, 10, 10], f32),
                         np.full(3, 30.0, f32), oracle.EARLY)
    assert p["argmax"][0] == 1


@pytest.mark.parametrize("mode", [oracle.LATE, oracle.EARLY])
def test_output_slew_is_worst_arc_slew(mode):
    # S_out = max (late) / min (early) over the gate's arcs of the slew-table lookup at the
    # arc's input slew and the output load; the lookup itself is pinned separately
    d = gen.make_design(**gen.CONFIGS["c1"])
    lib = gen.make_library()
    at, sl = gen.make_pi(d)
    load, nd, ni = oracle.delay_calc(d)
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, at, sl, mode)
    gate_of = np.repeat(np.arange(d.n_gates), np.diff(d.gate_arc_ptr))
    s_arc = np.empty(d.n_arcs, f32)
    d_arc = np.empty(d.n_arcs, f32)
    for a in range(d.n_arcs):
        L = load[d.n_pi + gate_of[a]]
        s_arc[a] = oracle.bilerp(lib.x, lib.y, lib.tab[d.arc_tbl[a], 1], p["slew_in"][a], L)[0]
        d_arc[a] = oracle.bilerp(lib.x, lib.y, lib.tab[d.arc_tbl[a], 0], p["slew_in"][a], L)[0]
    assert np.array_equal(d_arc, p["arc_delay"])
    red = np.maximum if mode == oracle.LATE else np.minimum
    worst = red.reduceat(s_arc, d.gate_arc_ptr[:-1])
    assert np.array_equal(worst, p["slew_drv"][d.n_pi:])
    # slews of input pins: quadrature of the driver slew and the net's spread (FP32, rounded)
    su = p["slew_drv"][d.arc_drv]
    assert np.array_equal(p["slew_in"], np.sqrt(su * su + ni))
