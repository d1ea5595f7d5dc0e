"""Pins of the oracle's RC delay calculation (step 2) against closed forms and an
independent O(n^2) moment definition.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from tests import tiny

HERE = os.path.dirname(os.path.abspath(__file__))


def _one_net_design(parent, R, C, taps, pincaps):
    """PI 0 drives the given net; each tap feeds a one-input gate; gate nets are 1 node."""
    gates = [[0] for _ in taps]
    nets = [(list(parent), list(R), list(C))] + [([-1], [0.0], [0.5]) for _ in taps]
    return tiny.design(1, gates, nets, pincaps=pincaps, taps=taps)


def test_single_rc_closed_form():
    # one resistor into one capacitor: impulse response exp(-t/tau)/tau, mean tau, variance tau^2
    d = _one_net_design([-1, 0], [0.0, 200.0], [0.0, 0.0], [1], [3.0])
    load, nd, ni, m1, m2, cd = oracle.delay_calc(d, moments=True)
    tau = 200.0 * 3.0 * 1e-3
    assert abs(m1[1] - tau) <= 1e-15 * tau
    assert abs((2 * m2[1] - m1[1] ** 2) - tau ** 2) <= 1e-14 * tau ** 2
    assert load[0] == np.float32(3.0)
    assert nd[0] == np.float32(tau)
    assert abs(ni[0] - np.float32(0.36)) <= 1e-7


@pytest.mark.parametrize("n", [1, 2, 5, 16, 100])
def test_uniform_chain_closed_form(n):
    # n equal segments R/n with caps C/n at nodes 1..n: far-end Elmore = RC(n+1)/(2n)
    Rt, Ct = 300.0, 4.0
    C = [0.0] + [Ct / n] * n
    R = [0.0] + [Rt / n] * n
    parent = list(range(-1, n))
    d = _one_net_design(parent, R, C, [n], [0.0])
    load, nd, ni, m1, m2, cd = oracle.delay_calc(d, moments=True)
    # inputs are FP32: use the rounded segment values, RC(n+1)/(2n) = r c n(n+1)/2
    r, c = float(np.float32(Rt / n)), float(np.float32(Ct / n))
    expect = r * c * n * (n + 1) / 2 * 1e-3
    assert abs(m1[n] - expect) <= 1e-13 * expect
    assert abs(expect - Rt * Ct * (n + 1) / (2 * n) * 1e-3) <= 1e-6 * expect
    assert abs(cd[0] - c * n) <= 1e-14 * c * n


def test_hand_chain_fixture():
    g = json.load(open(os.path.join(HERE, "golden", "hand_chain.json")))
    R = [0.0 if r is None else r for r in g["edge_R_ohm"]]
    d = _one_net_design([-1, 0, 1], R, g["wire_cap_fF"], [g["sink_node"]], [g["sink_pin_cap_fF"]])
    load, nd, ni, m1, m2, cd = oracle.delay_calc(d, moments=True)
    e = g["expect"]
    np.testing.assert_allclose(cd[:3], e["downstream_cap_fF"], rtol=1e-15)
    np.testing.assert_allclose(m1[:3], e["m1_ps"], rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(m2[:3], e["m2_ps2"], rtol=1e-14, atol=1e-300)
    assert load[0] == np.float32(e["load_fF"])
    assert abs(float(ni[0]) - e["imp2_sink_ps2"]) <= 1e-7 * e["imp2_sink_ps2"]
    # propagate through the sink: AT = 10 + 0.896, slew = sqrt(400 + 0.671744)
    from paper_2203_08395_amd import gen
    lib = gen.make_library(n_tables=1, seed=1)
    p = oracle.propagate(d, lib.x, lib.y, lib.tab, load, nd, ni,
                         np.array([g["pi_at_ps"]], np.float32), np.array([g["pi_slew_ps"]], np.float32))
    ulp = np.spacing(np.float32(e["sink_at_ps"]))
    assert abs(float(p["at_in"][0]) - e["sink_at_ps"]) <= ulp
    ulp = np.spacing(np.float32(e["sink_slew_ps"]))
    assert abs(float(p["slew_in"][0]) - e["sink_slew_ps"]) <= ulp


def _rph_moments(parent, R, Ctot):
    """Rubinstein-Penfield-Horowitz: m1_k = sum_j R_kj C_j, m2_k = sum_j R_kj C_j m1_j,
    R_kj = resistance shared by the root->k and root->j paths.  O(n^2), written from the sets."""
    n = len(parent)
    paths = []
    for k in range(n):
        s, v = set(), k
        while v > 0:
            s.add(v)
            v = parent[v]
        paths.append(s)
    Rkj = np.zeros((n, n))
    for k in range(n):
        for j in range(n):
            Rkj[k, j] = sum(R[e] for e in paths[k] & paths[j])
    m1 = (Rkj * np.asarray(Ctot)[None, :]).sum(axis=1) * 1e-3
    m2 = (Rkj * (np.asarray(Ctot) * m1)[None, :]).sum(axis=1) * 1e-3
    return m1, m2


@pytest.mark.parametrize("seed", range(8))
def test_two_pass_matches_rph_on_random_trees(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    parent = [-1] + [int(rng.integers(0, k)) for k in range(1, n)]
    R = [0.0] + list(rng.uniform(10, 500, n - 1).astype(np.float32).astype(float))
    C = list(rng.uniform(0.1, 5, n).astype(np.float32).astype(float))
    ns = int(rng.integers(1, 6))
    taps = [int(t) for t in rng.integers(0, n, ns)]
    caps = list(rng.uniform(1, 4, ns).astype(np.float32).astype(float))
    d = _one_net_design(parent, R, C, taps, caps)
    load, nd, ni, m1, m2, cd = oracle.delay_calc(d, moments=True)
    Ctot = np.array(C, dtype=np.float64)
    for t, c in zip(taps, caps):
        Ctot[t] += c
    e1, e2 = _rph_moments(parent, R, Ctot)
    np.testing.assert_allclose(m1[:n], e1, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(m2[:n], e2, rtol=1e-12, atol=1e-300)
    assert abs(load[0] - np.float32(Ctot.sum())) <= np.spacing(np.float32(Ctot.sum()))
    # Elmore bounds: R_path*Cd(sink) <= m1(sink) <= R_path*load
    for i, t in enumerate(taps):
        v, rp = t, 0.0
        while v > 0:
            rp += R[v]
            v = parent[v]
        assert rp * cd[t] * 1e-3 <= m1[t] * (1 + 1e-12)
        assert m1[t] <= rp * Ctot.sum() * 1e-3 * (1 + 1e-12)
        assert ni[i] >= 0.0


def test_generated_design_load_equals_total_cap():
    from paper_2203_08395_amd import gen
    d = gen.make_design(**gen.CONFIGS["c1"])
    load, nd, ni = oracle.delay_calc(d)
    tot = np.zeros(d.n_drivers)
    np.add.at(tot, np.repeat(np.arange(d.n_drivers), np.diff(d.net_node_ptr)), d.node_C.astype(np.float64))
    np.add.at(tot, d.arc_drv, d.arc_pincap.astype(np.float64))
    np.testing.assert_allclose(load, tot, rtol=2e-7)
    assert (nd > 0).all() and (ni >= 0).all()


def test_bad_tap_is_rejected():
    d = _one_net_design([-1, 0], [0.0, 100.0], [1.0, 1.0], [1], [1.0])
    d.arc_tap[0] = 5
    with pytest.raises(oracle.OracleError):
        oracle.delay_calc(d)
