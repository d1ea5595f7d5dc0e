"""Seeded synthetic timing designs, cell libraries and per-view inputs.

This module only draws inputs. It holds none of the timing arithmetic: no
levelization, no RC moments, no table interpolation, no propagation. Both the
CPU oracle (through the tests and the benchmark's CPU leg) and the HIP path
consume exactly the arrays it returns.

Design model (the paper states no netlist model; the timing experiment of
Section IV-A only says a timer analyses a million-gate design per view):

* drivers: primary inputs 0..n_pi-1, then gate outputs n_pi..n_pi+G-1;
* gate g has k >= 1 input pins, its cell arcs ``gate_arc_ptr[g]..gate_arc_ptr[g+1]-1``;
  arc a joins input pin a (a sink of driver ``arc_drv[a]``'s net) to g's output;
* every driver owns an RC net with nodes ``net_node_ptr[d]..net_node_ptr[d+1]-1``;
  local node 0 is the driver tap, ``node_parent`` is local with parent < child,
  ``node_R`` is the resistance of the edge parent->node (ohm), ``node_C`` the wire cap
  at the node (fF); input pin a taps local node ``arc_tap[a]`` with ``arc_pincap[a]`` fF;
* a driver with no sink is a timing endpoint.

Gate ids are randomly permuted, so the input numbering is not a level order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_AXIS = 7
AXIS_X = np.array([5.0 * 100.0 ** (i / 6.0) for i in range(N_AXIS)], dtype=np.float32)   # input slew, ps
AXIS_Y = np.array([200.0 ** (j / 6.0) for j in range(N_AXIS)], dtype=np.float32)         # load, fF
CORNER_KAPPAS = (0.8, 1.0, 1.1, 1.3)


@dataclasses.dataclass
class Design:
    n_pi: int
    n_gates: int
    gate_arc_ptr: np.ndarray   # int32[G+1]
    arc_drv: np.ndarray        # int32[A]
    arc_tbl: np.ndarray        # int32[A]
    arc_tap: np.ndarray        # int32[A]
    arc_pincap: np.ndarray     # float32[A]
    net_node_ptr: np.ndarray   # int32[D+1]
    node_parent: np.ndarray    # int32[M]
    node_R: np.ndarray         # float32[M]
    node_C: np.ndarray         # float32[M]
    n_levels_built: int = 0    # level count the generator aimed for (metadata only)

    @property
    def n_drivers(self) -> int:
        return self.n_pi + self.n_gates

    @property
    def n_arcs(self) -> int:
        return int(self.arc_drv.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.node_R.shape[0])

    @property
    def n_pins(self) -> int:
        # primary inputs + gate outputs + gate input pins
        return self.n_drivers + self.n_arcs

    def counts(self) -> dict:
        return {"pins": self.n_pins, "pi": self.n_pi, "gates": self.n_gates,
                "arcs": self.n_arcs, "drivers": self.n_drivers, "rc_nodes": self.n_nodes}


@dataclasses.dataclass
class Library:
    x: np.ndarray       # float32[7] input-slew axis (ps)
    y: np.ndarray       # float32[7] load axis (fF)
    tab: np.ndarray     # float32[K, 2, 7, 7]: [table][delay|slew][slew index][load index]

    @property
    def n_tables(self) -> int:
        return int(self.tab.shape[0])


def _fanin(rng: np.random.Generator, kind: str, n: int) -> np.ndarray:
    if kind == "uniform4":
        return rng.integers(1, 5, size=n).astype(np.int64)
    if kind == "geom":
        k = rng.geometric(0.4, size=n)
        bad = k > 16
        while bad.any():                      # truncation by redrawing = conditioning on k <= 16
            k[bad] = rng.geometric(0.4, size=int(bad.sum()))
            bad = k > 16
        return k.astype(np.int64)
    if kind.startswith("fixed"):
        return np.full(n, int(kind[5:]), dtype=np.int64)
    raise ValueError(kind)


def _expected_fanin(kind: str) -> float:
    if kind == "uniform4":
        return 2.5
    if kind == "geom":
        p, q = 0.4, 0.6
        w = np.array([q ** (k - 1) * p for k in range(1, 17)])
        return float((w * np.arange(1, 17)).sum() / w.sum())
    return float(kind[5:])


def _rc_nets(rng, n_drv, m_lo, m_hi, tree):
    m = rng.integers(m_lo, m_hi + 1, size=n_drv).astype(np.int64)
    ptr = np.zeros(n_drv + 1, dtype=np.int64)
    np.cumsum(m, out=ptr[1:])
    tot = int(ptr[-1])
    local = np.arange(tot, dtype=np.int64) - np.repeat(ptr[:-1], m)
    if tree:
        # random recursive tree: parent of local node k is uniform on 0..k-1
        u = rng.random(tot)
        parent = np.floor(u * local).astype(np.int64)
    else:
        parent = local - 1
    parent[local == 0] = -1
    R = rng.uniform(10.0, 500.0, size=tot).astype(np.float32)
    R[local == 0] = 0.0
    C = rng.uniform(0.1, 5.0, size=tot).astype(np.float32)
    return m, ptr, parent, R, C


def make_design(n_pins: int, n_levels: int, fanin: str = "uniform4", seed: int = 1,
                n_fanout64: int = 0, m_range=(2, 8), tree: bool = False,
                n_tables: int = 128, shuffle: bool = True) -> Design:
    """Random levelized DAG of about ``n_pins`` pins in ``n_levels`` gate levels.

    Each gate at level l takes one input from a driver at level l-1 and its other
    inputs from distinct drivers drawn uniformly over all levels below l, so the
    gate levels are exactly 1..n_levels.  ``n_fanout64`` drivers are rewired to
    drive exactly 64 sinks.  Nets are RC chains (or random recursive trees) with
    ``m_range`` nodes, R ~ U[10,500] ohm, C ~ U[0.1,5] fF; pin caps ~ U[1,4] fF.
    """
    rng = np.random.default_rng(seed)
    kbar = _expected_fanin(fanin)
    G = max(n_levels, int(round(n_pins / (1.0 + kbar + 1.0 / n_levels))))
    n_pi = max(2, int(round(G / n_levels)))
    per = np.full(n_levels, G // n_levels, dtype=np.int64)
    per[: G % n_levels] += 1
    gstart = np.zeros(n_levels + 1, dtype=np.int64)
    np.cumsum(per, out=gstart[1:])

    kmax = 16 if fanin == "geom" else (4 if fanin == "uniform4" else int(fanin[5:]))
    rows = np.full((G, kmax), -1, dtype=np.int64)     # generation ids of input drivers, col 0 = level-defining
    ks = np.zeros(G, dtype=np.int64)
    for lv in range(n_levels):
        g0, g1 = int(gstart[lv]), int(gstart[lv + 1])
        ng = g1 - g0
        if lv == 0:
            plo, phi = 0, n_pi
        else:
            plo, phi = n_pi + int(gstart[lv - 1]), n_pi + int(gstart[lv])
        n_earlier = n_pi + g0                         # drivers with level < lv+1
        k = np.minimum(_fanin(rng, fanin, ng), n_earlier)
        ks[g0:g1] = k
        M = rng.integers(0, n_earlier, size=(ng, kmax))
        M[:, 0] = rng.integers(plo, phi, size=ng)
        valid = np.arange(kmax)[None, :] < k[:, None]
        while True:
            dup = np.zeros_like(valid)
            for c in range(1, kmax):
                same = (M[:, :c] == M[:, c:c + 1]) & valid[:, :c]
                dup[:, c] = valid[:, c] & same.any(axis=1)
            if not dup.any():
                break
            M[dup] = rng.integers(0, n_earlier, size=int(dup.sum()))
        M[~valid] = -1
        rows[g0:g1] = M

    gate_level = np.repeat(np.arange(1, n_levels + 1), per)
    drv_level = np.concatenate([np.zeros(n_pi, dtype=np.int64), gate_level])

    if n_fanout64 > 0:
        fo = np.bincount(rows[rows >= 0], minlength=n_pi + G)
        cand = np.nonzero(drv_level <= n_levels - 2)[0]
        chosen = rng.choice(cand, size=min(n_fanout64, cand.size), replace=False)
        for d in chosen:
            need = 64 - int(fo[d])
            if need <= 0:
                continue
            lv = int(drv_level[d])
            pool = np.arange(int(gstart[lv]), G)       # gates above d's level
            pool = pool[(ks[pool] >= 2) & ~(rows[pool] == d).any(axis=1)]
            if pool.size < need:
                continue
            pick = rng.choice(pool, size=need, replace=False)
            col = 1 + np.floor(rng.random(need) * (ks[pick] - 1)).astype(np.int64)
            old = rows[pick, col]
            rows[pick, col] = d
            np.subtract.at(fo, old, 1)
            fo[d] += need

    # shuffle the input order inside each gate, then the gate ids
    if shuffle:
        keys = rng.random((G, kmax))
        keys[rows < 0] = 2.0
        order = np.argsort(keys, axis=1, kind="stable")
        rows = np.take_along_axis(rows, order, axis=1)
        perm = rng.permutation(G)                      # generation gate j -> final gate perm[j]
    else:
        perm = np.arange(G)
    inv = np.empty(G, dtype=np.int64)
    inv[perm] = np.arange(G)
    drv_map = np.concatenate([np.arange(n_pi), n_pi + perm])
    rows_f = rows[inv]                                  # final gate order
    ks_f = ks[inv]
    gate_arc_ptr = np.zeros(G + 1, dtype=np.int64)
    np.cumsum(ks_f, out=gate_arc_ptr[1:])
    valid = rows_f >= 0
    arc_drv = drv_map[rows_f[valid]]                    # row-major: gates in order, inputs in order
    A = arc_drv.shape[0]
    D = n_pi + G

    m, net_ptr, parent, R, C = _rc_nets(rng, D, m_range[0], m_range[1], tree)
    # sink taps: a net's first sink (lowest arc id) taps the far end, others a uniform node 1..M-1
    order = np.argsort(arc_drv, kind="stable")
    sd = arc_drv[order]
    first = np.ones(A, dtype=bool)
    first[1:] = sd[1:] != sd[:-1]
    md = m[sd]
    tap_sorted = np.where(first, md - 1, 1 + np.floor(rng.random(A) * (md - 1)).astype(np.int64))
    arc_tap = np.empty(A, dtype=np.int64)
    arc_tap[order] = tap_sorted
    arc_pincap = rng.uniform(1.0, 4.0, size=A).astype(np.float32)
    arc_tbl = rng.integers(0, n_tables, size=A)

    return Design(
        n_pi=int(n_pi), n_gates=int(G),
        gate_arc_ptr=gate_arc_ptr.astype(np.int32), arc_drv=arc_drv.astype(np.int32),
        arc_tbl=arc_tbl.astype(np.int32), arc_tap=arc_tap.astype(np.int32),
        arc_pincap=arc_pincap, net_node_ptr=net_ptr.astype(np.int32),
        node_parent=parent.astype(np.int32), node_R=R, node_C=C, n_levels_built=int(n_levels))


def make_library(n_tables: int = 128, seed: int = 7, kappas=(1.0,), bilinear: bool = False) -> Library:
    """K delay/slew 7x7 table pairs on the shared geometric axes.

    delay = a + b*x + c*y + e*sqrt(x*y) with a~U[2,10] ps, b~U[0.05,0.3], c~U[0.5,3] ps/fF,
    e~U[0,0.2] (e = 0 when ``bilinear``); slew = a' + b'*x + c'*y with a'~U[3,8], b'~U[0.05,0.2],
    c'~U[1,2.5].  Sampled in FP64, rounded to FP32; a corner's tables are fl32(kappa*T) in FP32.
    Returns tables shaped [len(kappas), K, 2, 7, 7] when several kappas are given.
    """
    rng = np.random.default_rng(seed)
    x = AXIS_X.astype(np.float64)[:, None]
    y = AXIS_Y.astype(np.float64)[None, :]
    tab = np.empty((n_tables, 2, N_AXIS, N_AXIS), dtype=np.float32)
    for t in range(n_tables):
        a, b, c = rng.uniform(2, 10), rng.uniform(0.05, 0.3), rng.uniform(0.5, 3.0)
        e = 0.0 if bilinear else rng.uniform(0.0, 0.2)
        a2, b2, c2 = rng.uniform(3, 8), rng.uniform(0.05, 0.2), rng.uniform(1.0, 2.5)
        tab[t, 0] = (a + b * x + c * y + e * np.sqrt(x * y)).astype(np.float32)
        tab[t, 1] = (a2 + b2 * x + c2 * y + 0.0 * x * y).astype(np.float32)
    out = []
    for kap in kappas:
        out.append(tab if kap == 1.0 else (np.float32(kap) * tab).astype(np.float32))
    tabs = out[0] if len(kappas) == 1 else np.stack(out)
    return Library(x=AXIS_X.copy(), y=AXIS_Y.copy(), tab=tabs)


def make_pi(design: Design, seed: int = 11):
    """Primary-input arrival ~ U[0,50] ps and slew ~ U[5,50] ps (FP32)."""
    rng = np.random.default_rng(seed)
    at = rng.uniform(0.0, 50.0, size=design.n_pi).astype(np.float32)
    sl = rng.uniform(5.0, 50.0, size=design.n_pi).astype(np.float32)
    return at, sl


def endpoint_ids(design: Design) -> np.ndarray:
    """Drivers with no sink, ascending: the endpoint ranks used by the RAT arrays."""
    fo = np.bincount(design.arc_drv, minlength=design.n_drivers)
    return np.nonzero(fo == 0)[0].astype(np.int32)


def make_rat(design: Design, n_levels: int, late_per_level: float = 62.0, hold: float = 60.0):
    """Endpoint required times: one clock for setup (late) and one hold bound (early).

    Late RAT = ``late_per_level`` ps x levels for every endpoint; early RAT = ``hold`` ps.
    """
    n_ep = endpoint_ids(design).shape[0]
    late = np.full(n_ep, np.float32(late_per_level * n_levels), dtype=np.float32)
    early = np.full(n_ep, np.float32(hold), dtype=np.float32)
    return late, early


# Named workloads (sizes and distributions of the timing configurations)
CONFIGS = {
    "c1": dict(n_pins=10_000, n_levels=50, fanin="uniform4", seed=1, n_fanout64=0),
    "c2": dict(n_pins=1_000_000, n_levels=300, fanin="geom", seed=2, n_fanout64=16),
    "c5": dict(n_pins=2_000_000, n_levels=400, fanin="geom", seed=5, n_fanout64=32),
}

# Endpoint required times per workload: the clock per level and the hold bound were
# picked once so that about 10% of endpoints fail setup and 5% fail hold on the seed.
RAT_PARAMS = {
    "c1": dict(late_per_level=77.7, hold=92.0),
    "c2": dict(late_per_level=72.9, hold=150.0),
    "c5": dict(late_per_level=72.9, hold=150.0),
}


def c3_designs(n_designs: int = 64, seed: int = 3):
    """Pin counts log-uniform on [5k, 500k], levels round(30*sqrt(P/5k))."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_designs):
        p = int(round(math.exp(rng.uniform(math.log(5e3), math.log(5e5)))))
        lv = int(round(30 * math.sqrt(p / 5e3)))
        out.append(dict(n_pins=p, n_levels=lv, fanin="geom", seed=seed * 1000 + i,
                        n_fanout64=int(round(16 * p / 1e6))))
    return out


@dataclasses.dataclass
class TreeSet:
    """RC-tree nets on their own (the learned-surrogate workload): net n has nodes
    net_node_ptr[n]..net_node_ptr[n+1]-1 (local node 0 = driver), its sinks are
    sink_ptr[n]..sink_ptr[n+1]-1 tapping local node sink_node[s] with sink_pincap[s];
    drv_slew[n] is the slew of the net's driver."""
    net_node_ptr: np.ndarray   # int32[N+1]
    node_parent: np.ndarray    # int32[M] local
    node_R: np.ndarray         # float32[M]
    node_C: np.ndarray         # float32[M]
    sink_ptr: np.ndarray       # int32[N+1]
    sink_node: np.ndarray      # int32[S] local node index
    sink_pincap: np.ndarray    # float32[S]
    drv_slew: np.ndarray       # float32[N]

    @property
    def n_nets(self) -> int:
        return int(self.net_node_ptr.shape[0] - 1)

    @property
    def n_sinks(self) -> int:
        return int(self.sink_node.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.node_R.shape[0])

    def subset(self, n0: int, n1: int) -> "TreeSet":
        a, b = int(self.net_node_ptr[n0]), int(self.net_node_ptr[n1])
        s0, s1 = int(self.sink_ptr[n0]), int(self.sink_ptr[n1])
        return TreeSet(
            net_node_ptr=(self.net_node_ptr[n0:n1 + 1] - a).astype(np.int32),
            node_parent=self.node_parent[a:b].copy(), node_R=self.node_R[a:b].copy(),
            node_C=self.node_C[a:b].copy(),
            sink_ptr=(self.sink_ptr[n0:n1 + 1] - s0).astype(np.int32),
            sink_node=self.sink_node[s0:s1].copy(), sink_pincap=self.sink_pincap[s0:s1].copy(),
            drv_slew=self.drv_slew[n0:n1].copy())


def make_rc_trees(n_nets: int, m_range=(2, 64), seed: int = 4) -> TreeSet:
    """Random recursive RC trees (parent of node k uniform on 0..k-1), M ~ U{m_range},
    R ~ U[10,500] ohm, wire C ~ U[0.1,5] fF; every leaf is a sink with pin cap U[1,4] fF;
    driver slew ~ U[5,50] ps."""
    rng = np.random.default_rng(seed)
    m, ptr, parent, R, C = _rc_nets(rng, n_nets, m_range[0], m_range[1], tree=True)
    tot = int(ptr[-1])
    has_child = np.zeros(tot, dtype=bool)
    net_of = np.repeat(np.arange(n_nets), m)
    nonroot = parent >= 0
    has_child[(ptr[:-1][net_of] + parent)[nonroot]] = True
    local = np.arange(tot) - np.repeat(ptr[:-1], m)
    leaf = ~has_child & (local > 0)
    sink_global = np.nonzero(leaf)[0]
    sink_net = net_of[sink_global]
    cnt = np.bincount(sink_net, minlength=n_nets)
    sptr = np.zeros(n_nets + 1, dtype=np.int64)
    np.cumsum(cnt, out=sptr[1:])
    return TreeSet(net_node_ptr=ptr.astype(np.int32), node_parent=parent.astype(np.int32), node_R=R, node_C=C,
                   sink_ptr=sptr.astype(np.int32), sink_node=local[sink_global].astype(np.int32),
                   sink_pincap=rng.uniform(1.0, 4.0, size=sink_global.shape[0]).astype(np.float32),
                   drv_slew=rng.uniform(5.0, 50.0, size=n_nets).astype(np.float32))
