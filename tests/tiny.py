"""Small hand-built designs for the CPU pins (no timing arithmetic here)."""
import numpy as np

from paper_2203_08395_amd.gen import Design


def design(n_pi, gates, nets, pincaps=None, tables=None, taps=None):
    """gates: list of input-driver lists; nets: per driver (parent, R, C) lists.

    Sinks tap the last node of their net unless ``taps`` gives the node per arc."""
    ptr = [0]
    drv = []
    for ins in gates:
        drv.extend(ins)
        ptr.append(len(drv))
    A = len(drv)
    D = n_pi + len(gates)
    assert len(nets) == D
    nptr = [0]
    par, R, C = [], [], []
    for (p, r, c) in nets:
        par.extend(p)
        R.extend(r)
        C.extend(c)
        nptr.append(len(par))
    nsz = np.diff(nptr)
    tap = [int(nsz[d]) - 1 for d in drv] if taps is None else list(taps)
    return Design(
        n_pi=n_pi, n_gates=len(gates),
        gate_arc_ptr=np.array(ptr, np.int32), arc_drv=np.array(drv, np.int32),
        arc_tbl=np.array(tables if tables is not None else [0] * A, np.int32),
        arc_tap=np.array(tap, np.int32),
        arc_pincap=np.array(pincaps if pincaps is not None else [2.0] * A, np.float32),
        net_node_ptr=np.array(nptr, np.int32), node_parent=np.array(par, np.int32),
        node_R=np.array(R, np.float32), node_C=np.array(C, np.float32))


def chain_net(R, C):
    """RC chain: node 0 = driver tap with wire cap C[0]; edge k-1 -> k has R[k]."""
    n = len(C)
    return (list(range(-1, n - 1)), [0.0] + list(R), list(C))


def wide_fanout_design(seed, n_pi=40, levels=24, width=60, big_levels=(6, 13), big_fanout=100):
    """A levelized random design in which one driver at each of ``big_levels`` feeds
    ``big_fanout`` extra gates (more sinks than one 64-lane tile holds), so the backward
    pass cannot tile that level and runs it as a level launch."""
    rng = np.random.default_rng(seed)
    gates, by_level = [], [list(range(n_pi))]
    nid = n_pi
    for l in range(1, levels + 1):
        ids = []
        lower = [u for lv in by_level for u in lv]
        for _ in range(width):
            ins = [int(rng.choice(by_level[l - 1]))] + [int(rng.choice(lower)) for _ in range(rng.integers(0, 3))]
            gates.append(ins)
            ids.append(nid)
            nid += 1
        by_level.append(ids)
    for lb in big_levels:
        b = by_level[lb][0]
        for _ in range(big_fanout):
            gates.append([b, int(rng.choice(by_level[lb - 1]))])
    D = n_pi + len(gates)
    nets = []
    for _ in range(D):
        m = int(rng.integers(2, 6))
        nets.append(chain_net(list(rng.uniform(10, 300, m - 1)), list(rng.uniform(0.2, 3, m))))
    A = sum(len(x) for x in gates)
    return design(n_pi, gates, nets, pincaps=list(rng.uniform(1, 4, A)), tables=list(rng.integers(0, 128, A)))
