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
