"""CPU oracle for levelized static timing analysis -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The product (the HIP library and its binding) never imports it, and it never
imports the product.  Both sides consume the arrays of the seeded input generator.

The computation lives in ``sta_oracle.c`` (plain C, FP64 delay calculation, FP32
propagation with no contraction); this module marshals numpy arrays into it and forms
the endpoint summaries:

* WNS = the minimum endpoint slack (exact, FP32);
* TNS = the sum of the negative endpoint slacks, computed exactly and rounded once to
  FP64 (``math.fsum``), so it does not depend on any summation order.

The paper (Heteroflow, Section IV-A) prints no timing formula or value; no pin here
comes from it.  Every function is pinned by the CPU tests against closed forms, brute
force on tiny graphs, an independent O(n^2) moment definition and invariants.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

LATE, EARLY = 0, 1


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "sta_oracle.c"))):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.orc_levelize.argtypes = [I, I, P, P, P, P]
    lib.orc_delay_calc.argtypes = [I, P, P, P, P, I, P, P, P, P, P, P, P, P, P]
    lib.orc_bilerp.argtypes = [P, P, P, ctypes.c_float, ctypes.c_float]
    lib.orc_bilerp.restype = ctypes.c_float
    lib.orc_bilerp_many.argtypes = [P, P, P, I, P, P, P]
    lib.orc_propagate.argtypes = [I, I, I, P, P, P, I, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_slack.argtypes = [I, I, I, P, P, P, P, P, P, P, P, P, P, P]
    for f in ("orc_levelize", "orc_delay_calc", "orc_propagate", "orc_slack"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(rc, what):
    if rc != 0:
        names = {-1: "E_ARG", -2: "E_RANGE", -3: "E_CYCLE"}
        raise OracleError(f"{what}: {names.get(rc, rc)}")


def levelize(d):
    """Step 1: level of every driver (PI 0, gate output 1 + max fanin level) and Kahn order."""
    lib = _load()
    D = d.n_pi + d.n_gates
    level = np.zeros(D, dtype=np.int32)
    topo = np.zeros(max(d.n_gates, 1), dtype=np.int32)
    gp, ad = _c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32)
    _check(lib.orc_levelize(d.n_pi, d.n_gates, _p(gp), _p(ad), _p(level), _p(topo)), "levelize")
    return level, topo[: d.n_gates]


def delay_calc(d, moments: bool = False):
    """Step 2 (FP64 per net): load per driver, Elmore delay and imp2 per sink arc (FP32 rounded).

    With ``moments`` also returns the FP64 node arrays (m1, m2, downstream cap)."""
    lib = _load()
    D, A, M = d.n_pi + d.n_gates, d.arc_drv.shape[0], d.node_R.shape[0]
    load = np.zeros(D, dtype=np.float32)
    nd = np.zeros(A, dtype=np.float32)
    ni = np.zeros(A, dtype=np.float32)
    m1 = np.zeros(M, dtype=np.float64) if moments else None
    m2 = np.zeros(M, dtype=np.float64) if moments else None
    cd = np.zeros(M, dtype=np.float64) if moments else None
    arrs = [_c(d.net_node_ptr, np.int32), _c(d.node_parent, np.int32), _c(d.node_R, np.float32),
            _c(d.node_C, np.float32), _c(d.arc_drv, np.int32), _c(d.arc_tap, np.int32),
            _c(d.arc_pincap, np.float32)]
    rc = lib.orc_delay_calc(D, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]), A,
                            _p(arrs[4]), _p(arrs[5]), _p(arrs[6]), _p(load), _p(nd), _p(ni),
                            _p(m1), _p(m2), _p(cd))
    _check(rc, "delay_calc")
    if moments:
        return load, nd, ni, m1, m2, cd
    return load, nd, ni


def bilerp(x, y, T, s, l):
    """Step 3: FP32 bilinear lookup of one 7x7 table at arrays of (slew, load)."""
    lib = _load()
    s = _c(np.atleast_1d(s), np.float32)
    l = _c(np.atleast_1d(l), np.float32)
    out = np.zeros(s.shape[0], dtype=np.float32)
    x, y, T = _c(x, np.float32), _c(y, np.float32), _c(T, np.float32)
    lib.orc_bilerp_many(_p(x), _p(y), _p(T), s.shape[0], _p(s), _p(l), _p(out))
    return out


def propagate(d, lib_x, lib_y, lib_tab, load, net_delay, net_imp2, pi_at, pi_slew, mode=LATE):
    """Steps 4-5 (FP32): arrival time and slew of every pin, arc delays and the argmax arc."""
    lib = _load()
    D, A, G = d.n_pi + d.n_gates, d.arc_drv.shape[0], d.n_gates
    tab = _c(lib_tab, np.float32)
    K = tab.shape[0]
    out = dict(at_drv=np.zeros(D, np.float32), slew_drv=np.zeros(D, np.float32),
               at_in=np.zeros(A, np.float32), slew_in=np.zeros(A, np.float32),
               arc_delay=np.zeros(A, np.float32), argmax=np.zeros(max(G, 1), np.int32))
    ins = [_c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32), _c(d.arc_tbl, np.int32),
           _c(lib_x, np.float32), _c(lib_y, np.float32), tab, _c(load, np.float32),
           _c(net_delay, np.float32), _c(net_imp2, np.float32), _c(pi_at, np.float32),
           _c(pi_slew, np.float32)]
    rc = lib.orc_propagate(int(mode), d.n_pi, G, _p(ins[0]), _p(ins[1]), _p(ins[2]), K,
                           _p(ins[3]), _p(ins[4]), _p(ins[5]), _p(ins[6]), _p(ins[7]), _p(ins[8]),
                           _p(ins[9]), _p(ins[10]), _p(out["at_drv"]), _p(out["slew_drv"]),
                           _p(out["at_in"]), _p(out["slew_in"]), _p(out["arc_delay"]),
                           _p(out["argmax"]))
    _check(rc, "propagate")
    out["argmax"] = out["argmax"][:G]
    return out


def endpoints(d):
    fo = np.bincount(np.asarray(d.arc_drv), minlength=d.n_pi + d.n_gates)
    return np.nonzero(fo == 0)[0]


def slack(d, net_delay, arc_delay, at_drv, at_in, ep_rat, mode=LATE):
    """Step 6 (FP32): required times and slacks of every pin, then WNS and TNS."""
    lib = _load()
    D, A, G = d.n_pi + d.n_gates, d.arc_drv.shape[0], d.n_gates
    out = dict(rat_drv=np.zeros(D, np.float32), rat_in=np.zeros(A, np.float32),
               slack_drv=np.zeros(D, np.float32), slack_in=np.zeros(A, np.float32))
    ins = [_c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32), _c(net_delay, np.float32),
           _c(arc_delay, np.float32), _c(at_drv, np.float32), _c(at_in, np.float32),
           _c(ep_rat, np.float32)]
    rc = lib.orc_slack(int(mode), d.n_pi, G, *[_p(a) for a in ins], _p(out["rat_drv"]),
                       _p(out["rat_in"]), _p(out["slack_drv"]), _p(out["slack_in"]))
    _check(rc, "slack")
    ep = endpoints(d)
    s = out["slack_drv"][ep]
    out["wns"] = np.float32(s.min()) if s.size else np.float32(np.inf)
    out["tns"] = tns(s)
    return out


def tns(endpoint_slack) -> float:
    """Exact sum of the negative endpoint slacks, rounded once to FP64."""
    s = np.asarray(endpoint_slack, dtype=np.float32)
    neg = s[s < 0].astype(np.float64)
    return math.fsum(neg.tolist())


def run(d, lib, pi_at, pi_slew, ep_rat_late, ep_rat_early=None, modes=(LATE,)):
    """Whole path for the given modes: delay calc, then propagate and slack per mode."""
    load, nd, ni = delay_calc(d)
    res = {"load": load, "net_delay": nd, "net_imp2": ni}
    for m in modes:
        rat = ep_rat_late if m == LATE else ep_rat_early
        p = propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, pi_at, pi_slew, m)
        s = slack(d, nd, p["arc_delay"], p["at_drv"], p["at_in"], rat, m)
        p.update(s)
        res["late" if m == LATE else "early"] = p
    return res
