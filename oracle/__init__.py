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
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

LATE, EARLY = 0, 1


class OracleError(RuntimeError):
    pass


def _load(par: bool = False):
    """The serial oracle, or (par) the OpenMP build of the same source."""
    global _lib, _lib_omp
    if (_lib_omp if par else _lib) is not None:
        return _lib_omp if par else _lib
    src = os.path.join(_HERE, "sta_oracle.c")
    if any(not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(src) for p in (_LIB_PATH, _LIB_OMP_PATH)):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_OMP_PATH if par else _LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.orc_levelize.argtypes = [I, I, P, P, P, P]
    for f in ("orc_delay_calc", "orc_delay_calc_lv"):
        getattr(lib, f).argtypes = [I, P, P, P, P, I, P, P, P, P, P, P, P, P, P]
    lib.orc_bilerp.argtypes = [P, P, P, ctypes.c_float, ctypes.c_float]
    lib.orc_bilerp.restype = ctypes.c_float
    lib.orc_bilerp_many.argtypes = [P, P, P, I, P, P, P]
    for f in ("orc_propagate", "orc_propagate_lv"):
        getattr(lib, f).argtypes = [I, I, I, P, P, P, I, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    for f in ("orc_slack", "orc_slack_lv"):
        getattr(lib, f).argtypes = [I, I, I, P, P, P, P, P, P, P, P, P, P, P]
    for f in ("orc_levelize", "orc_delay_calc", "orc_propagate", "orc_slack", "orc_delay_calc_lv",
              "orc_propagate_lv", "orc_slack_lv", "orc_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [I]
    lib.orc_set_threads.restype = None
    if par:
        _lib_omp = lib
    else:
        _lib = lib
    return lib


def threads(n=None) -> int:
    """Threads of the OpenMP build: sets them when n is given; returns the count in use."""
    lib = _load(True)
    if n is not None:
        lib.orc_set_threads(int(n))
    return int(lib.orc_num_threads())


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


def delay_calc(d, moments: bool = False, par: bool = False):
    """Step 2 (FP64 per net): load per driver, Elmore delay and imp2 per sink arc (FP32 rounded).

    With ``moments`` also returns the FP64 node arrays (m1, m2, downstream cap).  With
    ``par`` the OpenMP build spreads the nets over its threads (same results)."""
    lib = _load(par)
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
    rc = (lib.orc_delay_calc_lv if par else lib.orc_delay_calc)(D, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]), A,
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


def propagate(d, lib_x, lib_y, lib_tab, load, net_delay, net_imp2, pi_at, pi_slew, mode=LATE, par=False):
    """Steps 4-5 (FP32): arrival time and slew of every pin, arc delays and the argmax arc.
    With ``par`` the OpenMP build runs level by level, each level's gates in parallel."""
    lib = _load(par)
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
    rc = (lib.orc_propagate_lv if par else lib.orc_propagate)(int(mode), d.n_pi, G, _p(ins[0]), _p(ins[1]), _p(ins[2]), K,
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


def slack(d, net_delay, arc_delay, at_drv, at_in, ep_rat, mode=LATE, par=False):
    """Step 6 (FP32): required times and slacks of every pin, then WNS and TNS.  With
    ``par`` the OpenMP build runs level by level from the top, in parallel per level."""
    lib = _load(par)
    D, A, G = d.n_pi + d.n_gates, d.arc_drv.shape[0], d.n_gates
    out = dict(rat_drv=np.zeros(D, np.float32), rat_in=np.zeros(A, np.float32),
               slack_drv=np.zeros(D, np.float32), slack_in=np.zeros(A, np.float32))
    ins = [_c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32), _c(net_delay, np.float32),
           _c(arc_delay, np.float32), _c(at_drv, np.float32), _c(at_in, np.float32),
           _c(ep_rat, np.float32)]
    rc = (lib.orc_slack_lv if par else lib.orc_slack)(int(mode), d.n_pi, G, *[_p(a) for a in ins], _p(out["rat_drv"]),
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


def run(d, lib, pi_at, pi_slew, ep_rat_late, ep_rat_early=None, modes=(LATE,), par=False):
    """Whole path for the given modes: delay calc, then propagate and slack per mode
    (``par``: the OpenMP build's level-parallel entry points)."""
    load, nd, ni = delay_calc(d, par=par)
    res = {"load": load, "net_delay": nd, "net_imp2": ni}
    for m in modes:
        rat = ep_rat_late if m == LATE else ep_rat_early
        p = propagate(d, lib.x, lib.y, lib.tab, load, nd, ni, pi_at, pi_slew, m, par=par)
        s = slack(d, nd, p["arc_delay"], p["at_drv"], p["at_in"], rat, m, par=par)
        p.update(s)
        res["late" if m == LATE else "early"] = p
    return res


# ---- RC-tree nets and the learned-surrogate reference --------------------------------

FEATURES = ("R_path", "load", "Cd_sink", "depth", "M", "n_sinks", "R_first", "C_path",
            "mean_R", "mean_C", "pin_cap", "drv_slew")


def tree_moments(T, features=False):
    """FP64 Elmore m1 and imp2 per sink, load per net, and optionally the 12 features."""
    lib = _load()
    f = lib.orc_tree_moments
    f.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 12
    f.restype = ctypes.c_int
    N, S = T.n_nets, T.n_sinks
    m1 = np.zeros(S, np.float64)
    imp2 = np.zeros(S, np.float64)
    load = np.zeros(N, np.float64)
    feat = np.zeros((S, 12), np.float64) if features else None
    arrs = [_c(T.net_node_ptr, np.int32), _c(T.node_parent, np.int32), _c(T.node_R, np.float32),
            _c(T.node_C, np.float32), _c(T.sink_ptr, np.int32), _c(T.sink_node, np.int32),
            _c(T.sink_pincap, np.float32), _c(T.drv_slew, np.float32)]
    _check(f(N, *[_p(a) for a in arrs], _p(m1), _p(imp2), _p(load), _p(feat)), "tree_moments")
    out = {"m1": m1, "imp2": imp2, "load": load}
    if features:
        out["feat"] = feat
    return out


def tree_targets(T, mom=None):
    """The surrogate's targets per sink, as the timing path defines them in FP32:
    delay = fl32(m1), slew = sqrt(S_drv^2 + fl32(imp2)) (FP32 operations)."""
    mom = mom if mom is not None else tree_moments(T)
    nd = mom["m1"].astype(np.float32)
    ni = mom["imp2"].astype(np.float32)
    net = np.repeat(np.arange(T.n_nets), np.diff(T.sink_ptr))
    s = T.drv_slew[net].astype(np.float32)
    slew = np.sqrt(s * s + ni).astype(np.float32)
    return np.stack([nd, slew], axis=1)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), via FP32, returned as FP64."""
    u = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


class MLP:
    """Reference of the 12-64-64-2 ReLU network (inputs padded to 16) in FP64.

    With ``quant`` the values the GPU feeds to its BF16 matrix products are rounded to
    bfloat16 at the same points: the input, the weights, both hidden activations, and in
    the backward pass the output error and both masked hidden gradients."""

    def __init__(self, params):
        self.p = {k: np.asarray(v, np.float64) for k, v in params.items()}

    @staticmethod
    def init(seed=0):
        rng = np.random.default_rng(seed)
        def he(o, i):
            return rng.standard_normal((o, i)) * np.sqrt(2.0 / i)
        W1 = np.zeros((64, 16))
        W1[:, :12] = he(64, 12)
        return {"W1": W1, "b1": np.zeros(64), "W2": he(64, 64), "b2": np.zeros(64),
                "W3": he(2, 64) * 0.5, "b3": np.zeros(2)}

    def forward(self, x, quant=True):
        q = bf16 if quant else (lambda a: np.asarray(a, np.float64))
        p = self.p
        xq = q(x)
        z1 = xq @ q(p["W1"]).T + p["b1"]
        h1 = q(np.maximum(z1, 0.0))
        z2 = h1 @ q(p["W2"]).T + p["b2"]
        h2 = q(np.maximum(z2, 0.0))
        y = h2 @ q(p["W3"]).T + p["b3"]
        return y, {"x": xq, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "quant": quant}

    def loss(self, x, t, quant=True):
        y, _ = self.forward(x, quant)
        return 0.5 * np.mean(np.sum((y - t) ** 2, axis=1))

    def grads(self, x, t, quant=True):
        """Gradients of loss = mean over the batch of 0.5*|y - t|^2."""
        q = bf16 if quant else (lambda a: np.asarray(a, np.float64))
        p = self.p
        y, c = self.forward(x, quant)
        B = x.shape[0]
        dy = (y - t) / B
        dyq = q(dy)
        g = {"W3": dyq.T @ c["h2"], "b3": dy.sum(0)}
        dz2 = (dyq @ q(p["W3"])) * (c["z2"] > 0)
        dz2q = q(dz2)
        g["W2"] = dz2q.T @ c["h1"]
        g["b2"] = dz2.sum(0)
        dz1 = (dz2q @ q(p["W2"])) * (c["z1"] > 0)
        dz1q = q(dz1)
        g["W1"] = dz1q.T @ c["x"]
        g["b1"] = dz1.sum(0)
        return g


def surrogate_targets(T, mom=None):
    """Normalized targets per sink, in FP64, rounded to FP32.

    With L = R_path*Cd(sink)*1e-3 and U = R_path*load*1e-3 (the two Elmore bounds: every
    edge on the path sees at least the sink's downstream cap and at most the whole net):
      alpha = (m1 - L) / (U - L)   (0 where U == L),     gamma = sqrt(imp2) / U  (0 where U == 0)."""
    mom = mom if mom is not None else tree_moments(T, features=True)
    f = mom["feat"]
    L = (f[:, 0] * f[:, 2]) * 1e-3
    U = (f[:, 0] * f[:, 1]) * 1e-3
    span = U - L
    alpha = np.where(span > 0, (mom["m1"] - L) / np.where(span > 0, span, 1.0), 0.0)
    gamma = np.where(U > 0, np.sqrt(mom["imp2"]) / np.where(U > 0, U, 1.0), 0.0)
    return np.stack([alpha, gamma], axis=1).astype(np.float32)


def decode(feat32, y):
    """Predicted (delay, slew) per sink in FP32 from the features and the network's
    (alpha, gamma):  delay = L + alpha*(U-L),  slew = sqrt(S^2 + (gamma*U)^2)."""
    f = np.asarray(feat32, np.float32)
    y = np.asarray(y, np.float32)
    k = np.float32(1e-3)
    L = (f[:, 0] * f[:, 2]) * k
    U = (f[:, 0] * f[:, 1]) * k
    d = L + y[:, 0] * (U - L)
    g = y[:, 1] * U
    s = np.sqrt(f[:, 11] * f[:, 11] + g * g)
    return d.astype(np.float32), s.astype(np.float32)


def norm_stats(feat):
    """Per-feature mean and 1/std of log(1 + feature) over the given rows (FP64, population
    std; 1/std = 1 where the std is 0)."""
    lf = np.log(np.asarray(feat, np.float64) + 1.0)
    mu = lf.mean(axis=0)
    sd = lf.std(axis=0)
    return mu, np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)


def mlp_input(feat, mu, rstd):
    """Network input: (log(1 + f) - mu) * rstd for the 12 features, padded with zeros to 16."""
    x = np.zeros((feat.shape[0], 16))
    x[:, :12] = (np.log(np.asarray(feat, np.float64) + 1.0) - mu) * rstd
    return x


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


N_BINS = 64
N_BUCKETS = 128


def error_bin(feat):
    """Calibration bin of a sink: 8 depth classes (1..7, >=8) x 8 net-size classes (M in
    steps of 8 nodes, M<=64; larger nets share the last class)."""
    depth = np.clip(np.asarray(feat)[:, 3].astype(np.int64), 1, 8) - 1
    msz = np.clip((np.asarray(feat)[:, 4].astype(np.int64) - 1) // 8, 0, 7)
    return depth * 8 + msz


def error_bucket(e):
    """Histogram bucket of a normalized FP32 error e >= 0, on quarter-octave edges that are
    exact in binary: with key = (biased exponent)*4 + (top two mantissa bits) of e, bucket
    k = clamp(508 - key, 0, 127).  Bucket 0 takes every e >= 1; bucket k > 0 holds the
    e in [edge(508 - k), edge(509 - k)), edge(key) being the FP32 value with bits key << 21."""
    e = np.ascontiguousarray(np.abs(np.asarray(e, np.float32)))
    key = (e.view(np.uint32) >> 21).astype(np.int64)
    return np.clip(508 - key, 0, N_BUCKETS - 1)


def bucket_bound(k):
    """Upper edge (exclusive) of bucket k > 0 as FP32; +inf for bucket 0."""
    if k <= 0:
        return np.inf
    return float(np.array([(509 - k) << 21], np.uint32).view(np.float32)[0])


def calibrate(feat, err, quantile=0.999, min_count=256):
    """Per (bin, output) upper bound of the `quantile` of the normalized error, read from a
    histogram of error buckets: the upper edge of the bucket where the count of errors in
    it and the buckets above first exceeds floor((1-quantile)*n).  Bins with fewer than
    `min_count` samples, or whose quantile falls in bucket 0, get +inf (always fall back)."""
    b = error_bin(feat)
    q = np.full((N_BINS, 2), np.inf)
    for o in range(2):
        hist = np.zeros((N_BINS, N_BUCKETS), np.int64)
        np.add.at(hist, (b, error_bucket(err[:, o])), 1)
        for i in range(N_BINS):
            n = hist[i].sum()
            if n < min_count:
                continue
            allow = int(np.floor((1.0 - quantile) * n))
            c = 0
            for k in range(N_BUCKETS):
                c += hist[i, k]
                if c > allow:
                    q[i, o] = bucket_bound(k)
                    break
    return q


# ---- adjoint of TNS and critical paths -----------------------------------------------

def tns_adjoint(d, res_mode, mode=LATE):
    """dTNS/dAT per driver and dTNS/d(arc delay) per cell arc (FP64 counts) by the chain
    rule through the saved argmax arcs, from a forward/slack result of this oracle."""
    lib = _load()
    f = lib.orc_tns_adjoint
    f.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 6
    f.restype = ctypes.c_int
    D, A = d.n_pi + d.n_gates, d.arc_drv.shape[0]
    g_at = np.zeros(D, np.float64)
    g_arc = np.zeros(A, np.float64)
    arrs = [_c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32), _c(res_mode["argmax"], np.int32),
            _c(res_mode["slack_drv"], np.float32)]
    _check(f(int(mode), d.n_pi, d.n_gates, *[_p(a) for a in arrs], _p(g_at), _p(g_arc)), "tns_adjoint")
    return g_at, g_arc


def _seg(axis, v):
    """Largest i in 0..5 with axis[i] <= v (FP32 comparisons), per element."""
    ax = np.asarray(axis, np.float32)
    v = np.asarray(v, np.float32)
    return np.sum(ax[None, 1:6] <= v[:, None], axis=1)


def bilerp64(x, y, T, s, l):
    """The bilinear lookup of one table per element in FP64 arithmetic (same segments as
    the FP32 lookup, no clamping).  T: [n][49]."""
    x64, y64 = np.asarray(x, np.float64), np.asarray(y, np.float64)
    i, j = _seg(x, s), _seg(y, l)
    tx = (np.asarray(s, np.float64) - x64[i]) / (x64[i + 1] - x64[i])
    ty = (np.asarray(l, np.float64) - y64[j]) / (y64[j + 1] - y64[j])
    T = np.asarray(T, np.float64)
    r = np.arange(T.shape[0])
    p = T[r, i * 7 + j] + tx * (T[r, (i + 1) * 7 + j] - T[r, i * 7 + j])
    q = T[r, i * 7 + j + 1] + tx * (T[r, (i + 1) * 7 + j + 1] - T[r, i * 7 + j + 1])
    return p + ty * (q - p), (q - p) / (y64[j + 1] - y64[j])


def load_slope(d, libr, res_mode, load, table_set=0):
    """d(delay of the argmax arc)/d(load) of every gate (FP64 arithmetic), slew held."""
    G = d.n_gates
    a = np.asarray(d.gate_arc_ptr[:-1]) + np.asarray(res_mode["argmax"][:G])
    tb = np.asarray(d.arc_tbl)[a]
    T = _tables(libr, table_set)
    _, slope = bilerp64(libr.x, libr.y, T[tb, 0], res_mode["slew_in"][a], np.asarray(load)[d.n_pi + np.arange(G)])
    return slope


def _tables(libr, table_set=0):
    """[n_tables][2][49] FP32 tables of one set ([sets][K][2][7][7] or [K][2][7][7])."""
    t = np.asarray(libr.tab, np.float32)
    if t.ndim == 5:
        t = t[table_set]
    return t.reshape(-1, 2, 49)


def tns_delta(d, arc_delay, net_delay, pi_at, ep_rat_drv, mode, pert_gate, pert_off, pert_delay):
    """FP64 TNS of the design and its change under each delay perturbation of one gate."""
    lib = _load()
    f = lib.orc_tns_delta
    f.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 6 + [ctypes.c_int] + [ctypes.c_void_p] * 5
    f.restype = ctypes.c_int
    n = len(pert_gate)
    base = np.zeros(1, np.float64)
    delta = np.zeros(max(n, 1), np.float64)
    arrs = [_c(d.gate_arc_ptr, np.int32), _c(d.arc_drv, np.int32), _c(arc_delay, np.float64),
            _c(net_delay, np.float64), _c(pi_at, np.float64), _c(ep_rat_drv, np.float64)]
    pg, po, pd = _c(pert_gate, np.int32), _c(pert_off, np.int32), _c(pert_delay, np.float64)
    _check(f(int(mode), d.n_pi, d.n_gates, *[_p(a) for a in arrs], n, _p(pg), _p(po), _p(pd), _p(base),
             _p(delta)), "tns_delta")
    return float(base[0]), delta[:n]


def _gate_of_arc(d):
    return np.repeat(np.arange(d.n_gates), np.diff(d.gate_arc_ptr))


def fd_arc_delay(d, arc_delay, net_delay, pi_at, ep_rat_drv, mode, arcs, h=1e-3):
    """Central differences of TNS (FP64) in the delays of the given cell arcs.  Returns
    (fd, clean): clean marks samples where the two one-sided differences agree (no tie of
    a maximum and no endpoint slack crossing zero within +-h)."""
    gate = _gate_of_arc(d)
    ptr = np.asarray(d.gate_arc_ptr)
    pg, po, pd = [], [0], []
    for a in arcs:
        g = gate[a]
        base = np.asarray(arc_delay[ptr[g]:ptr[g + 1]], np.float64)
        for sgn in (1.0, -1.0):
            x = base.copy()
            x[a - ptr[g]] += sgn * h
            pg.append(g)
            pd.extend(x.tolist())
            po.append(len(pd))
    _, dl = tns_delta(d, arc_delay, net_delay, pi_at, ep_rat_drv, mode, pg, po, pd)
    dp, dm = dl[0::2], dl[1::2]
    fd = (dp - dm) / (2 * h)
    clean = np.abs(dp + dm) <= 1e-9 * (1.0 + np.abs(dp) + np.abs(dm))
    return fd, clean


def fd_load(d, libr, res_mode, load, net_delay, pi_at, ep_rat_drv, mode, gates, h=1e-3, table_set=0):
    """Central differences of TNS (FP64) in the load of the given gates' output nets: the
    delays of all the gate's arcs are re-evaluated by the FP64 bilinear lookup at load +-h
    (and at the load itself, the reference point), input slews held."""
    T = _tables(libr, table_set)
    ptr = np.asarray(d.gate_arc_ptr)
    arc_delay = np.asarray(res_mode["arc_delay"], np.float64).copy()
    pg, po, pd = [], [0], []
    for g in gates:
        a = np.arange(ptr[g], ptr[g + 1])
        L0 = float(load[d.n_pi + g])
        for dl in (h, -h, 0.0):
            val, _ = bilerp64(libr.x, libr.y, T[np.asarray(d.arc_tbl)[a], 0], res_mode["slew_in"][a],
                              np.full(a.size, L0 + dl))
            pg.append(g)
            pd.extend(val.tolist())
            po.append(len(pd))
    _, dl_ = tns_delta(d, arc_delay, net_delay, pi_at, ep_rat_drv, mode, pg, po, pd)
    dp, dm, d0 = dl_[0::3], dl_[1::3], dl_[2::3]
    fd = (dp - dm) / (2 * h)
    clean = np.abs(dp + dm - 2 * d0) <= 1e-9 * (1.0 + np.abs(dp) + np.abs(dm))
    return fd, clean


def ep_rat_by_driver(d, ep_rat):
    """Endpoint required times (by endpoint rank) spread into a per-driver FP64 array."""
    r = np.zeros(d.n_pi + d.n_gates, np.float64)
    r[endpoints(d)] = np.asarray(ep_rat, np.float64)
    return r


def critical_paths(d, res_mode, k):
    """The k worst endpoints (slack, then rank) and their argmax paths back to a primary
    input: lists of drivers (endpoint first) and of the cell arcs leading into them."""
    ep = endpoints(d)
    s = np.asarray(res_mode["slack_drv"], np.float32)[ep]
    order = np.lexsort((np.arange(ep.size), s))[:k]
    paths = []
    for r in order:
        u = int(ep[r])
        drv, arcs = [u], []
        while u >= d.n_pi:
            g = u - d.n_pi
            a = int(d.gate_arc_ptr[g] + res_mode["argmax"][g])
            arcs.append(a)
            u = int(d.arc_drv[a])
            drv.append(u)
        paths.append((int(r), float(s[r]), drv, arcs))
    return paths
