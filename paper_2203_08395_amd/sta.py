"""Python binding of libsta.so: argument marshalling only.

Every step of the timing path runs in the library's HIP kernels; this module allocates
the device buffers with torch (device memory and the current stream are all torch
provides), fills the C structs and raises ``StaError`` on a non-OK status.  There is no
CPU fallback: without the built library (``python -m paper_2203_08395_amd.build``) every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsta.so")

STA_LATE, STA_EARLY = 0, 1
STA_DC_FP64, STA_DC_FP32 = 0, 1
MAX_VIEWS = 8
_STATUS = {0: "OK", -1: "E_ARG", -2: "E_RANGE", -3: "E_CYCLE", -4: "E_NONFINITE", -5: "E_ALLOC", -6: "E_HIP"}

_P = ctypes.c_void_p


class StaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = _STATUS.get(status, str(status))


class DesignDesc(ctypes.Structure):
    _fields_ = [("n_pi", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("n_tables", ctypes.c_int32),
                ("gate_arc_ptr", _P), ("arc_drv", _P), ("arc_tbl", _P), ("arc_tap", _P), ("arc_pincap", _P),
                ("net_node_ptr", _P), ("node_parent", _P), ("node_R", _P), ("node_C", _P)]


class Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_pi", "n_gates", "n_drivers", "n_arcs", "n_nodes", "n_pins", "n_levels", "n_endpoints",
                 "max_fanin", "max_fanout", "max_net_nodes", "n_fwd_tiles", "n_bwd_tiles")] + \
               [("graph_bytes", ctypes.c_size_t), ("scratch_bytes", ctypes.c_size_t)]


class SpanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("fwd_spans", "fwd_spans_fused", "fwd_span_launches", "fwd_level_launches", "fwd_span_gates",
                 "fwd_span_arcs", "fwd_span_arcs_computed", "fwd_span_tiles", "bwd_spans", "bwd_spans_fused",
                 "bwd_span_launches", "bwd_level_launches", "bwd_span_drivers", "bwd_span_arcs",
                 "bwd_span_slots_computed", "bwd_span_tiles")]


class LibraryC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_float * 7), ("y", ctypes.c_float * 7), ("tables", _P),
                ("n_sets", ctypes.c_int32), ("n_tables", ctypes.c_int32)]


class ViewsC(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("mode", ctypes.c_int32 * MAX_VIEWS),
                ("table_set", ctypes.c_int32 * MAX_VIEWS)]


class NetOut(ctypes.Structure):
    _fields_ = [("load", _P), ("net_delay", _P), ("net_imp2", _P), ("arc_load", _P)]


class TimingOut(ctypes.Structure):
    _fields_ = [("drv_ts", _P), ("arc_ts", _P), ("arc_delay", _P), ("argmax", _P)]


class SlackOut(ctypes.Structure):
    _fields_ = [("drv_rat", _P), ("arc_rat", _P), ("drv_slack", _P), ("arc_slack", _P), ("tns", _P), ("wns", _P)]


_lib = None

EXPORTS = ("sta_last_error", "sta_build_graph", "sta_build_graph_spans", "sta_graph_sizes", "sta_graph_perm", "sta_graph_upload",
           "sta_graph_free", "sta_delay_calc", "sta_propagate", "sta_slack", "sta_slack_noalloc", "sta_set_schedule", "sta_set_level_fusion",
           "sta_graph_spans", "sta_graph_span_list", "sta_profile_begin", "sta_profile_end")


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


def load_library():
    """Load libsta.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_08395_amd.build`")
    # torch first, so that libsta binds to the HIP runtime torch already uses (one runtime
    # per process: device pointers and streams from torch are then valid in libsta)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    lib.sta_last_error.restype = ctypes.c_char_p
    lib.sta_last_error.argtypes = []
    lib.sta_build_graph.argtypes = [ctypes.POINTER(DesignDesc), ctypes.POINTER(_P)]
    lib.sta_build_graph_spans.argtypes = [ctypes.POINTER(DesignDesc), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(_P)]
    lib.sta_graph_sizes.argtypes = [_P, ctypes.POINTER(Sizes)]
    lib.sta_graph_perm.argtypes = [_P, _P, _P, _P, _P, _P]
    lib.sta_graph_upload.argtypes = [_P, _P, ctypes.c_size_t, _P]
    lib.sta_graph_free.argtypes = [_P]
    lib.sta_graph_free.restype = None
    lib.sta_delay_calc.argtypes = [_P, ctypes.c_int, ctypes.POINTER(NetOut), _P]
    lib.sta_propagate.argtypes = [_P, ctypes.POINTER(LibraryC), ctypes.POINTER(ViewsC), _P,
                                  ctypes.POINTER(NetOut), ctypes.POINTER(TimingOut), _P]
    lib.sta_slack.argtypes = [_P, ctypes.POINTER(ViewsC), ctypes.POINTER(NetOut), ctypes.POINTER(TimingOut), _P,
                              ctypes.POINTER(SlackOut), _P, ctypes.c_size_t, _P]
    lib.sta_slack_noalloc.argtypes = [_P, ctypes.POINTER(ViewsC), ctypes.POINTER(NetOut), ctypes.POINTER(TimingOut),
                                      _P, ctypes.POINTER(SlackOut), _P]
    lib.sta_set_schedule.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
    lib.sta_set_level_fusion.argtypes = [_P, ctypes.c_int32]
    lib.sta_graph_spans.argtypes = [_P, ctypes.POINTER(SpanInfo)]
    lib.sta_graph_span_list.argtypes = [_P, _P, _P]
    lib.sta_profile_begin.argtypes = []
    lib.sta_profile_end.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    for f in ("sta_build_graph", "sta_build_graph_spans", "sta_graph_sizes", "sta_graph_perm", "sta_graph_upload",
              "sta_delay_calc",
              "sta_propagate", "sta_slack", "sta_slack_noalloc", "sta_set_schedule", "sta_set_level_fusion",
              "sta_graph_spans",
              "sta_graph_span_list", "sta_profile_begin", "sta_profile_end"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st, what):
    if st != 0:
        msg = load_library().sta_last_error().decode(errors="replace")
        raise StaError(st, msg or what)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(t):
    return None if t is None else _P(t.data_ptr())


def _stream(torch, device):
    return _P(torch.cuda.current_stream(device).cuda_stream)


class Graph:
    """A levelized design (host side built by sta_build_graph); ``upload`` places it on a GPU."""

    def __init__(self, design, n_tables=None, span_levels=None):
        """span_levels: (forward, backward) longest fused span in levels, each 1..8
        (sta_build_graph_spans); None: the library's (8, 8)."""
        lib = load_library()
        self._keep = [_np(design.gate_arc_ptr, np.int32), _np(design.arc_drv, np.int32),
                      _np(design.arc_tbl, np.int32), _np(design.arc_tap, np.int32),
                      _np(design.arc_pincap, np.float32), _np(design.net_node_ptr, np.int32),
                      _np(design.node_parent, np.int32), _np(design.node_R, np.float32),
                      _np(design.node_C, np.float32)]
        if n_tables is None:
            n_tables = int(self._keep[2].max()) + 1 if self._keep[2].size else 1
        d = DesignDesc(int(design.n_pi), int(design.n_gates), n_tables,
                       *[_P(a.ctypes.data) for a in self._keep])
        h = _P()
        if span_levels is None:
            _check(lib.sta_build_graph(ctypes.byref(d), ctypes.byref(h)), "sta_build_graph")
        else:
            _check(lib.sta_build_graph_spans(ctypes.byref(d), int(span_levels[0]), int(span_levels[1]),
                                             ctypes.byref(h)), "sta_build_graph_spans")
        self.span_levels = tuple(span_levels) if span_levels is not None else (8, 8)
        self._h = h
        self._keep = None
        s = Sizes()
        _check(lib.sta_graph_sizes(h, ctypes.byref(s)), "sta_graph_sizes")
        self.sizes = {f: int(getattr(s, f)) for f, _ in Sizes._fields_}
        D, A, G, E = (self.sizes[k] for k in ("n_drivers", "n_arcs", "n_gates", "n_endpoints"))
        self.drv_input = np.zeros(D, np.int32)
        self.arc_input = np.zeros(A, np.int32)
        self.gate_input = np.zeros(G, np.int32)
        self.level = np.zeros(D, np.int32)
        self.ep_driver = np.zeros(E, np.int32)
        _check(lib.sta_graph_perm(h, *[_P(a.ctypes.data) if a.size else None for a in
                                       (self.drv_input, self.arc_input, self.gate_input, self.level,
                                        self.ep_driver)]), "sta_graph_perm")
        self.dev = None
        self.device = None

    def upload(self, device="cuda"):
        import torch
        lib = load_library()
        nb = max(self.sizes["graph_bytes"], 256)
        self.dev = torch.empty(nb, dtype=torch.uint8, device=device)
        self.device = self.dev.device
        _check(lib.sta_graph_upload(self._h, _P(self.dev.data_ptr()), nb, _stream(torch, self.device)),
               "sta_graph_upload")
        return self

    def set_schedule(self, view_max_arcs_per_level, use_graphs=True):
        """0: one launch per level; -1: default choice; n: view schedule up to n arcs per
        level.  use_graphs: replay the level schedule's launches from a captured hipGraph."""
        _check(load_library().sta_set_schedule(self._h, int(view_max_arcs_per_level), int(bool(use_graphs))),
               "sta_set_schedule")
        return self

    def set_level_fusion(self, enable):
        """Fused spans: up to eight gate levels per forward launch and eight driver levels
        per backward launch, any view count (default on)."""
        _check(load_library().sta_set_level_fusion(self._h, int(bool(enable))), "sta_set_level_fusion")
        return self

    @property
    def spans(self):
        """The fusion plan: fused spans, launches and the work they cover."""
        si = SpanInfo()
        _check(load_library().sta_graph_spans(self._h, ctypes.byref(si)), "sta_graph_spans")
        return {f: int(getattr(si, f)) for f, _ in SpanInfo._fields_}

    def span_list(self):
        """(forward, backward) spans as int32 arrays of rows (first or top level, last or
        bottom level, fused), in launch order."""
        sp = self.spans
        fwd = np.zeros((sp["fwd_spans"], 3), np.int32)
        bwd = np.zeros((sp["bwd_spans"], 3), np.int32)
        _check(load_library().sta_graph_span_list(self._h, fwd.ctypes.data if fwd.size else None,
                                                  bwd.ctypes.data if bwd.size else None), "sta_graph_span_list")
        return fwd, bwd

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sta_graph_free(h)
            self._h = None

    # maps from internal (level) order to input order
    def drv_to_input(self, x):
        out = np.empty_like(x)
        out[self.drv_input] = x
        return out

    def arc_to_input(self, x):
        out = np.empty_like(x)
        out[self.arc_input] = x
        return out

    def gate_to_input(self, x):
        out = np.empty_like(x)
        out[self.gate_input] = x
        return out


def make_views(modes, table_sets=None):
    v = ViewsC()
    v.n_views = len(modes)
    for i, m in enumerate(modes):
        v.mode[i] = int(m)
        v.table_set[i] = int(table_sets[i]) if table_sets is not None else 0
    return v


def make_library(x, y, tables):
    """tables: device tensor [n_sets, K, 2, 7, 7] (or [K, 2, 7, 7]) float32."""
    L = LibraryC()
    for i in range(7):
        L.x[i] = float(np.float32(x[i]))
        L.y[i] = float(np.float32(y[i]))
    if tables.dim() == 4:
        tables = tables.unsqueeze(0)
    L.tables = _P(tables.data_ptr())
    L.n_sets = int(tables.shape[0])
    L.n_tables = int(tables.shape[1])
    L._tensor = tables
    return L


def delay_calc(g: Graph, precision=STA_DC_FP64, out=None):
    import torch
    D, A = g.sizes["n_drivers"], g.sizes["n_arcs"]
    if out is None:
        out = alloc_net(g)
    no = _netout(out)
    _check(load_library().sta_delay_calc(g.handle, int(precision), ctypes.byref(no), _stream(torch, g.device)),
           "sta_delay_calc")
    return out


def _netout(nd):
    return NetOut(_ptr(nd["load"]), _ptr(nd["net_delay"]), _ptr(nd["net_imp2"]), _ptr(nd["arc_load"]))


def alloc_net(g: Graph):
    import torch
    D, A = g.sizes["n_drivers"], g.sizes["n_arcs"]
    return {"load": torch.empty(max(D, 1), dtype=torch.float32, device=g.device),
            "net_delay": torch.empty(max(A, 1), dtype=torch.float32, device=g.device),
            "net_imp2": torch.empty(max(A, 1), dtype=torch.float32, device=g.device),
            "arc_load": torch.empty(max(A, 1), dtype=torch.float32, device=g.device)}


def alloc_timing(g: Graph, n_views):
    import torch
    D, A, G = g.sizes["n_drivers"], g.sizes["n_arcs"], g.sizes["n_gates"]
    dev = g.device
    return {"drv_ts": torch.empty((max(D, 1), n_views, 2), dtype=torch.float32, device=dev),
            "arc_ts": torch.empty((max(A, 1), n_views, 2), dtype=torch.float32, device=dev),
            "arc_delay": torch.empty((max(A, 1), n_views), dtype=torch.float32, device=dev),
            "argmax": torch.empty((max(G, 1), n_views), dtype=torch.uint8, device=dev)}


def propagate(g: Graph, lib: LibraryC, views: ViewsC, pi_ts, nd, out=None):
    """pi_ts: device [n_pi, V, 2] float32 (arrival, slew) of the primary inputs."""
    import torch
    if out is None:
        out = alloc_timing(g, views.n_views)
    to = TimingOut(_ptr(out["drv_ts"]), _ptr(out["arc_ts"]), _ptr(out["arc_delay"]), _ptr(out["argmax"]))
    no = _netout(nd)
    _check(load_library().sta_propagate(g.handle, ctypes.byref(lib), ctypes.byref(views), _ptr(pi_ts),
                                        ctypes.byref(no), ctypes.byref(to), _stream(torch, g.device)),
           "sta_propagate")
    return out


def alloc_slack(g: Graph, n_views):
    import torch
    D, A = g.sizes["n_drivers"], g.sizes["n_arcs"]
    dev = g.device
    return {"drv_rat": torch.empty((max(D, 1), n_views), dtype=torch.float32, device=dev),
            "arc_rat": torch.empty((max(A, 1), n_views), dtype=torch.float32, device=dev),
            "drv_slack": torch.empty((max(D, 1), n_views), dtype=torch.float32, device=dev),
            "arc_slack": torch.empty((max(A, 1), n_views), dtype=torch.float32, device=dev),
            "tns": torch.empty(n_views, dtype=torch.float64, device=dev),
            "wns": torch.empty(n_views, dtype=torch.float32, device=dev),
            "scratch": torch.empty(g.sizes["scratch_bytes"], dtype=torch.uint8, device=dev)}


def slack(g: Graph, views: ViewsC, nd, timing, ep_rat, out=None):
    """ep_rat: device [E, V] float32 required time of each endpoint (rank order)."""
    import torch
    if out is None:
        out = alloc_slack(g, views.n_views)
    to = TimingOut(_ptr(timing["drv_ts"]), _ptr(timing["arc_ts"]), _ptr(timing["arc_delay"]),
                   _ptr(timing["argmax"]))
    so = SlackOut(_ptr(out["drv_rat"]), _ptr(out["arc_rat"]), _ptr(out["drv_slack"]), _ptr(out["arc_slack"]),
                  _ptr(out["tns"]), _ptr(out["wns"]))
    no = _netout(nd)
    _check(load_library().sta_slack(g.handle, ctypes.byref(views), ctypes.byref(no), ctypes.byref(to),
                                    _ptr(ep_rat), ctypes.byref(so), _ptr(out["scratch"]),
                                    out["scratch"].numel(), _stream(torch, g.device)), "sta_slack")
    return out


def slack_noalloc(g: Graph, views: ViewsC, nd, timing, ep_rat, out):
    """sta_slack_noalloc: sta_slack with the library's static device scratch (no scratch
    argument; the caller's outputs ``out`` must exist: this call allocates nothing)."""
    import torch
    to = TimingOut(_ptr(timing["drv_ts"]), _ptr(timing["arc_ts"]), _ptr(timing["arc_delay"]),
                   _ptr(timing["argmax"]))
    so = SlackOut(_ptr(out["drv_rat"]), _ptr(out["arc_rat"]), _ptr(out["drv_slack"]), _ptr(out["arc_slack"]),
                  _ptr(out["tns"]), _ptr(out["wns"]))
    no = _netout(nd)
    _check(load_library().sta_slack_noalloc(g.handle, ctypes.byref(views), ctypes.byref(no), ctypes.byref(to),
                                            _ptr(ep_rat), ctypes.byref(so), _stream(torch, g.device)),
           "sta_slack_noalloc")
    return out


def profile_begin():
    _check(load_library().sta_profile_begin(), "sta_profile_begin")


def profile_end():
    """{kernel name: (launches, total ms)} of the launches since profile_begin (HIP events)."""
    cap = 32
    arr = (KernelStat * cap)()
    n = ctypes.c_int32(0)
    _check(load_library().sta_profile_end(arr, cap, ctypes.byref(n)), "sta_profile_end")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, cap))}


# ---- analyses: adjoint of TNS, critical paths (include/sta_analysis.h) -----------------

class AdjointOut(ctypes.Structure):
    _fields_ = [("g_drv_at", _P), ("g_arc_delay", _P), ("g_net_delay", _P), ("g_load", _P)]


class PathsOut(ctypes.Structure):
    _fields_ = [("ep_rank", _P), ("slack", _P), ("len", _P), ("drv", _P), ("arc", _P)]


MAX_PATHS = 64
ANALYSIS_EXPORTS = ("sta_tns_adjoint", "sta_arc_load", "sta_paths_scratch_bytes", "sta_critical_paths")
_ana_bound = False


def _ana():
    global _ana_bound
    lib = load_library()
    if not _ana_bound:
        lib.sta_tns_adjoint.argtypes = [_P, ctypes.POINTER(LibraryC), ctypes.POINTER(ViewsC), ctypes.POINTER(NetOut),
                                        ctypes.POINTER(TimingOut), ctypes.POINTER(SlackOut),
                                        ctypes.POINTER(AdjointOut), _P]
        lib.sta_arc_load.argtypes = [_P, ctypes.POINTER(NetOut), _P]
        lib.sta_paths_scratch_bytes.argtypes = []
        lib.sta_paths_scratch_bytes.restype = ctypes.c_size_t
        lib.sta_critical_paths.argtypes = [_P, ctypes.POINTER(ViewsC), ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(TimingOut), ctypes.POINTER(SlackOut),
                                           ctypes.POINTER(PathsOut), _P, ctypes.c_size_t, _P]
        for f in ("sta_tns_adjoint", "sta_arc_load", "sta_critical_paths"):
            getattr(lib, f).restype = ctypes.c_int
        _ana_bound = True
    return lib


def _timingout(t):
    return TimingOut(_ptr(t["drv_ts"]), _ptr(t["arc_ts"]), _ptr(t["arc_delay"]), _ptr(t["argmax"]))


def _slackout(o):
    return SlackOut(_ptr(o["drv_rat"]), _ptr(o["arc_rat"]), _ptr(o["drv_slack"]), _ptr(o["arc_slack"]),
                    _ptr(o["tns"]), _ptr(o["wns"]))


def alloc_adjoint(g: Graph, n_views, arcs=True, load=True):
    import torch
    D, A = g.sizes["n_drivers"], g.sizes["n_arcs"]
    dev = g.device
    out = {"g_drv_at": torch.empty((max(D, 1), n_views), dtype=torch.float32, device=dev)}
    if arcs:
        out["g_arc_delay"] = torch.empty((max(A, 1), n_views), dtype=torch.float32, device=dev)
        out["g_net_delay"] = torch.empty((max(A, 1), n_views), dtype=torch.float32, device=dev)
    if load:
        out["g_load"] = torch.empty((max(D, 1), n_views), dtype=torch.float32, device=dev)
    return out


def tns_adjoint(g: Graph, lib: LibraryC, views: ViewsC, nd, timing, slack_out, out=None):
    """Gradients of every view's TNS (see sta_tns_adjoint); device tensors, internal order."""
    import torch
    if out is None:
        out = alloc_adjoint(g, views.n_views)
    ao = AdjointOut(_ptr(out.get("g_drv_at")), _ptr(out.get("g_arc_delay")), _ptr(out.get("g_net_delay")),
                    _ptr(out.get("g_load")))
    no, to, so = _netout(nd), _timingout(timing), _slackout(slack_out)
    _check(_ana().sta_tns_adjoint(g.handle, ctypes.byref(lib) if lib is not None else None, ctypes.byref(views),
                                  ctypes.byref(no), ctypes.byref(to), ctypes.byref(so), ctypes.byref(ao),
                                  _stream(torch, g.device)), "sta_tns_adjoint")
    return out


def arc_load(g: Graph, nd):
    import torch
    no = _netout(nd)
    _check(_ana().sta_arc_load(g.handle, ctypes.byref(no), _stream(torch, g.device)), "sta_arc_load")


def critical_paths(g: Graph, views: ViewsC, view, k, timing, slack_out):
    """The k worst endpoints of one view and their argmax paths (device tensors)."""
    import torch
    L = g.sizes["n_levels"]
    dev = g.device
    out = {"ep_rank": torch.empty(k, dtype=torch.int32, device=dev),
           "slack": torch.empty(k, dtype=torch.float32, device=dev),
           "len": torch.empty(k, dtype=torch.int32, device=dev),
           "drv": torch.empty((k, L + 1), dtype=torch.int32, device=dev),
           "arc": torch.empty((k, max(L, 1)), dtype=torch.int32, device=dev)}
    lib = _ana()
    nb = lib.sta_paths_scratch_bytes()
    scratch = torch.empty(nb, dtype=torch.uint8, device=dev)
    po = PathsOut(_ptr(out["ep_rank"]), _ptr(out["slack"]), _ptr(out["len"]), _ptr(out["drv"]), _ptr(out["arc"]))
    _check(lib.sta_critical_paths(g.handle, ctypes.byref(views), int(view), int(k), ctypes.byref(_timingout(timing)),
                                  ctypes.byref(_slackout(slack_out)), ctypes.byref(po), _ptr(scratch), nb,
                                  _stream(torch, dev)), "sta_critical_paths")
    return out


# ---- batches of designs (include/sta_batch.h) --------------------------------------------

BATCH_EXPORTS = ("sta_batch_workspace_bytes", "sta_batch_create", "sta_batch_delay_calc", "sta_batch_propagate",
                 "sta_batch_slack", "sta_batch_set_tiling", "sta_batch_info", "sta_batch_free")
BATCH_PERSISTENT, BATCH_LEVELS, BATCH_SPANS = 0, 1, 2


class BatchDesignC(ctypes.Structure):
    _fields_ = [("g", _P), ("pi_ts", _P), ("nd", ctypes.POINTER(NetOut)), ("out", ctypes.POINTER(TimingOut)),
                ("schedule", ctypes.c_int32), ("ep_rat", _P), ("sl", ctypes.POINTER(SlackOut))]


class BatchPlanC(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("span_designs", "persistent_designs", "level_designs",
                                              "persistent_units", "fwd_steps", "fwd_span_tiles", "bwd_steps",
                                              "bwd_span_tiles", "slack_designs", "dc_launches")]


_batch_bound = False


def _batch_lib():
    global _batch_bound
    lib = load_library()
    if not _batch_bound:
        lib.sta_batch_workspace_bytes.argtypes = [ctypes.POINTER(BatchDesignC), ctypes.c_int32, ctypes.c_int32]
        lib.sta_batch_workspace_bytes.restype = ctypes.c_size_t
        lib.sta_batch_create.argtypes = [ctypes.POINTER(BatchDesignC), ctypes.c_int32, ctypes.POINTER(LibraryC),
                                         ctypes.POINTER(ViewsC), _P, ctypes.c_size_t, ctypes.POINTER(_P)]
        lib.sta_batch_delay_calc.argtypes = [_P, ctypes.c_int, ctypes.c_int32, _P]
        lib.sta_batch_propagate.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, _P]
        lib.sta_batch_slack.argtypes = [_P, ctypes.c_int32, _P]
        lib.sta_batch_set_tiling.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
        lib.sta_batch_info.argtypes = [_P, ctypes.POINTER(BatchPlanC)]
        lib.sta_batch_free.argtypes = [_P]
        lib.sta_batch_free.restype = None
        for f in ("sta_batch_create", "sta_batch_delay_calc", "sta_batch_propagate", "sta_batch_slack",
                  "sta_batch_set_tiling", "sta_batch_info"):
            getattr(lib, f).restype = ctypes.c_int
        _batch_bound = True
    return lib


class Batch:
    """Several uploaded graphs sharing one library and view set, run together.

    entries: list of (graph, pi_ts tensor, net dict, timing dict, schedule) or
    (graph, pi_ts, net dict, timing dict, schedule, ep_rat tensor, slack dict); the slack
    dict is the output of ``alloc_slack`` (its scratch is not used)."""

    def __init__(self, entries, lib: LibraryC, views: ViewsC):
        import torch
        blib = _batch_lib()
        self._keep = []
        arr = (BatchDesignC * max(len(entries), 1))()
        for i, e in enumerate(entries):
            g, pi, nd, tm, sched = e[:5]
            ep_rat, sl = (e[5], e[6]) if len(e) > 5 else (None, None)
            no, to = _netout(nd), _timingout(tm)
            so = _slackout(sl) if sl is not None else None
            self._keep += [g, pi, nd, tm, no, to, ep_rat, sl, so]
            arr[i] = BatchDesignC(g.handle, _ptr(pi), ctypes.pointer(no), ctypes.pointer(to), int(sched),
                                  _ptr(ep_rat), ctypes.pointer(so) if so is not None else None)
        self._arr = arr
        self.device = entries[0][0].device if entries else torch.device("cuda")
        nb = blib.sta_batch_workspace_bytes(arr, len(entries), views.n_views)
        if nb == 0:
            raise StaError(-1, "sta_batch_workspace_bytes: bad design list")
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        h = _P()
        self._views, self._lib = views, lib
        _check(blib.sta_batch_create(arr, len(entries), ctypes.byref(lib), ctypes.byref(views),
                                     _ptr(self.workspace), nb, ctypes.byref(h)), "sta_batch_create")
        self._h = h

    def delay_calc(self, precision=None, use_graph=True):
        import torch
        prec = STA_DC_FP64 if precision is None else precision
        _check(_batch_lib().sta_batch_delay_calc(self._h, int(prec), int(use_graph), _stream(torch, self.device)),
               "sta_batch_delay_calc")

    def propagate(self, use_graph=True, blocks=0):
        import torch
        _check(_batch_lib().sta_batch_propagate(self._h, int(use_graph), int(blocks), _stream(torch, self.device)),
               "sta_batch_propagate")

    def slack(self, use_graph=True):
        import torch
        _check(_batch_lib().sta_batch_slack(self._h, int(use_graph), _stream(torch, self.device)),
               "sta_batch_slack")

    def set_tiling(self, fwd_views_per_wave, bwd_views_per_wave):
        _check(_batch_lib().sta_batch_set_tiling(self._h, int(fwd_views_per_wave), int(bwd_views_per_wave)),
               "sta_batch_set_tiling")
        return self

    def info(self):
        p = BatchPlanC()
        _check(_batch_lib().sta_batch_info(self._h, ctypes.byref(p)), "sta_batch_info")
        return {f: int(getattr(p, f)) for f, _ in BatchPlanC._fields_}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sta_batch_free(h)
            self._h = None
