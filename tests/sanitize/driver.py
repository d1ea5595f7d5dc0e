"""Drives the sanitizer builds of the oracle and of libsta's host code (run in a child
process with the sanitizer runtimes preloaded): levelization, delay calculation,
propagation and slack of the oracle, and graph build, sizes, maps, fusion plan and every
validation error of the host library, on seeded designs and planted bad inputs."""
import ctypes
import sys

import numpy as np

sys.path.insert(0, sys.argv[3])
import oracle  # noqa: E402
from paper_2203_08395_amd import gen, sta  # noqa: E402


def main():
    proc = ctypes.CDLL(None)
    assert hasattr(proc, "__asan_init") and hasattr(proc, "__ubsan_handle_add_overflow"), "sanitizers not loaded"
    oracle._LIB_PATH = sys.argv[1]
    oracle._LIB_OMP_PATH = sys.argv[1]
    host = ctypes.CDLL(sys.argv[2])
    P = ctypes.c_void_p
    host.sta_build_graph.argtypes = [P, P]
    host.sta_graph_sizes.argtypes = [P, P]
    host.sta_graph_perm.argtypes = [P] * 6
    host.sta_graph_spans.argtypes = [P, P]
    host.sta_graph_span_list.argtypes = [P, P, P]
    host.sta_graph_free.argtypes = [P]
    host.sta_last_error.restype = ctypes.c_char_p
    designs = [gen.make_design(**gen.CONFIGS["c1"]),
               gen.make_design(n_pins=40000, n_levels=60, fanin="geom", seed=93, n_fanout64=2),
               gen.make_design(n_pins=200, n_levels=5, fanin="uniform4", seed=94)]
    lib = gen.make_library()
    for d in designs:
        pa, ps = gen.make_pi(d)
        late, early = gen.make_rat(d, 10, late_per_level=70.0, hold=120.0)
        oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY))
        oracle.run(d, lib, pa, ps, late, early, modes=(oracle.LATE, oracle.EARLY), par=True)
        oracle.levelize(d)
        keep = [np.ascontiguousarray(a, dt) for a, dt in (
            (d.gate_arc_ptr, np.int32), (d.arc_drv, np.int32), (d.arc_tbl, np.int32), (d.arc_tap, np.int32),
            (d.arc_pincap, np.float32), (d.net_node_ptr, np.int32), (d.node_parent, np.int32),
            (d.node_R, np.float32), (d.node_C, np.float32))]

        def build(arrs, n_tables=lib.n_tables):
            desc = sta.DesignDesc(int(d.n_pi), int(d.n_gates), n_tables, *[P(a.ctypes.data) for a in arrs])
            h = P()
            st = host.sta_build_graph(ctypes.byref(desc), ctypes.byref(h))
            return st, h

        st, h = build(keep)
        assert st == 0, host.sta_last_error()
        s = sta.Sizes()
        assert host.sta_graph_sizes(h, ctypes.byref(s)) == 0
        D, A, G, E = s.n_drivers, s.n_arcs, s.n_gates, s.n_endpoints
        maps = [np.zeros(n, np.int32) for n in (D, A, G, D, E)]
        assert host.sta_graph_perm(h, *[P(m.ctypes.data) if m.size else None for m in maps]) == 0
        info = sta.SpanInfo()
        assert host.sta_graph_spans(h, ctypes.byref(info)) == 0
        fwd = np.zeros((info.fwd_spans, 3), np.int32)
        bwd = np.zeros((info.bwd_spans, 3), np.int32)
        assert host.sta_graph_span_list(h, P(fwd.ctypes.data), P(bwd.ctypes.data)) == 0
        host.sta_graph_free(h)
        # planted errors: range, table, non-finite, cycle
        bad = [a.copy() for a in keep]
        bad[1][0] = D + 5
        assert build(bad)[0] == sta_status("E_RANGE")
        bad = [a.copy() for a in keep]
        bad[2][-1] = lib.n_tables
        assert build(bad)[0] == sta_status("E_RANGE")
        bad = [a.copy() for a in keep]
        bad[7][1] = np.nan
        assert build(bad)[0] == sta_status("E_NONFINITE")
        bad = [a.copy() for a in keep]
        g_last = d.n_gates - 1
        a0, a1 = int(d.gate_arc_ptr[0]), int(d.gate_arc_ptr[g_last])
        bad[1][a0], bad[3][a0] = d.n_pi + g_last, 0          # gate 0 reads the last gate ...
        bad[1][a1], bad[3][a1] = d.n_pi + 0, 0               # ... and the last gate reads gate 0
        assert build(bad)[0] == sta_status("E_CYCLE")
    print("sanitized host code and oracle: clean", flush=True)


def sta_status(name):
    return {v: k for k, v in sta._STATUS.items()}[name]


if __name__ == "__main__":
    main()
