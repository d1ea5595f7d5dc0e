"""Host-side checks of the C ABI: exported symbols, graph build, levelization and the
validation errors.  No GPU is touched (sta_build_graph is host only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen, sta
from tests import tiny

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="sta.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(sta_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = sta.load_library()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sta.EXPORTS)


def test_library_exports_every_surrogate_symbol():
    from paper_2203_08395_amd import surrogate
    lib = surrogate._lib()
    names = _declared("sta_surrogate.h")
    assert len(names) == 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(surrogate.EXPORTS)


def test_library_exports_every_analysis_symbol():
    lib = sta._ana()
    names = _declared("sta_analysis.h")
    assert len(names) == 4
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sta.ANALYSIS_EXPORTS)
    assert lib.sta_paths_scratch_bytes() == 128 * 64 * 8
    assert lib.sta_tns_adjoint(None, None, None, None, None, None, None, None) == -1
    assert lib.sta_critical_paths(None, None, 0, 1, None, None, None, None, 0, None) == -1


def test_timing_calls_validate_before_launching():
    """Null arguments and a graph that is not uploaded are errors, caught on the host."""
    lib = sta.load_library()
    assert lib.sta_propagate(None, None, None, None, None, None, None) == -1
    g = sta.Graph(_ok_design(), n_tables=4)
    L = sta.LibraryC()
    v = sta.ViewsC()
    no, to = sta.NetOut(), sta.TimingOut()
    st = lib.sta_propagate(g.handle, ctypes.byref(L), ctypes.byref(v), None, ctypes.byref(no), ctypes.byref(to), None)
    assert st == -1 and b"not uploaded" in lib.sta_last_error()
    st = lib.sta_delay_calc(g.handle, 0, ctypes.byref(no), None)
    assert st == -1 and b"not uploaded" in lib.sta_last_error()


def test_surrogate_host_validation_without_gpu():
    """Argument errors are caught before any launch (no device pointer is touched)."""
    from paper_2203_08395_amd import surrogate
    lib = surrogate._lib()
    assert lib.sta_tree_dataset(None, None, None, None, None, None, None) == -1
    t = surrogate.TreesC(-1, 0)
    assert lib.sta_tree_exact(ctypes.byref(t), None, None, None, None, None, None) == -1
    assert lib.sta_mlp_train_step(None, None, None, None, None, None, None, None, 0, None, None, 0, None) == -1
    assert lib.sta_mlp_grad_scratch_bytes(0) == 0
    assert lib.sta_mlp_grad_scratch_bytes(33) == 2 * 5380 * 4
    assert lib.sta_mlp_grad_scratch_bytes(10 ** 6) == 1024 * 5380 * 4
    assert lib.sta_surrogate_calibrate(None, None, None, 10, 1.5, 0, None, None, 0, None) == -1
    assert lib.sta_mlp_norm_scratch_bytes() == 256 * 24 * 8
    assert lib.sta_surrogate_cal_scratch_bytes() == 64 * 2 * 128 * 4
    # empty tree set: nothing to launch
    t0 = surrogate.TreesC(0, 0)
    assert lib.sta_tree_exact(ctypes.byref(t0), None, None, None, None, None, None) == 0


@pytest.mark.parametrize("cfg", ["c1", "small_geom"])
def test_levels_and_numbering_match_oracle(cfg):
    if cfg == "c1":
        d = gen.make_design(**gen.CONFIGS["c1"])
    else:
        d = gen.make_design(n_pins=20000, n_levels=60, fanin="geom", seed=9, n_fanout64=3)
    g = sta.Graph(d, n_tables=128)
    lv, _ = oracle.levelize(d)
    assert np.array_equal(g.drv_to_input(g.level), lv)
    assert g.sizes["n_levels"] == lv.max()
    # internal order is level order, PIs first and unchanged
    assert np.all(np.diff(g.level) >= 0)
    assert np.array_equal(g.drv_input[:d.n_pi], np.arange(d.n_pi))
    assert np.array_equal(np.sort(g.drv_input), np.arange(d.n_drivers))
    assert np.array_equal(np.sort(g.arc_input), np.arange(d.n_arcs))
    # arcs of a gate stay contiguous and in input order
    gi = g.gate_input
    k_int = np.diff(d.gate_arc_ptr)[gi]
    ptr = np.concatenate([[0], np.cumsum(k_int)])
    for i in range(0, d.n_gates, 97):
        q = gi[i]
        assert np.array_equal(g.arc_input[ptr[i]:ptr[i + 1]], np.arange(d.gate_arc_ptr[q], d.gate_arc_ptr[q + 1]))
    ep = oracle.endpoints(d)
    assert np.array_equal(g.drv_input[g.ep_driver], ep)
    s = g.sizes
    assert s["n_pins"] == d.n_pins and s["n_endpoints"] == ep.size
    assert s["graph_bytes"] > 0 and s["scratch_bytes"] > 0


def _expect(status, d, n_tables=4):
    with pytest.raises(sta.StaError) as e:
        sta.Graph(d, n_tables=n_tables)
    assert e.value.name == status, str(e.value)
    return str(e.value)


def _ok_design():
    nets = [tiny.chain_net([100.0, 200.0], [0.5, 0.5, 0.5]) for _ in range(5)]
    return tiny.design(2, [[0, 1], [2], [3, 0]], nets, tables=[0, 1, 2, 3, 0])


def test_valid_small_design_builds():
    g = sta.Graph(_ok_design(), n_tables=4)
    assert g.sizes["n_levels"] == 3
    assert list(g.level) == [0, 0, 1, 2, 3]


def test_cycle():
    nets = [tiny.chain_net([100.0], [1.0, 1.0])] * 3
    msg = _expect("E_CYCLE", tiny.design(1, [[0, 2], [1]], nets))
    assert "cycle" in msg
    _expect("E_CYCLE", tiny.design(1, [[0, 1]], nets[:2]))        # self loop


def test_range_errors():
    d = _ok_design(); d.arc_drv[1] = 9
    _expect("E_RANGE", d)
    d = _ok_design(); d.arc_drv[0] = -1
    _expect("E_RANGE", d)
    d = _ok_design(); d.arc_tbl[2] = 4
    _expect("E_RANGE", d)
    d = _ok_design(); d.arc_tap[0] = 3
    _expect("E_RANGE", d)
    d = _ok_design(); d.node_parent[2] = 2
    _expect("E_RANGE", d)
    d = _ok_design(); d.node_parent[3] = 0           # node 0 of net 1 must have no parent
    _expect("E_RANGE", d)


def test_nonfinite_errors():
    for field, idx in (("node_R", 1), ("node_C", 4), ("arc_pincap", 2)):
        for bad in (np.nan, np.inf, -1.0):
            d = _ok_design()
            getattr(d, field)[idx] = bad
            _expect("E_NONFINITE", d)


def test_arg_errors():
    d = _ok_design(); d.gate_arc_ptr[1] = 0            # a gate without inputs
    _expect("E_ARG", d)
    wide = tiny.design(65, [list(range(65))], [tiny.chain_net([1.0], [1.0, 1.0])] * 66)
    _expect("E_ARG", wide, n_tables=1)                 # fanin above the maximum
    big = tiny.design(1, [[0]], [tiny.chain_net([1.0] * 256, [1.0] * 257), tiny.chain_net([1.0], [1.0, 1.0])])
    _expect("E_ARG", big, n_tables=1)                  # RC net above the node maximum
    _expect("E_ARG", _ok_design(), n_tables=0)


def test_empty_design_builds():
    d = tiny.design(0, [], [])
    g = sta.Graph(d, n_tables=1)
    assert g.sizes["n_drivers"] == 0 and g.sizes["n_levels"] == 0


def test_pi_only_design():
    d = tiny.design(3, [], [tiny.chain_net([5.0], [1.0, 1.0])] * 3)
    g = sta.Graph(d, n_tables=1)
    assert g.sizes["n_endpoints"] == 3 and g.sizes["n_levels"] == 0


def test_library_exports_every_batch_symbol():
    lib = sta._batch_lib()
    names = _declared("sta_batch.h")
    assert len(names) == 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sta.BATCH_EXPORTS)
    # host-side validation, no device memory touched
    assert lib.sta_batch_workspace_bytes(None, -1, 4) == 0
    assert lib.sta_batch_workspace_bytes(None, 0, 0) == 0
    assert lib.sta_batch_delay_calc(None, 0, 1, None) == -1
    assert lib.sta_batch_propagate(None, 1, 0, None) == -1
    assert lib.sta_batch_slack(None, 1, None) == -1
    assert lib.sta_batch_info(None, None) == -1
    assert lib.sta_batch_set_tiling(None, 1, 1) == -1


def test_span_length_caps():
    """sta_build_graph_spans: lengths outside 1..8 are refused; within, every span is at
    most that long and the levelization does not change."""
    d = gen.make_design(n_pins=6000, n_levels=40, fanin="geom", seed=9, n_fanout64=1)
    for bad in ((0, 8), (8, 0), (9, 8), (8, 9)):
        with pytest.raises(sta.StaError):
            sta.Graph(d, n_tables=128, span_levels=bad)
    ref = sta.Graph(d, n_tables=128)
    for caps in ((1, 1), (3, 5), (8, 2)):
        g = sta.Graph(d, n_tables=128, span_levels=caps)
        f, b = g.span_list()
        assert np.all(f[:, 1] - f[:, 0] + 1 <= caps[0]) and np.all(b[:, 0] - b[:, 1] + 1 <= caps[1])
        assert f[0, 0] == 1 and f[-1, 1] == d_levels(ref) and b[0, 0] == d_levels(ref) and b[-1, 1] == 0
        np.testing.assert_array_equal(g.level, ref.level)
        np.testing.assert_array_equal(g.drv_input, ref.drv_input)
        assert g.spans["fwd_span_arcs"] == ref.spans["fwd_span_arcs"] == d.n_arcs
    g1 = sta.Graph(d, n_tables=128, span_levels=(1, 1))
    assert g1.spans["fwd_span_launches"] == d_levels(ref)


def d_levels(g):
    return g.sizes["n_levels"]
