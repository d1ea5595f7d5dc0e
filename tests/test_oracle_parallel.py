"""The OpenMP build of the oracle (level by level, each level's gates, drivers and nets
spread over threads) against the serial build (Kahn order), bit for bit, at several
thread counts.  The per-gate arithmetic is one routine in both; this checks that the
level order and the threads change nothing."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen


def _bits(x):
    x = np.ascontiguousarray(x)
    return x.view(np.uint32) if x.dtype == np.float32 else x.view(np.uint64) if x.dtype == np.float64 else x


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("case", ["c1", "geom"])
def test_parallel_oracle_equals_serial(case, threads):
    if case == "c1":
        cfg = gen.CONFIGS["c1"]
        rp = gen.RAT_PARAMS["c1"]
    else:
        cfg = dict(n_pins=60000, n_levels=80, fanin="geom", seed=91, n_fanout64=2)
        rp = dict(late_per_level=70.0, hold=120.0)
    d = gen.make_design(**cfg)
    lib = gen.make_library()
    pa, ps = gen.make_pi(d)
    late, early = gen.make_rat(d, cfg["n_levels"], **rp)
    assert oracle.threads(threads) == threads
    modes = (oracle.LATE, oracle.EARLY)
    a = oracle.run(d, lib, pa, ps, late, early, modes=modes)
    b = oracle.run(d, lib, pa, ps, late, early, modes=modes, par=True)
    for k in ("load", "net_delay", "net_imp2"):
        np.testing.assert_array_equal(_bits(a[k]), _bits(b[k]), err_msg=k)
    for m in ("late", "early"):
        for k, v in a[m].items():
            if isinstance(v, np.ndarray):
                np.testing.assert_array_equal(_bits(v), _bits(b[m][k]), err_msg=f"{m} {k}")
        assert a[m]["tns"] == b[m]["tns"] and _bits(np.float32(a[m]["wns"])) == _bits(np.float32(b[m]["wns"]))


def test_parallel_moments_equal_serial():
    d = gen.make_design(n_pins=20000, n_levels=40, fanin="geom", seed=92, n_fanout64=1)
    oracle.threads(4)
    a = oracle.delay_calc(d, moments=True)
    b = oracle.delay_calc(d, moments=True, par=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(_bits(x), _bits(y))
