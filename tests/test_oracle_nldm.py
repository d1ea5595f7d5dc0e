"""Pins of the oracle's NLDM lookup (step 3).  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2203_08395_amd import gen


def _bilinear_table(a, b, c, e):
    x = gen.AXIS_X.astype(np.float64)[:, None]
    y = gen.AXIS_Y.astype(np.float64)[None, :]
    return (a + b * x + c * y + e * x * y).astype(np.float32)


@pytest.mark.parametrize("seed", range(5))
def test_reproduces_bilinear_function_inside_and_outside(seed):
    # a table sampled from f = a + b x + c y + e x y is reproduced exactly in real
    # arithmetic anywhere, extrapolation included; FP32 leaves a few ulps
    rng = np.random.default_rng(seed)
    a, b, c, e = rng.uniform(1, 10), rng.uniform(0.05, 0.3), rng.uniform(0.5, 3), rng.uniform(0, 0.01)
    T = _bilinear_table(a, b, c, e)
    s = rng.uniform(1.0, 700.0, 4000).astype(np.float32)
    l = rng.uniform(0.5, 260.0, 4000).astype(np.float32)
    v = oracle.bilerp(gen.AXIS_X, gen.AXIS_Y, T, s, l).astype(np.float64)
    sd, ld = s.astype(np.float64), l.astype(np.float64)
    f = a + b * sd + c * ld + e * sd * ld
    scale = np.abs(T).max() * (1 + np.maximum(sd / 500.0, ld / 200.0))
    assert np.all(np.abs(v - f) <= 4e-6 * scale)


def test_grid_points_exact():
    lib = gen.make_library(n_tables=4, seed=3)
    for t in range(4):
        T = lib.tab[t, 0]
        for i in range(7):
            for j in range(7):
                v = oracle.bilerp(lib.x, lib.y, T, lib.x[i], lib.y[j])[0]
                if i < 6 and j < 6:
                    assert v == T[i, j]
                else:
                    assert abs(v - T[i, j]) <= 2 * np.spacing(T[i, j])


def test_segment_rule_below_and_above_axis():
    # below x[0] the first segment extrapolates; above x[6] the last one does
    T = _bilinear_table(3.0, 0.25, 0.0, 0.0)      # depends on slew only: 3 + 0.25 s
    for s in [0.5, 2.0, 4.999, 600.0, 1000.0]:
        v = oracle.bilerp(gen.AXIS_X, gen.AXIS_Y, T, np.float32(s), np.float32(10.0))[0]
        assert abs(v - (3.0 + 0.25 * s)) <= 1e-5 * (3.0 + 0.25 * s)


def test_axis_transpose_would_fail():
    # delay depends on load only: swapping the axes or the table indices would break this
    T = _bilinear_table(2.0, 0.0, 1.5, 0.0)
    s = np.float32(50.0)
    for l in [1.0, 3.0, 14.0, 100.0, 200.0]:
        v = oracle.bilerp(gen.AXIS_X, gen.AXIS_Y, T, s, np.float32(l))[0]
        assert abs(v - (2.0 + 1.5 * l)) <= 1e-5 * (2.0 + 1.5 * l)


def test_monotone_tables_give_monotone_results():
    lib = gen.make_library(n_tables=8, seed=9)
    rng = np.random.default_rng(0)
    for t in range(8):
        for k in (0, 1):
            T = lib.tab[t, k]
            s = np.sort(rng.uniform(5, 500, 500)).astype(np.float32)
            l = np.full(500, np.float32(rng.uniform(1, 200)), np.float32)
            v = oracle.bilerp(lib.x, lib.y, T, s, l)
            assert np.all(np.diff(v) >= -2 * np.spacing(np.abs(v[1:])))
            l = np.sort(rng.uniform(1, 200, 500)).astype(np.float32)
            s = np.full(500, np.float32(rng.uniform(5, 500)), np.float32)
            v = oracle.bilerp(lib.x, lib.y, T, s, l)
            assert np.all(np.diff(v) >= -2 * np.spacing(np.abs(v[1:])))
