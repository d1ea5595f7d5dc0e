"""Pins of the RC-tree and learned-surrogate reference (CPU only).

Tree moments are checked against the path-overlap definition of the RC-tree moments
(independent of the sweep order the reference uses), a uniform chain in closed form, the
Elmore bounds, and brute-force features.  The network reference is checked against
central finite differences, torch's bfloat16 rounding and torch's Adam."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08395_amd import gen


def _path(par, k):
    out = []
    while k != 0:
        out.append(k)
        k = par[k]
    return out


def _brute_tree(T, n):
    """m1, m2 of every node of net n from the definition: m1(k) = sum_v C_v R(k, v),
    m2(k) = sum_v C_v R(k, v) m1(v), R(k, v) = resistance shared by the root paths."""
    a, b = T.net_node_ptr[n], T.net_node_ptr[n + 1]
    par = T.node_parent[a:b]
    R = T.node_R[a:b].astype(np.float64)
    C = T.node_C[a:b].astype(np.float64).copy()
    for s in range(T.sink_ptr[n], T.sink_ptr[n + 1]):
        C[T.sink_node[s]] += T.sink_pincap[s]
    M = b - a
    paths = [set(_path(par, k)) for k in range(M)]
    Rs = np.array([[sum(R[e] for e in paths[k] & paths[v]) for v in range(M)] for k in range(M)])
    m1 = (Rs * C[None, :]).sum(1) * 1e-3
    m2 = (Rs * (C * m1)[None, :]).sum(1) * 1e-3
    return m1, m2, C, paths


def test_tree_moments_match_path_overlap_definition():
    T = gen.make_rc_trees(40, m_range=(2, 20), seed=11)
    mom = oracle.tree_moments(T, features=True)
    for n in range(T.n_nets):
        m1, m2, C, paths = _brute_tree(T, n)
        for s in range(T.sink_ptr[n], T.sink_ptr[n + 1]):
            k = T.sink_node[s]
            assert mom["m1"][s] == pytest.approx(m1[k], rel=1e-12)
            assert mom["imp2"][s] == pytest.approx(max(0.0, 2 * m2[k] - m1[k] ** 2), rel=1e-9, abs=1e-9 * m1[k] ** 2)
        assert mom["load"][n] == pytest.approx(C.sum(), rel=1e-14)


def test_tree_features_brute_force():
    T = gen.make_rc_trees(30, m_range=(2, 24), seed=12)
    f = oracle.tree_moments(T, features=True)["feat"]
    for n in range(T.n_nets):
        a, b = T.net_node_ptr[n], T.net_node_ptr[n + 1]
        par = T.node_parent[a:b]
        R = T.node_R[a:b].astype(np.float64)
        Cw = T.node_C[a:b].astype(np.float64)
        _, _, C, paths = _brute_tree(T, n)
        M = b - a
        sub = [C[[v for v in range(M) if k in paths[v] or v == k]].sum() for k in range(M)]
        ns = T.sink_ptr[n + 1] - T.sink_ptr[n]
        for s in range(T.sink_ptr[n], T.sink_ptr[n + 1]):
            k = T.sink_node[s]
            p = _path(par, k)
            exp = [R[p].sum(), C.sum(), sub[k], len(p), M, ns, R[p[-1]], C[p].sum(),
                   R[1:].mean(), Cw.mean(), T.sink_pincap[s], T.drv_slew[n]]
            np.testing.assert_allclose(f[s], exp, rtol=1e-12)


def test_chain_closed_form():
    # one chain of n nodes, equal r and c, one sink at the far end
    for n in (2, 5, 9):
        r, c, cp = 100.0, 2.0, 3.0
        T = gen.TreeSet(net_node_ptr=np.array([0, n], np.int32), node_parent=np.arange(-1, n - 1, dtype=np.int32),
                        node_R=np.full(n, r, np.float32), node_C=np.full(n, c, np.float32),
                        sink_ptr=np.array([0, 1], np.int32), sink_node=np.array([n - 1], np.int32),
                        sink_pincap=np.array([cp], np.float32), drv_slew=np.array([10.0], np.float32))
        T.node_R[0] = 0.0
        mom = oracle.tree_moments(T)
        m1 = r * (c * n * (n - 1) / 2 + (n - 1) * cp) * 1e-3
        assert mom["m1"][0] == pytest.approx(m1, rel=1e-14)
        assert mom["load"][0] == pytest.approx(n * c + cp, rel=1e-14)


def test_elmore_bounds_and_target_decode():
    T = gen.make_rc_trees(3000, seed=13)
    mom = oracle.tree_moments(T, features=True)
    f = mom["feat"]
    L = f[:, 0] * f[:, 2] * 1e-3
    U = f[:, 0] * f[:, 1] * 1e-3
    assert np.all(L <= mom["m1"] * (1 + 1e-12)) and np.all(mom["m1"] <= U * (1 + 1e-12))
    t = oracle.surrogate_targets(T, mom)
    assert np.all((t[:, 0] >= 0) & (t[:, 0] <= 1)) and np.all(t[:, 1] >= 0)
    d, s = oracle.decode(f.astype(np.float32), t)
    exact = oracle.tree_targets(T, mom)
    np.testing.assert_allclose(d, exact[:, 0], rtol=2e-6, atol=1e-6)
    np.testing.assert_allclose(s, exact[:, 1], rtol=2e-6, atol=1e-6)


def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e-3])])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16(x), ref)


def _fd_check(quant):
    p = oracle.MLP.init(3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((48, 16))
    x[:, 12:] = 0
    t = rng.standard_normal((48, 2)) * 0.3
    g = oracle.MLP(p).grads(x, t, quant=quant)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            if k == "W1" and idx % 16 >= 12:
                continue
            h = 1e-6
            pp = {kk: v.copy() for kk, v in p.items()}
            pp[k].reshape(-1)[idx] += h
            lp = oracle.MLP(pp).loss(x, t, quant=False)
            pp[k].reshape(-1)[idx] -= 2 * h
            lm = oracle.MLP(pp).loss(x, t, quant=False)
            fd = (lp - lm) / (2 * h)
            yield k, g[k].reshape(-1)[idx], fd


def test_mlp_gradients_central_differences():
    for k, an, fd in _fd_check(quant=False):
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_mlp_quantized_path_is_exact_on_dyadic_values():
    """With inputs, weights and every intermediate value short dyadic rationals, all the
    BF16 rounding points are exact, so the quantized forward and gradients must equal the
    FP64 ones (and hence the finite differences above)."""
    rng = np.random.default_rng(6)
    def sparse_rows(o, i, nnz):
        W = np.zeros((o, i))
        for r in range(o):
            W[r, rng.choice(i, nnz, replace=False)] = rng.choice([-0.25, 0.25], nnz)
        return W
    W1 = np.zeros((64, 16))
    W1[:, :12] = rng.choice([-0.25, 0.0, 0.25], (64, 12))
    p = {"W1": W1, "b1": rng.choice([-0.25, 0.0, 0.25], 64), "W2": sparse_rows(64, 64, 4),
         "b2": rng.choice([-0.25, 0.0, 0.25], 64), "W3": sparse_rows(2, 64, 4), "b3": np.array([0.25, -0.25])}
    x = np.zeros((4, 16))
    x[:, :12] = rng.choice([-1.0, 0.0, 1.0], (4, 12))
    mlp = oracle.MLP(p)
    y, _ = mlp.forward(x, quant=False)
    t = y - rng.choice([-0.25, 0.25], y.shape)
    yq, _ = mlp.forward(x, quant=True)
    np.testing.assert_array_equal(yq, y)
    g0, g1 = mlp.grads(x, t, quant=False), mlp.grads(x, t, quant=True)
    for k in g0:
        np.testing.assert_array_equal(g1[k], g0[k])
    assert any(np.abs(g0[k]).sum() > 0 for k in ("W1", "W2"))


def test_mlp_forward_matches_torch_float64():
    p = oracle.MLP.init(5)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((100, 16))
    y, _ = oracle.MLP(p).forward(x, quant=False)
    tp = {k: torch.from_numpy(v) for k, v in p.items()}
    h = torch.relu(torch.from_numpy(x) @ tp["W1"].T + tp["b1"])
    h = torch.relu(h @ tp["W2"].T + tp["b2"])
    np.testing.assert_allclose(y, (h @ tp["W3"].T + tp["b3"]).numpy(), rtol=1e-12, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(50)
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = oracle.adam(p, g, m, v, step, 1e-2)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_calibration_bound_is_a_quantile_upper_bound():
    rng = np.random.default_rng(4)
    n = 60000
    feat = np.ones((n, 12))
    feat[:, 3] = rng.integers(1, 12, n)
    feat[:, 4] = rng.integers(2, 65, n)
    err = np.abs(rng.standard_normal((n, 2)) * 10.0 ** rng.uniform(-4, -1, (n, 2))).astype(np.float32)
    q = oracle.calibrate(feat, err, quantile=0.999, min_count=256)
    b = oracle.error_bin(feat)
    for i in range(oracle.N_BINS):
        sel = b == i
        for o in range(2):
            e = err[sel, o]
            if e.size < 256:
                assert np.isinf(q[i, o])
                continue
            allow = int(np.floor(0.001 * e.size))
            assert np.sum(e >= q[i, o]) <= allow
            # one bucket lower would exceed the allowance: the bound is tight to a bucket
            k = 509 - (int(np.array([q[i, o]], np.float32).view(np.uint32)[0]) >> 21)
            lower = oracle.bucket_bound(k + 1)
            assert np.sum(e >= lower) > allow


def test_error_buckets_are_monotone_and_exact_on_edges():
    e = np.array([0.0, 2.0 ** -40, 0.001, 0.5, 0.625, 0.7499, 0.75, 1.0, 7.0], np.float32)
    k = oracle.error_bucket(e)
    assert list(k) == sorted(k, reverse=True)
    for kk in range(1, 127):
        lo = np.float32(oracle.bucket_bound(kk + 1))
        assert oracle.error_bucket(np.array([lo], np.float32))[0] == kk
        assert oracle.error_bucket(np.array([np.nextafter(lo, np.float32(0))], np.float32))[0] == kk + 1 or kk == 126


def test_norm_stats_hand_values():
    """Hand-computed statistics of log(1 + f): a constant feature (std 0 -> rstd 1), a
    two-valued feature whose population std is 1/2 (the sample std would be larger), and
    features whose logs are equally spaced."""
    n = 6
    feat = np.zeros((n, 12))
    feat[:, 0] = 3.0                                   # log 4 everywhere: mean log 4, rstd 1
    feat[:, 1] = [0.0, np.e - 1.0] * 3                 # logs 0, 1: mean 1/2, population std 1/2
    feat[:, 2] = [0.0, 1.0, 3.0, 7.0, 0.0, 1.0]        # logs (0, 1, 2, 3, 0, 1) * log 2
    feat[:, 3] = 0.0                                   # log 0 + 1 = 0: mean 0, rstd 1
    mu, rstd = oracle.norm_stats(feat)
    assert mu[0] == pytest.approx(np.log(4.0), rel=1e-15) and rstd[0] == 1.0
    assert mu[1] == pytest.approx(0.5, rel=1e-15) and rstd[1] == pytest.approx(2.0, rel=1e-14)
    # logs 0,1,2,3,0,1 (x log 2): mean 7/6, E[k^2] = 15/6, variance 15/6 - 49/36 = 41/36
    assert mu[2] == pytest.approx(7.0 / 6.0 * np.log(2.0), rel=1e-14)
    assert rstd[2] == pytest.approx(1.0 / (np.log(2.0) * np.sqrt(41.0 / 36.0)), rel=1e-14)
    assert mu[3] == 0.0 and rstd[3] == 1.0


def test_mlp_input_hand_values():
    """x = (log(1 + f) - mu) * rstd on the 12 features, zero in the 4 pad columns: a zero
    feature gives the finite value -mu * rstd (log f would give -inf)."""
    feat = np.zeros((2, 12))
    feat[0, 0] = np.e - 1.0        # log(1 + f) = 1
    feat[1, 5] = 3.0               # log 4
    mu = np.full(12, 0.25)
    rstd = np.full(12, 4.0)
    x = oracle.mlp_input(feat, mu, rstd)
    assert x.shape == (2, 16)
    assert x[0, 0] == pytest.approx(3.0, rel=1e-15)                      # (1 - 1/4) * 4
    assert x[0, 1] == -1.0 and x[1, 0] == -1.0                            # zero feature: -mu * rstd
    assert x[1, 5] == pytest.approx((np.log(4.0) - 0.25) * 4.0, rel=1e-15)
    assert np.all(x[:, 12:] == 0.0)
    assert np.all(np.isfinite(x))


def test_error_bin_hand_values():
    """Bins of (depth, nodes) pairs written out by hand from the rule: depth class
    clamp(depth, 1, 8) - 1 (so 7 and 8 differ, 8 and 9 share), size class (M - 1) // 8
    clamped to 0..7 (so M = 8 | 9 and M = 64 | 65 straddle or share the edges)."""
    cases = [  # (depth, M, bin)
        (1, 2, 0), (1, 8, 0), (1, 9, 1), (1, 64, 7), (1, 65, 7), (1, 200, 7),
        (0, 5, 0),                                          # depth below 1 joins class 1
        (2, 17, 8 + 2), (7, 8, 48), (7, 9, 49), (8, 8, 56), (8, 9, 57), (8, 64, 63),
        (9, 65, 63), (30, 33, 56 + 4), (3, 1, 16),
    ]
    feat = np.zeros((len(cases), 12))
    feat[:, 3] = [c[0] for c in cases]
    feat[:, 4] = [c[1] for c in cases]
    assert list(oracle.error_bin(feat)) == [c[2] for c in cases]
