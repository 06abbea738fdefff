"""Pins for the oracle's CDF-model pieces (feature, targets, loss and gradient, Adam, splitters).

Closed forms: special parameter settings where the network reduces to a constant or to
a single hinge, Mitchell's error bound for the log feature, the first Adam step
(an update of lr * sign(g)), and exact quantile splitters when the model equals the
empirical mid-CDF.  Gradients: central differences of the oracle's own loss (exact for
the parameters the loss is quadratic in, and away from hinge kinks for the others).
"""
import math

import numpy as np
import pytest

import oracle

H = 64


def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) from state 0: its first outputs are the
    published sequence (the same stream as Java's SplittableRandom(0).nextLong(), whose first
    value is -2152535657050944081)."""
    got = [int(v) for v in oracle.splitmix64(0, 4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert got[0] == (1 << 64) - 2152535657050944081


def test_sample_bernoulli_uses_stream_and_kept_fraction():
    """Row i is kept iff the (i+1)-th output of the pinned stream is below frac * 2^64, and the
    kept count lies in a 5-sigma binomial band."""
    n, seed = 400_000, 987654321
    keys = np.arange(n, dtype=np.int64) * 5 - 7
    z = oracle.splitmix64(seed, n)
    for frac in (0.01, 0.25):
        s = oracle.sample_bernoulli(keys, seed, frac)
        thr = np.uint64(int(frac * 2**64))
        assert np.array_equal(s, keys[z < thr])
        sd = math.sqrt(n * frac * (1 - frac))
        assert abs(len(s) - n * frac) < 5 * sd
    assert np.array_equal(oracle.sample_bernoulli(keys[:1000], seed, 1.0), keys[:1000])
    assert len(oracle.sample_bernoulli(keys[:1000], seed, 0.0)) == 0


def test_feature_exact_values():
    L = 40
    scale = np.float32(1.0 / (L * 2**23))
    kmin = 100
    x = oracle.cdf_feature([100, 101, 102, 99, -5], kmin, scale)
    assert x[0] == 0.0 and x[3] == 0.0 and x[4] == 0.0
    assert x[1] == np.float32(np.float32(2**23) * scale)                    # log2(2) = 1
    assert x[2] == np.float32(np.float32(2**23 + 2**22) * scale)            # 1 + 0.5 (Mitchell)


def test_feature_mitchell_bound_and_monotone():
    rng = np.random.default_rng(0)
    kmin = 1
    L = 41
    scale = np.float32(1.0 / (L * 2**23))
    keys = np.sort(np.concatenate([rng.integers(1, 2**40, 3000), np.arange(1, 2000)])).astype(np.int64)
    x = oracle.cdf_feature(keys, kmin, scale).astype(np.float64)
    assert np.all(np.diff(x) >= 0)
    lg = np.log2((keys - kmin + 1).astype(np.float64))
    err = lg - x * L
    # Mitchell: 0 <= log2(v) - (l + frac) <= 0.0861; plus FP32 rounding of the fixed point
    assert err.min() > -1e-5 and err.max() < 0.0861 + 1e-5


def test_targets_mid_cdf():
    n = 10
    t = oracle.cdf_targets(np.arange(n))
    assert np.array_equal(t, np.array([(2 * i + 1) / (2 * n) for i in range(n)], np.float32))
    assert np.all(oracle.cdf_targets(np.full(7, 3)) == np.float32(0.5))
    assert oracle.cdf_targets(np.array([1, 1, 2])).tolist() == [np.float32(1 / 3)] * 2 + [np.float32(5 / 6)]


def _params(w1, b1, w2, b2):
    return np.concatenate([w1, b1, w2, [b2]]).astype(np.float32)


def test_loss_constant_network_closed_form():
    rng = np.random.default_rng(1)
    x = rng.random(500).astype(np.float32)
    t = rng.random(500).astype(np.float32)
    b2 = 0.3
    p = _params(rng.normal(size=H), rng.normal(size=H), np.zeros(H), b2)
    loss, g = oracle.mlp_loss_grad(p, x, t)
    e = np.float64(np.float32(b2)) - t.astype(np.float64)
    assert loss == pytest.approx(np.mean(e**2), rel=1e-12)
    assert g[3 * H] == pytest.approx(2 * np.mean(e), rel=1e-12)
    assert np.all(g[:2 * H] == 0)          # no gradient flows through w2 == 0


def test_loss_single_hinge_closed_form():
    """One live unit relu(x - 0.5) with w2 = 1: y = max(x - 0.5, 0)."""
    x = np.linspace(0, 1, 101, dtype=np.float32)
    t = np.zeros_like(x)
    w1 = np.zeros(H); b1 = np.full(H, -1.0); w2 = np.zeros(H)
    w1[5], b1[5], w2[5] = 1.0, -0.5, 1.0
    p = _params(w1, b1, w2, 0.0)
    loss, g = oracle.mlp_loss_grad(p, x, t)
    y = np.maximum(x.astype(np.float64) - 0.5, 0)
    assert loss == pytest.approx(np.mean(y**2), rel=1e-12)
    assert oracle.mlp_forward(p, x) == pytest.approx(y, abs=1e-15)
    # d/db1 of mean(y^2) = mean(2 y * 1[z>0])
    assert g[H + 5] == pytest.approx(np.mean(2 * y), rel=1e-12)
    assert g[H + 4] == 0.0 and g[4] == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_central_differences(seed):
    rng = np.random.default_rng(seed)
    n = 400
    x = np.sort(rng.random(n)).astype(np.float32)
    t = np.sort(rng.random(n)).astype(np.float32)
    p = _params(rng.normal(1, 0.3, H), -rng.random(H), rng.normal(0, 0.1, H), 0.05)
    _, g = oracle.mlp_loss_grad(p, x, t)
    h = 2.0**-12
    for j in list(rng.choice(3 * H + 1, 40, replace=False)) + [3 * H, 2 * H + 3]:
        pp, pm = p.copy(), p.copy()
        pp[j] += np.float32(h)
        pm[j] -= np.float32(h)
        hh = (float(pp[j]) - float(pm[j])) / 2
        lp, _ = oracle.mlp_loss_grad(pp, x, t)
        lm, _ = oracle.mlp_loss_grad(pm, x, t)
        fd = (lp - lm) / (2 * hh)
        if j >= 2 * H:        # loss is exactly quadratic in w2, b2: central difference exact
            assert fd == pytest.approx(g[j], rel=1e-7, abs=1e-12)
        else:                 # hinge kinks: at most a few samples change side within +-h
            assert abs(fd - g[j]) <= 1e-3 * max(1.0, abs(g[j])) + 4 * abs(p[2 * H + j % H]) / n


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    p = rng.normal(size=3 * H + 1).astype(np.float32)
    g = rng.normal(size=3 * H + 1).astype(np.float32)
    g[7] = 0.0
    p0 = p.copy()
    m = np.zeros_like(p); v = np.zeros_like(p)
    oracle.adam_step(p, m, v, g, 1, lr=1e-2)
    step = p0.astype(np.float64) - p.astype(np.float64)
    expect = 1e-2 * np.sign(g.astype(np.float64))
    assert np.allclose(step, expect, atol=2e-7 * np.maximum(1, np.abs(p0)) + 1e-9)
    assert p[7] == p0[7]
    assert np.allclose(m, 0.1 * g, rtol=1e-6) and np.allclose(v, 0.001 * g.astype(np.float64)**2, rtol=1e-5)


def test_splitters_exact_quantiles():
    """Model == empirical mid-CDF on distinct keys: s_j is the key at ceil(j n / P - 1/2)."""
    n, P = 1000, 8
    keys = np.arange(n, dtype=np.int64) * 3 + 11
    y = (2 * np.arange(n) + 1) / (2 * n)
    s = oracle.splitters_from_cdf(keys, y, P)
    expect = [keys[math.ceil(j * n / P - 0.5)] for j in range(1, P)]
    assert s.tolist() == expect


def test_splitters_isolate_heavy_key_and_envelope():
    """A key holding half of the sample crosses several quantiles: it becomes a singleton
    partition [k, k+1).  A non-monotone model is read through its running maximum."""
    keys = np.sort(np.concatenate([np.arange(100), np.full(200, 500), np.arange(1000, 1100)])).astype(np.int64)
    t = oracle.cdf_targets(keys).astype(np.float64)
    s = oracle.splitters_from_cdf(keys, t, 8)
    assert 500 in s.tolist() and 501 in s.tolist()
    ids = oracle.part_ids_range(keys, s)
    pid = ids[keys == 500][0]
    assert set(keys[ids == pid].tolist()) == {500}
    assert np.all(np.diff(s) > 0)
    y = t.copy()
    y[150] = 0.0          # a dip does not move splitters (running maximum)
    assert oracle.splitters_from_cdf(keys, y, 8).tolist() == s.tolist()
