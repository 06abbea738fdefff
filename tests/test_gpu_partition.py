"""GPU parity of partitioning and of the CDF-model kernels against the oracle, via the C ABI.

Partition ids, histograms, boundary arrays and the stable scatter are integer results and
must match exactly.  The network's FP32 outputs are compared with the oracle's double-precision
forward pass within a derived rounding bound.  Splitters are integers chosen from model values:
the oracle's rule runs on the oracle's own forward values, and the GPU's splitters must equal
its result wherever no model value lies within that bound of a quantile j/P at a crossing.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

GiB = 1 << 30
F01 = float(np.float32(0.01))   # the sampling fraction as the library stores it (FP32)


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(4 * GiB)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def pinned(vx, a):
    hb = vx.HostBuffer(len(a), a.dtype)
    hb.array[:] = a
    return hb


def _say(*a):
    print(*a, flush=True)


def _keys(n, seed=0):
    rng = np.random.default_rng(seed)
    k = np.concatenate([rng.zipf(1.3, n // 2), rng.integers(-2**62, 2**62, n - n // 2)]).astype(np.int64)
    rng.shuffle(k)
    return k


def _expect(ids, P, key, pays):
    order, b = oracle.cluster_boundary(ids, P)
    return oracle.histogram(ids, P), b, key[order.astype(np.int64)], [p[order.astype(np.int64)] for p in pays]


def _torch_empty_like(a):
    import torch
    return torch.empty(len(a), dtype=torch.int64 if a.dtype == np.int64 else torch.int32, device="cuda")


@pytest.mark.parametrize("P", [1, 2, 16, 1024])
def test_radix_hash_device_scatter(gpu, ctx, P):
    key = _keys(300_007, 1)
    pay = [np.arange(len(key), dtype=np.int64) * 7, (np.arange(len(key)) % 1000).astype(np.int32)]
    ok, op = _torch_empty_like(key), [_torch_empty_like(p) for p in pay]
    _say("radix hash device", P)
    r = ctx.partition(dev(key), [dev(p) for p in pay], method="radix_hash", n_parts=P, out_key=ok, out_pays=op)
    log2p = (P - 1).bit_length()
    h, b, ck, cp = _expect(oracle.part_ids_hash(key, log2p), P, key, pay)
    assert r["n_parts"] == P and np.array_equal(r["hist"], h) and np.array_equal(r["boundary"], b)
    assert np.array_equal(ok.cpu().numpy(), ck)
    for o, e in zip(op, cp):
        assert np.array_equal(o.cpu().numpy(), e)


def test_radix_bits_host_streamed_scatter(gpu, ctx, monkeypatch):
    """Host-resident input in many chunks, written to host memory by zero-copy stores."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 40_000))
    key = _keys(1_000_003, 2)
    pay = [np.arange(len(key), dtype=np.int64)]
    hk, hp = pinned(gpu, key), [pinned(gpu, p) for p in pay]
    ok, op = gpu.HostBuffer(len(key), np.int64), [gpu.HostBuffer(len(key), np.int64)]
    _say("radix bits host streamed")
    r = ctx.partition(hk, hp, method="radix_bits", n_parts=64, shift=3, out_key=ok, out_pays=op)
    h, b, ck, cp = _expect(oracle.part_ids_bits(key, 3, 6), 64, key, pay)
    assert np.array_equal(r["hist"], h) and np.array_equal(r["boundary"], b)
    assert np.array_equal(ok.array, ck) and np.array_equal(op[0].array, cp[0])


def test_range_given_splitters_and_hist_only(gpu, ctx):
    key = _keys(200_000, 3)
    spl = np.array([-2**61, -5, 0, 1, 2, 3, 10, 1000, 2**40], np.int64)
    _say("range given")
    r = ctx.partition(dev(key), method="range", splitters=spl)
    ids = oracle.part_ids_range(key, spl)
    assert r["n_parts"] == len(spl) + 1
    assert np.array_equal(r["hist"], oracle.histogram(ids, len(spl) + 1))
    assert np.array_equal(r["boundary"], oracle.cluster_boundary(ids, len(spl) + 1)[1])
    with pytest.raises(gpu.VxError):
        ctx.partition(dev(key), method="range", splitters=spl[::-1].copy())


def test_partition_edges(gpu, ctx):
    _say("partition edges")
    e = np.zeros(0, np.int64)
    r = ctx.partition(dev(np.zeros(1, np.int64))[:0], method="radix_hash", n_parts=8)
    assert r["hist"].sum() == 0 and r["boundary"].tolist() == [0] * 9
    same = np.full(5000, 42, np.int64)
    r = ctx.partition(dev(same), method="radix_hash", n_parts=8)
    assert sorted(r["hist"].tolist()) == [0] * 7 + [5000]
    assert r["imbalance"] == 8.0
    del e


def test_quantile_splitters_exact(gpu, ctx):
    """Sample (SplitMix64 Bernoulli), GPU radix sort, mid-CDF targets, splitter rule:
    identical to the oracle's sample, sort, targets and rule."""
    rng = np.random.default_rng(4)
    key = np.concatenate([rng.zipf(1.1, 1_500_000), rng.integers(1, 2**40, 500_000)]).astype(np.int64)
    rng.shuffle(key)
    seed, P = 12345, 64
    _say("quantile splitters")
    r = ctx.partition(pinned(gpu, key), method="quantile", n_parts=P, seed=seed, sample_frac=0.01)
    s = np.sort(oracle.sample_bernoulli(key, seed, F01))
    t = oracle.cdf_targets(s).astype(np.float64)
    exp = oracle.splitters_from_cdf(s, t, P)
    assert np.array_equal(r["splitters"], exp)
    ids = oracle.part_ids_range(key, exp)
    assert np.array_equal(r["hist"], oracle.histogram(ids, len(exp) + 1))
    # the heavy key 1 (about 30% of rows) carries several quantiles: a singleton partition
    assert 1 in exp.tolist() and 2 in exp.tolist()


def _fwd_bound(params, x):
    """Rounding bound for the GPU's FP32 network value (mlp_eval: y = b2, then for each hidden unit
    in order z = fma(w1, x, b1) and, if z > 0, y = fma(w2, z, y)).

    Both sides agree on which units are active: fma rounds the exact w1 x + b1 once and the oracle
    forms w1 x exactly in double before adding b1, and rounding keeps the sign.  With u = 2^-24,
    each of the m + 1 terms (b2 and w2_j z_j over the m active units) passes through at most m + 1
    roundings (its own z, then the fma chain), so |y_gpu - y| <= gamma_{m+1} (|b2| + sum |w2_j z_j|),
    gamma_k = k u / (1 - k u).  gamma_66 (m <= 64) also covers the oracle's double rounding."""
    H = 64
    u = 2.0**-24
    w1, b1, w2 = (params[:H].astype(np.float64), params[H:2 * H].astype(np.float64),
                  params[2 * H:3 * H].astype(np.float64))
    z = x.astype(np.float64)[:, None] * w1 + b1
    S = abs(float(params[3 * H])) + (np.abs(w2 * z) * (z > 0)).sum(1)
    g = 66 * u / (1 - 66 * u)
    return g * S


def _crossings(y, P):
    """For each quantile j/P (j = 1..P-1): the first index where the running maximum reaches it."""
    env = np.maximum.accumulate(y)
    return np.searchsorted(env, np.arange(1, P) / P, side="left")


@pytest.mark.parametrize("seed", [0, 1])
def test_cdf_forward_parity(gpu, ctx, seed):
    """vx_cdf_forward (the evaluation that also places the splitters) against the oracle's forward
    pass, element by element within the derived FP32 bound: random parameters over [0, 1), and the
    initial knots on the features of a Zipf sample."""
    rng = np.random.default_rng(seed)
    n = 200_000
    x = rng.random(n).astype(np.float32)
    x[:3] = [0.0, 1.0 - 2**-24, 0.5]
    p = np.concatenate([rng.normal(1, 0.5, 64), -rng.random(64), rng.normal(0, 0.1, 64), [0.02]]).astype(np.float32)
    s = np.sort(rng.zipf(1.2, 50_000)).astype(np.int64)
    xz = oracle.cdf_feature(s, s[0], oracle.feature_scale(s[0], s[-1]))
    p0 = np.concatenate([np.ones(64), -np.arange(64) / 64, np.full(64, 1 / 64), [0]]).astype(np.float32)
    _say("cdf forward parity", seed)
    for xs, ps in ((x, p), (xz, p0)):
        y_g = ctx.cdf_forward(dev(xs), ps).astype(np.float64)
        y_o = oracle.mlp_forward(ps, xs)
        b = _fwd_bound(ps, xs)
        err = np.abs(y_g - y_o)
        assert np.all(err <= b), float((err / np.maximum(b, 1e-300)).max())
        assert b.max() < 1e-4 * max(1.0, np.abs(y_o).max())        # the bound is not vacuous


def test_learned_splitters_exact(gpu, ctx):
    """Splitters of the GPU-trained model against the oracle's rule run on the oracle's own
    sample, features and forward values.  Where no model value lies within the forward bound of a
    quantile at its crossing, the GPU's splitters must equal the oracle's exactly.  At a quantile
    that is that close, either side of it is a correct reading, so the GPU's splitters must then
    equal the rule applied to its own forward values, which are checked against the oracle's
    within the bound, and every splitter that no such quantile can move must still be there."""
    rng = np.random.default_rng(5)
    key = np.concatenate([rng.zipf(1.1, 800_000), rng.integers(1, 2**40, 200_000)]).astype(np.int64)
    seed, P = 777, 32
    _say("learned splitters")
    r = ctx.partition(dev(key), method="learned", n_parts=P, seed=seed, sample_frac=0.01, train_steps=60)
    model = r["model"]
    s = np.sort(oracle.sample_bernoulli(key, seed, F01))
    x = oracle.cdf_feature(s, s[0], oracle.feature_scale(s[0], s[-1]))
    y_o = oracle.mlp_forward(model, x)
    b = _fwd_bound(model, x)
    exp = oracle.splitters_from_cdf(s, y_o, P)
    y_g = ctx.cdf_forward(dev(x), model).astype(np.float64)
    assert np.all(np.abs(y_g - y_o) <= b)
    lo, hi = _crossings(y_o + b, P), _crossings(y_o - b, P)
    n = len(s)
    near = [j for j in range(P - 1) if s[min(lo[j], n - 1)] != s[min(hi[j], n - 1)] or (lo[j] < n) != (hi[j] < n)]
    print("quantiles within the forward bound at their crossing:", len(near), "of", P - 1, flush=True)
    got = r["splitters"]
    if not near:
        assert np.array_equal(got, exp)
    else:
        assert np.array_equal(got, oracle.splitters_from_cdf(s, y_g, P))
        moved = set()
        for j in near:
            moved |= {int(s[i]) for i in range(lo[j], min(hi[j] + 1, n))}
        moved |= {k + 1 for k in moved}
        assert {int(k) for k in exp} - moved <= {int(k) for k in got}
    assert r["final_loss"] > 0 and np.isfinite(r["final_loss"])
    assert np.array_equal(r["hist"], oracle.histogram(oracle.part_ids_range(key, got), len(got) + 1))


def _grad_bound(params, x, t):
    """Rounding bound for the GPU gradient, per component.

    The GPU evaluates z = fma(w1, x, b1) (one rounding: |dz| <= u |z|), h = relu(z),
    p = w2 * h (one rounding) and y = b2 + (butterfly sum of 64 p's: 6 roundings) in FP32,
    u = 2^-24, so |dy_i| <= 7u (|b2| + sum_j |w2_j h_ij|) + 2u sum_j |w2_j h_ij|.  The activation
    pattern is the same on both sides: fma rounds the exact w1 x + b1 once, the oracle forms the
    exact product w1 x in double before adding b1, and rounding keeps the sign.
    Every gradient term is (2/n) e_i a_ic with a_ic in {w2_j x_i [z>0], w2_j [z>0], h_ij, 1};
    the FP64 accumulation adds nothing visible and the result is rounded to FP32 (u |g|).
    Hence |dg_c| <= (2/n) sum_i (|dy_i| |a_ic| + |e_i| 2u |a_ic|) + u |g_c|."""
    H = 64
    u = 2.0**-24
    w1, b1, w2, b2 = (params[:H].astype(np.float64), params[H:2 * H].astype(np.float64),
                      params[2 * H:3 * H].astype(np.float64), float(params[3 * H]))
    xd = x.astype(np.float64)[:, None]
    z = xd * w1 + b1
    h = np.maximum(z, 0)
    S = np.abs(b2) + np.abs(w2 * h).sum(1)
    y = b2 + (w2 * h).sum(1)
    e = np.abs(y - t.astype(np.float64))
    dy = 7 * u * S + 2 * u * np.abs(w2 * h).sum(1)
    n = len(x)
    act = (z > 0).astype(np.float64)
    a_w1 = np.abs(w2) * np.abs(xd) * act
    a_b1 = np.abs(w2) * act
    a_w2 = h

    def term(a):
        return (2 / n) * ((dy[:, None] * a).sum(0) + (e[:, None] * (2 * u * a)).sum(0))

    return np.concatenate([term(a_w1), term(a_b1), term(a_w2), [(2 / n) * dy.sum()]])


@pytest.mark.parametrize("seed", [0, 1])
def test_cdf_gradient_parity(gpu, ctx, seed):
    import torch
    rng = np.random.default_rng(seed)
    n = 50_000
    x = np.sort(rng.random(n)).astype(np.float32)
    t = ((np.arange(n) + 0.5) / n).astype(np.float32)
    p = np.concatenate([rng.normal(1, 0.3, 64), -rng.random(64), rng.normal(0, 0.05, 64), [0.01]]).astype(np.float32)
    _say("cdf gradient parity", seed)
    loss_g, g_g = ctx.cdf_loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), p)
    loss_o, g_o = oracle.mlp_loss_grad(p, x, t)
    bound = _grad_bound(p, x, t)
    u = 2.0**-24
    err = np.abs(g_g.astype(np.float64) - g_o)
    assert np.all(err <= bound + u * np.abs(g_o) + 1e-30), (err / (bound + 1e-30)).max()
    assert abs(loss_g - loss_o) <= 1e-6 * loss_o


def test_cdf_train_deterministic_and_descends(gpu, ctx):
    import torch
    rng = np.random.default_rng(3)
    s = np.sort(rng.zipf(1.2, 100_000)).astype(np.int64)
    x = oracle.cdf_feature(s, s[0], oracle.feature_scale(s[0], s[-1]))
    t = oracle.cdf_targets(s)
    H = 64
    p0 = np.concatenate([np.ones(H), -np.arange(H) / H, np.full(H, 1 / H), [0]]).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    _say("cdf train")
    p1, l1 = ctx.cdf_train(xd, td, p0, 100)
    p2, l2 = ctx.cdf_train(xd, td, p0, 100)
    assert np.array_equal(p1, p2) and l1 == l2
    l0, _ = oracle.mlp_loss_grad(p0, x, t)
    assert l1 < 0.5 * l0
    # one step against the oracle's Adam step from the oracle's gradient
    q, _ = ctx.cdf_train(xd, td, p0, 1)
    _, g = oracle.mlp_loss_grad(p0, x, t)
    qo, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    oracle.adam_step(qo, m, v, g.astype(np.float32), 1)
    big = np.abs(g) > 1e-3 * np.abs(g).max()     # sign of tiny components is rounding-dependent
    assert np.allclose(q[big], qo[big], rtol=0, atol=1e-6)


def _oracle_train(p0, x, t, steps, lr=1e-2, flip=None):
    """The oracle's trajectory: full-batch Adam from p0 with the trainer's cosine learning rate,
    each step from the oracle's gradient rounded to FP32.  flip (a numpy Generator): every
    gradient component moved one FP32 ulp up or down at random, to measure how far rounding
    alone carries the trajectory."""
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k in range(1, steps + 1):
        _, g = oracle.mlp_loss_grad(p, x, t)
        g = g.astype(np.float32)
        if flip is not None:
            g = np.nextafter(g, np.where(flip.random(len(g)) < 0.5, -np.inf, np.inf).astype(np.float32))
        oracle.adam_step(p, m, v, g, k, lr=lr * (1 + np.cos(np.pi * (k - 1) / steps)) / 2)
    return p, oracle.mlp_loss_grad(p, x, t)[0]


def test_cdf_train_trajectory_parity(gpu, ctx):
    """50 training steps on the GPU against the oracle's 50 steps from the same start (its gradient
    and its Adam step, both pinned on their own): the final loss and the model's outputs on the
    training points agree within 100 times what a one-ulp change of every gradient component does
    to the oracle's own trajectory (about 1e-7 here), and never closer than 1e-5 is required."""
    import torch
    rng = np.random.default_rng(3)
    s = np.sort(rng.zipf(1.2, 100_000)).astype(np.int64)
    x = oracle.cdf_feature(s, s[0], oracle.feature_scale(s[0], s[-1]))
    t = oracle.cdf_targets(s)
    H, steps = 64, 50
    p0 = np.concatenate([np.ones(H), -np.arange(H) / H, np.full(H, 1 / H), [0]]).astype(np.float32)
    po, lo = _oracle_train(p0, x, t, steps)
    pf, lf = _oracle_train(p0, x, t, steps, flip=np.random.default_rng(1))
    yo, yf = oracle.mlp_forward(po, x), oracle.mlp_forward(pf, x)
    tol_y = max(1e-5, 100 * float(np.abs(yo - yf).max()))
    tol_l = max(1e-5, 100 * abs(lo - lf) / lo)
    _say("cdf train trajectory", steps, "tolerances", tol_y, tol_l)
    pg, lg = ctx.cdf_train(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), p0, steps)
    assert lo < 0.5 * oracle.mlp_loss_grad(p0, x, t)[0]            # the oracle's run does train
    assert abs(lg - lo) <= tol_l * lo, (lg, lo)
    yg = oracle.mlp_forward(pg, x)
    assert float(np.abs(yg - yo).max()) <= tol_y, float(np.abs(yg - yo).max())


def test_auto_method_reports_estimates(gpu, ctx):
    rng = np.random.default_rng(8)
    key = rng.zipf(1.1, 2_000_000).astype(np.int64)
    _say("auto method")
    r = ctx.partition(dev(key), method="auto", n_parts=64, seed=5, train_steps=40)
    assert r["est_imbalance_radix"] > 1.0 and r["est_imbalance_range"] > 0
    # AUTO picks among radix-hash, the trained model's splitters and the sample quantiles (these
    # when their singletons hold clearly more of the sample, as after only 40 training steps)
    assert r["method_used"] in (gpu.VX_PART_RADIX_HASH, gpu.VX_PART_LEARNED, gpu.VX_PART_QUANTILE)
    assert r["hist"].sum() == len(key)


def _largest_table_partition(r):
    """Rows of the largest partition that has to be joined through a hash table: every partition
    except the singletons [s, s + 1), whose single key is resolved from its counts."""
    spl = np.asarray(r["splitters"], np.int64)
    hist = np.asarray(r["hist"], np.int64)
    single = np.zeros(len(hist), bool)
    if len(spl) > 1:
        single[1:len(spl)] = spl[1:] == spl[:-1] + 1
    return int(hist[~single].max()), int(hist[single].sum())


def test_trained_network_gain(gpu, ctx):
    """What training buys on Zipf(1.1) keys: the trained CDF network's splitters isolate the heavy
    keys and balance the rest, so its largest table-joined partition is several times smaller than
    with the same network untrained (initial weights) or with radix-hash partitioning, whose
    partition holding the heaviest key takes about a tenth of all rows.  The sample quantiles of the
    same sorted sample (no network) are the control for the network itself: on these keys the
    trained network only matches them, it does not beat them."""
    rng = np.random.default_rng(21)
    key = rng.zipf(1.1, 2_000_000).astype(np.int64)
    n, P = len(key), 64
    _say("trained network gain")
    got = {}
    for m in ("learned", "untrained", "quantile", "radix_hash"):
        r = ctx.partition(dev(key), method=m, n_parts=P, seed=3, sample_frac=0.02, train_steps=300)
        assert r["hist"].sum() == n
        got[m] = _largest_table_partition(r) if m != "radix_hash" else (int(r["hist"].max()), 0)
    mean = n / P
    print("largest table-joined partition / mean:", {m: round(v[0] / mean, 2) for m, v in got.items()},
          "singleton rows:", {m: v[1] for m, v in got.items()}, flush=True)
    assert got["learned"][1] > 0.1 * n               # heavy keys go to singleton partitions
    assert got["learned"][0] * 3 < got["untrained"][0]
    assert got["learned"][0] * 3 < got["radix_hash"][0]
    assert got["radix_hash"][0] > 0.09 * n
    # the network against the sample quantiles it was fit to: within 1.5x either way
    assert got["learned"][0] < 1.5 * got["quantile"][0] and got["quantile"][0] < 1.5 * got["learned"][0]


# ----------------------------------------------------------------------------- partitioned join

def _zipf_join(n_b, n_p, seed):
    rng = np.random.default_rng(seed)
    bk = rng.zipf(1.1, n_b).astype(np.int64)
    bp = rng.integers(0, 1 << 32, n_b).astype(np.int64)
    pk = rng.zipf(1.1, n_p).astype(np.int64)
    return bk, bp, pk


@pytest.mark.parametrize("method", ["radix_hash", "radix_bits", "learned", "quantile", "untrained", "auto"])
def test_partitioned_join_methods_exact(gpu, ctx, method, monkeypatch):
    """Every partitioner gives the oracle's exact aggregates (many chunks per side)."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 50_000))
    bk, bp, pk = _zipf_join(300_000, 1_000_001, 6)
    _say("partitioned join", method)
    got, st, used = ctx.join_partitioned(pinned(gpu, bk), [pinned(gpu, bp)], pinned(gpu, pk), method=method,
                                         n_parts=64, seed=9, train_steps=80)
    assert got == oracle.join_agg(bk, [bp], pk, [])
    if method in ("learned", "quantile"):
        assert st["singleton_rows"] > 0.1 * (len(bk) + len(pk))
    if method == "radix_hash":
        assert st["singleton_rows"] == 0 and st["n_parts"] == 64


@pytest.mark.parametrize("placement", ["0", "1"])
def test_partitioned_join_clustered_copy_placement(gpu, ctx, placement, monkeypatch):
    """The clustered build side in pinned host memory (read back by zero-copy) or in device
    memory gives the same exact aggregates and per-partition results."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 40_000))
    monkeypatch.setenv("VX_PJ_DEVICE", placement)
    bk, bp, pk = _zipf_join(250_000, 600_001, 13)
    _say("clustered copy placement", placement)
    got, st, used, per = ctx.join_partitioned(pinned(gpu, bk), [pinned(gpu, bp)], pinned(gpu, pk),
                                              method="learned", n_parts=32, seed=4, train_steps=60,
                                              per_partition=True)
    assert got == oracle.join_agg(bk, [bp], pk, [])
    assert [sum(x) % (1 << 64) for x in zip(*per)] == got
    assert (st["zc_bytes"] == 0) == (placement == "1")


@pytest.mark.parametrize("placement", ["0", "1"])
@pytest.mark.parametrize("method", ["learned", "radix_hash"])
def test_partitioned_join_int32_no_payload_one_partition(gpu, ctx, placement, method, monkeypatch):
    """int32 keys (with the empty-marker key), no build payload, and a single partition, on both
    placements of the clustered copy."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 30_000))
    monkeypatch.setenv("VX_PJ_DEVICE", placement)
    i32 = np.iinfo(np.int32)
    rng = np.random.default_rng(31)
    bk = rng.zipf(1.2, 200_000).astype(np.int32)
    pk = rng.zipf(1.2, 333_333).astype(np.int32)
    bk[::5000] = i32.min
    pk[::7000] = i32.min
    _say("partitioned int32", method, placement)
    got, st, used = ctx.join_partitioned(dev(bk), [], pinned(gpu, pk), method=method, n_parts=32, seed=2,
                                         train_steps=40)
    assert got == oracle.join_agg(bk, [], pk, [])
    got1 = ctx.join_partitioned(dev(bk), [], dev(pk), method=method, n_parts=1, seed=2, train_steps=20)[0]
    assert got1 == got


def test_partitioned_join_per_partition_radix(gpu, ctx):
    bk, bp, pk = _zipf_join(100_000, 300_000, 7)
    _say("partitioned per-partition")
    got, st, used, per = ctx.join_partitioned(dev(bk), [dev(bp)], dev(pk), method="radix_hash", n_parts=16,
                                              per_partition=True)
    ib, ip = oracle.part_ids_hash(bk, 4), oracle.part_ids_hash(pk, 4)
    for p in range(16):
        assert per[p] == oracle.join_agg(bk[ib == p], [bp[ib == p]], pk[ip == p], [])
    assert [sum(x) % (1 << 64) for x in zip(*per)] == got


def test_partitioned_join_edges(gpu, ctx):
    i64 = np.iinfo(np.int64)
    _say("partitioned edges")
    bk = np.array([i64.min, i64.min, 5, 5, 5, i64.max], np.int64)
    bp = np.array([1, 2, 3, 4, 5, 6], np.int64)
    pk = np.array([i64.min, 5, 5, i64.max, 7], np.int64)
    for m in ("radix_hash", "quantile"):
        got = ctx.join_partitioned(dev(bk), [dev(bp)], dev(pk), method=m, n_parts=4, sample_frac=1.0)[0]
        assert got == oracle.join_agg(bk, [bp], pk, [])
    e = np.zeros(0, np.int64)
    assert ctx.join_partitioned(dev(bk), [dev(bp)], dev(np.zeros(1, np.int64))[:0], method="radix_hash",
                                n_parts=4)[0] == [0, 0]
    same = np.full(10_000, 3, np.int64)
    got = ctx.join_partitioned(dev(same), [dev(same)], dev(same[:77]), method="learned", n_parts=8,
                               sample_frac=0.5, train_steps=10)[0]
    assert got == oracle.join_agg(same, [same], same[:77], [])
    del e


def test_partitioned_join_auto_on_scrambled_keys(gpu, ctx, monkeypatch):
    """Zipf keys scrambled by a bijection keep their heavy keys but lose the order that the learned
    model's log-scale feature relies on.  AUTO must still isolate the heavy keys (with the learned
    splitters, or else the sample quantiles) instead of falling back to radix-hash, and stay exact."""
    import datagen
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 50_000))
    bk, bp, pk = _zipf_join(300_000, 1_000_001, 31)
    datagen.scramble40(bk)
    datagen.scramble40(pk)
    _say("partitioned join auto, scrambled keys")
    got, st, used = ctx.join_partitioned(pinned(gpu, bk), [pinned(gpu, bp)], pinned(gpu, pk), method="auto",
                                         n_parts=64, seed=9, train_steps=80)
    assert got == oracle.join_agg(bk, [bp], pk, [])
    assert used in (gpu.VX_PART_LEARNED, gpu.VX_PART_QUANTILE)
    # the heaviest key alone holds about 9.5% of the rows; radix-hash would isolate none
    assert st["singleton_rows"] > 0.05 * (len(bk) + len(pk))
