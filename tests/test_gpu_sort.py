"""GPU parity of the out-of-core sort (Sec. 6.1) against the oracle, through the C ABI.

The sorted column must equal the oracle's sorted order element by element, for single and
many runs (pass 2 regroup + merge tree, ragged last run), int64 and int32 keys, pinned host
and device columns, and the degenerate inputs (empty, one key, all equal, already sorted,
reversed, the extreme values).
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

GiB, MiB = 1 << 30, 1 << 20


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(2 * GiB)
    yield c
    c.close()


def pinned(vx, a):
    hb = vx.HostBuffer(len(a), a.dtype)
    hb.array[:] = a
    return hb


def _say(*a):
    print(*a, flush=True)


def _keys(n, dtype, seed):
    rng = np.random.default_rng(seed)
    info = np.iinfo(dtype)
    k = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    if n > 100:
        k[:4] = [info.min, info.max, 0, -1]
        k[10:n // 10] = k[10]                   # a long run of one value
    return k


@pytest.mark.parametrize("n,chunk", [(100_003, 0), (1_000_003, 65_536), (50_000, 1024), (300_001, 100_000),
                                     (5_000_003, 0)])
def test_sort_host_int64(gpu, ctx, n, chunk):
    """One run, 16 runs with a ragged last one, 49 runs (a deep merge tree), 4 runs, and one run of
    611 digit tiles (the column scan's blocks hold 5 tiles each, the last one a single tile)."""
    k = _keys(n, np.int64, n)
    want = oracle.sort(k)
    h = pinned(gpu, k)
    _say("sort int64 host", n, chunk)
    st = ctx.sort(h, chunk_rows=chunk)
    assert np.array_equal(h.array, want)
    assert st["chunks"] == (1 if chunk == 0 else -(-n // chunk))
    assert st["rows"] == n


@pytest.mark.parametrize("n,chunk", [(777_777, 100_000), (5000, 0)])
def test_sort_int32_heavy_duplicates(gpu, ctx, n, chunk):
    rng = np.random.default_rng(3)
    k = rng.integers(-50, 50, n).astype(np.int32)
    k[::101] = np.iinfo(np.int32).min
    k[::103] = np.iinfo(np.int32).max
    want = oracle.sort(k).astype(np.int32)
    h = pinned(gpu, k)
    _say("sort int32", n, chunk)
    ctx.sort(h, chunk_rows=chunk)
    assert np.array_equal(h.array, want)


@pytest.mark.parametrize("n,chunk", [(300_001, 65_536), (3 * 8192 + 1, 0), (8192, 0)])
def test_sort_int32_full_range(gpu, ctx, n, chunk):
    """int32 keys over the whole range: every digit value in each of the 4 digit passes, the sign
    digit last; runs of whole 8192-key tiles plus a ragged tile, one key past a tile, and one
    exact tile."""
    rng = np.random.default_rng(11)
    k = rng.integers(np.iinfo(np.int32).min, np.iinfo(np.int32).max, n, dtype=np.int64, endpoint=True)
    k = k.astype(np.int32)
    want = oracle.sort(k).astype(np.int32)
    h = pinned(gpu, k)
    _say("sort int32 full range", n, chunk)
    ctx.sort(h, chunk_rows=chunk)
    assert np.array_equal(h.array, want)


def test_sort_device_column_many_runs(gpu, ctx):
    import torch
    k = _keys(400_000, np.int64, 5)
    want = oracle.sort(k)
    t = torch.from_numpy(k.copy()).cuda()
    _say("sort device column")
    st = ctx.sort(t, chunk_rows=30_000)
    assert st["chunks"] == 14
    assert np.array_equal(t.cpu().numpy(), want)


@pytest.mark.parametrize("case", ["empty", "one", "two", "equal", "sorted", "reversed", "extremes"])
def test_sort_degenerate(gpu, ctx, case):
    i64 = np.iinfo(np.int64)
    k = {"empty": np.zeros(0, np.int64), "one": np.array([7], np.int64), "two": np.array([5, -5], np.int64),
         "equal": np.full(70_001, 42, np.int64), "sorted": np.arange(-35_000, 35_001, dtype=np.int64),
         "reversed": np.arange(35_000, -35_001, -1, dtype=np.int64),
         "extremes": np.tile(np.array([i64.max, i64.min, 0, -1, 1], np.int64), 20_000)}[case]
    want = oracle.sort(k)
    if len(k) == 0:
        ctx.sort(np.zeros(0, np.int64))
        return
    h = pinned(gpu, k)
    ctx.sort(h, chunk_rows=8192)
    assert np.array_equal(h.array, want)


def test_sort_small_budget_auto_runs(gpu):
    """The automatic run length under a small budget: several runs, still exact."""
    k = datagen.sort_keys(3_000_000)
    want = oracle.sort(k)
    c = gpu.Context(64 * MiB)
    try:
        h = pinned(gpu, k)
        _say("sort small budget")
        st = c.sort(h)
        assert st["chunks"] > 1
        assert np.array_equal(h.array, want)
    finally:
        c.close()


def test_sort_errors(gpu, ctx):
    bad = gpu.Col(None, 3, 0)
    d = gpu.SortDesc(bad, 10, 0, 0, 0)
    st = gpu.Stats()
    assert gpu.lib().vx_sort(ctx.h, d, st) == gpu.VX_EINVAL
    with pytest.raises(gpu.VxError) as e:
        ctx.sort(np.arange(1000, dtype=np.int64))     # pageable memory
    assert e.value.status == gpu.VX_ENOTPINNED
