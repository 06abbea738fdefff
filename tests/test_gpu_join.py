"""GPU parity of the plain / streamed join against the oracle, through the C ABI.

Every aggregate is an integer modulo 2^64, so the bar is bit-exact equality.
"""
import os

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

M64 = 1 << 64
GiB = 1 << 30


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(8 * GiB)
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


@pytest.mark.parametrize("hashed", [False, True])
@pytest.mark.parametrize("lanes", ["1", "4", "8"])
def test_plain_device_resident_ragged(gpu, ctx, lanes, hashed, monkeypatch):
    """The recipe's keys fill their range, so the build is laid out directly unless VX_HASHED."""
    monkeypatch.setenv("VX_BUILD_LANES", lanes)
    bkey, bpay, pkey = datagen.plain_join(10007, 300_001, seed=3)
    _say("plain ragged lanes", lanes, "hashed", hashed)
    got, st = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), hashed=hashed)
    assert got == oracle.join_agg(bkey, [bpay], pkey, [])


def test_plain_full_size_device_resident(gpu, ctx):
    """Plain in-memory join at full size: 2^20 unique int32 build keys, 2^24 probes."""
    bkey, bpay, pkey = datagen.plain_join()
    _say("plain full size")
    exp = oracle.join_agg(bkey, [bpay], pkey, [])
    for hashed in (False, True):
        got, st = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), hashed=hashed)
        assert got == exp
    assert 0.45 < got[0] / len(pkey) < 0.55


def test_edge_cases_empty_and_extremes(gpu, ctx):
    i64 = np.iinfo(np.int64)
    i32 = np.iinfo(np.int32)
    e = np.zeros(0, np.int64)
    k = np.arange(100, dtype=np.int64)
    _say("edge: empty")
    assert ctx.join_plain(dev(e), [dev(e)], dev(k))[0] == [0, 0]
    assert ctx.join_plain(dev(k), [dev(k)], dev(e))[0] == [0, 0]
    _say("edge: sentinel keys int64")
    bkey = np.array([i64.min, i64.max, 0, -1, 5], np.int64)
    bpay = np.array([11, 22, 33, 44, 55], np.int64)
    pkey = np.array([i64.min, i64.max, i64.max, 7, -1, i64.min, i64.min, 0], np.int64)
    ppay = np.array([1, 2, 3, 4, 5, 6, 7, 8], np.int64)
    exp = oracle.join_agg(bkey, [bpay], pkey, [ppay])
    assert ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)])[0] == exp
    _say("edge: sentinel keys int32")
    bk = np.array([i32.min, i32.max, 0], np.int32)
    bp = np.array([i32.min, i32.max, -7], np.int32)
    pk = np.array([i32.min, i32.min, i32.max, 3], np.int32)
    assert ctx.join_plain(dev(bk), [dev(bp)], dev(pk))[0] == oracle.join_agg(bk, [bp], pk, [])


def test_all_match_no_match(gpu, ctx):
    n = 50_000
    bkey = np.arange(n, dtype=np.int32)
    bpay = np.arange(n, dtype=np.int32) * 3 - 7
    allm = np.tile(bkey, 3)
    nom = np.arange(n, 2 * n, dtype=np.int32)
    _say("all/no match")
    assert ctx.join_plain(dev(bkey), [dev(bpay)], dev(allm))[0] == oracle.join_agg(bkey, [bpay], allm, [])
    assert ctx.join_plain(dev(bkey), [dev(bpay)], dev(nom))[0] == [0, 0]


def test_duplicate_in_unique_build_rejected(gpu, ctx):
    bkey = np.array([1, 2, 3, 2], np.int64)
    _say("dup key")
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_plain(dev(bkey), [], dev(bkey))
    assert ei.value.status == gpu.VX_EDUPKEY
    bkey = np.array([np.iinfo(np.int64).min] * 2, np.int64)      # duplicate sentinel key
    with pytest.raises(gpu.VxError):
        ctx.join_plain(dev(bkey), [], dev(bkey))


def test_preagg_duplicates_heavy(gpu, ctx):
    """Pre-aggregating table: a single key 10^6 times plus a Zipf tail, on both sides."""
    rng = np.random.default_rng(9)
    bkey = np.concatenate([np.full(1_000_000, 42), rng.zipf(1.2, 300_000)]).astype(np.int64)
    rng.shuffle(bkey)
    bpay = rng.integers(0, 1 << 32, len(bkey)).astype(np.int64)
    pkey = np.concatenate([np.full(1000, 42), rng.zipf(1.2, 200_000)]).astype(np.int64)
    ppay = rng.integers(-(1 << 40), 1 << 40, len(pkey)).astype(np.int64)
    _say("preagg heavy")
    got = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)], unique=False)[0]
    assert got == oracle.join_agg(bkey, [bpay], pkey, [ppay])


@pytest.mark.parametrize("late_mat", [0, 1, -1, 2])
@pytest.mark.parametrize("n_buffers", [2, 3])
def test_streamed_probe_modes(gpu, ctx, late_mat, n_buffers):
    """Host-resident probe side streamed in many chunks (ragged last chunk); every
    late-materialization mode and buffer count gives the same exact aggregates."""
    nb, np_ = 1 << 16, 1_000_003
    bk, b0, b1 = datagen.stream_build(nb, seed=5)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=5)
    hk, h0, h1 = pinned(gpu, pk), pinned(gpu, p0), pinned(gpu, p1)
    _say("streamed probe", late_mat, n_buffers)
    got, st = ctx.join_plain(pinned(gpu, bk), [pinned(gpu, b0), pinned(gpu, b1)], hk, [h0, h1],
                             late_mat=late_mat, chunk_rows=65_537, n_buffers=n_buffers)
    assert got == oracle.join_agg(bk, [b0, b1], pk, [p0, p1])
    assert st["chunks"] == (np_ + 65_536) // 65_537
    if late_mat == 1:
        assert st["zc_mask"] == 3 and st["sdma_bytes"] == np_ * 8
    if late_mat == 0:
        assert st["zc_mask"] == 0 and st["sdma_bytes"] == np_ * 24


def test_streamed_per_chunk_aggregates(gpu, ctx):
    nb, np_ = 5000, 200_000
    bk, b0, b1 = datagen.stream_build(nb, seed=8)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=8, match_frac=0.5)
    t = ctx.build(dev(bk), [dev(b0), dev(b1)])
    cr = 30_000
    _say("per-chunk aggregates")
    tot, st, per = t.probe(pinned(gpu, pk), [pinned(gpu, p0), pinned(gpu, p1)], chunk_rows=cr,
                           chunk_aggs=True, late_mat=1)
    pb = oracle.PreparedBuild(bk, [b0, b1])
    for c, row in enumerate(per):
        sl = slice(c * cr, (c + 1) * cr)
        assert row == pb.probe(pk[sl], [p0[sl], p1[sl]])
    assert [sum(x) % M64 for x in zip(*per)] == tot
    t.destroy()


def test_budget_and_pinning_errors(gpu):
    c = gpu.Context(4 << 20)      # 4 MiB budget: table of 2^20 rows cannot fit
    bkey, bpay, pkey = datagen.plain_join(1 << 20, 1 << 10, seed=1)
    _say("budget error")
    with pytest.raises(gpu.VxError) as ei:
        c.join_plain(dev(bkey), [dev(bpay)], dev(pkey))
    assert ei.value.status == gpu.VX_EBUDGET
    # the context stays usable after the failure
    assert c.join_plain(dev(bkey[:1000]), [dev(bpay[:1000])], dev(pkey))[0] == \
        oracle.join_agg(bkey[:1000], [bpay[:1000]], pkey, [])
    _say("pageable host memory rejected")
    with pytest.raises(gpu.VxError) as ei:
        c.join_plain(dev(bkey[:10]), [], np.ascontiguousarray(pkey))
    assert ei.value.status == gpu.VX_ENOTPINNED
    c.close()


def test_streamed_budget_forces_smaller_chunks(gpu):
    """A budget that holds the table but not default-sized chunks: the executor shrinks chunks."""
    nb, np_ = 1 << 12, 3_000_000
    bk, b0, b1 = datagen.stream_build(nb, seed=12)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=12)
    c = gpu.Context(6 << 20)
    _say("budget-limited chunks")
    got, st = c.join_plain(dev(bk), [dev(b0), dev(b1)], pinned(gpu, pk), [pinned(gpu, p0), pinned(gpu, p1)],
                           late_mat=0)
    assert got == oracle.join_agg(bk, [b0, b1], pk, [p0, p1])
    assert st["chunk_rows"] * 24 * 2 < (6 << 20)
    c.close()


def test_calibration_properties(gpu, ctx):
    """vx_calibrate: link rates are positive and bounded by PCIe 5.0 x16, the zero-copy granule is a
    power of two between 8 and 2048 bytes, and device memory reads faster than the link."""
    _say("calibration")
    c = ctx.calibrate(256 << 20)
    assert 5 < c["h2d_gbs"] < 64 and 5 < c["zc_read_gbs"] < 64
    g = c["zc_granule"]
    assert 8 <= g <= 2048 and g & (g - 1) == 0
    assert c["hbm_read_gbs"] > 4 * c["h2d_gbs"]
    assert 5 < c["d2h_gbs"] < 64 and 0 < c["zc_write_gbs"] < 64
    assert 5 < c["duplex_sdma_gbs"] < 128 and 5 < c["duplex_zcw_gbs"] < 128 and 5 < c["duplex_zcr_gbs"] < 128


@pytest.mark.parametrize("pdt", [np.int64, np.int32])
def test_zero_copy_granules_counted(gpu, pdt):
    """zc_bytes of a zero-copy probe is 128 B (the granule before any calibration) times the
    granules that hold a matching row, counted in each payload column.  The columns are
    page-aligned and the chunks a multiple of 64 rows, so no granule is split between two waves
    and the count equals the distinct granules of the matching rows, computed here from the keys."""
    nb, np_ = 1 << 12, (1 << 18) + 77
    bk, b0, b1 = datagen.stream_build(nb, seed=5)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=5)
    p0, p1 = p0.astype(pdt), p1.astype(pdt)
    hosts = [pinned(gpu, a) for a in (pk, p0, p1)]
    _say("zero-copy granule count", np.dtype(pdt).name)
    try:
        with gpu.Context(1 << 30) as c:
            got, st = c.join_plain(dev(bk), [dev(b0), dev(b1)], hosts[0], hosts[1:], late_mat=gpu.VX_LATE_ZC,
                                   chunk_rows=1 << 15, count_zc=True)
            got2, st2 = c.join_plain(dev(bk), [dev(b0), dev(b1)], hosts[0], hosts[1:], late_mat=gpu.VX_LATE_ZC,
                                     chunk_rows=1 << 15)
        assert got == oracle.join_agg(bk, [b0, b1], pk, [p0, p1]) and got2 == got
        assert st["zc_mask"] == 3 and st["zc_counted"] == 1 and st2["zc_counted"] == 0
        rows = np.nonzero(np.isin(pk, bk))[0]          # unique build keys: a row matches iff its key is built
        granules = len(np.unique(rows * np.dtype(pdt).itemsize // 128))
        assert 0.05 < len(rows) / np_ < 0.15
        assert st["zc_bytes"] == 2 * 128 * granules
        # without the count, the wire model's estimate: within 2% of the count at this size
        assert abs(st2["zc_bytes"] - st["zc_bytes"]) < 0.02 * st["zc_bytes"]
    finally:
        for h in hosts:
            h.free()


def test_zero_copy_granules_unaligned_column(gpu):
    """A payload column that starts 3 elements into its allocation: a granule can then straddle two
    waves' rows, and each wave counts the granules of its own 64 rows (each wave's gather moves
    them).  Expected: per block of 64 rows (the waves' rows: chunks are a multiple of 64 rows),
    the distinct 128-byte granules of its matching rows, at their byte addresses."""
    nb, np_ = 1 << 12, (1 << 17) + 5
    bk, b0, b1 = datagen.stream_build(nb, seed=6)
    pk, p0, _ = datagen.stream_probe(nb, np_, seed=6)
    kh = pinned(gpu, pk)
    ph = gpu.HostBuffer(np_ + 3, np.int64)
    ph.array[3:] = p0
    _say("zero-copy granules, unaligned column")
    try:
        with gpu.Context(1 << 30) as c:
            got, st = c.join_plain(dev(bk), [dev(b0)], kh, [ph.array[3:]], late_mat=gpu.VX_LATE_ZC,
                                   chunk_rows=1 << 14, count_zc=True)
        assert got == oracle.join_agg(bk, [b0], pk, [p0])
        rows = np.nonzero(np.isin(pk, bk))[0]
        addr = (3 + rows) * 8                       # byte offset from the allocation (page-aligned)
        per_wave = np.unique(np.stack([rows // 64, addr // 128]), axis=1).shape[1]
        assert per_wave > len(np.unique(addr // 128))     # some granules straddle two waves
        assert st["zc_bytes"] == 128 * per_wave
    finally:
        kh.free()
        ph.free()
