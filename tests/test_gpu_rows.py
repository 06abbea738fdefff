"""GPU parity of the materialized join output (vx_probe_rows) against the oracle's join rows.

The GPU writes rows in no particular order; each test sorts them by probe row index and
compares every column exactly (integer work: bit-exact).
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

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


def _check(got_rows, got_b, got_p, n_out, bk, bps, pk, pps):
    erow, eb, ep = oracle.join_rows(bk, bps, pk, pps)
    assert n_out == len(erow)
    row = np.asarray(got_rows[:n_out], np.uint64)
    order = np.argsort(row, kind="stable")
    assert np.array_equal(row[order], erow)
    for g, e in zip(got_b, eb):
        assert np.array_equal(np.asarray(g[:n_out], np.int64)[order], e)
    for g, e in zip(got_p, ep):
        assert np.array_equal(np.asarray(g[:n_out], np.int64)[order], e)


def test_rows_device_resident_ragged(gpu, ctx):
    bkey, bpay, pkey = datagen.plain_join(20011, 300_007, seed=23)
    ppay = (np.arange(len(pkey), dtype=np.int64) * 13 - 5).astype(np.int32)
    t = ctx.build(dev(bkey), [dev(bpay)])
    _say("rows device-resident")
    agg, st, n_out, (row, bc, pc) = t.probe_rows(dev(pkey), [dev(ppay)])
    _check(row, bc, pc, n_out, bkey, [bpay], pkey, [ppay])
    assert agg == oracle.join_agg(bkey, [bpay], pkey, [ppay])
    t.destroy()


@pytest.mark.parametrize("late_mat", [-1, 0, 1])
def test_rows_streamed_host_probe(gpu, ctx, late_mat):
    nb, np_ = 1 << 15, 700_001
    bk, b0, b1 = datagen.stream_build(nb, seed=29)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=29, match_frac=0.2)
    t = ctx.build(pinned(gpu, bk), [pinned(gpu, b0), pinned(gpu, b1)])
    _say("rows streamed", late_mat)
    agg, st, n_out, (row, bc, pc) = t.probe_rows(pinned(gpu, pk), [pinned(gpu, p0), pinned(gpu, p1)],
                                                 late_mat=late_mat, chunk_rows=65_537)
    _check(row, bc, pc, n_out, bk, [b0, b1], pk, [p0, p1])
    assert agg == oracle.join_agg(bk, [b0, b1], pk, [p0, p1])
    assert st["chunks"] == (np_ + 65_536) // 65_537
    t.destroy()


def test_rows_to_device_memory_and_skipped_columns(gpu, ctx):
    import torch
    bkey, bpay, pkey = datagen.plain_join(5000, 80_000, seed=31)
    t = ctx.build(dev(bkey), [dev(bpay)])
    cap = 80_000
    row = torch.zeros(cap, dtype=torch.int64, device="cuda")
    bcol = torch.zeros(cap, dtype=torch.int64, device="cuda")
    _say("rows to device memory")
    agg, st, n_out, _ = t.probe_rows(dev(pkey), [], out=(row, [bcol], []))
    _check(row.cpu().numpy().view(np.uint64), [bcol.cpu().numpy()], [], n_out, bkey, [bpay], pkey, [])
    # a skipped build column: rows still written
    agg2, _, n2, _ = t.probe_rows(dev(pkey), [], out=(row, [None], []))
    assert n2 == n_out and agg2 == agg
    t.destroy()


def test_rows_edges(gpu, ctx):
    i64 = np.iinfo(np.int64)
    bk = np.array([i64.min, i64.max, 0, -1], np.int64)
    bp = np.array([10, 20, 30, 40], np.int64)
    pk = np.array([i64.max, 5, i64.min, -1, i64.min, 0], np.int64)
    pp = np.array([1, 2, 3, 4, 5, 6], np.int64)
    t = ctx.build(dev(bk), [dev(bp)])
    _say("rows edges")
    agg, st, n_out, (row, bc, pc) = t.probe_rows(dev(pk), [dev(pp)])
    _check(row, bc, pc, n_out, bk, [bp], pk, [pp])
    # no matches
    agg, st, n_out, _ = t.probe_rows(dev(np.array([7, 8, 9], np.int64)), [])
    assert n_out == 0 and agg == [0, 0]
    # capacity: 5 matches, room for 3
    with pytest.raises(gpu.VxError) as ei:
        t.probe_rows(dev(pk), [dev(pp)], cap=3)
    assert ei.value.status == gpu.VX_ECAPACITY and "n_out 5" in str(ei.value)
    t.destroy()
    tp = ctx.build(dev(bk), [dev(bp)], unique=False)
    with pytest.raises(gpu.VxError) as ei:
        tp.probe_rows(dev(pk), [])
    assert ei.value.status == gpu.VX_EUNSUPPORTED
    tp.destroy()


def test_rows_zero_copy_granules_counted(gpu):
    """zc_bytes of a zero-copy rows probe, counted by the kernels: 128 B (the granule before any
    calibration) times the granules that hold a matching row, in each of the two payload columns
    (one count stands for both, as they share width and offset), as in the aggregate-only probe.
    Page-aligned columns and chunks of a multiple of 64 rows keep each granule in one wave."""
    nb, np_ = 1 << 12, (1 << 18) + 77
    bk, b0, b1 = datagen.stream_build(nb, seed=5)
    pk, p0, p1 = datagen.stream_probe(nb, np_, seed=5)
    hosts = [pinned(gpu, a) for a in (pk, p0, p1)]
    _say("rows zero-copy granule count")
    try:
        with gpu.Context(1 << 30) as c:
            t = c.build(dev(bk), [dev(b0), dev(b1)])
            agg, st, n_out, (row, bc, pc) = t.probe_rows(hosts[0], hosts[1:], late_mat=gpu.VX_LATE_ZC,
                                                         chunk_rows=1 << 15, count_zc=True)
            _check(row, bc, pc, n_out, bk, [b0, b1], pk, [p0, p1])
            t.destroy()
        assert st["zc_mask"] == 3 and st["zc_counted"] == 1
        rows = np.nonzero(np.isin(pk, bk))[0]
        granules = len(np.unique(rows * 8 // 128))
        assert st["zc_bytes"] == 2 * 128 * granules
    finally:
        for h in hosts:
            h.free()
