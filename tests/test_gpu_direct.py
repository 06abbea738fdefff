"""GPU parity of direct-layout tables (key k in slot k - min) against the oracle and against the
hash layout of the same build (VX_HASHED), through the C ABI.

A build over device-resident keys whose range is no wider than the hash table's capacity is laid
out directly.  When the build is unique and its n keys are exactly the n values of their range
(no empty-marker key), the table is dense: payloads only, every key of the range present.
Results must not depend on the layout: every aggregate and every materialized row is compared
exactly.  Covered: dense and gapped ranges, the empty-marker key beside a range, ranges at the
ends of int32 and int64, probes below, inside and above the range, duplicates (rejected for
unique builds, also when they leave the row count equal to the range's width; aggregated for
pre-aggregating ones), dense tables without payloads and with mixed-width payloads, streamed
host probes, and the materialized rows.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

GiB = 1 << 30


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


def _slot_bytes(key_dtype, pay_dtypes):
    off = np.dtype(key_dtype).itemsize
    for p in pay_dtypes:
        s = np.dtype(p).itemsize
        off = (off + s - 1) // s * s + s
    b = 8
    while b < off:
        b *= 2
    return b


def _dense_bytes(n, pay_dtypes):
    """Dense table: n payload slots (the payloads packed, a power of two >= 4 bytes; none without
    payloads), n presence bytes, each 256-byte aligned, and the 256-byte side record."""
    off = 0
    for p in pay_dtypes:
        s = np.dtype(p).itemsize
        off = (off + s - 1) // s * s + s
    b = 4 if off else 0
    while b and b < off:
        b *= 2
    a256 = lambda v: (v + 255) // 256 * 256
    return a256(n * b) + a256(n) + 256


def _probes(rng, lo, n, m, dtype):
    """m probe keys: most inside [lo, lo + n), the rest just below or above it, clipped to the type."""
    info = np.iinfo(dtype)
    k = rng.integers(lo - n // 4, lo + n + n // 4, m, dtype=np.int64, endpoint=True)
    return np.clip(k, info.min, info.max).astype(dtype)


@pytest.mark.parametrize("lanes", ["1", "4", "8"])
@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_direct_dense_matches_hashed_and_oracle(gpu, ctx, lanes, dtype, monkeypatch):
    """2^16 keys filling [base, base + 2^16): the direct table has 2^16 slots, the hash table 2^17.
    The lane count applies to the hash build; a direct build always takes one lane per row."""
    monkeypatch.setenv("VX_BUILD_LANES", lanes)
    rng = np.random.default_rng(int(lanes) + np.dtype(dtype).itemsize)
    n, base = 1 << 16, -12_345
    bkey = (rng.permutation(n) + base).astype(dtype)
    bpay = rng.integers(-2**31, 2**31, n).astype(np.int32)
    pkey = _probes(rng, base, n, 300_001, dtype)
    ppay = rng.integers(-2**40, 2**40, len(pkey)).astype(np.int64)
    exp = oracle.join_agg(bkey, [bpay], pkey, [ppay])
    _say("direct dense", lanes, np.dtype(dtype).name)
    got_d, st_d = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)])
    got_h, st_h = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)], hashed=True)
    assert got_d == exp and got_h == exp
    sb = _slot_bytes(dtype, [np.int32])
    assert st_d["table_bytes"] == _dense_bytes(n, [np.int32])
    assert st_h["table_bytes"] == 2 * n * sb + 256


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_direct_gaps_and_empty_marker(gpu, ctx, dtype):
    """Keys with gaps (3000 of a 5000-wide range) plus the empty-marker key, which lives outside
    the slots; probes hit keys, gaps, both sides of the range and the marker."""
    info = np.iinfo(dtype)
    rng = np.random.default_rng(31)
    base = 1000
    bkey = np.concatenate([rng.permutation(5000)[:3000] + base, [info.min]]).astype(dtype)
    rng.shuffle(bkey)
    bp0 = rng.integers(-2**31, 2**31, len(bkey)).astype(np.int32)
    bp1 = rng.integers(-2**62, 2**62, len(bkey)).astype(np.int64)
    pkey = np.concatenate([_probes(rng, base, 5000, 50_000, dtype), np.full(17, info.min, dtype),
                           np.array([info.max, info.min + 1, 0, -1], dtype)])
    exp = oracle.join_agg(bkey, [bp0, bp1], pkey, [])
    _say("direct gaps + marker", np.dtype(dtype).name)
    got_d, _ = ctx.join_plain(dev(bkey), [dev(bp0), dev(bp1)], dev(pkey))
    got_h, _ = ctx.join_plain(dev(bkey), [dev(bp0), dev(bp1)], dev(pkey), hashed=True)
    assert got_d == exp and got_h == exp


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("end", ["top", "bottom"])
def test_direct_at_type_extremes(gpu, ctx, dtype, end):
    """Ranges ending at the type's maximum, or starting just above its minimum (the marker)."""
    info = np.iinfo(dtype)
    n = 4096
    rng = np.random.default_rng(5)
    lo = int(info.max) - n + 1 if end == "top" else int(info.min) + 1
    bkey = (rng.permutation(n).astype(np.int64) + lo).astype(dtype)
    bpay = rng.integers(-2**62, 2**62, n).astype(np.int64)
    pkey = np.concatenate([bkey[::3], np.array([info.max, info.min, info.min + 1, 0, -1,
                                                lo - 1 if end == "top" else lo + n], np.int64).astype(dtype)])
    _say("direct extremes", np.dtype(dtype).name, end)
    got, st = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey))
    assert got == oracle.join_agg(bkey, [bpay], pkey, [])
    assert st["table_bytes"] == _dense_bytes(n, [np.int64])


@pytest.mark.parametrize("dup", [0, 500, 999])
def test_direct_duplicate_rejected(gpu, ctx, dup):
    """A repeated key at either end or inside the range fails the unique build."""
    bkey = np.concatenate([np.arange(1000), [dup]]).astype(np.int32)
    _say("direct duplicate", dup)
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_plain(dev(bkey), [], dev(bkey))
    assert ei.value.status == gpu.VX_EDUPKEY


@pytest.mark.parametrize("swap", [(500, 0), (0, 999), (999, 0)])
def test_dense_duplicate_rejected(gpu, ctx, swap):
    """n keys spanning a range n wide but with one key repeated (so another is missing): the row
    count matches the range, and the build must still fail."""
    bkey = np.arange(1000, dtype=np.int64)
    bkey[swap[0]] = swap[1]
    _say("dense duplicate", swap)
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_plain(dev(bkey), [dev(bkey)], dev(np.arange(-5, 1005, dtype=np.int64)))
    assert ei.value.status == gpu.VX_EDUPKEY
    with pytest.raises(gpu.VxError) as ei:
        ctx.build(dev(bkey), [dev(bkey)])
    assert ei.value.status == gpu.VX_EDUPKEY


@pytest.mark.parametrize("pays", [(), (np.int32, np.int64), (np.int64, np.int32, np.int32)])
def test_dense_payload_layouts(gpu, ctx, pays):
    """Dense tables without payloads and with mixed-width payloads, against the hash layout and the
    oracle; a key range one short of the rows (the empty-marker key added) is not dense."""
    rng = np.random.default_rng(61 + len(pays))
    n, base = 40_000, 3_000_000_000
    bkey = (rng.permutation(n) + base).astype(np.int64)
    bp = [rng.integers(np.iinfo(p).min, np.iinfo(p).max, n, dtype=np.int64, endpoint=True).astype(p) for p in pays]
    pkey = _probes(rng, base, n, 250_007, np.int64)
    ppay = rng.integers(-2**62, 2**62, len(pkey)).astype(np.int64)
    exp = oracle.join_agg(bkey, bp, pkey, [ppay])
    _say("dense payloads", [np.dtype(p).name for p in pays])
    got_d, st_d = ctx.join_plain(dev(bkey), [dev(x) for x in bp], dev(pkey), [dev(ppay)])
    got_h, _ = ctx.join_plain(dev(bkey), [dev(x) for x in bp], dev(pkey), [dev(ppay)], hashed=True)
    assert got_d == exp and got_h == exp
    assert st_d["table_bytes"] == _dense_bytes(n, pays)
    # the empty-marker key makes n + 1 rows over an n-wide range: a keyed direct table
    mk = np.concatenate([bkey, [np.iinfo(np.int64).min]])
    mp = [np.concatenate([x, x[:1]]) for x in bp]
    pk2 = np.concatenate([pkey, np.full(9, np.iinfo(np.int64).min)])
    pp2 = np.concatenate([ppay, ppay[:9]])
    got, st = ctx.join_plain(dev(mk), [dev(x) for x in mp], dev(pk2), [dev(pp2)])
    assert got == oracle.join_agg(mk, mp, pk2, [pp2])
    assert st["table_bytes"] != _dense_bytes(n, pays)


def test_direct_preagg(gpu, ctx):
    """A pre-aggregating build whose keys repeat inside a narrow range takes the direct layout."""
    rng = np.random.default_rng(12)
    bkey = rng.integers(-300, 700, 200_000).astype(np.int64)
    bkey[::1000] = np.iinfo(np.int64).min
    bpay = rng.integers(0, 1 << 40, len(bkey)).astype(np.int64)
    pkey = rng.integers(-400, 800, 100_000).astype(np.int64)
    pkey[::777] = np.iinfo(np.int64).min
    ppay = rng.integers(-(1 << 40), 1 << 40, len(pkey)).astype(np.int64)
    exp = oracle.join_agg(bkey, [bpay], pkey, [ppay])
    _say("direct preagg")
    got_d, st_d = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)], unique=False)
    got_h, st_h = ctx.join_plain(dev(bkey), [dev(bpay)], dev(pkey), [dev(ppay)], unique=False, hashed=True)
    assert got_d == exp and got_h == exp
    assert st_d["table_bytes"] < st_h["table_bytes"]


@pytest.mark.parametrize("late_mat", [0, 1])
def test_direct_table_streamed_host_probe(gpu, ctx, late_mat):
    """A direct table probed by a pinned host column in several chunks."""
    rng = np.random.default_rng(40 + late_mat)
    n = 50_000
    bkey = (rng.permutation(n) + 7).astype(np.int64)
    bpay = rng.integers(-2**31, 2**31, n).astype(np.int32)
    pkey = _probes(rng, 7, 2 * n, 1_000_003, np.int64)
    ppay = rng.integers(-2**62, 2**62, len(pkey)).astype(np.int64)
    t = ctx.build(dev(bkey), [dev(bpay)])
    try:
        _say("direct streamed", late_mat)
        got, st = t.probe(pinned(gpu, pkey), [pinned(gpu, ppay)], late_mat=late_mat, chunk_rows=100_000)
    finally:
        t.destroy()
    assert got == oracle.join_agg(bkey, [bpay], pkey, [ppay])
    assert st["chunks"] == 11


def test_direct_table_rows(gpu, ctx):
    """The join's rows from a direct table, sorted by probe row and compared column by column."""
    rng = np.random.default_rng(77)
    n = 30_000
    bkey = (rng.permutation(n) - 15_000).astype(np.int32)
    bpay = rng.integers(-2**31, 2**31, n).astype(np.int32)
    pkey = _probes(rng, -15_000, n, 200_003, np.int32)
    ppay = rng.integers(-2**31, 2**31, len(pkey)).astype(np.int32)
    t = ctx.build(dev(bkey), [dev(bpay)])
    try:
        _say("direct rows")
        agg, st, n_out, (row, bc, pc) = t.probe_rows(dev(pkey), [dev(ppay)])
    finally:
        t.destroy()
    erow, eb, ep = oracle.join_rows(bkey, [bpay], pkey, [ppay])
    assert n_out == len(erow)
    r = np.asarray(row[:n_out], np.uint64)
    order = np.argsort(r, kind="stable")
    assert np.array_equal(r[order], erow)
    assert np.array_equal(np.asarray(bc[0][:n_out], np.int64)[order], eb[0])
    assert np.array_equal(np.asarray(pc[0][:n_out], np.int64)[order], ep[0])
    assert agg == oracle.join_agg(bkey, [bpay], pkey, [ppay])


def test_host_keys_stay_hashed(gpu, ctx):
    """Host-resident build keys are not measured (that pass would cross the host link)."""
    n = 1 << 12
    bkey = np.arange(n, dtype=np.int32)
    _say("host keys hashed")
    got, st = ctx.join_plain(pinned(gpu, bkey), [], dev(bkey))
    assert got == [n]
    assert st["table_bytes"] == 2 * n * 8 + 256


def test_build_flag_errors(gpu, ctx):
    """VX_HASHED only qualifies VX_UNIQUE or VX_PREAGG; alone, or with unknown bits, it is rejected."""
    import ctypes as C
    k = dev(np.arange(100, dtype=np.int64))
    for flags in (gpu.VX_HASHED, gpu.VX_UNIQUE | gpu.VX_PREAGG, gpu.VX_UNIQUE | 8):
        d = gpu.BuildDesc(gpu.col(k), None, 0, flags, 100, 0.0, 0)
        h = C.c_void_p()
        assert gpu.lib().vx_build(ctx.h, C.byref(d), C.byref(h)) == gpu.VX_EINVAL
        assert not h.value
