"""GPU parity of the two-table radix join (the hash-join case study, Sec. 6.2) against the
oracle, through the C ABI.

Every result is an integer sum mod 2^64 and must match exactly: the whole join's (count,
SUM(A.val), SUM(B.val)), and each partition's, which the oracle computes by joining the rows of
both tables that its own partition function sends to that partition.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

GiB, MiB = 1 << 30, 1 << 20
M64 = 1 << 64


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(2 * GiB)
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


def _per_partition(ak, aps, bk, bps, ia, ib, P):
    out = []
    for p in range(P):
        ma, mb = ia == p, ib == p
        out.append(oracle.join_agg(ak[ma], [x[ma] for x in aps], bk[mb], [x[mb] for x in bps]))
    return out


def test_radix_join_recipe_one_partition(gpu, ctx):
    """The workload recipe at a small size: A's table fits, so nothing is clustered and both
    tables are read in place from pinned host memory."""
    na, nb = 1 << 18, (1 << 19) + 3
    ak, av = datagen.radix_a(na)
    bk, bv = datagen.radix_b(na, nb)
    _say("radix join one partition", na, nb)
    got, st = ctx.join_radix(pinned(gpu, ak), [pinned(gpu, av)], pinned(gpu, bk), [pinned(gpu, bv)])
    assert got == oracle.join_agg(ak, [av], bk, [bv])
    assert got[0] == nb
    assert st["n_parts"] == 1 and st["chunks"] == 1
    assert st["zc_bytes"] == na * 16 + nb * 16


@pytest.mark.parametrize("placement", [1, 2])
def test_radix_join_clustered(gpu, ctx, placement, monkeypatch):
    """Both tables clustered into 16 partitions by raw key bits over several pass-1 chunks (ragged
    tails), the clustered copies in pinned host memory (1) or in the arena (2)."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 50_000))
    na, nb = 300_001, 700_003
    ak, av = datagen.radix_a(na, seed=11)
    bk, bv = datagen.radix_b(na, nb, seed=11)
    bk[::97] += na                     # some B rows match nothing
    _say("radix join clustered, placement", placement)
    got, st, per = ctx.join_radix(pinned(gpu, ak), [pinned(gpu, av)], pinned(gpu, bk), [pinned(gpu, bv)],
                                  n_parts=16, placement=placement, per_partition=True)
    assert got == oracle.join_agg(ak, [av], bk, [bv])
    ia, ib = oracle.part_ids_bits(ak, 0, 4), oracle.part_ids_bits(bk, 0, 4)
    assert per == _per_partition(ak, [av], bk, [bv], ia, ib, 16)
    assert st["n_parts"] == 16 and st["chunks"] == 16
    # pass 1 copies every tuple in; pass 2 reads the clustered copies from host memory again (in
    # place or copied in) only when they live there
    pass2_host = st["zc_bytes"] + st["sdma_bytes"] - (na + nb) * 16
    assert (pass2_host == (na + nb) * 16) == (placement == 1)
    assert (pass2_host == 0) == (placement == 2)


@pytest.mark.parametrize("shift,P", [(5, 32), (0, 1024)])
def test_radix_join_raw_bits_shift(gpu, ctx, shift, P, monkeypatch):
    """Raw key bits from a shift, and the largest partition count, on device-resident tables
    with duplicate keys on both sides."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 70_000))
    rng = np.random.default_rng(shift + P)
    ak = rng.integers(0, 1 << 20, 250_000).astype(np.int64)
    bk = rng.integers(0, 1 << 20, 400_000).astype(np.int64)
    av = rng.integers(-2**40, 2**40, 250_000).astype(np.int64)
    bv = rng.integers(-2**40, 2**40, 400_000).astype(np.int64)
    _say("radix join raw bits", shift, P)
    got, st, per = ctx.join_radix(dev(ak), [dev(av)], dev(bk), [dev(bv)], n_parts=P, shift=shift,
                                  per_partition=True)
    assert got == oracle.join_agg(ak, [av], bk, [bv])
    lg = P.bit_length() - 1
    ia, ib = oracle.part_ids_bits(ak, shift, lg), oracle.part_ids_bits(bk, shift, lg)
    assert per == _per_partition(ak, [av], bk, [bv], ia, ib, P)


@pytest.mark.parametrize("pays", ["both", "a", "b", "none"])
def test_radix_join_hash_int32_duplicates_sentinel(gpu, ctx, pays, monkeypatch):
    """int32 keys partitioned by the 64-bit mix, heavy duplicates on both sides, the table's
    empty-marker key present on both sides, and every payload combination."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 40_000))
    i32 = np.iinfo(np.int32)
    rng = np.random.default_rng(5)
    ak = rng.zipf(1.3, 120_000).astype(np.int32)
    bk = rng.zipf(1.3, 260_001).astype(np.int32)
    ak[::3001] = i32.min
    bk[::4001] = i32.min
    av = rng.integers(i32.min, i32.max, len(ak)).astype(np.int32)
    bv = rng.integers(i32.min, i32.max, len(bk)).astype(np.int32)
    aps = [av] if pays in ("both", "a") else []
    bps = [bv] if pays in ("both", "b") else []
    _say("radix join int32 hash", pays)
    got, st, per = ctx.join_radix(pinned(gpu, ak), [pinned(gpu, x) for x in aps], pinned(gpu, bk),
                                  [pinned(gpu, x) for x in bps], n_parts=8, hash=True, per_partition=True)
    assert got == oracle.join_agg(ak, aps, bk, bps)
    ia, ib = oracle.part_ids_hash(ak, 3), oracle.part_ids_hash(bk, 3)
    assert per == _per_partition(ak, aps, bk, bps, ia, ib, 8)


@pytest.mark.parametrize("P", [1, 2])
def test_radix_join_slices(gpu, P, monkeypatch):
    """A partition whose A rows exceed the largest table the arena holds is built in slices,
    each probed by all of B's rows of that partition (all keys even: with raw bit 0 every row
    lands in partition 0)."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(8 * 65_536))
    na, nb = 1 << 18, (1 << 19) + 11
    ak, av = datagen.radix_a(na, seed=21)
    bk, bv = datagen.radix_b(na, nb, seed=21)
    ak, bk = ak * 2, bk * 2
    c = gpu.Context(16 * MiB)
    try:
        _say("radix join slices", P)
        got, st = ctx_join(c, gpu, ak, av, bk, bv, P)
    finally:
        c.close()
    assert got == oracle.join_agg(ak, [av], bk, [bv])
    assert st["chunks"] >= 2, st


def ctx_join(c, gpu, ak, av, bk, bv, P):
    if P == 1:
        return c.join_radix(dev(ak), [dev(av)], dev(bk), [dev(bv)], n_parts=1)
    return c.join_radix(pinned(gpu, ak), [pinned(gpu, av)], pinned(gpu, bk), [pinned(gpu, bv)], n_parts=P)


@pytest.mark.parametrize("na,nb", [(0, 1000), (1000, 0), (0, 0)])
def test_radix_join_empty(gpu, ctx, na, nb):
    ak, av = datagen.radix_a(max(na, 1))
    bk, bv = datagen.radix_b(max(na, 1), max(nb, 1))
    got, st = ctx.join_radix(dev(ak[:na]), [dev(av[:na])], dev(bk[:nb]), [dev(bv[:nb])], n_parts=4)
    assert got == [0, 0, 0]


def test_radix_join_errors(gpu, ctx):
    k = dev(np.arange(100, dtype=np.int64))
    k32 = dev(np.arange(100, dtype=np.int32))
    with pytest.raises(gpu.VxError) as e:
        ctx.join_radix(k, [k], k, [k], n_parts=3)
    assert e.value.status == gpu.VX_EINVAL
    with pytest.raises(gpu.VxError) as e:
        ctx.join_radix(k, [k, k], k, [k])
    assert e.value.status == gpu.VX_EUNSUPPORTED
    with pytest.raises(gpu.VxError) as e:
        ctx.join_radix(k, [k], k32, [k32])
    assert e.value.status == gpu.VX_EINVAL
    with pytest.raises(gpu.VxError) as e:
        ctx.join_radix(k, [k], k, [k], n_parts=4, placement=3)
    assert e.value.status == gpu.VX_EINVAL
