"""Parity of the skewed partitioned join on its own input generator: Zipf(1.1) keys over ranks
[1, 2^40] by rejection-inversion (datagen.skew_build / skew_probe), the build side clustered into
about 200 range partitions (learned, sample-quantile) or 256 radix-hash partitions, with heavy
keys in singleton partitions and the clustered copy in device or in pinned host memory.

Scaled down (2^22 build x 2^24 probe rows) every partitioner and both placements are compared
with the oracle's join over all rows, and the learned method partition by partition.  A 48 MiB
budget makes the partition tables outgrow the arena, so the probe side streams once per group
of resident tables.  At full size (2^30 x 2^32, 48 GiB pinned, 32 GiB budget) two table
partitions are compared with the oracle on the rows that fall in them, and the three heaviest
keys' singleton partitions with their closed form mB(k) mP(k), sumB(k) mP(k) counted from the
arrays.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

GiB = 1 << 30
MiB = 1 << 20
M64 = 1 << 64
NB, NP = 1 << 22, 1 << 24


def _say(*a):
    print(*a, flush=True)


def _pinned(vx, a):
    hb = vx.HostBuffer(len(a), a.dtype)
    hb.array[:] = a
    return hb


@pytest.fixture(scope="module")
def skew(gpu):
    bk, bp = datagen.skew_build(NB)
    pk = datagen.skew_probe(NP)
    _say("skew workload scaled: oracle over", NB, "x", NP, "rows")
    exp = oracle.join_agg(bk, [bp], pk, [])
    H = [_pinned(gpu, a) for a in (bk, bp, pk)]
    yield bk, bp, pk, H, exp
    for h in H:
        h.free()


@pytest.fixture(scope="module")
def ctx4(gpu):
    c = gpu.Context(4 * GiB)
    yield c
    c.close()


def _singletons(spl):
    return [(int(spl[i - 1]), i) for i in range(1, len(spl)) if spl[i] == spl[i - 1] + 1]


@pytest.mark.parametrize("method,placement", [("learned", "0"), ("learned", "1"), ("quantile", "0"),
                                              ("quantile", "1"), ("radix_hash", "2"), ("auto", "2")])
def test_skew_scaled_methods_exact(gpu, ctx4, skew, method, placement, monkeypatch):
    monkeypatch.setenv("VX_CHUNK_BYTES", str(2 * MiB))
    monkeypatch.setenv("VX_PJ_DEVICE", placement)
    bk, bp, pk, H, exp = skew
    _say("skew scaled", method, "placement", placement)
    got, st, used = ctx4.join_partitioned(H[0], [H[1]], H[2], method=method, n_parts=256, seed=7,
                                          train_steps=300)
    assert got == exp
    assert st["chunks"] == NP * 8 // (2 * MiB)
    if method == "radix_hash":
        assert st["n_parts"] == 256 and st["singleton_rows"] == 0
    else:
        assert used in (gpu.VX_PART_LEARNED, gpu.VX_PART_QUANTILE)
        assert st["n_parts"] >= 128
        assert st["singleton_rows"] > 0.15 * (NB + NP)      # the heaviest keys need no table
    if placement in ("0", "1"):
        assert (st["zc_bytes"] == 0) == (placement == "1")


def test_skew_scaled_learned_per_partition(gpu, ctx4, skew, monkeypatch):
    """Every partition of the learned splitters against the oracle on its own rows."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(2 * MiB))
    bk, bp, pk, H, exp = skew
    _say("skew scaled per partition")
    got, st, used, per = ctx4.join_partitioned(H[0], [H[1]], H[2], method="learned", n_parts=256, seed=7,
                                               train_steps=300, per_partition=True)
    r = ctx4.partition(H[0], method="learned", n_parts=256, seed=7, train_steps=300)
    spl = r["splitters"]
    P = len(spl) + 1
    assert st["n_parts"] == P and got == exp
    ib, ip = oracle.part_ids_range(bk, spl), oracle.part_ids_range(pk, spl)
    assert np.array_equal(oracle.histogram(ib, P), r["hist"])
    for p in range(P):
        mb, mp = ib == p, ip == p
        assert per[p] == oracle.join_agg(bk[mb], [bp[mb]], pk[mp], []), f"partition {p}"
    assert len(_singletons(spl)) >= 5


def test_skew_small_budget_table_groups(gpu, skew, monkeypatch):
    """A 48 MiB arena cannot hold every partition's compact table at once: the clustered copy goes
    to pinned host memory and the probe side is streamed once per group of resident tables."""
    monkeypatch.setenv("VX_CHUNK_BYTES", str(2 * MiB))
    bk, bp, pk, H, exp = skew
    _say("skew scaled, 48 MiB budget")
    with gpu.Context(48 * MiB) as c:
        got, st, used = c.join_partitioned(H[0], [H[1]], H[2], method="learned", n_parts=256, seed=7,
                                           train_steps=300)
    print("probe-side host-to-device bytes:", st["sdma_bytes"], "for", NP * 8, "bytes of keys", flush=True)
    assert got == exp
    assert st["zc_bytes"] > 0                          # clustered copy read back from host memory
    assert st["sdma_bytes"] >= 2 * NP * 8                   # at least two passes over the probe keys


# ----------------------------------------------------------------------------- full size

def _chunked(n, step=1 << 27):
    return [(r0, min(n, r0 + step)) for r0 in range(0, n, step)]


def test_skew_full_size(gpu):
    nb, np_ = 1 << 30, 1 << 32
    _say("full-size skewed join: allocating 48 GiB pinned")
    bk, bp, pk = gpu.HostBuffer(nb, np.int64), gpu.HostBuffer(nb, np.int64), gpu.HostBuffer(np_, np.int64)
    try:
        for r0, r1 in _chunked(nb):
            datagen.skew_build(r1 - r0, out=(bk.array[r0:r1], bp.array[r0:r1]), row0=r0)
        for r0, r1 in _chunked(np_):
            datagen.skew_probe(r1 - r0, out=pk.array[r0:r1], row0=r0)
        _say("generated; learned and radix-hash joins")
        with gpu.Context(32 * GiB) as ctx:
            tot, st, used, per = ctx.join_partitioned(bk, [bp], pk, method="learned", n_parts=256, seed=7,
                                                      per_partition=True)
            r = ctx.partition(bk, method="learned", n_parts=256, seed=7)
            tot_r, st_r, _ = ctx.join_partitioned(bk, [bp], pk, method="radix_hash", n_parts=256, seed=7)
        assert tot == tot_r and st_r["n_parts"] == 256
        spl = r["splitters"]
        P = len(spl) + 1
        assert st["n_parts"] == P and [sum(x) % M64 for x in zip(*per)] == tot
        ex = cf.ThreadPoolExecutor(16)
        # the three heaviest keys: singleton partitions [k, k + 1) resolved from counts
        single = dict(_singletons(spl))
        _say("singleton closed forms")

        def heavy(lo, hi, b):
            kb = bk.array[lo:hi] if b else pk.array[lo:hi]
            out = []
            for k in (1, 2, 3):
                m = kb == k
                out.append((int(m.sum()), int(bp.array[lo:hi][m].view(np.uint64).sum(dtype=np.uint64)) if b else 0))
            return out

        hb = list(ex.map(lambda c: heavy(c[0], c[1], True), _chunked(nb)))
        hp = list(ex.map(lambda c: heavy(c[0], c[1], False), _chunked(np_)))
        for i, k in enumerate((1, 2, 3)):
            assert k in single, f"key {k} has no singleton partition"
            mB = sum(x[i][0] for x in hb)
            sB = sum(x[i][1] for x in hb)
            mP = sum(x[i][0] for x in hp)
            assert per[single[k]] == [mB * mP % M64, sB * mP % M64], f"key {k}"
        # two table partitions against the oracle on the rows that fall in them
        table_parts = [p for p in range(1, P - 1) if p not in single.values()]
        for p in (table_parts[len(table_parts) // 2], P - 1):
            lo = int(spl[p - 1])
            hi = int(spl[p]) if p < P - 1 else None
            _say("oracle on partition", p, "keys from", lo)

            def pick(c, col, pay):
                k = col.array[c[0]:c[1]]
                m = (k >= lo) & (k < hi) if hi is not None else k >= lo
                return k[m], (pay.array[c[0]:c[1]][m] if pay is not None else None)

            b = list(ex.map(lambda c: pick(c, bk, bp), _chunked(nb)))
            q = list(ex.map(lambda c: pick(c, pk, None), _chunked(np_)))
            kb = np.concatenate([x[0] for x in b])
            assert len(kb) == int(r["hist"][p])
            want = oracle.join_agg(kb, [np.concatenate([x[1] for x in b])], np.concatenate([x[0] for x in q]), [])
            assert per[p] == want, f"partition {p}"
        ex.shutdown()
    finally:
        for h in (bk, bp, pk):
            h.free()
