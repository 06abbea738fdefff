"""GPU parity of the batched join (queue-draining build and probe kernels in one HIP graph, and
the per-job baseline of two launches per join)."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

GiB = 1 << 30
M64 = 1 << 64


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Context(8 * GiB)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(*a):
    print(*a, flush=True)


def _jobs(n_jobs, seed, b_lo=1 << 10, b_hi=1 << 16):
    b, p = datagen.batch_sizes(n_jobs, seed=seed, b_lo=b_lo, b_hi=b_hi)
    return [datagen.batch_job(j, int(b[j]), int(p[j]), seed=seed) for j in range(n_jobs)]


@pytest.mark.parametrize("mode", [1, 0])
def test_batch_matches_oracle(gpu, ctx, mode):
    jobs = _jobs(24, 41)
    _say("batch mode", mode)
    got, st = ctx.join_batch([dev(j[0]) for j in jobs], [dev(j[1]) for j in jobs], [dev(j[2]) for j in jobs],
                             mode=mode)
    for (bk, bp, pk), g in zip(jobs, got):
        assert g == oracle.join_agg(bk, [bp], pk, [])
    assert st["rows"] == sum(len(j[2]) for j in jobs)


def test_batch_explicit_configs_and_graph_replay(gpu, ctx):
    jobs = _jobs(16, 42)
    exp = [oracle.join_agg(bk, [bp], pk, []) for bk, bp, pk in jobs]
    args = ([dev(j[0]) for j in jobs], [dev(j[1]) for j in jobs], [dev(j[2]) for j in jobs])
    for tile, block, lf in ((64, 256, 0.5), (1024, 512, 0.7), (65536, 256, 0.9)):
        _say("batch config", tile, block, lf)
        got, _ = ctx.join_batch(*args, tile_rows=tile, block=block, load_factor=lf)
        assert got == exp
    # replays of the cached graph, with eager work in between
    import torch
    for r in range(3):
        got, st = ctx.join_batch(*args, tile_rows=1024, block=512, load_factor=0.7)
        assert got == exp
        torch.cuda.synchronize()
        _ = (args[2][0] + 1).sum().item()
    # one graph: build phase, bit count of the direct tables (these jobs' keys fill their ranges), and
    # the probe by regions: count, scan and scatter of the probe sides whose tables exceed the stage,
    # then the region probe
    assert st["kernel_launches"] == 6 and st["n_parts"] > 0


def test_batch_edges(gpu, ctx):
    i32 = np.iinfo(np.int32)
    bk = [np.array([i32.min, 1, 2], np.int32), np.zeros(0, np.int32), np.array([5], np.int32)]
    bp = [np.array([7, 8, 9], np.int32), np.zeros(0, np.int32), np.array([-3], np.int32)]
    pk = [np.array([i32.min, i32.min, 2, 3], np.int32), np.array([1, 2], np.int32), np.zeros(0, np.int32)]
    _say("batch edges")
    for mode in (0, 1):
        got, _ = ctx.join_batch([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk], mode=mode,
                                tile_rows=64, block=256, load_factor=0.5)
        assert got == [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_batch([dev(np.array([1, 1], np.int32))], [None], [dev(np.array([1], np.int32))],
                       tile_rows=64, block=256, load_factor=0.5)
    assert ei.value.status == gpu.VX_EDUPKEY


def test_batch_hash_duplicate_detected(gpu, ctx):
    """A repeated key with a different payload in a hash-table job (the insert that claims key and
    payload in one 64-bit compare-and-swap finds the key already there), and in a job whose keys
    would take a direct table but are forced into a hash table; both modes."""
    rng = np.random.default_rng(8)
    k = np.unique(rng.integers(-10**9, 10**9, 20_000)).astype(np.int32)
    rng.shuffle(k)
    k = np.concatenate([k, k[:1]])
    pay = rng.integers(-100, 100, len(k)).astype(np.int32)
    pay[-1] = pay[0] + 1
    cases = [([dev(k)], [dev(pay)], False),
             ([dev(np.array([0, 1, 1, 3], np.int32))], [dev(np.array([5, 6, 7, 8], np.int32))], True)]
    for bks, bps, hashed in cases:
        for mode in (0, 1):
            _say("batch hash duplicate", len(bks[0]), "hashed", hashed, "mode", mode)
            with pytest.raises(gpu.VxError) as ei:
                ctx.join_batch(bks, bps, [dev(np.array([1, 2], np.int32))], mode=mode, hashed=hashed,
                               tile_rows=1024, block=256, load_factor=0.5)
            assert ei.value.status == gpu.VX_EDUPKEY


@pytest.mark.parametrize("kt", [np.int32, np.int64])
def test_batch_without_payloads(gpu, ctx, kt):
    """Jobs with no payload column: counts only (the sums stay 0).  Direct tables then hold
    nothing to read (a probe key in range is a match); hash tables (an insert claims key and a
    zero payload at once) of 512 KiB and more have their probe sides partitioned, with the
    forced-hash flag for every job; in the graph and in the per-job baseline."""
    rng = np.random.default_rng(12)
    bk = [(rng.permutation(n).astype(np.int64) - 5).astype(kt) for n in (3000, 70_000)]
    bk.append(np.unique(rng.integers(-10**6, 10**6, 40_000)).astype(kt))
    pk = [np.concatenate([rng.integers(int(k.min()) - 100, int(k.max()) + 100, 3 * len(k)).astype(kt),
                          k[rng.integers(0, len(k), len(k))]]) for k in bk]
    exp = [oracle.join_agg(a, [], c, []) + [0] for a, c in zip(bk, pk)]
    args = ([dev(x) for x in bk], [None] * len(bk), [dev(x) for x in pk])
    for hashed in (False, True):
        for mode in (0, 1):
            _say("batch without payloads", kt.__name__, "hashed", hashed, "mode", mode)
            got, _ = ctx.join_batch(*args, mode=mode, hashed=hashed, tile_rows=1024, block=256, load_factor=0.7)
            assert got == exp


def test_batch_int64_keys(gpu, ctx):
    rng = np.random.default_rng(3)
    bk = [rng.permutation(1 << 40)[:0] if False else np.unique(rng.integers(-2**60, 2**60, n)).astype(np.int64)
          for n in (1000, 5000, 300)]
    bp = [rng.integers(-2**40, 2**40, len(k)).astype(np.int64) for k in bk]
    pk = [np.concatenate([k[::2], rng.integers(-2**60, 2**60, 3 * len(k))]).astype(np.int64) for k in bk]
    _say("batch int64")
    got, _ = ctx.join_batch([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk])
    assert got == [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]


def test_batch_direct_tables(gpu, ctx):
    """Jobs whose build keys fill their range exactly take a direct table: a mix of such jobs
    (int32 ranges anywhere, one starting at the empty-marker key) and hash-table jobs, in both
    modes, and with the keys changed in place between calls (the choice is made again)."""
    import torch
    i32 = np.iinfo(np.int32)
    rng = np.random.default_rng(8)
    bk, bp, pk = [], [], []
    for j, (n, base) in enumerate([(5000, 0), (3000, -1500), (777, i32.min), (4096, 10**9), (2000, None)]):
        k = (rng.permutation(n) + base).astype(np.int32) if base is not None else \
            np.unique(rng.integers(-10**6, 10**6, n)).astype(np.int32)
        bk.append(k)
        bp.append(rng.integers(i32.min, i32.max, len(k)).astype(np.int32))
        lo = int(k.min())
        pk.append(rng.integers(max(i32.min, lo - 500), min(i32.max, lo + 2 * len(k)), 6 * len(k)).astype(np.int32))
    exp = [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    dk = [dev(x) for x in bk]
    args = (dk, [dev(x) for x in bp], [dev(x) for x in pk])
    for mode in (0, 1):
        _say("batch direct tables, mode", mode)
        got, st = ctx.join_batch(*args, mode=mode, tile_rows=1024, block=256, load_factor=0.5)
        assert got == exp
    # job 0's keys no longer fill their range (one key moved far away), job 4's now do
    bk[0][0] = 10**8
    bk[4] = np.arange(len(bk[4]), dtype=np.int32) * 1 + 7
    dk[0].copy_(torch.from_numpy(bk[0]))
    dk[4].copy_(torch.from_numpy(bk[4]))
    exp = [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    got, _ = ctx.join_batch(*args, tile_rows=1024, block=256, load_factor=0.5)
    assert got == exp


def test_batch_direct_duplicate_detected(gpu, ctx):
    """Keys 0, 1, 1, 3 fill the range 0..3 by count but not by value: the direct table's bitmap
    sees the second 1."""
    for mode in (0, 1):
        with pytest.raises(gpu.VxError) as ei:
            ctx.join_batch([dev(np.array([0, 1, 1, 3], np.int32))], [None], [dev(np.array([2], np.int32))],
                           mode=mode, tile_rows=64, block=256, load_factor=0.5)
        assert ei.value.status == gpu.VX_EDUPKEY


def test_batch_direct_int64(gpu, ctx):
    rng = np.random.default_rng(9)
    bk = [(rng.permutation(n) + off).astype(np.int64) for n, off in ((3000, -2**62), (1024, 2**40), (1, 5))]
    bp = [rng.integers(-2**40, 2**40, len(k)).astype(np.int64) for k in bk]
    pk = [np.concatenate([k[::3], k.min() - 1 - np.arange(50), k.max() + 1 + np.arange(50)]).astype(np.int64)
          for k in bk]
    _say("batch direct int64")
    got, _ = ctx.join_batch([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk])
    assert got == [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_mixed_xcd_placement(gpu, ctx, mode):
    """Jobs whose tables exceed 3/4 of an XCD's L2 (spread over every XCD) beside jobs pinned to
    one XCD, hash and direct tables, and an empty job: every job's result must match the oracle."""
    rng = np.random.default_rng(17)
    sizes = [(1 << 20, 3_000_000), (3 << 18, 2_000_000), (1 << 19, 1_500_000), (5000, 40_000), (0, 1000)]
    sizes += [(int(n), int(10 * n)) for n in rng.integers(1000, 60_000, 12)]
    bk, bp, pk = [], [], []
    for i, (nb, npr) in enumerate(sizes):
        if i % 3 == 1:    # unique keys with gaps: a hash table
            k = np.unique(rng.integers(-2**30, 2**30, int(nb * 1.01) + 10)).astype(np.int32)[:nb]
            rng.shuffle(k)
        else:             # a permutation of a range: a direct table
            k = (rng.permutation(nb) + int(rng.integers(-2**20, 2**20))).astype(np.int32)
        bk.append(k)
        bp.append(rng.integers(-2**31, 2**31, nb).astype(np.int32))
        lo = int(k.min()) if nb else 0
        hi = int(k.max()) if nb else 1
        pk.append(np.concatenate([rng.choice(k, npr // 2) if nb else np.zeros(0, np.int32),
                                  rng.integers(lo - 1000, hi + 1000, npr - (npr // 2 if nb else 0))]).astype(np.int32))
    exp = [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    _say("batch mixed placement, mode", mode)
    got, _ = ctx.join_batch([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk], mode=mode,
                            tile_rows=8192, block=256, load_factor=0.5)
    assert got == exp


def test_batch_budget_error_then_success(gpu):
    """A batch whose tables do not fit the arena fails with VX_EBUDGET and leaves no cached graph
    behind: a smaller batch on the same context then runs, and the large one fails again."""
    MiB = 1 << 20
    c = gpu.Context(64 * MiB)
    try:
        rng = np.random.default_rng(23)
        big = np.unique(rng.integers(-2**31, 2**31 - 1, 5_000_000)).astype(np.int32)[:4_000_000]   # hash: 64 MiB of slots
        small_k = [rng.permutation(1000).astype(np.int32), np.array([3, 9, -4], np.int32)]
        small_p = [rng.integers(-2**31, 2**31, len(k)).astype(np.int32) for k in small_k]
        probes = [rng.integers(-10, 1010, 5000).astype(np.int32), np.array([9, 9, 1], np.int32)]
        _say("batch budget error")
        for _ in range(2):
            with pytest.raises(gpu.VxError) as ei:
                c.join_batch([dev(big)], [dev(big)], [dev(big[:100])], tile_rows=8192, block=256, load_factor=0.5)
            assert ei.value.status == gpu.VX_EBUDGET
            got, _ = c.join_batch([dev(x) for x in small_k], [dev(x) for x in small_p], [dev(x) for x in probes],
                                  tile_rows=8192, block=256, load_factor=0.5)
            assert got == [oracle.join_agg(a, [b], p, []) for a, b, p in zip(small_k, small_p, probes)]
    finally:
        c.close()


def test_batch_cache_gives_the_arena_back(gpu):
    """A graph-mode batch keeps its tables in the arena for the next call with the same jobs; any
    other call gets them back first.  Four direct jobs of 2^20 keys hold about 16.5 MiB of a 48 MiB
    arena; a plain join whose hashed table needs 32 MiB then still runs, and the arena's use
    returns to its level before the batch."""
    jobs = [datagen.plain_join(1 << 20, 1 << 20, seed=50 + j) for j in range(4)]
    exp = [oracle.join_agg(bk, [bp], pk, []) for bk, bp, pk in jobs]
    args = ([dev(j[0]) for j in jobs], [dev(j[1]) for j in jobs], [dev(j[2]) for j in jobs])
    bk, bp, pk = datagen.plain_join(1 << 21, 1 << 20, seed=9)
    want = oracle.join_agg(bk, [bp], pk, [])
    d = [dev(x) for x in (bk, bp, pk)]
    _say("batch arena retention")
    with gpu.Context(48 << 20) as c:
        base = c.arena_used()
        got, st = c.join_batch(*args, tile_rows=4096, block=256, load_factor=0.5)
        assert got == exp
        held = c.arena_used() - base
        assert held >= 16 << 20
        assert (48 << 20) - base - held < 32 << 20           # the join's table would not fit beside it
        assert c.join_plain(d[0], [d[1]], d[2], hashed=True)[0] == want
        assert c.arena_used() == base
        got, _ = c.join_batch(*args, tile_rows=4096, block=256, load_factor=0.5)   # graph built again
        assert got == exp


def test_batch_hashed_flag(gpu, ctx):
    """VX_HASHED puts every job in a hash table even when its keys fill their range; graph and
    per-job baseline agree with the oracle either way."""
    jobs = _jobs(12, 45)
    exp = [oracle.join_agg(bk, [bp], pk, []) for bk, bp, pk in jobs]
    args = ([dev(j[0]) for j in jobs], [dev(j[1]) for j in jobs], [dev(j[2]) for j in jobs])
    _say("batch hashed flag")
    for mode in (0, 1):
        got_h, st_h = ctx.join_batch(*args, mode=mode, hashed=True, tile_rows=2048, block=256, load_factor=0.5)
        got_d, st_d = ctx.join_batch(*args, mode=mode, tile_rows=2048, block=256, load_factor=0.5)
        assert got_h == exp and got_d == exp
        assert st_h["table_bytes"] > st_d["table_bytes"]   # hash slots of 8 B at load 0.5 against 4 B payloads


def _part_jobs(rng, kt):
    """Jobs for the partitioned probe path: direct-table jobs (ranges at 0, at the type's minimum and
    maximum, negative) and hash-table jobs (one holding the empty-marker key), probe sides from empty
    to ragged multiples of the partition tile."""
    info = np.iinfo(kt)
    bk, bp, pk = [], [], []
    specs = [(5000, 0, 4097), (20000, int(info.min), 50000), (70001, int(info.max) - 70000, 123457),
             (300000, -12345, 200003), (16384, 7, 0), (9000, None, 4096), (40000, None, 99999),
             (123456, None, 4095), (60000, "min", 70000)]
    for n, base, m in specs:
        if base is None or base == "min":
            k = np.unique(rng.integers(-10**6 if kt == np.int32 else -2**62, 10**6 if kt == np.int32 else 2**62,
                                       n + n // 8)).astype(kt)[:n]
            rng.shuffle(k)
            if base == "min":
                k[0] = info.min
        else:
            k = (rng.permutation(n).astype(np.int64) + base).astype(kt)
        bk.append(k)
        bp.append(rng.integers(-2**31, 2**31, n).astype(np.int32))
        lo, hi = int(k.min()), int(k.max())
        span_lo = max(int(info.min), lo - n // 2)
        span_hi = min(int(info.max), hi + n) if base is not None and base != "min" else hi
        rand = rng.integers(span_lo, span_hi, m // 2, dtype=np.int64, endpoint=True).astype(kt)
        hits = k[rng.integers(0, n, m - m // 2)]
        q = np.concatenate([rand, hits])
        rng.shuffle(q)
        if base == "min" and m:
            q[:50] = info.min
        pk.append(q)
    return bk, bp, pk


@pytest.mark.parametrize("kt", [np.int32, np.int64])
def test_batch_partitioned_probe(gpu, kt, monkeypatch):
    """The probe by regions: tables of at most the LDS stage probed whole from the jobs' own keys,
    larger ones cut into regions with the probe side partitioned into one array per region, regions
    staged in LDS or (past the region-count cap) read from device memory; direct and hash tables
    (whose probe keys outside the build keys' range are dropped).  Stages of 1 KiB and 64 KiB, and
    the probe through the tile map alone, against the oracle, with graph replays."""
    rng = np.random.default_rng(19 if kt == np.int32 else 23)
    bk, bp, pk = _part_jobs(rng, kt)
    exp = [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    args = ([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk])
    for stage_kb in ("1", "64"):
        monkeypatch.setenv("VX_BATCH_STAGE_KB", stage_kb)
        for hashed in (False, True):
            for tile, block, lf in ((1024, 256, 0.5), (65536, 512, 0.7)):
                _say("batch by regions", kt.__name__, "stage KiB", stage_kb, "hashed", hashed, "config", tile, block, lf)
                with gpu.Context(2 * GiB) as c:
                    for rep in range(2):
                        got, st = c.join_batch(*args, hashed=hashed, tile_rows=tile, block=block, load_factor=lf)
                        assert got == exp, f"replay {rep}"
                assert st["n_parts"] >= 4                       # jobs whose probe side was partitioned
                # jobs probed by regions: all but the one with no probe rows, unless its table fits the stage
                assert st["survivors"] == len(bk) - (1 if stage_kb == "1" or hashed else 0)
                # build phase, count, scan, scatter, region probe, and the direct tables' bit count
                assert st["kernel_launches"] == 5 + (0 if hashed else 1)
    monkeypatch.setenv("VX_BATCH_REGIONS", "0")
    with gpu.Context(2 * GiB) as c:
        got, st = c.join_batch(*args, tile_rows=1024, block=256, load_factor=0.5)
    assert got == exp and st["n_parts"] == 0 and st["kernel_launches"] == 3


@pytest.mark.parametrize("kt,pt", [(np.int32, np.int32), (np.int64, np.int32), (np.int64, np.int64)])
def test_batch_direct_tables_larger_than_l2(gpu, ctx, kt, pt):
    """Direct tables of 6 MB and more of payloads (their probe sides partitioned into regions),
    beside a direct table that fits an L2 and a hash table, int32 and int64 payloads: against the
    oracle in the graph (two replays, the tuned and an explicit configuration) and in the per-job
    baseline."""
    rng = np.random.default_rng(31)
    info = np.iinfo(kt)
    specs = [(1_500_001, -700_000), (1_000_003, int(info.max) - 1_000_002), (400_000, 12), (200_000, None)]
    bk, bp, pk = [], [], []
    for n, base in specs:
        if base is None:
            k = np.unique(rng.integers(-10**9, 10**9, n + n // 8)).astype(kt)[:n]
            rng.shuffle(k)
        else:
            k = (rng.permutation(n).astype(np.int64) + base).astype(kt)
        bk.append(k)
        bp.append(rng.integers(np.iinfo(pt).min, np.iinfo(pt).max, n, dtype=np.int64, endpoint=True).astype(pt))
        lo = max(int(info.min), int(k.min()) - n // 4)
        hi = min(int(info.max), int(k.max()) + n // 4)
        q = np.concatenate([rng.integers(lo, hi, n, dtype=np.int64, endpoint=True).astype(kt), k[rng.integers(0, n, n)]])
        rng.shuffle(q)
        pk.append(q)
    exp = [oracle.join_agg(a, [b], c, []) for a, b, c in zip(bk, bp, pk)]
    args = ([dev(x) for x in bk], [dev(x) for x in bp], [dev(x) for x in pk])
    for cfg in ({}, {"tile_rows": 8192, "block": 512, "load_factor": 0.7}):
        _say("batch large direct tables", kt.__name__, pt.__name__, "config", cfg)
        for rep in range(2):
            got, _ = ctx.join_batch(*args, **cfg)
            assert got == exp, f"replay {rep}"
    got, _ = ctx.join_batch(*args, mode=1)
    assert got == exp


def test_batch_direct_large_duplicate_detected(gpu, ctx):
    """A repeated key in a direct table of 1.2 M keys (filling their range by count, one value
    missing) is found by the presence count, in the graph and in the per-job baseline."""
    rng = np.random.default_rng(5)
    n = 1_200_000
    k = rng.permutation(n).astype(np.int32)
    lo, hi = int(np.argmin(k)), int(np.argmax(k))
    i, j = [x for x in range(10) if x not in (lo, hi)][:2]
    k[i] = k[j]
    for mode in (0, 1):
        with pytest.raises(gpu.VxError) as ei:
            ctx.join_batch([dev(k)], [dev(rng.integers(0, 100, n).astype(np.int32))], [dev(k[:1000])], mode=mode,
                           tile_rows=8192, block=512, load_factor=0.5)
        assert ei.value.status == gpu.VX_EDUPKEY
