"""Full-size parity of the streamed join in the launch configuration bench.py times, with its
rows materialized as well.

2^26 build rows and 2^31 host-resident probe rows (48 GiB pinned), 16 GiB budget, automatic
late materialization.  The oracle's hash map of 2^26 keys is too slow to build here, so the
expected aggregates come from the generator's closed form (each probe row knows the build row it
matches), which tests/test_oracle_join.py pins to the oracle at small scale.  Every aggregate,
the per-chunk aggregates of sampled chunks, and a second run (determinism) are compared exactly.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

M64 = 1 << 64
GiB = 1 << 30


def test_streamed_join_full_size_closed_form(gpu):
    import torch
    nb, np_ = 1 << 26, 1 << 31
    print("full-size streamed join: allocating 49 GiB pinned", flush=True)
    H = {}
    for name, n, dt in (("bk", nb, np.int64), ("b0", nb, np.int32), ("b1", nb, np.int32),
                        ("pk", np_, np.int64), ("p0", np_, np.int64), ("p1", np_, np.int64)):
        H[name] = gpu.HostBuffer(n, dt)
    try:
        datagen.stream_build(nb, out=(H["bk"].array, H["b0"].array, H["b1"].array))
        step = 1 << 27
        for r0 in range(0, np_, step):
            datagen.stream_probe(nb, step, out=(H["pk"].array[r0:r0 + step], H["p0"].array[r0:r0 + step],
                                                H["p1"].array[r0:r0 + step]), row0=r0)
        print("generated; running the join", flush=True)
        cap = int(np_ * 0.1 * 1.01)
        for name, dt in (("row", np.uint64), ("ob0", np.int64), ("ob1", np.int64), ("op0", np.int64),
                         ("op1", np.int64)):
            H[name] = gpu.HostBuffer(cap, dt)
        with gpu.Context(16 * GiB) as ctx:
            t = ctx.build(H["bk"], [H["b0"], H["b1"]])
            tot, st, per = t.probe(H["pk"], [H["p0"], H["p1"]], chunk_aggs=True,
                                   chunk_rows=(64 << 20) // 8)
            tot2, _ = t.probe(H["pk"], [H["p0"], H["p1"]])
            print("materializing the join's rows", flush=True)
            out = (H["row"].array, [H["ob0"].array, H["ob1"].array], [H["op0"].array, H["op1"].array])
            tot3, _, n_out, _ = t.probe_rows(H["pk"], [H["p0"], H["p1"]], out=out, cap=cap)
            t.destroy()
        assert tot3 == tot and n_out == tot[0]
        assert tot == tot2
        assert st["chunks"] == 256 and st["zc_mask"] == 3
        print("closed form over", np_, "rows", flush=True)
        b0 = H["b0"].array.astype(np.int64)
        b1 = H["b1"].array.astype(np.int64)
        exp = [0, 0, 0, 0, 0]
        cr = st["chunk_rows"]
        hit = np.empty(cr, np.int64)
        for c in range(np_ // cr):
            r0 = c * cr
            datagen.fill_probe_fk(datagen.SEED_STREAM, datagen.COL_BKEY, nb, 0.1, hit_row=hit, row0=r0)
            h = hit >= 0
            rows = hit[h]
            vals = [int(h.sum()), int(b0[rows].sum()), int(b1[rows].sum()),
                    int(H["p0"].array[r0:r0 + cr][h].sum()), int(H["p1"].array[r0:r0 + cr][h].sum())]
            if c in (0, 77, np_ // cr - 1):
                assert per[c] == [v % M64 for v in vals], f"chunk {c}"
                # the materialized rows of this chunk: exactly its matching rows, with their values
                row = H["row"].array[:n_out]
                sel = np.nonzero((row >= r0) & (row < r0 + cr))[0]
                order = np.argsort(row[sel])
                got_rows = row[sel][order].astype(np.int64) - r0
                exp_rows = np.nonzero(h)[0]
                assert np.array_equal(got_rows, exp_rows), f"rows of chunk {c}"
                assert np.array_equal(H["ob0"].array[:n_out][sel][order], b0[hit[h]])
                assert np.array_equal(H["ob1"].array[:n_out][sel][order], b1[hit[h]])
                assert np.array_equal(H["op0"].array[:n_out][sel][order], H["p0"].array[r0:r0 + cr][h])
                assert np.array_equal(H["op1"].array[:n_out][sel][order], H["p1"].array[r0:r0 + cr][h])
            exp = [e + v for e, v in zip(exp, vals)]
        assert tot == [e % M64 for e in exp]
        assert [sum(x) % M64 for x in zip(*per)] == tot
    finally:
        for h in H.values():
            h.free()


def test_batch_full_size_closed_form(gpu):
    """256 joins at full size (build 2^10..2^22 rows, probe 10..100x), one graph launch; each job
    checked against its closed form (dense permutation keys: count = #{probe < n_build},
    SUM = sum of pay_of_key[probe]), which tests/test_oracle_join.py pins to the oracle."""
    import torch
    b, p = datagen.batch_sizes(256)
    print(f"batch full size: {int(p.sum())} probe rows", flush=True)
    jobs = [datagen.batch_job(j, int(b[j]), int(p[j])) for j in range(256)]
    dev = [[torch.from_numpy(a).cuda() for a in job] for job in jobs]
    with gpu.Context(32 * GiB) as ctx:
        got, st = ctx.join_batch([x[0] for x in dev], [x[1] for x in dev], [x[2] for x in dev])
    del dev
    print("batch full size: closed forms", flush=True)
    for j, (bk, bp, pk) in enumerate(jobs):
        pay_of_key = np.empty(len(bk), np.int64)
        pay_of_key[bk] = bp
        hit = pk < len(bk)
        exp = [int(hit.sum()), int(pay_of_key[pk[hit]].sum()) % M64]
        assert got[j] == exp, f"job {j}"


def test_radix_join_full_size(gpu):
    """The two-table radix join at the size bench.py times: A and B of 2^29 rows each (16 B
    tuples, 8 GiB per table, pinned), 4 GiB budget, automatic partition count.  The whole join
    is checked against the generator's closed form (every B row matches the one A row with its
    key), which tests/test_oracle_radix_join.py pins to the oracle; two sampled partitions are
    checked against the oracle itself on the rows both tables send to them."""
    import oracle
    n = 1 << 29
    print("full-size radix join: allocating 32 GiB pinned", flush=True)
    ak, av, bk, bv = (gpu.HostBuffer(n, np.int64) for _ in range(4))
    try:
        step = 1 << 27
        for r0 in range(0, n, step):
            datagen.radix_a(n, out=(ak.array[r0:r0 + step], av.array[r0:r0 + step]), row0=r0)
            datagen.radix_b(n, step, out=(bk.array[r0:r0 + step], bv.array[r0:r0 + step]), row0=r0)
        print("generated; running the join", flush=True)
        with gpu.Context(4 * GiB) as ctx:
            tot, st, per = ctx.join_radix(ak, [av], bk, [bv], per_partition=True)
            tot2, _ = ctx.join_radix(ak, [av], bk, [bv])
        assert tot == tot2
        P = st["n_parts"]
        assert P == 16 and st["chunks"] == 16
        print("closed form", flush=True)
        a_of_key = np.empty(n, np.uint64)
        a_of_key[ak.array] = av.array.view(np.uint64)
        want = [n, int(a_of_key[bk.array].sum(dtype=np.uint64)), int(bv.array.view(np.uint64).sum(dtype=np.uint64))]
        del a_of_key
        assert tot == want
        assert [sum(x) % M64 for x in zip(*per)] == tot
        for p in (0, P - 1):
            print("oracle on partition", p, flush=True)
            ma, mb = (ak.array & (P - 1)) == p, (bk.array & (P - 1)) == p
            assert per[p] == oracle.join_agg(ak.array[ma], [av.array[ma]], bk.array[mb], [bv.array[mb]])
    finally:
        for h in (ak, av, bk, bv):
            h.free()


def test_sort_full_size(gpu):
    """The out-of-core sort at the size bench.py times: 2^31 int64 keys uniform over all values,
    pinned (16 GiB), 4 GiB budget (32 runs).  The output must be in order and hold the input's
    multiset: equal sum mod 2^64, xor and count; and sampled output positions must hold the key
    of that rank in the regenerated input (counted directly: #{x < key} <= position <
    #{x <= key})."""
    n = 1 << 31
    print("full-size sort: 16 GiB pinned", flush=True)
    h = gpu.HostBuffer(n, np.int64)
    try:
        step = 1 << 27
        sums = [0, 0]
        for r0 in range(0, n, step):
            v = datagen.sort_keys(step, out=h.array[r0:r0 + step], row0=r0).view(np.uint64)
            sums[0] = (sums[0] + int(v.sum(dtype=np.uint64))) % M64
            sums[1] ^= int(np.bitwise_xor.reduce(v))
        with gpu.Context(4 * GiB) as ctx:
            st = ctx.sort(h)
        assert st["chunks"] == 32
        print("checking order and multiset", flush=True)
        got = [0, 0]
        prev = None
        for r0 in range(0, n, step):
            a = h.array[r0:r0 + step]
            assert np.all(a[1:] >= a[:-1]) and (prev is None or prev <= a[0])
            prev = a[-1]
            v = a.view(np.uint64)
            got[0] = (got[0] + int(v.sum(dtype=np.uint64))) % M64
            got[1] ^= int(np.bitwise_xor.reduce(v))
        assert got == sums
        print("sampled ranks", flush=True)
        pos = [0, 12_345_678, n // 2 + 7, n - 1]
        keys = [int(h.array[p]) for p in pos]
        less = [0] * len(pos)
        leq = [0] * len(pos)
        buf = np.empty(step, np.int64)
        for r0 in range(0, n, step):
            datagen.sort_keys(step, out=buf, row0=r0)
            for i, k in enumerate(keys):
                less[i] += int(np.count_nonzero(buf < k))
                leq[i] += int(np.count_nonzero(buf <= k))
        for p, lo, hi in zip(pos, less, leq):
            assert lo <= p < hi, (p, lo, hi)
    finally:
        h.free()
