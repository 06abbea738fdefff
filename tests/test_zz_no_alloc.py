"""The no-allocation entry point, vx_join_plain_noalloc, against the plain join of vx_join_agg
(the same build and probe kernels with the table in a context's arena), through the C ABI.

Two calls in a row share the library's fixed device array; the second, on a smaller input, must
not see the first one's table.  Aggregates are integers mod 2^64, so the bar is equality.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

M64 = 1 << 64


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(*a):
    print(*a, flush=True)


def _run(gpu, out, bk, bps, pk, pps, unique=True):
    import torch
    out.fill_(-1)                      # the entry point must clear what it accumulates into
    gpu.join_plain_noalloc(bk, bps, pk, pps, out, unique=unique)
    torch.cuda.synchronize()
    return [int(v) % M64 for v in out.cpu().tolist()]


def test_noalloc_matches_join_agg_two_calls(gpu):
    import torch
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    with gpu.Context(1 << 30) as c:
        # the in-memory join at full size (2^20 unique int32 keys fill the array's largest table),
        # then a smaller, ragged one
        for nb, np_, seed in ((1 << 20, 1 << 24, 1), (10007, 300_001, 2)):
            bk, bp, pk = (_dev(x) for x in datagen.plain_join(nb, np_, seed=seed))
            _say("noalloc plain", nb, np_)
            want, _ = c.join_plain(bk, [bp], pk, hashed=True)
            got = _run(gpu, out, bk, [bp], pk, [])
            assert got[9] == 0
            assert got[:2] == want and got[2:9] == [0] * 7


def test_noalloc_int64_payloads_and_preagg(gpu):
    import torch
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    with gpu.Context(1 << 30) as c:
        bk, b0, b1 = datagen.stream_build(1 << 16, seed=8)
        pk, p0, p1 = datagen.stream_probe(1 << 16, 1 << 20, seed=8)
        d = [_dev(x) for x in (bk, b0, b1, pk, p0, p1)]
        _say("noalloc int64 keys, 2 + 2 payloads")
        want, _ = c.join_plain(d[0], d[1:3], d[3], d[4:6], hashed=True)
        got = _run(gpu, out, d[0], d[1:3], d[3], d[4:6])
        assert got[9] == 0 and got[:5] == want
        # duplicates on both sides through a pre-aggregating table, then a smaller unique join
        rng = np.random.default_rng(9)
        kb = rng.integers(-50, 50, 20_000).astype(np.int64)
        vb = rng.integers(-2**40, 2**40, 20_000).astype(np.int64)
        kp = rng.integers(-60, 60, 70_001).astype(np.int64)
        _say("noalloc pre-aggregated")
        want, _ = c.join_plain(_dev(kb), [_dev(vb)], _dev(kp), unique=False, hashed=True)
        got = _run(gpu, out, _dev(kb), [_dev(vb)], _dev(kp), [], unique=False)
        assert got[9] == 0 and got[:2] == want
        bk, bp, pk = (_dev(x) for x in datagen.plain_join(1000, 5000, seed=3))
        want, _ = c.join_plain(bk, [bp], pk, hashed=True)
        assert _run(gpu, out, bk, [bp], pk, [])[:2] == want


def test_noalloc_errors(gpu):
    import torch
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    _say("noalloc errors")
    big = _dev(np.arange((1 << 20) + 1, dtype=np.int32))
    with pytest.raises(gpu.VxError) as e:
        gpu.join_plain_noalloc(big, [big], big, [], out)
    assert e.value.status == gpu.VX_EBUDGET and "scratch" in str(e.value)
    host = np.arange(10, dtype=np.int32)
    with pytest.raises(gpu.VxError) as e:
        gpu.join_plain_noalloc(host, [], _dev(host), [], out)
    assert e.value.status == gpu.VX_EINVAL
    # a repeated key in a unique build is reported in the error word, not by the call
    k = _dev(np.array([3, 1, 3], np.int32))
    got = _run(gpu, out, k, [], k, [])
    assert got[9] & 1
