"""GPU parity of the star join + GROUP BY against the oracle, through the C ABI (bit-exact)."""
import numpy as np
import pytest

import datagen
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


def _random_star(rng, rows=(13, 40, 64, 25), nf=3000, groups=(0, 3), key_dtype=np.int32):
    dims = []
    for d, n in enumerate(rows):
        key = rng.permutation(2 * n)[:n].astype(key_dtype)
        filt = rng.integers(0, 4, n).astype(np.int32)
        grp = rng.integers(-3, 9, n).astype(np.int32) if d in groups else None
        dims.append(dict(key=key, filt=filt, lo=0, hi=int(rng.integers(0, 3)), group=grp))
    fks = [rng.integers(-2, 2 * len(dims[d]["key"]) + 2, nf).astype(key_dtype) for d in range(len(rows))]
    meas = [rng.integers(-2**31, 2**31 - 1, nf, dtype=np.int64, endpoint=True).astype(np.int32) for _ in range(3)]
    return dims, fks, meas


def _check(got, exp):
    g, c, s, st = got
    eg, ec, es = exp
    assert np.array_equal(g, eg) and np.array_equal(c, ec) and np.array_equal(s, es)


def _dev_dims(dims):
    return [dict(key=dev(d["key"]), filt=dev(d["filt"]), lo=d["lo"], hi=d["hi"],
                 group=None if d["group"] is None else dev(d["group"])) for d in dims]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_star_tiny_device_resident(gpu, ctx, seed):
    dims, fks, meas = _random_star(np.random.default_rng(seed))
    _say("star tiny", seed)
    exp = oracle.star_groupby(dims, fks, meas)
    _check(ctx.join_star(_dev_dims(dims), [dev(f) for f in fks], [dev(m) for m in meas]), exp)


@pytest.mark.parametrize("late_mat", [0, 1, -1, 2])
def test_star_host_streamed_modes(gpu, ctx, late_mat):
    rng = np.random.default_rng(11)
    dims, fks, meas = _random_star(rng, rows=(100, 700, 3000, 1000), nf=500_003)
    _say("star streamed late_mat", late_mat)
    exp = oracle.star_groupby(dims, fks, meas)
    got = ctx.join_star(_dev_dims(dims), [pinned(gpu, f) for f in fks], [pinned(gpu, m) for m in meas],
                        late_mat=late_mat, chunk_rows=40_000, count_zc=late_mat == 1)
    _check(got, exp)
    st = got[3]
    assert st["chunks"] == (500_003 + 39_999) // 40_000
    if late_mat == 0:
        assert st["zc_mask"] == 0
    if late_mat == 1:
        assert st["zc_mask"] == (1 << 7) - 2      # every column but the first probed key
        # counted zero-copy traffic: dimensions are probed in ascending filter selectivity (stable);
        # each later foreign key is read for the rows alive before it, the measures for the
        # survivors, each in 128-byte granules of 32 int32 rows (page-aligned columns, chunks of
        # 40,000 rows = 625 waves, so no granule is split between two waves)
        passing = [d["key"][(d["filt"] >= d["lo"]) & (d["filt"] <= d["hi"])] for d in dims]
        sel = [len(p) / len(d["key"]) for p, d in zip(passing, dims)]
        order = sorted(range(len(dims)), key=lambda k: sel[k])
        alive = np.ones(len(fks[0]), bool)
        granules = 0
        for pos, k in enumerate(order):
            if pos:
                granules += len(np.unique(np.nonzero(alive)[0] * 4 // 128))
            alive &= np.isin(fks[k], passing[k])
        granules += len(meas) * len(np.unique(np.nonzero(alive)[0] * 4 // 128))
        assert st["survivors"] == int(alive.sum())
        assert st["zc_counted"] == 1 and st["zc_bytes"] == 128 * granules


def test_star_ssb_shape_medium(gpu, ctx):
    """Four dimensions with the benchmark's filter selectivities and group attributes, reduced sizes."""
    rows = (2556, 20_000, 300_000, 200_000)
    dims = datagen.star_dims(seed=4, rows=rows)
    fks, meas = datagen.star_fact(3_000_000, seed=4, rows=rows)
    _say("star ssb-shaped medium")
    exp = oracle.star_groupby(dims, fks, meas)
    hdims = [dict(key=pinned(gpu, d["key"]), filt=pinned(gpu, d["filt"]), lo=0, hi=0,
                  group=None if d["group"] is None else pinned(gpu, d["group"])) for d in dims]
    got = ctx.join_star(hdims, [pinned(gpu, f) for f in fks], [pinned(gpu, m) for m in meas],
                        chunk_rows=1 << 20)
    _check(got, exp)
    assert got[3]["survivors"] == int(exp[1].sum())


def test_star_edge_cases(gpu, ctx):
    rng = np.random.default_rng(5)
    dims, fks, meas = _random_star(rng)
    _say("star: no survivors")
    nod = [dict(d, lo=100, hi=200) for d in dims]
    g, c, s, st = ctx.join_star(_dev_dims(nod), [dev(f) for f in fks], [dev(m) for m in meas])
    assert len(g) == 0 and st["survivors"] == 0
    _say("star: empty fact table")
    g, c, s, st = ctx.join_star(_dev_dims(dims), [dev(f[:0]) for f in fks], [dev(m[:0]) for m in meas])
    assert len(g) == 0
    _say("star: duplicate dimension key")
    bad = [dict(d) for d in dims]
    k = bad[1]["key"].copy()
    k[3] = k[7]
    bad[1]["key"] = k
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_star(_dev_dims(bad), [dev(f) for f in fks], [dev(m) for m in meas])
    assert ei.value.status == gpu.VX_EDUPKEY
    _say("star: group capacity")
    exp = oracle.star_groupby(dims, fks, meas)
    with pytest.raises(gpu.VxError) as ei:
        ctx.join_star(_dev_dims(dims), [dev(f) for f in fks], [dev(m) for m in meas], groups_cap=2)
    assert ei.value.status == gpu.VX_ECAPACITY


def test_star_sentinel_keys_and_negative_groups(gpu, ctx):
    """INT32_MIN as a dimension key and foreign key; group (-1, -1) (all-ones group code)."""
    i32 = np.iinfo(np.int32)
    d0 = dict(key=np.array([i32.min, 1, 2, i32.max], np.int32), filt=np.zeros(4, np.int32), lo=0, hi=0,
              group=np.array([-1, 5, -1, 7], np.int32))
    d1 = dict(key=np.array([i32.min, 3, 4], np.int32), filt=np.array([0, 0, 1], np.int32), lo=0, hi=0,
              group=np.array([-1, -1, 2], np.int32))
    f0 = np.array([i32.min, 1, 2, i32.max, 9, i32.min], np.int32)
    f1 = np.array([i32.min, 3, i32.min, 4, 3, 3], np.int32)
    m = [np.array([1, 2, 3, 4, 5, 6], np.int32)]
    exp = oracle.star_groupby([d0, d1], [f0, f1], m)
    _say("star sentinel")
    _check(ctx.join_star(_dev_dims([d0, d1]), [dev(f0), dev(f1)], [dev(x) for x in m]), exp)
    assert (-1, -1) in [tuple(r) for r in exp[0].tolist()]


def test_star_full_size_dense_closed_form(gpu):
    """Full size: 600,000,000 fact rows (16.8 GB pinned), dimensions of 2,556 / 200,000 /
    3,000,000 / 2,000,000 rows.  Expected groups from direct-array lookups (dense dimension keys),
    the closed form tests/test_oracle_star_partition.py pins to the oracle."""
    nf = 600_000_000
    rows = datagen.STAR_DIM_ROWS
    dims = datagen.star_dims()
    _say("star full size: allocating pinned fact table")
    fk_h = [gpu.HostBuffer(nf, np.int32) for _ in range(4)]
    ms_h = [gpu.HostBuffer(nf, np.int32) for _ in range(3)]
    try:
        step = 1 << 26
        for r0 in range(0, nf, step):
            r1 = min(nf, r0 + step)
            datagen.star_fact(r1 - r0, rows=rows, out=([h.array[r0:r1] for h in fk_h],
                                                       [h.array[r0:r1] for h in ms_h]), row0=r0)
        _say("star full size: running")
        with gpu.Context(16 * GiB) as c:
            g, cnt, sums, st = c.join_star(_dev_dims(dims), fk_h, ms_h, groups_cap=4096)
        _say(f"star full size: {st['total_ms']:.1f} ms, {st['survivors']} survivors, zc_mask {st['zc_mask']}")
        _say("star full size: closed form")
        acc = {}
        for r0 in range(0, nf, step):
            r1 = min(nf, r0 + step)
            ok = np.ones(r1 - r0, bool)
            for d, dim in enumerate(dims):
                ok &= dim["filt"][fk_h[d].array[r0:r1]] == 0
            code = (dims[0]["group"][fk_h[0].array[r0:r1][ok]].astype(np.int64) * 1000 +
                    dims[3]["group"][fk_h[3].array[r0:r1][ok]])
            u, inv = np.unique(code, return_inverse=True)
            cs = np.bincount(inv)
            ss = [None] * 3
            for mcol in range(3):
                s = np.zeros(len(u), np.int64)
                np.add.at(s, inv, ms_h[mcol].array[r0:r1][ok].astype(np.int64))
                ss[mcol] = s
            for i, key in enumerate(u.tolist()):
                a = acc.setdefault(key, [0, 0, 0, 0])
                a[0] += int(cs[i])
                for mcol in range(3):
                    a[1 + mcol] += int(ss[mcol][i])
        keys = sorted(acc)
        assert g[:, 0].tolist() == [k // 1000 for k in keys]
        assert g[:, 1].tolist() == [k % 1000 for k in keys]
        assert cnt.tolist() == [acc[k][0] for k in keys]
        assert sums.tolist() == [[acc[k][1 + m] % (1 << 64) for m in range(3)] for k in keys]
        assert len(keys) == 700
    finally:
        for h in fk_h + ms_h:
            h.free()
