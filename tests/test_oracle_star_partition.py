"""Pins for the oracle's star join + GROUP BY, partitioning and late-materialization rule."""
import json
import os

import numpy as np
import pytest

import datagen
import oracle

M64 = 1 << 64
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- star join

def star_brute(dims, fks, meas):
    """Nested loops: every fact row against every dimension row (the definition)."""
    groups = {}
    nfact = len(fks[0])
    for i in range(nfact):
        g = []
        ok = True
        for d, dim in enumerate(dims):
            hits = [r for r in range(len(dim["key"])) if int(dim["key"][r]) == int(fks[d][i])]
            hits = [r for r in hits if dim["lo"] <= int(dim["filt"][r]) <= dim["hi"]]
            if not hits:
                ok = False
                break
            if dim.get("group") is not None and len(g) < 2:
                g.append(int(dim["group"][hits[0]]))
        if not ok:
            continue
        while len(g) < 2:
            g.append(0)
        acc = groups.setdefault(tuple(g), [0] + [0] * len(meas))
        acc[0] += 1
        for c, m in enumerate(meas):
            acc[1 + c] = (acc[1 + c] + int(m[i])) % M64
    return sorted(groups.items())


def _as_list(res):
    g, cnt, sums = res
    return [((int(a), int(b)), [int(c)] + [int(x) for x in s]) for (a, b), c, s in zip(g, cnt, sums)]


def test_star_brute_force_tiny():
    rng = np.random.default_rng(5)
    for trial in range(6):
        dims = []
        for d, n in enumerate((13, 40, 64, 25)):
            key = rng.permutation(2 * n)[:n].astype(np.int32)    # sparse unique keys
            filt = rng.integers(0, 4, n).astype(np.int32)
            grp = rng.integers(-3, 9, n).astype(np.int32) if d in (0, 3) else None
            dims.append(dict(key=key, filt=filt, lo=0, hi=int(rng.integers(0, 3)), group=grp))
        nf = 300
        fks = [rng.integers(-2, 2 * len(dims[d]["key"]) + 2, nf).astype(np.int32) for d in range(4)]
        meas = [rng.integers(-2**31, 2**31 - 1, nf, dtype=np.int64, endpoint=True).astype(np.int32)
                for _ in range(3)]
        assert _as_list(oracle.star_groupby(dims, fks, meas)) == star_brute(dims, fks, meas)


def test_star_dense_closed_form():
    """Dense dimension keys 0..n-1: filters and groups are direct array lookups."""
    rows = (100, 2000, 5000, 3000)
    dims = datagen.star_dims(seed=9, rows=rows)
    fks, meas = datagen.star_fact(100_000, seed=9, rows=rows)
    ok = np.ones(len(fks[0]), bool)
    for d, dim in enumerate(dims):
        ok &= (dim["filt"][fks[d]] >= dim["lo"]) & (dim["filt"][fks[d]] <= dim["hi"])
    g0 = dims[0]["group"][fks[0][ok]].astype(np.int64)
    g1 = dims[3]["group"][fks[3][ok]].astype(np.int64)
    code = g0 * 1000 + g1
    uniq, inv = np.unique(code, return_inverse=True)
    cnt = np.bincount(inv)
    res_g, res_c, res_s = oracle.star_groupby(dims, fks, meas)
    assert np.array_equal(res_g[:, 0], uniq // 1000)
    assert np.array_equal(res_g[:, 1], uniq % 1000)
    assert np.array_equal(res_c, cnt.astype(np.uint64))
    for c in range(3):
        s = np.zeros(len(uniq), np.int64)
        np.add.at(s, inv, meas[c][ok].astype(np.int64))
        assert np.array_equal(res_s[:, c], s.astype(np.uint64))
    # 1/7 * 1/5 * 1/25 * 1 survivors, 7 x 100 groups
    assert abs(ok.mean() - 1 / 875) < 0.001
    assert len(uniq) <= 700


def test_star_duplicate_dim_key_rejected():
    d = dict(key=np.array([1, 1], np.int32), filt=np.zeros(2, np.int32), lo=0, hi=0, group=None)
    with pytest.raises(ValueError):
        oracle.star_groupby([d], [np.array([1], np.int32)], [np.array([1], np.int32)])


def test_star_no_survivors_and_empty_fact():
    dims = datagen.star_dims(seed=1, rows=(10, 10, 10, 10))
    for d in dims:
        d["lo"], d["hi"] = 100, 200          # nothing passes
    fks, meas = datagen.star_fact(1000, seed=1, rows=(10, 10, 10, 10))
    g, c, s = oracle.star_groupby(dims, fks, meas)
    assert len(g) == 0
    g, c, s = oracle.star_groupby(dims, [f[:0] for f in fks], [m[:0] for m in meas])
    assert len(g) == 0


# ----------------------------------------------------------------------------- partitioning

def test_boundary_closed_form_and_stable_order():
    """find_boundary == exclusive prefix sum of the histogram; clustering is a stable sort."""
    rng = np.random.default_rng(2)
    for nparts in (1, 2, 7, 64, 1000):
        n = int(rng.integers(0, 5000))
        ids = rng.integers(0, nparts, n).astype(np.uint32)
        if nparts > 3 and n:
            ids[ids == 1] = 2          # force empty groups, including a leading one
            ids[ids == 0] = 3
        order, b = oracle.cluster_boundary(ids, nparts)
        hist = oracle.histogram(ids, nparts)
        assert np.array_equal(hist, np.bincount(ids, minlength=nparts).astype(np.uint64))
        assert int(hist.sum()) == n
        expect_b = np.concatenate([[0], np.cumsum(hist)]).astype(np.uint64)
        assert np.array_equal(b, expect_b)
        assert np.array_equal(order, np.argsort(ids, kind="stable").astype(np.uint64))


def test_boundary_paper_example():
    """The paper's find_boundary illustration (Sec. 6.2.1): four 3-bit tuples clustered on
    their two low bits into four groups; group 1 is empty so its entry equals the next
    boundary.  Only the facts stated in the text are fixed by the fixture."""
    with open(os.path.join(GOLDEN, "find_boundary_example.json")) as f:
        ex = json.load(f)
    keys = np.array(ex["keys_consistent_with_text"], np.int64)
    ids = oracle.part_ids_bits(keys, 0, ex["hash_bits"])
    order, b = oracle.cluster_boundary(ids, ex["groups"])
    assert len(b) == ex["groups"] + 1
    for idx, val in ex["boundary_entries_stated"].items():
        assert int(b[int(idx)]) == val
    assert int(b[-1]) == len(keys)


def test_part_ids_bits_paper_radix():
    """Raw low-bit radix ids (the paper uses key bits 0..23): id == key & (2^b - 1)."""
    keys = np.array([0, 1, 2**24 - 1, 2**24, 2**24 + 5, -1, 2**40 + 3], np.int64)
    ids = oracle.part_ids_bits(keys, 0, 24)
    assert ids.tolist() == [0, 1, 2**24 - 1, 0, 5, 2**24 - 1, 3]
    assert oracle.part_ids_bits(keys, 2, 1).tolist() == [0, 0, 1, 0, 1, 1, 0]


def test_part_ids_hash_properties():
    """The radix-hash id is the top bits of a bijective 64-bit mix: zero maps to zero,
    distinct keys spread uniformly, and the ids are nested across log2p."""
    keys = np.arange(1, 200_001, dtype=np.int64)
    assert oracle.part_ids_hash(np.zeros(1, np.int64), 8)[0] == 0
    ids8 = oracle.part_ids_hash(keys, 8)
    counts = np.bincount(ids8, minlength=256)
    chi2 = float(((counts - len(keys) / 256) ** 2 / (len(keys) / 256)).sum())
    assert chi2 < 400          # 255 dof; mean 255, sd ~22.6
    ids4 = oracle.part_ids_hash(keys, 4)
    assert np.array_equal(ids4, ids8 >> 4)
    assert oracle.part_ids_hash(keys, 0).max() == 0


# The published inverse of the MurmurHash3 64-bit finalizer (the "unmix" used to invert it):
# the xor-shift by 33 undoes itself, and these are the inverses of its two multipliers mod 2^64.
_UNMIX = (0x9CB4B2F8129337DB, 0x4F74430C22A54005)


def _unmix64(h):
    m = (1 << 64) - 1
    h ^= h >> 33
    h = (h * _UNMIX[0]) & m
    h ^= h >> 33
    h = (h * _UNMIX[1]) & m
    h ^= h >> 33
    return h


def test_hash64_inverted_by_published_unmix():
    """The finalizer's output, run through its published inverse, gives the key back.  A wrong
    multiplier, shift or step order in the oracle's finalizer breaks this for almost every key."""
    rng = np.random.default_rng(11)
    keys = np.concatenate([rng.integers(-2**63, 2**63 - 1, 2000, dtype=np.int64),
                           np.array([0, 1, -1, 2**63 - 1, -2**63, 2**40, 12345], np.int64)])
    h = oracle.hash64(keys)
    assert h[len(keys) - 7] == 0                     # fmix64(0) = 0
    back = [_unmix64(int(v)) for v in h]
    assert back == [int(k) & ((1 << 64) - 1) for k in keys]
    # the radix-hash id is the finalizer's top log2p bits
    for log2p in (1, 7, 12):
        assert np.array_equal(oracle.part_ids_hash(keys, log2p), (h >> np.uint64(64 - log2p)).astype(np.uint32))


def test_part_ids_range_is_upper_bound():
    rng = np.random.default_rng(4)
    keys = rng.integers(-1000, 1000, 5000).astype(np.int64)
    spl = np.unique(rng.integers(-1200, 1200, 9)).astype(np.int64)
    ids = oracle.part_ids_range(keys, spl)
    assert np.array_equal(ids, np.searchsorted(spl, keys, side="right").astype(np.uint32))
    assert oracle.part_ids_range(keys, np.zeros(0, np.int64)).max() == 0


def test_late_materialization_threshold_paper_value():
    """Sec. 6.3: 4-byte elements, a 64-byte LLC line and four GPUs give TH = 1/64."""
    assert oracle.late_mat_threshold(4, 64, 4) == 1 / 64
    assert oracle.late_mat_threshold(8, 128, 1) == 1 / 16
