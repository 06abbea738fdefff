"""Pins of the oracle for the out-of-core sort (Sec. 6.1).

The sort's result has a plain definition (the keys in ascending signed order), pinned to numpy's
sort and to the permutation and order invariants.  The merge phase's regroup step cuts every
sorted run at one global rank; the oracle states it as a definition (the rank smallest elements
of the union, ties from lower-numbered runs first), pinned here by its invariants and by a
worked example.
"""
import numpy as np
import pytest

import oracle

I64 = np.iinfo(np.int64)


@pytest.mark.parametrize("dtype", [np.int64, np.int32])
@pytest.mark.parametrize("n", [0, 1, 2, 1000, 100_003])
def test_sort_matches_numpy(dtype, n):
    rng = np.random.default_rng(n)
    info = np.iinfo(dtype)
    k = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    if n > 10:
        k[:3] = [info.min, info.max, 0]
        k[3:n // 3] = k[3]                      # a long run of one value
    got = oracle.sort(k)
    assert np.array_equal(got, np.sort(k.astype(np.int64)))
    assert np.all(got[1:] >= got[:-1])
    assert np.array_equal(np.unique(got, return_counts=True)[1], np.unique(k, return_counts=True)[1])


def test_merge_cuts_worked_example():
    # union in order: 1(run 0) 2(run 0) 2(run 0) 2(run 1) 3(run 1) 5(run 0)
    runs = [np.array([1, 2, 2, 5]), np.array([2, 3])]
    want = {0: [0, 0], 1: [1, 0], 2: [2, 0], 3: [3, 0], 4: [3, 1], 5: [3, 2], 6: [4, 2]}
    for r, c in want.items():
        assert list(oracle.merge_cuts(runs, r)) == c


@pytest.mark.parametrize("seed", range(4))
def test_merge_cuts_invariants(seed):
    rng = np.random.default_rng(seed)
    runs = [np.sort(rng.integers(-20, 20, int(rng.integers(0, 40)))) for _ in range(int(rng.integers(1, 7)))]
    runs[0] = np.concatenate([[I64.min], runs[0], [I64.max]])
    total = sum(len(r) for r in runs)
    for r in range(total + 1):
        cut = oracle.merge_cuts(runs, r)
        assert int(cut.sum()) == r and all(0 <= c <= len(x) for c, x in zip(cut, runs))
        taken = np.concatenate([x[:c] for x, c in zip(runs, cut)] + [np.zeros(0, np.int64)])
        rest = np.concatenate([x[c:] for x, c in zip(runs, cut)] + [np.zeros(0, np.int64)])
        if len(taken) and len(rest):
            assert taken.max() <= rest.min()
            v = taken.max()
            # ties at the cut value: a later run takes some only if every earlier run took all of its own
            partial = [j for j, (x, c) in enumerate(zip(runs, cut)) if c < len(x) and x[c] == v]
            took = [j for j, (x, c) in enumerate(zip(runs, cut)) if c > 0 and x[c - 1] == v]
            if partial and took:
                assert max(took) <= min(partial)


def test_regroup_then_merge_is_the_sort():
    rng = np.random.default_rng(9)
    runs = [np.sort(rng.integers(-1000, 1000, int(rng.integers(50, 400)))) for _ in range(9)]
    allk = np.concatenate(runs)
    C = 333
    ranks = list(range(0, len(allk), C)) + [len(allk)]
    cuts = [oracle.merge_cuts(runs, r) for r in ranks]
    parts = [np.sort(np.concatenate([x[a:b] for x, a, b in zip(runs, lo, hi)]))
             for lo, hi in zip(cuts[:-1], cuts[1:])]
    assert all(len(p) == hi - lo for p, lo, hi in zip(parts, ranks[:-1], ranks[1:]))
    assert np.array_equal(np.concatenate(parts), np.sort(allk))


# ---- the library's host-side regroup step (no GPU work), against the oracle's definition

@pytest.mark.parametrize("seed", range(6))
def test_library_merge_cuts_match_oracle(seed):
    import paper_2502_09541_amd as vx
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(1, 9))
    lo, hi = (-30, 30) if seed % 2 else (I64.min, I64.max)
    runs = [np.sort(rng.integers(lo, hi, int(rng.integers(0, 60)), dtype=np.int64)) for _ in range(k)]
    if seed == 3:
        runs[0] = np.concatenate([[I64.min] * 3, runs[0], [I64.max] * 2])
    total = sum(len(r) for r in runs)
    for r in range(total + 1):
        assert list(vx.merge_cuts(runs, r)) == list(oracle.merge_cuts(runs, r)), r


def test_library_merge_cuts_rejects_rank_past_end():
    import paper_2502_09541_amd as vx
    with pytest.raises(vx.VxError) as e:
        vx.merge_cuts([np.arange(5)], 6)
    assert e.value.status == vx.VX_EINVAL
