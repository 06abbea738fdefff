"""Pins of the oracle for the two-table radix join (the hash-join case study, Sec. 6.2).

The query is SUM(A.val + B.val) over the pairs with A.key == B.key.  The oracle answers it with
its join aggregate (count, SUM over pairs of A's payload, SUM over pairs of B's payload), so
the pair sum is the two payload sums added mod 2^64.  Pinned here by:
- nested-loop brute force of the query itself on tiny inputs with duplicates on both sides;
- the decomposition the radix join relies on: a partition function of the key sends both rows
  of every pair to one partition, so the per-partition joins add up to the whole join;
- closed forms of the workload recipe (unique permutation keys in A, foreign keys in B).
"""
import numpy as np
import pytest

import datagen
import oracle

M64 = 1 << 64


def _brute(ak, av, bk, bv):
    cnt = sa = sb = pair = 0
    for i in range(len(ak)):
        for j in range(len(bk)):
            if ak[i] == bk[j]:
                cnt += 1
                sa += int(av[i])
                sb += int(bv[j])
                pair += int(av[i]) + int(bv[j])
    return cnt, sa % M64, sb % M64, pair % M64


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pair_sum_brute_force(seed):
    rng = np.random.default_rng(seed)
    na, nb = 150, 230
    ak = rng.integers(0, 40, na).astype(np.int64)
    bk = rng.integers(0, 50, nb).astype(np.int64)
    ak[:3] = np.iinfo(np.int64).min     # the GPU table's empty marker is an ordinary key here
    bk[:2] = np.iinfo(np.int64).min
    av = rng.integers(-2**62, 2**62, na).astype(np.int64)
    bv = rng.integers(-2**62, 2**62, nb).astype(np.int64)
    cnt, sa, sb, pair = _brute(ak, av, bk, bv)
    got = oracle.join_agg(ak, [av], bk, [bv])
    assert got == [cnt, sa, sb]
    assert (got[1] + got[2]) % M64 == pair


@pytest.mark.parametrize("fn,P,shift", [("bits", 4, 0), ("bits", 16, 3), ("hash", 8, 0), ("bits", 1, 0)])
def test_partition_decomposition(fn, P, shift):
    rng = np.random.default_rng(7)
    ak = rng.integers(0, 3000, 5000).astype(np.int64)
    bk = rng.integers(0, 4000, 9000).astype(np.int64)
    av = rng.integers(0, 2**32, 5000).astype(np.int64)
    bv = rng.integers(0, 2**32, 9000).astype(np.int64)
    log2p = P.bit_length() - 1
    if fn == "bits":
        ia, ib = oracle.part_ids_bits(ak, shift, log2p), oracle.part_ids_bits(bk, shift, log2p)
    else:
        ia, ib = oracle.part_ids_hash(ak, log2p), oracle.part_ids_hash(bk, log2p)
    whole = oracle.join_agg(ak, [av], bk, [bv])
    tot = [0, 0, 0]
    for p in range(P):
        ma, mb = ia == p, ib == p
        r = oracle.join_agg(ak[ma], [av[ma]], bk[mb], [bv[mb]])
        tot = [(x + y) % M64 for x, y in zip(tot, r)]
    assert tot == whole
    assert whole[0] > 0


def test_recipe_closed_form():
    na, nb = 1 << 16, (1 << 17) + 5
    ak, av = datagen.radix_a(na)
    bk, bv = datagen.radix_b(na, nb)
    assert np.array_equal(np.sort(ak), np.arange(na))      # unique keys: a permutation of [0, n_a)
    a_of_key = np.empty(na, np.uint64)
    a_of_key[ak] = av.astype(np.uint64)
    want = [nb, int(a_of_key[bk].sum(dtype=np.uint64)), int(bv.astype(np.uint64).sum(dtype=np.uint64))]
    assert oracle.join_agg(ak, [av], bk, [bv]) == want
