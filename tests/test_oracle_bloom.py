"""Pins of the oracle's Bloom-filter visited set (section 4.3 variant of Algorithm 1):
the hash definition worked by hand, the reduction to the exact visited set when no
false positive can occur, the closed form when the filter saturates after the entry
points, and hand-built false-positive and same-group cases."""

import itertools

import numpy as np

import oracle
from oracle.bloom import BloomFilter
from synth.data import gmm_points


def _csr(rows):
    rowptr = [0]
    flat = []
    for r in rows:
        flat.extend(r)
        rowptr.append(len(flat))
    return np.asarray(rowptr, dtype=np.int64), np.asarray(flat, dtype=np.int64)


def test_hash_bits_worked_by_hand():
    f = BloomFilter(8)
    assert f.bits(0) == (0, 0)
    # 1 * A: the top byte of each multiplier (0x9E3779B1, 0x85EBCA77)
    assert f.bits(1) == (0x9E, 0x85)
    # 2 * 0x9E3779B1 = 0x1_3C6E_F362 -> 0x3C6EF362 mod 2^32; 2 * 0x85EBCA77 = 0x1_0BD7_94EE
    assert f.bits(2) == (0x3C, 0x0B)
    assert BloomFilter(32).bits(3) == ((3 * 0x9E3779B1) % 2 ** 32, (3 * 0x85EBCA77) % 2 ** 32)


def _small_graph(n=600, dim=10, comps=3, seed=21, R=12):
    from synth.graph import build_graph, padded_to_csr
    X = gmm_points(seed, n, dim, comps)
    rowptr, nbrs = padded_to_csr(build_graph(X, R, device="cpu"))
    return X, rowptr, nbrs


def test_without_false_positives_equals_exact_visited_set():
    # at 2^32 bits each hash is injective on node ids, so a node can only be reported
    # visited if both of its bits were set by other nodes' other hash, which does not
    # happen on this graph: the variant reduces to Algorithm 1 with an exact set
    X, rowptr, nbrs = _small_graph()
    Q = gmm_points(22, 12, 10, 3, stream_offset=1)
    for i, q in enumerate(Q):
        for ef in (8, 40):
            ex = oracle.greedy_search(q, X, rowptr, nbrs, ef, [i, 300 + i])
            bl = oracle.greedy_search(q, X, rowptr, nbrs, ef, [i, 300 + i], bloom_log2=32)
            assert bl["ids"].tolist() == ex["ids"].tolist()
            assert (bl["dists"] == ex["dists"]).all()
            assert (bl["n_exp"], bl["n_dist"]) == (ex["n_exp"], ex["n_dist"])


def test_saturated_filter_keeps_only_the_entry_points():
    # one-bit hashes into 2 bits: once the entry points have set both bits every other
    # node counts as visited, so C is the best ef entries by brute force and every
    # entry in C is expanded without scoring anything
    X, rowptr, nbrs = _small_graph()
    q = gmm_points(23, 1, 10, 3, stream_offset=1)[0]
    entries = [3, 50, 77, 120, 200, 411, 512, 599]
    f = BloomFilter(1)
    for e in entries:
        f.add(e)
    assert f.bits_set == {0, 1}
    for ef in (3, 8, 20):
        r = oracle.greedy_search(q, X, rowptr, nbrs, ef, entries, bloom_log2=1)
        d = oracle.as_f32(((X[entries].astype(np.float64) - q) ** 2).sum(1))
        order = sorted(range(len(entries)), key=lambda j: (d[j], entries[j]))[:ef]
        assert r["ids"].tolist() == [entries[j] for j in order]
        assert r["dists"].tolist() == [float(d[j]) for j in order]
        assert r["n_dist"] == len(entries)
        assert r["n_exp"] == min(ef, len(entries))


def test_false_positive_is_never_scored():
    # a -> b -> c: c's two bits are already set by a and b, so c is skipped even though
    # the exact visited set would score it
    f = BloomFilter(4)
    a, b, c = next((a, b, c) for a, b, c in itertools.permutations(range(1, 40), 3)
                   if set(f.bits(c)) <= set(f.bits(a)) | set(f.bits(b))
                   and not set(f.bits(b)) <= set(f.bits(a)))
    rows = [[] for _ in range(40)]
    rows[a], rows[b] = [b], [c]
    rowptr, nbrs = _csr(rows)
    X = gmm_points(24, 40, 4, 2)
    q = X[c] + 0.01  # c would be the best answer
    ex = oracle.greedy_search(q, X, rowptr, nbrs, 4, [a])
    bl = oracle.greedy_search(q, X, rowptr, nbrs, 4, [a], bloom_log2=4)
    assert sorted(ex["ids"].tolist()) == sorted([a, b, c]) and ex["ids"][0] == c
    assert sorted(bl["ids"].tolist()) == sorted([a, b]) and bl["n_dist"] == 2


def test_one_group_is_tested_before_it_is_marked():
    # x and y share both bits: listed in one group both are scored; met in a later
    # group y counts as visited; an id repeated in one group is scored twice, listed once
    f = BloomFilter(4)
    x, y = next((x, y) for x, y in itertools.combinations(range(1, 200), 2) if f.bits(x) == f.bits(y))
    X = gmm_points(25, 200, 4, 2)
    q = gmm_points(26, 1, 4, 2, stream_offset=1)[0]
    empty = _csr([[] for _ in range(200)])
    r = oracle.greedy_search(q, X, *empty, 8, [x, y], bloom_log2=4)
    assert sorted(r["ids"].tolist()) == sorted([x, y]) and r["n_dist"] == 2
    rows = [[] for _ in range(200)]
    rows[x] = [y]
    r = oracle.greedy_search(q, X, *_csr(rows), 8, [x], bloom_log2=4)
    assert r["ids"].tolist() == [x] and r["n_dist"] == 1
    r = oracle.greedy_search(q, X, *empty, 8, [x, x, x], bloom_log2=4)
    assert r["ids"].tolist() == [x] and r["n_dist"] == 3
    # entry points come in groups of 64: a repeat in the next group counts as visited
    r = oracle.greedy_search(q, X, *empty, 8, [x] + [-1] * 63 + [x], bloom_log2=4)
    assert r["ids"].tolist() == [x] and r["n_dist"] == 1
