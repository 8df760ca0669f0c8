"""Pins of the oracle's expansion-width variant of Algorithm 1 (two unchecked entries
expanded per step; not the paper's algorithm): a hand-worked example where it reaches a
node that width 1 drops, and the exact kNN when the list can hold every node."""

import numpy as np

import oracle
from synth.data import gmm_points


def _csr(rows):
    rowptr = [0]
    flat = []
    for r in rows:
        flat.extend(r)
        rowptr.append(len(flat))
    return np.asarray(rowptr, dtype=np.int64), np.asarray(flat, dtype=np.int64)


def test_hand_example_width_two_expands_an_entry_that_width_one_drops():
    # 1-d points, query at 0: a = 5 (25), b = 6 (36), c = 4 (16), g = 1 (1); a -> c, b -> g.
    # Width 1, ef 2, entries [a, b]: expanding a inserts c, the resize drops b, then c has
    # no out-edge: C = [c, a]; expansions a, c; distances a, b, c.
    # Width 2: a and b are expanded together, c and g inserted, the resize keeps [g, c],
    # both expanded: C = [g, c]; expansions a, b, g, c; distances a, b, c, g.
    a, b, c, g = 0, 1, 2, 3
    X = np.array([[5.0], [6.0], [4.0], [1.0]])
    rowptr, nbrs = _csr([[c], [g], [], []])
    q = np.array([0.0])
    r1 = oracle.greedy_search(q, X, rowptr, nbrs, 2, [a, b])
    assert r1["ids"].tolist() == [c, a] and r1["dists"].tolist() == [16.0, 25.0]
    assert (r1["n_exp"], r1["n_dist"]) == (2, 3)
    r2 = oracle.greedy_search(q, X, rowptr, nbrs, 2, [a, b], width=2)
    assert r2["ids"].tolist() == [g, c] and r2["dists"].tolist() == [1.0, 16.0]
    assert (r2["n_exp"], r2["n_dist"]) == (4, 4)
    assert r2["checked"].all()


def test_width_two_with_a_list_of_every_node_is_exact_knn():
    from synth.graph import build_graph, padded_to_csr
    X = gmm_points(31, 400, 8, 3)
    rowptr, nbrs = padded_to_csr(build_graph(X, 10, device="cpu"))
    Q = gmm_points(32, 8, 8, 3, stream_offset=1)
    gt, _ = oracle.exact_knn(X, Q, 10)
    for i, q in enumerate(Q):
        for bloom in (None, 32):
            r = oracle.greedy_search(q, X, rowptr, nbrs, X.shape[0], [i], precision="f64", width=2,
                                     bloom_log2=bloom)
            # the repaired graph reaches every node; with the Bloom filter a node met in both
            # rows of one step is scored twice (both are tested before either is marked)
            assert r["n_dist"] == X.shape[0] if bloom is None else r["n_dist"] >= X.shape[0]
            assert r["ids"].size == X.shape[0] and r["ids"][:10].tolist() == gt[i].tolist()
