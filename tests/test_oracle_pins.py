"""Pins for the CPU oracle: hand-worked examples, closed forms, invariants and
special cases that reduce to library routines.  None of these compare the
oracle with itself; each is chosen so that a plausible slip (a dropped term,
a wrong sign or index, a transposed operand, a missing visited mark, a wrong
tie-break) fails at least one of them.
"""

import json
import os
import random

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle.sampling import csr_from_padded
from synth.data import gmm_points, make_rng


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _csr(rows):
    rowptr = [0]
    flat = []
    for r in rows:
        flat.extend(r)
        rowptr.append(len(flat))
    return np.asarray(rowptr, dtype=np.int64), np.asarray(flat, dtype=np.int64)


# ---------------------------------------------------------------- metric / knn

def test_knn_and_recall_hand_examples(golden_dir):
    g = _load(golden_dir, "knn_recall_examples.json")
    ids, d = oracle.exact_knn(np.array(g["knn"]["points"]), np.array([g["knn"]["query"]]), 5)
    assert ids[0].tolist() == g["knn"]["ids"]
    np.testing.assert_allclose(d[0], g["knn"]["dists"], rtol=0, atol=1e-12)
    r = g["recall"]
    assert oracle.recall_at_k(np.array(r["found"]), np.array(r["truth"]), r["k"]) == pytest.approx(r["value"])


def test_knn_matches_scipy_argsort():
    X = gmm_points(11, 400, 12, 4)
    Q = gmm_points(12, 30, 12, 4, stream_offset=1)
    ids, d = oracle.exact_knn(X, Q, 7)
    full = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    for i in range(Q.shape[0]):
        ref = np.argsort(full[i], kind="stable")[:7]
        assert ids[i].tolist() == ref.tolist()
        np.testing.assert_allclose(d[i], full[i][ref], rtol=1e-12)
    # inner product: smallest -<q,x> first
    ids_ip, _ = oracle.exact_knn(X, Q, 5, "ip")
    ref_ip = np.argsort(-(Q.astype(np.float64) @ X.astype(np.float64).T), axis=1, kind="stable")[:, :5]
    assert (ids_ip == ref_ip).all()


def test_recall_of_truth_is_one():
    X = gmm_points(3, 200, 8, 3)
    ids, _ = oracle.exact_knn(X, X[:20], 10)
    assert oracle.recall_at_k(ids, ids, 10) == 1.0


# ---------------------------------------------------------------- projection

def test_projection_hand_example(golden_dir):
    g = _load(golden_dir, "projection_axes.json")
    V, w, mu = oracle.fit_projection(np.array(g["points"]), g["d_r"], center=g["center"])
    np.testing.assert_allclose(w, g["eigenvalues"], atol=1e-12)
    np.testing.assert_allclose(V, g["V"], atol=1e-12)
    np.testing.assert_allclose(mu, g["mean"], atol=1e-12)


@pytest.mark.parametrize("center", [True, False])
def test_projection_orthonormal_and_svd(center):
    X = gmm_points(5, 500, 24, 6) + 3.0  # non-zero mean: centring matters
    V, w, mu = oracle.fit_projection(X, 24, center=center)
    np.testing.assert_allclose(V.T @ V, np.eye(24), atol=1e-12)
    X64 = X.astype(np.float64)
    A = X64 - X64.mean(0) if center else X64
    s = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(w, s ** 2 / X.shape[0], rtol=1e-10, atol=1e-12)


def test_full_rank_projection_preserves_distances():
    X = gmm_points(6, 300, 16, 4)
    V, _, _ = oracle.fit_projection(X, 16)
    Y = oracle.project(X, V)
    a = cdist(X.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    b = cdist(Y, Y, "sqeuclidean")
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-9)
    # inner products too
    np.testing.assert_allclose(Y @ Y.T, X.astype(np.float64) @ X.astype(np.float64).T, rtol=1e-12, atol=1e-9)


def test_primary_plus_residual_split():
    X = gmm_points(7, 300, 20, 5)
    V, _, _ = oracle.fit_projection(X, 20)
    q, x = X[0].astype(np.float64), X[1:].astype(np.float64)
    prim = oracle.project(x, V[:, :8])
    res = oracle.project(x, V[:, 8:])
    qp, qs = oracle.project(q[None], V[:, :8])[0], oracle.project(q[None], V[:, 8:])[0]
    full = ((x - q) ** 2).sum(1)
    split = ((prim - qp) ** 2).sum(1) + ((res - qs) ** 2).sum(1)
    np.testing.assert_allclose(split, full, rtol=1e-12)


def test_eckart_young_residual_energy():
    X = gmm_points(8, 600, 16, 5) + 1.5
    V, w, mu = oracle.fit_projection(X, 6)
    A = X.astype(np.float64) - mu
    resid = A - (A @ V) @ V.T
    np.testing.assert_allclose((resid ** 2).sum(), X.shape[0] * w[6:].sum(), rtol=1e-9)
    # Ky Fan: captured variance equals the top eigenvalues' sum
    C = A.T @ A / X.shape[0]
    np.testing.assert_allclose(np.trace(V.T @ C @ V), w[:6].sum(), rtol=1e-10)


# ---------------------------------------------------------------- traversal

def test_traverse_hand_examples(golden_dir):
    g = _load(golden_dir, "traverse_examples.json")
    for c in g["cases"]:
        rowptr, nbrs = _csr(c["rows"])
        r = oracle.greedy_search(np.array(c["query"]), np.array(c["points"], dtype=np.float64),
                                 rowptr, nbrs, c["ef"], c["entries"])
        assert r["ids"].tolist() == c["ids"], c["name"]
        np.testing.assert_allclose(r["dists"], c["dists"], rtol=1e-7, atol=0, err_msg=c["name"])
        assert r["n_exp"] == c["n_exp"], c["name"]
        assert r["n_dist"] == c["n_dist"], c["name"]


def test_near_tie_margin_hand_examples(golden_dir):
    """The margin that excuses a divergence from the oracle, worked by hand: each case
    isolates one kind of decision (initial resize, choice of the node to expand, resize
    after an expansion, order of the final list, inner-product keys, width 2, an exact
    tie), so a gap taken at the wrong position or between the wrong keys fails one."""
    g = _load(golden_dir, "margin_examples.json")
    for c in g["traverse"]:
        rowptr, nbrs = _csr(c["rows"])
        r = oracle.greedy_search(np.array(c["query"]), np.array(c["points"], dtype=np.float64), rowptr, nbrs,
                                 c["ef"], c["entries"], c["metric"], width=c["width"])
        assert r["ids"].tolist() == c["ids"], c["name"]
        assert (r["n_exp"], r["n_dist"]) == (c["n_exp"], c["n_dist"]), c["name"]
        num, den = c["margin"]
        assert r["margin"] == num / den, (c["name"], r["margin"], num / den)
    rt = g["route"]
    cent = np.array(rt["centroids"], dtype=np.float64)
    for c in rt["cases"]:
        cl, gap = oracle.route(np.array(c["query"]), cent)
        assert cl == c["cluster"], c["name"]
        assert gap == c["gap"][0] / c["gap"][1], (c["name"], gap)
    se = g["select_entries"]
    P = np.array(se["pivots"], dtype=np.float64)
    for c in se["cases"]:
        ids, _, cl, margin = oracle.select_entries(np.array([c["query"]]), np.array(se["centroids"]),
                                                   np.array(se["buckets"]), P, se["pivot_ids"], c["E"])
        assert int(cl[0]) == c["cluster"] and ids[0].tolist() == c["entry_ids"], c["name"]
        assert margin[0] == c["margin"][0] / c["margin"][1], (c["name"], margin[0])


def _small_graph(n=600, dim=10, comps=3, seed=21, R=12):
    from synth.graph import build_graph, padded_to_csr
    X = gmm_points(seed, n, dim, comps)
    adj = build_graph(X, R, device="cpu")
    rowptr, nbrs = padded_to_csr(adj)
    return X, rowptr, nbrs


def test_large_ef_returns_exact_knn_of_reachable_set():
    X, rowptr, nbrs = _small_graph()
    Q = gmm_points(22, 15, 10, 3, stream_offset=1)
    gt, gd = oracle.exact_knn(X, Q, 10)
    for i, q in enumerate(Q):
        r = oracle.greedy_search(q, X, rowptr, nbrs, X.shape[0], [0], precision="f64")
        assert r["n_dist"] == X.shape[0]  # the repaired graph reaches every node
        assert r["ids"][:10].tolist() == gt[i].tolist()
        np.testing.assert_allclose(r["dists"][:10], gd[i], rtol=1e-12)
        # in the paper's single precision the distances are the fp32-rounded exact ones
        r32 = oracle.greedy_search(q, X, rowptr, nbrs, X.shape[0], [0])
        assert (r32["dists"][:10] == gd[i].astype(np.float32).astype(np.float64)).all()


def test_complete_graph_one_expansion_sees_everything():
    X = gmm_points(23, 40, 5, 2)
    rows = [[v for v in range(40) if v != u] for u in range(40)]
    rowptr, nbrs = _csr(rows)
    q = gmm_points(24, 1, 5, 2, stream_offset=1)[0]
    gt, _ = oracle.exact_knn(X, q[None], 8)
    r = oracle.greedy_search(q, X, rowptr, nbrs, 8, [17])
    assert r["n_dist"] == 40
    assert r["ids"].tolist() == gt[0].tolist()
    assert r["checked"].all()


def _bounded_insertion_search(q, X, rowptr, nbrs, ef, entries):
    """Independent formulation: a bounded sorted insertion that never lets C exceed ef."""
    import bisect
    q = q.astype(np.float64)
    seen = set()
    keys, checked = [], {}

    def offer(v):
        d = float(((X[v].astype(np.float64) - q) ** 2).sum())
        key = (d, v)
        if len(keys) == ef and key > keys[-1]:
            return
        bisect.insort(keys, key)
        checked[v] = False
        if len(keys) > ef:
            keys.pop()
    for e in entries:
        if e not in seen:
            seen.add(e)
            offer(e)
    steps = 0
    while True:
        u = next((k[1] for k in keys if not checked[k[1]]), None)
        if u is None:
            break
        checked[u] = True
        steps += 1
        for v in nbrs[rowptr[u]:rowptr[u + 1]]:
            v = int(v)
            if v not in seen:
                seen.add(v)
                offer(v)
    return [k[1] for k in keys], steps, len(seen)


def test_insert_then_resize_equals_bounded_insertion_and_row_order_free():
    X, rowptr, nbrs = _small_graph(seed=31)
    Q = gmm_points(32, 12, 10, 3, stream_offset=1)
    rnd = random.Random(5)
    shuffled = nbrs.copy()
    for u in range(len(rowptr) - 1):
        seg = shuffled[rowptr[u]:rowptr[u + 1]].tolist()
        rnd.shuffle(seg)
        shuffled[rowptr[u]:rowptr[u + 1]] = seg
    for ef in (1, 4, 16, 40):
        for i, q in enumerate(Q):
            ent = [i * 7 % 600, (i * 13 + 5) % 600]
            a = oracle.greedy_search(q, X, rowptr, nbrs, ef, ent)
            ids, steps, nd = _bounded_insertion_search(q, X, rowptr, nbrs, ef, ent)
            assert a["ids"].tolist() == ids
            assert a["n_exp"] == steps and a["n_dist"] == nd
            assert a["n_exp"] <= a["n_dist"]
            assert a["n_dist"] == len(a["visited"])
            b = oracle.greedy_search(q, X, rowptr, shuffled, ef, ent)
            assert b["ids"].tolist() == a["ids"].tolist()


def test_forgetting_visited_nodes_outside_c_does_not_change_result():
    """Design property used by the GPU kernel: a visited cache that may forget
    nodes (but never reports an unvisited node as visited), combined with
    de-duplication against C, reproduces Algorithm 1 exactly."""
    X, rowptr, nbrs = _small_graph(seed=41)
    Q = gmm_points(42, 10, 10, 3, stream_offset=1)
    for ef in (2, 8, 32):
        for q in Q:
            ref = oracle.greedy_search(q, X, rowptr, nbrs, ef, [3, 300])
            q64 = q.astype(np.float64)
            cache = set()
            C = []  # [(d, id), checked]

            def ins(cands):
                nonlocal C
                for v in cands:
                    d = float(((X[v].astype(np.float64) - q64) ** 2).sum())
                    if any(c[0][1] == v for c in C):
                        continue  # duplicate of a member of C
                    C.append([(d, v), False])
                C.sort(key=lambda c: c[0])
                C = C[:ef]
            ins([3, 300])
            cache.update([3, 300])
            steps = 0
            while True:
                pos = next((i for i, c in enumerate(C) if not c[1]), None)
                if pos is None:
                    break
                C[pos][1] = True
                u = C[pos][0][1]
                steps += 1
                new = [int(v) for v in nbrs[rowptr[u]:rowptr[u + 1]] if int(v) not in cache]
                cache.update(new)
                ins(new)
                if steps % 3 == 0:
                    cache = set()  # forget everything
            assert [c[0][1] for c in C] == ref["ids"].tolist()
            assert steps == ref["n_exp"]


# ---------------------------------------------------------------- sampling / subgraph

def test_sampling_hand_examples(golden_dir):
    g = _load(golden_dir, "sampling_examples.json")
    rowptr, nbrs = _csr(g["rows"])
    for c in g["cases"]:
        s = oracle.sample_nodes(rowptr, nbrs, np.array(g["order"]), c["n_target"], c["mode"])
        assert np.nonzero(s)[0].tolist() == c["members"], c


def test_sampling_counts_and_determinism():
    X, rowptr, nbrs = _small_graph(seed=51)
    n = X.shape[0]
    order = make_rng(9, 0).permutation(n)
    for mode in ("uniform", "seed_expand"):
        for target in (0, 1, 150, n):
            s = oracle.sample_nodes(rowptr, nbrs, order, target, mode)
            assert s.sum() == target
            assert (s == oracle.sample_nodes(rowptr, nbrs, order, target, mode)).all()
    u = oracle.sample_nodes(rowptr, nbrs, order, 150, "uniform")
    assert set(np.nonzero(u)[0]) == set(order[:150].tolist())


def test_subgraph_invariants_and_detection():
    from synth.graph import build_subgraph_csr
    X, rowptr, nbrs = _small_graph(seed=61)
    order = make_rng(10, 0).permutation(X.shape[0])
    s = oracle.sample_nodes(rowptr, nbrs, order, 150, "seed_expand")
    sr, sn = build_subgraph_csr(X, s, 12, device="cpu")
    assert oracle.check_subgraph(sr, sn, s, 12) == []
    # a planted edge into an unsampled node is reported
    bad = sn.copy()
    u = int(np.nonzero(s)[0][0])
    outside = int(np.nonzero(~s)[0][0])
    bad[sr[u]] = outside
    assert any("unsampled" in p for p in oracle.check_subgraph(sr, bad, s, 12))
    # rho = 1: every node sampled, the subgraph is the full graph
    full = oracle.sample_nodes(rowptr, nbrs, order, X.shape[0], "seed_expand")
    assert full.all()


# ---------------------------------------------------------------- entry selection

def test_entries_hand_example(golden_dir):
    g = _load(golden_dir, "entries_example.json")
    P = np.array(g["pivots"], dtype=np.float64)
    b, c = oracle.balanced_kmeans(P, g["r"], g["init"], g["iters"])
    assert b.tolist() == g["buckets"]
    np.testing.assert_allclose(c, g["centroids"], atol=1e-12)
    ids, d, cl, _ = oracle.select_entries(np.array([g["query"]]), c, b, P, g["pivot_ids"], g["E"])
    assert int(cl[0]) == g["cluster"]
    assert ids[0].tolist() == g["entry_ids"]
    np.testing.assert_allclose(d[0], g["entry_dists"], atol=1e-12)


def test_balanced_buckets_are_equal_and_disjoint():
    P = gmm_points(71, 512, 8, 7)
    init = make_rng(3, 1).choice(512, 32, replace=False)
    b, c = oracle.balanced_kmeans(P, 32, init)
    assert b.shape == (32, 16)
    assert sorted(b.ravel().tolist()) == list(range(512))
    np.testing.assert_allclose(c, np.stack([P[row].astype(np.float64).mean(0) for row in b]), rtol=1e-12)
    b2, _ = oracle.balanced_kmeans(P, 32, init)
    assert (b == b2).all()


def test_one_cluster_is_brute_force_over_pivots():
    P = gmm_points(72, 96, 6, 3)
    Q = gmm_points(73, 20, 6, 3, stream_offset=1)
    pid = np.arange(1000, 1096)
    b, c = oracle.balanced_kmeans(P, 1, [0])
    ids, d, cl, _ = oracle.select_entries(Q, c, b, P, pid, 10)
    # single-precision keys: the exact distance rounded once to fp32, ties by node id
    full = cdist(Q.astype(np.float64), P.astype(np.float64), "sqeuclidean").astype(np.float32)
    for i in range(Q.shape[0]):
        ref = np.lexsort((pid, full[i]))[:10]
        assert ids[i].tolist() == (pid[ref]).tolist()
        assert (d[i] == full[i][ref]).all()
    ids64, d64, _, _ = oracle.select_entries(Q, c, b, P, pid, 10, precision="f64")
    full64 = cdist(Q.astype(np.float64), P.astype(np.float64), "sqeuclidean")
    for i in range(Q.shape[0]):
        ref = np.argsort(full64[i], kind="stable")[:10]
        assert ids64[i].tolist() == (pid[ref]).tolist()
        np.testing.assert_allclose(d64[i], full64[i][ref], rtol=1e-12)


def test_fes_work_matches_complexity_table():
    """Table 2, FES (general): m*n*d/r multiply-adds when buckets are equal."""
    m, n, d, r = 20, 64, 6, 4
    P = gmm_points(74, n, d, 4)
    Q = gmm_points(75, m, d, 4, stream_offset=1)
    b, c = oracle.balanced_kmeans(P, r, [0, 1, 2, 3])
    _, _, cl, _ = oracle.select_entries(Q, c, b, P, np.arange(n), 4)
    scored = sum(len(b[k]) for k in cl) * d
    assert scored == m * n * d // r


# ---------------------------------------------------------------- stages 2 and 3

def test_stages_hand_example(golden_dir):
    g = _load(golden_dir, "stages_example.json")
    X = np.array(g["points"], dtype=np.float64)
    q = np.array(g["query"], dtype=np.float64)
    sr, sn = _csr(g["sub_rows"])
    fr, fn = _csr(g["full_rows"])
    r = oracle.refine(q, X, sr, sn, g["beam"], g["ef_cpu"], steps=g["steps"])
    assert r["ids"].tolist() == g["refine_ids"]
    np.testing.assert_allclose(r["dists"], g["refine_dists"], atol=1e-12)
    assert sorted(r["visited"]) == g["refine_visited"]
    assert r["n_dist"] == g["refine_n_dist"]
    ids, d, f = oracle.final_traversal(q, X, fr, fn, r["ids"], r["dists"], r["visited"], g["ef_cpu"], g["k"])
    assert ids.tolist() == g["final_ids"]
    np.testing.assert_allclose(d, g["final_dists"], atol=1e-12)
    assert f["n_exp"] == g["final_n_exp"] and f["n_dist"] == g["final_n_dist"]


def test_pipeline_margin_hand_example(golden_dir):
    """The whole search's margin combines the entry cut with every stage's decisions."""
    g = _load(golden_dir, "pipeline_margin_example.json")
    X = np.array(g["points"], dtype=np.float64)
    V = np.array(g["V"], dtype=np.float64)
    sr, sn = _csr(g["sub_rows"])
    fr, fn = _csr(g["full_rows"])
    P = X[g["pivot_ids"]]
    for c in g["cases"]:
        ids, d, cnt, margin = oracle.pipeline(np.array([g["query"]]), X, V, fr, fn, sr, sn, X @ V,
                                              np.array(g["centroids"]), np.array(g["buckets"]), P, g["pivot_ids"],
                                              k=g["k"], ef_gpu=g["ef_gpu"], ef_cpu=g["ef_cpu"], E=g["E"],
                                              use_gpu_stage=c["use_gpu_stage"], with_margin=True)
        assert ids[0].tolist() == c["ids"] and d[0].tolist() == c["dists"], c["name"]
        assert cnt[0].tolist() == c["counters"], (c["name"], cnt[0])
        assert margin[0] == c["margin"][0] / c["margin"][1], (c["name"], margin[0])
        # the same search started from given reduced queries (here q V itself)
        ids2, _, _, m2 = oracle.pipeline(np.array([g["query"]]), X, V, fr, fn, sr, sn, X @ V,
                                         np.array(g["centroids"]), np.array(g["buckets"]), P, g["pivot_ids"],
                                         k=g["k"], ef_gpu=g["ef_gpu"], ef_cpu=g["ef_cpu"], E=g["E"],
                                         use_gpu_stage=c["use_gpu_stage"], with_margin=True,
                                         Qr=np.array([g["query"]]) @ V)
        assert ids2[0].tolist() == c["ids"] and m2[0] == margin[0]


def test_refine_without_steps_is_a_rerank_by_full_distance():
    X, rowptr, nbrs = _small_graph(seed=81)
    q = gmm_points(82, 1, 10, 3, stream_offset=1)[0]
    beam = [5, 99, 17, 250, -1]
    r = oracle.refine(q, X, rowptr, nbrs, beam, 3, steps=0)
    full = cdist(q[None].astype(np.float64), X[[5, 99, 17, 250]].astype(np.float64), "sqeuclidean")[0]
    full = full.astype(np.float32)  # single-precision keys, rounded once
    order = np.argsort(full, kind="stable")[:3]
    assert r["ids"].tolist() == [[5, 99, 17, 250][i] for i in order]
    assert (r["dists"] == full[order]).all()


def test_graceful_degradation_is_plain_greedy_search_and_exact_at_large_ef():
    X, rowptr, nbrs = _small_graph(seed=91)
    n = X.shape[0]
    Q = gmm_points(92, 6, 10, 3, stream_offset=1)
    V, _, _ = oracle.fit_projection(X, 4)
    Xr = oracle.project(X, V)
    P_ids = np.arange(0, 64)
    b, c = oracle.balanced_kmeans(Xr[P_ids], 2, [0, 1])
    gt, _ = oracle.exact_knn(X, Q, 10)
    ids, _, cnt = oracle.pipeline(Q, X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids,
                                  k=10, ef_gpu=16, ef_cpu=n, E=8, use_gpu_stage=False)
    assert (ids == gt).all()
    ids2, _, _ = oracle.pipeline(Q, X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids,
                                 k=10, ef_gpu=16, ef_cpu=n, E=8)
    assert (ids2 == gt).all()


def test_gpu_only_special_case_is_exact_knn_with_every_node_and_full_rank():
    # every node sampled (the subgraph is the full graph), d_r = D, and a list that holds
    # every node: stage 1 alone finds all of them and the best k by full distance are the
    # exact k nearest neighbours, with or without the refinement steps
    X, rowptr, nbrs = _small_graph(seed=93)
    n, D = X.shape
    Q = gmm_points(94, 6, 10, 3, stream_offset=1)
    V, _, _ = oracle.fit_projection(X, D)
    Xr = oracle.project(X, V)
    P_ids = np.arange(0, 64)
    b, c = oracle.balanced_kmeans(Xr[P_ids], 2, [0, 1])
    gt, gd = oracle.exact_knn(X, Q, 10)
    for refine in (False, True):
        ids, d, cnt = oracle.pipeline(Q, X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids,
                                      k=10, ef_gpu=n, ef_cpu=n, E=8, use_refine=refine, use_final=False)
        assert (ids == gt).all()
        assert (d == gd.astype(np.float32).astype(np.float64)).all()
        assert (cnt[:, 0] == n).all() and (cnt[:, 2] == 0).all()


def test_fixed_entries_pipeline_is_exact_at_large_ef_and_equals_fes_for_its_own_entries():
    # without entry selection every query starts from the same predefined nodes; on a
    # connected graph a list that holds every node still returns the exact kNN, with and
    # without the GPU stage; and a query given its own FES entries as the fixed set gets
    # the FES pipeline's result
    X, rowptr, nbrs = _small_graph(seed=95)
    n = X.shape[0]
    Q = gmm_points(96, 5, 10, 3, stream_offset=1)
    V, _, _ = oracle.fit_projection(X, 4)
    Xr = oracle.project(X, V)
    P_ids = np.arange(0, 64)
    b, c = oracle.balanced_kmeans(Xr[P_ids], 2, [0, 1])
    gt, _ = oracle.exact_knn(X, Q, 10)
    for gpu in (True, False):
        ids, _, _ = oracle.pipeline(Q, X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids, k=10,
                                    ef_gpu=n, ef_cpu=n, E=1, use_gpu_stage=gpu, fixed_entries=[7])
        assert (ids == gt).all()
    Qr = oracle.as_f32(oracle.project(Q, V))
    ent, _, _, _ = oracle.select_entries(Qr, c, b, Xr[P_ids], P_ids, 4)
    for i in range(Q.shape[0]):
        a = oracle.pipeline(Q[i:i + 1], X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids, k=5,
                            ef_gpu=8, ef_cpu=8, E=4)
        f = oracle.pipeline(Q[i:i + 1], X, V, rowptr, nbrs, rowptr, nbrs, Xr, c, b, Xr[P_ids], P_ids, k=5,
                            ef_gpu=8, ef_cpu=8, E=4, fixed_entries=ent[i])
        assert (a[0] == f[0]).all() and (a[1] == f[1]).all() and (a[2] == f[2]).all()
