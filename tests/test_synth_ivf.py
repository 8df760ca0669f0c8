"""The IVF-restricted graph builder used for the 10^7-row workloads, pinned on the CPU.

With every list probed, each row's probe set is the whole base set, so the builder must
return exactly the exact builder's graph (same candidates, same pruning, same reverse
step, same repair).  With fewer lists probed the graph is approximate but must still be
a valid fixture: degree at most R, no self loops or repeated ids, rows ordered by
(distance, id), every row reachable from the medoid."""

import numpy as np
import pytest
import torch

from synth.data import gmm_points
from synth.graph import build_graph, medoid_of
from synth.ivf import build_graph_ivf, coarse_kmeans, ivf_candidates, reached_gpu
from synth.knn import exact_knn


@pytest.fixture(scope="module")
def pts():
    return gmm_points(7, 3000, 16, 20)


def test_all_lists_probed_equals_the_exact_builder(pts):
    exact = build_graph(pts, 12, device="cpu")
    ivf = build_graph_ivf(pts, 12, n_lists=8, nprobe=8, device="cpu")
    assert (exact == ivf).all()


def test_candidates_with_every_list_are_the_exact_knn(pts):
    x32 = torch.as_tensor(pts)
    cen, assign = coarse_kmeans(x32, 6, seed=3)
    ids, d = ivf_candidates(x32, x32.double(), cen, assign, nprobe=6, cand=10)
    ref, ref_d = exact_knn(pts, None, 10, "l2", device="cpu", exclude_self=True)
    assert (ids.numpy() == ref).all()
    assert np.array_equal(d.numpy(), ref_d)


def test_partial_probe_gives_a_valid_connected_graph(pts):
    R = 12
    adj = build_graph_ivf(pts, R, n_lists=16, nprobe=3, device="cpu")
    n = pts.shape[0]
    assert adj.shape == (n, R)
    x = pts.astype(np.float64)
    for u in range(n):
        row = adj[u][adj[u] >= 0]
        assert u not in row
        assert len(set(row.tolist())) == len(row)
        # padding only at the end; rows ordered by (distance, id)
        assert (adj[u][len(row):] == -1).all()
        d = ((x[row] - x[u]) ** 2).sum(1)
        keys = list(zip(d.tolist(), row.tolist()))
        assert keys == sorted(keys)
    seen = reached_gpu(torch.as_tensor(adj).long(), medoid_of(pts)).numpy()
    assert seen.all()
    # an approximate graph, but most rows keep the exact builder's neighbours
    exact = build_graph(pts, R, device="cpu")
    assert (adj == exact).all(1).mean() > 0.8


def test_breadth_first_reachability_on_a_hand_built_graph():
    adj = torch.tensor([[1, -1], [2, -1], [0, 1], [4, -1], [-1, -1]])
    assert reached_gpu(adj, 0).tolist() == [True, True, True, False, False]
    assert reached_gpu(adj, 3).tolist() == [False, False, False, True, True]


def test_repair_path_matches_the_exact_builder():
    # degree 3 on well separated blobs leaves parts unreachable until the repair links them
    from synth.graph import _reached_from, add_reverse, rng_prune
    X = gmm_points(11, 2000, 8, 40)
    x64 = torch.as_tensor(X).double()
    ids, d = exact_knn(X, None, 3, "l2", device="cpu", exclude_self=True)
    raw = add_reverse(x64, rng_prune(x64, torch.as_tensor(ids), torch.as_tensor(d), 3), 3).numpy()
    assert not _reached_from(raw, medoid_of(X)).all()
    exact = build_graph(X, 3, device="cpu")
    ivf = build_graph_ivf(X, 3, n_lists=4, nprobe=4, device="cpu")
    assert (exact == ivf).all()
    assert reached_gpu(torch.as_tensor(ivf).long(), medoid_of(X)).all()
