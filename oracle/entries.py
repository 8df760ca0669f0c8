"""Fast entry selection (section 5; Algorithm 2; Table 2).

Entry vectors (pivots) are grouped into r coarse clusters of equal size (the
layout EV[r][n/r][d] of Algorithm 2).  Each query is routed to its nearest
centroid and only that cluster's pivots are scored; the best E of them seed
the traversal.  With r = 1 this is brute force over all pivots (section 5,
complexity analysis).

Readings where the paper is silent:
* clustering: Lloyd's k-means in squared L2 on the pivots' reduced vectors,
  seeded from r given distinct pivots, a fixed number of iterations, then a
  balanced assignment that fills buckets of exactly n/r in the order of
  (distance, pivot position, cluster); centroids are the final bucket means.
  Clustering and routing use squared L2 for both metrics; pivot scores use the
  workload metric.
* ties: routing takes the lowest cluster index, entries are ordered by
  (distance, node id).
* E (entries per query) is a parameter; the same value is given to both sides.
* distances that decide routing and the top-E are single-precision values
  (section 6.1): exact, then rounded once to fp32 (``precision="f64"`` keeps fp64).

The bucket contents are "parity unpinned" against the paper (no worked
example exists); they are pinned by the invariants in the tests.
"""

from __future__ import annotations

import numpy as np

from .metric import as_f32, delta_many


def _sqdist(a, b) -> np.ndarray:
    """Squared L2 between every row of a and every row of b, direct form, fp64."""
    out = np.empty((a.shape[0], b.shape[0]))
    for j in range(b.shape[0]):
        diff = a - b[j][None, :]
        out[:, j] = np.einsum("ij,ij->i", diff, diff)
    return out


def balanced_kmeans(P, r: int, init_idx, iters: int = 10):
    """Return (buckets int [r][n/r] of pivot positions, centroids fp64 [r][d])."""
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    if r <= 0 or n % r != 0:
        raise ValueError("pivot count must be a multiple of r")
    cap = n // r
    C = P[np.asarray(init_idx, dtype=np.int64)].copy()
    for _ in range(iters):
        D = _sqdist(P, C)
        assign = np.argmin(D, axis=1)  # first minimum = lowest cluster index
        for c in range(r):
            members = P[assign == c]
            if members.shape[0] > 0:
                C[c] = members.sum(0) / members.shape[0]
    D = _sqdist(P, C)
    p_idx, c_idx = np.meshgrid(np.arange(n), np.arange(r), indexing="ij")
    order = np.lexsort((c_idx.ravel(), p_idx.ravel(), D.ravel()))
    owner = np.full(n, -1, dtype=np.int64)
    size = np.zeros(r, dtype=np.int64)
    for flat in order:
        p, c = divmod(int(flat), r)
        if owner[p] < 0 and size[c] < cap:
            owner[p] = c
            size[c] += 1
    buckets = np.stack([np.nonzero(owner == c)[0] for c in range(r)])
    centroids = np.stack([P[buckets[c]].sum(0) / cap for c in range(r)])
    return buckets, centroids


def route(qr, centroids, precision: str = "f32"):
    """(nearest centroid index, relative gap to the runner-up) for one reduced query."""
    qr = np.asarray(qr, dtype=np.float64)
    d = delta_many(qr, centroids, "l2")
    if precision == "f32":
        d = as_f32(d)
    c = int(np.argmin(d))
    if d.shape[0] < 2:
        return c, np.inf
    s = np.sort(d)
    return c, (s[1] - s[0]) / max(abs(s[1]), 1e-300)


def select_entries(Qr, centroids, buckets, P, pivot_ids, E: int, metric: str = "l2", precision: str = "f32"):
    """Top-E pivots of the routed cluster for each query.

    Returns (entry ids int64 [m][E], distances fp64 [m][E], cluster int [m],
    margin fp64 [m]); rows are padded with (-1, +inf) when a cluster holds
    fewer than E pivots.  ``margin`` is the smallest relative gap among the
    decisions taken for that query (routing and the first E+1 scores).
    """
    Qr = np.asarray(Qr, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    pivot_ids = np.asarray(pivot_ids, dtype=np.int64)
    m = Qr.shape[0]
    ids = np.full((m, E), -1, dtype=np.int64)
    dists = np.full((m, E), np.inf)
    clusters = np.zeros(m, dtype=np.int64)
    margins = np.full(m, np.inf)
    for i in range(m):
        c, gap = route(Qr[i], centroids, precision)
        clusters[i] = c
        members = np.asarray(buckets[c], dtype=np.int64)
        d = delta_many(Qr[i], P[members], metric)
        if precision == "f32":
            d = as_f32(d)
        nid = pivot_ids[members]
        order = np.lexsort((nid, d))
        take = order[:E]
        ids[i, :take.size] = nid[take]
        dists[i, :take.size] = d[take]
        head = d[order[:E + 1]]
        if head.size >= 2:
            rel = np.diff(head) / np.maximum(np.maximum(np.abs(head[1:]), np.abs(head[:-1])), 1e-300)
            gap = min(gap, float(rel.min()))
        margins[i] = gap
    return ids, dists, clusters, margins
