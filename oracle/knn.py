"""Exact top-k by brute force (the problem definition, section 2.1; ground truth of
the recall metric, section 6.1).

Every (query, base) distance is computed directly in fp64 and each row is
ordered by the key (distance, id), so equal distances resolve to the smaller
id.
"""

from __future__ import annotations

import numpy as np

from .metric import delta_many


def exact_knn(X, Q, k: int, metric: str = "l2"):
    """Return (ids int64 [m][k], dists fp64 [m][k]); k is clipped to N."""
    X = np.asarray(X, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = X.shape[0]
    k = min(k, n)
    ids = np.empty((Q.shape[0], k), dtype=np.int64)
    dists = np.empty((Q.shape[0], k), dtype=np.float64)
    all_ids = np.arange(n)
    for i, q in enumerate(Q):
        d = delta_many(q, X, metric)
        order = np.lexsort((all_ids, d))[:k]
        ids[i] = order
        dists[i] = d[order]
    return ids, dists
