"""Distances and the recall metric (fp64).

* Squared Euclidean distance is the unit of work in the paper's complexity
  analysis (section 5, Table 2) and the distance of Algorithm 1; the square root
  is never taken because it does not change any ranking.
* Inner-product workloads use delta = -<q, x> so that smaller is better
  everywhere (a reading: the paper evaluates Euclidean data and unit-norm
  embeddings, where both orders agree).
* recall@k = |retrieved_k intersect groundtruth_k| / k, averaged over queries
  (section 6.1, Metrics).
* Precision of the search: the paper computes distances in single precision
  (section 6.1, setup).  Where a distance decides an order (Algorithm 1's list,
  the entry top-E, routing), the oracle uses the fp32 value nearest to the exact
  distance: computed in fp64, rounded once (``as_f32``).  The exact kNN of the
  problem definition stays in fp64.
"""

from __future__ import annotations

import numpy as np


def delta(q, x, metric: str = "l2") -> float:
    """Distance between two vectors, fp64, direct form."""
    q = np.asarray(q, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    if metric == "l2":
        diff = q - x
        return float(np.dot(diff, diff))
    if metric == "ip":
        return float(-np.dot(q, x))
    raise ValueError(metric)


def delta_many(q, xs, metric: str = "l2") -> np.ndarray:
    """Distance from q to every row of xs, fp64, direct form."""
    q = np.asarray(q, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    if xs.shape[0] == 0:
        return np.zeros(0)
    if metric == "l2":
        diff = xs - q[None, :]
        return np.einsum("ij,ij->i", diff, diff)
    if metric == "ip":
        return -(xs @ q)
    raise ValueError(metric)


def recall_at_k(found, truth, k: int) -> float:
    """Mean of |found[:k] & truth[:k]| / k over the query rows (section 6.1)."""
    found = np.asarray(found)
    truth = np.asarray(truth)
    total = 0
    for f, t in zip(found, truth):
        f = [int(v) for v in f[:k] if v >= 0]
        total += len(set(f) & set(int(v) for v in t[:k]))
    return total / (k * max(1, truth.shape[0]))


def as_f32(d):
    """Round fp64 distances once to the nearest float32 (returned as fp64 values)."""
    return np.asarray(d, dtype=np.float64).astype(np.float32).astype(np.float64)
