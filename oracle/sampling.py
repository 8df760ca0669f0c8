"""Graph sampling and the subgraph layout (section 4.1 stage 1; section 4.3 subgraph management).

Sampling: seed nodes are drawn uniformly at random and each seed brings in its
1-hop out-neighbours (the frontier) until the target count is reached.  The
random draw is an input: ``order`` is a permutation of [0, N) and seeds are
taken in that order.  Readings:
* ``seed_expand``: walk ``order``; a seed not yet sampled is added, then its
  out-neighbours in stored order, stopping exactly at ``n_target``;
* ``uniform``: the first ``n_target`` entries of ``order`` (no expansion).

Subgraph layout: unsampled nodes keep their id and a row with out-degree 0,
and every edge into them is removed, so no id remapping is needed.
"""

from __future__ import annotations

import numpy as np


def sample_nodes(rowptr, nbrs, order, n_target: int, mode: str = "seed_expand") -> np.ndarray:
    """Boolean membership mask of the sampled set S, |S| = n_target."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.shape[0] - 1
    if not 0 <= n_target <= n:
        raise ValueError("n_target out of range")
    in_s = np.zeros(n, dtype=bool)
    if mode == "uniform":
        for s in order[:n_target]:
            in_s[int(s)] = True
        return in_s
    if mode != "seed_expand":
        raise ValueError(mode)
    count = 0
    for s in order:
        if count >= n_target:
            break
        s = int(s)
        if in_s[s]:
            continue
        in_s[s] = True
        count += 1
        for v in nbrs[rowptr[s]:rowptr[s + 1]]:
            if count >= n_target:
                break
            v = int(v)
            if not in_s[v]:
                in_s[v] = True
                count += 1
    return in_s


def check_subgraph(rowptr, nbrs, in_s, max_degree: int) -> list:
    """Every violated subgraph invariant, as readable strings (empty list = valid)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.shape[0] - 1
    problems = []
    for u in range(n):
        row = [int(v) for v in nbrs[rowptr[u]:rowptr[u + 1]]]
        if not in_s[u] and row:
            problems.append(f"unsampled node {u} has out-edges")
        if len(row) > max_degree:
            problems.append(f"node {u} degree {len(row)} > {max_degree}")
        if len(set(row)) != len(row):
            problems.append(f"node {u} has duplicate neighbours")
        for v in row:
            if v == u:
                problems.append(f"self loop at {u}")
            elif not 0 <= v < n:
                problems.append(f"edge {u}->{v} out of range")
            elif not in_s[v]:
                problems.append(f"edge {u}->{v} enters an unsampled node")
    return problems


def padded_from_csr(rowptr, nbrs, width: int) -> np.ndarray:
    """[N][width] neighbour table, rows in stored order, padded with -1."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    n = rowptr.shape[0] - 1
    out = np.full((n, width), -1, dtype=np.int64)
    for u in range(n):
        row = nbrs[rowptr[u]:rowptr[u + 1]]
        out[u, :len(row)] = row
    return out


def csr_from_padded(adj):
    """Inverse of padded_from_csr (drops the -1 padding)."""
    adj = np.asarray(adj)
    rowptr = [0]
    flat = []
    for row in adj:
        kept = [int(v) for v in row if v >= 0]
        flat.extend(kept)
        rowptr.append(len(flat))
    return np.asarray(rowptr, dtype=np.int64), np.asarray(flat, dtype=np.int64)
