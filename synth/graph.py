"""Proximity-graph fixtures standing in for the externally trained graph index.

Recipe (the paper reuses a FAISS-built HNSW base layer; FAISS is not available
here, so a graph of the same kind is built from scratch):

1. exact ``cand``-NN of every node (fp64 order, ties by id);
2. neighbour-selection heuristic of HNSW (relative-neighbourhood pruning): scan
   candidates nearest first, drop ``c`` if an already kept ``s`` is closer to
   ``c`` than the node itself, stop at ``R`` kept;
3. reverse edges are added, each node's union of forward and (nearest ``R``)
   reverse candidates is pruned again with the same rule when it exceeds ``R``;
4. connectivity repair: nodes not reachable from the medoid are hung off the
   nearest reachable node that still has a free slot (and linked back when the
   new node has room), so every node is reachable from the medoid.

Node sampling and the subgraph's reconnection use the same builder on the
sampled rows only; the result is stored over all N rows with unsampled rows
empty.  Rows are sorted by (distance, id).
"""

from __future__ import annotations

import numpy as np
import torch
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import breadth_first_order, connected_components

from .knn import exact_knn, pick_device


def _pair_dist64(vecs: torch.Tensor) -> torch.Tensor:
    """Squared L2 between all candidate pairs, [b][c][c] fp64."""
    nrm = (vecs ** 2).sum(-1)
    g = torch.bmm(vecs, vecs.transpose(1, 2).contiguous())
    return (nrm[:, :, None] + nrm[:, None, :] - 2.0 * g).clamp(min=0.0)


@torch.no_grad()
def rng_prune(x64: torch.Tensor, cand: torch.Tensor, cdist: torch.Tensor, R: int,
              keep_all_if_fits: bool = False, chunk: int = 0) -> torch.Tensor:
    """HNSW-style selection over sorted candidate rows; returns kept ids [n][R] (-1 pad).
    Rows are processed in chunks (0: sized so that a chunk's gathered vectors take about
    1 GiB on a GPU, 8,192 rows on the CPU); every row is decided on its own."""
    n, c = cand.shape
    if chunk <= 0:
        chunk = 8192 if cand.device.type != "cuda" else \
            max(8192, min(1 << 16, (1 << 30) // max(1, c * x64.shape[1] * 8)))
    out = torch.full((n, R), -1, dtype=torch.int64, device=cand.device)
    for a in range(0, n, chunk):
        ci = cand[a:a + chunk]
        cd = cdist[a:a + chunk]
        b = ci.shape[0]
        valid = ci >= 0
        if keep_all_if_fits:
            cnt = valid.sum(1)
        vecs = x64[ci.clamp(min=0)]
        P = _pair_dist64(vecs)
        keep = torch.zeros((b, c), dtype=torch.bool, device=ci.device)
        count = torch.zeros(b, dtype=torch.int64, device=ci.device)
        for i in range(c):
            blocked = ((P[:, i, :] < cd[:, i:i + 1]) & keep).any(1)
            take = valid[:, i] & ~blocked & (count < R)
            if keep_all_if_fits:
                take = take | (valid[:, i] & (cnt <= R))
            keep[:, i] = take
            count += take.long()
        # compact kept ids preserving order
        pos = torch.cumsum(keep.long(), 1) - 1
        rows = torch.arange(b, device=ci.device)[:, None].expand(b, c)
        sel = keep & (pos < R)
        blk = torch.full((b, R), -1, dtype=torch.int64, device=ci.device)
        blk[rows[sel], pos[sel]] = ci[sel]
        out[a:a + b] = blk
    return out


@torch.no_grad()
def add_reverse(x64: torch.Tensor, fwd: torch.Tensor, R: int, block: int = 1 << 22) -> torch.Tensor:
    """Every row's forward neighbours united with the rows that point to it, cut to the
    nearest 2R by (fp64 distance, id) and re-pruned to R (rows holding at most R keep all).
    The proposals are gathered one block of target rows at a time, so that memory stays
    bounded at 10^8 rows."""
    dev = fwd.device
    n = fwd.shape[0]
    width = 2 * R
    pairs = max(1 << 16, (1 << 31) // (8 * x64.shape[1]))  # ~2 GiB per gathered operand
    out = torch.full((n, R), -1, dtype=torch.int64, device=dev)
    for a in range(0, n, block):
        b = min(n, a + block)
        nb_ = b - a
        f = fwd[a:b]
        fm = f >= 0
        node_f = torch.arange(a, b, device=dev)[:, None].expand_as(f)[fm]
        nbr_f = f[fm]
        # reverse proposals: the sources u of edges u -> v with v in [a, b)
        hit = (fwd >= a) & (fwd < b)
        src, col = torch.nonzero(hit, as_tuple=True)
        node_r = fwd[src, col]
        del hit, col
        key = torch.unique(torch.cat([node_f - a, node_r - a]) * n + torch.cat([nbr_f, src]))
        del node_f, nbr_f, node_r, src
        node, nbr = key // n + a, key % n
        del key
        dist = torch.empty(node.shape[0], dtype=torch.float64, device=dev)
        for p in range(0, node.shape[0], pairs):
            dist[p:p + pairs] = ((x64[node[p:p + pairs]] - x64[nbr[p:p + pairs]]) ** 2).sum(-1)
        # group by node, ascending (dist, id)
        o = torch.argsort(nbr, stable=True)
        node, nbr, dist = node[o], nbr[o], dist[o]
        o = torch.argsort(dist, stable=True)
        node, nbr, dist = node[o], nbr[o], dist[o]
        o = torch.argsort(node, stable=True)
        node, nbr, dist = node[o], nbr[o], dist[o]
        counts = torch.bincount(node - a, minlength=nb_)
        starts = torch.cumsum(counts, 0) - counts
        rank = torch.arange(node.shape[0], device=dev) - starts[node - a]
        sel = rank < width
        cand = torch.full((nb_, width), -1, dtype=torch.int64, device=dev)
        cd = torch.full((nb_, width), float("inf"), dtype=torch.float64, device=dev)
        cand[node[sel] - a, rank[sel]] = nbr[sel]
        cd[node[sel] - a, rank[sel]] = dist[sel]
        out[a:b] = rng_prune(x64, cand, cd, R, keep_all_if_fits=True)
    return out


def _csr(adj: np.ndarray, n: int) -> csr_matrix:
    rows = np.repeat(np.arange(n), adj.shape[1])
    cols = adj.reshape(-1)
    m = cols >= 0
    return csr_matrix((np.ones(int(m.sum()), dtype=np.int8), (rows[m], cols[m])), shape=(n, n))


def _reached_from(adj: np.ndarray, start: int) -> np.ndarray:
    order = breadth_first_order(_csr(adj, adj.shape[0]), start, directed=True, return_predecessors=False)
    r = np.zeros(adj.shape[0], dtype=bool)
    r[order] = True
    return r


def _append(adj: np.ndarray, u: int, v: int) -> bool:
    row = adj[u]
    if (row == v).any():
        return True
    free = np.nonzero(row < 0)[0]
    if free.size == 0:
        return False
    row[free[0]] = v
    return True


def _repair(X: np.ndarray, adj: np.ndarray, medoid: int, device) -> np.ndarray:
    return _repair_with(X, adj, medoid, device, _reached_from)


def _repair_with(X: np.ndarray, adj: np.ndarray, medoid: int, device, reached_fn, nearest_fn=None) -> np.ndarray:
    """Link one node of every source strongly connected component of the unreached part
    from its nearest reached node (with a free slot); repeat until all are reached.
    ``reached_fn(adj, start)`` gives the rows reachable from ``start`` (bool [n]);
    ``nearest_fn(rows, allowed)`` the nearest allowed row of each given row (exact kNN by
    default)."""
    n, R = adj.shape
    for _ in range(16):
        reached = reached_fn(adj, medoid)
        if reached.all():
            return adj
        un = np.nonzero(~reached)[0]
        pos = np.full(n, -1, dtype=np.int64)
        pos[un] = np.arange(un.size)
        rows = adj[un]
        valid = (rows >= 0) & ~reached[np.clip(rows, 0, None)]
        src = np.repeat(np.arange(un.size), R)[valid.ravel()]
        dst = pos[rows[valid]]
        g = csr_matrix((np.ones(src.size, dtype=np.int8), (src, dst)), shape=(un.size, un.size))
        ncomp, lab = connected_components(g, directed=True, connection="strong")
        has_in = np.zeros(ncomp, dtype=bool)
        cross = lab[src] != lab[dst]
        has_in[lab[dst[cross]]] = True
        _, first = np.unique(lab, return_index=True)  # smallest member of every component
        reps = un[first[~has_in]]
        host_ok = reached & (adj < 0).any(1)
        if not host_ok.any():
            host_ok = reached
        if nearest_fn is None:
            near, _ = exact_knn(X, X[reps], 1, "l2", device=device, candidate_mask=host_ok)
            near = near[:, 0]
        else:
            near = nearest_fn(reps, host_ok)
        for u, h in zip(reps.tolist(), near.tolist()):
            if not _append(adj, int(h), int(u)):
                adj[int(h), -1] = u
            _append(adj, int(u), int(h))
    if not reached_fn(adj, medoid).all():
        raise RuntimeError("connectivity repair did not converge")
    return adj


def medoid_of(X: np.ndarray) -> int:
    mu = X.astype(np.float64).mean(0)
    d = ((X.astype(np.float64) - mu) ** 2).sum(1)
    return int(np.argmin(d))


@torch.no_grad()
def build_graph(X: np.ndarray, R: int, cand: int | None = None, *, device=None,
                repair: bool = True) -> np.ndarray:
    """Degree-<=R proximity graph over the rows of X as a padded [n][R] int32 array."""
    dev = pick_device(device)
    n = X.shape[0]
    cand = R if cand is None else cand
    cand = min(cand, n - 1)
    ids, dist = exact_knn(X, None, cand, "l2", device=dev, exclude_self=True)
    x64 = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev).double()
    ci = torch.as_tensor(ids).to(dev)
    cd = torch.as_tensor(dist).to(dev)
    fwd = rng_prune(x64, ci, cd, R)
    full = add_reverse(x64, fwd, R)
    adj = full.cpu().numpy()
    # rows sorted by (distance, id)
    adj = _sort_rows(X, adj, dev)
    if repair:
        adj = _repair(X, adj, medoid_of(X), dev)
        adj = _sort_rows(X, adj, dev)
    return adj.astype(np.int32)


@torch.no_grad()
def _sort_rows(X: np.ndarray, adj: np.ndarray, device=None) -> np.ndarray:
    """Order every row by (distance to the row's node, id); -1 padding last."""
    dev = pick_device(device)
    x = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev).double()
    a_all = torch.as_tensor(adj).to(dev).long()
    out = torch.full_like(a_all, -1)
    step = 16384
    big = torch.iinfo(torch.int64).max
    for a in range(0, adj.shape[0], step):
        blk = a_all[a:a + step]
        v = x[blk.clamp(min=0)]
        d = ((v - x[a:a + step, None, :]) ** 2).sum(-1)
        d = torch.where(blk >= 0, d, torch.full_like(d, float("inf")))
        key_id = torch.where(blk >= 0, blk, torch.full_like(blk, big))
        o = torch.argsort(key_id, dim=1, stable=True)
        blk, d = torch.gather(blk, 1, o), torch.gather(d, 1, o)
        o = torch.argsort(d, dim=1, stable=True)
        out[a:a + step] = torch.gather(blk, 1, o)
    return out.cpu().numpy()


@torch.no_grad()
def leading_components(X: np.ndarray, dims: int, device=None) -> np.ndarray:
    """The ``dims`` leading eigenvectors of X's centred second moment (fp64), [D][dims]."""
    dev = pick_device(device)
    x = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    G = torch.zeros((x.shape[1], x.shape[1]), dtype=torch.float64, device=dev)
    mu = torch.zeros(x.shape[1], dtype=torch.float64, device=dev)
    for a in range(0, x.shape[0], 1 << 20):
        xa = x[a:a + (1 << 20)].double()
        G += xa.T @ xa
        mu += xa.sum(0)
    n = x.shape[0]
    C = (G / n - torch.outer(mu / n, mu / n)).cpu().numpy()
    w, V = np.linalg.eigh(C)
    return V[:, ::-1][:, :dims].copy()


def build_graph_projected(X: np.ndarray, R: int, dims: int, *, device=None, builder=None) -> np.ndarray:
    """Graph for high-dimensional rows: candidates, pruning and repair on the ``dims``
    leading principal components (``builder``, the exact builder by default), then every
    row ordered by the full distance.  Distances in the projected space under-estimate the
    full ones by the residual energy only, so the near candidates are largely the same
    rows; the full-space scoring of those candidates would cost D / dims times more."""
    V = leading_components(X, dims, device)
    Xp = (X.astype(np.float64) @ V).astype(np.float32)
    build = builder or (lambda Y, R_: build_graph(Y, R_, device=device))
    adj = build(Xp, R)
    return _sort_rows(X, adj.astype(np.int64), device).astype(np.int32)


def padded_to_csr(adj: np.ndarray):
    """[n][R] padded rows -> (rowptr int64 [n+1], nbrs int32)."""
    deg = (adj >= 0).sum(1)
    rowptr = np.zeros(adj.shape[0] + 1, dtype=np.int64)
    np.cumsum(deg, out=rowptr[1:])
    nbrs = adj[adj >= 0].astype(np.int32)
    return rowptr, nbrs


def build_subgraph_csr(X: np.ndarray, mask: np.ndarray, R: int, cand: int | None = None, *,
                       device=None):
    """Reconnect the sampled rows with the same builder; CSR over all N rows."""
    sel = np.nonzero(mask)[0]
    local = build_graph(X[sel], R, cand, device=device)
    glob = np.where(local >= 0, sel[np.clip(local, 0, None)], -1)
    n = X.shape[0]
    full = np.full((n, R), -1, dtype=np.int64)
    full[sel] = glob
    return padded_to_csr(full)
