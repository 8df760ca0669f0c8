"""Proximity graphs for the 10^7-10^8-row workloads, from IVF-restricted candidates.

The exact builder (``synth.graph``) scores every pair of rows, which is out of reach at
tens of millions of rows.  This builder restricts each row's candidates to an inverted
file (IVF) probe set and otherwise follows the same recipe, so that with every list
probed it returns exactly the exact builder's graph:

1. coarse clustering: seeded k-means (Lloyd) over a seeded sample of the rows into
   ``n_lists`` lists, then every row joins the list of its nearest centroid;
2. candidates: a list's rows share one probe set, the rows of the ``nprobe`` lists whose
   centroids are nearest to that list's centroid (its own list first); each row scores
   the probe set with an fp32 GEMM on vectors centred at its list's centroid (the
   distance is translation invariant, and centring keeps the expanded form's
   cancellation small), keeps the nearest ``cand + margin`` and re-ranks them by the
   direct fp64 distance, ties by id, to the nearest ``cand``;
3. neighbour selection of HNSW (relative-neighbourhood pruning) down to ``R``, reverse
   edges and re-pruning, rows ordered by (distance, id), and connectivity repair from
   the medoid: the exact builder's own steps (reachability is a breadth-first search on
   the GPU here, which scales to 10^8 rows).

Probing fewer lists than all of them loses a candidate only when one of the row's true
``cand`` nearest rows sits in an unprobed list; the graph then differs from the exact
one there, as FAISS-style approximate graphs do.
"""

from __future__ import annotations

import numpy as np
import torch

from .data import make_rng
from .graph import _repair_with, _sort_rows, add_reverse, medoid_of, padded_to_csr, rng_prune
from .knn import pick_device


@torch.no_grad()
def coarse_kmeans(x32: torch.Tensor, n_lists: int, seed: int, iters: int = 8, sample: int = 256):
    """Seeded Lloyd k-means over a seeded sample of at most ``sample * n_lists`` rows, then
    the nearest centroid of every row (ties by the lower list).  Returns (centroids fp32
    [n_lists][d], assignment int64 [n])."""
    n = x32.shape[0]
    dev = x32.device
    rng = make_rng(seed, 0x1F1F)
    m = min(n, sample * n_lists)
    rows = np.sort(rng.choice(n, size=m, replace=False)) if m < n else np.arange(n)
    xs = x32[torch.as_tensor(rows, device=dev)]
    init = rng.choice(m, size=n_lists, replace=False)
    cen = xs[torch.as_tensor(np.sort(init), device=dev)].clone()
    for _ in range(iters):
        a = _nearest(xs, cen)
        s = torch.zeros_like(cen).index_add_(0, a, xs)
        c = torch.bincount(a, minlength=n_lists).to(cen.dtype)
        nz = c > 0
        cen[nz] = s[nz] / c[nz, None]
    return cen, _nearest(x32, cen)


def _nearest(x: torch.Tensor, cen: torch.Tensor) -> torch.Tensor:
    cn = (cen.double() ** 2).sum(1).float()
    rows = max(1024, (1 << 30) // (4 * cen.shape[0]))  # ~1 GiB of scores per block
    out = torch.empty(x.shape[0], dtype=torch.int64, device=x.device)
    for a in range(0, x.shape[0], rows):
        s = cn[None, :] - 2.0 * (x[a:a + rows] @ cen.T)
        out[a:a + rows] = torch.argmin(s, dim=1)
    return out


@torch.no_grad()
def ivf_candidates(x32: torch.Tensor, x64: torch.Tensor, cen: torch.Tensor, assign: torch.Tensor,
                   nprobe: int, cand: int, margin: int = 16, rows_per_gemm: int = 4096, log=None):
    """Nearest ``cand`` rows of every row among its list's probe set (itself excluded):
    (ids int64 [n][cand], -1 padded; fp64 distances [n][cand], +inf padded), rows ordered
    by (distance, id)."""
    dev = x32.device
    n = x32.shape[0]
    L = cen.shape[0]
    nprobe = min(nprobe, L)
    order = torch.argsort(assign, stable=True)
    counts = torch.bincount(assign, minlength=L)
    starts = torch.cumsum(counts, 0) - counts
    # probe lists of every list: its own first, then the nearest other centroids (ties by
    # the lower list)
    c64 = cen.double()
    cn = (c64 ** 2).sum(1)
    probes = torch.empty((L, nprobe), dtype=torch.int64, device=dev)
    for a in range(0, L, 2048):
        dc = cn[a:a + 2048, None] + cn[None, :] - 2.0 * (c64[a:a + 2048] @ c64.T)
        r = torch.arange(dc.shape[0], device=dev)
        dc[r, a + r] = -1.0
        probes[a:a + 2048] = torch.argsort(dc, dim=1, stable=True)[:, :nprobe]
    probes = probes.cpu().numpy()
    out_i = torch.full((n, cand), -1, dtype=torch.int64, device=dev)
    out_d = torch.full((n, cand), float("inf"), dtype=torch.float64, device=dev)
    starts_h, counts_h = starts.cpu().numpy(), counts.cpu().numpy()
    for c in range(L):
        if log is not None and c % 8192 == 0 and c:
            log(f"ivf: candidates of {c} of {L} lists")
        if counts_h[c] == 0:
            continue
        probe = torch.cat([order[starts_h[p]:starts_h[p] + counts_h[p]] for p in probes[c]])
        xp = x32[probe] - cen[c][None, :]
        pn = (xp.double() ** 2).sum(1).float()
        members = order[starts_h[c]:starts_h[c] + counts_h[c]]
        kk = min(cand + margin, probe.shape[0] - 1)
        if kk <= 0:
            continue
        for a in range(0, members.shape[0], rows_per_gemm):
            mb = members[a:a + rows_per_gemm]
            xm = x32[mb] - cen[c][None, :]
            s = pn[None, :] - 2.0 * (xm @ xp.T)
            # a member's own row: position a + i of the probe set (its list comes first)
            r = torch.arange(mb.shape[0], device=dev)
            s[r, a + r] = float("inf")
            _, loc = torch.topk(s, kk, dim=1, largest=False, sorted=False)
            ids = probe[loc]
            vecs = x64[ids]
            d = ((vecs - x64[mb][:, None, :]) ** 2).sum(-1)
            o1 = torch.argsort(ids, dim=1, stable=True)
            ids, d = torch.gather(ids, 1, o1), torch.gather(d, 1, o1)
            o2 = torch.argsort(d, dim=1, stable=True)
            ids, d = torch.gather(ids, 1, o2)[:, :cand], torch.gather(d, 1, o2)[:, :cand]
            w = ids.shape[1]
            out_i[mb, :w] = ids
            out_d[mb, :w] = d
    return out_i, out_d


@torch.no_grad()
def reached_gpu(adj: torch.Tensor, start: int) -> torch.Tensor:
    """Rows reachable from ``start`` along the padded rows of ``adj`` (breadth first)."""
    n = adj.shape[0]
    seen = torch.zeros(n, dtype=torch.bool, device=adj.device)
    seen[start] = True
    front = torch.tensor([start], dtype=torch.int64, device=adj.device)
    while front.numel() > 0:
        nxt = adj[front].reshape(-1)
        nxt = nxt[nxt >= 0]
        nxt = torch.unique(nxt[~seen[nxt]])
        seen[nxt] = True
        front = nxt
    return seen


@torch.no_grad()
def build_graph_ivf(X: np.ndarray, R: int, *, n_lists: int | None = None, nprobe: int = 8,
                    cand: int | None = None, seed: int = 0, device=None, repair: bool = True,
                    log=None) -> np.ndarray:
    """Degree-<=R proximity graph over the rows of X (padded [n][R] int32), candidates
    restricted to ``nprobe`` IVF lists of about 1,024 rows each unless ``n_lists`` is given."""
    import time
    dev = pick_device(device)
    n = X.shape[0]
    cand = min(R if cand is None else cand, n - 1)
    L = n_lists if n_lists is not None else max(1, n // 1024)
    say = log or (lambda msg: None)
    t = time.time()
    x32 = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    x64 = x32.double()
    cen, assign = coarse_kmeans(x32, L, seed)
    say(f"ivf: {L} lists over {n} rows in {time.time() - t:.1f}s")
    t = time.time()
    ci, cd = ivf_candidates(x32, x64, cen, assign, nprobe, cand, log=say)
    del assign
    say(f"ivf: {cand} candidates per row from {min(nprobe, L)} lists in {time.time() - t:.1f}s")
    t = time.time()
    fwd = rng_prune(x64, ci, cd, R)
    del ci, cd
    say(f"ivf: forward lists pruned in {time.time() - t:.1f}s")
    full = add_reverse(x64, fwd, R)
    del fwd
    say(f"ivf: pruned, reverse edges added in {time.time() - t:.1f}s")
    del x64
    if dev.type == "cuda":
        torch.cuda.empty_cache()
    t = time.time()
    adj = _sort_rows(X, full.cpu().numpy(), dev)
    del full
    if repair:
        xn = (x32.double() ** 2).sum(1)

        def nearest(rows, allowed):
            # nearest allowed row by the direct fp64 distance among the 64 best of an fp32
            # scan (ties by id), with the vectors already on the device
            ok = torch.as_tensor(allowed).to(dev)
            q = x32[torch.as_tensor(rows).to(dev)]
            out = []
            blk = max(1, min(256, (1 << 30) // (8 * n)))  # ~1 GiB of scores per block
            for a in range(0, q.shape[0], blk):
                qa = q[a:a + blk]
                sc = (xn[None, :] - 2.0 * (qa.double() @ x32.double().T)).float() if n <= 1 << 20 else \
                    xn.float()[None, :] - 2.0 * (qa @ x32.T)
                sc[:, ~ok] = float("inf")
                _, cand = torch.topk(sc, min(64, n), dim=1, largest=False)
                d = ((x32[cand].double() - qa.double()[:, None, :]) ** 2).sum(-1)
                d = torch.where(ok[cand], d, torch.full_like(d, float("inf")))
                key_id = torch.argsort(cand, dim=1, stable=True)
                cand, d = torch.gather(cand, 1, key_id), torch.gather(d, 1, key_id)
                out.append(torch.gather(cand, 1, torch.argsort(d, dim=1, stable=True)[:, :1])[:, 0])
            return torch.cat(out).cpu().numpy()

        adj = _repair_with(X, adj, medoid_of(X), dev,
                           lambda a, s: reached_gpu(torch.as_tensor(a).to(dev), s).cpu().numpy(), nearest)
        adj = _sort_rows(X, adj, dev)
    del x32
    say(f"ivf: rows ordered, connected from the medoid in {time.time() - t:.1f}s")
    return adj.astype(np.int32)


def build_subgraph_csr_ivf(X: np.ndarray, mask: np.ndarray, R: int, *, nprobe: int = 8, seed: int = 0,
                           device=None, log=None):
    """The sampled rows reconnected by the IVF builder; CSR over all N rows."""
    sel = np.nonzero(mask)[0]
    local = build_graph_ivf(X[sel], R, nprobe=nprobe, seed=seed, device=device, log=log)
    glob = np.where(local >= 0, sel[np.clip(local, 0, None)], -1)
    n = X.shape[0]
    full = np.full((n, R), -1, dtype=np.int32)
    full[sel] = glob
    return padded_to_csr(full)
