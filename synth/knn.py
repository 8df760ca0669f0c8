"""Exact k-nearest-neighbour search used to build graph fixtures and recall ground truth.

Candidates come from an fp32 GEMM scan with a safety margin; the final order
is decided by fp64 distances recomputed directly, with ties broken by the
smaller id.  Runs on whatever torch device is given (the GPU when building the
million-row fixtures, the CPU for small ones).
"""

from __future__ import annotations

import numpy as np
import torch


def pick_device(device=None) -> torch.device:
    if device is not None:
        return torch.device(device)
    return torch.device("cuda" if torch.cuda.is_available() else "cpu")


def _rank_exact(x64: torch.Tensor, q64: torch.Tensor, cand: torch.Tensor, metric: str, k: int):
    """Re-rank candidate ids [b][c] by fp64 distance, ties by id; return top-k."""
    vecs = x64[cand.clamp(min=0)]  # [b][c][d]
    if metric == "l2":
        d = ((vecs - q64[:, None, :]) ** 2).sum(-1)
    else:
        d = -(vecs * q64[:, None, :]).sum(-1)
    d = torch.where(cand >= 0, d, torch.full_like(d, float("inf")))
    # order by id, then stable order by distance => (distance, id) lexicographic
    o1 = torch.argsort(cand, dim=1, stable=True)
    cand, d = torch.gather(cand, 1, o1), torch.gather(d, 1, o1)
    o2 = torch.argsort(d, dim=1, stable=True)
    cand, d = torch.gather(cand, 1, o2), torch.gather(d, 1, o2)
    return cand[:, :k], d[:, :k]


@torch.no_grad()
def exact_knn(X, Q, k: int, metric: str = "l2", *, device=None, exclude_self: bool = False,
              margin: int = 16, budget_bytes: int | None = None, candidate_mask=None,
              fp64_scores: bool = False):
    """Exact top-k of each row of Q among rows of X.

    Returns (ids int64 [m][k], dists float64 [m][k]) as numpy arrays.  With
    ``exclude_self`` the query set is X itself and row i never returns i.
    ``candidate_mask`` (bool [n]) restricts the search to the marked rows.
    ``fp64_scores`` takes the candidates from fp64 scores instead of an fp32 GEMM (for sets
    whose nearest scores lie closer together than the fp32 products' rounding).
    """
    dev = pick_device(device)
    old_tf32 = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    try:
        xt = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
        qt = xt if Q is None else torch.as_tensor(np.ascontiguousarray(Q, dtype=np.float32)).to(dev)
        n, m = xt.shape[0], qt.shape[0]
        kk = min(k + margin, n)
        x64 = xt.double()
        xn64 = (x64 ** 2).sum(1)
        xn = xn64.float()
        bias = None
        if candidate_mask is not None:
            cm = torch.as_tensor(np.asarray(candidate_mask, dtype=bool)).to(dev)
            bias = torch.where(cm, torch.zeros(n, device=dev), torch.full((n,), float("inf"), device=dev))
        if budget_bytes is None:
            budget_bytes = (6 << 30) if dev.type == "cuda" else (1 << 29)
        # a chunk's score matrix also stays below 2^30 elements (top-k over larger tensors
        # is not to be relied on)
        width = 8 if fp64_scores else 4
        bs = int(max(1, min(m, budget_bytes // max(1, width * n), (1 << 30) // max(1, n))))
        out_i = np.empty((m, min(k, n)), dtype=np.int64)
        out_d = np.empty((m, min(k, n)), dtype=np.float64)
        for q0 in range(0, m, bs):
            q = qt[q0:q0 + bs]
            if fp64_scores:
                q64 = q.double()
                s = (xn64[None, :] - 2.0 * (q64 @ x64.T)) if metric == "l2" else -(q64 @ x64.T)
            elif metric == "l2":
                s = xn[None, :] - 2.0 * (q @ xt.T)
            else:
                s = -(q @ xt.T)
            if bias is not None:
                s = s + bias[None, :]
            if exclude_self:
                r = torch.arange(q.shape[0], device=dev)
                s[r, q0 + r] = float("inf")
            _, idx = torch.topk(s, kk, dim=1, largest=False, sorted=False)
            del s
            if exclude_self:
                r = torch.arange(q.shape[0], device=dev)
                idx = torch.where(idx == (q0 + r)[:, None], torch.full_like(idx, -1), idx)
            if bias is not None:
                idx = torch.where(bias[idx.clamp(min=0)] == 0, idx, torch.full_like(idx, -1))
            ci, cd = _rank_exact(x64, q.double(), idx, metric, min(k, n))
            out_i[q0:q0 + bs] = ci.cpu().numpy()
            out_d[q0:q0 + bs] = cd.cpu().numpy()
        return out_i, out_d
    finally:
        torch.backends.cuda.matmul.allow_tf32 = old_tf32


def recall_at_k(found: np.ndarray, truth: np.ndarray, k: int) -> float:
    """Mean over queries of |found_k intersect truth_k| / k."""
    found = np.asarray(found)[:, :k]
    truth = np.asarray(truth)[:, :k]
    hits = 0
    for f, t in zip(found, truth):
        hits += len(set(f[f >= 0].tolist()) & set(t.tolist()))
    return hits / (k * max(1, len(truth)))
