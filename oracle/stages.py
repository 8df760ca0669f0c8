"""The three search stages and the full pipeline (section 4.1).

1. GPU piloting: Algorithm 1 on the sampled subgraph with reduced vectors,
   started from the entries that fast entry selection returns.
2. Residual refinement: complete distances for the stage-1 candidates (primary
   plus residual part, which in exact arithmetic is the full distance and is
   computed here directly on the full vectors), a re-ranking, then two loop
   steps of Algorithm 1 on the subgraph with full distances; the outputs are
   the re-ranked candidates and the visited set.
3. Final traversal: Algorithm 1 on the full graph with full vectors, starting
   from the stage-2 candidates (all unchecked again, because the full graph's
   edges differ) with the stage-2 visited set pre-populated.

Only the candidate list crosses from stage 1 to stage 2 (section 4.1 summary:
the query goes to the GPU, a small candidate set comes back), so stage 2
starts with the handed-off ids as its visited set.  With stage 1 switched off
the pipeline is plain Algorithm 1 from the entries (graceful degradation,
section 4.1 summary).  The effective final list size is max(ef, k) because
k <= ef (section 2.2).
"""

from __future__ import annotations

import numpy as np

from .entries import select_entries
from .metric import as_f32, delta_many
from .projection import project
from .traverse import greedy_search


def gpu_stage(qr, Xr, sub_rowptr, sub_nbrs, entries, ef: int, metric: str = "l2", bloom_log2=None, width: int = 1):
    """Stage 1 for one reduced query: Algorithm 1 on the subgraph (with the exact visited
    set, or the Bloom filter of section 4.3 when bloom_log2 is given)."""
    return greedy_search(qr, Xr, sub_rowptr, sub_nbrs, ef, entries, metric, bloom_log2=bloom_log2, width=width)


def refine(q, X, sub_rowptr, sub_nbrs, beam_ids, ef_cpu: int, metric: str = "l2", steps: int = 2):
    """Stage 2 for one query; returns the Algorithm 1 result dict plus total n_dist."""
    ids = [int(v) for v in beam_ids if v >= 0]
    d = as_f32(delta_many(q, X[np.asarray(ids, dtype=np.int64)], metric)) if ids else np.zeros(0)
    res = greedy_search(q, X, sub_rowptr, sub_nbrs, ef_cpu, (), metric,
                        initial=list(zip(d.tolist(), ids)), max_steps=steps)
    res["n_dist"] += len(ids)
    return res


def final_traversal(q, X, rowptr, nbrs, cand_ids, cand_dists, visited, ef_cpu: int, k: int,
                    metric: str = "l2"):
    """Stage 3 for one query; returns (ids [k], dists [k], result dict), padded with (-1, inf)."""
    ef = max(ef_cpu, k)
    res = greedy_search(q, X, rowptr, nbrs, ef, (), metric,
                        initial=list(zip(np.asarray(cand_dists).tolist(), np.asarray(cand_ids).tolist())),
                        visited=visited)
    ids = np.full(k, -1, dtype=np.int64)
    dists = np.full(k, np.inf)
    take = min(k, res["ids"].size)
    ids[:take] = res["ids"][:take]
    dists[:take] = res["dists"][:take]
    return ids, dists, res


def _order_gap(keys) -> float:
    """Smallest relative gap between neighbouring values of an ordered sequence."""
    gap = np.inf
    for a, b in zip(keys, keys[1:]):
        gap = min(gap, abs(b - a) / max(abs(a), abs(b), 1e-300))
    return gap


def pipeline(Q, X, V, rowptr, nbrs, sub_rowptr, sub_nbrs, Xr, centroids, buckets, pivot_vecs,
             pivot_ids, *, k: int, ef_gpu: int, ef_cpu: int, E: int, metric: str = "l2",
             refine_steps: int = 2, use_gpu_stage: bool = True, use_refine: bool = True, bloom_log2=None,
             use_final: bool = True, width: int = 1, Qr=None, with_margin: bool = False, fixed_entries=None):
    """All stages for every query; returns (ids [m][k], dists [m][k], counters [m][4]).

    counters = (stage-1 distances, stage-2 distances, stage-3 distances, stage-3 steps).
    use_final=False skips stage 3 and returns the best k of the stage-2 list by full
    distance (with every node sampled and d_r = D this is the GPU-only special case).

    Qr: the reduced queries [m][d_r] to route and search with; by default q^T V_d computed
    here exactly (fp64) and rounded once to fp32: the search computes in single precision
    (section 6.1), and the reduced query is held like the reduced base vectors X_r, which
    the caller passes already rounded.

    with_margin=True appends margin [m]: per query, the smallest relative gap over every
    comparison that decided its result (routing, the entry cut, each stage's Algorithm 1
    decisions, and the order of the k returned keys).

    fixed_entries: node ids every query starts from instead of the entries fast entry
    selection picks (the predefined entry points section 5 contrasts FES with; the
    ablation without FES); no routing or entry cut is decided then.
    """
    if not use_final and not use_gpu_stage:
        raise ValueError("without the GPU stage the final traversal must run")
    Q = np.asarray(Q, dtype=np.float64)
    Qr = as_f32(project(Q, V)) if Qr is None else np.asarray(Qr, dtype=np.float64)
    m = Q.shape[0]
    if fixed_entries is None:
        entries, _, _, e_margin = select_entries(Qr, centroids, buckets, pivot_vecs, pivot_ids, E, metric)
    else:
        entries = np.tile(np.asarray(fixed_entries, dtype=np.int64)[None, :], (m, 1))
        e_margin = np.full(m, np.inf)
    out_i = np.full((m, k), -1, dtype=np.int64)
    out_d = np.full((m, k), np.inf)
    counters = np.zeros((m, 4), dtype=np.int64)
    margins = np.full(m, np.inf)
    for i in range(m):
        margin = float(e_margin[i])
        if use_gpu_stage:
            g = gpu_stage(Qr[i], Xr, sub_rowptr, sub_nbrs, entries[i], ef_gpu, metric, bloom_log2, width)
            counters[i, 0] = g["n_dist"]
            margin = min(margin, g["margin"])
            if use_refine:
                r = refine(Q[i], X, sub_rowptr, sub_nbrs, g["ids"], ef_cpu, metric, refine_steps)
                counters[i, 1] = r["n_dist"]
                margin = min(margin, r["margin"])
                c_ids, c_d, vis = r["ids"], r["dists"], r["visited"]
            else:
                c_ids = g["ids"]
                c_d = as_f32(delta_many(Q[i], X[c_ids], metric)) if c_ids.size else np.zeros(0)
                counters[i, 1] = c_ids.size
                vis = set(int(v) for v in c_ids)
            if use_final:
                ids, d, f = final_traversal(Q[i], X, rowptr, nbrs, c_ids, c_d, vis, ef_cpu, k, metric)
                margin = min(margin, f["margin"])
            else:
                order = sorted(range(len(c_ids)), key=lambda j: (float(c_d[j]), int(c_ids[j])))
                # the cut after the k-th key and the order of the k kept
                margin = min(margin, _order_gap([float(c_d[j]) for j in order[:min(ef_cpu, k) + 1]]))
                order = order[:min(ef_cpu, k)]
                ids = np.full(k, -1, dtype=np.int64)
                d = np.full(k, np.inf)
                ids[:len(order)] = [int(c_ids[j]) for j in order]
                d[:len(order)] = [float(c_d[j]) for j in order]
                f = {"n_dist": 0, "n_exp": 0}
        else:
            ef = max(ef_cpu, k)
            f = greedy_search(Q[i], X, rowptr, nbrs, ef, entries[i], metric)
            margin = min(margin, f["margin"])
            ids = np.full(k, -1, dtype=np.int64)
            d = np.full(k, np.inf)
            t = min(k, f["ids"].size)
            ids[:t], d[:t] = f["ids"][:t], f["dists"][:t]
        counters[i, 2] = f["n_dist"]
        counters[i, 3] = f["n_exp"]
        out_i[i], out_d[i] = ids, d
        margins[i] = margin
    if with_margin:
        return out_i, out_d, counters, margins
    return out_i, out_d, counters
