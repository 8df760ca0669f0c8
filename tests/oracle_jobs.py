"""Oracle runs over many queries for the GPU parity tests, spread over the host cores.

The functions here only slice the inputs and call the oracle (`oracle.pipeline`,
`oracle.greedy_search`); the worker processes are started by `oracle.parallel`, which
memory-maps the arrays.  Nothing here computes any part of the method.
"""

from __future__ import annotations

import numpy as np

import oracle
from oracle.parallel import map_queries

# the arrays every pipeline job reads, by name
PIPELINE_ARRAYS = ("Q", "Qr", "X", "V", "rp", "nb", "sr", "sn", "Xr", "cent", "buckets", "P", "pivots")


def _pipeline_job(a, item):
    rows, kw = item
    rows = np.asarray(rows, dtype=np.int64)
    return oracle.pipeline(a["Q"][rows], a["X"], a["V"], a["rp"], a["nb"], a["sr"], a["sn"], a["Xr"], a["cent"],
                           a["buckets"], a["P"], a["pivots"], Qr=a["Qr"][rows], with_margin=True, **kw)


def pipeline(arrays: dict, jobs, procs=None, chunk: int = 16):
    """jobs: [(rows, oracle.pipeline keyword arguments)], each rows an index array into
    arrays["Q"] / arrays["Qr"].  Returns, per job, (ids, dists, counters, margins) for
    its rows, in order."""
    items, owner = [], []
    for j, (rows, kw) in enumerate(jobs):
        rows = np.asarray(rows, dtype=np.int64)
        for lo in range(0, rows.size, chunk):
            items.append((rows[lo:lo + chunk], kw))
            owner.append(j)
    arr = {name: arrays[name] for name in PIPELINE_ARRAYS}
    parts = map_queries(_pipeline_job, items, arr, procs)
    out = []
    for j in range(len(jobs)):
        mine = [p for p, o in zip(parts, owner) if o == j]
        if not mine:
            k = jobs[j][1]["k"]
            out.append((np.zeros((0, k), np.int64), np.zeros((0, k)), np.zeros((0, 4), np.int64), np.zeros(0)))
            continue
        out.append(tuple(np.concatenate([p[c] for p in mine]) for c in range(4)))
    return out


def _traverse_job(a, item):
    rows, ef, metric, kw = item
    res = []
    n = a["Xr"].shape[0]
    for i in rows:
        ent = a["entries"][i]
        ent = np.where((ent >= 0) & (ent < n), ent, -1)
        r = oracle.greedy_search(a["Qr"][i], a["Xr"], a["sr"], a["sn"], int(ef if np.ndim(ef) == 0 else ef[i]),
                                 ent, metric, **kw)
        res.append({"ids": r["ids"], "dists": r["dists"], "n_exp": r["n_exp"], "n_dist": r["n_dist"],
                    "margin": r["margin"]})
    return res


def traverse(Qr, Xr64, sr, sn, entries, rows, ef, metric="l2", procs=None, chunk: int = 8, **kw):
    """oracle.greedy_search for the queries `rows` (stage 1: reduced queries, reduced
    vectors, subgraph); ef is one size or an array of per-query sizes indexed like Qr."""
    rows = np.asarray(rows, dtype=np.int64)
    arrays = dict(Qr=Qr, Xr=Xr64, sr=sr, sn=sn, entries=entries)
    if np.ndim(ef):
        arrays["ef"] = np.asarray(ef)
    items = [(rows[lo:lo + chunk], ef if np.ndim(ef) == 0 else None, metric, kw)
             for lo in range(0, rows.size, chunk)]
    if np.ndim(ef):
        parts = map_queries(_traverse_job_ragged, items, arrays, procs)
    else:
        parts = map_queries(_traverse_job, items, arrays, procs)
    return [r for p in parts for r in p]


def _traverse_job_ragged(a, item):
    rows, _, metric, kw = item
    b = dict(a)
    return _traverse_job(b, (rows, a["ef"], metric, kw))
