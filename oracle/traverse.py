"""Greedy best-first search, Algorithm 1 ("ANNS by Greedy Search"), section 2.2.

The candidate list C holds (distance, id, checked) entries.  Each loop step
takes the first unchecked entry u, marks it checked, computes the distance of
every not-yet-visited out-neighbour of u (marking it visited), inserts it, and
finally resizes C to ef.  The search ends when C holds no unchecked entry.

Readings where the paper is silent:
* order: C is ordered by the key (distance, id), a strict total order;
* entry points: each entry is marked visited and scored once when C is
  initialised (entries already visited, or equal to -1, are skipped), and the
  initial C is resized to ef (the first expansion is the same either way);
* visited is an exact set, one distance per visited node, so
  n_dist = |visited|; ``bloom_log2`` selects the paper's lossy filter instead
  (section 4.3; its readings are in ``oracle.bloom``);
* expansion width is one node per loop step, as printed; ``width=2`` is a variant
  (not the paper's): each step takes the first two unchecked entries of C, marks
  both, and scores the unvisited out-neighbours of both (first node's row, then
  the second's) as one group before the resize;
* distances are single-precision values (section 6.1): each is computed exactly
  and rounded once to fp32 before it enters C (``precision="f64"`` keeps fp64).

Inputs for the later stages: ``initial`` seeds C with already scored
(distance, id) pairs, ``visited`` pre-populates the visited set and
``max_steps`` bounds the number of loop steps (the refinement stage runs two).

The returned ``margin`` is the smallest relative gap over the comparisons that
steer Algorithm 1: the first unchecked entry against the next unchecked one
(which node line 5 expands), the last kept key against the first key dropped by
each resize (line 11), and neighbouring keys of the final list (its order).
When it is tiny, a different rounding of the distances may legitimately change
the result.
"""

from __future__ import annotations

import numpy as np

from .bloom import ENTRY_GROUP, BloomFilter
from .metric import as_f32, delta_many


def _rel_gap(a: float, b: float) -> float:
    return abs(b - a) / max(abs(a), abs(b), 1e-300)


def _resize_gap(sorted_keys, ef: int) -> float:
    """Gap at the resize boundary (kept key ef-1 against dropped key ef)."""
    if len(sorted_keys) <= ef:
        return np.inf
    return _rel_gap(sorted_keys[ef - 1][0], sorted_keys[ef][0])


def greedy_search(q, vectors, rowptr, nbrs, ef: int, entries=(), metric: str = "l2", *,
                  initial=None, visited=None, max_steps=None, precision: str = "f32", bloom_log2=None,
                  width: int = 1):
    """Run Algorithm 1 for one query.

    q        query vector (any float dtype; used in fp64)
    vectors  base vectors indexed by node id
    rowptr, nbrs   CSR out-neighbours in stored order
    Returns a dict with ``ids``/``dists`` (C in key order, at most ef),
    ``checked`` flags, ``n_exp`` (loop steps), ``n_dist`` (distances computed
    here), ``visited`` (the final set, or the Bloom filter) and ``margin``.
    """
    if ef < 1:
        raise ValueError("ef must be >= 1")
    if width not in (1, 2):
        raise ValueError("width must be 1 or 2")
    if bloom_log2 is not None and (initial is not None or visited is not None):
        raise ValueError("the Bloom filter variant starts from entry points only")
    q = np.asarray(q, dtype=np.float64)
    seen = set() if visited is None else set(int(v) for v in visited)
    bloom = BloomFilter(bloom_log2) if bloom_log2 is not None else None
    n_dist = 0

    def score(ids):
        d = delta_many(q, vectors[np.asarray(ids)], metric)
        return as_f32(d) if precision == "f32" else d
    # line 3: C <- EP
    C = []  # list of [key=(distance, id), checked]
    if initial is not None:
        for d, v in initial:
            C.append([(float(d), int(v)), False])
            seen.add(int(v))
    fresh = []
    if bloom is not None:
        entries = [int(e) for e in entries]
        for g in range(0, len(entries), ENTRY_GROUP):
            fresh += bloom.fresh_of_group(entries[g:g + ENTRY_GROUP])
    else:
        for e in entries:
            e = int(e)
            if e < 0 or e in seen:
                continue
            seen.add(e)
            fresh.append(e)
    if fresh:
        ds = score(fresh)
        n_dist += len(fresh)
        in_c = set()
        for d, v in zip(ds, fresh):
            if v not in in_c:  # an id listed twice in a group enters C once
                in_c.add(v)
                C.append([(float(d), v), False])
    C.sort(key=lambda c: c[0])
    margin = _resize_gap([c[0] for c in C], ef)
    del C[ef:]
    n_exp = 0
    while max_steps is None or n_exp < max_steps:
        # line 5: the first unchecked node in C (the first `width` of them)
        unchecked = [i for i, c in enumerate(C) if not c[1]][:width + 1]
        if not unchecked:
            break  # line 12: no unchecked node left
        chosen = unchecked[:width]
        if len(unchecked) > width:  # which nodes are expanded: the last chosen vs the next
            margin = min(margin, _rel_gap(C[chosen[-1]][0][0], C[unchecked[width]][0][0]))
        group = []
        for pos in chosen:
            C[pos][1] = True
            u = C[pos][0][1]
            group.extend(int(v) for v in nbrs[rowptr[u]:rowptr[u + 1]])
        n_exp += len(chosen)
        # lines 6-10: unvisited out-neighbours, mark, score, insert
        new = []
        if bloom is not None:
            new = bloom.fresh_of_group(group)
        else:
            for v in group:
                if v not in seen:
                    seen.add(v)
                    new.append(v)
        if new:
            ds = score(new)
            n_dist += len(new)
            in_c = {c[0][1] for c in C}
            for d, v in zip(ds, new):
                if v not in in_c:
                    in_c.add(v)
                    C.append([(float(d), v), False])
            C.sort(key=lambda c: c[0])
            margin = min(margin, _resize_gap([c[0] for c in C], ef))
        # line 11: C.resize(ef)
        del C[ef:]
    for a, b in zip(C, C[1:]):
        margin = min(margin, _rel_gap(a[0][0], b[0][0]))
    return {
        "ids": np.asarray([c[0][1] for c in C], dtype=np.int64),
        "dists": np.asarray([c[0][0] for c in C], dtype=np.float64),
        "checked": np.asarray([c[1] for c in C], dtype=bool),
        "n_exp": n_exp,
        "n_dist": n_dist,
        "visited": bloom if bloom is not None else seen,
        "margin": margin,
    }
