"""Shared GPU-versus-oracle checks (imported by the GPU test modules)."""

import numpy as np
import torch

import oracle
import paper_2503_21206_amd as pa
from tests.parity import TIE, DistTally


def _t(a, dev, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev).contiguous()


def say(msg):
    print(msg, flush=True)


def traverse_check(dev, w, Xr_host, Xr_dev, entries, ef, qidx, metric="l2", cache_log2=0, expect_reset=False,
                   outputs=None, bloom_log2=None, width=1, refs=None):
    """Stage-1 traversal of the queries qidx against the oracle.  With `outputs` = (ids,
    dists, counters) rows of an earlier launch for exactly those queries, those are checked
    instead of launching the kernel here.  bloom_log2: the Bloom-filter visited set of
    2^bloom_log2 bits on both sides; width: entries expanded per step on both sides.
    refs: the oracle's results for qidx, already computed (tests.oracle_jobs.traverse)."""
    Qr = w["Qr32"][qidx]
    if outputs is None:
        adj = _t(w["sub_adj"].astype(np.int32), dev)
        ids, d, cnt = pa.gpu_traverse(_t(Qr, dev), Xr_dev, adj, _t(entries[qidx].astype(np.int32), dev), ef,
                                      metric, cache_log2, bloom_log2=-1 if bloom_log2 is None else bloom_log2,
                                      width=width)
        torch.cuda.synchronize()
        ids, d, cnt = ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy()
    else:
        ids, d, cnt = outputs
    assert (cnt[:, 3] == 0).all()
    Xr64 = Xr_host.astype(np.float64) if refs is None else None
    bad = 0
    tally = DistTally()
    n = Xr_host.shape[0]
    for j, i in enumerate(qidx):
        if refs is not None:
            r = refs[j]
        else:
            ent_i = np.where((entries[i] >= 0) & (entries[i] < n), entries[i], -1)  # the kernel skips the others
            r = oracle.greedy_search(Qr[j], Xr64, w["sr"], w["sn"], ef, ent_i, metric, bloom_log2=bloom_log2,
                                     width=width)
        k = r["ids"].size
        ref = np.full(ef, -1)
        ref[:k] = r["ids"]
        if not (ids[j] == ref).all():
            assert r["margin"] <= TIE, (i, ids[j][:8], ref[:8], r["margin"])
            bad += 1
            continue
        assert (ids[j][k:] == -1).all() and (d[j][k:] == np.inf).all()
        tally.check(d[j][:k], r["dists"], i)
        if r["margin"] > TIE:
            assert cnt[j, 0] == r["n_exp"]
            if cnt[j, 2] == 0:
                assert cnt[j, 1] == r["n_dist"]
            else:
                assert cnt[j, 1] >= r["n_dist"]
    off = tally.done()
    say(f"  {len(qidx)} queries: {bad} id divergences, {off} of {tally.n} distances 1 ulp off")
    if expect_reset:
        assert (cnt[:, 2] > 0).any()
    assert bad <= max(1, len(qidx) // 1000), bad
    return ids, d, cnt




def library_qr(dev, Q, V, centroids):
    """The library's own reduced queries and routed clusters (pa_project_route: the fp32
    MFMA product the search pipeline computes), as host arrays."""
    Qr, cl = pa.project_route(_t(Q, dev), _t(V, dev), _t(centroids, dev))
    torch.cuda.synchronize()
    return Qr.cpu().numpy(), cl.cpu().numpy()


def pipeline_check(ids, d, ref, what, cnt=None):
    """Search results [m][k] against oracle.pipeline's (ids, dists, counters, margins) for
    the same queries.  An ordered result list may differ only where the oracle's margin over
    every decision of the search is at most two ulps, on at most 0.1% of the queries (at
    least one); the distances of equal lists are within 1 ulp.  With the library's
    counters [m][8], the host stages' distance and step counts must equal the oracle's,
    and stage 1's as well where the visited cache never forgot a node."""
    oi, od, oc, om = ref
    m = ids.shape[0]
    assert oi.shape == ids.shape, (what, oi.shape, ids.shape)
    bad = 0
    tally = DistTally()
    for i in range(m):
        if not (ids[i] == oi[i]).all():
            assert om[i] <= TIE, (what, i, ids[i][:8], oi[i][:8], om[i])
            bad += 1
            continue
        tally.check(d[i], od[i], (what, i))
        if cnt is not None and om[i] > TIE:
            if cnt[i, 2] == 0:
                assert cnt[i, 1] == oc[i, 0], (what, i, "stage-1 distances", cnt[i, 1], oc[i, 0])
            assert cnt[i, 3] == oc[i, 1], (what, i, "stage-2 distances", cnt[i, 3], oc[i, 1])
            assert cnt[i, 4] == oc[i, 2], (what, i, "stage-3 distances", cnt[i, 4], oc[i, 2])
            assert cnt[i, 5] == oc[i, 3], (what, i, "stage-3 steps", cnt[i, 5], oc[i, 3])
    off = tally.done()
    say(f"  {what}: {m} queries, {bad} lists differ (near ties), {off} of {tally.n} distances 1 ulp off")
    assert bad <= max(1, m // 1000), (what, bad)
    return bad
