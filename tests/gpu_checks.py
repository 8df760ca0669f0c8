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
                   outputs=None, bloom_log2=None, width=1):
    """Stage-1 traversal of the queries qidx against the oracle.  With `outputs` = (ids,
    dists, counters) rows of an earlier launch for exactly those queries, those are checked
    instead of launching the kernel here.  bloom_log2: the Bloom-filter visited set of
    2^bloom_log2 bits on both sides; width: entries expanded per step on both sides."""
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
    Xr64 = Xr_host.astype(np.float64)
    bad = 0
    tally = DistTally()
    n = Xr_host.shape[0]
    for j, i in enumerate(qidx):
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


