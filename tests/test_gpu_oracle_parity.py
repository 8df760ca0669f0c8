"""End-to-end parity with the oracle: every search form the library offers, run through
the C-ABI on the 10K x 96 workload, against `oracle.pipeline` on the same inputs.

Both sides compute the reduced queries themselves: the oracle as the exact product
rounded once to fp32, the library with its compensated projection, which gives the same
bits (checked here: at most a 1e-4 fraction of the values may differ, by one ulp).  The
lists must be the oracle's on at least 99.9% of the queries, a differing query only where
the oracle's margin over every decision of its search (routing, the entry cut, every
Algorithm 1 step of stages 1-3, the order of the returned keys) is at most two fp32 ulps;
distances within 1 ulp; the host stages' counters equal.  Covered: the default pipeline, the Bloom visited filter, expansion
width 2, stage 1 without refinement (stage mask 1), no GPU stage (mask 2), the GPU-only
special case (masks 5 and 7), top-100, the compact layout, per-request (k, ef) through
the serving loop, and the per-query list sizes of the ragged traversal."""

import numpy as np
import pytest

import oracle
import paper_2503_21206_amd as pa
from synth import node_order
from tests import oracle_jobs
from tests.gpu_checks import _t, library_qr, pipeline_check, say
from tests.parity import TIE, DistTally, ulp_diff
from tests.workload import build_tiny, device_tables, oracle_entries

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pa.device_init(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def tiny():
    return build_tiny(device="cpu")


def _ulp_fraction(got, want):
    u = ulp_diff(got, want)
    assert (u <= 1).all(), np.argwhere(u > 1)[:4]
    return float((u != 0).mean())


@pytest.fixture(scope="module")
def lib_qr(dev, tiny):
    """The library's reduced queries and routed clusters, checked against the oracle's
    reduced queries (never fed to the oracle)."""
    Qr, cl = library_qr(dev, tiny["Q"], tiny["V32"], tiny["cent32"])
    frac = _ulp_fraction(Qr, tiny["Qr32"])
    say(f"library projection of the queries: {frac:.2e} of the values one ulp from the oracle's")
    assert frac <= 1e-4
    # per-row results: the same bits whatever the batch around a query
    Qr2, cl2 = library_qr(dev, tiny["Q"][333:700], tiny["V32"], tiny["cent32"])
    assert (Qr2.view(np.uint32) == Qr[333:700].view(np.uint32)).all() and (cl2 == cl[333:700]).all()
    return Qr, cl


def test_projection_of_the_base_set_is_the_rounded_exact_product(dev, tiny):
    say("pa_project of the 10,000 base vectors (f32, f16, bf16) against the oracle's rounded product")
    Xt, Vt = _t(tiny["X"], dev), _t(tiny["V32"], dev)
    y32 = pa.project(Xt, Vt, "f32").cpu().numpy()
    frac = _ulp_fraction(y32, tiny["Xr32"])
    say(f"  {frac:.2e} of the fp32 values one ulp off")
    assert frac <= 1e-4
    y16 = pa.project(Xt, Vt, "f16").cpu().numpy().astype(np.float32)
    assert np.mean(y16 != tiny["Xr32"].astype(np.float16).astype(np.float32)) <= 1e-4


def _arrays(tiny, Xr=None, **over):
    """Oracle inputs: the workload's own arrays (reduced queries: the oracle's)."""
    a = dict(Q=tiny["Q"], Qr=tiny["Qr32"], X=tiny["X"], V=tiny["V32"], rp=tiny["rp"], nb=tiny["nb"], sr=tiny["sr"],
             sn=tiny["sn"], Xr=tiny["Xr32"] if Xr is None else Xr, cent=tiny["cent32"], buckets=tiny["buckets"],
             P=tiny["P32"], pivots=tiny["pivots"])
    a.update(over)
    return a


def _index(tiny, xr="f32", compact=False):
    s = tiny["spec"]
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype=xr, r=s.r, threads=4,
                                  compact=compact))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    idx.set_projection(tiny["V32"])
    mask = idx.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
    assert (mask == tiny["mask"]).all()
    idx.build_subgraph(mask, tiny["sr"], tiny["sn"])
    idx.build_entries(tiny["pivots"], tiny["init"], 10)
    _, b, c = idx.state()  # the library's buckets and centroids are the oracle's
    assert (b == tiny["pivots"][tiny["buckets"]]).all() and (c.view(np.uint32) == tiny["cent32"].view(np.uint32)).all()
    return idx


def test_routing_on_the_library_projection(dev, tiny, lib_qr):
    say("routing: pa_project_route's clusters against the oracle's routing of its own reduced queries")
    _, cl = lib_qr
    Qr = tiny["Qr32"]
    bad = 0
    for i in range(Qr.shape[0]):
        c, gap = oracle.route(Qr[i], tiny["cent32"].astype(np.float64))
        if c != cl[i]:
            assert gap <= TIE, (i, c, cl[i], gap)
            bad += 1
    say(f"  {Qr.shape[0]} queries, {bad} routed differently (near ties)")
    assert bad <= max(1, Qr.shape[0] // 1000)


def test_entries_on_the_library_projection(dev, tiny, lib_qr):
    say("FES entries of the library's reduced queries and clusters against the oracle's")
    Qr, cl = lib_qr
    EV, EVn, EVid = device_tables(tiny)
    E = 8
    ids, d = pa.select_entries(_t(Qr, dev), _t(cl.astype(np.int32), dev), _t(EV, dev), _t(EVn, dev), _t(EVid, dev),
                               E)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    oi, od, _, margin = oracle_entries(tiny, E)
    nq = Qr.shape[0]
    tally = DistTally()
    bad = 0
    for i in range(nq):
        if not (ids[i] == oi[i]).all():
            assert margin[i] <= TIE, (i, ids[i], oi[i], margin[i])
            bad += 1
            continue
        tally.check(d[i], od[i], i)
    tally.done()
    say(f"  {nq} queries, {bad} entry lists differ (near ties)")
    assert bad <= max(1, nq // 1000)


SEARCH_FORMS = [
    # name, search keyword arguments, oracle keyword arguments, queries
    ("default", dict(batch=300), dict(), 1000),
    ("bloom", dict(batch=300, bloom=True), dict(bloom_log2=15), 1000),
    ("width2", dict(width=2), dict(width=2), 1000),
    ("stage1_no_refine", dict(stage_mask=1), dict(use_refine=False), 1000),
    ("no_gpu_stage", dict(stage_mask=2), dict(use_gpu_stage=False), 1000),
    ("serial_sub_batches", dict(batch=300, serial=True), dict(), 1000),
    ("fixed_entries", dict(fixed_entries=True), dict(fixed_entries="F"), 1000),
    ("fixed_entries_no_gpu_stage", dict(fixed_entries=True, stage_mask=2), dict(fixed_entries="F",
                                                                            use_gpu_stage=False), 1000),
]


def _fixed_entries(tiny, E):
    """The predefined entries of the library's fixed mode, from the oracle's buckets: entry
    e is pivot e // r of bucket e % r."""
    b = tiny["pivots"][tiny["buckets"]]
    r = b.shape[0]
    return np.array([b[e % r, e // r] for e in range(E)], dtype=np.int64)


def test_search_forms_match_the_oracle(dev, tiny, lib_qr):
    idx = _index(tiny)
    Q = tiny["Q"]
    jobs, outs = [], []
    for name, skw, okw, nq in SEARCH_FORMS:
        say(f"Index.search form {name}: {nq} queries, k 10, ef 64/64")
        ids, d, cnt, st = idx.search(Q[:nq], 10, 64, 64, with_counters=True, **skw)
        outs.append((name, ids, d, cnt))
        okw = {k: (_fixed_entries(tiny, 8) if v == "F" else v) for k, v in okw.items()}
        jobs.append((np.arange(nq), dict(k=10, ef_gpu=64, ef_cpu=64, E=8, **okw)))
    say("oracle pipeline for every form (host worker processes)")
    refs = oracle_jobs.pipeline(_arrays(tiny), jobs)
    gt, _ = oracle.exact_knn(tiny["X"], Q, 10)
    for (name, ids, d, cnt), ref in zip(outs, refs):
        pipeline_check(ids, d, ref, name, cnt)
        say(f"  {name}: recall@10 {oracle.recall_at_k(ids, gt[:ids.shape[0]], 10):.4f}")
    idx.close()


def test_top100_matches_the_oracle(dev, tiny, lib_qr):
    idx = _index(tiny)
    nq = 300
    say(f"Index.search top-100: {nq} queries, ef_gpu 320, ef_cpu 160")
    ids, d, cnt, _ = idx.search(tiny["Q"][:nq], 100, 320, 160, with_counters=True)
    ref, = oracle_jobs.pipeline(_arrays(tiny), [(np.arange(nq), dict(k=100, ef_gpu=320, ef_cpu=160, E=8))])
    pipeline_check(ids, d, ref, "top-100", cnt)
    gt, _ = oracle.exact_knn(tiny["X"], tiny["Q"][:nq], 100)
    say(f"  recall@100 {oracle.recall_at_k(ids, gt, 100):.4f}")
    idx.close()


def test_compact_layout_matches_the_oracle(dev, tiny, lib_qr):
    Xr16 = tiny["Xr32"].astype(np.float16).astype(np.float32)
    idx = _index(tiny, "f16", compact=True)
    assert idx.info()["xr_rows"] == int(tiny["mask"].sum())
    nq = 1000
    say("compact layout (sampled rows only, fp16): Index.search against the oracle on the dequantised rows")
    ids, d, cnt, _ = idx.search(tiny["Q"][:nq], 10, 64, 64, with_counters=True, batch=300)
    ids2, d2, cnt2, _ = idx.search(tiny["Q"][:nq], 10, 64, 64, with_counters=True, stage_mask=2)
    # the entry table holds the pivots' fp32 rows (the same buckets as the full layout)
    a = _arrays(tiny, Xr=Xr16)
    refs = oracle_jobs.pipeline(a, [(np.arange(nq), dict(k=10, ef_gpu=64, ef_cpu=64, E=8)),
                                    (np.arange(nq), dict(k=10, ef_gpu=64, ef_cpu=64, E=8, use_gpu_stage=False))])
    pipeline_check(ids, d, refs[0], "compact fp16", cnt)
    pipeline_check(ids2, d2, refs[1], "compact fp16, no GPU stage", cnt2)
    idx.close()


def test_gpu_only_special_case_matches_the_oracle(dev, tiny):
    say("GPU-only special case: every node sampled, d_r = D, no final traversal; against the oracle")
    s = tiny["spec"]
    X, Q = tiny["X"], tiny["Q"][:500]
    D = X.shape[1]
    V64, _, _ = oracle.fit_projection(X, D, s.metric)
    V32 = V64.astype(np.float32)
    Xr = oracle.project(X, V32).astype(np.float32)
    full = np.ones(X.shape[0], dtype=np.uint8)
    pivots = tiny["pivots"]
    idx = pa.Index(pa.IndexConfig(dim=D, d_r=D, metric=s.metric, xr_dtype="f32", r=s.r, threads=4))
    idx.set_data(X, tiny["rp"], tiny["nb"])
    idx.set_projection(V32)
    idx.build_subgraph(full, tiny["rp"], tiny["nb"])
    idx.build_entries(pivots, tiny["init"], 10)
    # the oracle clusters the same pivots from the same seeds; the library's buckets agree
    b, c = oracle.balanced_kmeans(Xr[pivots].astype(np.float64), s.r, tiny["init"])
    c = c.astype(np.float32)
    _, lb, lc = idx.state()
    assert (lb == pivots[b]).all() and (lc.view(np.uint32) == c.view(np.uint32)).all()
    Qr = oracle.project(Q, V32).astype(np.float32)
    a = dict(Q=Q, Qr=Qr, X=X, V=V32, rp=tiny["rp"], nb=tiny["nb"], sr=tiny["rp"], sn=tiny["nb"], Xr=Xr, cent=c,
             buckets=b, P=Xr[pivots], pivots=pivots)
    outs, jobs = [], []
    for mask, refine in ((5, False), (7, True)):
        ids, d, cnt, _ = idx.search(Q, 10, 64, 64, stage_mask=mask, with_counters=True)
        assert (cnt[:, 4] == 0).all() and (cnt[:, 0] > 0).all()
        outs.append((mask, ids, d, cnt))
        jobs.append((np.arange(Q.shape[0]), dict(k=10, ef_gpu=64, ef_cpu=64, E=8, use_refine=refine,
                                                 use_final=False)))
    refs = oracle_jobs.pipeline(a, jobs)
    for (mask, ids, d, cnt), ref in zip(outs, refs):
        pipeline_check(ids, d, ref, f"stage_mask {mask}", cnt)
    with pytest.raises(pa.PilotannError):  # the final traversal cannot be skipped without the GPU stage
        idx.search(Q[:4], 10, 64, 64, stage_mask=6)
    idx.close()


def _requests(tiny, n, seed=11):
    rng = np.random.default_rng(seed)
    ks = rng.choice([10, 50, 100], size=n)
    efs = rng.choice([64, 128, 256, 512], size=n)
    return [(i, int(ks[i]), int(efs[i])) for i in range(n)]


def test_server_results_match_the_oracle(dev, tiny, lib_qr):
    idx = _index(tiny)
    n = 160
    reqs = _requests(tiny, n)
    say(f"server: {n} requests with k in {{10, 50, 100}} and ef in {{64, ..., 512}}, against the oracle")
    srv = pa.Server(idx, hbm_budget=1 << 30, max_batch=48, streams=3, threads=4)
    for tag, k, ef in reqs:
        srv.submit(tiny["Q"][tag], k, ef, tag)
    srv.drain()
    got = {r["tag"]: r for r in srv.poll(1000)}
    st = srv.stats()
    srv.close()
    assert st["completed"] == n and st["max_batch"] > 1
    n_b = tiny["spec"].n_pivots // tiny["spec"].r
    groups = {}
    for tag, k, ef in reqs:
        groups.setdefault((k, max(ef, k)), []).append(tag)
    keys = sorted(groups)
    jobs = [(np.asarray(groups[key]), dict(k=key[0], ef_gpu=key[1], ef_cpu=key[1], E=min(key[1], n_b)))
            for key in keys]
    refs = oracle_jobs.pipeline(_arrays(tiny), jobs)
    for key, ref in zip(keys, refs):
        tags = groups[key]
        ids = np.stack([got[t]["ids"] for t in tags])
        d = np.stack([got[t]["dists"] for t in tags])
        pipeline_check(ids, d, ref, f"server k={key[0]} ef={key[1]}")
    idx.close()


def test_ragged_traverse_matches_the_oracle(dev, tiny):
    say("gpu_traverse_ragged: per-query ef in {1, 8, 33, 64, 100, 256, 512} against the oracle")
    ent, _, _, _ = oracle_entries(tiny, 8)
    rng = np.random.default_rng(4)
    m = 400
    efs = rng.choice([1, 8, 33, 64, 100, 256, 512], size=m).astype(np.int32)
    Qr = tiny["Qr32"][:m]
    ids, d, cnt = pa.gpu_traverse_ragged(_t(Qr, dev), _t(tiny["Xr32"], dev), _t(tiny["sub_adj"].astype(np.int32), dev),
                                         _t(ent[:m].astype(np.int32), dev), _t(efs, dev))
    ids, d, cnt = ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy()
    # a row of list size ef starts from its first min(E, ef) entries
    ent_use = np.where(np.arange(8)[None, :] < np.minimum(efs, 8)[:, None], ent[:m], -1)
    refs = oracle_jobs.traverse(Qr, tiny["Xr32"].astype(np.float64), tiny["sr"], tiny["sn"], ent_use,
                                np.arange(m), efs)
    tally = DistTally()
    bad = 0
    for i, r in enumerate(refs):
        ef = int(efs[i])
        ref = np.full(ef, -1)
        ref[:r["ids"].size] = r["ids"]
        assert (ids[i, ef:] == -1).all()
        if not (ids[i, :ef] == ref).all():
            assert r["margin"] <= TIE, (i, ef, r["margin"])
            bad += 1
            continue
        tally.check(d[i, :r["ids"].size], r["dists"], i)
        if r["margin"] > TIE:
            assert cnt[i, 0] == r["n_exp"]
            if cnt[i, 2] == 0:
                assert cnt[i, 1] == r["n_dist"]
    off = tally.done()
    say(f"  {m} queries, {bad} differ (near ties), {off} distances 1 ulp off")
    assert bad <= max(1, m // 1000)


def test_ragged_traverse_with_bloom_filter_and_width_two_matches_the_oracle(dev, tiny):
    say("gpu_traverse with per-query ef in {8, 33, 64, 100}, the Bloom filter (2^15 bits) and width 2")
    ent, _, _, _ = oracle_entries(tiny, 8)
    rng = np.random.default_rng(6)
    m = 300
    efs = rng.choice([8, 33, 64, 100], size=m).astype(np.int32)
    Qr = tiny["Qr32"][:m]
    ids, d, cnt = pa.gpu_traverse_ragged(_t(Qr, dev), _t(tiny["Xr32"], dev), _t(tiny["sub_adj"].astype(np.int32), dev),
                                         _t(ent[:m].astype(np.int32), dev), _t(efs, dev), bloom_log2=15, width=2)
    ids, d, cnt = ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy()
    assert (cnt[:, 2] == 0).all()
    ent_use = np.where(np.arange(8)[None, :] < np.minimum(efs, 8)[:, None], ent[:m], -1)
    refs = oracle_jobs.traverse(Qr, tiny["Xr32"].astype(np.float64), tiny["sr"], tiny["sn"], ent_use,
                                np.arange(m), efs, bloom_log2=15, width=2)
    bad = 0
    tally = DistTally()
    for i, r in enumerate(refs):
        ef = int(efs[i])
        ref = np.full(ef, -1)
        ref[:r["ids"].size] = r["ids"]
        if not (ids[i, :ef] == ref).all():
            assert r["margin"] <= TIE, (i, ef, r["margin"])
            bad += 1
            continue
        tally.check(d[i, :r["ids"].size], r["dists"], i)
        if r["margin"] > TIE:
            assert cnt[i, 0] == r["n_exp"] and cnt[i, 1] == r["n_dist"]
    tally.done()
    assert bad <= max(1, m // 1000)
