"""GPU parity: every stage-isolated entry point against the oracle on the same
seeded inputs (the 10K x 96 workload: several tiles, a ragged tail), plus edge
cases.  The bar (see tests/parity.py for the reasoning):
* distances: the correctly rounded fp32 value on both sides, so within 1 ulp of
  the oracle's everywhere and identical on all but a 1e-4 fraction;
* ids: the ordered list equals the oracle's; a query may differ only where the
  oracle's near-tie margin is at most two ulps, and on at most 0.1% of queries;
* counters equal wherever the ids are equal, no near tie occurred and the
  visited cache never reset.
The projection is compared against the rounded exact product (it is the same bits on
all but a tiny fraction of the values) and against its rigorous error bound.
"""

import numpy as np
import pytest

import oracle
import paper_2503_21206_amd as pa
from tests.gpu_checks import traverse_check as _traverse_check
from tests.parity import TIE, DistTally
from tests.workload import build_tiny, device_tables, oracle_entries, to_bf16, to_f16

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


def _t(a, dev, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev).contiguous()


def say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------ projection

def test_projection_within_its_error_bound(dev, tiny):
    say("project tiny X (10000x96 -> 32) and a ragged 37-row slice")
    X, V = tiny["X"], tiny["V32"]
    for rows in (X, X[:37]):
        Y = pa.project(_t(rows, dev), _t(V, dev), "f32").cpu().numpy()
        ref = rows.astype(np.float64) @ V.astype(np.float64)
        bound = 2 * 96 * 2.0 ** -24 * (np.abs(rows.astype(np.float64)) @ np.abs(V.astype(np.float64)))
        assert (np.abs(Y - ref) <= bound + 1e-30).all()


def test_projection_converters_bit_exact(dev, tiny):
    say("project with f16 / bf16 outputs")
    Xt, Vt = _t(tiny["X"][:1000], dev), _t(tiny["V32"], dev)
    y32 = pa.project(Xt, Vt, "f32").cpu().numpy()
    y16 = pa.project(Xt, Vt, "f16").cpu().numpy()
    ybf = pa.project(Xt, Vt, "bf16").float().cpu().numpy()
    assert (y16.view(np.uint16) == y32.astype(np.float16).view(np.uint16)).all()
    assert (ybf == to_bf16(y32)).all()


def test_gram_f64_and_fit_projection(dev, tiny):
    say("gram_f64 on tiny X, then fit_projection")
    X = tiny["X"]
    G = torch.zeros((96, 96), dtype=torch.float64, device=dev)
    cs = torch.zeros((96,), dtype=torch.float64, device=dev)
    pa.gram_f64(_t(X[:6000], dev), G, cs, accumulate=False)
    pa.gram_f64(_t(X[6000:], dev), G, cs, accumulate=True)
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    np.testing.assert_allclose(G.cpu().numpy(), X64.T @ X64, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(cs.cpu().numpy(), X64.sum(0), rtol=1e-12, atol=1e-9)
    V, w, mu = pa.fit_projection(X, 32, center=True)
    np.testing.assert_allclose(w, tiny["evals"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(mu, tiny["mean"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(V.T.astype(np.float64) @ V, np.eye(32), atol=2e-6)
    # same subspace where the eigengap allows it (Davis-Kahan), and the same captured variance
    Vo = tiny["V64"]
    C = np.cov(X64.T, bias=True)
    np.testing.assert_allclose(np.trace(V.T.astype(np.float64) @ C @ V), tiny["evals"][:32].sum(), rtol=1e-6)
    gap = (tiny["evals"][31] - tiny["evals"][32]) / tiny["evals"][0]
    if gap > 1e-6:
        P1 = V.astype(np.float64) @ V.T
        P2 = Vo @ Vo.T
        assert np.linalg.norm(P1 - P2, 2) <= 1e-5 / gap


# ------------------------------------------------------------ entry selection

def _fes_check(dev, w, E, Qr, metric="l2"):
    EV, EVn, EVid = device_tables(w)
    oi, od, ocl, margin = oracle_entries(w, E, Qr)
    ids, d = pa.select_entries(_t(Qr, dev), _t(ocl.astype(np.int32), dev), _t(EV, dev), _t(EVn, dev),
                               _t(EVid, dev), E, metric)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    tally = DistTally()
    bad = 0
    for i in range(Qr.shape[0]):
        if not (ids[i] == oi[i]).all():
            assert margin[i] <= TIE, (i, ids[i], oi[i], margin[i])
            bad += 1
            continue
        tally.check(d[i], od[i], i)
    tally.done()
    return bad


def test_select_entries(dev, tiny):
    say("select_entries E=8 (bucket size 8) and E=12 (padded)")
    bad = _fes_check(dev, tiny, 8, tiny["Qr32"])
    assert bad <= tiny["Q"].shape[0] // 1000
    _fes_check(dev, tiny, 12, tiny["Qr32"][:100])
    _fes_check(dev, tiny, 3, tiny["Qr32"][:5])


def test_route_and_entries_with_64_buckets(dev, tiny):
    say("r = 64 buckets (one per lane of a wavefront): routing, select_entries E=4, and the index build")
    from synth import kmeans_init_choice
    s = tiny["spec"]
    r = 64
    init = kmeans_init_choice(s.n_pivots, r, s.seed)
    b, cent = oracle.balanced_kmeans(tiny["P32"], r, init)
    w = dict(tiny, buckets=b, cent32=cent.astype(np.float32))
    Q, V = tiny["Q"], tiny["V32"]
    _, cl = pa.project_route(_t(Q, dev), _t(V, dev), _t(w["cent32"], dev))
    cl = cl.cpu().numpy()
    bad = 0
    for i in range(Q.shape[0]):
        c, margin = oracle.route(tiny["Qr32"][i], w["cent32"].astype(np.float64))
        if c != cl[i]:
            assert margin <= TIE, (i, c, cl[i], margin)
            bad += 1
    assert bad <= max(1, Q.shape[0] // 1000)
    assert _fes_check(dev, w, 4, tiny["Qr32"]) <= Q.shape[0] // 1000
    # the index clusters its pivots into the same 64 buckets and searches with them
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, r=r, threads=4))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    idx.set_projection(V)
    idx.build_subgraph(tiny["mask"], tiny["sr"], tiny["sn"])
    idx.build_entries(tiny["pivots"], init, 10)
    _, buckets, _ = idx.state()  # balanced: 64 buckets of 4, every pivot once
    assert buckets.shape == (r, s.n_pivots // r) and np.array_equal(np.sort(buckets.ravel()), np.sort(tiny["pivots"]))
    ids, d, _, _ = idx.search(Q, 10, 64, 64)
    rec = oracle.recall_at_k(ids, oracle.exact_knn(tiny["X"], Q, 10)[0], 10)
    say(f"  recall@10 {rec:.4f}")
    assert rec >= 0.9
    idx.close()


# ------------------------------------------------------------ traversal

def test_traverse_f32_parity(dev, tiny):
    say("gpu_traverse f32 ef=64, 1000 queries")
    ent, _, _, _ = oracle_entries(tiny, 8)
    Xr = _t(tiny["Xr32"], dev)
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 64, np.arange(tiny["Q"].shape[0]))


def test_traverse_edge_cases(dev, tiny):
    ent, _, _, _ = oracle_entries(tiny, 8)
    Xr = _t(tiny["Xr32"], dev)
    say("gpu_traverse ef=1, ragged batches m=1 and m=3")
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 1, np.arange(200))
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 16, np.array([5]))
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 16, np.array([7, 8, 9]))
    say("gpu_traverse ef=512 (maximum), 40 queries")
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 512, np.arange(40))
    say("gpu_traverse tiny visited cache (forced resets) stays exact")
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, 64, np.arange(100), cache_log2=8, expect_reset=True)
    say("gpu_traverse with -1 / out-of-range entries and an empty entry list")
    bad = ent.copy()
    bad[:, 0] = -1
    bad[:, 1] = 10 ** 6
    bad[:, 2] = -7
    _traverse_check(dev, tiny, tiny["Xr32"], Xr, bad, 32, np.arange(50))
    Qr = _t(tiny["Qr32"][:4], dev)
    adj = _t(tiny["sub_adj"].astype(np.int32), dev)
    ids, d, cnt = pa.gpu_traverse(Qr, Xr, adj, torch.empty((4, 0), dtype=torch.int32, device=dev), 8)
    assert (ids.cpu().numpy() == -1).all() and (cnt.cpu().numpy()[:, :2] == 0).all()
    say("gpu_traverse m=0")
    ids, d, cnt = pa.gpu_traverse(Qr[:0], Xr, adj, torch.empty((0, 8), dtype=torch.int32, device=dev), 8)
    assert ids.shape == (0, 8)
    with pytest.raises(pa.PilotannError):
        pa.gpu_traverse(Qr, Xr, adj, _t(ent[:4].astype(np.int32), dev), 513)


def test_traverse_bloom_filter_parity(dev, tiny):
    ent, _, _, _ = oracle_entries(tiny, 8)
    Xr = _t(tiny["Xr32"], dev)
    for lg, ef, nq in ((13, 64, 300), (15, 64, 300), (18, 32, 300), (16, 200, 60)):
        say(f"gpu_traverse with the Bloom visited filter: 2^{lg} bits, ef={ef}, {nq} queries")
        _, _, cnt = _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, ef, np.arange(nq), bloom_log2=lg)
        assert (cnt[:, 2] == 0).all()
    say("Bloom filter with fp16 rows and duplicate / out-of-range entries")
    xh = to_f16(tiny["Xr32"])
    bad = ent.copy()
    bad[:, 1] = bad[:, 0]
    bad[:, 2] = 10 ** 6
    _traverse_check(dev, tiny, np.asarray(xh, dtype=np.float32), _t(np.asarray(xh, dtype=np.float32), dev,
                    torch.float16), bad, 48, np.arange(200), bloom_log2=14)
    Qr = _t(tiny["Qr32"][:4], dev)
    adj = _t(tiny["sub_adj"].astype(np.int32), dev)
    with pytest.raises(pa.PilotannError):  # a filter below 128 bits per list entry
        pa.gpu_traverse(Qr, Xr, adj, _t(ent[:4].astype(np.int32), dev), 256, bloom_log2=13)


def test_traverse_width_two_parity(dev, tiny):
    ent, _, _, _ = oracle_entries(tiny, 8)
    Xr = _t(tiny["Xr32"], dev)
    for ef, bloom, cl, nq in ((64, None, 0, 300), (16, None, 0, 200), (200, None, 0, 60), (64, 15, 0, 200),
                              (64, None, 8, 100)):
        say(f"gpu_traverse, two entries expanded per step: ef={ef}, Bloom 2^{bloom} bits, cache_log2={cl}")
        _traverse_check(dev, tiny, tiny["Xr32"], Xr, ent, ef, np.arange(nq), cache_log2=cl, bloom_log2=bloom,
                        width=2)
    say("width 2 with fp16 rows")
    xh = np.asarray(to_f16(tiny["Xr32"]), dtype=np.float32)
    _traverse_check(dev, tiny, xh, _t(xh, dev, torch.float16), ent, 48, np.arange(200), width=2)
    Qr = _t(tiny["Qr32"][:4], dev)
    adj33 = _t(np.full((tiny["X"].shape[0], 33), -1, np.int32), dev)
    with pytest.raises(pa.PilotannError):  # two rows of more than 32 ids do not fit one wavefront
        pa.gpu_traverse(Qr, Xr, adj33, _t(ent[:4].astype(np.int32), dev), 16, width=2)
    say("Index.search with width 2: recall against width 1")
    s = tiny["spec"]
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f32", r=s.r, threads=4))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    idx.set_projection(tiny["V32"])
    idx.build_subgraph(tiny["mask"], tiny["sr"], tiny["sn"])
    idx.build_entries(tiny["pivots"], tiny["init"], 10)
    gt, _ = oracle.exact_knn(tiny["X"], tiny["Q"], 10)
    r1 = oracle.recall_at_k(idx.search(tiny["Q"], 10, 64, 64)[0], gt, 10)
    ids2, _, cnt2, _ = idx.search(tiny["Q"], 10, 64, 64, width=2, with_counters=True)
    r2 = oracle.recall_at_k(ids2, gt, 10)
    say(f"  recall@10 width 1 {r1:.4f}, width 2 {r2:.4f}")
    assert r2 >= r1 - 0.01
    idx.close()


def test_traverse_exact_ties_and_near_ties(dev, tiny):
    # every row repeated (equal distances: the id decides) and a copy nudged by one ulp
    # (distances a few units apart in fp32): the plain scores cannot order these, so the
    # steps are decided on exactly re-scored keys, and the lists must still be the oracle's
    say("gpu_traverse on rows with exact duplicates and one-ulp neighbours, exact and Bloom visited sets")
    base = tiny["Xr32"][:3000]
    nudged = np.nextafter(base, np.float32(np.inf)).astype(np.float32)
    Xr = np.concatenate([base, base, nudged]).astype(np.float32)
    n = Xr.shape[0]
    rng = np.random.default_rng(5)
    R = 16
    rows = []
    for u in range(n):  # a random graph over the copies, with the copies of u linked
        k = u % 3000
        nb = set(rng.choice(n, R - 2, replace=False).tolist()) | {k, k + 3000}
        nb.discard(u)
        rows.append(sorted(nb)[:R])
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    nbrs = np.concatenate([np.asarray(r, dtype=np.int64) for r in rows])
    w = dict(Qr32=tiny["Qr32"][:200], sr=rp, sn=nbrs, sub_adj=oracle.padded_from_csr(rp, nbrs, R))
    ent = rng.choice(n, (200, 8)).astype(np.int64)
    for bloom in (None, 16):
        _traverse_check(dev, w, Xr, _t(Xr, dev), ent, 32, np.arange(200), bloom_log2=bloom)


def test_traverse_f16_and_bf16(dev, tiny):
    ent, _, _, _ = oracle_entries(tiny, 8)
    for name, conv, tdt in (("f16", to_f16, torch.float16), ("bf16", to_bf16, torch.bfloat16)):
        say(f"gpu_traverse {name} reduced vectors ef=64, 500 queries")
        xh = conv(tiny["Xr32"])
        Xr = _t(np.asarray(xh, dtype=np.float32), dev, tdt)
        _traverse_check(dev, tiny, np.asarray(xh, dtype=np.float32), Xr, ent, 64, np.arange(500))


def test_traverse_deterministic_and_batch_invariant(dev, tiny):
    say("gpu_traverse twice + alone-vs-batch")
    ent, _, _, _ = oracle_entries(tiny, 8)
    Xr = _t(tiny["Xr32"], dev)
    adj = _t(tiny["sub_adj"].astype(np.int32), dev)
    Qr = _t(tiny["Qr32"], dev)
    E = _t(ent.astype(np.int32), dev)
    a = [x.cpu().numpy() for x in pa.gpu_traverse(Qr, Xr, adj, E, 96)]
    b = [x.cpu().numpy() for x in pa.gpu_traverse(Qr, Xr, adj, E, 96)]
    for x, y in zip(a, b):
        assert (x.view(np.uint8) == y.view(np.uint8)).all()
    for i in (0, 17, 999):
        s = [x.cpu().numpy() for x in pa.gpu_traverse(Qr[i:i + 1], Xr, adj, E[i:i + 1], 96)]
        assert (s[0][0] == a[0][i]).all() and (s[1][0].view(np.uint32) == a[1][i].view(np.uint32)).all()


def test_traverse_inner_product(dev):
    say("gpu_traverse inner product on unit-norm anisotropic data (4000 x 64 -> 32)")
    from synth.data import anisotropic_points
    from synth.graph import build_graph, padded_to_csr
    X = anisotropic_points(77, 4000, 64, 16)
    Q = anisotropic_points(78, 200, 64, 16, stream_offset=1)
    adj = build_graph(X, 16, device="cpu")
    rp, nb = padded_to_csr(adj)
    V, _, _ = oracle.fit_projection(X, 32, "ip")
    V32 = V.astype(np.float32)
    Xr = oracle.project(X, V32).astype(np.float32)
    Qr = oracle.project(Q, V32).astype(np.float32)
    ent = np.stack([np.arange(0, 4000, 500)] * 200).astype(np.int32)
    w = dict(Qr32=Qr, sub_adj=adj, sr=rp, sn=nb)
    _traverse_check(dev, w, Xr, _t(Xr, dev), ent, 48, np.arange(200), metric="ip")


# ------------------------------------------------------------ full pipeline

def test_index_pipeline_matches_oracle(dev, tiny):
    say("Index: set_data, set_projection, sample, build_subgraph, build_entries, search")
    s = tiny["spec"]
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f32", r=s.r, threads=4))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    idx.set_projection(tiny["V32"])
    from synth import node_order
    mask = idx.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
    assert (mask == tiny["mask"]).all()
    idx.build_subgraph(mask, tiny["sr"], tiny["sn"])
    idx.build_entries(tiny["pivots"], tiny["init"], 10)
    V, b, c = idx.state()
    assert (V == tiny["V32"]).all()
    Q = tiny["Q"]
    ids, d, cnt, st = idx.search(Q, 10, 64, 64, with_counters=True, batch=300)
    assert st["beam_launches"] == 4 and st["beam_ms"] > 0
    # (the results themselves are compared with the oracle in test_gpu_oracle_parity.py)
    # queries already resident in HBM: identical results, no upload
    Qd = _t(Q, dev)
    ids_d, d_d, _, _ = idx.search(Q, 10, 64, 64, batch=300, Q_dev=Qd)
    assert (ids_d == ids).all() and (d_d.view(np.uint32) == d.view(np.uint32)).all()
    import ctypes
    opts = pa.SearchOpts(64, 64, 0, 0, 0, 0, 0, 0, Q.ctypes.data, 0, 1)  # a host pointer is refused
    out_i = np.empty((Q.shape[0], 10), np.int64)
    out_d = np.empty((Q.shape[0], 10), np.float32)
    st = pa.lib().pa_search(idx._h, Q.ctypes.data_as(ctypes.c_void_p), Q.shape[0], 10, ctypes.byref(opts),
                            out_i.ctypes.data_as(ctypes.c_void_p), out_d.ctypes.data_as(ctypes.c_void_p), None, None)
    assert st == -1
    # stage 1 with the paper's Bloom visited filter (automatic size: 2^15 bits at ef 64) never
    # resets; no GPU stage = plain greedy search from the FES entries (no stage-1 counters)
    _, _, cnt_b, _ = idx.search(Q, 10, 64, 64, with_counters=True, batch=300, bloom=True)
    assert (cnt_b[:, 2] == 0).all()
    _, _, cnt0, _ = idx.search(Q[:100], 10, 64, 64, stage_mask=2, with_counters=True)
    assert (cnt0[:, 0] == 0).all()
    idx.close()


def test_compact_layout_matches_full_layout(dev, tiny, tmp_path):
    say("Index with X_r and the subgraph for the sampled nodes only, against the full layout")
    s = tiny["spec"]
    Q = tiny["Q"]
    out = {}
    for compact in (False, True):
        idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f16", r=s.r, threads=4,
                                      compact=compact))
        idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
        if compact:  # the subgraph first: the rows are written when the projection arrives
            idx.build_subgraph(tiny["mask"], tiny["sr"], tiny["sn"])
            assert idx.info()["xr_rows"] == 0
            idx.set_projection(tiny["V32"])
        else:
            idx.set_projection(tiny["V32"])
            idx.build_subgraph(tiny["mask"], tiny["sr"], tiny["sn"])
        idx.build_entries(tiny["pivots"], tiny["init"], 10)
        info = idx.info()
        ids, d, cnt, _ = idx.search(Q, 10, 64, 64, with_counters=True, batch=300)
        ids0, d0, _, _ = idx.search(Q[:200], 10, 64, 64, stage_mask=2)  # GPU stage off: FES ids on the host
        idsb, _, _, _ = idx.search(Q, 10, 64, 64, batch=300, bloom=True)
        out[compact] = dict(info=info, ids=ids, d=d, cnt=cnt, ids0=ids0, d0=d0, idsb=idsb)
        if compact:
            path = str(tmp_path / "compact.pidx")
            idx.save(path)
            idx2 = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f16", r=s.r,
                                           threads=4, compact=True))
            idx2.set_data(tiny["X"], tiny["rp"], tiny["nb"])
            idx2.load(path)
            assert idx2.info()["xr_rows"] == info["xr_rows"]
            i2, d2, _, _ = idx2.search(Q, 10, 64, 64, batch=300)
            assert (i2 == ids).all() and (d2.view(np.uint32) == d.view(np.uint32)).all()
            idx2.close()
            with pytest.raises(pa.PilotannError):  # a full-layout index refuses a compact checkpoint
                idx3 = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f16", r=s.r))
                idx3.set_data(tiny["X"], tiny["rp"], tiny["nb"])
                idx3.load(path)
        idx.close()
    full, comp = out[False], out[True]
    n_s = int(tiny["mask"].sum())
    say(f"  rows on the device {full['info']['xr_rows']} -> {comp['info']['xr_rows']}, "
        f"HBM {full['info']['hbm_bytes']} -> {comp['info']['hbm_bytes']} bytes")
    assert full["info"]["xr_rows"] == tiny["X"].shape[0] and comp["info"]["xr_rows"] == n_s
    assert comp["info"]["hbm_bytes"] < full["info"]["hbm_bytes"]
    # device ids keep the node order, so every decision and every result is the same
    assert (comp["ids"] == full["ids"]).all() and (comp["d"].view(np.uint32) == full["d"].view(np.uint32)).all()
    assert (comp["cnt"][:, 0] == full["cnt"][:, 0]).all()
    assert (comp["ids0"] == full["ids0"]).all() and (comp["d0"].view(np.uint32) == full["d0"].view(np.uint32)).all()
    gt, _ = oracle.exact_knn(tiny["X"], Q, 10)
    rb_full, rb_comp = oracle.recall_at_k(full["idsb"], gt, 10), oracle.recall_at_k(comp["idsb"], gt, 10)
    say(f"  Bloom filter (hashes of node ids vs device ids): recall {rb_full:.4f} vs {rb_comp:.4f}")
    assert abs(rb_full - rb_comp) <= 0.01


def test_memory_model_predicts_the_index_bytes(dev, tiny):
    say("memory-bounded mode: the HBM model against the bytes three index forms hold, and the planner's budget")
    s = tiny["spec"]
    Q = tiny["Q"]
    N = tiny["X"].shape[0]
    rho = int(tiny["mask"].sum()) / N
    n_p = len(tiny["pivots"])

    def build(compact, xr, piv, budget=0):
        idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype=xr, r=s.r, threads=4,
                                      compact=compact, pivot_dtype=piv, hbm_budget=budget))
        idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
        idx.set_projection(tiny["V32"])
        idx.build_subgraph(tiny["mask"], tiny["sr"], tiny["sn"])
        idx.build_entries(tiny["pivots"], tiny["init"], 10)
        return idx

    for compact, xr, piv in ((True, "f16", "f32"), (False, "f32", "f32"), (True, "bf16", "fp8")):
        idx = build(compact, xr, piv)
        R_sub = idx.info()["R_sub"]
        shape = pa.memory_shape(N, s.dim, R_sub, n_p, s.r, xr, piv, compact)
        assert idx.info()["hbm_bytes"] == pa.hbm_bytes(shape, rho, s.d_r), (compact, xr, piv)
        idx.search(Q, 10, 64, 64, batch=300)
        shape = pa.memory_shape(N, s.dim, R_sub, n_p, s.r, xr, piv, compact, queries=Q.shape[0], batch=300,
                                ef_gpu=64)
        assert idx.info()["hbm_bytes"] == pa.hbm_bytes(shape, rho, s.d_r), (compact, xr, piv)
        idx.close()
    # the planner's pair for a budget of exactly its bytes: the index builds and searches
    # within it, and one byte less is refused when the search buffers are allocated
    shape = pa.memory_shape(N, s.dim, R_sub, n_p, s.r, "f16", queries=Q.shape[0], batch=300, ef_gpu=64)
    need = pa.hbm_bytes(shape, rho, s.d_r)
    assert pa.plan_memory(shape, need, [rho], [16, s.d_r, 2 * s.d_r]) == (rho, s.d_r, need)
    idx = build(True, "f16", "f32", budget=need)
    ids, _, _, _ = idx.search(Q, 10, 64, 64, batch=300)
    assert idx.info()["hbm_bytes"] == need and (ids >= 0).all()
    idx.close()
    idx = build(True, "f16", "f32", budget=need - 1)
    with pytest.raises(pa.PilotannError) as e:
        idx.search(Q, 10, 64, 64, batch=300)
    assert e.value.status == -4  # PA_EHBM
    idx.close()


# ------------------------------------------------------------ large buckets and the FP8 form

def _big_bucket_tables(tiny, n_p=4096, r=2):
    from synth import kmeans_init_choice, pivot_choice
    S = np.nonzero(tiny["mask"])[0]
    pivots = pivot_choice(np.arange(tiny["X"].shape[0]), n_p, 77)
    P = tiny["Xr32"][pivots]
    b, c = oracle.balanced_kmeans(P, r, kmeans_init_choice(n_p, r, 77), iters=3)
    EV = P[b].astype(np.float32)
    EVn = (EV.astype(np.float64) ** 2).sum(-1).astype(np.float32)
    EVid = pivots[b].astype(np.int32)
    del S
    return P, pivots, b, c.astype(np.float32), EV, EVn, EVid


@pytest.mark.parametrize("n_p,r,E", [(4096, 2, 32), (4096, 4, 64), (4096, 8, 64), (4096, 32, 128)])
def test_select_entries_chunked_large_bucket(dev, tiny, n_p, r, E):
    # buckets of 2,048 pivots (candidate list shrunk chunk by chunk), 1,024 and 512 (scores
    # in registers) and 128 (one chunk), the last with E equal to the bucket size
    say(f"select_entries with {n_p // r}-pivot buckets, E={E}")
    P, pivots, b, cent, EV, EVn, EVid = _big_bucket_tables(tiny, n_p, r)
    Qr = tiny["Qr32"][:300]
    oi, od, ocl, margin = oracle.select_entries(Qr, cent.astype(np.float64), b, P, pivots, E)
    ids, d = pa.select_entries(_t(Qr, dev), _t(ocl.astype(np.int32), dev), _t(EV, dev), _t(EVn, dev), _t(EVid, dev),
                               E)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    tally = DistTally()
    bad = 0
    for i in range(Qr.shape[0]):
        if not (ids[i] == oi[i]).all():
            assert margin[i] <= TIE, (i, margin[i])
            bad += 1
            continue
        tally.check(d[i], od[i], i)
    tally.done()
    assert bad <= 1


@pytest.mark.parametrize("n_p,r", [(4096, 2), (8192, 2), (4096, 8)])
def test_select_entries_fp8_preselect_then_fp32_rerank(dev, tiny, n_p, r):
    # buckets of 2,048 and 512 pivots (scores in registers) and 4,096 (candidate list)
    say(f"select_entries_fp8 with {n_p // r}-pivot buckets, E=16, K=64")
    P, pivots, b, cent, EV, EVn, EVid = _big_bucket_tables(tiny, n_p, r)
    codes, scales = pa.quantize_fp8_rows(EV.reshape(-1, EV.shape[-1]))
    EV8 = codes.reshape(EV.shape)
    EVs = scales.reshape(EV.shape[:2])
    Qr = tiny["Qr32"][:300]
    oi, od, ocl, _ = oracle.select_entries(Qr, cent.astype(np.float64), b, P, pivots, 16)
    ids, d = pa.select_entries_fp8(_t(Qr, dev), _t(ocl.astype(np.int32), dev), _t(EV, dev), _t(EV8, dev),
                                   _t(EVs, dev), _t(EVn, dev), _t(EVid, dev), 16, 64)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    overlap = np.mean([len(set(ids[i]) & set(oi[i])) / 16 for i in range(Qr.shape[0])])
    exact = np.mean([(ids[i] == oi[i]).all() for i in range(Qr.shape[0])])
    say(f"fp8 pre-selection: overlap@16 {overlap:.4f}, identical lists {exact:.4f}")
    assert overlap >= 0.99
    # every returned distance is the correctly rounded fp32 distance of its pivot
    Xr64 = tiny["Xr32"].astype(np.float64)
    tally = DistTally()
    for i in range(Qr.shape[0]):
        tally.check(d[i], oracle.as_f32(oracle.delta_many(Qr[i], Xr64[ids[i]])), i)
    tally.done()



def _ord_f32(v):
    u = np.asarray(v, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return np.where(u & 0x80000000, (~u) & 0xFFFFFFFF, u | 0x80000000)


@pytest.mark.parametrize("n_b,K,E,d", [(512, 64, 16, 32), (2048, 256, 256, 32), (2048, 256, 64, 32),
                                       (4096, 256, 64, 32), (2048, 1024, 256, 128), (2048, 1024, 256, 256)])
def test_fp8_preselection_exact_on_integer_data(dev, n_b, K, E, d):
    # Small integers make every FP8 product sum exact in fp32 whatever the MFMA's order, so
    # the K best by (FP8 score, position) are known exactly, ties included (integer data has
    # many equal scores).  Buckets of 512 and 2,048 pivots keep the scores in registers
    # (2,048: the narrowed K-th search), 4,096 the candidate list; E = K = 256 emits the whole
    # pre-selection, re-scored exactly and ordered by (distance, node id).  K = 1,024 lists
    # fill most of the LDS: at d = 128 with 256-pivot chunks, at d = 256 with 128-pivot chunks.
    say(f"select_entries_fp8 on integer data: {n_b}-pivot buckets, d={d}, K={K}, E={E}")
    rng = np.random.default_rng(n_b + K + E + d)
    m, r = 300, 2
    Q = rng.integers(-3, 4, (m, d)).astype(np.float32)
    EV = rng.integers(-3, 4, (r, n_b, d)).astype(np.float32)
    EVid = rng.permutation(r * n_b).astype(np.int32).reshape(r, n_b)
    cl = rng.integers(0, r, m).astype(np.int32)
    codes, scales = pa.quantize_fp8_rows(EV.reshape(-1, d))
    ids, dist = pa.select_entries_fp8(_t(Q, dev), _t(cl, dev), _t(EV, dev), _t(codes.reshape(r, n_b, d), dev),
                                      _t(scales.reshape(r, n_b), dev),
                                      _t((EV.astype(np.float64) ** 2).sum(-1).astype(np.float32), dev), _t(EVid, dev),
                                      E, K, "ip")
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    # expected: the query's e4m3 codes (scale max|q| / 448, round to nearest even), exact
    # integer-multiple products, the score -acc * (s_q * s_p) in fp32
    dec = lambda c: torch.from_numpy(np.ascontiguousarray(c)).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    p8 = dec(codes).reshape(r, n_b, d)
    amax = np.abs(Q).max(1)
    sq = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    q8 = torch.from_numpy((Q / sq[:, None]).astype(np.float32)).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    ps = scales.reshape(r, n_b)
    for i in range(m):
        c = cl[i]
        acc = (p8[c] @ q8[i]).astype(np.float32)  # exact sums of exact products
        score = -(acc * (sq[i] * ps[c]))
        order = np.lexsort((np.arange(n_b), _ord_f32(score)))  # by (score, position)
        pre = order[:K]
        exact = (-(EV[c][pre].astype(np.float64) @ Q[i].astype(np.float64))).astype(np.float32)
        key = (_ord_f32(exact) << np.uint64(32)) | EVid[c][pre].astype(np.uint64)
        top = np.argsort(key, kind="stable")[:E]
        assert (ids[i] == EVid[c][pre][top]).all(), i
        assert (dist[i].view(np.uint32) == exact[top].view(np.uint32)).all(), i

def test_index_with_fp8_pivots(dev, tiny):
    say("Index with fp8 pivots: search recall close to the fp32-pivot index")
    s = tiny["spec"]
    from synth import node_order
    out = {}
    for pdt in ("f32", "fp8"):
        idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, r=s.r, threads=4, pivot_dtype=pdt))
        idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
        idx.set_projection(tiny["V32"])
        mask = idx.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
        idx.build_subgraph(mask, tiny["sr"], tiny["sn"])
        idx.build_entries(tiny["pivots"], tiny["init"], 10)
        out[pdt], _, _, _ = idx.search(tiny["Q"], 10, 64, 64)
        idx.close()
    gt, _ = oracle.exact_knn(tiny["X"], tiny["Q"], 10)
    r32, r8 = oracle.recall_at_k(out["f32"], gt, 10), oracle.recall_at_k(out["fp8"], gt, 10)
    say(f"recall@10 f32 pivots {r32:.4f}, fp8 pivots {r8:.4f}")
    assert r8 >= r32 - 0.01
