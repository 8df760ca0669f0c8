"""The code paths of the large configurations at small N: the 768-d inner-product form
(bf16 reduced vectors, d_r = 128, degree 48, 20% subgraph, FP8 pivots re-ranked in fp32)
and the 96-d form with fp16 reduced vectors at d_r = 48.  Same recipes as the full-size
workloads, fewer vectors; parity against the oracle as in the other GPU tests."""

import dataclasses

import numpy as np
import pytest

import oracle
import paper_2503_21206_amd as pa
from synth import SPECS, base_vectors, kmeans_init_choice, node_order, pivot_choice, query_vectors
from synth.graph import build_graph, build_subgraph_csr, padded_to_csr
from tests.gpu_checks import _t, say, traverse_check
from tests.parity import DistTally
from tests.workload import to_bf16, to_f16

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _fixture(spec):
    dev = "cuda"
    X, Q = base_vectors(spec), query_vectors(spec)
    adj = build_graph(X, spec.degree, device=dev)
    rp, nb = padded_to_csr(adj)
    mask = oracle.sample_nodes(rp, nb, node_order(spec.n, spec.seed), round(spec.rho * spec.n), spec.sample_mode)
    sr, sn = build_subgraph_csr(X, mask, spec.degree, device=dev)
    V64, _, _ = oracle.fit_projection(X, spec.d_r, spec.metric)
    V32 = V64.astype(np.float32)
    Xr32 = oracle.project(X, V32).astype(np.float32)
    Qr32 = oracle.project(Q, V32).astype(np.float32)
    S = np.nonzero(mask)[0]
    deg = sr[1:] - sr[:-1]
    pivots = pivot_choice(S[deg[S] > 0], spec.n_pivots, spec.seed)
    init = kmeans_init_choice(spec.n_pivots, spec.r, spec.seed)
    R_sub = int((sr[1:] - sr[:-1]).max())
    return dict(spec=spec, X=X, Q=Q, rp=rp, nb=nb, mask=mask, sr=sr, sn=sn, V32=V32, Xr32=Xr32, Qr32=Qr32,
                pivots=pivots, init=init, sub_adj=oracle.padded_from_csr(sr, sn, R_sub))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pa.device_init(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ip768(dev):
    say("fixture: 50,000 x 768 unit-norm anisotropic, inner product, degree 48, d_r 128, rho 0.2")
    return _fixture(dataclasses.replace(SPECS["aniso10m"], name="aniso50k", n=50_000, queries=200, n_pivots=8192))


@pytest.fixture(scope="module")
def l2_96(dev):
    say("fixture: 50,000 x 96 nested mixture, L2, degree 32, d_r 48, rho 0.25")
    return _fixture(dataclasses.replace(SPECS["gmm100m"], name="gmm50k", n=50_000, queries=300, n_pivots=2048))


def _entries(w, E, Xr_for_pivots):
    P = Xr_for_pivots[w["pivots"]].astype(np.float64)
    b, c = oracle.balanced_kmeans(P, w["spec"].r, w["init"])
    ids, d, cl, margin = oracle.select_entries(w["Qr32"], c, b, P, w["pivots"], E, w["spec"].metric)
    return ids, d, cl, b, c


def test_ip768_bf16_traversal(dev, ip768):
    say("gpu_traverse: 768-d IP, bf16 X_r (d_r 128), degree 48, ef 128, 200 queries")
    w = ip768
    xb = to_bf16(w["Xr32"])
    ent, _, _, _, _ = _entries(w, 32, w["Xr32"])
    traverse_check(dev, w, xb, _t(xb, dev, torch.bfloat16), ent, 128, np.arange(200), metric="ip")


def test_ip768_fp8_entries(dev, ip768):
    say("select_entries_fp8: 8,192 pivots in 32 buckets of 256, d_r 128, E 32, K 128; exact re-score")
    w = ip768
    E = 32
    oi, od, ocl, b, c = _entries(w, E, w["Xr32"])
    P = w["Xr32"][w["pivots"]]
    EV = P[b].astype(np.float32)
    EVn = (EV.astype(np.float64) ** 2).sum(-1).astype(np.float32)
    EVid = w["pivots"][b].astype(np.int32)
    codes, scales = pa.quantize_fp8_rows(EV.reshape(-1, EV.shape[-1]))
    ids, d = pa.select_entries_fp8(_t(w["Qr32"], dev), _t(ocl.astype(np.int32), dev), _t(EV, dev),
                                   _t(codes.reshape(EV.shape), dev), _t(scales.reshape(EV.shape[:2]), dev),
                                   _t(EVn, dev), _t(EVid, dev), E, 4 * E, "ip")
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    overlap = np.mean([len(set(ids[i]) & set(oi[i])) / E for i in range(ids.shape[0])])
    same = np.mean([(ids[i] == oi[i]).all() for i in range(ids.shape[0])])
    say(f"  fp8 pre-selection: overlap@{E} {overlap:.4f}, identical lists {same:.4f}")
    assert overlap >= 0.99
    tally = DistTally()
    for i in range(ids.shape[0]):
        tally.check(d[i], oracle.as_f32(oracle.delta_many(w["Qr32"][i], w["Xr32"][ids[i]], "ip")), i)
    tally.done()


def test_ip768_index_bf16_fp8(dev, ip768):
    say("Index: 768-d IP, bf16 X_r, fp8 pivots; search 200 queries at ef 128")
    w = ip768
    s = w["spec"]
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric="ip", xr_dtype="bf16", r=s.r, threads=4,
                                  pivot_dtype="fp8"))
    idx.set_data(w["X"], w["rp"], w["nb"])
    idx.set_projection(w["V32"])
    idx.build_subgraph(w["mask"], w["sr"], w["sn"])
    idx.build_entries(w["pivots"], w["init"], 10)
    ids, d, cnt, st = idx.search(w["Q"], 10, 128, 128, with_counters=True)
    gt, _ = oracle.exact_knn(w["X"], w["Q"], 10, "ip")
    rec = oracle.recall_at_k(ids, gt, 10)
    say(f"  recall@10 {rec:.4f}, mean stage-1 distances {cnt[:, 1].mean():.0f}, stage-3 {cnt[:, 4].mean():.0f}")
    assert rec >= 0.9
    tally = DistTally()
    for i in range(ids.shape[0]):
        tally.check(d[i], oracle.as_f32(oracle.delta_many(w["Q"][i], w["X"][ids[i]], "ip")), i)
    tally.done()
    idx.close()


def test_l2_96_fp16_traversal_and_index(dev, l2_96):
    w = l2_96
    s = w["spec"]
    say("gpu_traverse: 96-d L2, fp16 X_r (d_r 48), ef 64, 300 queries")
    xh = np.asarray(to_f16(w["Xr32"]), dtype=np.float32)
    ent, _, _, _, _ = _entries(w, 16, w["Xr32"])
    traverse_check(dev, w, xh, _t(xh, dev, torch.float16), ent, 64, np.arange(300))
    say("Index: 96-d L2, fp16 X_r; search 300 queries at ef 64")
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric="l2", xr_dtype="f16", r=s.r, threads=4))
    idx.set_data(w["X"], w["rp"], w["nb"])
    idx.set_projection(w["V32"])
    idx.build_subgraph(w["mask"], w["sr"], w["sn"])
    idx.build_entries(w["pivots"], w["init"], 10)
    ids, d, _, _ = idx.search(w["Q"], 10, 64, 64)
    gt, _ = oracle.exact_knn(w["X"], w["Q"], 10)
    rec = oracle.recall_at_k(ids, gt, 10)
    say(f"  recall@10 {rec:.4f}")
    assert rec >= 0.9
    tally = DistTally()
    for i in range(ids.shape[0]):
        tally.check(d[i], oracle.as_f32(oracle.delta_many(w["Q"][i], w["X"][ids[i]])), i)
    tally.done()
    idx.close()


def test_ip768_compact_layout_matches_full(dev, ip768):
    say("Index: 768-d IP, bf16 X_r, fp8 pivots; compact layout against the full layout, and a checkpoint round trip")
    w = ip768
    s = w["spec"]
    out = []
    for compact in (False, True):
        idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric="ip", xr_dtype="bf16", r=s.r, threads=4,
                                      pivot_dtype="fp8", compact=compact))
        idx.set_data(w["X"], w["rp"], w["nb"])
        idx.set_projection(w["V32"])
        idx.build_subgraph(w["mask"], w["sr"], w["sn"])
        idx.build_entries(w["pivots"], w["init"], 10)
        ids, d, _, _ = idx.search(w["Q"], 10, 128, 128)
        out.append((ids, d, idx.info()))
        idx.close()
    (i0, d0, f0), (i1, d1, f1) = out
    assert (i0 == i1).all() and (d0.view(np.uint32) == d1.view(np.uint32)).all()
    assert f1["xr_rows"] == int(w["mask"].sum()) and f1["hbm_bytes"] < f0["hbm_bytes"]
