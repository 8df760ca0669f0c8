"""Serving loop and per-query list sizes on the GPU: each request's result is
bit-identical alone, in a mixed micro-batch, and through the batch search; the
HBM budget makes requests queue instead of failing; errors are reported."""

import numpy as np
import pytest

import paper_2503_21206_amd as pa
from synth import node_order
from tests.workload import build_tiny, oracle_entries

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


@pytest.fixture(scope="module")
def index(dev, tiny):
    s = tiny["spec"]
    idx = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f32", r=s.r, threads=4))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    idx.set_projection(tiny["V32"])
    mask = idx.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
    idx.build_subgraph(mask, tiny["sr"], tiny["sn"])
    idx.build_entries(tiny["pivots"], tiny["init"], 10)
    yield idx
    idx.close()


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev)


def test_ragged_traverse_rows_equal_single_size_runs(dev, tiny):
    print("gpu_traverse_ragged with ef in {8,16,32,64,100} vs per-size runs", flush=True)
    ent, _, _, _ = oracle_entries(tiny, 8)
    rng = np.random.default_rng(3)
    m = 300
    efs = rng.choice([8, 16, 32, 64, 100], size=m).astype(np.int32)
    Qr = _t(tiny["Qr32"][:m], dev)
    Xr = _t(tiny["Xr32"], dev)
    adj = _t(tiny["sub_adj"].astype(np.int32), dev)
    E = _t(ent[:m].astype(np.int32), dev)
    ids, d, cnt = pa.gpu_traverse_ragged(Qr, Xr, adj, E, _t(efs, dev))
    ids, d, cnt = ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy()
    for ef in np.unique(efs):
        sel = np.nonzero(efs == ef)[0]
        e_use = min(8, int(ef))
        a_ids, a_d, a_cnt = pa.gpu_traverse(Qr[sel], Xr, adj, E[sel][:, :e_use].contiguous(), int(ef))
        a_ids, a_d, a_cnt = a_ids.cpu().numpy(), a_d.cpu().numpy(), a_cnt.cpu().numpy()
        assert (ids[sel, :ef] == a_ids).all()
        assert (d[sel, :ef].view(np.uint32) == a_d.view(np.uint32)).all()
        assert (cnt[sel] == a_cnt).all()
        assert (ids[sel, ef:] == -1).all()


def _requests(tiny, n, seed=7):
    rng = np.random.default_rng(seed)
    ks = rng.choice([10, 50, 100], size=n)
    efs = rng.choice([64, 128, 256, 512], size=n)
    return [(i, tiny["Q"][i], int(ks[i]), int(efs[i])) for i in range(n)]


def test_server_result_is_the_same_alone_in_the_mix_and_in_batch_search(dev, tiny, index):
    reqs = _requests(tiny, 120)
    srv = pa.Server(index, hbm_budget=1 << 30, max_batch=64, streams=3, threads=4)
    print("server: 120 mixed requests submitted at once", flush=True)
    for tag, q, k, ef in reqs:
        srv.submit(q, k, ef, tag)
    srv.drain()
    mixed = {r["tag"]: r for r in srv.poll(1000)}
    st = srv.stats()
    assert st["completed"] == 120 and st["bytes_in_flight"] == 0
    assert st["max_batch"] > 1
    print("server: the same requests one at a time", flush=True)
    for tag, q, k, ef in reqs[:40]:
        srv.submit(q, k, ef, tag)
        srv.drain()
        alone = srv.poll(10)
        assert len(alone) == 1
        a = alone[0]
        b = mixed[tag]
        assert (a["ids"] == b["ids"]).all() and (a["dists"].view(np.uint32) == b["dists"].view(np.uint32)).all()
        assert a["t_submit_us"] <= a["t_admit_us"] <= a["t_done_us"]
    srv.close()
    print("server vs batch search at the same (k, ef)", flush=True)
    for tag, q, k, ef in reqs[:30]:
        ef = max(ef, k)  # the server raises ef to k
        ids, d, _, _ = index.search(q[None], k, ef, ef)
        assert (ids[0] == mixed[tag]["ids"]).all()
        assert (d[0].view(np.uint32) == mixed[tag]["dists"].view(np.uint32)).all()


def _batch_bytes(spec, m, ef):
    """Device bytes of a micro-batch of m requests at list size ef (the server's documented
    footprint: each buffer rounded up to 256 bytes)."""
    al = lambda b: (b + 255) // 256 * 256
    e = min(ef, spec.n_pivots // spec.r)
    return (al(4 * m * spec.dim) + al(4 * m * spec.d_r) + al(4 * m) + 2 * al(4 * m * e) + 2 * al(4 * m * ef)
            + al(16 * m) + al(4 * m) + al(4 * (3 * spec.r + 2 + m)))


def test_server_budget_makes_requests_queue(dev, tiny, index):
    s = tiny["spec"]
    # the index first, then two slots that each hold a micro-batch of three requests at
    # ef 512 but not four
    held = index.info()["hbm_bytes"]
    per_slot = _batch_bytes(s, 3, 512)
    assert _batch_bytes(s, 4, 512) > per_slot
    srv = pa.Server(index, hbm_budget=held + 2 * per_slot, max_batch=64, streams=2, threads=2)
    print("server: budget of the index plus two slots of three requests at ef 512, 30 submitted", flush=True)
    for i in range(30):
        srv.submit(tiny["Q"][i], 10, 512, i)
    srv.drain()
    res = {r["tag"]: r for r in srv.poll(100)}
    st = srv.stats()
    srv.close()
    # the server's arenas are released with it
    assert index.info()["hbm_bytes"] == held
    assert len(res) == 30 and st["max_batch"] <= 3 and st["batches"] >= 10
    ids, d, _, _ = index.search(tiny["Q"][:30], 10, 512, 512)
    for i in range(30):
        assert (res[i]["ids"] == ids[i]).all()


def test_server_budget_below_the_index_is_refused(dev, tiny, index):
    held = index.info()["hbm_bytes"]
    with pytest.raises(pa.PilotannError) as e:
        pa.Server(index, hbm_budget=held + 1000, streams=2, threads=1)
    assert e.value.status == -4  # PA_EHBM


def test_server_rejects_bad_requests(dev, tiny, index):
    srv = pa.Server(index, hbm_budget=index.info()["hbm_bytes"] + (64 << 20), max_k=100, threads=1)
    q = tiny["Q"][0]
    with pytest.raises(pa.PilotannError) as e:
        srv.submit(q, 0, 64, 1)
    assert e.value.status == -1
    with pytest.raises(pa.PilotannError) as e:
        srv.submit(q, 101, 128, 1)
    assert e.value.status == -1
    with pytest.raises(pa.PilotannError) as e:
        srv.submit(q, 10, 513, 1)
    assert e.value.status == -1
    bad = q.copy()
    bad[3] = np.nan
    with pytest.raises(pa.PilotannError) as e:
        srv.submit(bad, 10, 64, 1)
    assert e.value.status == -6
    srv.close()


def test_server_on_the_compact_layout_matches_the_full_layout(dev, tiny, index):
    s = tiny["spec"]
    comp = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f32", r=s.r, threads=4,
                                   compact=True))
    comp.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    comp.set_projection(tiny["V32"])
    mask = comp.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
    comp.build_subgraph(mask, tiny["sr"], tiny["sn"])
    comp.build_entries(tiny["pivots"], tiny["init"], 10)
    reqs = _requests(tiny, 60)
    out = []
    for idx in (index, comp):
        srv = pa.Server(idx, hbm_budget=1 << 30, max_batch=32, streams=2, threads=4)
        for tag, q, k, ef in reqs:
            srv.submit(q, k, ef, tag)
        srv.drain()
        out.append({r["tag"]: r for r in srv.poll(1000)})
        srv.close()
    print("server: 60 requests on the full and on the compact layout", flush=True)
    for tag, _, _, _ in reqs:
        a, b = out[0][tag], out[1][tag]
        assert (a["ids"] == b["ids"]).all() and (a["dists"].view(np.uint32) == b["dists"].view(np.uint32)).all()
    comp.close()
