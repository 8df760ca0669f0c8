"""Index checkpoint: save, load into a fresh index, identical search results; corrupt
files and mismatched parameters are refused without touching the index."""

import numpy as np
import pytest

import paper_2503_21206_amd as pa
from synth import node_order
from tests.workload import build_tiny

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pa.device_init(0)
    return build_tiny(device="cpu")


def _index(tiny, **over):
    s = tiny["spec"]
    cfg = dict(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f16", r=s.r, threads=4)
    cfg.update(over)
    idx = pa.Index(pa.IndexConfig(**cfg))
    idx.set_data(tiny["X"], tiny["rp"], tiny["nb"])
    return idx


def test_save_load_round_trip(tiny, tmp_path):
    print("checkpoint: build, save, load into a fresh index, search both", flush=True)
    s = tiny["spec"]
    a = _index(tiny)
    a.set_projection(tiny["V32"])
    mask = a.sample_nodes(node_order(s.n, s.seed), round(s.rho * s.n), s.sample_mode)
    a.build_subgraph(mask, tiny["sr"], tiny["sn"])
    a.build_entries(tiny["pivots"], tiny["init"], 10)
    Q = tiny["Q"][:300]
    ids_a, d_a, cnt_a, _ = a.search(Q, 10, 64, 64, with_counters=True)
    path = str(tmp_path / "tiny.pidx")
    a.save(path)
    b = _index(tiny)
    assert b.info()["built"] == 1
    b.load(path)
    info = b.info()
    assert info["built"] == 15 and info["n_pivots"] == s.n_pivots and info["R_sub"] == a.info()["R_sub"]
    ids_b, d_b, cnt_b, _ = b.search(Q, 10, 64, 64, with_counters=True)
    assert (ids_a == ids_b).all() and (d_a.view(np.uint32) == d_b.view(np.uint32)).all() and (cnt_a == cnt_b).all()
    Va, ba, ca = a.state()
    Vb, bb, cb = b.state()
    assert (Va == Vb).all() and (ba == bb).all() and (ca == cb).all()

    print("checkpoint: corrupt byte, truncation, wrong parameters, wrong N", flush=True)
    raw = bytearray(open(path, "rb").read())
    bad = bytearray(raw)
    bad[len(bad) // 2] ^= 0x40  # one flipped bit inside a section
    open(path + ".bad", "wb").write(bytes(bad))
    open(path + ".short", "wb").write(bytes(raw[: len(raw) - 100]))
    for p in (path + ".bad", path + ".short", str(tmp_path / "missing.pidx")):
        with pytest.raises(pa.PilotannError) as e:
            b.load(p)
        assert e.value.status == -9
    # a failed load leaves the loaded index as it was
    ids_c, d_c, _, _ = b.search(Q, 10, 64, 64)
    assert (ids_c == ids_a).all()
    c = _index(tiny, xr_dtype="f32")
    with pytest.raises(pa.PilotannError) as e:
        c.load(path)
    assert e.value.status == -1 and c.info()["built"] == 1
    small = pa.Index(pa.IndexConfig(dim=s.dim, d_r=s.d_r, metric=s.metric, xr_dtype="f16", r=s.r, threads=2))
    rp = tiny["rp"][:1001].copy()
    small.set_data(tiny["X"][:1000], rp, np.where(tiny["nb"][: rp[-1]] < 1000, tiny["nb"][: rp[-1]], 0))
    with pytest.raises(pa.PilotannError) as e:
        small.load(path)
    assert e.value.status == -1
    with pytest.raises(pa.PilotannError) as e:
        _index(tiny).save(str(tmp_path / "unbuilt.pidx"))
    assert e.value.status == -2
    for x in (a, b, c, small):
        x.close()
