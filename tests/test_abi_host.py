"""The C-ABI library: it loads, exports every declared symbol, and its host-only
entry points (sampling, subgraph validation, clustering, eigensolver, stages
2-3) agree with the oracle.  No GPU needed."""

import os
import re

import numpy as np
import pytest

import oracle
import paper_2503_21206_amd as pa
from synth.data import gmm_points, make_rng
from tests.parity import TIE, DistTally

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return pa.lib()


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:pa_status|const char\*|int32_t|int64_t)\s+(pa_[a-z0-9_]+)\s*\(", text, re.M))
    return names


def test_every_declared_symbol_is_exported(L):
    decl = _declared()
    assert len(decl) >= 25
    for name in decl:
        assert hasattr(L, name), name
    assert decl == set(pa.symbols())
    assert pa.abi_version() == 12


def _csr(rows):
    rowptr = [0]
    flat = []
    for r in rows:
        flat.extend(r)
        rowptr.append(len(flat))
    return np.asarray(rowptr, dtype=np.int64), np.asarray(flat, dtype=np.int32)


def test_sample_nodes_matches_oracle(golden_dir):
    import json
    g = json.load(open(os.path.join(golden_dir, "sampling_examples.json")))
    rowptr, nbrs = _csr(g["rows"])
    for c in g["cases"]:
        m = pa.sample_nodes(rowptr, nbrs, g["order"], c["n_target"], c["mode"])
        assert np.nonzero(m)[0].tolist() == c["members"]
    from synth.graph import build_graph, padded_to_csr
    X = gmm_points(101, 800, 8, 4)
    rp, nb = padded_to_csr(build_graph(X, 10, device="cpu"))
    order = make_rng(7, 0).permutation(800)
    for mode in ("uniform", "seed_expand"):
        for t in (0, 1, 199, 800):
            a = pa.sample_nodes(rp, nb, order, t, mode)
            b = oracle.sample_nodes(rp, nb, order, t, mode)
            assert (a == b).all()


def test_sample_nodes_rejects_bad_input():
    rowptr, nbrs = _csr([[1], [0]])
    with pytest.raises(pa.PilotannError) as e:
        pa.sample_nodes(rowptr, nbrs, [0, 1], 3)
    assert e.value.status == -1
    with pytest.raises(pa.PilotannError):
        pa.sample_nodes(rowptr, nbrs, [0, 0], 2, "uniform")  # not a permutation


def test_check_subgraph_accepts_valid_and_names_violations():
    from synth.graph import build_graph, build_subgraph_csr, padded_to_csr
    X = gmm_points(102, 500, 8, 3)
    rp, nb = padded_to_csr(build_graph(X, 10, device="cpu"))
    order = make_rng(8, 0).permutation(500)
    mask = oracle.sample_nodes(rp, nb, order, 125, "seed_expand")
    sr, sn = build_subgraph_csr(X, mask, 10, device="cpu")
    pa.check_subgraph(sr, sn, mask, 10)
    u = int(np.nonzero(mask)[0][0])
    outside = int(np.nonzero(~mask)[0][0])
    bad = sn.copy()
    bad[sr[u]] = outside
    with pytest.raises(pa.PilotannError, match="unsampled"):
        pa.check_subgraph(sr, bad, mask, 10)
    bad = sn.copy()
    bad[sr[u]] = u
    with pytest.raises(pa.PilotannError, match="self loop"):
        pa.check_subgraph(sr, bad, mask, 10)
    with pytest.raises(pa.PilotannError, match="degree"):
        pa.check_subgraph(sr, sn, mask, 1)


def test_build_entries_matches_oracle_buckets():
    P = gmm_points(103, 1024, 16, 20)
    init = make_rng(9, 1).choice(1024, 32, replace=False)
    b, c = pa.build_entries(P, 32, init, 10)
    ob, oc = oracle.balanced_kmeans(P, 32, init, 10)
    assert (b == ob).all()
    # both take each final centroid as the fp64 mean of its bucket's rows in position order
    assert (c.view(np.uint32) == oc.astype(np.float32).view(np.uint32)).all()


def test_build_entries_hand_example(golden_dir):
    import json
    g = json.load(open(os.path.join(golden_dir, "entries_example.json")))
    b, c = pa.build_entries(np.array(g["pivots"], dtype=np.float32), g["r"], g["init"], g["iters"])
    assert b.tolist() == g["buckets"]
    np.testing.assert_allclose(c, g["centroids"], atol=1e-6)


def test_eigh_matches_oracle_and_hand_example(golden_dir):
    import json
    g = json.load(open(os.path.join(golden_dir, "projection_axes.json")))
    M, _ = oracle.projection.second_moment(np.array(g["points"]), True)
    w, V = pa.eigh_f64(M)
    np.testing.assert_allclose(w, g["eigenvalues"], atol=1e-12)
    np.testing.assert_allclose(V[:, :2], g["V"], atol=1e-12)
    X = gmm_points(104, 2000, 24, 30) + 1.0
    M, _ = oracle.projection.second_moment(X, True)
    w, V = pa.eigh_f64(M)
    Vo, wo, _ = oracle.fit_projection(X, 24)
    np.testing.assert_allclose(w, wo, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(24), atol=1e-12)
    # eigenvectors agree up to the shared sign rule where eigenvalues are separated
    gaps = np.minimum(np.abs(np.diff(wo, prepend=np.inf)), np.abs(np.diff(wo, append=-np.inf)))
    for j in range(24):
        if gaps[j] > 1e-6 * wo[0]:
            np.testing.assert_allclose(V[:, j], Vo[:, j], atol=1e-8)


@pytest.fixture(scope="module")
def tiny():
    from synth import SPECS, base_vectors, query_vectors
    from synth.graph import build_graph, build_subgraph_csr, padded_to_csr
    s = SPECS["tiny"]
    X = base_vectors(s)
    Q = query_vectors(s, 60)
    adj = build_graph(X, 32, device="cpu")
    rp, nb = padded_to_csr(adj)
    order = make_rng(s.seed + 3, 0).permutation(s.n)
    mask = oracle.sample_nodes(rp, nb, order, round(s.rho * s.n), s.sample_mode)
    sr, sn = build_subgraph_csr(X, mask, 32, device="cpu")
    return dict(X=X, Q=Q, rp=rp, nb=nb, adj=adj, mask=mask, sr=sr, sn=sn,
                sub_adj=oracle.padded_from_csr(sr, sn, 32))


def test_cpu_stages_match_oracle(tiny):
    X, Q = tiny["X"], tiny["Q"]
    rng = make_rng(11, 0)
    S = np.nonzero(tiny["mask"])[0]
    beams = np.stack([rng.choice(S, 48, replace=False) for _ in range(Q.shape[0])]).astype(np.int32)
    beams[:, -3:] = -1  # padding is skipped
    for steps, ef_cpu, k in ((2, 32, 10), (0, 16, 10), (-1, 24, 30)):
        ids, d, cnt = pa.cpu_stages(X, tiny["sub_adj"], tiny["adj"], Q, beams, ef_cpu, k, steps, threads=4)
        bad = 0
        tally = DistTally()
        for i in range(Q.shape[0]):
            m2 = np.inf
            if steps >= 0:
                r = oracle.refine(Q[i], X, tiny["sr"], tiny["sn"], beams[i], ef_cpu, steps=steps)
                c_ids, c_d, vis, n2, m2 = r["ids"], r["dists"], r["visited"], r["n_dist"], r["margin"]
            else:
                b = beams[i][beams[i] >= 0]
                c_d = oracle.as_f32(oracle.delta_many(Q[i], X[b]))
                c_ids, vis, n2 = b, set(b.tolist()), b.size
            oi, od, f = oracle.final_traversal(Q[i], X, tiny["rp"], tiny["nb"], c_ids, c_d, vis, ef_cpu, k)
            if not (ids[i] == oi).all():
                assert min(m2, f["margin"]) <= TIE, (i, m2, f["margin"])
                bad += 1
                continue
            tally.check(d[i], od, i)
            if min(m2, f["margin"]) > TIE:
                assert cnt[i, 0] == n2 and cnt[i, 1] == f["n_dist"] and cnt[i, 2] == f["n_exp"]
        tally.done()
        assert bad <= max(1, Q.shape[0] // 1000), bad


def test_cpu_search_is_plain_greedy_search(tiny):
    X, Q = tiny["X"], tiny["Q"]
    entries = np.tile(np.array([0, 4000, 9999], dtype=np.int32), (Q.shape[0], 1))
    ids, d, cnt = pa.cpu_search(X, tiny["adj"], Q, entries, 40, 10, threads=3)
    tally = DistTally()
    bad = 0
    for i in range(Q.shape[0]):
        r = oracle.greedy_search(Q[i], X, tiny["rp"], tiny["nb"], 40, entries[i])
        if (ids[i] == r["ids"][:10]).all():
            tally.check(d[i], r["dists"][:10], i)
            if r["margin"] > TIE:
                assert cnt[i, 1] == r["n_dist"] and cnt[i, 2] == r["n_exp"]
        else:
            assert r["margin"] <= TIE
            bad += 1
    tally.done()
    assert bad <= max(1, Q.shape[0] // 1000), bad


def test_cpu_stages_hand_example(golden_dir):
    import json
    g = json.load(open(os.path.join(golden_dir, "stages_example.json")))
    X = np.array(g["points"], dtype=np.float32)
    sub = oracle.padded_from_csr(*_csr(g["sub_rows"]), 2)
    full = oracle.padded_from_csr(*_csr(g["full_rows"]), 2)
    ids, d, cnt = pa.cpu_stages(X, sub, full, np.array([g["query"]], dtype=np.float32),
                                np.array([g["beam"]], dtype=np.int32), g["ef_cpu"], g["k"], g["steps"], threads=1)
    assert ids[0].tolist() == g["final_ids"]
    np.testing.assert_allclose(d[0], g["final_dists"], rtol=2.0 ** -23)  # fp32 rounding of the worked values
    assert cnt[0].tolist() == [g["refine_n_dist"], g["final_n_dist"], g["final_n_exp"], 0]


def test_empty_batches_and_argument_errors(tiny):
    X = tiny["X"]
    ids, d, cnt = pa.cpu_stages(X, tiny["sub_adj"], tiny["adj"], np.zeros((0, 96), np.float32),
                                np.zeros((0, 4), np.int32), 8, 5)
    assert ids.shape == (0, 5)
    with pytest.raises(pa.PilotannError) as e:
        pa.cpu_stages(X, tiny["sub_adj"], tiny["adj"], tiny["Q"][:2], np.zeros((2, 4), np.int32), 0, 5)
    assert e.value.status == -1
    with pytest.raises(pa.PilotannError):
        pa.build_entries(np.zeros((10, 4), np.float32), 3, [0, 1, 2])  # 10 % 3 != 0
    with pytest.raises(pa.PilotannError) as e:
        pa.build_entries(np.full((4, 2), np.nan, np.float32), 2, [0, 1])
    assert e.value.status == -6


def test_fp8_row_encoding_matches_torch_e4m3fn():
    import torch
    rng = np.random.default_rng(5)
    X = (rng.standard_normal((300, 64)) * rng.uniform(1e-6, 10, size=(300, 1))).astype(np.float32)
    X[3] = 0.0
    X[4, :5] = [448e-3, -1e-9, 2.5e-7, 3.0, -3.0]
    codes, scales = pa.quantize_fp8_rows(X)
    amax = np.abs(X).max(1)
    np.testing.assert_array_equal(scales, np.where(amax > 0, amax / np.float32(448.0), 1.0).astype(np.float32))
    ref = torch.tensor(X / scales[:, None]).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(codes, ref)
    # the largest magnitude of every non-zero row encodes to +-448
    nz = amax > 0
    assert (np.abs(torch.tensor(codes).view(torch.float8_e4m3fn).float().numpy()).max(1)[nz] == 448).all()


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library every call raises: the binding has no fallback of its own."""
    import subprocess
    import sys
    code = (
        "import numpy as np, paper_2503_21206_amd as pa\n"
        f"pa.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
        "pa._lib = None\n"
        "for call in (lambda: pa.abi_version(),\n"
        "             lambda: pa.sample_nodes(np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(1, np.int64), 1),\n"
        "             lambda: pa.cpu_search(np.zeros((4, 8), np.float32), np.full((4, 2), -1, np.int32),\n"
        "                                   np.zeros((1, 8), np.float32), np.zeros((1, 1), np.int32), 4, 1)):\n"
        "    try:\n"
        "        call()\n"
        "    except RuntimeError as e:\n"
        "        assert 'missing' in str(e), e\n"
        "    else:\n"
        "        raise SystemExit('a call returned without the library')\n"
        "print('ok')\n"
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_hbm_model_hand_sums_and_planner_choice():
    """The device-byte model of the memory-bounded mode, worked by hand on a small shape,
    and the planner's rule (largest ratio that fits, then the largest width)."""
    shape = pa.memory_shape(N=1000, dim=32, R_sub=8, n_pivots=64, r=4, xr_dtype="f16")
    # rho 0.25 -> 250 sampled rows, d_r 16, 2-byte rows: V 4*32*16 = 2048, X_r 250*16*2 = 8000,
    # adjacency 4*250*8 = 8000, id map 4*250 = 1000, pivots 4*64*(16+2) = 4608, centroids
    # 4*4*16 = 256
    assert pa.hbm_bytes(shape, 0.25, 16) == 2048 + 8000 + 8000 + 1000 + 4608 + 256
    full = pa.memory_shape(N=1000, dim=32, R_sub=8, n_pivots=64, r=4, xr_dtype="f16", compact=False)
    assert pa.hbm_bytes(full, 0.25, 16) == 2048 + 32000 + 32000 + 4608 + 256  # every row, no id map
    fp8 = pa.memory_shape(N=1000, dim=32, R_sub=8, n_pivots=64, r=4, xr_dtype="f16", pivot_dtype="fp8")
    assert pa.hbm_bytes(fp8, 0.25, 16) == 23912 + 64 * (16 + 4)
    # 10 queries, ef 8, E = min(8, 64/4): 10*(4*32 + 4*16 + 4 + 8*8 + 8*8 + 16) + 4*(3*4 + 2 + 10)
    q = pa.memory_shape(N=1000, dim=32, R_sub=8, n_pivots=64, r=4, xr_dtype="f16", queries=10, ef_gpu=8)
    assert pa.hbm_bytes(q, 0.25, 16) == 23912 + 3400 + 96
    qd = pa.memory_shape(N=1000, dim=32, R_sub=8, n_pivots=64, r=4, xr_dtype="f16", queries=10, ef_gpu=8,
                         q_on_device=True)
    assert pa.hbm_bytes(qd, 0.25, 16) == 23912 + 3400 + 96 - 10 * 4 * 32
    rhos, widths = [0.1, 0.25, 0.5], [16, 32]
    cost = {(r_, d_): pa.hbm_bytes(shape, r_, d_) for r_ in rhos for d_ in widths}
    assert cost[(0.5, 16)] < cost[(0.5, 32)] and cost[(0.25, 32)] < cost[(0.5, 16)]
    # a budget between (0.25, 32) and (0.5, 16): the largest ratio that fits is 0.25, at its widest
    assert pa.plan_memory(shape, cost[(0.5, 16)] - 1, rhos, widths) == (0.25, 32, cost[(0.25, 32)])
    assert pa.plan_memory(shape, cost[(0.5, 16)], rhos, widths) == (0.5, 16, cost[(0.5, 16)])
    assert pa.plan_memory(shape, 10 ** 12, rhos, widths) == (0.5, 32, cost[(0.5, 32)])
    with pytest.raises(pa.PilotannError) as e:
        pa.plan_memory(shape, cost[(0.1, 16)] - 1, rhos, widths)
    assert e.value.status == -4  # PA_EHBM: nothing fits
    wide = pa.memory_shape(N=1000, dim=512, R_sub=8, n_pivots=64, r=4)
    with pytest.raises(pa.PilotannError):
        pa.hbm_bytes(wide, 0.25, 272)  # above the largest reduced width the library builds
    for bad_rho, bad_w in ((0.0, 16), (1.5, 16), (0.25, 24), (0.25, 48)):
        with pytest.raises(pa.PilotannError) as e:
            pa.plan_memory(shape, 10 ** 12, [bad_rho], [bad_w])
        assert e.value.status == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_bench_roofline_counts_the_algorithmic_bytes():
    """The beam kernel's algorithmic bytes per query: 4*d_r (query) + 4*E (entries) + 8*ef
    (list out) + 4*R per expansion (adjacency row) + s*d_r per distance (reduced row)."""
    import types
    import bench
    spec = types.SimpleNamespace(name="hand", queries=10, d_r=64, degree=32, n=1_000_000, rho=0.25)
    agg = {"n_exp1": 650, "n_dist1": 8670, "beam_launches": 2, "beam_ms": 1.0}
    r = bench.roofline(spec, agg, 2, 64, 64, 4, "f32")
    # the traversal's tables: 250,000 sampled rows of 256 + 128 bytes fit the 256 MB cache
    assert r["working_set_bytes"] == 250_000 * 384 and r["served_from"] == "infinity_cache"
    big = types.SimpleNamespace(name="hand", queries=10, d_r=48, degree=32, n=32_000_000, rho=0.25)
    assert bench.roofline(big, agg, 2, 64, 64, 2, "f16")["served_from"] == "hbm"
    # 20 queries * (256 + 256 + 512) + 650 * 128 + 8670 * 256 = 20480 + 83200 + 2219520 bytes
    # over two launches of 0.5 ms each
    assert r["bytes_per_launch"] == (20480 + 83200 + 2219520) // 2
    assert abs(r["achieved"] - 2323200 / 2 / 0.5e-3 / 1e9) < 0.05
    assert r["peak"] == 8000.0 and r["traffic"] is None  # no profile for this workload
    # with |visited| counted separately (766 per query instead of the kernel's 867 evaluations,
    # which include re-scores after forget events) the method's bytes use |visited|
    r = bench.roofline(spec, agg, 2, 64, 64, 4, "f32", visited=766.0)
    method = 20480 + 83200 + 20 * 766 * 256
    assert r["bytes_per_launch"] == method // 2 and r["kernel_bytes_per_launch"] == (20480 + 83200 + 2219520) // 2
    assert abs(r["frac"] - method / 2 / 0.5e-3 / 1e9 / 8000.0) < 1e-4
