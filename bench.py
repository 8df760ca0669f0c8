#!/usr/bin/env python3
"""Benchmark: QPS at recall@10 = 0.95 of the full PilotANN search on one MI355X.

Workload (default ``gmm1m``): N = 1,000,000 base vectors, d = 128, fp32, a
1,024-component Gaussian mixture; 10,000 queries; L2; k = 10; graph degree 32;
projection to 64 dims; 25% subgraph (seed + 1-hop expansion); 4,096 pivots in 32
buckets.  Two forms are measured on the same GPU: reduced vectors stored in
fp32 and in fp16 (fp32 arithmetic), both followed by fp32 refinement and final
traversal on the host.  For each form the smallest ef of the sweep reaching
recall@10 >= 0.95 is found first (untimed), then ``--warmup`` untimed searches and
three runs of ``--steps`` timed searches of all queries at that ef; ``value`` is the
median run.  A step starts from the queries in host memory: their upload to the GPU
is inside it.  One JSON line goes to stdout; progress goes to stderr.

Roofline: the stage-1 traversal kernel is the dominant GPU kernel.  Its
algorithmic bytes per query are 4*d_r (query) + 4*E (entries) + 4*R per
expansion (adjacency row) + s*d_r per visited node (gathered reduced row, s =
bytes per element; |visited| counted in an extra untimed search whose visited
cache never forgets) + 8*ef (list out); the kernel's own bytes (its distance
evaluations, re-scores after cache forgets included) are reported beside them.
The launch duration comes from HIP events recorded around every launch on the
library's stream during the timed steps.  Peak = 8 TB/s HBM.  ``traffic`` is the
HBM traffic per launch that rocprofv3's FETCH_SIZE and WRITE_SIZE counters
measured for the same kernel and configuration, each scaled by what the counter
reads for a copy of known size; it is read from the committed counter summary
and reported only while the kernel's sources still hash to the value recorded
there (null otherwise).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20  # MI355X's last-level cache in front of HBM
PROFILES = os.path.join(ROOT, "profiles")
BEAM_SOURCES = ("k_beam.hip", "ffloat.hpp", "common.hpp")


def beam_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in BEAM_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_21206_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, form, ef_gpu):
    """Counter-measured HBM bytes per beam launch, if the summary for this workload and form
    (profiles/beam_kernel_<workload>_<form>_traffic.txt) matches this kernel and run."""
    try:
        with open(os.path.join(PROFILES, f"beam_kernel_{workload}_{form}_traffic.txt")) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if (kv.get("source_hash") != beam_source_hash() or kv.get("workload") != workload
            or kv.get("form") != form or kv.get("ef_gpu") != str(ef_gpu)):
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def large(spec):
    """Workloads whose exact kNN graph is out of reach (the IVF-restricted builder is used)."""
    return spec.n >= 4_000_000


def check_ground_truth(X, Q, gt, spec, device, n=64):
    """Recomputes the first n queries' top k one query at a time (fp64 distances over every
    row, ties by id) and stops the run if any differs from the batched ground truth."""
    import torch
    x = torch.as_tensor(X).to(device)
    bad = 0
    for i in range(min(n, Q.shape[0])):
        q = torch.as_tensor(Q[i]).to(device).double()
        d = torch.empty(x.shape[0], dtype=torch.float64, device=device)
        for a in range(0, x.shape[0], 1 << 22):
            xa = x[a:a + (1 << 22)].double()
            d[a:a + (1 << 22)] = ((xa - q) ** 2).sum(1) if spec.metric == "l2" else -(xa @ q)
        top = torch.topk(d, spec.k + 16, largest=False).indices
        dd = d[top]
        order = sorted(range(top.shape[0]), key=lambda j: (float(dd[j]), int(top[j])))
        ref = [int(top[j]) for j in order[:spec.k]]
        bad += int(ref != [int(v) for v in gt[i][:spec.k]])
    log(f"ground truth re-derived for {min(n, Q.shape[0])} queries one at a time: {bad} differ")
    if bad:
        raise RuntimeError(f"batched ground truth differs from the per-query recomputation on {bad} queries")


def build_fixture(spec, device, cache=None, nprobe=64):
    """Base set, queries, full graph and ground truth.  The graph of a large workload comes
    from the IVF-restricted builder; ``cache`` (a directory) keeps the graph, the ground
    truth and the subgraph between runs (the vectors are regenerated from their seeds)."""
    from synth import base_vectors, query_vectors, node_order, pivot_choice, kmeans_init_choice
    from synth.graph import build_graph, build_graph_projected, build_subgraph_csr, padded_to_csr
    from synth.ivf import build_graph_ivf, build_subgraph_csr_ivf
    from synth.knn import exact_knn
    wide = spec.dim >= 512  # graph from the 128 leading principal components

    def graph_of(Xa):
        if wide:
            inner = (lambda Y, R: build_graph_ivf(Y, R, nprobe=nprobe, seed=spec.seed, device=device, log=log)) \
                if large(spec) else None
            return build_graph_projected(Xa, spec.degree, 128, device=device, builder=inner)
        if large(spec):
            return build_graph_ivf(Xa, spec.degree, nprobe=nprobe, seed=spec.seed, device=device, log=log)
        return build_graph(Xa, spec.degree, device=device)
    t = time.time()
    X = base_vectors(spec)
    Q = query_vectors(spec)
    log(f"data {X.shape} + {Q.shape} in {time.time() - t:.1f}s")
    tag = f"{spec.name}_n{spec.n}_q{spec.queries}_R{spec.degree}_p{nprobe}"
    path = (lambda what: os.path.join(cache, f"{tag}_{what}.npy")) if cache else None
    if cache and os.path.exists(path("adj")) and os.path.exists(path("gt")):
        adj, gt = np.load(path("adj")), np.load(path("gt"))
        log(f"graph and ground truth from {cache}")
    else:
        t = time.time()
        adj = graph_of(X)
        log(f"full graph: mean degree {(adj >= 0).sum(1).mean():.2f} in {time.time() - t:.1f}s")
        t = time.time()
        # candidates from an fp32 GEMM, re-ranked in fp64; at 10^7 rows of 768-d unit vectors
        # the nearest scores lie closer together than the fp32 products' rounding, so those
        # workloads take their candidates from fp64 scores (checked below on 64 queries)
        gt, _ = exact_knn(X, Q, spec.k, spec.metric, device=device,
                          budget_bytes=(32 << 30) if large(spec) else None,
                          fp64_scores=large(spec) and wide)
        log(f"ground truth in {time.time() - t:.1f}s")
        if large(spec):
            check_ground_truth(X, Q, gt, spec, device)
        if cache:
            os.makedirs(cache, exist_ok=True)
            np.save(path("adj"), adj)
            np.save(path("gt"), gt)
    rp, nb = padded_to_csr(adj)
    if wide:
        def sub_builder(Xa, mask, R, device=None):
            sel = np.nonzero(mask)[0]
            local = graph_of(Xa[sel])
            full = np.full((Xa.shape[0], R), -1, dtype=np.int32)
            full[sel] = np.where(local >= 0, sel[np.clip(local, 0, None)], -1)
            return padded_to_csr(full)
    elif large(spec):
        def sub_builder(Xa, mask, R, device=None):
            return build_subgraph_csr_ivf(Xa, mask, R, nprobe=nprobe, seed=spec.seed + 3, device=device, log=log)
    else:
        sub_builder = build_subgraph_csr
    if cache:
        def cached_sub(Xa, mask, R, device=None, _b=sub_builder):
            f = os.path.join(cache, f"{tag}_sub_{int(mask.sum())}.npz")
            if os.path.exists(f):
                with np.load(f) as d:
                    if d["mask"].shape == mask.shape and (d["mask"] == mask).all():
                        log(f"subgraph from {cache}")
                        return d["sr"], d["sn"]
            sr, sn = _b(Xa, mask, R, device=device)
            np.savez(f + ".tmp.npz", mask=mask, sr=sr, sn=sn)
            os.replace(f + ".tmp.npz", f)
            return sr, sn
        builder = cached_sub
    else:
        builder = sub_builder
    return dict(X=X, Q=Q, adj=adj, rp=rp, nb=nb, gt=gt, order=node_order(spec.n, spec.seed),
                pivot_choice=pivot_choice, kmeans_init_choice=kmeans_init_choice,
                build_subgraph_csr=builder, device=device,
                graph=("candidates and pruning on the 128 leading principal components, rows ordered by the "
                       "full distance" if wide else "full vectors")
                + (f", IVF-restricted candidates ({nprobe} lists of ~1,024 rows probed)" if large(spec)
                   else ", exact candidates"))


def build_index(spec, fx, xr_dtype, shared, compact=False):
    import paper_2503_21206_amd as pa
    t = time.time()
    idx = pa.Index(pa.IndexConfig(dim=spec.dim, d_r=spec.d_r, metric=spec.metric, xr_dtype=xr_dtype, r=spec.r,
                                  compact=compact, pivot_dtype=spec.pivot_dtype))
    idx.set_data(fx["X"], fx["rp"], fx["nb"])
    if "V" not in shared:
        idx.fit_projection()
        shared["V"] = idx.projection()
    else:
        idx.set_projection(shared["V"])
    n_target = round(spec.rho * spec.n)
    mask = idx.sample_nodes(fx["order"], n_target, spec.sample_mode)
    if "sub" not in shared:
        ts = time.time()
        sr, sn = fx["build_subgraph_csr"](fx["X"], mask, spec.degree, device=fx["device"])
        shared["sub"] = (mask, sr, sn)
        log(f"subgraph reconnected over {int(mask.sum())} nodes in {time.time() - ts:.1f}s")
    mask, sr, sn = shared["sub"]
    idx.build_subgraph(mask, sr, sn)
    if "pivots" not in shared:
        S = np.nonzero(mask)[0]
        deg = sr[1:] - sr[:-1]
        shared["pivots"] = fx["pivot_choice"](S[deg[S] > 0], spec.n_pivots, spec.seed)
        shared["init"] = fx["kmeans_init_choice"](spec.n_pivots, spec.r, spec.seed)
    idx.build_entries(shared["pivots"], shared["init"], 10)
    log(f"index ({xr_dtype}) built in {time.time() - t:.1f}s")
    return idx


def recall(ids, gt, k):
    from synth.knn import recall_at_k
    return recall_at_k(ids, gt, k)


def sweep(idx, spec, fx, target, efs):
    """Find the fastest (ef_gpu, ef_cpu) pair reaching the target recall.

    ef_cpu walks up the workload's sweep; for each value ef_gpu takes ef_cpu and 2*ef_cpu
    (the GPU list is cheap).  The walk stops at the first ef_cpu that reaches the target,
    since larger ef_cpu only adds host work."""
    curve = []
    hits = []
    for ef_cpu in efs:
        for ef_gpu in sorted({ef_cpu, min(512, 2 * ef_cpu)}):
            idx.search(fx["Q"][:1000], spec.k, ef_gpu, ef_cpu)  # warm caches for this pair
            ids, _, _, st = idx.search(fx["Q"], spec.k, ef_gpu, ef_cpu)
            rec = recall(ids, fx["gt"], spec.k)
            qps = fx["Q"].shape[0] / (st["wall_ms"] / 1e3)
            curve.append({"ef_gpu": ef_gpu, "ef_cpu": ef_cpu, "recall": round(rec, 5), "qps": round(qps, 1)})
            log(f"  ef_gpu={ef_gpu:4d} ef_cpu={ef_cpu:4d} recall@{spec.k}={rec:.4f} qps={qps:,.0f}")
            if rec >= target:
                hits.append((qps, ef_gpu, ef_cpu))
        if hits:
            break
    if not hits:
        return None, curve
    best = max(hits)
    return (best[1], best[2]), curve


def timed(idx, spec, fx, ef, steps, warmup, resident=False, **kw):
    """W untimed and K timed searches of every query at (ef_gpu, ef_cpu).  Each timed step
    is the whole search from host queries: the upload of the queries to the GPU (pinned
    staging, host-to-device copy), projection, routing, FES, stage 1, the hand-off and the
    host stages.  resident=True passes a device copy of the queries made before the timed
    region instead (no upload inside it), for comparison."""
    import torch
    ef_gpu, ef_cpu = ef
    Qd = torch.as_tensor(fx["Q"]).to("cuda").contiguous() if resident else None
    for _ in range(warmup):
        idx.search(fx["Q"], spec.k, ef_gpu, ef_cpu, Q_dev=Qd, **kw)
    torch.cuda.synchronize()
    agg = None
    t0 = time.perf_counter()
    for _ in range(steps):
        ids, _, _, st = idx.search(fx["Q"], spec.k, ef_gpu, ef_cpu, Q_dev=Qd, **kw)
        if agg is None:
            agg = {k: 0.0 for k in st}
        for k, v in st.items():
            agg[k] += v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = recall(ids, fx["gt"], spec.k)
    return dt, agg, rec


def timed_median(idx, spec, fx, ef, steps, warmup, runs=3, **kw):
    """`runs` timed runs of `steps` searches each (after one warm-up phase); returns the run
    with the median time (dt, agg, recall) and every run's queries per second."""
    res = []
    for i in range(runs):
        res.append(timed(idx, spec, fx, ef, steps, warmup if i == 0 else 0, **kw))
    order = sorted(range(runs), key=lambda i: res[i][0])
    med = res[order[runs // 2]]
    return med, [round(spec.queries * steps / r[0], 1) for r in res]


def visited_per_query(idx, spec, fx, ef, **kw):
    """|visited| of stage 1 per query (the method's distance evaluations, Algorithm 1 with
    an exact visited set): counted in one untimed search with the largest visited cache, in
    which no query forgets a node (checked), so the kernel's count is |visited|.  None if a
    forget event still happened."""
    _, _, cnt, _ = idx.search(fx["Q"], spec.k, ef[0], ef[1], cache_log2=13, with_counters=True, **kw)
    if (cnt[:, 2] != 0).any():
        return None
    return float(cnt[:, 1].mean())


def cpu_only(idx, spec, fx, target, steps):
    """The library with the GPU stage switched off: plain Algorithm 1 on the full graph on
    the host cores from the FES entries (graceful degradation, section 4.1), the analogue
    of the CPU graph search the paper compares against.  Smallest swept ef reaching the
    target recall, then `steps` timed searches."""
    import torch
    curve, chosen = [], None
    for ef in sorted(set(spec.ef) | {24, 40, 80, 160}):
        ids, _, _, st = idx.search(fx["Q"], spec.k, ef, ef, stage_mask=2)
        rec = recall(ids, fx["gt"], spec.k)
        curve.append({"ef": ef, "recall": round(rec, 5), "qps": round(fx["Q"].shape[0] / (st["wall_ms"] / 1e3), 1)})
        log(f"  cpu-only ef={ef:4d} recall@{spec.k}={rec:.4f}")
        if rec >= target:
            chosen = ef
            break
    if chosen is None:
        return {"curve": curve, "value": None}
    t0 = time.perf_counter()
    agg = 0
    for _ in range(steps):
        ids, _, cnt, st = idx.search(fx["Q"], spec.k, chosen, chosen, stage_mask=2, with_counters=True)
        agg += int(cnt[:, 4].sum())
    dt = time.perf_counter() - t0
    return {"value": round(spec.queries * steps / dt, 1), "unit": "queries/s", "ef": chosen,
            "recall": round(recall(ids, fx["gt"], spec.k), 5), "mean_n_dist": round(agg / (spec.queries * steps), 1),
            "curve": curve}


def ablation(idx, spec, fx, ef, steps=2):
    """The paper's ablation (Table 5): components removed one after another, at the chosen
    (ef_gpu, ef_cpu), all queries in sub-batches of 2,048: the full pipeline (the host
    stages of a sub-batch overlap the GPU stage of the next ones); without pipelining (the
    host waits for the GPU stage of every sub-batch); then also without fast entry
    selection (every query starts from the same predefined pivots); then also without the
    residual refinement (stage 2); then also without GPU piloting (Algorithm 1 on the full
    graph on the host from the predefined entries).  Each row reports QPS, recall and the
    host's full-distance evaluations per query; two single removals are added for
    reference."""
    rows = [("full", {"batch": 2048}),
            ("-pipelining", {"batch": 2048, "serial": True}),
            ("-pipelining -fes", {"batch": 2048, "serial": True, "fixed_entries": True}),
            ("-pipelining -fes -refinement", {"batch": 2048, "serial": True, "fixed_entries": True,
                                              "stage_mask": 1}),
            ("-pipelining -fes -refinement -gpu_piloting", {"batch": 2048, "serial": True, "fixed_entries": True,
                                                            "stage_mask": 2}),
            ("only -fes", {"batch": 2048, "fixed_entries": True}),
            ("only -refinement", {"batch": 2048, "stage_mask": 1})]
    out = {"what": "Table 5 rows, cumulative; ef_gpu/ef_cpu fixed at the timed pair; sub-batches of 2,048",
           "ef_gpu": ef[0], "ef_cpu": ef[1], "rows": {}}
    for name, kw in rows:
        idx.search(fx["Q"], spec.k, ef[0], ef[1], **kw)
        t0 = time.perf_counter()
        n2 = n3 = 0
        for _ in range(steps):
            ids, _, cnt, st = idx.search(fx["Q"], spec.k, ef[0], ef[1], with_counters=True, **kw)
            n2 += int(cnt[:, 3].sum())
            n3 += int(cnt[:, 4].sum())
        dt = time.perf_counter() - t0
        m = spec.queries * steps
        out["rows"][name] = {"qps": round(m / dt, 1), "recall": round(recall(ids, fx["gt"], spec.k), 5),
                             "host_distances_per_query": round((n2 + n3) / m, 1)}
        log(f"  ablation {name}: {out['rows'][name]}")
    return out


def top100(idx, spec, fx, target, steps=2):
    """k = 100: the fastest (ef_gpu, ef_cpu) with recall@100 >= target (ef >= k)."""
    import torch
    from synth.knn import exact_knn
    gt100, _ = exact_knn(fx["X"], fx["Q"], 100, spec.metric, device="cuda")
    curve, best = [], None
    for ef_cpu in (100, 128, 160, 192, 256, 384, 512):
        hit = []
        for ef_gpu in sorted({ef_cpu, min(512, 2 * ef_cpu)}):
            idx.search(fx["Q"][:1000], 100, ef_gpu, ef_cpu)
            ids, _, _, st = idx.search(fx["Q"], 100, ef_gpu, ef_cpu)
            rec = recall(ids, gt100, 100)
            qps = fx["Q"].shape[0] / (st["wall_ms"] / 1e3)
            curve.append({"ef_gpu": ef_gpu, "ef_cpu": ef_cpu, "recall": round(rec, 5), "qps": round(qps, 1)})
            log(f"  k=100 ef_gpu={ef_gpu} ef_cpu={ef_cpu} recall@100={rec:.4f} qps={qps:,.0f}")
            if rec >= target:
                hit.append((qps, ef_gpu, ef_cpu))
        if hit:
            best = max(hit)
            break
    if best is None:
        return {"value": None, "curve": curve}
    _, ef_gpu, ef_cpu = best
    t0 = time.perf_counter()
    for _ in range(steps):
        ids, _, _, _ = idx.search(fx["Q"], 100, ef_gpu, ef_cpu)
    dt = time.perf_counter() - t0
    return {"value": round(spec.queries * steps / dt, 1), "unit": "queries/s", "metric": "recall@100",
            "ef_gpu": ef_gpu, "ef_cpu": ef_cpu, "recall": round(recall(ids, gt100, 100), 5), "curve": curve}


MFMA_PEAK_TFLOPS = {"f32": 157.3, "fp8": 5000.0}


def gemm_leg(spec, fx, V, reps=20):
    """The MFMA kernels on their own, timed with HIP events on the stream they run on:
    the query projection and the FES pivot scoring at the bench shape (fp32), and the FES
    at the 768-d inner-product shape of the large configuration (d_r = 128, 65,536 FP8
    pivots in 32 buckets, E = 64, K = 256).  Algorithmic FLOPs: 2*m*D*d_r for the
    projection and 2*m*(n_p/r)*d_r for the pivot product (Table 2, FES general); the
    pre-selection sort and the exact re-score are extra work on top."""
    import torch
    import paper_2503_21206_amd as pa
    from synth.data import make_rng
    dev = torch.device("cuda")
    rng = make_rng(spec.seed, 90)
    out = {}

    def timed_call(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    m = spec.queries
    Q = torch.as_tensor(fx["Q"]).to(dev)
    Vt = torch.as_tensor(V).to(dev)
    ms = timed_call(lambda: pa.project(Q, Vt, "f32"))
    fl = 2.0 * m * spec.dim * spec.d_r
    out["projection"] = {"shape": f"{m} x {spec.dim} -> {spec.d_r}", "ms": round(ms, 4),
                         "tflops": round(fl / ms / 1e9, 2), "peak": MFMA_PEAK_TFLOPS["f32"],
                         "frac": round(fl / ms / 1e9 / MFMA_PEAK_TFLOPS["f32"], 4), "dtype": "f32"}

    def fes_case(name, m, d, r, n_b, E, K, dtype, metric):
        Qr = torch.as_tensor(rng.standard_normal((m, d)).astype(np.float32)).to(dev)
        EV = rng.standard_normal((r, n_b, d)).astype(np.float32)
        EVn = torch.as_tensor((EV.astype(np.float64) ** 2).sum(-1).astype(np.float32)).to(dev)
        EVid = torch.as_tensor(np.arange(r * n_b, dtype=np.int32).reshape(r, n_b)).to(dev)
        cl = torch.as_tensor(rng.integers(0, r, m).astype(np.int32)).to(dev)
        EVd = torch.as_tensor(EV).to(dev)
        if dtype == "fp8":
            codes, scales = pa.quantize_fp8_rows(EV.reshape(-1, d))
            E8 = torch.as_tensor(codes.reshape(r, n_b, d)).to(dev)
            Es = torch.as_tensor(scales.reshape(r, n_b)).to(dev)
            fn = lambda: pa.select_entries_fp8(Qr, cl, EVd, E8, Es, EVn, EVid, E, K, metric)
        else:
            fn = lambda: pa.select_entries(Qr, cl, EVd, EVn, EVid, E, metric)
        ms = timed_call(fn)
        fl = 2.0 * m * n_b * d
        out[name] = {"shape": f"{m} queries x {r} buckets of {n_b} pivots x {d} dims, E={E}"
                              + (f", K={K}" if dtype == "fp8" else ""),
                     "ms": round(ms, 4), "tflops": round(fl / ms / 1e9, 2), "peak": MFMA_PEAK_TFLOPS[dtype],
                     "frac": round(fl / ms / 1e9 / MFMA_PEAK_TFLOPS[dtype], 5), "dtype": dtype}

    for args in (("fes_f32", m, spec.d_r, spec.r, spec.n_pivots // spec.r, 64, 0, "f32", spec.metric),
                 ("fes_fp8_768d", m, 128, 32, 65536 // 32, 64, 256, "fp8", "ip")):
        try:
            fes_case(*args)
        except pa.PilotannError as e:  # a shape this device cannot hold is reported, not fatal
            out[args[0]] = {"error": str(e)}
    return out


def roofline(spec, agg, steps, ef, E, xr_bytes, form, visited=None):
    """Beam-kernel bytes and time per launch; ef is the stage-1 list size.

    Algorithmic bytes per query (the method's own work): 4*d_r (query) + 4*E (entries) +
    4*R per expansion (adjacency row) + s*d_r per visited node (its reduced row, gathered
    once: Algorithm 1 scores each visited node once) + 8*ef (list out); |visited| comes
    from `visited` (per query, counted with a visited cache that never forgets), the
    expansions from the timed launches' counters.  The kernel's own bytes count its
    distance evaluations instead, which include the re-scores after visited-cache forget
    events; both are reported, the fraction is the method's."""
    m = spec.queries * steps
    fixed = m * (4 * spec.d_r + 4 * E + 8 * ef) + agg["n_exp1"] * 4 * spec.degree
    kernel = fixed + agg["n_dist1"] * xr_bytes * spec.d_r
    method = fixed + (visited * m if visited is not None else agg["n_dist1"]) * xr_bytes * spec.d_r
    launches = agg["beam_launches"]
    avg_ms = agg["beam_ms"] / launches
    achieved = method / launches / (avg_ms / 1e3) / 1e9
    # the traversal's tables: the sampled nodes' reduced rows and subgraph adjacency rows
    n_sub = round(spec.rho * spec.n)
    working_set = n_sub * (xr_bytes * spec.d_r + 4 * spec.degree)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "working_set_bytes": int(working_set),
            "served_from": "infinity_cache" if working_set <= INFINITY_CACHE_BYTES else "hbm",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(spec.name, form, ef),
            "kernel": "beam_kernel", "bytes_per_launch": int(method / launches),
            "kernel_bytes_per_launch": int(kernel / launches),
            "kernel_frac": round(kernel / launches / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "visited_per_query": None if visited is None else round(visited, 2),
            "distance_evaluations_per_query": round(agg["n_dist1"] / m, 2),
            "avg_launch_ms": round(avg_ms, 4), "launches": int(launches)}


def precision_leg(idx, spec, fx, shared, form, ef, n=1000):
    """Distance error of a form against fp64 on its unquantised reduced vectors, at stage 1
    and at the output, on the first n queries.  Stage 1 runs through the stage-isolated
    calls on the same tables the index holds (the projection kernel rounds X V to the
    form, the pivots' fp32 rows feed entry selection), and returns correctly rounded
    distances of the stored rows; the reference is the fp64 distance between Q V and X V
    (V the fp32 projection).  The output distances are the host stages' full distances,
    compared with fp64 full distances."""
    import torch
    import paper_2503_21206_amd as pa
    dev = torch.device("cuda")
    n = min(n, spec.queries)
    V = shared["V"]
    Vt = torch.as_tensor(V).to(dev)
    mask, sr, sn = shared["sub"]
    _, buckets, cent = idx.state()
    Xd = torch.as_tensor(fx["X"]).to(dev)
    Xr = pa.project(Xd, Vt, form)
    del Xd
    piv = buckets.reshape(-1).astype(np.int64)
    EV = pa.project(torch.as_tensor(fx["X"][piv]).to(dev), Vt, "f32").reshape(spec.r, -1, spec.d_r)
    EVn = (EV.double() ** 2).sum(-1).float()
    EVid = torch.as_tensor(buckets).to(dev)
    Q = fx["Q"][:n]
    Qr, cl = pa.project_route(torch.as_tensor(Q).to(dev), Vt, torch.as_tensor(cent).to(dev))
    E = min(ef[0], spec.n_pivots // spec.r)
    ent, _ = pa.select_entries(Qr, cl, EV.contiguous(), EVn, EVid, E, spec.metric)
    R_sub = int((sr[1:] - sr[:-1]).max())
    adj = pa.pack_adjacency(sr, sn, R_sub)
    ids, d, _ = pa.gpu_traverse(Qr, Xr, adj, ent, ef[0], spec.metric)
    torch.cuda.synchronize()
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    del Xr, adj
    ok = ids >= 0
    V64 = V.astype(np.float64)
    q64 = Q.astype(np.float64) @ V64
    rows = fx["X"][ids[ok]].astype(np.float64) @ V64
    qq = q64[np.nonzero(ok)[0]]
    ref = ((qq - rows) ** 2).sum(1) if spec.metric == "l2" else -(qq * rows).sum(1)
    err1 = np.abs(d[ok] - ref) / np.maximum(np.abs(ref), 1e-30)
    oi, od, _, _ = idx.search(Q, spec.k, ef[0], ef[1])
    okk = oi >= 0
    xo = fx["X"][oi[okk]].astype(np.float64)
    qo = Q.astype(np.float64)[np.nonzero(okk)[0]]
    ref_o = ((qo - xo) ** 2).sum(1) if spec.metric == "l2" else -(qo * xo).sum(1)
    err_o = np.abs(od[okk].astype(np.float64) - ref_o) / np.maximum(np.abs(ref_o), 1e-30)
    out = {"queries": n, "stage1_max_rel_err": float(f"{err1.max():.3g}"),
           "stage1_mean_rel_err": float(f"{err1.mean():.3g}"),
           "output_max_rel_err": float(f"{err_o.max():.3g}"),
           "what": "max/mean |delta - delta_64| / |delta_64| over every returned (id, distance): stage 1 against "
                   "fp64 distances of the unquantised reduced vectors (Q V, X V), output against fp64 full "
                   "distances"}
    log(f"  precision {form}: {out}")
    return out


def memory_leg(spec, fx, shared, ef, full_info, steps):
    """Memory-bounded layout (X_r and the device subgraph for the sampled nodes only, fp16
    rows) at several sampling ratios: HBM held by the index (and the library's model of
    it), QPS and recall at ef; then the (rho, d_r) the planner picks for a few budgets."""
    import dataclasses
    import paper_2503_21206_amd as pa
    out = {"what": "compact layout, fp16 X_r, ef_gpu/ef_cpu as timed; hbm_bytes = index tables and search "
                   "buffers on the device",
           "full_layout_rho_0.25": {"hbm_bytes": full_info["hbm_bytes"], "xr_rows": full_info["xr_rows"]},
           "points": []}
    for rho in (0.1, 0.25, 0.5, 0.75):
        sp = dataclasses.replace(spec, rho=rho)
        sh = {"V": shared["V"]} if rho != spec.rho else shared
        idx = build_index(sp, fx, "f16", sh, compact=True)
        dt, agg, rec = timed(idx, sp, fx, ef, steps, 1)
        info = idx.info()
        # the library's HBM model for the same shape (the timed searches upload the queries)
        shape = pa.memory_shape(sp.n, sp.dim, info["R_sub"], sp.n_pivots, sp.r, "f16", queries=sp.queries,
                                ef_gpu=ef[0])
        out["points"].append({"rho": rho, "hbm_bytes": info["hbm_bytes"],
                              "model_hbm_bytes": pa.hbm_bytes(shape, info["xr_rows"] / sp.n, sp.d_r),
                              "xr_rows": info["xr_rows"],
                              "qps": round(sp.queries * steps / dt, 1), "recall": round(rec, 5),
                              "mean_n_dist3": round(agg["n_dist3"] / (sp.queries * steps), 1)})
        log(f"  compact rho={rho}: {out['points'][-1]}")
        idx.close()
    # the planner's choice per HBM budget over the (rho, d_r) grid, at the reconnection
    # degree cap (the subgraph's padded degree is at most that)
    shape = pa.memory_shape(spec.n, spec.dim, spec.degree, spec.n_pivots, spec.r, "f16", queries=spec.queries,
                            ef_gpu=ef[0])
    rhos, widths = [0.1, 0.25, 0.5, 0.75, 1.0], [32, 64, 128]
    out["plan"] = {"rhos": rhos, "d_r": widths, "choices": []}
    for mb in (32, 64, 128, 256):
        try:
            rho, d_r, b = pa.plan_memory(shape, mb << 20, rhos, widths)
            out["plan"]["choices"].append({"budget_mib": mb, "rho": rho, "d_r": d_r, "hbm_bytes": b})
        except pa.PilotannError:
            out["plan"]["choices"].append({"budget_mib": mb, "rho": None})
    log(f"  plan: {out['plan']['choices']}")
    return out


def bucket_leg(idx32, spec, fx, shared, ef, target, steps):
    """FES with r = 64 buckets (one per lane of a 64-wide wavefront; the paper's r = 32
    matches a 32-wide warp) against the r = 32 index: recall at the same ef, the fastest
    swept pair that reaches the target recall, and both indexes timed alternately at their
    own pairs (the host stages' speed drifts within a run)."""
    import dataclasses
    sp = dataclasses.replace(spec, r=64)
    sh = {k: shared[k] for k in ("V", "sub", "pivots")}
    sh["init"] = fx["kmeans_init_choice"](spec.n_pivots, sp.r, spec.seed)
    idx = build_index(sp, fx, "f32", sh)
    _, _, rec_same = timed(idx, sp, fx, ef, 1, 0)
    out = {"r": 64, "recall_at_r32_ef": {"ef_gpu": ef[0], "ef_cpu": ef[1], "recall": round(rec_same, 5)}}
    ef64, curve = sweep(idx, sp, fx, target, sorted(set(sp.ef) | {40, 56}))  # finer near the target
    out["curve"] = curve
    if ef64 is not None:
        best = {32: (0.0, None, None), 64: (0.0, None, None)}
        for _ in range(2):
            for r, ix, e in ((64, idx, ef64), (32, idx32, ef)):
                dt, agg, rec = timed(ix, sp if r == 64 else spec, fx, e, steps, 1)
                q = spec.queries * steps / dt
                if q > best[r][0]:
                    best[r] = (q, rec, agg)
        for r, e in ((64, ef64), (32, ef)):
            q, rec, agg = best[r]
            out[f"r{r}_at_target"] = {"ef_gpu": e[0], "ef_cpu": e[1], "qps": round(q, 1), "recall": round(rec, 5),
                                      "mean_n_dist3": round(agg["n_dist3"] / (spec.queries * steps), 1),
                                      "fes_ms_per_step": round(agg["fes_ms"] / steps, 3)}
    idx.close()
    log(f"  buckets: { {k: v for k, v in out.items() if k != 'curve'} }")
    return out


def ratio_sweep(spec, fx, shared, ef, steps):
    """The paper's (rho, d_r / D) grid, compact layout with fp16 rows at a fixed ef: recall,
    QPS and HBM per point (opt-in: nine index builds)."""
    import dataclasses
    subs, Vs, out = {}, {spec.d_r: shared["V"]}, []
    for d_r in (32, 64, 128):
        for rho in (0.1, 0.25, 0.5):
            sp = dataclasses.replace(spec, rho=rho, d_r=d_r)
            sh = dict(subs.get(rho, {}))
            if d_r in Vs:
                sh["V"] = Vs[d_r]
            idx = build_index(sp, fx, "f16", sh, compact=True)
            Vs[d_r] = sh["V"]
            subs[rho] = {k: sh[k] for k in ("sub", "pivots", "init")}
            dt, agg, rec = timed(idx, sp, fx, ef, steps, 1)
            info = idx.info()
            out.append({"rho": rho, "d_r": d_r, "recall": round(rec, 5), "qps": round(sp.queries * steps / dt, 1),
                        "hbm_bytes": info["hbm_bytes"],
                        "beam_ms_per_step": round(agg["beam_ms"] / steps, 3),
                        "mean_n_dist3": round(agg["n_dist3"] / (sp.queries * steps), 1)})
            log(f"  ratio sweep: {out[-1]}")
            idx.close()
    return {"what": f"compact layout, fp16 X_r, ef_gpu/ef_cpu = {ef}", "points": out}


def gpu_only_leg(spec, fx, target, steps):
    """The paper's GPU-only special case: every node sampled (the subgraph is the full
    graph), d_r = D in fp32, stage 1 alone finds the candidates and the host only re-ranks
    the list by full distance (no final traversal).  Smallest swept ef_gpu reaching the
    target recall, then `steps` timed searches."""
    import torch
    import paper_2503_21206_amd as pa
    t = time.time()
    idx = pa.Index(pa.IndexConfig(dim=spec.dim, d_r=spec.dim, metric=spec.metric, xr_dtype="f32", r=spec.r))
    idx.set_data(fx["X"], fx["rp"], fx["nb"])
    idx.fit_projection()
    try:
        idx.build_subgraph(np.ones(spec.n, dtype=np.uint8), fx["rp"], fx["nb"])
    except pa.PilotannError as e:  # e.g. a full-graph degree above the traversal's limit
        idx.close()
        return {"error": str(e)}
    deg = fx["rp"][1:] - fx["rp"][:-1]
    pivots = fx["pivot_choice"](np.nonzero(deg > 0)[0], spec.n_pivots, spec.seed)
    idx.build_entries(pivots, fx["kmeans_init_choice"](spec.n_pivots, spec.r, spec.seed), 10)
    log(f"gpu-only index built in {time.time() - t:.1f}s")
    curve, chosen = [], None
    for ef in (32, 64, 96, 128, 192, 256, 384, 512):
        ids, _, _, st = idx.search(fx["Q"], spec.k, ef, ef, stage_mask=5)
        rec = recall(ids, fx["gt"], spec.k)
        curve.append({"ef_gpu": ef, "recall": round(rec, 5), "qps": round(fx["Q"].shape[0] / (st["wall_ms"] / 1e3), 1)})
        log(f"  gpu-only ef={ef:4d} recall@{spec.k}={rec:.4f}")
        if rec >= target:
            chosen = ef
            break
    out = {"what": "every node sampled, d_r = D fp32, stage 1 on the GPU, host re-rank of the stage-1 list only",
           "curve": curve, "value": None}
    if chosen is not None:
        agg = None
        t0 = time.perf_counter()
        for _ in range(steps):
            ids, _, _, st = idx.search(fx["Q"], spec.k, chosen, chosen, stage_mask=5)
            agg = st if agg is None else {k: agg[k] + v for k, v in st.items()}
        dt = time.perf_counter() - t0
        out.update({"value": round(spec.queries * steps / dt, 1), "unit": "queries/s", "ef_gpu": chosen,
                    "recall": round(recall(ids, fx["gt"], spec.k), 5),
                    "beam_ms_per_step": round(agg["beam_ms"] / steps, 3),
                    "fes_ms_per_step": round(agg["fes_ms"] / steps, 3)})
    idx.close()
    return out


def cpu_baseline(spec, fx, shared, ef_pair, budget_s, plain_ef=None):
    """The oracle, timed on the host cores in worker processes (one per core): the full
    pipeline (its own fp64 projection, clustering of the same pivots, stages 1-3) at the
    timed (ef_gpu, ef_cpu), and plain Algorithm 1 on the full graph from the same FES
    entries at `plain_ef` (the CPU-only leg's ef), each on a bounded sample of queries sized
    from a short serial calibration so that it takes about budget_s seconds."""
    import oracle
    from oracle.parallel import host_cores
    from tests import oracle_jobs
    t = time.time()
    X = fx["X"]
    V, _, _ = oracle.fit_projection(X, spec.d_r, spec.metric)
    V32 = V.astype(np.float32)
    Xr = oracle.project(X, V32).astype(np.float32)
    Qr = oracle.project(fx["Q"], V32).astype(np.float32)
    mask, sr, sn = shared["sub"]
    P = Xr[shared["pivots"]]
    buckets, cent = oracle.balanced_kmeans(P.astype(np.float64), spec.r, shared["init"])
    cent = cent.astype(np.float32)
    log(f"oracle setup {time.time() - t:.1f}s")
    ef_gpu, ef_cpu = ef_pair
    E = min(ef_gpu, spec.n_pivots // spec.r)
    cores = host_cores()
    arrays = dict(Q=fx["Q"], Qr=Qr, X=X, V=V32, rp=fx["rp"], nb=fx["nb"], sr=sr, sn=sn, Xr=Xr, cent=cent,
                  buckets=buckets, P=P, pivots=shared["pivots"])
    out = {"unit": "queries/s", "cores": cores, "kind": "oracle"}

    def leg(kw, label):
        t0 = time.perf_counter()  # serial calibration on a few queries
        n_cal = 8
        oracle.pipeline(fx["Q"][:n_cal], X, V32, fx["rp"], fx["nb"], sr, sn, Xr, cent, buckets, P,
                        shared["pivots"], Qr=Qr[:n_cal], metric=spec.metric, **kw)
        rate1 = n_cal / (time.perf_counter() - t0)
        n = int(min(spec.queries, max(cores * 4, rate1 * cores * budget_s)))
        rows = np.arange(n)
        t0 = time.perf_counter()
        res, = oracle_jobs.pipeline(arrays, [(rows, dict(metric=spec.metric, **kw))], procs=cores, chunk=8)
        dt = time.perf_counter() - t0
        rec = recall(res[0], fx["gt"][:n], spec.k)
        log(f"  oracle {label}: {n} queries on {cores} processes in {dt:.1f}s, recall {rec:.4f}")
        return {"value": round(n / dt, 2), "sample": f"first {n} of {spec.queries} queries, {label}, {dt:.1f}s "
                                                     f"on {cores} worker processes", "recall": round(rec, 5)}

    full = leg(dict(k=spec.k, ef_gpu=ef_gpu, ef_cpu=ef_cpu, E=E), f"full pipeline at ef_gpu={ef_gpu} ef_cpu={ef_cpu}")
    out.update(value=full["value"], sample=full["sample"], recall=full["recall"])
    if plain_ef is not None:
        out["plain_algorithm1"] = leg(dict(k=spec.k, ef_gpu=plain_ef, ef_cpu=plain_ef, E=E, use_gpu_stage=False),
                                      f"Algorithm 1 on the full graph from the FES entries at ef={plain_ef}")
    return out


def serve_batch_bytes(spec, m, ef):
    """Device bytes of a serving micro-batch of m requests at list size ef (the footprint the
    server's admission charges, from the header's formula)."""
    al = lambda b: (b + 255) // 256 * 256
    e = min(ef, spec.n_pivots // spec.r)
    return (al(4 * m * spec.dim) + al(4 * m * spec.d_r) + al(4 * m) + 2 * al(4 * m * e) + 2 * al(4 * m * ef)
            + al(16 * m) + al(4 * m) + al(4 * (3 * spec.r + 2 + m)))


def serve_bench(idx, spec, fx, rates, seconds, budget):
    """Open-loop Poisson arrivals at each rate; latency from the scheduled arrival time.

    Requests draw k from {10, 50, 100} and ef from {64, 128, 256, 512}.  The submitting
    loop never waits for completions; latency = completion - scheduled arrival, so a
    client that falls behind is charged to the system (no coordinated omission)."""
    import paper_2503_21206_amd as pa
    from synth.data import make_rng, OFF_ARRIVAL
    out = []
    Q = fx["Q"]
    for rate in rates:
        srv = pa.Server(idx, hbm_budget=budget, max_batch=1024, streams=3)
        rng = make_rng(spec.seed + OFF_ARRIVAL, int(rate))
        n = int(rate * seconds)
        gaps = rng.exponential(1.0 / rate, size=n)
        sched = np.cumsum(gaps)
        ks = rng.choice([10, 50, 100], size=n)
        efs = rng.choice([64, 128, 256, 512], size=n)
        qi = rng.integers(0, Q.shape[0], size=n)
        submit_py = np.zeros(n)
        t0 = time.perf_counter()
        results = []
        i = 0
        while i < n:
            now = time.perf_counter() - t0
            while i < n and sched[i] <= now:
                submit_py[i] = time.perf_counter() - t0
                srv.submit(Q[qi[i]], int(ks[i]), int(efs[i]), i)
                i += 1
            results.extend(srv.poll(4096))
            if i < n:
                wait = sched[i] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3))
        srv.drain()
        results.extend(srv.poll(1 << 20))
        t_end = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        by_tag = {r["tag"]: r for r in results}
        # server clock -> python clock via each request's own submit timestamp
        lat = []
        hits = 0
        for tag, r in by_tag.items():
            offset = r["t_submit_us"] / 1e6 - submit_py[tag]
            arrival = sched[tag] + offset
            lat.append(r["t_done_us"] / 1e6 - arrival)
            hits += len(set(r["ids"][:10].tolist()) & set(fx["gt"][qi[tag]][:10].tolist()))
        lat = np.array(lat) * 1e3
        out.append({"offered_qps": rate, "achieved_qps": round(len(by_tag) / t_end, 1),
                    "p50_ms": round(float(np.percentile(lat, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat, 99)), 3),
                    "recall@10": round(hits / (10 * len(by_tag)), 4), "requests": len(by_tag),
                    "micro_batches": st["batches"], "largest_micro_batch": st["max_batch"]})
        log(f"serve rate={rate}: {out[-1]}")
    return out


def flat_leg(args, spec):
    """The same shape on a flat mixture (1,024 well separated blobs, centres ~ N(0, 4I)):
    fixture, fp32 index, the sweep to the target recall (or its end), then one timed run."""
    fx = build_fixture(spec, "cuda")
    shared = {}
    idx = build_index(spec, fx, "f32", shared)
    ef, curve = sweep(idx, spec, fx, args.target, spec.ef)
    out = {"workload": f"{spec.name}: N={spec.n} d={spec.dim} {spec.components}-component flat GMM "
                       f"(centres ~ N(0, 4I)), otherwise as the headline", "curve": curve, "value": None}
    if ef is not None:
        dt, agg, rec = timed(idx, spec, fx, ef, max(1, min(args.steps, 5)), 1)
        out.update(value=round(spec.queries * max(1, min(args.steps, 5)) / dt, 1), unit="queries/s",
                   ef_gpu=ef[0], ef_cpu=ef[1], recall=round(rec, 5))
    else:
        out["note"] = f"recall@{spec.k} stays below {args.target} over the whole ef sweep"
    idx.close()
    log(f"  flat mixture: { {k: v for k, v in out.items() if k != 'curve'} }")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gmm1m")
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-only", action="store_true", help="skip the GPU-stage-off comparison leg")
    ap.add_argument("--no-gemm", action="store_true", help="skip the MFMA kernel leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the ablation and top-100 legs")
    ap.add_argument("--no-bloom", action="store_true",
                    help="skip the stage-1 variant legs (Bloom filter, expansion width 2) of each form")
    ap.add_argument("--ratio-sweep", action="store_true", help="add the (rho, d_r) grid (nine index builds)")
    ap.add_argument("--forms", default="f32,f16")
    ap.add_argument("--serve-rates", default="2000,5000,10000,20000,50000")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-budget", type=int, default=32 << 30)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device-to-device copy kernel (counter calibration for profiles)")
    ap.add_argument("--calibration-only", action="store_true",
                    help="run only the 1 GiB copy kernel of --copy-calibration and exit")
    ap.add_argument("--no-flat", dest="flat", action="store_false",
                    help="skip the flat-mixture leg (the same shape, centres ~ N(0, 4I))")
    ap.add_argument("--ef", default="",
                    help="ef_gpu,ef_cpu to time directly instead of sweeping for the target recall")
    ap.add_argument("--n", type=int, default=0,
                    help="base rows (the first n rows of the workload's base set; 0: all of them)")
    ap.add_argument("--queries", type=int, default=0, help="queries (the first ones; 0: the workload's count)")
    ap.add_argument("--nprobe", type=int, default=64, help="IVF lists probed per row by the large-N graph builder")
    ap.add_argument("--fixture-cache", default="",
                    help="directory that keeps the graph, ground truth and subgraph between runs")
    ap.add_argument("--no-precision", action="store_true", help="skip the per-form distance-error leg")
    ap.add_argument("--kernels-only", action="store_true",
                    help="time only the MFMA kernels (projection, FES) on synthetic inputs of the workload's "
                         "shape and print their JSON; no fixture, no search")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibration_only:
        copy_calibration()
        return
    import paper_2503_21206_amd as pa
    from synth import SPECS
    pa.device_init(0)
    import dataclasses
    spec = SPECS[args.workload]
    if args.n:
        spec = dataclasses.replace(spec, n=args.n)
    if args.queries:
        spec = dataclasses.replace(spec, queries=args.queries)
    if args.kernels_only:
        from synth import query_vectors
        from synth.data import make_rng
        Qk = query_vectors(spec)
        Vk = np.linalg.qr(make_rng(spec.seed, 91).standard_normal((spec.dim, spec.d_r)))[0].astype(np.float32)
        print(json.dumps({"kernels": gemm_leg(spec, {"Q": Qk}, Vk),
                          "workload": f"{spec.name} query shape, random orthonormal projection"}), flush=True)
        return
    fx = build_fixture(spec, "cuda", cache=args.fixture_cache or None, nprobe=args.nprobe)
    shared = {}
    forms = {}
    serving = None
    baseline_cpu_only = None
    extra = {}
    for form in args.forms.split(","):
        idx = build_index(spec, fx, form, shared)
        if args.ef:
            ef, curve = tuple(int(x) for x in args.ef.split(",")), []
        else:
            log(f"sweep {form}")
            ef, curve = sweep(idx, spec, fx, args.target, spec.ef)
        if ef is None:
            ef = (spec.ef[-1], spec.ef[-1])
            log(f"  target recall not reached; timing at ef={ef}")
        (dt, agg, rec), runs = timed_median(idx, spec, fx, ef, args.steps, args.warmup)
        E = min(ef[0], spec.n_pivots // spec.r)
        xr_bytes = 4 if form == "f32" else 2
        qps = spec.queries * args.steps / dt
        visited = visited_per_query(idx, spec, fx, ef)
        dtr, _, _ = timed(idx, spec, fx, ef, args.steps, 1, resident=True)
        forms[form] = {
            "value": round(qps, 1), "ef_gpu": ef[0], "ef_cpu": ef[1], "recall": round(rec, 5),
            "ms_per_step": round(dt * 1e3 / args.steps, 3), "runs_qps": runs,
            "queries_resident_in_hbm_qps": round(spec.queries * args.steps / dtr, 1),
            "roofline": roofline(spec, agg, args.steps, ef[0], E, xr_bytes, form, visited),
            "gpu_stage": {"beam_ms_per_step": round(agg["beam_ms"] / args.steps, 3),
                          "fes_ms_per_step": round(agg["fes_ms"] / args.steps, 3),
                          "host_wait_ms_per_step": round(agg["host_wait_ms"] / args.steps, 3),
                          "mean_n_exp1": round(agg["n_exp1"] / (spec.queries * args.steps), 1),
                          "mean_n_dist1": round(agg["n_dist1"] / (spec.queries * args.steps), 1),
                          "mean_n_dist2": round(agg["n_dist2"] / (spec.queries * args.steps), 1),
                          "mean_n_dist3": round(agg["n_dist3"] / (spec.queries * args.steps), 1),
                          "forget_events": int(agg["n_reset1"])},
            "curve": curve,
        }
        log(f"{form}: ef={ef} recall={rec:.4f} qps={qps:,.0f} roofline={forms[form]['roofline']}")
        if not args.no_precision:
            forms[form]["precision"] = precision_leg(idx, spec, fx, shared, form, ef)
            if form != "f32" and "f32" in forms and (forms["f32"]["ef_gpu"], forms["f32"]["ef_cpu"]) != ef:
                e32 = (forms["f32"]["ef_gpu"], forms["f32"]["ef_cpu"])
                _, _, rec32 = timed(idx, spec, fx, e32, 1, 0)
                forms[form]["precision"]["recall_at_f32_ef"] = {"ef_gpu": e32[0], "ef_cpu": e32[1],
                                                                "recall": round(rec32, 5)}
            if form != "f32" and "f32" in forms:
                r32 = forms["f32"]["recall"]
                mine = forms[form]["precision"].get("recall_at_f32_ef", {}).get("recall", rec)
                forms[form]["precision"]["recall_loss_vs_f32"] = round(r32 - mine, 5)
        if not args.no_bloom:  # stage-1 variants at the same ef
            variants = {"bloom": ("the Bloom-filter visited set of section 4.3 (automatic size, 32 bits per "
                                  "cache slot) instead of the exact cache", True, 1),
                        "width2": ("two unchecked entries expanded per step (not the paper's Algorithm 1)", False, 2),
                        "bloom+width2": ("both", True, 2)}
            if spec.degree > 32:  # expansion width 2 takes subgraph degrees up to 32
                variants = {"bloom": variants["bloom"]}
            forms[form]["variants"] = {}
            for name, (what, bloom, width) in variants.items():
                dtb, aggb, recb = timed(idx, spec, fx, ef, args.steps, args.warmup, bloom=bloom, width=width)
                vis_b = aggb["n_dist1"] / (spec.queries * args.steps) if bloom else \
                    visited_per_query(idx, spec, fx, ef, width=width)
                forms[form]["variants"][name] = {
                    "what": what, "value": round(spec.queries * args.steps / dtb, 1), "recall": round(recb, 5),
                    "ms_per_step": round(dtb * 1e3 / args.steps, 3),
                    "roofline": roofline(spec, aggb, args.steps, ef[0], E, xr_bytes, f"{form}+{name}", vis_b),
                    "mean_n_exp1": round(aggb["n_exp1"] / (spec.queries * args.steps), 1),
                    "mean_n_dist1": round(aggb["n_dist1"] / (spec.queries * args.steps), 1)}
                log(f"{form} {name}: recall={recb:.4f} roofline={forms[form]['variants'][name]['roofline']}")
        if form == "f32" and not args.no_cpu_only:
            log("cpu-only (GPU stage off)")
            baseline_cpu_only = cpu_only(idx, spec, fx, args.target, max(1, min(args.steps, 3)))
        if form == "f32" and not args.no_extra:
            log("ablation")
            extra["ablation"] = ablation(idx, spec, fx, ef)
            log("top-100")
            extra["top100"] = top100(idx, spec, fx, args.target)
            log("gpu-only special case")
            extra["gpu_only"] = gpu_only_leg(spec, fx, args.target, max(1, min(args.steps, 3)))
            log("64 buckets")
            extra["fes_64_buckets"] = bucket_leg(idx, spec, fx, shared, ef, args.target,
                                                 max(1, min(args.steps, 3)))
        if form == "f16" and args.ratio_sweep:
            log("ratio sweep")
            extra["ratio_sweep"] = ratio_sweep(spec, fx, shared, ef, max(1, min(args.steps, 3)))
        if form == "f16" and not args.no_extra:
            log("memory-bounded layout")
            extra["memory_bounded"] = memory_leg(spec, fx, shared, ef, idx.info(), max(1, min(args.steps, 3)))
        if form == "f16" and args.serve_rates:
            rates = [float(x) for x in args.serve_rates.split(",") if x]
            serving = {"index_hbm_bytes": idx.info()["hbm_bytes"],
                       "rates": serve_bench(idx, spec, fx, rates, args.serve_seconds, args.serve_budget)}
            # a budget that binds: the index plus three slots of 32 requests at list size 512
            tight = serving["index_hbm_bytes"] + 3 * serve_batch_bytes(spec, 32, 512)
            low = [r for r in rates if r <= 20000][-2:]
            log(f"serving under a binding budget of {tight} bytes")
            serving["binding_budget"] = {
                "hbm_budget": tight,
                "what": "index bytes + 3 slots holding 32 requests at ef 512 each (more at smaller ef)",
                "rates": serve_bench(idx, spec, fx, low, args.serve_seconds, tight)}
        idx.close()
    if args.flat and not args.no_extra and args.workload + "_flat" in SPECS and not args.n:
        log("flat mixture (centres ~ N(0, 4I)) at the same shape")
        extra["flat_mixture"] = flat_leg(args, SPECS[args.workload + "_flat"])
    main_form = "f32" if "f32" in forms else next(iter(forms))
    f = forms[main_form]
    out = {
        "metric": "QPS at recall@10=0.95 on 1 MI355X (FP32 form; FP16 form alongside)",
        "value": f["value"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{spec.name}: N={spec.n} d={spec.dim} {spec.metric} k={spec.k} "
                               f"{spec.components}-component {'mixture' if spec.kind != 'aniso' else 'anisotropic mixture'}"
                               f", {spec.queries} queries, degree {spec.degree}, "
                               f"d_r={spec.d_r}, rho={spec.rho} {spec.sample_mode}, {spec.n_pivots} pivots/"
                               f"{spec.r} buckets; graph from {fx['graph']}", "ef_gpu": f["ef_gpu"], "ef_cpu": f["ef_cpu"],
                   "recall": f["recall"],
                   "host_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))},
        "roofline": f["roofline"],
        "forms": forms,
    }
    out.update(extra)
    if not args.no_gemm:
        log("MFMA kernels on their own")
        out["gemm"] = gemm_leg(spec, fx, shared["V"])
    if baseline_cpu_only is not None:
        co = dict(baseline_cpu_only)
        co["what"] = ("this library with the GPU stage off: Algorithm 1 on the full graph on the host cores from "
                      "the FES entries, smallest ef reaching the target recall")
        if co.get("value"):
            co["speedup_of_value"] = round(f["value"] / co["value"], 2)
        out["cpu_only"] = co
    if serving is not None:
        out["serving"] = {"workload": f"{spec.name} index, fp16 reduced vectors; Poisson arrivals, k in "
                                      f"{{10,50,100}}, ef in {{64,128,256,512}}, {args.serve_seconds}s per rate, "
                                      f"HBM budget {args.serve_budget} B (index + slot arenas)", **serving}
    if not args.no_cpu_baseline:
        plain_ef = baseline_cpu_only.get("ef") if baseline_cpu_only else f["ef_cpu"]
        out["cpu_baseline"] = cpu_baseline(spec, fx, shared, (f["ef_gpu"], f["ef_cpu"]), args.cpu_budget, plain_ef)
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        copy_calibration()


def copy_calibration():
    """One elementwise kernel that reads 1 GiB and writes 1 GiB: what a counter reads for
    it scales the same counter on the other kernels to bytes."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    log("copy calibration: 1073741824 bytes read, 1073741824 bytes written")


if __name__ == "__main__":
    main()
