"""Small seeded workloads for the parity tests: synthetic inputs plus the
oracle's view of every stage (computed on the CPU, never from the library)."""

from __future__ import annotations

import numpy as np

import oracle
from synth import SPECS, base_vectors, query_vectors, node_order, pivot_choice, kmeans_init_choice
from synth.graph import build_graph, build_subgraph_csr, padded_to_csr


def to_f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16)


def to_bf16(x):
    """Round-to-nearest-even float32 -> bfloat16, returned as float32 values."""
    import torch
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).float().numpy()


def build_tiny(n_queries: int | None = None, spec_name: str = "tiny", device=None):
    """The 10K x 96 workload with oracle-side projection, subgraph, pivots and buckets."""
    s = SPECS[spec_name]
    X = base_vectors(s)
    Q = query_vectors(s, n_queries)
    adj = build_graph(X, s.degree, device=device)
    rp, nb = padded_to_csr(adj)
    order = node_order(s.n, s.seed)
    mask = oracle.sample_nodes(rp, nb, order, round(s.rho * s.n), s.sample_mode)
    sr, sn = build_subgraph_csr(X, mask, s.degree, device=device)
    R_sub = int(max(1, (sr[1:] - sr[:-1]).max()))
    V64, w, mu = oracle.fit_projection(X, s.d_r, s.metric)
    V32 = V64.astype(np.float32)
    Xr32 = oracle.project(X, V32).astype(np.float32)  # fp64 product of the fp32 inputs, rounded once
    Qr32 = oracle.project(Q, V32).astype(np.float32)
    S = np.nonzero(mask)[0]
    deg = sr[1:] - sr[:-1]
    S_out = S[deg[S] > 0]
    pivots = pivot_choice(S_out, s.n_pivots, s.seed)
    init = kmeans_init_choice(s.n_pivots, s.r, s.seed)
    P32 = Xr32[pivots]
    buckets, cent = oracle.balanced_kmeans(P32, s.r, init)
    return dict(spec=s, X=X, Q=Q, adj=adj, rp=rp, nb=nb, mask=mask, sr=sr, sn=sn, R_sub=R_sub,
                sub_adj=oracle.padded_from_csr(sr, sn, R_sub), V64=V64, V32=V32, evals=w, mean=mu,
                Xr32=Xr32, Qr32=Qr32, pivots=pivots, init=init, P32=P32, buckets=buckets,
                cent32=cent.astype(np.float32))


def oracle_entries(w, E, Qr=None):
    """Oracle FES entries for every query (on the fp32-rounded reduced queries)."""
    Qr = w["Qr32"] if Qr is None else Qr
    ids, d, cl, margin = oracle.select_entries(Qr, w["cent32"].astype(np.float64), w["buckets"], w["P32"],
                                               w["pivots"], E, w["spec"].metric)
    return ids, d, cl, margin


def device_tables(w, E_unused=None):
    """EV / EVnorm / EVid laid out bucket-major from the oracle's buckets."""
    b = w["buckets"]
    EV = w["P32"][b]  # [r][n_b][d]
    EVn = (EV.astype(np.float64) ** 2).sum(-1).astype(np.float32)
    EVid = w["pivots"][b].astype(np.int32)
    return EV.astype(np.float32), EVn, EVid
