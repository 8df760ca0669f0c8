"""Python binding of libpilotann (the PilotANN GPU stage for MI355X).

Argument marshalling only: every step runs in the library's HIP kernels or host
C++.  Device buffers are torch tensors on the GPU (torch supplies memory and the
current stream); host buffers are numpy arrays.  The names follow the C ABI in
``include/pilotann.h`` without the ``pa_`` prefix.  Importing works without a
GPU; the library itself is loaded on first use and a missing build raises.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpilotann.so")

PA_OK = 0
PA_METRIC_L2, PA_METRIC_IP = 0, 1
PA_F32, PA_F16, PA_BF16, PA_FP8E4M3 = 0, 1, 2, 3
PA_SAMPLE_UNIFORM, PA_SAMPLE_SEED_EXPAND = 0, 1
PA_VISITED_EXACT, PA_VISITED_BLOOM = 0, 1
PA_ENTRIES_FES, PA_ENTRIES_FIXED = 0, 1
PA_MAX_EF = 512

METRICS = {"l2": PA_METRIC_L2, "ip": PA_METRIC_IP}
DTYPES = {"f32": PA_F32, "f16": PA_F16, "bf16": PA_BF16}


class PilotannError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"pilotann status {status}: {message}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("d_r", C.c_int32), ("metric", C.c_int32), ("xr_dtype", C.c_int32),
                ("r", C.c_int32), ("refine_steps", C.c_int32), ("threads", C.c_int32),
                ("device", C.c_int32), ("hbm_budget", C.c_int64), ("pivot_dtype", C.c_int32),
                ("preselect", C.c_int32), ("compact", C.c_int32)]


class SearchOpts(C.Structure):
    _fields_ = [("ef_gpu", C.c_int32), ("ef_cpu", C.c_int32), ("E", C.c_int32), ("batch", C.c_int32),
                ("stage_mask", C.c_int32), ("cache_log2", C.c_int32), ("threads", C.c_int32),
                ("handoff", C.c_int32), ("q_dev", C.c_void_p), ("visited", C.c_int32), ("width", C.c_int32),
                ("entries", C.c_int32), ("serial", C.c_int32)]


class TraverseOpts(C.Structure):
    _fields_ = [("visited", C.c_int32), ("cache_log2", C.c_int32), ("width", C.c_int32), ("ef_dev", C.c_void_p)]


class SearchStats(C.Structure):
    _fields_ = [("wall_ms", C.c_double), ("beam_ms", C.c_double), ("fes_ms", C.c_double),
                ("beam_launches", C.c_int64), ("n_exp1", C.c_int64), ("n_dist1", C.c_int64),
                ("n_dist2", C.c_int64), ("n_dist3", C.c_int64), ("n_exp3", C.c_int64),
                ("n_reset1", C.c_int64), ("host_wait_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class IndexInfo(C.Structure):
    _fields_ = [("N", C.c_int64), ("R_full", C.c_int32), ("R_sub", C.c_int32), ("n_pivots", C.c_int32),
                ("built", C.c_int32), ("hbm_bytes", C.c_int64), ("xr_rows", C.c_int64)]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_batch", C.c_int32), ("streams", C.c_int32),
                ("threads", C.c_int32), ("max_k", C.c_int32)]


class MemoryShape(C.Structure):
    _fields_ = [("N", C.c_int64), ("dim", C.c_int32), ("xr_dtype", C.c_int32), ("pivot_dtype", C.c_int32),
                ("compact", C.c_int32), ("R_sub", C.c_int32), ("n_pivots", C.c_int32), ("r", C.c_int32),
                ("queries", C.c_int64), ("batch", C.c_int32), ("ef_gpu", C.c_int32), ("E", C.c_int32),
                ("q_on_device", C.c_int32)]


class ResultInfo(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("k", C.c_int32), ("ef", C.c_int32), ("t_submit_us", C.c_double),
                ("t_admit_us", C.c_double), ("t_done_us", C.c_double)]


_P = C.c_void_p
_I32, _I64, _F64 = C.c_int32, C.c_int64, C.c_double

# name -> argument types (every function returns int32 status except where noted)
_SIGS = {
    "pa_abi_version": [],
    "pa_device_init": [_I32],
    "pa_gram_f64": [_P, _I64, _I32, _P, _P, _I32, _P],
    "pa_eigh_f64": [_P, _I32, _P, _P],
    "pa_fit_projection": [_P, _I64, _I32, _I32, _I32, _P, _P, _P],
    "pa_project": [_P, _I64, _I32, _P, _I32, _P, _I32, _P],
    "pa_project_route": [_P, _I64, _I32, _P, _I32, _P, _I32, _P, _P, _P],
    "pa_sample_nodes": [_I64, _P, _P, _P, _I64, _I32, _P],
    "pa_check_subgraph": [_I64, _P, _P, _P, _I32],
    "pa_pack_adjacency": [_I64, _P, _P, _I32, _P, _P],
    "pa_build_entries": [_P, _I32, _I32, _I32, _P, _I32, _P, _P],
    "pa_select_entries": [_P, _P, _I64, _I32, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P],
    "pa_select_entries_noalloc": [_P, _P, _I64, _I32, _P, _P, _P, _I32, _I32, _I32, _I32, _P, _P, _P],
    "pa_gpu_traverse": [_P, _I64, _I32, _P, _I32, _I64, _P, _I32, _P, _I32, _I32, _I32, C.POINTER(TraverseOpts), _P,
                        _P, _P, _P],
    "pa_cpu_stages": [_P, _I64, _I32, _P, _I32, _P, _I32, _P, _I64, _P, _I32, _I32, _I32, _I32, _I32, _I32,
                      _P, _P, _P],
    "pa_cpu_search": [_P, _I64, _I32, _P, _I32, _P, _I64, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P],
    "pa_index_create": [C.POINTER(Params), C.POINTER(_P)],
    "pa_index_destroy": [_P],
    "pa_index_set_data": [_P, _P, _I64, _P, _P],
    "pa_index_fit_projection": [_P, _I32],
    "pa_index_set_projection": [_P, _P],
    "pa_index_sample_nodes": [_P, _P, _I64, _I32, _P],
    "pa_index_build_subgraph": [_P, _P, _P, _P],
    "pa_index_build_entries": [_P, _P, _I32, _P, _I32],
    "pa_index_get_state": [_P, _P, _P, _P],
    "pa_index_get_info": [_P, C.POINTER(IndexInfo)],
    "pa_index_save": [_P, C.c_char_p],
    "pa_index_load": [_P, C.c_char_p],
    "pa_index_device_tables": [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                               C.POINTER(_P), C.POINTER(_P)],
    "pa_search": [_P, _P, _I64, _I32, C.POINTER(SearchOpts), _P, _P, _P, C.POINTER(SearchStats)],
    "pa_quantize_fp8_rows": [_P, _I64, _I32, _P, _P],
    "pa_select_entries_fp8": [_P, _P, _I64, _I32, _P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32, _P, _P, _P],
    "pa_server_create": [_P, C.POINTER(ServerParams), C.POINTER(_P)],
    "pa_server_submit": [_P, _P, _I32, _I32, C.c_uint64],
    "pa_server_poll": [_P, _I32, C.POINTER(ResultInfo), _P, _P, C.POINTER(_I32)],
    "pa_server_drain": [_P],
    "pa_server_stats": [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)],
    "pa_server_destroy": [_P],
    "pa_hbm_bytes": [C.POINTER(MemoryShape), _F64, _I32],
    "pa_plan_memory": [C.POINTER(MemoryShape), _I64, _P, _I32, _P, _I32, C.POINTER(_F64), C.POINTER(_I32),
                       C.POINTER(_I64)],
}
_RESTYPES = {"pa_hbm_bytes": C.c_int64}  # the others return an int32 status

_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2503_21206_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname: loaded first, it is the one
        # this library binds to as well (loaded after this library, torch finds no GPU)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        h = C.CDLL(LIB_PATH)
        h.pa_last_error.restype = C.c_char_p
        h.pa_last_error.argtypes = []
        for name, args in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = _RESTYPES.get(name, C.c_int32)
        _lib = h
    return _lib


def symbols():
    """Names of the C entry points this binding knows."""
    return ["pa_last_error", *_SIGS.keys()]


def _check(status: int):
    if status != PA_OK:
        raise PilotannError(status, lib().pa_last_error().decode())


def last_error() -> str:
    return lib().pa_last_error().decode()


def abi_version() -> int:
    return lib().pa_abi_version()


# ------------------------------------------------------------------ helpers

def _host(a, dtype):
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data_as(_P)


def _dev(t, dtype=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _torch_dtype(dt: int):
    import torch
    return {PA_F32: torch.float32, PA_F16: torch.float16, PA_BF16: torch.bfloat16}[dt]


# ------------------------------------------------------------------ stateless calls

def device_init(device: int = 0):
    _check(lib().pa_device_init(device))


def gram_f64(X, G, colsum, accumulate: bool = False, stream=None):
    import torch
    n, D = X.shape
    if tuple(G.shape) != (D, D) or tuple(colsum.shape) != (D,):
        raise ValueError("G must be [D][D] and colsum [D]")
    _check(lib().pa_gram_f64(_dev(X, torch.float32, "X"), n, D, _dev(G, torch.float64, "G"),
                             _dev(colsum, torch.float64, "colsum"), int(accumulate), _stream(stream)))


def eigh_f64(A):
    A, pa_ = _host(A, np.float64)
    D = A.shape[0]
    w = np.empty(D, dtype=np.float64)
    V = np.empty((D, D), dtype=np.float64)
    _check(lib().pa_eigh_f64(pa_, D, w.ctypes.data_as(_P), V.ctypes.data_as(_P)))
    return w, V


def fit_projection(X, d_r: int, center: bool = True):
    """SVD projection fitted on the GPU (FP64 moment) -> (V [D][d_r] fp32, evals, mean)."""
    X, px = _host(X, np.float32)
    N, D = X.shape
    V = np.empty((D, d_r), dtype=np.float32)
    w = np.empty(D, dtype=np.float64)
    mu = np.empty(D, dtype=np.float64)
    _check(lib().pa_fit_projection(px, N, D, d_r, int(center), V.ctypes.data_as(_P), w.ctypes.data_as(_P),
                                   mu.ctypes.data_as(_P)))
    return V, w, mu


def project(X, V, dtype: str = "f32", stream=None):
    import torch
    n, D = X.shape
    d_r = V.shape[1]
    if V.shape[0] != D:
        raise ValueError("V must be [D][d_r]")
    dt = DTYPES[dtype]
    Y = torch.empty((n, d_r), dtype=_torch_dtype(dt), device=X.device)
    _check(lib().pa_project(_dev(X, torch.float32, "X"), n, D, _dev(V, torch.float32, "V"), d_r, _dev(Y), dt,
                            _stream(stream)))
    return Y


def project_route(Q, V, centroids, stream=None):
    import torch
    m, D = Q.shape
    d_r = V.shape[1]
    if V.shape[0] != D or centroids.dim() != 2 or centroids.shape[1] != d_r:
        raise ValueError("V must be [D][d_r] and centroids [r][d_r]")
    Qr = torch.empty((m, d_r), dtype=torch.float32, device=Q.device)
    cl = torch.empty((m,), dtype=torch.int32, device=Q.device)
    _check(lib().pa_project_route(_dev(Q, torch.float32, "Q"), m, D, _dev(V, torch.float32, "V"), d_r,
                                  _dev(centroids, torch.float32, "centroids"), centroids.shape[0], _dev(Qr),
                                  _dev(cl), _stream(stream)))
    return Qr, cl


def sample_nodes(rowptr, nbrs, order, n_target: int, mode: str = "seed_expand"):
    rowptr, prp = _host(rowptr, np.int64)
    nbrs, pnb = _host(nbrs, np.int32)
    order, por = _host(order, np.int64)
    N = rowptr.shape[0] - 1
    mask = np.zeros(N, dtype=np.uint8)
    md = PA_SAMPLE_UNIFORM if mode == "uniform" else PA_SAMPLE_SEED_EXPAND
    _check(lib().pa_sample_nodes(N, prp, pnb, por, n_target, md, mask.ctypes.data_as(_P)))
    return mask.astype(bool)


def check_subgraph(rowptr, nbrs, mask, R: int):
    rowptr, prp = _host(rowptr, np.int64)
    nbrs, pnb = _host(nbrs, np.int32)
    mask, pm = _host(mask, np.uint8)
    _check(lib().pa_check_subgraph(rowptr.shape[0] - 1, prp, pnb, pm, R))


def pack_adjacency(rowptr, nbrs, R: int, device="cuda", stream=None):
    import torch
    rowptr, prp = _host(rowptr, np.int64)
    nbrs, pnb = _host(nbrs, np.int32)
    N = rowptr.shape[0] - 1
    adj = torch.empty((N, R), dtype=torch.int32, device=device)
    _check(lib().pa_pack_adjacency(N, prp, pnb, R, _dev(adj), _stream(stream)))
    return adj


def build_entries(P, r: int, init, iters: int = 10):
    P, pp = _host(P, np.float32)
    init, pi = _host(init, np.int32)
    n_p, d = P.shape
    buckets = np.empty((r, n_p // r), dtype=np.int32)
    cent = np.empty((r, d), dtype=np.float32)
    _check(lib().pa_build_entries(pp, n_p, d, r, pi, iters, buckets.ctypes.data_as(_P), cent.ctypes.data_as(_P)))
    return buckets, cent


def quantize_fp8_rows(X):
    """Host FP8 e4m3 encoding with one scale per row -> (codes uint8 [n][d], scales fp32 [n])."""
    X, px = _host(X, np.float32)
    n, d = X.shape
    codes = np.empty((n, d), dtype=np.uint8)
    scales = np.empty(n, dtype=np.float32)
    _check(lib().pa_quantize_fp8_rows(px, n, d, codes.ctypes.data_as(_P), scales.ctypes.data_as(_P)))
    return codes, scales


def select_entries(Qr, cluster, EV, EVnorm, EVid, E: int, metric: str = "l2", stream=None):
    """EV [r][n_b][d], EVnorm [r][n_b], EVid [r][n_b] device tensors."""
    import torch
    m, d = Qr.shape
    r, n_b = EVid.shape
    if tuple(EV.shape) != (r, n_b, d) or tuple(EVnorm.shape) != (r, n_b) or tuple(cluster.shape) != (m,):
        raise ValueError("EV [r][n_b][d], EVnorm [r][n_b] and cluster [m] must match Qr and EVid")
    ids = torch.empty((m, E), dtype=torch.int32, device=Qr.device)
    dist = torch.empty((m, E), dtype=torch.float32, device=Qr.device)
    _check(lib().pa_select_entries(_dev(Qr, torch.float32, "Qr"), _dev(cluster, torch.int32, "cluster"), m, d,
                                   _dev(EV, torch.float32, "EV"), _dev(EVnorm, torch.float32, "EVnorm"),
                                   _dev(EVid, torch.int32, "EVid"), r, n_b, E, METRICS[metric], _dev(ids),
                                   _dev(dist), _stream(stream)))
    return ids, dist


def select_entries_noalloc(Qr, cluster, EV, EVnorm, EVid, ids, dist, E: int, metric: str = "l2", stream=None):
    """pa_select_entries_noalloc: as select_entries, into caller-owned ids [m][E] int32 and
    dist [m][E] fp32 device tensors; the library allocates nothing on the device."""
    import torch
    m, d = Qr.shape
    r, n_b = EVid.shape
    if tuple(EV.shape) != (r, n_b, d) or tuple(EVnorm.shape) != (r, n_b) or tuple(cluster.shape) != (m,):
        raise ValueError("EV [r][n_b][d], EVnorm [r][n_b] and cluster [m] must match Qr and EVid")
    if tuple(ids.shape) != (m, E) or tuple(dist.shape) != (m, E):
        raise ValueError("ids and dist must be [m][E]")
    _check(lib().pa_select_entries_noalloc(_dev(Qr, torch.float32, "Qr"), _dev(cluster, torch.int32, "cluster"), m,
                                           d, _dev(EV, torch.float32, "EV"), _dev(EVnorm, torch.float32, "EVnorm"),
                                           _dev(EVid, torch.int32, "EVid"), r, n_b, E, METRICS[metric],
                                           _dev(ids, torch.int32, "ids"), _dev(dist, torch.float32, "dist"),
                                           _stream(stream)))
    return ids, dist


def select_entries_fp8(Qr, cluster, EV, EV8, EVscale, EVnorm, EVid, E: int, K: int, metric: str = "l2",
                       stream=None):
    """FP8 FES: EV8 [r][n_b][d] uint8 codes and EVscale [r][n_b] fp32 row scales, fp32 EV for re-rank."""
    import torch
    m, d = Qr.shape
    r, n_b = EVid.shape
    if tuple(EV.shape) != (r, n_b, d) or tuple(EV8.shape) != (r, n_b, d) or tuple(EVscale.shape) != (r, n_b) \
            or tuple(EVnorm.shape) != (r, n_b) or tuple(cluster.shape) != (m,):
        raise ValueError("EV, EV8 [r][n_b][d], EVscale, EVnorm [r][n_b] and cluster [m] must match")
    ids = torch.empty((m, E), dtype=torch.int32, device=Qr.device)
    dist = torch.empty((m, E), dtype=torch.float32, device=Qr.device)
    _check(lib().pa_select_entries_fp8(_dev(Qr, torch.float32, "Qr"), _dev(cluster, torch.int32, "cluster"), m, d,
                                       _dev(EV, torch.float32, "EV"), _dev(EV8, torch.uint8, "EV8"),
                                       _dev(EVscale, torch.float32, "EVscale"), _dev(EVnorm, torch.float32, "EVnorm"),
                                       _dev(EVid, torch.int32, "EVid"), r, n_b, E, K, METRICS[metric], _dev(ids),
                                       _dev(dist), _stream(stream)))
    return ids, dist


def gpu_traverse(Qr, Xr, adj, entries, ef: int, metric: str = "l2", cache_log2: int = 0, stream=None,
                 bloom_log2: int = -1, width: int = 1, efs=None):
    """Stage 1 on device tensors -> (ids [m][ef] int32, dists [m][ef] fp32, counters [m][4] int32).
    bloom_log2 >= 0 selects the Bloom-filter visited set of 2^bloom_log2 bits (0: automatic);
    width 2 expands the first two unchecked entries per step; efs [m] (device int32): a list
    size per query, with ef the largest (pa_gpu_traverse)."""
    import torch
    m, d_r = Qr.shape
    N, R = adj.shape
    dt = {torch.float32: PA_F32, torch.float16: PA_F16, torch.bfloat16: PA_BF16}[Xr.dtype]
    if tuple(Xr.shape) != (N, d_r):
        raise ValueError(f"Xr must be [{N}][{d_r}] to match adj and Qr, got {tuple(Xr.shape)}")
    if entries.dim() != 2 or entries.shape[0] != m:
        raise ValueError("entries must be [m][E]")
    if efs is not None and tuple(efs.shape) != (m,):
        raise ValueError("efs must be [m]")
    E = entries.shape[1]
    ids = torch.empty((m, ef), dtype=torch.int32, device=Qr.device)
    dist = torch.empty((m, ef), dtype=torch.float32, device=Qr.device)
    cnt = torch.empty((m, 4), dtype=torch.int32, device=Qr.device)
    if bloom_log2 < 0:
        opts = TraverseOpts(PA_VISITED_EXACT, cache_log2, width, None)
    else:
        opts = TraverseOpts(PA_VISITED_BLOOM, 0 if bloom_log2 == 0 else bloom_log2 - 5, width, None)
        if bloom_log2 != 0 and not 13 <= bloom_log2 <= 18:
            raise PilotannError(-1, "bloom_log2 must be 0 or 13..18")
    if efs is not None:
        opts.ef_dev = _dev(efs, torch.int32, "efs")
    _check(lib().pa_gpu_traverse(_dev(Qr, torch.float32, "Qr"), m, d_r, _dev(Xr, name="Xr"), dt, N,
                                 _dev(adj, torch.int32, "adj"), R, _dev(entries, torch.int32, "entries"), E, ef,
                                 METRICS[metric], C.byref(opts), _dev(ids), _dev(dist), _dev(cnt), _stream(stream)))
    return ids, dist, cnt


def gpu_traverse_ragged(Qr, Xr, adj, entries, efs, metric: str = "l2", stream=None, **kw):
    """Stage 1 with a per-query list size efs [m] (device int32) -> rows of stride max(efs)."""
    m = Qr.shape[0]
    if tuple(efs.shape) != (m,):
        raise ValueError("efs must be [m]")
    ef_max = int(efs.max().item()) if m else 1
    return gpu_traverse(Qr, Xr, adj, entries, ef_max, metric, stream=stream, efs=efs, **kw)


def cpu_stages(X, sub_adj, full_adj, Q, beam, ef_cpu: int, k: int, refine_steps: int = 2,
               metric: str = "l2", threads: int = 0):
    X, px = _host(X, np.float32)
    sub_adj, ps = _host(sub_adj, np.int32)
    full_adj, pf = _host(full_adj, np.int32)
    Q, pq = _host(Q, np.float32)
    beam, pb = _host(beam, np.int32)
    N, D = X.shape
    m = Q.shape[0]
    if sub_adj.shape[0] != N or full_adj.shape[0] != N or Q.shape[1] != D or beam.shape[0] != m:
        raise ValueError("adjacency tables need N rows, Q [m][D], beam [m][n_beam]")
    ids = np.empty((m, k), dtype=np.int64)
    dist = np.empty((m, k), dtype=np.float32)
    cnt = np.empty((m, 4), dtype=np.int32)
    _check(lib().pa_cpu_stages(px, N, D, ps, sub_adj.shape[1], pf, full_adj.shape[1], pq, m, pb, beam.shape[1],
                               ef_cpu, k, refine_steps, METRICS[metric], threads, ids.ctypes.data_as(_P),
                               dist.ctypes.data_as(_P), cnt.ctypes.data_as(_P)))
    return ids, dist, cnt


def cpu_search(X, full_adj, Q, entries, ef: int, k: int, metric: str = "l2", threads: int = 0):
    X, px = _host(X, np.float32)
    full_adj, pf = _host(full_adj, np.int32)
    Q, pq = _host(Q, np.float32)
    entries, pe = _host(entries, np.int32)
    N, D = X.shape
    m = Q.shape[0]
    if full_adj.shape[0] != N or Q.shape[1] != D or entries.shape[0] != m:
        raise ValueError("adjacency needs N rows, Q [m][D], entries [m][E]")
    ids = np.empty((m, k), dtype=np.int64)
    dist = np.empty((m, k), dtype=np.float32)
    cnt = np.empty((m, 4), dtype=np.int32)
    _check(lib().pa_cpu_search(px, N, D, pf, full_adj.shape[1], pq, m, pe, entries.shape[1], ef, k,
                               METRICS[metric], threads, ids.ctypes.data_as(_P), dist.ctypes.data_as(_P),
                               cnt.ctypes.data_as(_P)))
    return ids, dist, cnt


# ------------------------------------------------------------------ index

def memory_shape(N: int, dim: int, R_sub: int, n_pivots: int, r: int = 32, xr_dtype: str = "f16",
                 pivot_dtype: str = "f32", compact: bool = True, queries: int = 0, batch: int = 0, ef_gpu: int = 64,
                 E: int = 0, q_on_device: bool = False) -> MemoryShape:
    """The shape pa_hbm_bytes and pa_plan_memory take (fields as in include/pilotann.h)."""
    return MemoryShape(N, dim, DTYPES[xr_dtype], {"f32": PA_F32, "fp8": PA_FP8E4M3}[pivot_dtype],
                       1 if compact else 0, R_sub, n_pivots, r, queries, batch, ef_gpu, E, 1 if q_on_device else 0)


def hbm_bytes(shape: MemoryShape, rho: float, d_r: int) -> int:
    """Device bytes an index of this shape holds at sampling ratio rho and width d_r."""
    b = lib().pa_hbm_bytes(C.byref(shape), float(rho), int(d_r))
    if b < 0:
        raise PilotannError(-1, f"invalid memory shape, ratio {rho} or width {d_r}")
    return int(b)


def plan_memory(shape: MemoryShape, hbm_budget: int, rhos, d_rs):
    """(rho, d_r, bytes): the candidate pair that fits hbm_budget with the largest rho, then
    the largest d_r (memory-bounded mode)."""
    rh = np.ascontiguousarray(rhos, dtype=np.float64)
    dr = np.ascontiguousarray(d_rs, dtype=np.int32)
    rho, d, b = C.c_double(), C.c_int32(), C.c_int64()
    _check(lib().pa_plan_memory(C.byref(shape), int(hbm_budget), rh.ctypes.data_as(_P), rh.size,
                                dr.ctypes.data_as(_P), dr.size, C.byref(rho), C.byref(d), C.byref(b)))
    return rho.value, d.value, b.value


@dataclass
class IndexConfig:
    dim: int
    d_r: int
    metric: str = "l2"
    xr_dtype: str = "f32"
    r: int = 32
    refine_steps: int = 2
    threads: int = 0
    device: int = 0
    hbm_budget: int = 0
    pivot_dtype: str = "f32"  # "f32" | "fp8"
    preselect: int = 0
    compact: bool = False  # X_r and the device subgraph for the sampled nodes only


class Index:
    """Owning wrapper of pa_index; the base vectors X stay borrowed (kept alive here)."""

    def __init__(self, cfg: IndexConfig):
        self.cfg = cfg
        p = Params(cfg.dim, cfg.d_r, METRICS[cfg.metric], DTYPES[cfg.xr_dtype], cfg.r, cfg.refine_steps,
                   cfg.threads, cfg.device, cfg.hbm_budget, {"f32": PA_F32, "fp8": PA_FP8E4M3}[cfg.pivot_dtype],
                   cfg.preselect, 1 if cfg.compact else 0)
        h = C.c_void_p()
        _check(lib().pa_index_create(C.byref(p), C.byref(h)))
        self._h = h
        self._X = None
        self.n_p = 0

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pa_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, X, rowptr, nbrs):
        X, px = _host(X, np.float32)
        rowptr, prp = _host(rowptr, np.int64)
        nbrs, pnb = _host(nbrs, np.int32)
        self._X = X  # borrowed by the library until destroy
        _check(lib().pa_index_set_data(self._h, px, X.shape[0], prp, pnb))

    def fit_projection(self, center: int = -1):
        _check(lib().pa_index_fit_projection(self._h, center))

    def set_projection(self, V):
        V, pv = _host(V, np.float32)
        _check(lib().pa_index_set_projection(self._h, pv))

    def sample_nodes(self, order, n_target: int, mode: str = "seed_expand"):
        order, po = _host(order, np.int64)
        mask = np.zeros(self._X.shape[0], dtype=np.uint8)
        md = PA_SAMPLE_UNIFORM if mode == "uniform" else PA_SAMPLE_SEED_EXPAND
        _check(lib().pa_index_sample_nodes(self._h, po, n_target, md, mask.ctypes.data_as(_P)))
        return mask.astype(bool)

    def build_subgraph(self, mask, rowptr, nbrs):
        mask, pm = _host(mask, np.uint8)
        rowptr, prp = _host(rowptr, np.int64)
        nbrs, pnb = _host(nbrs, np.int32)
        _check(lib().pa_index_build_subgraph(self._h, pm, prp, pnb))

    def build_entries(self, pivot_ids, init, iters: int = 10):
        pivot_ids, pp = _host(pivot_ids, np.int32)
        init, pi = _host(init, np.int32)
        _check(lib().pa_index_build_entries(self._h, pp, pivot_ids.shape[0], pi, iters))
        self.n_p = pivot_ids.shape[0]

    def info(self):
        inf = IndexInfo()
        _check(lib().pa_index_get_info(self._h, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in inf._fields_}

    def save(self, path: str):
        """Write the built index (projection, reduced vectors, subgraph, entry table) to path."""
        _check(lib().pa_index_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Replace projection, subgraph and entries with a checkpoint written by save()."""
        _check(lib().pa_index_load(self._h, os.fsencode(path)))
        self.n_p = self.info()["n_pivots"]

    def projection(self):
        V = np.empty((self.cfg.dim, self.cfg.d_r), dtype=np.float32)
        _check(lib().pa_index_get_state(self._h, V.ctypes.data_as(_P), None, None))
        return V

    def state(self):
        r, d_r, D = self.cfg.r, self.cfg.d_r, self.cfg.dim
        V = np.empty((D, d_r), dtype=np.float32)
        b = np.empty((r, self.n_p // r), dtype=np.int32)
        c = np.empty((r, d_r), dtype=np.float32)
        _check(lib().pa_index_get_state(self._h, V.ctypes.data_as(_P), b.ctypes.data_as(_P), c.ctypes.data_as(_P)))
        return V, b, c

    def device_tables(self):
        ptrs = [_P() for _ in range(7)]
        _check(lib().pa_index_device_tables(self._h, *[C.byref(p) for p in ptrs]))
        names = ["Xr", "adj", "V", "centroids", "EV", "EVnorm", "EVid"]
        return {n: (p.value or 0) for n, p in zip(names, ptrs)}

    def search(self, Q, k: int, ef_gpu: int, ef_cpu: int = 0, E: int = 0, batch: int = 0, stage_mask: int = 0,
               cache_log2: int = 0, threads: int = 0, with_counters: bool = False, handoff: int = 0,
               Q_dev=None, bloom: bool = False, width: int = 1, fixed_entries: bool = False,
               serial: bool = False):
        """Q_dev: optional torch tensor on the index's device holding the same [m][dim] fp32
        queries as Q; the GPU stage then reads them from HBM instead of uploading Q.
        bloom: stage 1 tracks visited nodes in the paper's Bloom filter (32 << cache_log2
        bits) instead of the exact set.  width 2: stage 1 expands two entries per step.
        fixed_entries: no entry selection, the same predefined pivots for every query.
        serial: the host stages wait for the GPU stage of every sub-batch (no pipelining)."""
        Q, pq = _host(Q, np.float32)
        m = Q.shape[0]
        if Q.ndim != 2 or Q.shape[1] != self.cfg.dim:
            raise ValueError(f"queries must be [m][{self.cfg.dim}]")
        qd = None
        if Q_dev is not None:
            import torch
            if (not Q_dev.is_cuda or Q_dev.dtype != torch.float32 or tuple(Q_dev.shape) != Q.shape
                    or not Q_dev.is_contiguous()):
                raise ValueError("Q_dev must be a contiguous float32 device tensor shaped like Q")
            torch.cuda.current_stream(Q_dev.device).synchronize()  # its writes are complete
            qd = Q_dev.data_ptr()
        ids = np.empty((m, k), dtype=np.int64)
        dist = np.empty((m, k), dtype=np.float32)
        cnt = np.empty((m, 8), dtype=np.int32) if with_counters else None
        opts = SearchOpts(ef_gpu, ef_cpu, E, batch, stage_mask, cache_log2, threads, handoff, qd, 1 if bloom else 0,
                          width, 1 if fixed_entries else 0, 1 if serial else 0)
        st = SearchStats()
        _check(lib().pa_search(self._h, pq, m, k, C.byref(opts), ids.ctypes.data_as(_P), dist.ctypes.data_as(_P),
                               cnt.ctypes.data_as(_P) if cnt is not None else None, C.byref(st)))
        return ids, dist, cnt, st.as_dict()


class Server:
    """Continuous-batching server over a built Index (see pa_server_* in the header)."""

    def __init__(self, index: Index, hbm_budget: int, max_batch: int = 0, streams: int = 0, threads: int = 0,
                 max_k: int = 128):
        self.index = index
        self.dim = index.cfg.dim
        self.max_k = max_k
        p = ServerParams(hbm_budget, max_batch, streams, threads, max_k)
        h = C.c_void_p()
        _check(lib().pa_server_create(index._h, C.byref(p), C.byref(h)))
        self._h = h

    def submit(self, q, k: int, ef: int, tag: int):
        q, pq = _host(q, np.float32)
        if q.shape != (self.dim,):
            raise ValueError(f"query must be [{self.dim}]")
        _check(lib().pa_server_submit(self._h, pq, k, ef, tag))

    def poll(self, max_results: int = 4096):
        info = (ResultInfo * max(1, max_results))()
        ids = np.empty((max(1, max_results), self.max_k), dtype=np.int64)
        dist = np.empty((max(1, max_results), self.max_k), dtype=np.float32)
        n = C.c_int32(0)
        _check(lib().pa_server_poll(self._h, max_results, info, ids.ctypes.data_as(_P), dist.ctypes.data_as(_P),
                                    C.byref(n)))
        out = []
        for i in range(n.value):
            r = info[i]
            out.append({"tag": r.tag, "k": r.k, "ef": r.ef, "t_submit_us": r.t_submit_us,
                        "t_admit_us": r.t_admit_us, "t_done_us": r.t_done_us,
                        "ids": ids[i, :r.k].copy(), "dists": dist[i, :r.k].copy()})
        return out

    def drain(self):
        _check(lib().pa_server_drain(self._h))

    def stats(self):
        v = [C.c_int64() for _ in range(5)]
        _check(lib().pa_server_stats(self._h, *[C.byref(x) for x in v]))
        return dict(zip(["submitted", "completed", "batches", "max_batch", "bytes_in_flight"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().pa_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
