"""Run the oracle over many queries in worker processes.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This module holds none of the
method's arithmetic: it only spreads independent per-query oracle calls over the host
cores.  The large arrays are written once to .npy files and memory-mapped read-only by
every worker, so N x d inputs are shared through the page cache instead of being copied.
Workers are started with the "spawn" method: they begin as fresh interpreters, hold no
GPU state of the parent and import nothing but NumPy and the oracle.
"""

from __future__ import annotations

import multiprocessing as mp
import os
import shutil
import tempfile

import numpy as np

_ARRAYS: dict = {}


def host_cores() -> int:
    """Cores this process may run on (affinity), capped at 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - non-Linux
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _init(folder: str, names: list) -> None:
    _ARRAYS.clear()
    for name in names:
        _ARRAYS[name] = np.load(os.path.join(folder, name + ".npy"), mmap_mode="r")


def _call(job):
    func, item = job
    return func(_ARRAYS, item)


def map_queries(func, items, arrays: dict, procs: int | None = None, chunksize: int = 1):
    """[func(arrays, item) for item in items], computed by `procs` worker processes.

    func must be a module-level function (it is sent to the workers by reference); it
    receives the arrays as read-only memory maps and one item.  With procs == 1 the calls
    run in this process on the arrays themselves."""
    items = list(items)
    procs = host_cores() if procs is None else max(1, int(procs))
    if procs == 1 or len(items) <= 1:
        return [func(arrays, it) for it in items]
    folder = tempfile.mkdtemp(prefix="oracle_pool_")
    old = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    try:
        for name, a in arrays.items():
            np.save(os.path.join(folder, name + ".npy"), np.ascontiguousarray(a))
        for k in old:  # one BLAS thread per worker: the workers already fill the cores
            os.environ[k] = "1"
        ctx = mp.get_context("spawn")
        with ctx.Pool(min(procs, len(items)), initializer=_init, initargs=(folder, list(arrays))) as pool:
            return pool.map(_call, [(func, it) for it in items], chunksize=chunksize)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
        shutil.rmtree(folder, ignore_errors=True)
