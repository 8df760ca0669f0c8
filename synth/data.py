"""Seeded base/query vectors and the random draws the method consumes.

Generator recipe (the same on every machine, independent of memory size):

* every stream is ``numpy.random.Generator(PCG64(SeedSequence([seed, *keys])))``;
* base/query rows are produced in fixed chunks of ``CHUNK`` rows, chunk ``c``
  drawing from its own stream ``[seed, c]`` so any row range can be
  regenerated without producing the rows before it;
* ``seed = 1000 * config + offset`` with offsets +0 base vectors, +1 queries,
  +3 node order for sampling, +4 pivots and k-means seeds, +5 arrivals,
  +6 spectral basis.

Gaussian mixtures (the 96/128-dim workloads): ``K`` equally likely components,
points = centre + N(0, I).  Flat mixtures (the 10K workload) draw centres
~ N(0, 4 I).  Nested mixtures (the 1M and 100M workloads) draw the same number of
leaf centres through a tree: level-1 centres ~ N(0, s1^2 I), each child =
parent + N(0, s_l^2 I), with branching ``levels`` and spreads ``spreads``; this
gives the multi-scale cluster structure of real embedding sets, where a flat
mixture of well separated blobs has no coarse structure at all.  Anisotropic mixtures (the
768-dim inner-product workloads, and the 96-dim L2 workload at 10^7-10^8 rows): a seeded
orthonormal basis ``B`` (QR of a Gaussian matrix, signs fixed so diag(R) > 0) and a
power-law spectrum ``lambda_i = 1 / i``; centres ``2 B diag(sqrt(lambda)) z``, points
``centre + B diag(sqrt(lambda)) eps``, then (inner-product workloads) every point scaled
to unit length.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHUNK = 1_000_000

OFF_BASE, OFF_QUERY, OFF_ORDER, OFF_PIVOT, OFF_ARRIVAL, OFF_BASIS = 0, 1, 3, 4, 5, 6


@dataclass(frozen=True)
class WorkloadSpec:
    """Shape and parameters of one synthetic workload."""

    name: str
    config: int
    n: int
    dim: int
    components: int
    queries: int
    metric: str  # "l2" | "ip"
    k: int
    degree: int
    d_r: int
    rho: float
    sample_mode: str  # "uniform" | "seed_expand"
    n_pivots: int
    ef: tuple
    kind: str = "gmm"  # "gmm" (flat) | "hgmm" (nested) | "aniso"
    unit_norm: bool = True  # aniso only: every point scaled to unit length
    centre_scale: float = 2.0  # aniso only: centres = centre_scale * B diag(sqrt(lambda)) z
    levels: tuple = ()
    spreads: tuple = ()
    r: int = 32
    xr_dtypes: tuple = ("f32",)
    pivot_dtype: str = "f32"  # "f32" | "fp8": precision of the entry pivots' scores
    extra: dict = field(default_factory=dict)

    @property
    def seed(self) -> int:
        return 1000 * self.config


SPECS = {
    "tiny": WorkloadSpec(
        name="tiny", config=1, n=10_000, dim=96, components=64, queries=1_000,
        metric="l2", k=10, degree=32, d_r=32, rho=0.25, sample_mode="uniform",
        n_pivots=256, ef=(64,), xr_dtypes=("f32",)),
    "gmm1m": WorkloadSpec(
        name="gmm1m", config=2, n=1_000_000, dim=128, components=1024,
        queries=10_000, metric="l2", k=10, degree=32, d_r=64, rho=0.25,
        sample_mode="seed_expand", n_pivots=4096,
        ef=(32, 48, 64, 96, 128, 192, 256, 384, 512), xr_dtypes=("f32", "f16"),
        kind="hgmm", levels=(8, 8, 16), spreads=(2.0, 1.0, 0.5)),
    "gmm1m_flat": WorkloadSpec(
        name="gmm1m_flat", config=2, n=1_000_000, dim=128, components=1024,
        queries=10_000, metric="l2", k=10, degree=32, d_r=64, rho=0.25,
        sample_mode="seed_expand", n_pivots=4096,
        ef=(32, 48, 64, 96, 128, 192, 256, 384, 512), xr_dtypes=("f32", "f16"), kind="gmm"),
    "aniso10m": WorkloadSpec(
        name="aniso10m", config=3, n=10_000_000, dim=768, components=1024,
        queries=10_000, metric="ip", k=10, degree=48, d_r=128, rho=0.20,
        sample_mode="seed_expand", n_pivots=65_536, ef=(32, 48, 64, 96, 128, 192, 256, 384, 512),
        kind="aniso", xr_dtypes=("bf16",), pivot_dtype="fp8"),
    "gmm100m": WorkloadSpec(
        name="gmm100m", config=4, n=100_000_000, dim=96, components=16_384,
        queries=100_000, metric="l2", k=10, degree=32, d_r=48, rho=0.25,
        sample_mode="seed_expand", n_pivots=16_384, ef=(64, 128, 256, 512),
        xr_dtypes=("f16",), kind="hgmm", levels=(16, 16, 64), spreads=(2.0, 1.0, 0.5)),
    # the 100M x 96 L2 shape with anisotropic components (power-law spectrum, not normalised)
    "aniso100m": WorkloadSpec(
        name="aniso100m", config=4, n=100_000_000, dim=96, components=16_384,
        queries=100_000, metric="l2", k=10, degree=32, d_r=48, rho=0.25,
        sample_mode="seed_expand", n_pivots=65_536, ef=(32, 48, 64, 96, 128, 192, 256, 384, 512),
        kind="aniso", unit_norm=False, centre_scale=1.0, xr_dtypes=("f16",)),
    "serve20m": WorkloadSpec(
        name="serve20m", config=5, n=20_000_000, dim=768, components=1024,
        queries=100_000, metric="ip", k=10, degree=48, d_r=128, rho=0.20,
        sample_mode="seed_expand", n_pivots=65_536, ef=(32, 48, 64, 96, 128, 192, 256, 384, 512),
        kind="aniso", xr_dtypes=("f16",)),
}


def make_rng(seed: int, *keys: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, keys...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, keys)])))


def gmm_centers(seed: int, components: int, dim: int) -> np.ndarray:
    """Mixture centres ~ N(0, 4 I) as float64 [components][dim]."""
    rng = make_rng(seed, 0x7FFF_FFFF)
    return 2.0 * rng.standard_normal((components, dim))


def nested_centers(seed: int, levels, spreads, dim: int) -> np.ndarray:
    """Leaf centres of a nested mixture, float64 [prod(levels)][dim]."""
    rng = make_rng(seed, 0x7FFF_FFFD)
    cur = np.zeros((1, dim))
    for branch, spread in zip(levels, spreads):
        kids = cur[:, None, :] + spread * rng.standard_normal((cur.shape[0], branch, dim))
        cur = kids.reshape(-1, dim)
    return cur


def _basis(seed: int, dim: int) -> np.ndarray:
    rng = make_rng(seed + OFF_BASIS, 0)
    g = rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def _aniso_model(seed: int, components: int, dim: int, centre_scale: float = 2.0):
    b = _basis(seed, dim)
    lam = 1.0 / np.arange(1, dim + 1, dtype=np.float64)
    scale = b * np.sqrt(lam)[None, :]  # B diag(sqrt(lambda))
    rng = make_rng(seed, 0x7FFF_FFFE)
    z = rng.standard_normal((components, dim))
    centres = centre_scale * z @ scale.T
    return centres, scale


def _chunk_rows(seed: int, stream_seed: int, chunk: int, n_rows: int, components: int,
                dim: int, kind: str, model, unit_norm: bool = True) -> np.ndarray:
    rng = make_rng(stream_seed, chunk)
    comp = rng.integers(0, components, size=n_rows)
    eps = rng.standard_normal((n_rows, dim))
    if kind in ("gmm", "hgmm"):
        x = model[comp] + eps
    else:
        centres, scale = model
        x = centres[comp] + eps @ scale.T
        if unit_norm:
            x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def _rows(spec: WorkloadSpec, stream_seed: int, total: int, start: int, stop: int) -> np.ndarray:
    if spec.kind == "gmm":
        model = gmm_centers(spec.seed, spec.components, spec.dim)
    elif spec.kind == "hgmm":
        model = nested_centers(spec.seed, spec.levels, spec.spreads, spec.dim)
        if model.shape[0] != spec.components:
            raise ValueError("nested levels must multiply to the component count")
    else:
        model = _aniso_model(spec.seed, spec.components, spec.dim, spec.centre_scale)
    start, stop = max(0, start), min(total, stop)
    out = np.empty((max(0, stop - start), spec.dim), dtype=np.float32)
    c0, c1 = start // CHUNK, (stop - 1) // CHUNK if stop > start else -1

    def fill(c):
        lo, hi = c * CHUNK, min(total, (c + 1) * CHUNK)
        block = _chunk_rows(spec.seed, stream_seed, c, hi - lo, spec.components, spec.dim,
                            spec.kind, model, spec.unit_norm)
        a, b = max(lo, start), min(hi, stop)
        out[a - start:b - start] = block[a - lo:b - lo]

    # chunks draw from their own streams, so their order of generation does not matter;
    # NumPy releases the interpreter lock while it fills them
    chunks = range(c0, c1 + 1)
    if len(chunks) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(16, len(chunks))) as ex:
            list(ex.map(fill, chunks))
    else:
        for c in chunks:
            fill(c)
    return out


def gmm_points(seed: int, n: int, dim: int, components: int, stream_offset: int = OFF_BASE) -> np.ndarray:
    """Gaussian-mixture rows without a WorkloadSpec (used by small tests)."""
    spec = WorkloadSpec(name="adhoc", config=0, n=n, dim=dim, components=components, queries=0,
                        metric="l2", k=10, degree=32, d_r=dim, rho=1.0, sample_mode="uniform",
                        n_pivots=32, ef=(16,))
    model = gmm_centers(seed, components, dim)
    out = np.empty((n, dim), dtype=np.float32)
    for c in range((n + CHUNK - 1) // CHUNK):
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        out[lo:hi] = _chunk_rows(seed, seed + stream_offset, c, hi - lo, components, dim, "gmm", model)
    del spec
    return out


def anisotropic_points(seed: int, n: int, dim: int, components: int,
                       stream_offset: int = OFF_BASE) -> np.ndarray:
    """Unit-norm anisotropic-mixture rows without a WorkloadSpec."""
    model = _aniso_model(seed, components, dim)
    out = np.empty((n, dim), dtype=np.float32)
    for c in range((n + CHUNK - 1) // CHUNK):
        lo, hi = c * CHUNK, min(n, (c + 1) * CHUNK)
        out[lo:hi] = _chunk_rows(seed, seed + stream_offset, c, hi - lo, components, dim, "aniso", model)
    return out


def base_vectors(spec: WorkloadSpec, start: int = 0, stop: int | None = None) -> np.ndarray:
    """Rows [start, stop) of the base set, float32 [rows][dim]."""
    stop = spec.n if stop is None else stop
    return _rows(spec, spec.seed + OFF_BASE, spec.n, start, stop)


def query_vectors(spec: WorkloadSpec, count: int | None = None) -> np.ndarray:
    """The first ``count`` queries (same mixture, independent draws)."""
    count = spec.queries if count is None else count
    return _rows(spec, spec.seed + OFF_QUERY, max(count, 1), 0, count)


def node_order(n: int, seed: int) -> np.ndarray:
    """Seeded permutation of [0, n) consumed by node sampling (int64)."""
    return make_rng(seed + OFF_ORDER, 0).permutation(n).astype(np.int64)


def pivot_choice(candidates: np.ndarray, n_pivots: int, seed: int) -> np.ndarray:
    """``n_pivots`` distinct node ids drawn uniformly from ``candidates`` (int32)."""
    cand = np.sort(np.asarray(candidates, dtype=np.int64))
    if n_pivots > cand.size:
        raise ValueError("more pivots than candidate nodes")
    idx = make_rng(seed + OFF_PIVOT, 0).choice(cand.size, size=n_pivots, replace=False)
    return cand[idx].astype(np.int32)


def kmeans_init_choice(n_pivots: int, r: int, seed: int) -> np.ndarray:
    """``r`` distinct pivot positions that seed the coarse clustering (int32)."""
    return make_rng(seed + OFF_PIVOT, 1).choice(n_pivots, size=r, replace=False).astype(np.int32)
