"""Seeded synthetic COO tensors and factor matrices.

This module only draws random inputs: coordinates, values and factor
matrices. It holds none of the MTTKRP or CP arithmetic, and both the FP64
oracle and the HIP path take their inputs from it.

Shapes follow the power-law workloads the suite measures (its Table 3 of
real tensors, Section 6): third- and fourth/fifth-order tensors with
densities between 1e-2 and 1e-14 and a few very heavy slices.  Where the
suite used real FROSTT / HaTen2 tensors, these seeded tensors stand in for
them.

Recipe (deterministic for a given spec and seed):
  * one ``numpy.random.Generator(PCG64)`` child stream per role, spawned from
    ``SeedSequence(seed)`` in a fixed order:
    [coords mode 0..N-1, values, factors mode 0..N-1, noise, fit-init];
  * Zipf(s) modes draw a rank k in 1..I_k with P(k) proportional to k^-s
    (finite support, inverse CDF on the float64 cumulative sum) and map it
    through a seeded random permutation of 0..I_k-1;
  * uniform modes draw integers uniformly in 0..I_k-1;
  * with ``distinct=True`` coordinates are drawn in rounds and the first
    ``nnz`` distinct tuples in draw order are kept (the draw order is the
    caller order of the tensor, so it is random, not sorted);
  * values are U(0,1) or lognormal(0,1), drawn in float32 for the kept
    tuples in order; factors are N(0,1) float32, row-major I_k x R.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 1902033170

_HASH_MUL = np.uint64(0x9E3779B97F4A7C15)


@dataclass(frozen=True)
class TensorSpec:
    """How to draw one synthetic sparse tensor."""

    name: str
    dims: Tuple[int, ...]
    nnz: int
    rank: int
    # per mode: None for uniform, else the Zipf exponent s
    zipf: Tuple[Optional[float], ...] = ()
    values: str = "uniform"  # "uniform" -> U(0,1); "lognormal" -> lognormal(0,1)
    distinct: bool = True
    seed: int = BASE_SEED

    @property
    def order(self) -> int:
        return len(self.dims)

    def scaled(self, nnz: int, dims: Optional[Sequence[int]] = None, seed: Optional[int] = None) -> "TensorSpec":
        """Same recipe at another size (used for small parity cases)."""
        return replace(self, nnz=int(nnz), dims=tuple(dims) if dims is not None else self.dims,
                       seed=self.seed if seed is None else int(seed),
                       name=f"{self.name}@nnz={nnz}")


# The measured workloads. Index 1..5 keeps the numbering used throughout the
# docs (1 = small parity case, 2 = headline, 3 = order 4, 4 = CP fit on the
# coordinates of 2, 5 = order-5 hypersparse mixed precision).
CONFIGS = {
    1: TensorSpec("uniform-100x80x60", (100, 80, 60), 20_000, 16, (None, None, None), "uniform", True,
                  BASE_SEED + 1),
    2: TensorSpec("zipf1.1-50Kx40Kx30K", (50_000, 40_000, 30_000), 50_000_000, 32, (1.1, 1.1, 1.1), "uniform",
                  True, BASE_SEED + 2),
    3: TensorSpec("zipf1.2-100Kx10Kx1Kx200", (100_000, 10_000, 1_000, 200), 100_000_000, 64,
                  (1.2, 1.2, None, None), "uniform", True, BASE_SEED + 3),
    4: TensorSpec("cp-planted-50Kx40Kx30K", (50_000, 40_000, 30_000), 50_000_000, 32, (1.1, 1.1, 1.1), "uniform",
                  True, BASE_SEED + 2),
    5: TensorSpec("zipf1.1-1Mx1Mx100Kx1Kx100", (1_000_000, 1_000_000, 100_000, 1_000, 100), 200_000_000, 64,
                  (1.1,) * 5, "lognormal", True, BASE_SEED + 5),
}


@dataclass
class CooTensor:
    """A COO tensor in caller order: inds[k][m] is the mode-k index of nonzero m."""

    dims: Tuple[int, ...]
    inds: np.ndarray  # uint32 [N, nnz], C-contiguous (one row per mode)
    vals: np.ndarray  # float32 [nnz]
    spec: Optional[TensorSpec] = None
    meta: dict = field(default_factory=dict)

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])


def streams(seed: int, order: int):
    """Child generators in the fixed order documented in the module header."""
    ss = np.random.SeedSequence(int(seed))
    kids = ss.spawn(2 * order + 3)
    gens = [np.random.Generator(np.random.PCG64(k)) for k in kids]
    return {
        "coords": gens[:order],
        "values": gens[order],
        "factors": gens[order + 1: 2 * order + 1],
        "noise": gens[2 * order + 1],
        "init": gens[2 * order + 2],
    }


class _ZipfSampler:
    """Inverse-CDF sampler for P(rank k) ~ k^-s, k = 1..I (finite support).

    Returns 0-based ranks equal to ``searchsorted(cdf, u, side='right')``
    exactly; a bin table over [0,1) settles most draws without a search.
    """

    def __init__(self, size: int, s: float):
        w = np.arange(1, size + 1, dtype=np.float64) ** (-float(s))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        self.cdf = cdf
        self.size = size
        nb = 1 << max(12, min(24, int(math.ceil(math.log2(64 * size)))))
        self.nbins = nb
        edges = np.arange(nb + 1, dtype=np.float64) / nb
        # rank of any u in [b/nb, (b+1)/nb) lies in [lo[b], hi[b]]
        self.lo = np.searchsorted(cdf, edges[:-1], side="right").astype(np.int64)
        self.hi = np.searchsorted(cdf, edges[1:], side="left").astype(np.int64)

    def ranks(self, u: np.ndarray) -> np.ndarray:
        b = (u * self.nbins).astype(np.int64)  # exact: power-of-two scaling
        r = self.lo[b]
        amb = np.flatnonzero(r != self.hi[b])
        if amb.size:
            r[amb] = np.searchsorted(self.cdf, u[amb], side="right")
        np.minimum(r, self.size - 1, out=r)
        return r


def _pack_words(dims: Sequence[int]):
    """Group modes into uint64 key words, each word's cell count < 2^63."""
    words, cur, prod = [], [], 1
    for k, d in enumerate(dims):
        if cur and prod * d >= (1 << 63):
            words.append(cur)
            cur, prod = [], 1
        cur.append(k)
        prod *= d
    words.append(cur)
    return words


def _keys(coords: Sequence[np.ndarray], dims: Sequence[int]):
    out = []
    for grp in _pack_words(dims):
        key = np.zeros(coords[0].shape[0], dtype=np.uint64)
        for k in grp:
            key *= np.uint64(dims[k])
            key += coords[k].astype(np.uint64)
        out.append(key)
    return out


def first_distinct(keys: Sequence[np.ndarray], threads: int = 8) -> np.ndarray:
    """Sorted positions of the first occurrence of each distinct key tuple."""
    n = keys[0].shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    h = keys[0].copy()
    for w in keys[1:]:
        h ^= w * _HASH_MUL
    h *= _HASH_MUL
    nb = 8 if n > 1_000_000 else 1
    bucket = (h >> np.uint64(61)).astype(np.int8) if nb == 8 else np.zeros(n, np.int8)
    del h

    def one(b):
        idx = np.flatnonzero(bucket == b)
        if idx.size == 0:
            return idx
        if len(keys) == 1:
            _, fi = np.unique(keys[0][idx], return_index=True)
            return idx[fi]
        sub = [w[idx] for w in keys]
        order = np.lexsort(tuple(reversed(sub)))  # stable: draw order kept among equals
        sorted_words = [w[order] for w in sub]
        newrun = np.ones(idx.size, dtype=bool)
        same = np.ones(idx.size - 1, dtype=bool)
        for w in sorted_words:
            same &= w[1:] == w[:-1]
        newrun[1:] = ~same
        return idx[order[newrun]]

    with ThreadPoolExecutor(max(1, min(threads, nb))) as ex:
        parts = list(ex.map(one, range(nb)))
    mask = np.zeros(n, dtype=bool)
    for p in parts:
        mask[p] = True
    return np.flatnonzero(mask)


def _draw_coords(spec: TensorSpec, gens, count: int, samplers, perms):
    """One batch of coordinates; each mode draws from its own stream, so the modes
    are drawn in parallel threads with the same result as one after another."""
    def one(k):
        d, g = spec.dims[k], gens[k]
        s = spec.zipf[k] if spec.zipf else None
        if s is None:
            return g.integers(0, d, size=count, dtype=np.int64).astype(np.uint32)
        return perms[k][samplers[k].ranks(g.random(count))]

    with ThreadPoolExecutor(len(spec.dims)) as ex:
        return list(ex.map(one, range(len(spec.dims))))


def make_coo(spec: TensorSpec, threads: int = 8) -> CooTensor:
    """Draw the COO tensor of ``spec`` (caller order = draw order)."""
    N = spec.order
    dims = tuple(int(d) for d in spec.dims)
    M = int(spec.nnz)
    cells = 1
    for d in dims:
        cells *= d
    if spec.distinct and M > cells:
        raise ValueError(f"{M} distinct nonzeros do not fit in {cells} cells")
    g = streams(spec.seed, N)
    zipf = spec.zipf if spec.zipf else (None,) * N
    all_uniform = all(s is None for s in zipf)
    if M == 0:
        inds = np.zeros((N, 0), dtype=np.uint32)
    elif spec.distinct and all_uniform and cells <= 50_000_000:
        lin = g["coords"][0].choice(cells, size=M, replace=False)
        inds = np.stack([c.astype(np.uint32) for c in np.unravel_index(lin, dims)])
    else:
        perms, samplers = [], []
        for k in range(N):
            if zipf[k] is None:
                perms.append(None)
                samplers.append(None)
            else:
                perms.append(g["coords"][k].permutation(dims[k]).astype(np.uint32))
                samplers.append(_ZipfSampler(dims[k], zipf[k]))
        kept = [np.zeros(0, dtype=np.uint32) for _ in range(N)]
        have, rate = 0, 0.8
        rounds = 0
        while True:
            need = M - have
            batch = int(math.ceil(need / max(rate, 0.02) * 1.05)) + 1024 if spec.distinct else need
            batch = min(batch, 150_000_000)
            new = _draw_coords(spec, g["coords"], batch, samplers, perms)
            cat = [np.concatenate([a, b]) for a, b in zip(kept, new)]
            del new
            if spec.distinct:
                first = first_distinct(_keys(cat, dims), threads)
                got = first.size - have
                rate = max(got / batch, 1e-3)
                first = first[:M]
                kept = [c[first] for c in cat]
            else:
                kept = [c[:M] for c in cat]
            del cat
            have = kept[0].shape[0]
            rounds += 1
            if have >= M:
                break
            if rounds > 64:
                raise RuntimeError("coordinate drawing did not converge")
        inds = np.ascontiguousarray(np.stack(kept))
    if spec.values == "uniform":
        vals = g["values"].random(M, dtype=np.float32)
    elif spec.values == "lognormal":
        vals = g["values"].lognormal(0.0, 1.0, M).astype(np.float32)
    elif spec.values == "ints":  # small integers 0..7: exact in FP32 sums
        vals = g["values"].integers(0, 8, M).astype(np.float32)
    else:
        raise ValueError(spec.values)
    return CooTensor(dims, np.ascontiguousarray(inds, dtype=np.uint32), vals, spec)


GENERATOR_VERSION = 1


def load_or_make_coo(spec: TensorSpec, cache_dir: Optional[str] = None) -> CooTensor:
    """make_coo with an optional on-disk cache keyed by the spec and generator version."""
    if not cache_dir:
        return make_coo(spec)
    import hashlib
    import os
    key = hashlib.sha256(repr((spec, GENERATOR_VERSION)).encode()).hexdigest()[:20]
    base = os.path.join(cache_dir, f"coo_{key}")
    if os.path.exists(base + "_vals.npy"):
        return CooTensor(tuple(spec.dims), np.load(base + "_inds.npy"), np.load(base + "_vals.npy"), spec)
    coo = make_coo(spec)
    try:
        os.makedirs(cache_dir, exist_ok=True)
        np.save(base + "_inds.npy", coo.inds)
        np.save(base + "_vals.npy", coo.vals)
    except OSError:  # no room for the cache: drop partial files, carry on uncached
        for suffix in ("_inds.npy", "_vals.npy"):
            try:
                os.remove(base + suffix)
            except OSError:
                pass
    return coo


def make_factors(spec: TensorSpec, rank: Optional[int] = None, scale: float = 1.0):
    """N(0, scale^2) float32 factor matrices, row-major I_k x R."""
    R = spec.rank if rank is None else int(rank)
    g = streams(spec.seed, spec.order)
    return [(gk.standard_normal((d, R), dtype=np.float32) * np.float32(scale)).astype(np.float32)
            for gk, d in zip(g["factors"], spec.dims)]


def make_init(spec: TensorSpec, rank: Optional[int] = None, scale: float = 1.0):
    """Independent N(0, scale^2) draw used as the starting point of a CP fit."""
    R = spec.rank if rank is None else int(rank)
    g = streams(spec.seed, spec.order)["init"]
    return [(g.standard_normal((d, R), dtype=np.float32) * np.float32(scale)).astype(np.float32)
            for d in spec.dims]


def make_noise(spec: TensorSpec, n: int) -> np.ndarray:
    """Standard normal draws (float64) for the additive noise of a planted fit."""
    return streams(spec.seed, spec.order)["noise"].standard_normal(n)


def cp_planted_scale(rank: int, order: int) -> float:
    """Factor std so that a planted rank-R order-N CP entry has unit variance."""
    return float(rank) ** (-1.0 / (2.0 * order))


def head_block(coo: CooTensor, spec: TensorSpec, sizes: Sequence[int]) -> CooTensor:
    """Sub-tensor on the Zipf head ranks 1..sizes[k] of each mode, re-indexed 0-based.

    With Zipf modes the head ranks hold the densest block of the tensor, so
    a 30x20x10 head block of a 50Kx40Kx30K Zipf(1.1) tensor is fully dense.
    """
    g = streams(spec.seed, spec.order)
    keep = np.ones(coo.nnz, dtype=bool)
    remap = []
    for k, d in enumerate(spec.dims):
        perm = g["coords"][k].permutation(d).astype(np.uint32)
        inv = np.full(d, -1, dtype=np.int64)
        inv[perm[: sizes[k]]] = np.arange(sizes[k])
        r = inv[coo.inds[k]]
        keep &= r >= 0
        remap.append(r)
    inds = np.stack([r[keep].astype(np.uint32) for r in remap])
    return CooTensor(tuple(int(s) for s in sizes), np.ascontiguousarray(inds), coo.vals[keep].copy(), None,
                     {"parent": spec.name})

