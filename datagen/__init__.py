"""Seeded synthetic inputs shaped like the paper's cross-modal workloads.

This module only draws random numbers; it holds none of the index method's
arithmetic, so the oracle and the GPU library can both consume its outputs.

The paper evaluates on Text-to-Image (10M x 200, inner product), LAION
(10M x 512, cosine) and WebVid (2.5M x 512, cosine), each with 10K
out-of-distribution text queries and a disjoint training-query set as large
as the base (Sec. 5.1, Table 1).  None of those datasets is available here;
the generators below stand in for them with Gaussian mixtures whose query
distribution is shifted by a fixed "modality gap" vector, so queries sit far
from the base and their true neighbours are spread apart (Sec. 3).

Two laws (all draws from numpy PCG64):

Isotropic mixture (the tiny d=64 config, whose spread is given as sigma):
  * centres c_j ~ N(0, I_d), normalised to unit norm; base and query
    mixtures use independent centre sets;
  * point = c_z + sigma * g, z ~ U{0..K-1}, g ~ N(0, I_d) (each component is
    N(c_z, sigma^2 I), sigma = 0.3).

Low-rank mixture (the d=200 / d=512 configs, whose spread is not given).
Real text and image embeddings have an intrinsic dimension far below d;
both modalities live in one shared semantic subspace:
  * U = a random orthonormal d x r basis (r = 32), shared by both sets;
  * latent centres c_j ~ N(0, I_r), independent sets for base and queries;
  * h = c_z + 0.5 g_r, point = (U h + a g_d) / sqrt(r), g ~ N(0, I), with
    a = 0.6 at d = 200 and a = 0.375 at d = 512: the off-subspace noise has
    the same norm (about 1.5 / sqrt(r) of the point) at both widths, next to
    a subspace part of norm about 1.1.  At a = 0.6 and d = 512 the noise
    would be twice the signal, and normalised rows would be nearly random
    directions with no usable neighbour structure.

For both laws a query is s (.) point' + G u, with point' from the query
mixture, u a fixed random unit vector (the "modality gap", norm G) and s a
per-dimension scale (all ones unless the config says otherwise); rows are
L2-normalised when the config is a cosine workload.
Seeds: 240808933 + 1000 * config + stream, one stream per role; the rows of
a role are drawn in chunks of 65,536, chunk c from PCG64 seeded with
(seed, c), so large sets are drawn on several threads with results that do
not depend on the thread count.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import os

import numpy as np

SEED_BASE = 240808933

# stream ids, one per independent role
S_BASE_CENTRES, S_BASE_POINTS, S_QUERY_CENTRES, S_GAP, S_SCALE, S_TRAIN, S_TEST, S_REQ, S_GRAPH, S_BASIS = range(10)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    cfg: int
    d: int
    n: int
    n_train: int
    n_test: int
    k_base: int
    k_query: int
    gap: float
    normalize: bool
    query_scale: tuple | None  # (lo, hi) of a uniform per-dimension scale
    Nq: int
    M: int
    sigma: float = 0.3
    latent: int = 0          # 0: isotropic law; r > 0: low-rank law with an r-dim shared subspace
    latent_spread: float = 0.5
    ambient_noise: float = 0.6


# The five workloads (d, N, centres, gap, normalisation, build parameters).
WORKLOADS = {
    1: Workload("tiny-ood-d64", 1, 64, 10_000, 10_000, 1_000, 16, 16, 1.0, True, None, 32, 32),
    2: Workload("t2i-like-d200", 2, 200, 1_000_000, 1_000_000, 10_000, 256, 256, 1.5, False, (0.5, 1.5), 100, 64,
                latent=32),
    3: Workload("clip-like-d512", 3, 512, 2_000_000, 2_000_000, 10_000, 1024, 1024, 0.8, True, None, 100, 64,
                latent=32, ambient_noise=0.375),
    4: Workload("serve-d200-10M", 4, 200, 10_000_000, 10_000_000, 10_000, 1024, 1024, 1.5, False, (0.5, 1.5), 100,
                64, latent=32),
    5: Workload("serve-fp8-d512-8M", 5, 512, 8_000_000, 8_000_000, 10_000, 1024, 1024, 0.8, True, None, 100, 64,
                latent=32, ambient_noise=0.375),
}


def seed_for(cfg: int, stream: int) -> int:
    return SEED_BASE + 1000 * cfg + stream


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(cfg, stream)))


def _unit_rows(a: np.ndarray) -> np.ndarray:
    nrm = np.linalg.norm(a.astype(np.float64), axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return (a / nrm).astype(np.float32)


def _centres(rng, k, d):
    return _unit_rows(rng.standard_normal((k, d), dtype=np.float32))


CHUNK = 1 << 16  # rows per independently seeded chunk


def _chunk_rng(seed: int, c: int) -> np.random.Generator:
    """The generator of chunk c of a role: PCG64 seeded from (seed, c), so a
    chunk's draws do not depend on the thread that makes them or on the
    other chunks."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=(c,))))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n, d, seed, fill):
    """An n x d float32 array whose chunk c (CHUNK rows) is fill(rng_c, rows)
    with rng_c = _chunk_rng(seed, c); chunks run on a thread pool (numpy's
    generators and BLAS release the interpreter lock)."""
    out = np.empty((n, d), dtype=np.float32)

    def work(c):
        s0 = c * CHUNK
        e = min(n, s0 + CHUNK)
        out[s0:e] = fill(_chunk_rng(seed, c), e - s0)

    nchunks = (n + CHUNK - 1) // CHUNK
    if nchunks <= 1:
        for c in range(nchunks):
            work(c)
    else:
        with cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def _mixture(seed, n, centres, sigma):
    k, d = centres.shape
    scale = np.float32(sigma)

    def fill(rng, m):
        z = rng.integers(0, k, size=m)
        g = rng.standard_normal((m, d), dtype=np.float32)
        return centres[z] + scale * g

    return _chunked(n, d, seed, fill)


def _lowrank_mixture(seed, n, basis, centres, spread, noise):
    d, r = basis.shape
    inv = np.float32(1.0 / np.sqrt(r))

    def fill(rng, m):
        z = rng.integers(0, centres.shape[0], size=m)
        h = centres[z] + np.float32(spread) * rng.standard_normal((m, r), dtype=np.float32)
        x = h @ basis.T
        x += np.float32(noise) * rng.standard_normal((m, d), dtype=np.float32)
        return x * inv

    return _chunked(n, d, seed, fill)


def _normalize_inplace(a: np.ndarray):
    def work(s0):
        a[s0:s0 + CHUNK] = _unit_rows(a[s0:s0 + CHUNK])

    with cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(0, a.shape[0], CHUNK)))


class Generator:
    """Draws base / training / test / request vectors for one workload.

    Sizes can be overridden (n, n_train, n_test) to get smaller instances of
    the same law, e.g. for tests.
    """

    def __init__(self, w: Workload | int, n=None, n_train=None, n_test=None, d=None):
        if isinstance(w, int):
            w = WORKLOADS[w]
        if d is not None:
            w = dataclasses.replace(w, d=d)
        self.w = dataclasses.replace(
            w,
            n=w.n if n is None else n,
            n_train=w.n_train if n_train is None else n_train,
            n_test=w.n_test if n_test is None else n_test,
        )
        cfg, d = self.w.cfg, self.w.d
        r = self.w.latent
        if r:
            self.basis = np.linalg.qr(rng_for(cfg, S_BASIS).standard_normal((d, r)))[0].astype(np.float32)
            self.base_centres = rng_for(cfg, S_BASE_CENTRES).standard_normal((self.w.k_base, r), dtype=np.float32)
            self.query_centres = rng_for(cfg, S_QUERY_CENTRES).standard_normal((self.w.k_query, r), dtype=np.float32)
        else:
            self.basis = None
            self.base_centres = _centres(rng_for(cfg, S_BASE_CENTRES), self.w.k_base, d)
            self.query_centres = _centres(rng_for(cfg, S_QUERY_CENTRES), self.w.k_query, d)
        u = rng_for(cfg, S_GAP).standard_normal(d)
        self.gap = (self.w.gap * u / np.linalg.norm(u)).astype(np.float32)
        if self.w.query_scale is not None:
            lo, hi = self.w.query_scale
            self.scale = rng_for(cfg, S_SCALE).uniform(lo, hi, size=d).astype(np.float32)
        else:
            self.scale = np.ones(d, dtype=np.float32)

    def _points(self, seed, n, centres):
        if self.basis is not None:
            return _lowrank_mixture(seed, n, self.basis, centres, self.w.latent_spread, self.w.ambient_noise)
        return _mixture(seed, n, centres, self.w.sigma)

    def base(self) -> np.ndarray:
        x = self._points(seed_for(self.w.cfg, S_BASE_POINTS), self.w.n, self.base_centres)
        if self.w.normalize:
            _normalize_inplace(x)
        return x

    def _queries(self, seed, n):
        q = self._points(seed, n, self.query_centres)
        q *= self.scale
        q += self.gap
        if self.w.normalize:
            _normalize_inplace(q)
        return q

    def train(self) -> np.ndarray:
        return self._queries(seed_for(self.w.cfg, S_TRAIN), self.w.n_train)

    def test(self) -> np.ndarray:
        return self._queries(seed_for(self.w.cfg, S_TEST), self.w.n_test)

    def in_distribution(self, n: int) -> np.ndarray:
        """Fresh draws from the base law (ID queries), for sanity ratios."""
        x = self._points(seed_for(self.w.cfg, S_TEST + 100), n, self.base_centres)
        if self.w.normalize:
            _normalize_inplace(x)
        return x

    def requests(self, n: int, rate: float, ks=(1, 10, 100), Ls=(32, 128, 512), seed_offset=0):
        """A Poisson request stream: arrival times (s), query vectors, k, L."""
        rng = rng_for(self.w.cfg, S_REQ + 10 * seed_offset)
        t = np.cumsum(rng.exponential(1.0 / rate, size=n))
        k = rng.choice(np.asarray(ks, dtype=np.int32), size=n)
        L = rng.choice(np.asarray(Ls, dtype=np.int32), size=n)
        q = self._queries(seed_for(self.w.cfg, S_REQ + 10 * seed_offset + 5), n)
        return t, q, k, L


def random_graph(n: int, deg: int, seed: int = 0):
    """A seeded random directed graph in CSR form (int64 offsets, uint32 ids).

    Every node gets `deg` distinct out-neighbours (no self loops), and node
    i -> i+1 (mod n) is always present so every node is reachable from any
    start.  Used as a structural stand-in for an index at sizes the oracle
    cannot build.
    """
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7 + seed))
    deg = min(deg, n - 1)
    rows = []
    for s in range(0, n, 1 << 16):
        e = min(n, s + (1 << 16))
        cand = rng.integers(0, n, size=(e - s, deg + 8), dtype=np.int64)
        for r in range(e - s):
            i = s + r
            nb = [(i + 1) % n] if n > 1 else []
            seen = set(nb) | {i}
            for c in cand[r]:
                if len(nb) >= deg:
                    break
                c = int(c)
                if c not in seen:
                    seen.add(c)
                    nb.append(c)
            while len(nb) < deg:
                c = int(rng.integers(0, n))
                if c not in seen:
                    seen.add(c)
                    nb.append(c)
            rows.append(np.sort(np.asarray(nb, dtype=np.uint32)))
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(r) for r in rows])
    indices = np.concatenate(rows).astype(np.uint32) if rows else np.zeros(0, np.uint32)
    return offsets, indices


def random_graph_fast(n: int, deg: int, seed: int = 0):
    """Vectorised variant of random_graph for large n (duplicates removed, so
    rows may hold slightly fewer than `deg` ids; the ring edge is kept)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 11 + seed))
    ids = rng.integers(0, n, size=(n, deg), dtype=np.int64)
    ids[:, 0] = (np.arange(n) + 1) % n
    ids.sort(axis=1)
    keep = np.ones_like(ids, dtype=bool)
    keep[:, 1:] = ids[:, 1:] != ids[:, :-1]
    keep &= ids != np.arange(n)[:, None]
    counts = keep.sum(axis=1)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    indices = ids[keep].astype(np.uint32)
    return offsets, indices
