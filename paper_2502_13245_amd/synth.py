"""Seeded synthetic workloads for range retrieval (inputs only).

This module draws vectors and nothing else: it holds no distance, search or
radius arithmetic, so the CPU oracle and the GPU library can both be fed from
it without sharing any of the method.  Every generator is a Gaussian mixture
drawn with numpy's PCG64, with independent streams (``SeedSequence.spawn``)
for centres, per-cluster scales, cluster weights/labels, point noise and
queries.  Queries come from the same mixture as the base points.

The shapes stand in for the paper's datasets (its Table 1): BIGANN-like
uint8 d=128, DEEP-like float32 d=96 unit-norm, MSTuring-like d=100 (int8
here), Wikipedia/MSMARCO-like d=768 unit-norm.  Two knobs shape the result
count distribution towards the paper's Table 2 (most queries empty, a heavy
tail): a per-cluster scale spread ``sigma * exp(U[-spread, spread])`` and Zipf
cluster weights ``w_k ~ 1 / (k + 1) ** zipf``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    base: np.ndarray
    queries: np.ndarray
    meta: dict = field(default_factory=dict)


def _streams(seed: int, k: int = 6):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def _labels(rng, k: int, m: int, zipf: float) -> np.ndarray:
    if zipf <= 0.0:
        return rng.integers(0, k, size=m)
    w = 1.0 / np.arange(1, k + 1, dtype=np.float64) ** zipf
    w /= w.sum()
    return rng.choice(k, size=m, p=w)


def gaussian_mixture_int(n: int, nq: int, d: int, k: int, sigma: float, seed: int, *,
                         signed: bool = False, center_std: float = 30.0,
                         spread: float = 0.0, zipf: float = 0.0, chunk: int = 1 << 18,
                         name: str = "gmm-int") -> Workload:
    """uint8 (centres U[0,255]) or int8 (centres clip(N(0, center_std^2))) mixture;
    points are clip(rint(c + sigma_k z)) into the type's range."""
    r_c, r_s, r_l, r_x, r_ql, r_qx = _streams(seed)
    if signed:
        centers = np.clip(r_c.normal(0.0, center_std, size=(k, d)), -127, 127)
        lo, hi, dt = -128, 127, np.int8
    else:
        centers = r_c.uniform(0.0, 255.0, size=(k, d))
        lo, hi, dt = 0, 255, np.uint8
    scale = sigma * np.exp(r_s.uniform(-spread, spread, size=k)) if spread > 0 else np.full(k, sigma)

    def draw(m, rl, rx):
        lab = _labels(rl, k, m, zipf)
        out = np.empty((m, d), dtype=dt)
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            z = rx.standard_normal(size=(b - a, d))
            v = centers[lab[a:b]] + scale[lab[a:b], None] * z
            out[a:b] = np.clip(np.rint(v), lo, hi).astype(dt)
        return out, lab

    base, lab = draw(n, r_l, r_x)
    queries, qlab = draw(nq, r_ql, r_qx)
    meta = dict(generator="gaussian_mixture_int", n=n, nq=nq, d=d, k=k, sigma=sigma, seed=seed,
                signed=signed, center_std=center_std if signed else None, spread=spread,
                zipf=zipf, dtype=str(np.dtype(dt)))
    return Workload(name, base, queries, meta)


def gaussian_mixture_unit(n: int, nq: int, d: int, k: int, sigma: float, seed: int, *,
                          spread: float = 0.0, zipf: float = 0.0, chunk: int = 1 << 17,
                          name: str = "gmm-unit") -> Workload:
    """float32 unit-norm mixture: centres g/|g|, points normalize(c + sigma_k z)."""
    r_c, r_s, r_l, r_x, r_ql, r_qx = _streams(seed)
    g = r_c.standard_normal(size=(k, d))
    centers = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    scale = sigma * np.exp(r_s.uniform(-spread, spread, size=k)) if spread > 0 else np.full(k, sigma)
    scale = scale.astype(np.float32)

    def draw(m, rl, rx):
        # noise drawn and combined in float32 (large d x n stays affordable);
        # the unit normalisation is done in float64
        lab = _labels(rl, k, m, zipf)
        out = np.empty((m, d), dtype=np.float32)
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            v = rx.standard_normal(size=(b - a, d), dtype=np.float32)
            v *= scale[lab[a:b], None]
            v += centers[lab[a:b]]
            nrm = np.sqrt(np.einsum("ij,ij->i", v, v, dtype=np.float64))
            out[a:b] = v / nrm[:, None].astype(np.float32)
        return out, lab

    base, _ = draw(n, r_l, r_x)
    queries, _ = draw(nq, r_ql, r_qx)
    meta = dict(generator="gaussian_mixture_unit", n=n, nq=nq, d=d, k=k, sigma=sigma, seed=seed,
                spread=spread, zipf=zipf, dtype="float32")
    return Workload(name, base, queries, meta)


def latent_mixture_f32(n: int, nq: int, d: int, k: int, sigma: float, seed: int, *,
                       latent: int = 16, within: int = 10, noise: float = 0.05,
                       spread: float = 0.35, zipf: float = 1.0, unit: bool = True,
                       chunk: int = 0, name: str = "latent-f32") -> Workload:
    """float32 mixture with low intrinsic dimension, like text or image
    embeddings.  Centres lie on a `latent`-dimensional Gaussian sheet
    (c = A u, per-coordinate std 1); each cluster varies along its own
    `within`-dimensional random basis with per-coordinate std sigma_k =
    sigma exp(U[-spread, spread]), plus isotropic noise of std `noise`.
    Zipf(`zipf`) cluster sizes.  With `unit` every row is scaled to norm 1
    (in float64).  Unlike centres drawn independently on the sphere, nearby
    centres exist at every scale, so a proximity graph can be navigated."""
    ss = np.random.SeedSequence(seed).spawn(7)
    r_c, r_s, r_l, r_x, r_ql, r_qx, r_b = [np.random.default_rng(x) for x in ss]
    A = r_c.standard_normal((d, latent)) / np.sqrt(latent)
    centers = r_c.standard_normal((k, latent)) @ A.T
    scale = sigma * np.exp(r_s.uniform(-spread, spread, size=k))
    basis = r_b.standard_normal((k, d, within)) / np.sqrt(within)
    if chunk <= 0:
        chunk = max(1024, (1 << 25) // d)  # bounds the float64 work array

    def draw(m, rl, rx):
        lab = _labels(rl, k, m, zipf)
        out = np.empty((m, d), dtype=np.float32)
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            L = lab[a:b]
            z = rx.standard_normal(size=(b - a, within)) * scale[L, None]
            v = centers[L] + noise * rx.standard_normal(size=(b - a, d))
            # the within-cluster part, one product per cluster present
            order = np.argsort(L, kind="stable")
            for grp in np.split(order, np.flatnonzero(np.diff(L[order])) + 1):
                v[grp] += z[grp] @ basis[L[grp[0]]].T
            if unit:
                v /= np.linalg.norm(v, axis=1, keepdims=True)
            out[a:b] = v.astype(np.float32)
        return out

    base = draw(n, r_l, r_x)
    queries = draw(nq, r_ql, r_qx)
    meta = dict(generator="latent_mixture_f32", n=n, nq=nq, d=d, k=k, sigma=sigma, seed=seed,
                latent=latent, within=within, noise=noise, spread=spread, zipf=zipf, unit=unit,
                dtype="float32")
    return Workload(name, base, queries, meta)


def latent_mixture_u8(n: int, nq: int, d: int, k: int, sigma: float, seed: int, *,
                      latent: int = 16, center_std: float = 40.0, within: int = 10,
                      noise: float = 4.0, spread: float = 0.35, zipf: float = 1.0,
                      dense_frac: float = 0.1, dense_sigma: float = 6.0, chunk: int = 1 << 16,
                      signed: bool = False, name: str = "latent-u8") -> Workload:
    """uint8 mixture with low intrinsic dimension, like image descriptors.

    Centres lie on a `latent`-dimensional Gaussian sheet around 127.5
    (c = 127.5 + A u, per-coordinate std `center_std`); each cluster varies
    along its own `within`-dimensional random basis with per-coordinate std
    sigma_k, plus isotropic noise of std `noise`; values are rounded and
    clipped to [0, 255].  sigma_k = sigma * exp(U[-spread, spread]), except a
    `dense_frac` share of clusters that are near-duplicate groups with
    sigma_k = dense_sigma * exp(U[-0.5, 0.5]).  Zipf(`zipf`) cluster weights
    set the cluster sizes, so a few dense groups hold thousands of points.
    With `signed` the sheet is centred at 0 and values are int8 in
    [-128, 127]."""
    ss = np.random.SeedSequence(seed).spawn(7)
    r_c, r_s, r_l, r_x, r_ql, r_qx, r_b = [np.random.default_rng(x) for x in ss]
    A = r_c.standard_normal((d, latent)) * (center_std / np.sqrt(latent))
    lo, hi, mid, dt = (-128.0, 127.0, 0.0, np.int8) if signed else (0.0, 255.0, 127.5, np.uint8)
    centers = np.clip(mid + r_c.standard_normal((k, latent)) @ A.T, lo, hi)
    scale = sigma * np.exp(r_s.uniform(-spread, spread, size=k))
    dense = r_s.random(k) < dense_frac
    scale[dense] = dense_sigma * np.exp(r_s.uniform(-0.5, 0.5, size=int(dense.sum())))
    basis = r_b.standard_normal((k, d, within)) / np.sqrt(within)

    def draw(m, rl, rx):
        lab = _labels(rl, k, m, zipf)
        out = np.empty((m, d), dtype=dt)
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            L = lab[a:b]
            z = rx.standard_normal(size=(b - a, within)) * scale[L, None]
            v = centers[L] + np.einsum("ndm,nm->nd", basis[L], z)
            v += noise * rx.standard_normal(size=(b - a, d))
            out[a:b] = np.clip(np.rint(v), lo, hi).astype(dt)
        return out

    base = draw(n, r_l, r_x)
    queries = draw(nq, r_ql, r_qx)
    meta = dict(generator="latent_mixture_u8", n=n, nq=nq, d=d, k=k, sigma=sigma, seed=seed,
                latent=latent, center_std=center_std, within=within, noise=noise, spread=spread,
                zipf=zipf, dense_frac=dense_frac, dense_sigma=dense_sigma,
                dtype="int8" if signed else "uint8")
    return Workload(name, base, queries, meta)


def permutation(n: int, seed: int) -> np.ndarray:
    """Seeded insertion order for graph construction (an input, like the data)."""
    return np.random.default_rng(np.random.SeedSequence([seed, 0x5EED])).permutation(n).astype(np.int64)


def random_graph(n: int, R: int, seed: int, min_deg: int = 1) -> np.ndarray:
    """Seeded random directed graph [n, R] int32, -1 padded: each node gets a
    uniform degree in [min_deg, R] and distinct out-neighbours != itself."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x6A]))
    adj = np.full((n, R), -1, dtype=np.int32)
    deg = rng.integers(min_deg, R + 1, size=n)
    for i in range(n):
        m = min(int(deg[i]), n - 1)
        if m <= 0:
            continue
        pick = rng.choice(n - 1, size=m, replace=False)
        pick = np.where(pick >= i, pick + 1, pick)
        adj[i, :m] = pick
    return adj


def random_graph_fast(n: int, R: int, seed: int) -> np.ndarray:
    """Large seeded random R-out graph without self loops or repeated edges
    (vectorised; repeats inside a row are replaced by -1)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x6B]))
    adj = rng.integers(0, n - 1, size=(n, R), dtype=np.int64)
    adj += adj >= np.arange(n)[:, None]
    s = np.sort(adj, axis=1)
    dup_sorted = np.zeros_like(s, dtype=bool)
    dup_sorted[:, 1:] = s[:, 1:] == s[:, :-1]
    s[dup_sorted] = n  # repeats sort to the end, then become -1 padding
    s.sort(axis=1)
    s[s == n] = -1
    return s.astype(np.int32)


# ---------------------------------------------------------------------------
# the workloads used by the tests and the benchmark
# ---------------------------------------------------------------------------

def shifted_graph(n: int, R: int, seed: int, chunk: int = 1 << 20) -> np.ndarray:
    """Seeded R-out graph for very large n, generated in O(n R) vector work:
    row i lists (i + h_i + o_j) mod n with R distinct offsets o_j in
    [1, n/2) and a per-row shift h_i in [0, n/2), so h_i + o_j lies in
    [1, n - 1): no self loops and no repeated ids.  No locality at all, like
    random_graph_fast, at a fraction of its cost."""
    if n < 4 or R >= n // 2:
        raise ValueError("shifted_graph needs n >= 4 and R < n / 2")
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5A]))
    off = rng.choice(np.arange(1, n // 2, dtype=np.int64), size=R, replace=False)
    adj = np.empty((n, R), np.int32)
    for s in range(0, n, chunk):
        i = np.arange(s, min(n, s + chunk), dtype=np.int64)
        h = rng.integers(0, n // 2, size=len(i), dtype=np.int64)
        adj[s:s + len(i)] = ((i + h)[:, None] + off[None, :]) % n
    return adj


def config_small_u8(seed: int = 0) -> Workload:
    """10,000 base + 1,000 queries, d=128 uint8, 100-centre mixture (sigma 20,
    per-cluster spread exp(U[-0.3, 0.3]))."""
    w = gaussian_mixture_int(10_000, 1_000, 128, 100, 20.0, seed, spread=0.3,
                             name="u8-10k-d128")
    return w


def config_1m_u8(seed: int = 1, n: int = 1_000_000, nq: int = 10_000) -> Workload:
    """1M base + 10,000 queries, d=128 uint8, 1,000-centre mixture (sigma 25)
    with low intrinsic dimension, Zipf cluster sizes and 10% near-duplicate
    groups: most queries empty at the benchmark radius, a heavy result tail."""
    return latent_mixture_u8(n, nq, 128, 1_000, 25.0, seed, name=f"u8-{n // 1000}k-d128")


def config_1m_f32(seed: int = 2, n: int = 1_000_000, nq: int = 10_000) -> Workload:
    """1M base + 10,000 queries, d=96 float32 unit-norm embeddings: 2,000
    clusters on a 16-dimensional sheet, Zipf cluster sizes."""
    return latent_mixture_f32(n, nq, 96, 2_000, 0.35, seed, name=f"f32-{n // 1000}k-d96")


def config_10m_i8(seed: int = 4, n: int = 10_000_000, nq: int = 100_000) -> Workload:
    """10M base + 100,000 queries, d=100 int8 with low intrinsic dimension:
    10,000 clusters on a 16-dim sheet centred at 0 (per-coordinate std 30),
    Zipf cluster sizes, 10% near-duplicate groups; values clipped to int8."""
    return latent_mixture_u8(n, nq, 100, 10_000, 20.0, seed, center_std=30.0, signed=True,
                             name=f"i8-{n // 1000}k-d100")


def config_i8(seed: int = 3, n: int = 10_000_000, nq: int = 100_000) -> Workload:
    """int8 d=100, 10,000 centres clip(N(0, 30^2)), Zipf cluster weights."""
    return gaussian_mixture_int(n, nq, 100, 10_000, 12.0, seed, signed=True, center_std=30.0,
                                spread=0.3, zipf=1.0, name=f"i8-{n // 1000}k-d100")
