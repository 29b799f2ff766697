"""Seeded synthetic point sets shaped like the paper's workloads.

This module only draws random inputs; it holds none of the method's
arithmetic (no distances, no thresholds, no tree).  Both the GPU path and the
CPU oracle are fed from here, so the two sides always see identical bytes.

Every generator uses ``numpy.random.default_rng(seed)`` and returns host
numpy arrays in the layout the library boundary expects:

* L2 / angular : float32 [n, dim], row-major.
* Hamming      : uint64  [n, bits // 64]  (``dim`` passed to the library = bits).
* Levenshtein  : uint8   [n, stride]; symbols < 0xFF, padded with 0xFF; the
                 string length is the index of the first 0xFF (or ``stride``).

The stand-ins replace datasets the paper uses but that are not available here
(Table I): ``c2`` stands in for the 1M x 128 Euclidean set, ``c3`` for the
256-bit Hamming set, ``c1`` for the small ~10^4-point Euclidean sets, ``c4``
for an edit-distance workload (the paper names edit distance but runs no such
experiment), ``c5`` for many independent clouds.
"""
from __future__ import annotations

import numpy as np

LEV_PAD = 0xFF


def c1_clusters(n_centers: int = 20, per_center: int = 1000, dim: int = 8,
                sigma: float = 0.05, seed: int = 1001) -> np.ndarray:
    """Isotropic Gaussian clusters: centers U[0,1]^dim, x = c + sigma*N(0,I)."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, 1.0, (n_centers, dim))
    lab = np.repeat(np.arange(n_centers), per_center)
    x = centers[lab] + sigma * rng.standard_normal((lab.size, dim))
    x = x[rng.permutation(lab.size)]
    return np.ascontiguousarray(x.astype(np.float32))


def c2_manifold(n: int = 1_000_000, seed: int = 1002, latent: int = 12,
                hidden: int = 64, dim: int = 128, noise: float = 0.01,
                chunk: int = 200_000) -> np.ndarray:
    """12-dim uniform latents through a random two-layer tanh map to 128-d.

    z ~ U[-1,1]^12; h = tanh(W1 z + b1), W1 ~ N(0, 1/12), b1 ~ N(0, 0.1^2);
    x = tanh(W2 h) + N(0, noise^2), W2 ~ N(0, 1/64).  The weights are drawn
    first, then the latents and noise chunk by chunk, so a prefix of the
    n = 10^6 set equals the smaller set drawn with the same seed.
    """
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0.0, np.sqrt(1.0 / latent), (hidden, latent))
    b1 = rng.normal(0.0, 0.1, hidden)
    w2 = rng.normal(0.0, np.sqrt(1.0 / hidden), (dim, hidden))
    out = np.empty((n, dim), dtype=np.float32)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        z = rng.uniform(-1.0, 1.0, (m, latent))
        h = np.tanh(z @ w1.T + b1)
        x = np.tanh(h @ w2.T) + rng.normal(0.0, noise, (m, dim))
        out[s:s + m] = x.astype(np.float32)
    return out


def c3_hamming(n: int = 2_000_000, n_centers: int = 4096, bits: int = 256,
               flip: float = 0.05, seed: int = 1003,
               chunk: int = 100_000) -> np.ndarray:
    """Binary codes: point i = center (i mod n_centers) with each bit flipped
    independently with probability ``flip``.  Packed little-endian into
    ``bits // 64`` uint64 words per point."""
    assert bits % 64 == 0
    rng = np.random.default_rng(seed)
    words = bits // 64
    centers = rng.integers(0, 2**64, (n_centers, words), dtype=np.uint64)
    out = np.empty((n, words), dtype=np.uint64)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        idx = (np.arange(s, s + m) % n_centers)
        flips = rng.random((m, bits)) < flip
        packed = np.packbits(flips, axis=1, bitorder="little")
        mask = packed.view(np.uint64).reshape(m, words)
        out[s:s + m] = centers[idx] ^ mask
    return out


def c4_strings(n: int = 100_000, n_seeds: int = 2000, min_len: int = 80,
               max_len: int = 120, alphabet: int = 4, p_edit: float = 0.03,
               stride: int = 128, seed: int = 1004) -> np.ndarray:
    """Strings over a 4-letter alphabet.  Point i copies seed (i mod n_seeds);
    each position is edited with probability ``p_edit``, the edit drawn
    uniformly from {substitute by a different symbol, insert a random symbol
    before it, delete it}.  Strings longer than ``stride`` are truncated."""
    rng = np.random.default_rng(seed)
    seeds = [rng.integers(0, alphabet, rng.integers(min_len, max_len + 1))
             .astype(np.uint8) for _ in range(n_seeds)]
    out = np.full((n, stride), LEV_PAD, dtype=np.uint8)
    for i in range(n):
        src = seeds[i % n_seeds]
        hit = rng.random(src.size) < p_edit
        if not hit.any():
            s = src
        else:
            kind = rng.integers(0, 3, src.size)
            sym = rng.integers(0, alphabet, src.size)
            shift = rng.integers(1, alphabet, src.size)
            res = []
            for k in range(src.size):
                c = int(src[k])
                if not hit[k]:
                    res.append(c)
                elif kind[k] == 0:      # substitute by a different symbol
                    res.append((c + int(shift[k])) % alphabet)
                elif kind[k] == 1:      # insert a random symbol before
                    res.append(int(sym[k]))
                    res.append(c)
                # kind 2: delete
            s = np.asarray(res, dtype=np.uint8)
        m = min(s.size, stride)
        out[i, :m] = s[:m]
    return out


def angular_dirs(n: int = 20_000, dim: int = 16, n_centers: int = 20,
                 spread: float = 0.15, seed: int = 1006) -> np.ndarray:
    """Directions clustered around random unit vectors, with random positive
    scales (the angular metric ignores length).  No zero rows."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n_centers, dim))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    lab = rng.integers(0, n_centers, n)
    x = c[lab] + spread * rng.standard_normal((n, dim))
    x *= rng.uniform(0.5, 2.0, (n, 1))
    return np.ascontiguousarray(x.astype(np.float32))


def c5_cloud_specs(n_clouds: int = 256, seed: int = 1005):
    """Per-cloud parameters of the many-clouds workload: size log-uniform in
    [1e3, 2e5], dim in {3, 16, 64}, 5..50 mixture components, and a target
    mean neighbour count log-uniform in [10, 300]."""
    rng = np.random.default_rng(seed)
    specs = []
    for c in range(n_clouds):
        n_c = int(round(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
        d_c = int(rng.choice([3, 16, 64]))
        k_c = int(rng.integers(5, 51))
        target = float(np.exp(rng.uniform(np.log(10.0), np.log(300.0))))
        specs.append(dict(cloud=c, n=n_c, dim=d_c, components=k_c,
                          target_nbrs=target, seed=int(rng.integers(0, 2**31))))
    return specs


def c5_cloud(spec: dict, n_override: int | None = None) -> np.ndarray:
    """One Gaussian-mixture cloud: component means U[0,1]^d, per-component
    sigma log-uniform in [0.01, 0.05], uniform labels."""
    rng = np.random.default_rng(spec["seed"])
    d, k = spec["dim"], spec["components"]
    n = spec["n"] if n_override is None else n_override
    means = rng.uniform(0.0, 1.0, (k, d))
    sig = np.exp(rng.uniform(np.log(0.01), np.log(0.05), k))
    lab = rng.integers(0, k, n)
    x = means[lab] + sig[lab, None] * rng.standard_normal((n, d))
    return np.ascontiguousarray(x.astype(np.float32))


def grid_points(k: int, dim: int) -> np.ndarray:
    """Integer lattice {0..k-1}^dim as float32 (closed-form test inputs)."""
    axes = np.meshgrid(*([np.arange(k)] * dim), indexing="ij")
    return np.ascontiguousarray(
        np.stack([a.ravel() for a in axes], axis=1).astype(np.float32))


def random_points(n: int, dim: int, seed: int, scale: float = 1.0,
                  duplicates: int = 0) -> np.ndarray:
    """Uniform points in [0, scale]^dim; the last ``duplicates`` rows copy
    earlier rows (exercises duplicate handling)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, scale, (n, dim)).astype(np.float32)
    if duplicates:
        src = rng.integers(0, n - duplicates, duplicates)
        x[n - duplicates:] = x[src]
    return np.ascontiguousarray(x)


def random_codes(n: int, bits: int, seed: int, n_centers: int = 8,
                 flip: float = 0.1) -> np.ndarray:
    """Small clustered Hamming codes for tests."""
    return c3_hamming(n=n, n_centers=n_centers, bits=bits, flip=flip,
                      seed=seed, chunk=max(1, n))


def random_strings(n: int, seed: int, n_seeds: int = 20, stride: int = 128,
                   min_len: int = 20, max_len: int = 100,
                   p_edit: float = 0.05) -> np.ndarray:
    """Small edited-string families for tests."""
    return c4_strings(n=n, n_seeds=n_seeds, min_len=min_len, max_len=max_len,
                      stride=stride, p_edit=p_edit, seed=seed)
