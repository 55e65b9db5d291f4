"""Seeded synthetic workloads.

This module only draws random inputs (numpy PCG64); it holds none of the
clustering method's arithmetic and imports nothing else from this package, so
both the GPU path's tests and the CPU oracle's tests can take their inputs from
it.  Every generator returns a C-contiguous float32 array of shape (n, d) whose
rows are randomly permuted (so vertex 0, the root of the tree, is a random
point).

Workloads (the paper's experiments use UCI data and random Gaussian data of
d = 5 and d = 40, Sec. 4.2; the shapes below stand in for them):

  gaussian_mixture_iso : C1-style, isotropic Gaussian blobs + uniform outliers.
  gaussian_mixture_aniso : C2-style, axis-aligned anisotropic blobs, Dirichlet
                           cluster sizes.
  image_like : C3-style, nonnegative 28x28 "images" quantised to 256 levels and
               stored as q/256 (exactly representable in bfloat16).
  sparse_communities : C4-style, 1 % nonzeros per row, lognormal values, 50
                       communities sharing support sets, stored dense.
  blobs128 : C5-style, 16 isotropic blobs in d = 128.
"""
from __future__ import annotations

import numpy as np

CONFIG_SEED_BASE = 1000

# name, n, d, k of the five standard workloads
CONFIGS = {
    1: dict(name="gmm-iso-n2000-d16", n=2000, d=16, k=5),
    2: dict(name="gmm-aniso-n50000-d64", n=50_000, d=64, k=20),
    3: dict(name="image-like-n200000-d784", n=200_000, d=784, k=10),
    4: dict(name="sparse-comm-n100000-d4096", n=100_000, d=4096, k=50),
    5: dict(name="blobs-n20000-d128", n=20_000, d=128, k=16),
}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _finish(X, rng):
    X = X[rng.permutation(X.shape[0])]
    return np.ascontiguousarray(X, dtype=np.float32)


def gaussian_mixture_iso(n=2000, d=16, n_clusters=5, outlier_frac=0.02, box=10.0, std=1.0, seed=1001):
    rng = _rng(seed)
    n_out = int(round(n * outlier_frac))
    n_in = n - n_out
    means = rng.uniform(-box, box, size=(n_clusters, d))
    lab = rng.integers(0, n_clusters, size=n_in)
    X_in = means[lab] + std * rng.standard_normal((n_in, d))
    lo, hi = X_in.min(axis=0), X_in.max(axis=0)
    X_out = rng.uniform(lo, hi, size=(n_out, d))
    return _finish(np.vstack([X_in, X_out]), rng)


def gaussian_mixture_aniso(n=50_000, d=64, n_clusters=20, box=20.0, std_lo=0.5, std_hi=2.0, seed=1002):
    rng = _rng(seed)
    props = rng.dirichlet(np.ones(n_clusters))
    sizes = rng.multinomial(n, props)
    means = rng.uniform(-box, box, size=(n_clusters, d))
    stds = rng.uniform(std_lo, std_hi, size=(n_clusters, d))
    parts = [means[c] + stds[c] * rng.standard_normal((sizes[c], d)) for c in range(n_clusters) if sizes[c]]
    return _finish(np.vstack(parts), rng)


def image_like(n=200_000, side=28, n_centres=10, noise=0.1, seed=1003):
    """Nonnegative image-like rows, values q/256 with q in 0..255."""
    rng = _rng(seed)
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    centres = np.zeros((n_centres, side * side))
    for c in range(n_centres):
        img = np.zeros((side, side))
        for _ in range(int(rng.integers(3, 7))):
            amp = rng.uniform(0.5, 1.0)
            width = rng.uniform(2.0, 4.0)
            cy, cx = rng.uniform(0, side, size=2)
            img += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * width * width))
        img = np.clip(img, 0.0, 1.0)
        img[img < 0.1] = 0.0
        centres[c] = img.ravel()
    lab = rng.integers(0, n_centres, size=n)
    X = np.empty((n, side * side), np.float32)
    chunk = 20_000
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        base = centres[lab[s:e]]
        x = np.clip(base * (1.0 + noise * rng.standard_normal(base.shape)), 0.0, 1.0)
        q = np.rint(255.0 * x)
        X[s:e] = (q / 256.0).astype(np.float32)
    return _finish(X, rng)


def sparse_communities(n=100_000, d=4096, n_comm=50, density=0.01, p_in=0.8, seed=1004):
    rng = _rng(seed)
    nnz = max(1, int(round(d * density)))
    supports = np.stack([rng.choice(d, size=nnz, replace=False) for _ in range(n_comm)])
    comm = rng.integers(0, n_comm, size=n)
    X = np.zeros((n, d), np.float32)
    chunk = 10_000
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        inside = rng.random((m, nnz)) < p_in
        pick = rng.integers(0, nnz, size=(m, nnz))
        cols_in = supports[comm[s:e]][np.arange(m)[:, None], pick]
        cols_out = rng.integers(0, d, size=(m, nnz))
        cols = np.where(inside, cols_in, cols_out)
        vals = rng.lognormal(0.0, 1.0, size=(m, nnz)).astype(np.float32)
        rows = np.repeat(np.arange(s, e), nnz)
        X[rows, cols.ravel()] = vals.ravel()
    return _finish(X, rng)


def blobs128(n=20_000, d=128, n_clusters=16, box=15.0, std=1.0, seed=1005):
    rng = _rng(seed)
    means = rng.uniform(-box, box, size=(n_clusters, d))
    lab = rng.integers(0, n_clusters, size=n)
    return _finish(means[lab] + std * rng.standard_normal((n, d)), rng)


def config(i: int, n: int | None = None, seed: int | None = None) -> np.ndarray:
    """Points of workload ``i`` (1..5), optionally at a smaller n with the same recipe."""
    c = CONFIGS[i]
    n = c["n"] if n is None else int(n)
    seed = CONFIG_SEED_BASE + i if seed is None else seed
    if i == 1:
        return gaussian_mixture_iso(n=n, d=c["d"], seed=seed)
    if i == 2:
        return gaussian_mixture_aniso(n=n, d=c["d"], seed=seed)
    if i == 3:
        return image_like(n=n, seed=seed)
    if i == 4:
        return sparse_communities(n=n, d=c["d"], seed=seed)
    if i == 5:
        return blobs128(n=n, d=c["d"], seed=seed)
    raise KeyError(i)


# ---------------------------------------------------------------- edge cases

def collinear(n=64, seed=7, dyadic=True):
    """Points on the line through direction (3, 4, 0) (tree = path, maximal
    depth).  With dyadic positions every distance is 5 * |dpos|, exact in FP32
    and FP64."""
    rng = _rng(seed)
    if dyadic:
        pos = np.cumsum(rng.integers(1, 9, size=n)).astype(np.float64) / 8.0
    else:
        pos = np.cumsum(rng.uniform(0.5, 1.5, size=n))
    X = np.zeros((n, 3))
    X[:, 0] = 3.0 * pos
    X[:, 1] = 4.0 * pos
    return _finish(X, rng)


def lattice(side=8, dim=2, seed=11):
    """Integer grid: every nearest-neighbour distance ties at 1."""
    rng = _rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(side)] * dim, indexing="ij"), -1).reshape(-1, dim)
    return _finish(g.astype(np.float64), rng)


def with_duplicates(n=200, d=5, n_dup=20, seed=13):
    """Random points where ``n_dup`` rows repeat earlier rows exactly (D = 0 ties)."""
    rng = _rng(seed)
    X = rng.standard_normal((n, d))
    src = rng.integers(0, n - n_dup, size=n_dup)
    X[n - n_dup:] = X[src]
    return _finish(X, rng)


def star_points(m=50, d=4, seed=17):
    """A centre and m points on a sphere around it: the MST is (nearly) a star."""
    rng = _rng(seed)
    v = rng.standard_normal((m, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    X = np.vstack([np.zeros((1, d)), v * (1.0 + 0.01 * rng.random((m, 1)))])
    return _finish(X, rng)


def uniform(n=100, d=3, seed=19):
    rng = _rng(seed)
    return _finish(rng.random((n, d)), rng)
