"""Seeded synthetic inputs (point clouds and strengths) for the FMM.

This module holds no arithmetic of the method: it only draws points and
strengths with numpy's PCG64 generator, so that the CPU oracle and the HIP
path read exactly the same bytes.  The distributions follow the paper's
experiments (uniform unit square; normal clouds and a 'layer', all rejected
into the unit square, Sec. 5.4) widened to the workloads this library is
measured on:

  uniform   uniform in [0,1)^2
  gauss10   10 Gaussian clusters, centres U[0.1,0.9]^2, sigma_c ~ U[0.01,0.05],
            equal counts, rejected into [0,1)^2
  circle    unit circle, angle U[0, 2pi), radius 1 + N(0, 1e-3)
  clusters  20 Gaussian clusters, centres U[0,1)^2, sigma_c ~ U[0.002,0.05],
            equal counts, rejected into [0,1)^2
  spiral    90% on an Archimedean spiral about (0.5, 0.5), r = 0.45 phi/phi_max,
            phi = phi_max sqrt(U), phi_max = 16 pi, plus isotropic N(0, 1e-4)
            noise; 10% uniform in [0,1)^2
  normal    N((0.5,0.5), variance 1/100) rejected into [0,1)^2 (Sec. 5.4)
  layer     x uniform, y ~ N(0.5, variance 1/100) rejected into [0,1)^2

Strengths are complex m = a + ib with a, b ~ N(0,1) i.i.d.
"""
from __future__ import annotations

import numpy as np

DISTRIBUTIONS = ("uniform", "gauss10", "circle", "clusters", "spiral", "normal", "layer")


def _reject_gaussians(rng, n, centres, sigmas):
    """Equal-count Gaussian clusters, each point redrawn until it lies in [0,1)^2."""
    k = len(centres)
    counts = np.full(k, n // k)
    counts[: n - counts.sum()] += 1
    out = np.empty((n, 2))
    pos = 0
    for c, s, cnt in zip(centres, sigmas, counts):
        pts = rng.normal(c, s, size=(cnt, 2))
        bad = ~np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        while bad.any():
            pts[bad] = rng.normal(c, s, size=(int(bad.sum()), 2))
            bad = ~np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        out[pos:pos + cnt] = pts
        pos += cnt
    return out


def _reject_fn(rng, n, draw):
    pts = draw(n)
    bad = ~np.all((pts >= 0.0) & (pts < 1.0), axis=1)
    while bad.any():
        pts[bad] = draw(int(bad.sum()))
        bad = ~np.all((pts >= 0.0) & (pts < 1.0), axis=1)
    return pts


def points(dist: str, n: int, seed: int, shape_seed: int | None = None) -> np.ndarray:
    """n points of distribution `dist` as a complex128 array (x + iy).  For
    the cluster distributions the cluster centres and widths are drawn first;
    shape_seed (default: seed) draws them from a generator of their own, so
    that an independent draw of the same distribution (the same clusters,
    other points) takes the shape seed of the first draw."""
    rng = np.random.Generator(np.random.PCG64(seed))
    srng = rng if shape_seed is None else np.random.Generator(np.random.PCG64(shape_seed))
    if dist == "uniform":
        xy = rng.random((n, 2))
    elif dist == "gauss10":
        cen = srng.uniform(0.1, 0.9, size=(10, 2))
        sig = srng.uniform(0.01, 0.05, size=10)
        xy = _reject_gaussians(rng, n, cen, sig)
    elif dist == "clusters":
        cen = srng.random((20, 2))
        sig = srng.uniform(0.002, 0.05, size=20)
        xy = _reject_gaussians(rng, n, cen, sig)
    elif dist == "circle":
        ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
        r = 1.0 + rng.normal(0.0, 1e-3, size=n)
        xy = np.stack([r * np.cos(ph), r * np.sin(ph)], axis=1)
    elif dist == "spiral":
        ns = (9 * n) // 10
        phmax = 16.0 * np.pi
        ph = phmax * np.sqrt(rng.random(ns))
        r = 0.45 * ph / phmax
        sp = np.stack([0.5 + r * np.cos(ph), 0.5 + r * np.sin(ph)], axis=1)
        sp += rng.normal(0.0, 1e-4, size=sp.shape)
        un = rng.random((n - ns, 2))
        xy = np.concatenate([sp, un])
        xy = xy[rng.permutation(n)]
    elif dist == "normal":
        xy = _reject_fn(rng, n, lambda k: rng.normal(0.5, 0.1, size=(k, 2)))
    elif dist == "layer":
        def draw(k):
            return np.stack([rng.random(k), rng.normal(0.5, 0.1, size=k)], axis=1)
        xy = _reject_fn(rng, n, draw)
    else:
        raise ValueError("unknown distribution %r" % dist)
    return np.ascontiguousarray(xy[:, 0] + 1j * xy[:, 1])


def strengths(n: int, seed: int) -> np.ndarray:
    """Complex strengths a + ib, a, b ~ N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ab = rng.standard_normal((n, 2))
    return np.ascontiguousarray(ab[:, 0] + 1j * ab[:, 1])


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices in [0, n), sorted (the error-check targets)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def pair_orders(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n truncation orders drawn uniformly from [lo, hi] (uint8), for tests of
    per-pair M2L orders."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n).astype(np.uint8)


# Training and validation draws of the learned order model: independent
# 2^20-point draws of the 20-cluster distribution (strength seed = seed + 100).
PORDER_TRAIN_SEEDS = (11, 12, 13, 14)
PORDER_VAL_SEED = 15

# The measured workloads: (name, sources, separate targets or None, seeds).
WORKLOADS = {
    "uniform10k": dict(dist="uniform", n=10_000, seed=1, mseed=101, nd=40, tgt=None),
    "uniform1M": dict(dist="uniform", n=1 << 20, seed=2, mseed=102, nd=45, tgt=("uniform", 102 + 100),
                      sel_seed=21),
    "gauss10_1M": dict(dist="gauss10", n=1 << 20, seed=3, mseed=103, nd=45, tgt=("gauss10", 103 + 100),
                       sel_seed=22),
    "circle1M": dict(dist="circle", n=1 << 20, seed=4, mseed=104, nd=45, tgt=("circle", 104 + 100),
                     sel_seed=23),
    "clusters4M": dict(dist="clusters", n=1 << 22, seed=5, mseed=105, nd=45, tgt=None, sel_seed=7),
    "spiral16M": dict(dist="spiral", n=1 << 24, seed=6, mseed=106, nd=45, tgt=None, sel_seed=8),
}


def workload(name: str, n: int | None = None):
    """(src, m, tgt) for a named workload; n overrides the size (same recipe).
    Targets of the separate-target workloads are an independent draw of the
    source distribution: the same clusters (shape seed of the sources), their
    own point seed."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else int(n)
    src = points(w["dist"], n, w["seed"])
    m = strengths(n, w["mseed"])
    tgt = None
    if w["tgt"] is not None:
        tgt = points(w["tgt"][0], n, w["tgt"][1], shape_seed=w["seed"])
    return src, m, tgt
