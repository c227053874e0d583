"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and builds point clouds, label sets and
test vectors.  It holds none of the method's arithmetic (no kernel sums, no
Laplacians, no eigen-solves, no Allen--Cahn steps), so both the CPU oracle and
the GPU library can be fed from it without sharing any method code.

Random numbers come from numpy's Philox4x32-10 bit generator (a counter-based
generator, Salmon et al., SC'11), seeded per purpose:

    base seed   = 1000 + config id
    labels      = base + 100
    Lanczos     = base + 200
    test vecs   = base + 300

The paper's own datasets (beach images, Pavia Center, the small multilayer
sets of its Table 1) are not available; the generators below stand in for them
with the same shapes, sizes and kinds of structure (clustered colour values,
dense pixel grids, many two-band layers).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1000
SEED_LABELS = 100
SEED_LANCZOS = 200
SEED_VECTORS = 300


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


# ----------------------------------------------------------------------------
# generic pieces
# ----------------------------------------------------------------------------
def gaussian_mixture(n: int, d: int, comps: int, std: float, seed: int,
                     mean_low=0.0, mean_high=1.0):
    """Isotropic Gaussian mixture with equal weights.  Returns (points n x d,
    component id per point)."""
    g = rng(seed)
    means = g.uniform(mean_low, mean_high, size=(comps, d))
    cls = g.integers(0, comps, size=n)
    pts = means[cls] + std * g.standard_normal((n, d))
    return np.ascontiguousarray(pts), cls.astype(np.int32)


def uniform_ball(n: int, d: int, radius: float, seed: int):
    """n points uniform in a d-ball: radius R*U^(1/d), direction from a
    normalised Gaussian draw."""
    g = rng(seed)
    v = g.standard_normal((n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radius * g.uniform(0.0, 1.0, size=n) ** (1.0 / d)
    return np.ascontiguousarray(v * r[:, None])


def circle_points(n: int, radius: float, d: int = 2, phase: float = 0.0):
    """n points equally spaced on a circle in the first two coordinates."""
    t = 2.0 * np.pi * (np.arange(n) + phase) / n
    p = np.zeros((n, d))
    p[:, 0] = radius * np.cos(t)
    p[:, 1] = radius * np.sin(t)
    return p


def median_pairwise_distance(points: np.ndarray, samples: int, seed: int) -> float:
    """Median of all pair distances among `samples` distinct nodes drawn
    uniformly (the kernel-width recipe of the image workload).  With an even
    number of pairs the median is the mean of the two middle order
    statistics."""
    g = rng(seed)
    n = points.shape[0]
    idx = g.choice(n, size=min(samples, n), replace=False)
    s = points[idx]
    diff = s[:, None, :] - s[None, :, :]
    dist = np.sqrt((diff ** 2).sum(-1))
    iu = np.triu_indices(len(idx), k=1)
    return float(np.median(dist[iu]))


def label_set(n: int, classes: np.ndarray, fraction: float, seed: int):
    """round(fraction*n) distinct nodes, uniform, carry their class; all
    others are -1 (unlabelled)."""
    g = rng(seed)
    cnt = int(round(fraction * n))
    idx = g.choice(n, size=cnt, replace=False)
    lab = np.full(n, -1, dtype=np.int32)
    lab[idx] = classes[idx]
    return lab


def test_vectors(n: int, b: int, seed: int):
    """n x b column-major (Fortran order) N(0,1) block."""
    g = rng(seed)
    return np.asfortranarray(g.standard_normal((n, b)))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config1(n: int = 2000):
    """Plain single-layer case: 5-component GMM in R^3, std 0.05, sigma 0.1."""
    base = SEED_BASE + 1
    pts, cls = gaussian_mixture(n, 3, 5, 0.05, base)
    return dict(name="gmm3d_n%d" % n, n=n, layers=[pts], sigma=[0.1], classes=cls,
                m=5, label_fraction=0.02, k=10, base_seed=base)


def config2(n: int = 100_000):
    """Single layer, uniform 3-D ball of radius 0.25, sigma 0.05."""
    base = SEED_BASE + 2
    pts = uniform_ball(n, 3, 0.25, base)
    return dict(name="ball3d_n%d" % n, n=n, layers=[pts], sigma=[0.05], classes=None,
                k=20, N=64, m_nfft=6, eps_B=1.0 / 16, base_seed=base)


def synthetic_image(h: int, w: int, seed: int, ellipses: int = 7, noise: float = 0.02):
    """Background plus `ellipses` random ellipses painted in order (8 regions
    for 7 ellipses).  Centres U[0,max)^2, semi-axes U[60,300] px scaled to
    the image size, angle U[0,pi); region RGB means U[0.1,0.9]^3; N(0,noise)
    per channel.  Returns (rgb h x w x 3, region id h x w)."""
    g = rng(seed)
    scale = min(h, w) / 1000.0
    region = np.zeros((h, w), dtype=np.int32)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    for e in range(ellipses):
        cy, cx = g.uniform(0, h), g.uniform(0, w)
        a, bax = g.uniform(60, 300, size=2) * scale
        ang = g.uniform(0, np.pi)
        c, s = np.cos(ang), np.sin(ang)
        u = (xx - cx) * c + (yy - cy) * s
        v = -(xx - cx) * s + (yy - cy) * c
        inside = (u / a) ** 2 + (v / bax) ** 2 <= 1.0
        region[inside] = e + 1
    means = g.uniform(0.1, 0.9, size=(ellipses + 1, 3))
    rgb = means[region] + noise * g.standard_normal((h, w, 3))
    return rgb, region


def box_mean3x3(img: np.ndarray) -> np.ndarray:
    """3x3 box mean with clamped (replicated) edges, per channel."""
    p = np.pad(img, ((1, 1), (1, 1), (0, 0)), mode="edge")
    h, w = img.shape[:2]
    acc = np.zeros_like(img)
    for dy in range(3):
        for dx in range(3):
            acc += p[dy:dy + h, dx:dx + w]
    return acc / 9.0


def config3(h: int = 1000, w: int = 1000):
    """Image-like three-layer graph: RGB (d=3), pixel xy (d=2), 3x3 mean RGB
    (d=3); sigma per layer = median pairwise distance of 1000 samples."""
    base = SEED_BASE + 3
    rgb, region = synthetic_image(h, w, base)
    n = h * w
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    l_rgb = np.ascontiguousarray(rgb.reshape(n, 3))
    l_xy = np.ascontiguousarray(np.stack([xx.ravel(), yy.ravel()], axis=1))
    l_mean = np.ascontiguousarray(box_mean3x3(rgb).reshape(n, 3))
    layers = [l_rgb, l_xy, l_mean]
    sig = [median_pairwise_distance(L, 1000, base + 10 + t) for t, L in enumerate(layers)]
    return dict(name="image%dx%d_3layer" % (h, w), n=n, layers=layers, sigma=sig,
                classes=region.ravel().astype(np.int32), m=8, label_fraction=0.01,
                k=20, N=64, m_nfft=5, eps_B=1.0 / 16, p_reg=5, base_seed=base)


def config4(h: int = 512, w: int = 512, bands: int = 104, layers: int = 52):
    """Hyperspectral-like cube: 6 smooth endmembers (sum of 3 Gaussian bumps
    over the band index, + 0.05), Dirichlet(1) abundances per pixel, N(0,0.01)
    noise; band pairs (i, i+52) form 52 two-dimensional layers, each with its
    own sigma and grid size N_t = (32, 64, 128)[t mod 3]."""
    base = SEED_BASE + 4
    g = rng(base)
    band = np.arange(bands, dtype=np.float64)
    E = np.full((6, bands), 0.05)
    for e in range(6):
        for _ in range(3):
            c = g.uniform(0, bands)
            wd = g.uniform(8, 30)
            amp = g.uniform(0.2, 1.0)
            E[e] += amp * np.exp(-0.5 * ((band - c) / wd) ** 2)
    n = h * w
    ab = g.exponential(1.0, size=(n, 6))
    ab /= ab.sum(1, keepdims=True)
    cube = ab @ E + 0.01 * g.standard_normal((n, bands))
    half = bands // 2
    Ls = [np.ascontiguousarray(cube[:, [i, i + half]]) for i in range(layers)]
    sig = [median_pairwise_distance(L, 1000, base + 10 + t) for t, L in enumerate(Ls)]
    Ns = [(32, 64, 128)[t % 3] for t in range(layers)]
    return dict(name="hyperspectral%dx%d_%dlayer" % (h, w, layers), n=n, layers=Ls,
                sigma=sig, N=Ns, classes=np.argmax(ab, axis=1).astype(np.int32), m=6,
                base_seed=base)


def config5(n: int = 10_000_000, layers: int = 3, comps: int = 10):
    """Large scale: 3 layers of d=3 in torus units; node class c_i from 10
    components; layer-t coordinates mu_{t,c_i} + 0.03 N(0,I) with means
    uniform in a ball of radius 0.15; points beyond radius 0.21875 are
    redrawn."""
    base = SEED_BASE + 5
    g = rng(base)
    cls = g.integers(0, comps, size=n).astype(np.int32)
    Ls = []
    for t in range(layers):
        mu = uniform_ball(comps, 3, 0.15, base + 20 + t)
        pts = mu[cls] + 0.03 * g.standard_normal((n, 3))
        bad = np.linalg.norm(pts, axis=1) > 0.21875
        while bad.any():
            idx = np.nonzero(bad)[0]
            pts[idx] = mu[cls[idx]] + 0.03 * g.standard_normal((len(idx), 3))
            bad[idx] = np.linalg.norm(pts[idx], axis=1) > 0.21875
        Ls.append(np.ascontiguousarray(pts))
    return dict(name="gmm3d_n%d_%dlayer" % (n, layers), n=n, layers=Ls,
                sigma=[0.02] * layers, classes=cls, m=10, label_fraction=0.005,
                k=30, N=128, m_nfft=8, base_seed=base)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
