"""Seeded synthetic 3DGS scenes and view directions.

Inputs only: nothing here computes any step of the coding path.  The same
arrays feed the CPU oracle and the GPU library.

Scene recipe (stands in for the real 3DGS scenes of the paper's experiments,
which are not available):
  * positions: ``clusters`` centres ~ U[0,1]^3; each primitive picks one
    uniformly and adds U[-0.05, 0.05]^3;
  * band 0 (DC) RGB: a ``comps``-component isotropic Gaussian mixture, means
    ~ U[0,1]^3, sigma 0.05, equal weights, clipped to [0,1];
  * bands k = 1..15: i.i.d. Laplace(0, 0.2 / (l+1)^2) per channel, where
    l = floor(sqrt(k)) is the SH degree of the band;
  * FP64 on the host, stored as FP32.
View directions: normalised N(0, I_3) draws, FP32.
"""
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def band_degree(k):
    return int(math.isqrt(k))


def make_scene(n, clusters=32, comps=64, seed=1, degree_mix=None, small=0.0):
    """Returns (pos float32[n][3], sh float32[n][16][3]).  With degree_mix
    (probabilities of SH degree 0..3), each primitive draws its degree L and
    its bands of higher degree are replaced by U[-small, small] values
    (exact zeros for small = 0): the view-dependent colour many primitives
    barely use."""
    rng = _rng(seed)
    centres = rng.uniform(0.0, 1.0, (clusters, 3))
    which = rng.integers(0, clusters, n)
    pos = centres[which] + rng.uniform(-0.05, 0.05, (n, 3))
    means = rng.uniform(0.0, 1.0, (comps, 3))
    comp = rng.integers(0, comps, n)
    sh = np.empty((n, 16, 3), np.float64)
    sh[:, 0, :] = np.clip(means[comp] + rng.normal(0.0, 0.05, (n, 3)), 0.0, 1.0)
    for k in range(1, 16):
        scale = 0.2 / (band_degree(k) + 1) ** 2
        sh[:, k, :] = rng.laplace(0.0, scale, (n, 3))
    if degree_mix is not None:
        L = rng.choice(4, size=n, p=np.asarray(degree_mix, np.float64))
        tiny = rng.uniform(-small, small, (n, 16, 3))
        for k in range(1, 16):
            drop = band_degree(k) > L
            sh[drop, k, :] = tiny[drop, k, :]
    return pos.astype(np.float32), sh.astype(np.float32)


def make_scene_device(n, clusters=32, comps=64, seed=1, device="cuda"):
    """The same recipe drawn with torch's generator on the device, for
    workloads too large to draw on the host (the batched and served
    benchmarks).  A different random stream from make_scene: use make_scene
    wherever the oracle sees the same inputs.  Returns device tensors
    (pos float32[n][3], sh float32[n][16][3])."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f = dict(device=device, generator=g)
    centres = torch.rand((clusters, 3), dtype=torch.float64, **f)
    which = torch.randint(0, clusters, (n,), **f)
    pos = centres[which] + (torch.rand((n, 3), dtype=torch.float64, **f) - 0.5) * 0.1
    means = torch.rand((comps, 3), dtype=torch.float64, **f)
    comp = torch.randint(0, comps, (n,), **f)
    sh = torch.empty((n, 16, 3), dtype=torch.float32, device=device)
    dc = means[comp] + torch.randn((n, 3), dtype=torch.float64, **f) * 0.05
    sh[:, 0, :] = dc.clamp_(0.0, 1.0).float()
    for k in range(1, 16):
        scale = 0.2 / (band_degree(k) + 1) ** 2
        u = torch.rand((n, 3), dtype=torch.float64, **f) - 0.5   # Laplace by inverse CDF
        sh[:, k, :] = (-scale * torch.sign(u) * torch.log1p(-2.0 * u.abs())).float()
    return pos.float().contiguous(), sh


def make_opacity(n, seed=1):
    """float32[n] opacities in (0, 1]: a mix of nearly opaque primitives,
    faint ones and a uniform middle, the spread a trained scene shows."""
    rng = _rng(seed + 104729)
    kind = rng.random(n)
    a = np.where(kind < 0.45, 1.0 - 0.1 * rng.random(n),
                 np.where(kind < 0.7, 0.05 * rng.random(n) + 1e-3, rng.random(n) * 0.999 + 1e-3))
    return a.astype(np.float32)


def make_dirs(v, seed=1):
    """float32[v][3] unit view directions."""
    rng = _rng(seed + 7919)
    d = rng.normal(0.0, 1.0, (v, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d.astype(np.float32)


def make_tiles(pos, view, tiles_x, tiles_y, seed=1, sigma=(1.5, 24.0), fov=60.0):
    """What a tile rasteriser's front end hands to its colour stage, drawn
    synthetically: per primitive a projected footprint (pixel-space mean and
    the conic a, b, c of a 2D Gaussian) and, per 16x16-pixel tile, the
    primitives whose 3-sigma box meets the tile, ordered front to back by the
    distance of their positions to ``view`` (ties by index).  The mean is the
    primitive's position seen by a pinhole camera at ``view`` looking at the
    scene centre (0.5, 0.5, 0.5) with a ``fov``-degree horizontal field over
    the image (primitives behind the camera, or whose 3-sigma box misses the
    image, are in no list), so a tile's primitives come from one region of the
    scene as a rasteriser's do; the footprint's standard deviations are
    log-uniform in ``sigma`` px at a uniform rotation.  Returns float32
    foot[n][5] (mx, my, a, b, c), uint32 tile_start[tiles + 1], uint32 lst
    (primitive ids; tile t = ty * tiles_x + tx)."""
    rng = _rng(seed + 15485863)
    n = pos.shape[0]
    W, H = 16 * tiles_x, 16 * tiles_y
    f = np.asarray(view, np.float64)
    fwd = np.array([0.5, 0.5, 0.5]) - f
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, [0.0, 1.0, 0.0])
    right = right / np.linalg.norm(right) if np.linalg.norm(right) > 1e-9 else np.array([1.0, 0.0, 0.0])
    up = np.cross(right, fwd)
    rel = pos.astype(np.float64) - f[None, :]
    z = rel @ fwd
    focal = 0.5 * W / math.tan(math.radians(fov) / 2)
    zs = np.where(z > 1e-6, z, 1.0)
    mx = np.where(z > 1e-6, 0.5 * W + focal * (rel @ right) / zs, -1e9)
    my = np.where(z > 1e-6, 0.5 * H - focal * (rel @ up) / zs, -1e9)
    mx = np.clip(mx, -1e7, 1e7)
    my = np.clip(my, -1e7, 1e7)
    s1 = np.exp(rng.uniform(math.log(sigma[0]), math.log(sigma[1]), n))
    s2 = np.exp(rng.uniform(math.log(sigma[0]), math.log(sigma[1]), n))
    th = rng.uniform(0.0, math.pi, n)
    c, s = np.cos(th), np.sin(th)
    # covariance R diag(s1^2, s2^2) R^T, conic = its inverse
    sxx = c * c * s1 * s1 + s * s * s2 * s2
    syy = s * s * s1 * s1 + c * c * s2 * s2
    sxy = c * s * (s1 * s1 - s2 * s2)
    det = sxx * syy - sxy * sxy
    foot = np.stack([mx, my, syy / det, -sxy / det, sxx / det], 1).astype(np.float32)
    depth = np.linalg.norm(pos.astype(np.float64) - np.asarray(view, np.float64)[None, :], axis=1)
    order = np.lexsort((np.arange(n), depth))
    r = 3.0 * np.maximum(s1, s2)
    x0 = np.clip(np.floor((mx - r) / 16), 0, tiles_x - 1).astype(np.int64)
    x1 = np.clip(np.floor((mx + r) / 16), -1, tiles_x - 1).astype(np.int64)
    y0 = np.clip(np.floor((my - r) / 16), 0, tiles_y - 1).astype(np.int64)
    y1 = np.clip(np.floor((my + r) / 16), -1, tiles_y - 1).astype(np.int64)
    on = ~((mx + r < 0) | (my + r < 0) | (mx - r >= W) | (my - r >= H))
    wx = np.where(on, x1 - x0 + 1, 0)
    cnt = np.where(on, wx * (y1 - y0 + 1), 0)[order]
    pr = np.repeat(order, cnt)                     # primitive of each (primitive, tile) entry, front to back
    local = np.arange(pr.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    t = (y0[pr] + local // wx[pr]) * tiles_x + x0[pr] + local % wx[pr]
    k = np.argsort(t, kind="stable")          # depth order kept within each tile
    lst = pr[k].astype(np.uint32)
    tile_start = np.zeros(tiles_x * tiles_y + 1, np.uint32)
    np.cumsum(np.bincount(t, minlength=tiles_x * tiles_y), out=tile_start[1:])
    return foot, tile_start, lst


def batch_sizes(n_scenes=64, lo=50_000, hi=2_000_000, seed=4):
    """Primitive counts drawn log-uniformly from [lo, hi] (rounded)."""
    rng = _rng(seed)
    return [int(round(math.exp(x))) for x in rng.uniform(math.log(lo), math.log(hi), n_scenes)]


# The five workloads (sizes and seeds) the tests and the benchmark use.
CONFIGS = {
    "small": dict(n=65_536, clusters=32, comps=64, seed=1, dirs=64),
    "mid": dict(n=1_048_576, clusters=32, comps=64, seed=2, dirs=64),
    "large": dict(n=3_145_728, clusters=256, comps=256, seed=3, dirs=1024, rate=6.0),
}
