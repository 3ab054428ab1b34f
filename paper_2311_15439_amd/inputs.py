"""Seeded synthetic inputs shared by the oracle checks and the GPU path.

This module only draws random numbers and lays them out; it holds none of the
encoding's arithmetic.  Every generator takes an explicit seed and uses
``numpy.random.default_rng``.

Workload shapes follow the paper's experiments: 2-D image fitting (random
pixel coordinates of a 16384^2 image), 3-D volume sampling (rays through the
unit cube with stratified samples), and an n-D dimension sweep.  The paper's
own photograph and scenes are not available; these inputs stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n_dims: int
    n_levels: int
    log2_T: int
    n_feat: int
    table_f16: bool
    n_min: float
    growth: float
    n_points: int
    table_init: float  # tables drawn from U(-table_init, table_init)
    seed_points: int
    seed_tables: int


def growth_from_ends(n_min: float, n_max: float, L: int) -> float:
    """Per-level growth factor of a geometric schedule given its two ends."""
    return (n_max / n_min) ** (1.0 / (L - 1))


# Workloads: the image fit, the volume, and the dimension sweep, at the
# sizes the paper's experiments use (Sec. 6), with synthetic contents.
PLAIN_2D = Workload("plain-2d n=2 L=4 T=2^14 F=2 f32", 2, 4, 14, 2, False, 16.0, 1.5, 1 << 16, 1.0, 1, 2)
IMAGE_2D = Workload("image-2d n=2 L=16 T=2^22 F=2 f16", 2, 16, 22, 2, True, 16.0,
                    growth_from_ends(16, 1 << 15, 16), 1 << 20, 1e-4, 3, 5)
VOLUME_3D = Workload("volume-3d n=3 L=16 T=2^19 F=2 f16", 3, 16, 19, 2, True, 16.0,
                     growth_from_ends(16, 2048, 16), 1 << 21, 1e-4, 6, 8)


def sweep_workload(n: int) -> Workload:
    return Workload(f"sweep n={n} L=8 T=2^20 F=2 f16", n, 8, 20, 2, True, 16.0,
                    growth_from_ends(16, 512, 8), 1 << 20, 1e-4, 10 + n, 20 + n)


def uniform_points(N: int, n: int, seed: int) -> np.ndarray:
    """x ~ U[0,1)^n, float32 [N, n]."""
    return np.random.default_rng(seed).random((N, n), dtype=np.float32)


def pixel_points(N: int, seed: int, width: int = 16384) -> np.ndarray:
    """Random pixel positions (i + u) / width of a width x width image."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, width, size=(N, 2))
    u = rng.random((N, 2))
    return ((i + u) / width).astype(np.float32)


def ray_points(n_rays: int, n_samples: int, seed: int, radius: float = 1.5) -> np.ndarray:
    """Stratified samples along random rays through the unit cube, ray-major
    ([n_rays * n_samples, 3] float32, sample k of ray r at r*n_samples + k).

    Origins lie on a sphere of the given radius around the cube centre; each
    ray aims at a uniform point inside the cube and is clipped to the cube
    (slab test); sample k sits at t0 + (k + u_k)(t1 - t0)/n_samples."""
    rng = np.random.default_rng(seed)
    centre = np.full(3, 0.5)
    d = rng.normal(size=(n_rays, 3))
    o = centre + radius * d / np.linalg.norm(d, axis=1, keepdims=True)
    tgt = rng.random((n_rays, 3))
    dirn = tgt - o
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirn
        ta = (0.0 - o) * inv
        tb = (1.0 - o) * inv
    t0 = np.max(np.minimum(ta, tb), axis=1)
    t1 = np.min(np.maximum(ta, tb), axis=1)
    t0 = np.maximum(t0, 0.0)
    u = rng.random((n_rays, n_samples))
    k = np.arange(n_samples)[None, :]
    t = t0[:, None] + (k + u) * ((t1 - t0)[:, None] / n_samples)
    p = o[:, None, :] + t[..., None] * dirn[:, None, :]
    return np.clip(p, 0.0, np.nextafter(np.float32(1), np.float32(0))).reshape(-1, 3).astype(np.float32)


def tables(L: int, T: int, F: int, scale: float, seed: int, f16: bool) -> np.ndarray:
    """Feature tables [L, T, F] drawn from U(-scale, scale); float32 or float16."""
    t = np.random.default_rng(seed).uniform(-scale, scale, size=(L, T, F))
    return t.astype(np.float16 if f16 else np.float32)


def dense_values(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


def mlp_weights(d_in: int, hidden: int, d_out: int, seed: int):
    """Row-major binary16 weights W1 [H, d_in], W2 [H, H], W3 [d_out, H],
    drawn uniformly with the fan-in scaled bound sqrt(6 / fan_in)."""
    rng = np.random.default_rng(seed)

    def u(o, i):
        b = math.sqrt(6.0 / i)
        return rng.uniform(-b, b, size=(o, i)).astype(np.float16)

    return u(hidden, d_in), u(hidden, hidden), u(d_out, hidden)


def features_f16(N: int, D: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-scale, scale, size=(N, D)).astype(np.float16)


def gradients(N: int, D: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-scale, scale, size=(N, D)).astype(np.float32)


def procedural_rgb(pts: np.ndarray, seed: int, n_blobs: int = 64, n_waves: int = 8) -> np.ndarray:
    """Synthetic RGB target at 2-D points: random Gaussian blobs plus
    sinusoids (stands in for the paper's gigapixel photograph)."""
    rng = np.random.default_rng(seed)
    c = rng.random((n_blobs, 2))
    s = np.exp(rng.uniform(np.log(2.0 ** -9), np.log(2.0 ** -3), n_blobs))
    col = rng.random((n_blobs, 3))
    om = rng.normal(size=(n_waves, 2)) * rng.uniform(4, 2 ** 12, (n_waves, 1))
    ph = rng.uniform(0, 2 * np.pi, n_waves)
    wc = rng.random((n_waves, 3)) * 0.15
    x = pts.astype(np.float64)
    out = np.zeros((len(x), 3))
    for b in range(n_blobs):
        r2 = ((x - c[b]) ** 2).sum(1)
        out += np.exp(-0.5 * r2 / s[b] ** 2)[:, None] * col[b]
    for k in range(n_waves):
        out += np.sin(x @ om[k] + ph[k])[:, None] * wc[k]
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def procedural_density(pts: np.ndarray, seed: int, n_blobs: int = 32) -> np.ndarray:
    """Synthetic (sigma, r, g, b) target at 3-D points: a sum of Gaussian
    blobs (stands in for the paper's scenes)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.15, 0.85, (n_blobs, 3))
    s = rng.uniform(0.02, 0.12, n_blobs)
    col = rng.random((n_blobs, 3))
    x = pts.astype(np.float64)
    sig = np.zeros(len(x))
    rgb = np.zeros((len(x), 3))
    for b in range(n_blobs):
        g = np.exp(-0.5 * ((x - c[b]) ** 2).sum(1) / s[b] ** 2)
        sig += g
        rgb += g[:, None] * col[b]
    rgb /= np.maximum(sig, 1e-6)[:, None]
    return np.concatenate([sig[:, None], rgb], 1).astype(np.float32)


def nd_workload(n: int) -> Workload:
    """An n-dimensional regression field for the accuracy comparison beyond
    three dimensions (standing in for the high-dimensional tasks of Sec. 6):
    16 levels of 2 features (the network's 32 inputs), resolutions
    16 -> 512, T = 2^20, 2^18 points per step."""
    return Workload(f"field n={n} L=16 T=2^20 F=2 f16", n, 16, 20, 2, True, 16.0,
                    growth_from_ends(16, 512, 16), 1 << 18, 1e-4, 40 + n, 50 + n)


def procedural_nd(pts: np.ndarray, seed: int, n_blobs: int = 48, n_waves: int = 6) -> np.ndarray:
    """Synthetic 3-channel target over [0,1]^n: a 0.25 base, anisotropic
    Gaussian blobs (widths 2^-4 .. 2^-2 per axis) and plane waves of up to
    24 cycles per unit, clipped to [0, 1]."""
    rng = np.random.default_rng(seed)
    n = pts.shape[1]
    c = rng.random((n_blobs, n))
    s = np.exp(rng.uniform(np.log(2.0 ** -4), np.log(2.0 ** -2), (n_blobs, n)))
    col = rng.random((n_blobs, 3))
    om = rng.normal(size=(n_waves, n))
    om *= (rng.uniform(2, 24, (n_waves, 1)) * 2 * np.pi / np.linalg.norm(om, axis=1, keepdims=True))
    ph = rng.uniform(0, 2 * np.pi, n_waves)
    wc = rng.random((n_waves, 3)) * 0.2
    x = pts.astype(np.float64)
    out = np.full((len(x), 3), 0.25)
    for b in range(n_blobs):
        r2 = (((x - c[b]) / s[b]) ** 2).sum(1)
        out += np.exp(-0.5 * r2)[:, None] * col[b]
    for k in range(n_waves):
        out += np.sin(x @ om[k] + ph[k])[:, None] * wc[k]
    return np.clip(out, 0.0, 1.0).astype(np.float32)
