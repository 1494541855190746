"""Seeded synthetic scalar fields on 3D regular grids.

This module only draws random numbers and evaluates closed-form fields; it
holds none of the persistence arithmetic. Both the CPU oracle (tests) and the
GPU path (tests, smoke, bench) take their inputs from here, so neither side
ever produces the other's inputs.

All fields are returned as C-contiguous float32 arrays shaped [nz, ny, nx]
(x fastest), computed in float64 and rounded to float32 (round to nearest
even). Vertex coordinates are normalised, p = (x/(nx-1), y/(ny-1), z/(nz-1)).

Workload recipes (they stand in for the volumetric benchmark datasets the
paper resamples to 192^3, and for its "Elevation" and "Random" stress cases):

* ``noise``        i.i.d. uniform [0,1) float32 drawn directly in float32
                   (2^24 distinct values, so ties are exercised).
* ``gaussians``    sum of k isotropic Gaussians, centre ~ U[0,1)^3, sigma ~
                   U[s_lo, s_hi] (fraction of the side), amplitude ~ U[-1,1],
                   drawn in that order per Gaussian; then r * (max g - min g)
                   * U[0,1) i.i.d. noise, drawn after all Gaussians.
* ``elevation``    a*x + b*y + c*z with generic positive a, b, c.
* ``radial``       -|p - c|^2 with an off-centre c.
"""
from __future__ import annotations

import os

import numpy as np

__all__ = ["noise", "gaussians", "elevation", "radial", "field_from_config",
           "serving_requests"]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def noise(shape, seed: int) -> np.ndarray:
    nz, ny, nx = shape
    rng = _rng(seed)
    return rng.random(nz * ny * nx, dtype=np.float32).reshape(nz, ny, nx)


def _quantise(v: np.ndarray) -> np.ndarray:
    """Round to multiples of 2^-24: the exponential's last bits (which differ
    between CPUs and numpy builds) then no longer reach the field."""
    return np.round(v * 16777216.0) / 16777216.0


def gaussians(shape, seed: int, k: int, noise_frac: float,
              sigma_range=(0.02, 0.15)) -> np.ndarray:
    """Sum of k Gaussians plus uniform noise, evaluated separably.

    The sum is taken term by term in a fixed order with elementwise float64
    operations (no BLAS, whose summation order depends on the CPU), on
    factors rounded to multiples of 2^-24, so that a seed gives the same
    float32 field on every machine."""
    nz, ny, nx = shape
    rng = _rng(seed)
    xs = np.arange(nx, dtype=np.float64) / max(nx - 1, 1)
    ys = np.arange(ny, dtype=np.float64) / max(ny - 1, 1)
    zs = np.arange(nz, dtype=np.float64) / max(nz - 1, 1)
    GX = np.empty((k, nx))
    AZY = np.empty((k, nz, ny))  # a_i gz_i[z] gy_i[y]
    for i in range(k):
        c = rng.random(3)
        s = rng.uniform(sigma_range[0], sigma_range[1])
        a = rng.uniform(-1.0, 1.0)
        inv = 1.0 / (2.0 * s * s)
        GX[i] = _quantise(np.exp(-((xs - c[0]) ** 2) * inv))
        gy = _quantise(np.exp(-((ys - c[1]) ** 2) * inv))
        gz = _quantise(np.exp(-((zs - c[2]) ** 2) * inv))
        AZY[i] = (a * gz)[:, None] * gy[None, :]
    g = np.empty((nz, ny, nx))

    def slab(z0, z1):
        acc = g[z0:z1]
        acc[...] = 0.0
        tmp = np.empty_like(acc)
        for i in range(k):  # fixed order: the same sum everywhere
            np.multiply(AZY[i, z0:z1, :, None], GX[i][None, None, :], out=tmp)
            np.add(acc, tmp, out=acc)

    step = max(1, (1 << 21) // max(1, ny * nx))
    bounds = [(z0, min(nz, z0 + step)) for z0 in range(0, nz, step)]
    if len(bounds) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1, len(bounds))) as pool:
            list(pool.map(lambda b: slab(*b), bounds))
    else:
        slab(0, nz)
    if noise_frac > 0.0:
        span = float(g.max() - g.min())
        step = max(1, (1 << 24) // max(1, ny * nx))
        for z0 in range(0, nz, step):  # noise drawn in C order, slab by slab
            z1 = min(nz, z0 + step)
            g[z0:z1] += (noise_frac * span) * rng.random((z1 - z0) * ny * nx).reshape(z1 - z0, ny, nx)
    return np.ascontiguousarray(g.astype(np.float32))


def elevation(shape, coeffs=(1.0, 1.7320508075688772, 2.23606797749979)) -> np.ndarray:
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b, c = coeffs
    return np.ascontiguousarray((a * x + b * y + c * z).astype(np.float32))


def radial(shape, centre_offset=(0.0123, -0.0071, 0.0042)) -> np.ndarray:
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) / max(nz - 1, 1), np.arange(ny) / max(ny - 1, 1),
                          np.arange(nx) / max(nx - 1, 1), indexing="ij")
    c = (0.5 + centre_offset[0], 0.5 + centre_offset[1], 0.5 + centre_offset[2])
    f = -((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    return np.ascontiguousarray(f.astype(np.float32))


# Named workloads. Sizes follow the configurations the method is measured on.
CONFIGS = {
    "noise16": dict(shape=(16, 16, 16), kind="noise"),
    "smooth256": dict(shape=(256, 256, 256), kind="gaussians", k=32, r=0.01),
    "smooth512": dict(shape=(512, 512, 512), kind="gaussians", k=64, r=0.005),
    "noise512": dict(shape=(512, 512, 512), kind="noise"),
    "diff96": dict(shape=(96, 96, 96), kind="gaussians", k=16, r=0.02),
}


def with_infinities(field: np.ndarray, seed: int, frac_pos: float = 0.1, frac_neg: float = 0.05) -> np.ndarray:
    """A copy of field with random vertices set to +inf / -inf, plus the whole
    x = 0 face at +inf and the last vertex at -inf (infinities on the grid
    boundary, where batched grids meet their separators)."""
    rng = _rng(seed)
    f = np.array(field, dtype=np.float32, copy=True)
    u = rng.random(f.shape)
    f[u < frac_pos] = np.inf
    f[u > 1.0 - frac_neg] = -np.inf
    f[..., 0] = np.inf
    f.reshape(-1)[-1] = -np.inf
    return f


def field_from_config(name: str, seed: int = 0, shape=None) -> np.ndarray:
    cfg = CONFIGS[name]
    shp = tuple(shape) if shape is not None else cfg["shape"]
    if cfg["kind"] == "noise":
        return noise(shp, seed)
    return gaussians(shp, seed, cfg["k"], cfg["r"])


def serving_requests(n: int, seed: int = 1000, side_range=(16, 128), k: int = 8,
                     noise_frac: float = 0.01, rate: float = 1.0):
    """Request stream for the serving workload: per request, grid sides drawn
    log-uniform in side_range per axis (anisotropic), a Gaussian mixture plus
    noise field seeded with seed + i, and a Poisson arrival time (rate per s).
    Yields (arrival_s, shape, field_seed)."""
    rng = _rng(seed)
    lo, hi = np.log(side_range[0]), np.log(side_range[1])
    t = 0.0
    out = []
    for i in range(n):
        sides = np.rint(np.exp(rng.uniform(lo, hi, size=3))).astype(int)
        t += rng.exponential(1.0 / rate)
        out.append((t, (int(sides[2]), int(sides[1]), int(sides[0])), seed + i))
    return out
