"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws points, normals, right-hand sides and instance
parameters. It holds none of the method's arithmetic (no tree, partition,
compression, precision rule or product), so both the HIP library and the CPU
oracle can be fed the same inputs without sharing any code of the method.

Point sets follow the paper's numerical section: P_square (uniform in a
hypercube) and P_circle (on the unit hypersphere); the configuration recipes
below add the interior-ball mix used for the nonsymmetric double-layer case.
All draws use ``numpy.random.default_rng(seed)`` in a fixed order: points
first, then anything else.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Kernel type codes (same numbering as the C header's hh_kernel_type).
LOG, INV_R, INV_R2, GAUSS, MATERN, DOUBLE_LAYER = 1, 2, 3, 4, 5, 6
KERNEL_NAMES = {LOG: "log", INV_R: "inv_r", INV_R2: "inv_r2", GAUSS: "gauss",
                MATERN: "matern", DOUBLE_LAYER: "double_layer"}

# Storage-format bits of the precision mask (same as the C header).
FMT_FP64, FMT_FP32, FMT_FP16, FMT_BF16 = 0, 1, 2, 3
MASK_ALL = 0xF
# 8-bit quarter precision q43 (1 sign, 4 exponent, 3 fraction bits) of the
# paper's format table: mask bit 4 of the oracle; not a storage format of the
# C header.
FMT_Q43 = 4


def uniform_cube(n: int, d: int, rng, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n points i.i.d. uniform in [lo, hi]^d, row-major (n, d) float64."""
    return lo + (hi - lo) * rng.random((n, d))


def sphere_surface(n: int, d: int, rng) -> np.ndarray:
    """n points uniform on the unit sphere surface in R^d (normalised Gaussians)."""
    g = rng.standard_normal((n, d))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def ball_interior(n: int, d: int, rng) -> np.ndarray:
    """n points uniform in the unit ball in R^d (direction times radius U^(1/d))."""
    g = rng.standard_normal((n, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / d)
    return g * r[:, None]


def unit_normals(n: int, d: int, rng) -> np.ndarray:
    """n random unit vectors in R^d (normalised standard Gaussians)."""
    g = rng.standard_normal((n, d))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def rhs(n: int, nrhs: int, rng, dtype=np.float64) -> np.ndarray:
    """Right-hand sides x ~ N(0, 1), shape (n, nrhs), C order."""
    return rng.standard_normal((n, nrhs)).astype(dtype)


@dataclass
class Problem:
    """One H_h problem instance: points plus every parameter hh_build takes."""
    name: str
    points: np.ndarray
    kernel: int
    tol: float
    eta: float
    switch_level: int          # -1 means "L - 1" (the paper's default choice)
    leaf_size: int
    scale: float = 1.0
    h: float = 1.0
    normals: np.ndarray | None = None
    mask: int = MASK_ALL
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def d(self) -> int:
        return int(self.points.shape[1])


def cfg_plain_small(seed: int = 101, n: int = 4096) -> Problem:
    """2D log|r| on N uniform points in [0,1]^2, leaf 64, eta 1, switch 2, tol 1e-8,
    formats {fp64, fp32, fp16}."""
    rng = np.random.default_rng(seed)
    pts = uniform_cube(n, 2, rng)
    return Problem("plain_2d_log", pts, LOG, 1e-8, 1.0, 2, 64,
                   mask=(1 << FMT_FP64) | (1 << FMT_FP32) | (1 << FMT_FP16), seed=seed)


def cfg_2d_inv_r(seed: int = 202, n: int = 1 << 18) -> Problem:
    """2D 1/r on N uniform points in [0,1]^2, leaf 128, eta 1, switch 4, tol 1e-6."""
    rng = np.random.default_rng(seed)
    pts = uniform_cube(n, 2, rng)
    return Problem("2d_inv_r", pts, INV_R, 1e-6, 1.0, 4, 128, seed=seed)


def cfg_3d_laplace(seed: int = 303, n: int = 1 << 20, switch_level: int = 3) -> Problem:
    """3D Laplace 1/(4 pi r) on N uniform points in [0,1]^3, leaf 256, eta 1.5,
    tol 1e-6. The tree depth is 4 here, so the switching level is the paper's
    default L-1 = 3."""
    rng = np.random.default_rng(seed)
    pts = uniform_cube(n, 3, rng)
    return Problem("3d_laplace", pts, INV_R, 1e-6, 1.5, switch_level, 256,
                   scale=1.0 / (4.0 * math.pi), seed=seed)


def cfg_batched(seed: int = 404, count: int = 512, nmin_log2: int = 10,
                nmax_log2: int = 16) -> list[Problem]:
    """Independent Gaussian-kernel instances exp(-r^2/h^2): N log-uniform in
    [2^nmin, 2^nmax], points uniform in the unit cube, h ~ U[0.05, 0.3], tol drawn
    from {1e-4, 1e-6, 1e-8}; leaf 64, eta sqrt(3), switch L-1."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(math.floor(2.0 ** rng.uniform(nmin_log2, nmax_log2)))
        h = float(rng.uniform(0.05, 0.3))
        tol = float(rng.choice([1e-4, 1e-6, 1e-8]))
        pts = uniform_cube(n, 3, rng)
        out.append(Problem(f"gauss_{t}", pts, GAUSS, tol, math.sqrt(3.0), -1, 64,
                           h=h, seed=seed, extra={"index": t}))
    return out


def cfg_double_layer(seed: int = 505, n: int = 1 << 19) -> Problem:
    """Nonsymmetric double-layer kernel n_j.(p_i-p_j)/|p_i-p_j|^3: half the points
    uniform on the unit sphere surface, half uniform in the unit ball, random unit
    normals n_j; leaf 256, eta 1.5, switch 3, tol 1e-6."""
    rng = np.random.default_rng(seed)
    ns = n // 2
    pts = np.concatenate([sphere_surface(ns, 3, rng), ball_interior(n - ns, 3, rng)])
    nrm = unit_normals(n, 3, rng)
    return Problem("double_layer", pts, DOUBLE_LAYER, 1e-6, 1.5, 3, 256,
                   normals=nrm, seed=seed)


def paper_cube(n: int, d: int, kernel: int, tol: float, leaf_size: int,
               switch_level: int = -1, seed: int = 7, eta: float | None = None) -> Problem:
    """The paper's P_square set: N uniform points in [-1,1]^d, eta = sqrt(d)."""
    rng = np.random.default_rng(seed)
    pts = uniform_cube(n, d, rng, -1.0, 1.0)
    return Problem(f"paper_{d}d", pts, kernel, tol,
                   math.sqrt(d) if eta is None else eta, switch_level, leaf_size, seed=seed)
