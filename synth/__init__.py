"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds geometry and random numbers only: point sets on closed
surfaces, boundary-element panels and right-hand sides.  It contains none of
the inverse-FMM arithmetic, so both the CPU oracle and the HIP path may import
it without sharing any of the method's code.

Every generator takes an explicit seed and uses numpy's PCG64 generator, so a
(generator, seed, size) triple always yields the same bytes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sphere_points",
    "ellipsoid_points",
    "cube_surface_points",
    "geometry_points",
    "uniform_rhs",
    "icosphere",
    "laplace_self_term",
    "ellipsoid_area",
    "batch_geometries",
]


def sphere_points(n: int, seed: int, radius: float = 1.0) -> np.ndarray:
    """n points i.i.d. uniform on the sphere of the given radius (normalised
    Gaussian vectors).  Returns an (n, 3) float64 array, row-major."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return np.ascontiguousarray(g * radius)


def ellipsoid_points(n: int, seed: int, axes=(1.0, 0.7, 0.3), jitter: float = 0.0) -> np.ndarray:
    """n points area-uniform on the ellipsoid with the given semi-axes.

    Sampling: normalised Gaussians mapped onto the ellipsoid, accepted with
    probability proportional to the local area element (rejection).  With
    jitter > 0 every point is then moved by jitter * max(axes) * U[-1, 1]^3.
    """
    rng = np.random.default_rng(seed)
    a = np.asarray(axes, dtype=np.float64)
    out = np.empty((0, 3))
    # Area element of the map u -> a*u (u on S^2) is |a| * |u / a| up to a
    # constant factor; its maximum is max_i (prod a / a_i).
    amax = np.prod(a) / np.min(a)
    while out.shape[0] < n:
        m = max(2 * (n - out.shape[0]), 1024)
        u = rng.standard_normal((m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        dens = np.prod(a) * np.linalg.norm(u / a, axis=1)
        keep = rng.random(m) * amax < dens
        out = np.concatenate([out, u[keep] * a], axis=0)
    out = out[:n]
    if jitter > 0.0:
        out = out + jitter * float(np.max(a)) * rng.uniform(-1.0, 1.0, size=out.shape)
    return np.ascontiguousarray(out)


def cube_surface_points(n: int, seed: int, half_side: float = 1.0) -> np.ndarray:
    """n points uniform on the surface of the cube [-half_side, half_side]^3."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-half_side, half_side, size=(n, 2))
    p = np.empty((n, 3))
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    for d in range(3):
        others = [e for e in range(3) if e != d]
        sel = axis == d
        p[sel, d] = sign[sel] * half_side
        p[sel, others[0]] = uv[sel, 0]
        p[sel, others[1]] = uv[sel, 1]
    return np.ascontiguousarray(p)


def geometry_points(shape: str, n: int, seed: int, **kw) -> np.ndarray:
    if shape == "sphere":
        return sphere_points(n, seed, **kw)
    if shape == "ellipsoid":
        return ellipsoid_points(n, seed, **kw)
    if shape == "cube":
        return cube_surface_points(n, seed, **kw)
    raise ValueError(f"unknown shape {shape!r}")


def uniform_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides with i.i.d. U[-1, 1] entries, shape (n, nrhs), column-major
    semantics (column k is right-hand side k)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(n, nrhs)))


def ellipsoid_area(axes=(1.0, 0.7, 0.3)) -> float:
    """Surface area of an ellipsoid (Knud Thomsen's approximation, relative
    error below 1.1 %)."""
    a, b, c = (float(x) for x in axes)
    p = 1.6075
    return 4.0 * np.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1.0 / p)


def laplace_self_term(n: int, area: float = 4.0 * np.pi) -> float:
    """Diagonal entry 1/(4 pi * 0.5 h) with h = sqrt(area / n): the self
    interaction of a point that stands for a patch of mean spacing h."""
    h = np.sqrt(area / n)
    return 1.0 / (4.0 * np.pi * 0.5 * h)


def icosphere(subdiv: int):
    """Unit icosphere: icosahedron refined `subdiv` times (each triangle split in
    four, new vertices pushed onto the sphere).  Returns (vertices (V,3),
    triangles (20*4^subdiv, 3) int64)."""
    t = (1.0 + np.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    verts = [row for row in v]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = np.empty((4 * f.shape[0], 3), dtype=np.int64)
        for k, (a, b, c) in enumerate(f):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * k + 0] = (a, ab, ca)
            nf[4 * k + 1] = (b, bc, ab)
            nf[4 * k + 2] = (c, ca, bc)
            nf[4 * k + 3] = (ab, bc, ca)
        f = nf
    return np.asarray(verts), f


def batch_geometries(count: int, base_seed: int, nmin: int = 2048, nmax: int = 32768):
    """The many-geometry workload: geometry g is a sphere (radius 1), an
    ellipsoid (semi-axes i.i.d. U[0.5, 2]) or a cube surface (half-side 1)
    according to g mod 3, with N_g uniform in [nmin, nmax].  Returns a list of
    (shape, points) pairs."""
    out = []
    for g in range(count):
        seed = base_seed + g
        rng = np.random.default_rng(seed)
        n = int(rng.integers(nmin, nmax + 1))
        shape = ("sphere", "ellipsoid", "cube")[g % 3]
        if shape == "ellipsoid":
            axes = tuple(rng.uniform(0.5, 2.0, size=3))
            pts = ellipsoid_points(n, seed + 100000, axes=axes)
        elif shape == "sphere":
            pts = sphere_points(n, seed + 100000)
        else:
            pts = cube_surface_points(n, seed + 100000)
        out.append((shape, pts))
    return out
