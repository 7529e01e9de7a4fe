"""Oracle: the collocation BEM of the Laplace Dirichlet problem on a sphere.

Test infrastructure only (see the package header).

Alg. 4 of the paper solves a boundary integral equation discretised with
piecewise-constant elements; its scatterer, kernel and quadrature are
Helmholtz-specific and deferred to its references.  The Laplace stand-in is
the first-kind (single-layer) equation

    int_Gamma sigma(y) / (4 pi |x - y|) dS_y = f(x),  x on Gamma,

collocated at the panel centroids c_i with one-point quadrature off the
diagonal: A_ij = area_j / (4 pi |c_i - c_j|).  The self term is the integral
of the kernel over the disc of the panel's area centred at c_i,
sqrt(area_i / pi) / 2.

Closed form (pins the discretisation): for the unit sphere and
f(x) = 1 / |x - x0| with |x0| = a < 1, the exterior potential is f itself and
the interior one is its Kelvin image 1 / (a |x - x0 / a^2|); the jump of the
normal derivative gives sigma(x) = (1 - a^2) / |x - x0|^3.
"""
from __future__ import annotations

import numpy as np


def panels(vertices: np.ndarray, triangles: np.ndarray):
    """Centroids (P, 3) and areas (P,) of flat triangles."""
    a = vertices[triangles[:, 0]]
    b = vertices[triangles[:, 1]]
    c = vertices[triangles[:, 2]]
    centroids = (a + b + c) / 3.0
    areas = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return centroids, areas


def self_terms(areas: np.ndarray) -> np.ndarray:
    """Integral of 1 / (4 pi r) over a disc of the given area, seen from its
    centre: (1 / (4 pi)) * 2 pi R = R / 2 with R = sqrt(area / pi)."""
    return np.sqrt(np.asarray(areas, dtype=np.float64) / np.pi) / 2.0


def point_source(x: np.ndarray, x0=(0.0, 0.0, 0.5)) -> np.ndarray:
    return 1.0 / np.linalg.norm(np.asarray(x) - np.asarray(x0, dtype=np.float64)[None, :], axis=1)


def exact_density(x: np.ndarray, x0=(0.0, 0.0, 0.5)) -> np.ndarray:
    """sigma on the unit sphere for f = 1 / |x - x0| (see the module header)."""
    x0 = np.asarray(x0, dtype=np.float64)
    a2 = float(x0 @ x0)
    d = np.linalg.norm(np.asarray(x) - x0[None, :], axis=1)
    return (1.0 - a2) / d ** 3


def dense_matrix(centroids: np.ndarray, areas: np.ndarray) -> np.ndarray:
    """The collocation matrix (small panel counts only)."""
    d = centroids[:, None, :] - centroids[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    np.fill_diagonal(r, 1.0)
    A = areas[None, :] / (4.0 * np.pi * r)
    np.fill_diagonal(A, self_terms(areas))
    return A
