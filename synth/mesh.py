"""Seeded tetrahedral sphere meshes (test and benchmark input only).

The paper's cells are spheres meshed with 2,000-5,000 vertices and roughly
10,000-30,000 tetrahedra (Sec. "Simulation setup"); its own mesh generator is
described only in the missing supporting information.  This module builds a
stand-in with the same shape statistics:

* interior points on a body-centred-cubic (BCC) lattice of spacing ``a`` with
  a small Gaussian jitter, kept strictly inside the sphere;
* surface points on a Fibonacci spiral of the unit sphere;
* a Delaunay tetrahedralisation of the union (scipy's Qhull);
* tetrahedra whose reference edge matrix has a 2-norm condition number above
  ``cond_max`` are dropped (flat slivers that Qhull leaves on the hull),
  and vertices no tetrahedron uses any more are removed.

Everything here is topology and geometry of the *input*: no strain energy or
force is evaluated.  The determinant used to orient tetrahedra is the signed
volume of the vertex simplex.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay


def bcc_spacing(n_target: int, radius: float = 1.0) -> float:
    """BCC lattice constant giving about ``n_target`` points in the ball.

    A BCC lattice holds 2 points per cube of side ``a``.
    """
    vol = 4.0 / 3.0 * np.pi * radius ** 3
    return float((2.0 * vol / n_target) ** (1.0 / 3.0))


def fibonacci_sphere(n: int, radius: float = 1.0) -> np.ndarray:
    """``n`` nearly uniform points on the sphere of the given radius."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _edge_matrices(x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Columns x^k - x^4 for k = 1..3 (vertex 4 is the local origin)."""
    x4 = x[tets[:, 3]]
    return np.stack([x[tets[:, 0]] - x4, x[tets[:, 1]] - x4,
                     x[tets[:, 2]] - x4], axis=2)


def signed_volumes6(x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Six times the signed volume of each tetrahedron."""
    return np.linalg.det(_edge_matrices(x, tets))


def condition_numbers(x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """2-norm condition number of each reference edge matrix."""
    s = np.linalg.svd(_edge_matrices(x, tets), compute_uv=False)
    with np.errstate(divide="ignore"):
        return s[:, 0] / s[:, 2]


def orient_positive(x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two vertices of every negatively oriented tetrahedron."""
    tets = tets.copy()
    neg = signed_volumes6(x, tets) < 0
    tets[neg, 0], tets[neg, 1] = tets[neg, 1].copy(), tets[neg, 0].copy()
    return tets


def compact(x: np.ndarray, tets: np.ndarray):
    """Drop unreferenced vertices and renumber the rest in their old order."""
    used = np.zeros(len(x), dtype=bool)
    used[tets.ravel()] = True
    new_id = np.cumsum(used) - 1
    return x[used], new_id[tets].astype(np.int32)


def unique_edges(tets: np.ndarray) -> np.ndarray:
    """The 6 edges of every tetrahedron, deduplicated, as (E, 2) sorted pairs."""
    pairs = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]])
    e = tets[:, pairs].reshape(-1, 2)
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def mean_edge_length(x: np.ndarray, tets: np.ndarray) -> float:
    e = unique_edges(tets)
    return float(np.linalg.norm(x[e[:, 0]] - x[e[:, 1]], axis=1).mean())


def boundary_faces(tets: np.ndarray) -> np.ndarray:
    """Faces used by exactly one tetrahedron, wound so that the right-hand
    normal points out of that tetrahedron (for positively oriented tets)."""
    # Face opposite vertex v of (0,1,2,3), with an outward winding for a
    # positively oriented tetrahedron.
    local = np.array([[1, 3, 2], [0, 2, 3], [0, 3, 1], [0, 1, 2]])
    f = tets[:, local].reshape(-1, 3)
    key = np.sort(f, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True,
                            return_counts=True)
    return f[cnt[inv.ravel()] == 1]


def sphere_mesh(n_target: int, seed: int, radius: float = 1.0,
                jitter: float = 0.02, cond_max: float = 100.0):
    """Tetrahedral mesh of a ball with about ``n_target`` vertices.

    Returns ``(x, tets)``: float64 (N, 3) reference positions and int32 (M, 4)
    vertex indices, every tetrahedron positively oriented.
    """
    rng = np.random.default_rng(seed)
    a = bcc_spacing(n_target, radius)
    n = int(np.ceil(radius / a)) + 1
    g = np.arange(-n, n + 1, dtype=np.float64) * a
    cube = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    lat = np.concatenate([cube, cube + 0.5 * a])
    lat = lat + rng.normal(0.0, jitter * a, size=lat.shape)
    lat = lat[np.linalg.norm(lat, axis=1) < radius - 0.5 * a]
    n_surf = int(round(1.1 * 4.0 * np.pi * radius ** 2 / a ** 2))
    pts = np.concatenate([lat, fibonacci_sphere(n_surf, radius)])
    tets = Delaunay(pts).simplices.astype(np.int32)
    tets = orient_positive(pts, tets)
    keep = condition_numbers(pts, tets) <= cond_max
    x, tets = compact(pts, tets[keep])
    return np.ascontiguousarray(x), np.ascontiguousarray(tets)


def ellipsoid(x: np.ndarray, axes) -> np.ndarray:
    """Reference positions of the ball scaled to semi-axes ``axes``."""
    return x * np.asarray(axes, dtype=np.float64)[None, :]


def mesh_stats(x: np.ndarray, tets: np.ndarray) -> dict:
    vol6 = signed_volumes6(x, tets)
    cond = condition_numbers(x, tets)
    deg = np.bincount(tets.ravel(), minlength=len(x))
    return {
        "nodes": int(len(x)), "tets": int(len(tets)),
        "tets_per_node": float(len(tets) / len(x)),
        "mean_edge": mean_edge_length(x, tets),
        "volume": float(vol6.sum() / 6.0),
        "cond_p50": float(np.percentile(cond, 50)),
        "cond_p99": float(np.percentile(cond, 99)),
        "cond_max": float(cond.max()),
        "node_degree_mean": float(deg.mean()),
        "node_degree_max": int(deg.max()),
    }
