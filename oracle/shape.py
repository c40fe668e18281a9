"""FP64 reference for the cell-shape diagnostics (test infrastructure only):
the Taylor deformation parameter (Sec. "Taylor deformation parameter", eqs.
taylor-deformation-parameter-definition, inertia-tensor-discretized and
inertia-tensor-ellipsoid-semiaxes) and the cell strain (eq. cell-strain).

Readings where the paper is silent or garbled:
  * the inertia tensor is taken about the cell's centre of mass (the
    volume-weighted mean of the tetrahedron centroids; the paper does not
    name the origin);
  * V_l is the current signed volume of tetrahedron l, det(deformed edges)/6
    with the orientation of its reference vertex order (negative for an
    inverted tetrahedron);
  * the semi-axis formula of the paper yields the squared semi-axes of a
    solid ellipsoid (principal moments (M/5)(b^2 + c^2), ...), so
    a_i = sqrt((5 / (2 M)) (...)), with M the total current volume (uniform
    density); a negative radicand (a point set flatter than any ellipsoid)
    gives a_i = 0;
  * d_max is the largest distance between two nodes of the cell and d_ref
    the reference diameter supplied by the caller (2 R for the paper's
    spherical cell).
"""
from __future__ import annotations

import numpy as np


def tet_volumes(x, y, tets):
    """Current signed volumes: det[y^1 - y^4, y^2 - y^4, y^3 - y^4] / 6 times
    the sign of the same determinant in the reference configuration."""
    def det(p):
        e = p[tets[:, :3]] - p[tets[:, 3:4]]          # (m, 3 edges, 3)
        return np.linalg.det(np.transpose(e, (0, 2, 1)))
    return det(np.asarray(y, np.float64)) * np.sign(det(np.asarray(x, np.float64))) / 6.0


def inertia_tensor(x, y, tets):
    """Discretised inertia tensor about the centre of mass: the sum over
    tetrahedra of V_l (|r|^2 delta_ij - r_i r_j), r the tetrahedron centroid
    minus the centre of mass.  Returns (I, total volume, centre of mass)."""
    y = np.asarray(y, np.float64)
    V = tet_volumes(x, y, tets)
    cen = y[tets].mean(axis=1)                        # tetrahedron centroids
    M = V.sum()
    com = (V[:, None] * cen).sum(axis=0) / M
    r = cen - com
    I = np.zeros((3, 3))
    for l in range(len(V)):
        I += V[l] * (np.dot(r[l], r[l]) * np.eye(3) - np.outer(r[l], r[l]))
    return I, M, com


def semi_axes(I, M):
    """a_1 <= a_2 <= a_3 from the eigenvalues theta_1 >= theta_2 >= theta_3
    of the inertia tensor (squared-semi-axis reading, see module doc)."""
    th = np.sort(np.linalg.eigvalsh(I))[::-1]
    sq = (5.0 / (2.0 * M)) * np.array([-th[0] + th[1] + th[2],
                                       th[0] - th[1] + th[2],
                                       th[0] + th[1] - th[2]])
    return np.sqrt(np.clip(sq, 0.0, None))


def taylor_deformation(a):
    """D = (a_3 - a_1) / (a_3 + a_1)."""
    return (a[2] - a[0]) / (a[2] + a[0])


def max_node_distance(y):
    """Largest distance between two nodes (all pairs, in blocks)."""
    y = np.asarray(y, np.float64)
    best = 0.0
    for s in range(0, len(y), 512):
        d = y[s:s + 512, None, :] - y[None, :, :]
        best = max(best, float((d * d).sum(axis=2).max()))
    return np.sqrt(best)


def cell_shape(x, y, tets, d_ref=None):
    """All diagnostics of one cell: dict with volume, centre of mass,
    semi-axes, D, d_max and (if d_ref is given) strain = (d_max - d_ref) /
    d_ref."""
    I, M, com = inertia_tensor(x, y, tets)
    a = semi_axes(I, M)
    dmax = max_node_distance(y)
    out = {"volume": M, "com": com, "axes": a, "D": taylor_deformation(a),
           "d_max": dmax}
    if d_ref is not None:
        out["strain"] = (dmax - d_ref) / d_ref
    return out
