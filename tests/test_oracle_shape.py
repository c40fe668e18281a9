"""Pins of the FP64 shape-diagnostics oracle (CPU): a hand-derived worked
example of the discretised inertia tensor, invariances, the solid-ellipsoid
closed form, and the cell strain of known point sets."""
import numpy as np
import pytest

from oracle import shape
from synth.mesh import sphere_mesh


def _regular_tet():
    """A regular tetrahedron with centroid 0 and edge sqrt(3)."""
    return np.array([[1.0, 0, -1 / np.sqrt(8)], [-0.5, np.sqrt(3) / 2, -1 / np.sqrt(8)],
                     [-0.5, -np.sqrt(3) / 2, -1 / np.sqrt(8)], [0, 0, 3 / np.sqrt(8)]]) \
        * np.array([1.0, 1.0, 1.0])


def _six_tets(d, e, g, scale=(1.0, 1.0, 1.0)):
    """Six disjoint copies of one tetrahedron with centroids at +-d e_x,
    +-e e_y, +-g e_z; the pair on axis k is scaled by scale[k] about its
    centroid."""
    t = _regular_tet()
    t -= t.mean(axis=0)
    pts, tets = [], []
    for k, (dist, s) in enumerate(zip((d, e, g), scale)):
        for sign in (1.0, -1.0):
            c = np.zeros(3)
            c[k] = sign * dist
            tets.append(np.arange(len(pts), len(pts) + 4))
            pts.extend(c + s * t)
    return np.array(pts), np.array(tets, dtype=np.int32)


def test_worked_example_six_tetrahedra():
    """Centroids r on the axes: the second moment is S = 2 diag(V_x d^2,
    V_y e^2, V_z g^2), I = tr(S) 1 - S, and with S_x > S_y > S_z the semi-axis
    formula gives a_k^2 = (5 / (2M)) 2 S_k, so a_k = sqrt(5 S_k / M) and
    D = (sqrt(S_x) - sqrt(S_z)) / (sqrt(S_x) + sqrt(S_z)).  The deformed
    configuration rescales the tetrahedra (current volumes differ from the
    reference ones), is translated and rotated."""
    d, e, g = 3.0, 2.0, 1.5
    x, tets = _six_tets(d, e, g)
    y0, _ = _six_tets(d, e, g, scale=(1.2, 0.9, 0.7))
    V1 = abs(np.linalg.det((_regular_tet()[:3] - _regular_tet()[3]).T)) / 6
    Vx, Vy, Vz = V1 * 1.2 ** 3, V1 * 0.9 ** 3, V1 * 0.7 ** 3
    Sx, Sy, Sz = 2 * Vx * d * d, 2 * Vy * e * e, 2 * Vz * g * g
    assert Sx > Sy > Sz
    M = 2 * (Vx + Vy + Vz)
    a_ref = np.sqrt(5 * np.array([Sz, Sy, Sx]) / M)
    D_ref = (np.sqrt(Sx) - np.sqrt(Sz)) / (np.sqrt(Sx) + np.sqrt(Sz))
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    for y in (y0, y0 @ Q.T + np.array([10.0, -4.0, 2.5])):
        out = shape.cell_shape(x, y, tets)
        assert abs(out["volume"] - M) <= 1e-13 * M
        assert np.allclose(out["axes"], a_ref, rtol=1e-12, atol=0)
        assert abs(out["D"] - D_ref) <= 1e-12


def test_volume_sign_and_reference_orientation():
    x = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    tets = np.array([[0, 1, 2, 3], [1, 0, 2, 3]], dtype=np.int32)
    V = shape.tet_volumes(x, x, tets)
    assert np.allclose(V, [1 / 6, 1 / 6], rtol=1e-15)
    y = x.copy()
    y[3, 2] = -0.5                       # pushed through the opposite face
    assert np.allclose(shape.tet_volumes(x, y, tets), [-1 / 12, -1 / 12])


@pytest.fixture(scope="module")
def sphere():
    return sphere_mesh(3000, 11)


def test_solid_ellipsoid_closed_form(sphere):
    """A unit sphere mapped by diag(1.4, 1.0, 0.6) is a solid ellipsoid with
    semi-axes (0.6, 1.0, 1.4): D = 0.4.  The discretised tensor (point
    masses at tetrahedron centroids, faceted surface) is exact up to
    O((h/R)^2): below 1 % on the semi-axes and the volume at this resolution
    (16.7k tetrahedra); D, a ratio, is much closer."""
    x, tets = sphere
    A = np.diag([1.4, 1.0, 0.6])
    out = shape.cell_shape(x, x @ A.T, tets, d_ref=2.0)
    assert np.allclose(out["axes"], [0.6, 1.0, 1.4], rtol=0.01, atol=0)
    assert abs(out["D"] - 0.4) <= 0.002
    assert abs(out["volume"] - 4 / 3 * np.pi * 1.4 * 0.6) <= 0.015 * out["volume"]
    # the longest node pair spans the major axis
    assert 2 * 1.4 * 0.995 <= out["d_max"] <= 2 * 1.4 + 1e-12
    assert abs(out["strain"] - (out["d_max"] - 2.0) / 2.0) <= 1e-15
    # undeformed: D ~ 0 and strain ~ 0
    out0 = shape.cell_shape(x, x, tets, d_ref=2.0)
    assert out0["D"] <= 0.01 and abs(out0["strain"]) <= 0.01


def test_max_node_distance_known_sets():
    rng = np.random.default_rng(3)
    pts = rng.normal(size=(700, 3)) * 0.1
    pts[123] = [2.0, 0, 0]
    pts[456] = [-1.0, 0.5, 0]
    assert abs(shape.max_node_distance(pts) - np.hypot(3.0, 0.5)) <= 1e-14
    # the maximum of a regular tetrahedron's vertices is its edge
    assert abs(shape.max_node_distance(_regular_tet()) - np.sqrt(3.0)) <= 1e-14
