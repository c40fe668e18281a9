"""The seeded input generators: determinism, shapes and the noise rule."""
import numpy as np
import pytest

import oracle
from synth.configs import (J_FLOOR, small_sphere_case, uneven_batch,
                           volume_ratios)
from synth.mesh import boundary_faces, mesh_stats, signed_volumes6, sphere_mesh


def test_sphere_mesh_deterministic_and_paper_sized():
    x1, t1 = sphere_mesh(1000, 5)
    x2, t2 = sphere_mesh(1000, 5)
    assert np.array_equal(x1, x2) and np.array_equal(t1, t2)
    s = mesh_stats(x1, t1)
    # ~1,000 nodes / ~5,000 tets, volume close to 4 pi / 3
    assert 950 < s["nodes"] < 1150 and 4800 < s["tets"] < 5800
    assert abs(s["volume"] - 4.18879) < 0.1
    assert s["cond_max"] <= 100.0
    assert (signed_volumes6(x1, t1) > 0).all()


def test_boundary_is_closed_and_outward():
    x, t = sphere_mesh(300, 1)
    bf = boundary_faces(t)
    an = np.cross(x[bf[:, 1]] - x[bf[:, 0]], x[bf[:, 2]] - x[bf[:, 0]])
    assert np.abs(an.sum(0)).max() < 1e-12
    # divergence theorem: (1/3) sum over faces of (centroid . n area) = V
    vol = (np.einsum("ij,ij->i", x[bf].mean(1), an) / 6.0).sum()
    assert abs(vol - signed_volumes6(x, t).sum() / 6.0) < 1e-12


def test_noise_rule_keeps_volume_ratio_floor():
    for seed in (1000, 1007):
        c = small_sphere_case(seed)
        J = volume_ratios(c.x, c.y.astype(np.float64), c.tets)
        assert J.min() >= J_FLOOR * np.linalg.det(c.A) * (1 - 1e-5)


def test_uneven_batch_layout():
    b = uneven_batch(n_cells=6, seed=3000, ladder=4)
    assert b.node_off[0] == 0 and b.tet_off[0] == 0
    assert b.n_nodes == len(b.x) == len(b.y) and b.n_tets == len(b.tets)
    for c in range(b.n_cells):
        cell = b.cell(c)
        assert cell.tets.min() >= 0 and cell.tets.max() < cell.n_nodes
        mu, kappa, w = cell.theta
        assert 0.5 <= mu <= 2 and 5 <= kappa / mu <= 50 and 0 <= w <= 1
    b2 = uneven_batch(n_cells=6, seed=3000, ladder=4)
    assert np.array_equal(b.y, b2.y)


def test_oracle_rejects_bad_meshes():
    x = np.array([[0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    with pytest.raises(ValueError):
        oracle.OracleMesh(x, np.array([[0, 1, 2, 4]], dtype=np.int32))
    with pytest.raises(ValueError):
        oracle.OracleMesh(x, np.array([[0, 1, 2, 2]], dtype=np.int32))
