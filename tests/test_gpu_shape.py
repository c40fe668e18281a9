"""Shape diagnostics on the GPU (cm_shape) against the FP64 oracle: current
volume, centre of mass, semi-axes and Taylor deformation D from the
discretised inertia tensor, largest node distance and cell strain.

Tolerances: the device forms the same float64 quantities from the same
float32 positions (exact float64 edge differences); only the summation order
and the eigen-solver (Jacobi vs LAPACK) differ, so the bars are float64
rounding bars: 1e-12 relative on volume, centre and d_max, 1e-10 on the
semi-axes and D (cancellation in the semi-axis combinations)."""
import numpy as np
import pytest

from gpu_util import require_gpu
from oracle import shape as oshape
from synth.configs import template_batch, uneven_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _check(cb, b, y_host, d_ref):
    import torch
    out = cb.shape(cb.to_device(y_host), d_ref).cpu().numpy()
    torch.cuda.synchronize()
    for c in range(b.n_cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        t0, t1 = b.tet_off[c], b.tet_off[c + 1]
        ref = oshape.cell_shape(b.x[n0:n1], y_host[n0:n1].astype(np.float64),
                                b.tets[t0:t1], d_ref[c])
        r = out[c]
        scale = np.abs(y_host[n0:n1]).max()
        assert abs(r[0] - ref["volume"]) <= 1e-12 * abs(ref["volume"])
        assert np.abs(r[1:4] - ref["com"]).max() <= 1e-12 * scale
        assert np.abs(r[4:7] - ref["axes"]).max() <= 1e-10 * ref["axes"].max()
        assert abs(r[7] - ref["D"]) <= 1e-10
        assert abs(r[8] - ref["d_max"]) <= 1e-12 * ref["d_max"]
        assert abs(r[9] - ref["strain"]) <= 1e-12 * max(1.0, abs(ref["strain"]))
    return out


def test_shape_against_oracle():
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=5, seed=81, tet_lo=500, tet_hi=9000, ladder=5)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    d_ref = np.linspace(1.8, 2.4, b.n_cells)
    out = _check(cb, b, b.y, d_ref)
    # far from the origin and rotated: same shape
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    y2 = (b.y.astype(np.float64) @ Q.T + np.array([30.0, -12.0, 7.0])
          ).astype(np.float32)
    out2 = _check(cb, b, y2, d_ref)
    assert np.abs(out2[:, 4:9] - out[:, 4:9]).max() <= 1e-5
    # bitwise repeatable
    again = cb.shape(cb.to_device(b.y), d_ref).cpu().numpy()
    assert np.array_equal(again, out)
    # without d_ref the strain is NaN
    assert np.isnan(cb.shape(cb.to_device(b.y)).cpu().numpy()[:, 9]).all()


def test_shape_of_shared_mesh_batch():
    from paper_2003_03130_amd import CellBatch
    b = template_batch(6, 700, seed=82)
    n, m = b.info["template_nodes"], b.info["template_tets"]
    tp = CellBatch.template(b.n_cells, b.x[:n], b.tets[:m])
    ds = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    d_ref = np.full(b.n_cells, 2.0)
    o1 = _check(tp, b, b.y, d_ref)
    o2 = ds.shape(ds.to_device(b.y), d_ref).cpu().numpy()
    assert np.array_equal(o1, o2)


def test_large_cell_many_pair_blocks():
    """One 20k-node cell: 79 x 80 / 2 node-pair blocks, several hundred
    tiles."""
    from paper_2003_03130_amd import CellBatch
    from synth.configs import paper_sphere_case
    c = paper_sphere_case(2003)
    cb = CellBatch.single(c.x, c.tets)
    out = cb.shape(cb.to_device(c.y), 2.0).cpu().numpy()[0]
    ref = oshape.cell_shape(c.x, c.y.astype(np.float64), c.tets, 2.0)
    assert abs(out[0] - ref["volume"]) <= 1e-12 * ref["volume"]
    assert np.abs(out[4:7] - ref["axes"]).max() <= 1e-10
    assert abs(out[8] - ref["d_max"]) <= 1e-12 * ref["d_max"]


def _interior_nodes(tets, n):
    """Nodes of a cell none of whose faces lies on the boundary (every face
    shared by exactly two tetrahedra)."""
    f = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                                tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]]), axis=1)
    _, inv, cnt = np.unique(f, axis=0, return_inverse=True, return_counts=True)
    bad = np.zeros(n, bool)
    bad[f[cnt[inv.ravel()] != 2].ravel()] = True
    used = np.zeros(n, bool)
    used[tets.ravel()] = True
    return np.flatnonzero(used & ~bad)


def test_inverted_cell_searches_all_node_pairs():
    """The pair search takes only boundary (and non-manifold or unused)
    nodes while a cell has no inverted tetrahedron; two interior nodes moved
    far out on opposite sides invert their tetrahedra and become the
    farthest pair, which the search must still find (the other cells keep
    the restricted search)."""
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=3, seed=83, tet_lo=8000, tet_hi=12000, ladder=3)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    y = b.y.copy()
    c = 1
    n0, n1 = b.node_off[c], b.node_off[c + 1]
    t0, t1 = b.tet_off[c], b.tet_off[c + 1]
    inner = _interior_nodes(b.tets[t0:t1], n1 - n0)
    centre = b.x[n0:n1].mean(axis=0)
    near = inner[np.argsort(np.linalg.norm(b.x[n0:n1][inner] - centre, axis=1))[:2]]
    y[n0 + near[0]] = centre + np.array([5.0, 0.0, 0.0])
    y[n0 + near[1]] = centre - np.array([5.0, 0.0, 0.0])
    d_ref = np.full(b.n_cells, 2.0)
    out = _check(cb, b, y, d_ref)
    assert abs(out[c, 8] - 10.0) <= 1e-5


def test_duplicated_tetrahedron_keeps_its_nodes_in_the_search():
    """A face shared by two tetrahedra on the same side (a duplicated
    tetrahedron) does not make its nodes interior: a cell of a doubled unit
    tetrahedron and a separate one 3 R away, nothing inverted, has its
    farthest pair between the two parts."""
    from paper_2003_03130_amd import CellBatch
    from synth.configs import batch_from_cells, Cell
    unit = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64)
    x = np.concatenate([unit, unit + np.array([3.0, 0.0, 0.0])])
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 3], [4, 5, 6, 7]], np.int32)
    b = batch_from_cells([Cell(x, tets, x.astype(np.float32), (1.0, 10.0, 0.5))])
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    out = _check(cb, b, b.y, np.array([2.0]))
    assert abs(out[0, 8] - np.sqrt(17.0)) <= 1e-12 * np.sqrt(17.0)
