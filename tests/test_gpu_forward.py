"""Forward parity of the HIP kernels against the FP64 oracle (GPU).

Tolerances: forces max|f_gpu - f_oracle| / max|f_oracle| <= 1e-5, energy
relative error <= 1e-6 (the float32 device path against the float64 oracle on
the same float32 positions).
"""
import numpy as np
import pytest

from gpu_util import force_rel_err, oracle_cell, rel_err, require_gpu, run_cell
from synth.configs import paper_sphere_case, small_sphere_case, uneven_batch

pytestmark = pytest.mark.gpu
F_TOL, E_TOL = 1e-5, 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("seed", range(1000, 1016))
def test_small_sphere_parity(seed):
    c = small_sphere_case(seed)
    _, f, E, ninv = run_cell(c)
    _, (fo, Eo, ninv_o) = oracle_cell(c)
    print(f"seed {seed}: force err {force_rel_err(f, fo):.2e} energy err "
          f"{rel_err(E, Eo):.2e}", flush=True)
    assert force_rel_err(f, fo) <= F_TOL
    assert rel_err(E, Eo) <= E_TOL
    assert ninv == ninv_o == 0


@pytest.mark.parametrize("seed", range(2000, 2016))
def test_paper_sphere_parity(seed):
    c = paper_sphere_case(seed)
    _, f, E, ninv = run_cell(c)
    _, (fo, Eo, ninv_o) = oracle_cell(c)
    print(f"seed {seed}: force err {force_rel_err(f, fo):.2e} energy err "
          f"{rel_err(E, Eo):.2e}", flush=True)
    assert force_rel_err(f, fo) <= F_TOL
    assert rel_err(E, Eo) <= E_TOL
    assert ninv == ninv_o


@pytest.mark.parametrize("order,tile", [(0, 64), (1, 320), (2, 4096),
                                        (2, 1024), (1, 2048)])
def test_orders_and_tile_sizes(order, tile):
    c = small_sphere_case(1003)
    _, f, E, _ = run_cell(c, order=order, tile_tets=tile)
    _, (fo, Eo, _) = oracle_cell(c)
    assert force_rel_err(f, fo) <= F_TOL and rel_err(E, Eo) <= E_TOL


def test_reference_configuration_gives_zero_force():
    c = small_sphere_case(1000)
    c.y = c.x.astype(np.float32)
    _, f, E, _ = run_cell(c)
    from synth.mesh import mean_edge_length
    h = mean_edge_length(c.x, c.tets)
    # only float32 rounding of the positions remains
    assert np.abs(f).max() <= 1e-5 * c.theta[0] * h * h
    assert abs(E) <= 1e-9


def test_inverted_tetrahedra_are_counted_and_match_the_oracle():
    c = small_sphere_case(1001)
    y = c.y.astype(np.float64)
    t = c.tets[123]
    # push one vertex through the opposite face
    face = y[t[1:]].mean(0)
    y[t[0]] = face + 0.6 * (face - y[t[0]])
    c.y = y.astype(np.float32)
    _, f, E, ninv = run_cell(c)
    _, (fo, Eo, ninv_o) = oracle_cell(c)
    assert ninv == ninv_o >= 1
    assert np.isfinite(f).all() and np.isfinite(E)
    assert force_rel_err(f, fo) <= F_TOL and rel_err(E, Eo) <= E_TOL


def test_bitwise_repeatable_and_launch_independent():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=24, seed=99, tet_lo=500, tet_hi=8000, ladder=6)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, tile_tets=512)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    f0, E0 = cb.forces(y)
    ref_f, ref_E = f0.clone(), E0.clone()
    from paper_2003_03130_amd import CellmechError
    tried = 0
    for waves, bpcu in [(1, 0), (2, 0), (4, 1), (8, 2), (1, 4), (2, 16)]:
        try:
            cb.set_launch(waves, bpcu)
        except CellmechError:  # does not fit in LDS for this tile size
            continue
        tried += 1
        f1, E1 = cb.forces(y)
        assert torch.equal(f1, ref_f) and torch.equal(E1, ref_E), (waves, bpcu)
    assert tried >= 4
    f2, E2 = cb.forces(y, percell=True)
    assert torch.equal(f2, ref_f) and torch.equal(E2, ref_E)


def test_batch_equals_single_cells():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=6, seed=5, tet_lo=500, tet_hi=5000, ladder=4)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    fb, Eb = cb.forces(cb.to_device(b.y))
    fb = cb.to_host(fb)
    Eb = Eb.cpu().numpy()
    for c in range(b.n_cells):
        cell = b.cell(c)
        _, f, E, _ = run_cell(cell)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        assert np.array_equal(f, fb[n0:n1]) and E == Eb[c]


def test_graph_replay_matches_eager():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=8, seed=6, tet_lo=500, tet_hi=5000, ladder=4)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    fe, Ee = cb.forces(y)
    fe, Ee = fe.clone(), Ee.clone()
    f = cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=cb.device)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cb.graph_capture(0, y, f, E, stream=s)
    for _ in range(4):
        f.zero_()
        E.zero_()
        cb.graph_launch(stream=s)
        s.synchronize()
        assert torch.equal(f, fe) and torch.equal(E, Ee)
        fe2, _ = cb.forces(y)  # eager work between replays
        torch.cuda.synchronize()


def test_state_and_parameter_errors():
    from paper_2003_03130_amd import CellBatch, CellmechError
    from paper_2003_03130_amd import _native as nat
    c = small_sphere_case(1000)
    cb = CellBatch.single(c.x, c.tets)
    y = cb.to_device(c.y)
    with pytest.raises(CellmechError) as ei:
        cb.forces(y)
    assert ei.value.status == nat.CM_ESTATE
    for bad in [(-1.0, 1.0, 0.5), (1.0, -2.0, 0.5), (1.0, 1.0, 1.5),
                (float("nan"), 1.0, 0.5)]:
        with pytest.raises(CellmechError) as ei:
            cb.set_params(*bad)
        assert ei.value.status == nat.CM_EINVAL
    with pytest.raises(CellmechError):
        cb.set_launch(3, 0)


def _tiny_cells():
    """A 1-tetrahedron cell, two tetrahedra sharing a face, a 5-tetrahedron
    cube split, and a 1,000-node sphere: tiles of one chunk with mostly empty
    lanes beside full tiles."""
    from synth.configs import Cell
    rng = np.random.default_rng(77)
    cube = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0],
                     [1, 0, 1], [0, 1, 1], [1, 1, 1]], np.float64)
    meshes = [
        (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64),
         np.array([[0, 1, 2, 3]], np.int32)),
        (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]],
                  np.float64),
         np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)),
        (cube, np.array([[0, 1, 2, 3], [1, 4, 2, 7], [1, 3, 5, 7],
                         [2, 3, 6, 7], [1, 2, 3, 7]], np.int32)),
    ]
    cells = []
    for k, (x, tets) in enumerate(meshes):
        A = np.eye(3) + 0.2 * rng.standard_normal((3, 3))
        y = x @ A.T + 0.02 * rng.standard_normal(x.shape)
        cells.append(Cell(x, tets, y.astype(np.float32), (1.0 + k, 15.0, 0.3)))
    cells.append(small_sphere_case(1007))
    return cells


def test_tiny_and_ragged_cells_against_the_oracle():
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import batch_from_cells
    cells = _tiny_cells()
    b = batch_from_cells(cells)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    f, E = cb.forces(y, n_inverted=ninv)
    from synth.configs import cotangent
    v = cotangent(b.n_nodes, 78)
    eb = torch.tensor([0.4, -0.2, 0.9, 0.1], dtype=torch.float64, device=cb.device)
    yb, tb = cb.backward(y, cb.to_device(v), eb)
    f, E, yb = cb.to_host(f), E.cpu().numpy(), cb.to_host(yb)
    tb = tb.cpu().numpy().reshape(-1, 3)
    for c, cell in enumerate(cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m, (fo, Eo, _) = oracle_cell(cell)
        assert force_rel_err(f[n0:n1], fo) <= F_TOL, c
        assert rel_err(E[c], Eo) <= E_TOL, c
        yo, to = m.backward(cell.y.astype(np.float64), cell.theta,
                            v[n0:n1].astype(np.float64), float(eb[c]))
        assert force_rel_err(yb[n0:n1], yo) <= F_TOL, c
        assert force_rel_err(tb[c], to) <= F_TOL, c
