"""Forward and backward in one tile pass (cm_forces_and_backward) on the GPU.
Its outputs -- forces, energies, inverted counts, ybar and the parameter
gradient -- must equal bit for bit those of cm_forces followed by
cm_forces_backward (the same per-tetrahedron arithmetic and summation
orders), under every tile size, order, launch shape, material regions and
shared-mesh batches, and match the FP64 oracle to the tolerances of the
separate passes (forces, ybar, thetabar max-normalised 1e-5, energy 1e-6)."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import force_rel_err, rel_err, require_gpu
from synth.configs import (cotangent, radial_regions, random_theta,
                           small_sphere_case, template_batch, uneven_batch)

pytestmark = pytest.mark.gpu
TOL, E_TOL = 1e-5, 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _separate(cb, y, fb, eb, n_cells):
    import torch
    ninv = torch.zeros(n_cells, dtype=torch.int32, device=cb.device)
    f, E = cb.forces(y, n_inverted=ninv)
    yb, tb = cb.backward(y, fb, eb)
    torch.cuda.synchronize()
    return [t.clone() for t in (f, E, ninv, yb, tb)]


def _fused(cb, y, fb, eb, n_cells):
    import torch
    ninv = torch.full((n_cells,), -1, dtype=torch.int32, device=cb.device)
    f, yb = cb.empty_nodes(), cb.empty_nodes()
    f.fill_(float("nan"))
    yb.fill_(float("nan"))
    f, E, yb, tb = cb.forces_and_backward(y, fb, eb, f=f, n_inverted=ninv,
                                          ybar=yb)
    torch.cuda.synchronize()
    return [f, E, ninv, yb, tb]


def _assert_equal(got, want, what=""):
    import torch
    names = ("f", "energy", "n_inverted", "ybar", "thetabar")
    for n, g, w in zip(names, got, want):
        assert torch.equal(g, w), f"{what} {n} differs"


@pytest.mark.parametrize("seed", [1000, 1007])
def test_fused_against_oracle(seed):
    import torch
    from paper_2003_03130_amd import CellBatch
    c = small_sphere_case(seed)
    v = cotangent(c.n_nodes, seed + 1)
    cb = CellBatch.single(c.x, c.tets)
    cb.set_params(*c.theta)
    y = cb.to_device(c.y)
    eb = torch.tensor([0.4], dtype=torch.float64, device=cb.device)
    f, E, ninv, yb, tb = _fused(cb, y, cb.to_device(v), eb, 1)
    m = oracle.OracleMesh(c.x, c.tets)
    y64 = c.y.astype(np.float64)
    fo, Eo, no = m.forces(y64, c.theta)
    yo, to = m.backward(y64, c.theta, v.astype(np.float64), 0.4)
    errs = (force_rel_err(cb.to_host(f), fo), rel_err(E.item(), Eo),
            force_rel_err(cb.to_host(yb), yo), force_rel_err(tb.cpu().numpy(), to))
    print(f"seed {seed}: force, energy, ybar, thetabar {errs}", flush=True)
    assert errs[0] <= TOL and errs[1] <= E_TOL
    assert errs[2] <= TOL and errs[3] <= TOL
    assert ninv.item() == no


def test_fused_equals_separate_passes_on_an_uneven_batch():
    """Cells of uneven size, each with its own cotangents and energy
    cotangent, under several launch shapes (a shape whose LDS does not fit
    runs with fewer waves per workgroup; results do not change)."""
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=12, seed=71, tet_lo=500, tet_hi=8000, ladder=5)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    fb = cb.to_device(cotangent(b.n_nodes, 72))
    eb = torch.linspace(-0.5, 1.5, b.n_cells, dtype=torch.float64, device=cb.device)
    want = _separate(cb, y, fb, eb, b.n_cells)
    from paper_2003_03130_amd import CellmechError
    tried = 0
    for waves, bpcu in [(1, 0), (2, 0), (4, 0), (8, 0), (1, 2), (2, 4)]:
        try:
            cb.set_launch(waves, bpcu)  # refused where the separate passes' LDS does not fit
        except CellmechError:
            continue
        print(f"launch {waves},{bpcu}", flush=True)
        _assert_equal(_fused(cb, y, fb, eb, b.n_cells), want, f"launch {waves},{bpcu}")
        tried += 1
    assert tried >= 4


@pytest.mark.parametrize("order,tile", [(0, 64), (3, 192), (1, 320), (3, 1024),
                                        (2, 4096)])
def test_fused_orders_and_tile_sizes(order, tile):
    """Tiles of 1, 3, 5, 16 and 64 chunks under every tile order: bitwise
    the separate passes, and within the oracle's tolerance."""
    import torch
    from paper_2003_03130_amd import CellBatch
    c = small_sphere_case(1003)
    v = cotangent(c.n_nodes, 1004)
    cb = CellBatch.single(c.x, c.tets, tile_tets=tile, order=order)
    cb.set_params(*c.theta)
    y = cb.to_device(c.y)
    fb = cb.to_device(v)
    eb = torch.tensor([-0.7], dtype=torch.float64, device=cb.device)
    try:
        got = _fused(cb, y, fb, eb, 1)
    except RuntimeError as e:
        if "LDS" not in str(e):
            raise
        pytest.skip(str(e))  # tile does not fit the LDS budget
    _assert_equal(got, _separate(cb, y, fb, eb, 1), f"order {order} tile {tile}")
    m = oracle.OracleMesh(c.x, c.tets)
    yo, to = m.backward(c.y.astype(np.float64), c.theta, v.astype(np.float64), -0.7)
    assert force_rel_err(cb.to_host(got[3]), yo) <= TOL
    assert force_rel_err(got[4].cpu().numpy(), to) <= TOL


def test_fused_hessian_vector_product_alone():
    """No energy cotangent and no parameter gradient (null ebar, thetabar,
    n_inverted through the C-ABI): the adjoint half is the Hessian-vector
    product alone, as in cm_forces_backward with the same nulls."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    c = small_sphere_case(1011)
    cb = CellBatch.single(c.x, c.tets)
    cb.set_params(*c.theta)
    y = cb.to_device(c.y)
    fb = cb.to_device(cotangent(c.n_nodes, 1012))
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    f1, yb1, f2, yb2 = (cb.empty_nodes() for _ in range(4))
    E1 = torch.empty(1, dtype=torch.float64, device=cb.device)
    E2 = torch.empty_like(E1)
    lib = nat.lib()
    nat.check(lib.cm_forces(cb._h, p(y), p(f1), p(E1), None, st))
    nat.check(lib.cm_forces_backward(cb._h, p(y), p(fb), None, p(yb1), None, st))
    nat.check(lib.cm_forces_and_backward(cb._h, p(y), p(f2), p(E2), None, p(fb), None,
                                         p(yb2), None, st))
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(E1, E2) and torch.equal(yb1, yb2)
    m = oracle.OracleMesh(c.x, c.tets)
    yo, _ = m.backward(c.y.astype(np.float64), c.theta,
                       cb.to_host(fb).astype(np.float64), 0.0)
    assert force_rel_err(cb.to_host(yb2), yo) <= TOL


def test_fused_with_regions_and_shared_mesh():
    """Material regions (three radial regions per cell, each with its own
    parameters) on a shared-mesh batch and on the same cells in distinct
    arrays: the fused pass equals the separate passes on both."""
    import torch
    from paper_2003_03130_amd import CellBatch
    b = template_batch(5, 1500, seed=81)
    n, m = b.info["template_nodes"], b.info["template_tets"]
    reg1 = radial_regions(b.x[:n], b.tets[:m])
    rng = np.random.default_rng(82)
    th = np.array([random_theta(rng) for _ in range(b.n_cells * 3)])
    tp = CellBatch.template(b.n_cells, b.x[:n], b.tets[:m], regions=reg1, n_regions=3)
    ds = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                   regions=np.tile(reg1, b.n_cells), n_regions=3)
    v = cotangent(b.n_nodes, 83)
    outs = []
    for cb in (tp, ds):
        cb.set_params(th[:, 0], th[:, 1], th[:, 2])
        y = cb.to_device(b.y)
        fb = cb.to_device(v)
        eb = torch.linspace(0.1, 0.9, b.n_cells, dtype=torch.float64, device=cb.device)
        got = _fused(cb, y, fb, eb, b.n_cells)
        _assert_equal(got, _separate(cb, y, fb, eb, b.n_cells))
        outs.append([cb.to_host(got[0]), got[1].cpu(), got[2].cpu(),
                     cb.to_host(got[3]), got[4].cpu()])
    for g, w in zip(*outs):
        assert np.array_equal(np.asarray(g), np.asarray(w))


def test_fused_graph_replays_and_aliasing_rejected():
    """Graph mode 6 (the fused pass) replayed three times, with eager work
    and synchronisations between the replays: every replay equals the
    separate passes.  Aliased outputs are refused before any launch."""
    import torch
    from paper_2003_03130_amd import CellBatch, CellmechError
    b = uneven_batch(n_cells=6, seed=91, tet_lo=800, tet_hi=4000, ladder=3)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    fb = cb.to_device(cotangent(b.n_nodes, 92))
    eb = torch.linspace(0.2, 0.7, b.n_cells, dtype=torch.float64, device=cb.device)
    want = _separate(cb, y, fb, eb, b.n_cells)
    f, yb = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=cb.device)
    ninv = torch.empty(b.n_cells, dtype=torch.int32, device=cb.device)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=cb.device)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cb.graph_capture(6, y, f, E, ninv, fb, eb, yb, tb, stream=s)
    for rep in range(3):
        for t in (f, yb):
            t.fill_(float("nan"))
        _separate(cb, y, fb, eb, b.n_cells)  # eager work between replays
        cb.graph_launch(stream=s)
        torch.cuda.synchronize()
        _assert_equal([f, E, ninv, yb, tb], want, f"replay {rep}")
    with pytest.raises(CellmechError, match="alias"):
        cb.forces_and_backward(y, fb, eb, f=f, ybar=f)
    with pytest.raises(CellmechError, match="alias"):
        cb.forces_and_backward(y, fb, eb, f=fb)


def test_fused_node_of_no_tetrahedron():
    """A node that no tetrahedron uses is a shared node with no slot: the
    fused finalize writes zero force and zero ybar for it, as the separate
    passes do, and every other output is bitwise theirs."""
    import torch
    from paper_2003_03130_amd import CellBatch
    c0, c1 = small_sphere_case(1021), small_sphere_case(1022)
    extra = np.array([[0.0, 0.0, 2.0]])
    x = np.concatenate([c0.x, extra, c1.x])
    y = np.concatenate([c0.y, extra, c1.y]).astype(np.float32)
    n0 = len(c0.x) + 1
    tets = np.concatenate([c0.tets, c1.tets])
    cb = CellBatch([0, n0, n0 + len(c1.x)], [0, len(c0.tets), len(tets)], x, tets)
    cb.set_params([c0.theta[0], c1.theta[0]], [c0.theta[1], c1.theta[1]],
                  [c0.theta[2], c1.theta[2]])
    yd = cb.to_device(y)
    fb = cb.to_device(cotangent(cb.n_nodes, 1023))
    eb = torch.tensor([0.3, 0.6], dtype=torch.float64, device=cb.device)
    want = _separate(cb, yd, fb, eb, 2)
    got = _fused(cb, yd, fb, eb, 2)
    _assert_equal(got, want)
    assert not cb.to_host(got[0])[len(c0.x)].any()
    assert not cb.to_host(got[3])[len(c0.x)].any()


def test_fused_tiny_and_ragged_cells():
    """A 1-tetrahedron cell, two tetrahedra sharing a face, a 5-tetrahedron
    cube and a sphere in one batch (tiles of one chunk with mostly empty
    lanes beside full tiles): bitwise the separate passes, and the oracle's
    forces, energies, ybar and thetabar per cell."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import batch_from_cells
    from test_gpu_forward import _tiny_cells
    cells = _tiny_cells()
    b = batch_from_cells(cells)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    v = cotangent(b.n_nodes, 79)
    fb = cb.to_device(v)
    ebh = np.array([0.4, -0.2, 0.9, 0.1])
    eb = torch.tensor(ebh, dtype=torch.float64, device=cb.device)
    got = _fused(cb, y, fb, eb, b.n_cells)
    _assert_equal(got, _separate(cb, y, fb, eb, b.n_cells))
    f, E, yb = cb.to_host(got[0]), got[1].cpu().numpy(), cb.to_host(got[3])
    tb = got[4].cpu().numpy().reshape(-1, 3)
    for c, cell in enumerate(cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        y64 = cell.y.astype(np.float64)
        fo, Eo, _ = m.forces(y64, cell.theta)
        yo, to = m.backward(y64, cell.theta, v[n0:n1].astype(np.float64), float(ebh[c]))
        assert force_rel_err(f[n0:n1], fo) <= TOL, c
        assert rel_err(E[c], Eo) <= E_TOL, c
        assert force_rel_err(yb[n0:n1], yo) <= TOL, c
        assert force_rel_err(tb[c], to) <= TOL, c
