"""Material regions on the GPU (cm_batch_create_regions): every tetrahedron
carries a region id and every (cell, region) its own (mu, kappa, w).
Against the FP64 oracle's region composition (tolerance 1e-5, as the
single-material tests); equal parameters in every region reduce to the
single-material cell; a one-region batch is bitwise the plain batch; a
shared-mesh batch with regions is bitwise the distinct-array one."""
import numpy as np
import pytest

import oracle
from gpu_util import force_rel_err, require_gpu
from synth.configs import (cotangent, radial_regions, random_theta,
                           template_batch, uneven_batch)

pytestmark = pytest.mark.gpu
TOL = 1e-5
R = 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _regions(b):
    return np.concatenate([
        radial_regions(b.x[b.node_off[c]:b.node_off[c + 1]],
                       b.tets[b.tet_off[c]:b.tet_off[c + 1]])
        for c in range(b.n_cells)])


def _thetas(n_cells, seed):
    rng = np.random.default_rng(seed)
    return np.array([random_theta(rng) for _ in range(n_cells * R)])


def _run(cb, b, th, v, eb):
    import torch
    cb.set_params(th[:, 0], th[:, 1], th[:, 2])
    y = cb.to_device(b.y)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    f, E = cb.forces(y, n_inverted=ninv)
    yb, tb = cb.backward(y, cb.to_device(v), eb)
    torch.cuda.synchronize()
    return (cb.to_host(f), E.cpu().numpy(), ninv.cpu().numpy(),
            cb.to_host(yb), tb.cpu().numpy().reshape(-1, 3))


def test_regions_against_oracle():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=4, seed=61, tet_lo=3000, tet_hi=9000, ladder=4)
    reg = _regions(b)
    th = _thetas(b.n_cells, 62)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, regions=reg,
                   n_regions=R)
    assert cb.n_mat == b.n_cells * R and cb.info["n_regions"] == R
    v = cotangent(b.n_nodes, 63)
    eb = torch.linspace(0.3, 0.9, b.n_cells, dtype=torch.float64,
                        device=cb.device)
    f, E, ninv, yb, tb = _run(cb, b, th, v, eb)
    ebh = eb.cpu().numpy()
    for c in range(b.n_cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        t0, t1 = b.tet_off[c], b.tet_off[c + 1]
        rm = oracle.RegionMesh(b.x[n0:n1], b.tets[t0:t1], reg[t0:t1], R)
        yd = b.y[n0:n1].astype(np.float64)
        thc = th[c * R:(c + 1) * R]
        fo, Eo, no = rm.forces(yd, thc)
        assert force_rel_err(f[n0:n1], fo) <= TOL
        assert abs(E[c] - Eo) <= 1e-6 * abs(Eo)
        assert ninv[c] == no
        yo, to = rm.backward(yd, thc, v[n0:n1].astype(np.float64), ebh[c])
        assert np.abs(yb[n0:n1] - yo).max() <= TOL * np.abs(yo).max()
        assert np.abs(tb[c * R:(c + 1) * R] - to).max() <= TOL * np.abs(to).max()


def test_equal_parameters_reduce_to_one_material():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=3, seed=64, tet_lo=2000, tet_hi=6000, ladder=3)
    reg = _regions(b)
    v = cotangent(b.n_nodes, 65)
    eb = torch.full((b.n_cells,), 0.4, dtype=torch.float64, device="cuda")
    plain = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    f0, E0, n0, y0, t0 = _run(plain, b, b.theta, v, eb)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, regions=reg,
                   n_regions=R)
    th = np.repeat(b.theta, R, axis=0)
    f, E, ninv, yb, tb = _run(cb, b, th, v, eb)
    # same quantities, computed with other tiles (other vertex orders in the
    # chunks, so other float32 roundings of B) and summation orders: equal
    # within the parity bars
    assert force_rel_err(f, f0.astype(np.float64)) <= TOL
    assert np.abs(E - E0).max() <= 1e-6 * np.abs(E0).max()
    assert np.array_equal(ninv, n0)
    assert np.abs(yb - y0).max() <= TOL * np.abs(y0).max()
    # the gradient of a shared parameter is the sum over the regions
    assert np.abs(tb.reshape(b.n_cells, R, 3).sum(1) - t0).max() \
        <= TOL * np.abs(t0).max()
    # all tetrahedra in region 0 of a one-region batch: bitwise the plain one
    one = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                    regions=np.zeros(b.n_tets, np.uint8), n_regions=1)
    got = _run(one, b, b.theta, v, eb)
    for g, w in zip(got, (f0, E0, n0, y0, t0)):
        assert np.array_equal(g, w)


def test_empty_region_and_template_with_regions():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = template_batch(4, 900, seed=66)
    n, m = b.info["template_nodes"], b.info["template_tets"]
    reg1 = radial_regions(b.x[:n], b.tets[:m])
    Rx = R + 1  # region 3 has no tetrahedra
    th = np.array([random_theta(np.random.default_rng(67 + k))
                   for k in range(b.n_cells * Rx)])
    v = cotangent(b.n_nodes, 68)
    eb = torch.full((b.n_cells,), 0.5, dtype=torch.float64, device="cuda")
    tp = CellBatch.template(b.n_cells, b.x[:n], b.tets[:m], regions=reg1,
                            n_regions=Rx)
    ds = CellBatch(b.node_off, b.tet_off, b.x, b.tets,
                   regions=np.tile(reg1, b.n_cells), n_regions=Rx)
    got, want = _run(tp, b, th, v, eb), _run(ds, b, th, v, eb)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    tb = got[4].reshape(b.n_cells, Rx, 3)
    assert (tb[:, 3] == 0).all() and (np.abs(tb[:, :3]) > 0).all()


def test_plate_adjoint_accumulates_every_region():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=2, seed=69, tet_lo=1000, tet_hi=2000, ladder=2)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, regions=_regions(b),
                   n_regions=R)
    cb.set_params(*_thetas(b.n_cells, 70).T)
    y = cb.to_device(b.y)
    lam_next = cb.to_device(cotangent(b.n_nodes, 71))
    ybar_el, tb_el = cb.backward(y, lam_next)
    plate = torch.tensor([[0.8, -1.0]] * b.n_cells, dtype=torch.float64,
                         device=cb.device)
    acc0 = torch.linspace(-1, 1, 3 * cb.n_mat, dtype=torch.float64,
                          device=cb.device)
    acc = acc0.clone()
    lam = cb.empty_nodes()
    cb.plate_step_adjoint(y, lam_next, ybar_el, plate, 100.0, 4e-3, lam,
                          None, None, 1.0, tb_el, acc)
    torch.cuda.synchronize()
    ref = acc0 + 4e-3 * tb_el
    assert (acc - ref).abs().max() <= 1e-14 * ref.abs().max()
