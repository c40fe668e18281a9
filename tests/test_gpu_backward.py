"""Backward (adjoint) parity of the HIP kernels (GPU): Hessian-vector product
and parameter gradient against the FP64 oracle's dual-number reference and
FP64 central differences.  Tolerance: max-normalised error <= 1e-5."""
import numpy as np
import pytest

import oracle
from gpu_util import force_rel_err, require_gpu
from synth.configs import (cotangent, paper_sphere_case, small_sphere_case,
                           uneven_batch)

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _gpu_backward(cell, fbar, ebar, **kw):
    import torch
    from paper_2003_03130_amd import CellBatch
    cb = CellBatch.single(cell.x, cell.tets, **kw)
    cb.set_params(*cell.theta)
    y = cb.to_device(cell.y)
    fb = cb.to_device(fbar) if fbar is not None else None
    eb = (torch.tensor([ebar], dtype=torch.float64, device=cb.device)
          if ebar is not None else None)
    ybar, tb = cb.backward(y, fb, eb)
    torch.cuda.synchronize()
    return cb, cb.to_host(ybar), tb.cpu().numpy()


def _max_rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / np.abs(b).max())


@pytest.mark.parametrize("seed", [1000, 1005, 1010])
def test_small_sphere_backward(seed):
    c = small_sphere_case(seed)
    v = cotangent(c.n_nodes, seed + 1)
    _, yb, tb = _gpu_backward(c, v, 0.3)
    m = oracle.OracleMesh(c.x, c.tets)
    yo, to = m.backward(c.y.astype(np.float64), c.theta, v, 0.3)
    print(f"seed {seed}: ybar {_max_rel(yb, yo):.2e} thetabar "
          f"{_max_rel(tb, to):.2e}", flush=True)
    assert _max_rel(yb, yo) <= TOL
    assert _max_rel(tb, to) <= TOL


@pytest.mark.parametrize("order,tile", [(0, 64), (3, 128), (3, 192), (1, 320),
                                        (3, 1024), (2, 4096)])
def test_backward_orders_and_tile_sizes(order, tile):
    """Tiles of 1, 2, 3, 5, 16 and 64 chunks (one, even and odd chunk counts
    in the kernel's two-register-set chunk pipeline) under every tile order."""
    c = small_sphere_case(1003)
    v = cotangent(c.n_nodes, 1004)
    try:
        _, yb, tb = _gpu_backward(c, v, -0.7, tile_tets=tile, order=order)
    except RuntimeError as e:
        if "LDS" not in str(e):
            raise
        pytest.skip(str(e))  # tile does not fit the LDS budget
    m = oracle.OracleMesh(c.x, c.tets)
    yo, to = m.backward(c.y.astype(np.float64), c.theta, v, -0.7)
    print(f"order {order} tile {tile}: ybar {_max_rel(yb, yo):.2e} "
          f"thetabar {_max_rel(tb, to):.2e}", flush=True)
    assert _max_rel(yb, yo) <= TOL
    assert _max_rel(tb, to) <= TOL


def test_differentiation_config_against_oracle_and_fd():
    """One ~110k-tet sphere, L = sum v.f with v ~ N(0, 1): ybar and
    dL/d(mu, kappa, w) against the oracle and FP64 central differences
    (h = 1e-6)."""
    c = paper_sphere_case(4000)
    v = cotangent(c.n_nodes, 4001)
    _, yb, tb = _gpu_backward(c, v, None)
    m = oracle.OracleMesh(c.x, c.tets)
    y64 = c.y.astype(np.float64)
    yo, to = m.backward(y64, c.theta, v, 0.0)
    print(f"ybar {_max_rel(yb, yo):.2e} thetabar {_max_rel(tb, to):.2e}")
    assert _max_rel(yb, yo) <= TOL and _max_rel(tb, to) <= TOL
    h = 1e-6
    fd_y = (m.forces(y64 + h * v, c.theta)[0]
            - m.forces(y64 - h * v, c.theta)[0]) / (2 * h)
    assert _max_rel(yb, fd_y) <= TOL
    fd_t = []
    for k in range(3):
        tp, tm = list(c.theta), list(c.theta)
        hk = h * max(1.0, abs(c.theta[k]))
        tp[k] += hk
        tm[k] -= hk
        fd_t.append(((v * m.forces(y64, tp)[0]).sum()
                     - (v * m.forces(y64, tm)[0]).sum()) / (2 * hk))
    fd_t = np.array(fd_t)
    print("thetabar gpu", tb, "fd", fd_t)
    assert _max_rel(tb, fd_t) <= TOL


def test_energy_cotangent_gives_minus_forces():
    import torch
    c = small_sphere_case(1002)
    cb, yb, tb = _gpu_backward(c, None, 1.0)
    f, E = cb.forces(cb.to_device(c.y))
    assert force_rel_err(yb, -cb.to_host(f).astype(np.float64)) <= 1e-6
    m = oracle.OracleMesh(c.x, c.tets)
    mu, kappa, w = c.theta
    y64 = c.y.astype(np.float64)
    _, EI, _ = m.forces(y64, (1.0, 0.0, 1.0))
    _, EK, _ = m.forces(y64, (1.0, 0.0, 0.0))
    _, EJ, _ = m.forces(y64, (0.0, 1.0, 0.5))
    want = np.array([w * EI + (1 - w) * EK, EJ, mu * (EI - EK)])
    assert _max_rel(tb, want) <= TOL


def test_hvp_symmetry_on_gpu():
    import torch
    from paper_2003_03130_amd import CellBatch
    c = paper_sphere_case(2003)
    cb = CellBatch.single(c.x, c.tets)
    cb.set_params(*c.theta)
    y = cb.to_device(c.y)
    u = cb.to_device(cotangent(c.n_nodes, 1))
    v = cb.to_device(cotangent(c.n_nodes, 2))
    Hu, _ = cb.backward(y, u)
    Hv, _ = cb.backward(y, v)
    a = float((u.double() * Hv.double()).sum())
    b = float((v.double() * Hu.double()).sum())
    scale = float((u.double() * Hv.double()).abs().sum())
    assert abs(a - b) <= 1e-5 * scale


def test_thetabar_linearity_closed_form_on_gpu():
    """dL/dtheta from the backward kernel equals the closed form obtained from
    three forward calls, since f is linear in (mu1, mu2, kappa)."""
    import torch
    from paper_2003_03130_amd import CellBatch
    c = small_sphere_case(1007)
    cb = CellBatch.single(c.x, c.tets)
    y = cb.to_device(c.y)
    v = cotangent(c.n_nodes, 3)
    vd = cb.to_device(v)
    out = {}
    for name, th in (("I", (1.0, 0.0, 1.0)), ("K", (1.0, 0.0, 0.0)),
                     ("J", (0.0, 1.0, 0.5))):
        cb.set_params(*th)
        f, E = cb.forces(y)
        out[name] = (float((vd.double() * f.double()).sum()), float(E.item()))
    mu, kappa, w = c.theta
    eb = 0.7
    want = np.array([
        w * out["I"][0] + (1 - w) * out["K"][0] + eb * (w * out["I"][1] + (1 - w) * out["K"][1]),
        out["J"][0] + eb * out["J"][1],
        mu * (out["I"][0] - out["K"][0] + eb * (out["I"][1] - out["K"][1]))])
    cb.set_params(*c.theta)
    _, tb = cb.backward(y, vd, torch.tensor([eb], dtype=torch.float64,
                                            device=cb.device))
    assert _max_rel(tb.cpu().numpy(), want) <= TOL


def test_batched_backward_deterministic_and_equal_percell():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=12, seed=21, tet_lo=500, tet_hi=8000, ladder=5)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, tile_tets=768)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    v = cb.to_device(cotangent(b.n_nodes, 9))
    eb = torch.linspace(0.1, 1.0, b.n_cells, dtype=torch.float64,
                        device=cb.device)
    y0, t0 = cb.backward(y, v, eb)
    y0, t0 = y0.clone(), t0.clone()
    for waves, bpcu in [(2, 0), (1, 2), (1, 8)]:
        cb.set_launch(waves, bpcu)
        y1, t1 = cb.backward(y, v, eb)
        assert torch.equal(y1, y0) and torch.equal(t1, t0)
    y2, t2 = cb.backward(y, v, eb, percell=True)
    assert torch.equal(y2, y0) and torch.equal(t2, t0)
    # against the oracle, cell by cell
    yb = cb.to_host(y0)
    tb = t0.cpu().numpy().reshape(-1, 3)
    vh = cb.to_host(v)
    for c in range(b.n_cells):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        yo, to = m.backward(cell.y.astype(np.float64), cell.theta,
                            vh[n0:n1].astype(np.float64), float(eb[c]))
        assert _max_rel(yb[n0:n1], yo) <= TOL
        assert _max_rel(tb[c], to) <= TOL


@pytest.mark.parametrize("n_regions", [1, 3])
def test_backward_restricted_to_flagged_cells(n_regions):
    """cm_forces_backward_cells: selected cells bitwise equal to the full
    backward, the others' ybar / thetabar entries untouched (sentinels),
    flags read through a strided column; with material regions the
    thetabar slots of a cell follow its flag."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import radial_regions
    b = uneven_batch(n_cells=12, seed=23, tet_lo=500, tet_hi=8000, ladder=5)
    kw = {}
    if n_regions > 1:
        kw = dict(regions=np.concatenate([
            radial_regions(b.x[b.node_off[c]:b.node_off[c + 1]],
                           b.tets[b.tet_off[c]:b.tet_off[c + 1]])
            for c in range(b.n_cells)]), n_regions=n_regions)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, **kw)
    th = np.repeat(b.theta, n_regions, axis=0)
    cb.set_params(th[:, 0], th[:, 1], th[:, 2])
    y = cb.to_device(b.y)
    v = cb.to_device(cotangent(b.n_nodes, 29))
    eb = torch.linspace(-0.5, 0.8, b.n_cells, dtype=torch.float64,
                        device=cb.device)
    y0, t0 = cb.backward(y, v, eb)
    y0, t0 = cb.to_host(y0), t0.cpu().numpy().reshape(b.n_cells, -1)
    sel = np.array([1, 0, 0, 1, 1, 0, 1, 0, 0, 0, 1, 1], np.float64)
    state = torch.zeros(b.n_cells, 5, dtype=torch.float64, device=cb.device)
    state[:, 3] = torch.from_numpy(sel).to(cb.device)
    yb = torch.full_like(cb.empty_nodes(), 7.0)
    tb = torch.full((3 * cb.n_mat,), -3.0, dtype=torch.float64,
                    device=cb.device)
    cb.backward(y, v, eb, yb, tb, cells=state[:, 3])
    y1, t1 = cb.to_host(yb), tb.cpu().numpy().reshape(b.n_cells, -1)
    for c in range(b.n_cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        if sel[c]:
            assert np.array_equal(y1[n0:n1], y0[n0:n1]), c
            assert np.array_equal(t1[c], t0[c]), c
        else:
            assert np.all(y1[n0:n1] == 7.0), c
            assert np.all(t1[c] == -3.0), c
    with pytest.raises(ValueError):
        cb.backward(y, v, eb, yb, tb, cells=state[:4, 3])
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    fn = nat.lib().cm_forces_backward_cells
    assert fn(cb._h, _ptr(y), _ptr(v), None, None, 1, _ptr(yb), None,
              _stream(None)) != 0
    assert fn(cb._h, _ptr(y), _ptr(v), None, _ptr(state), 0, _ptr(yb), None,
              _stream(None)) != 0


def test_graph_forward_backward_replay():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=8, seed=22, tet_lo=500, tet_hi=5000, ladder=4)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y = cb.to_device(b.y)
    v = cb.to_device(cotangent(b.n_nodes, 4))
    eb = torch.full((b.n_cells,), 0.5, dtype=torch.float64, device=cb.device)
    fe, Ee = cb.forces(y)
    ye, te = cb.backward(y, v, eb)
    fe, Ee, ye, te = fe.clone(), Ee.clone(), ye.clone(), te.clone()
    f, yb = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=cb.device)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=cb.device)
    s = torch.cuda.Stream()
    # 1: forward then backward; 3: the same as per-cell launches; 4 and 5:
    # forward and backward as parallel branches (batched, per cell)
    for mode in (1, 3, 4, 5):
        with torch.cuda.stream(s):
            cb.graph_capture(mode, y, f, E, None, v, eb, yb, tb, stream=s)
        for _ in range(3):
            for t in (f, E, yb, tb):
                t.zero_()
            torch.cuda.synchronize()
            cb.graph_launch(stream=s)
            s.synchronize()
            assert torch.equal(f, fe) and torch.equal(E, Ee)
            assert torch.equal(yb, ye) and torch.equal(tb, te)
            cb.forces(y)
            torch.cuda.synchronize()


def test_autograd_function():
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.autograd import mr_forces
    c = small_sphere_case(1009)
    cb = CellBatch.single(c.x, c.tets)
    y = cb.to_device(c.y).requires_grad_(True)
    theta = torch.tensor([c.theta], dtype=torch.float64, device=cb.device,
                         requires_grad=True)
    v = cotangent(c.n_nodes, 5)
    vd = cb.to_device(v)
    f, E = mr_forces(y, theta, cb)
    L = (f.double() * vd.double()).sum() + 0.25 * E.sum()
    L.backward()
    m = oracle.OracleMesh(c.x, c.tets)
    yo, to = m.backward(c.y.astype(np.float64), c.theta, v, 0.25)
    assert _max_rel(cb.to_host(y.grad), yo) <= TOL
    assert _max_rel(theta.grad.cpu().numpy().ravel(), to) <= TOL
