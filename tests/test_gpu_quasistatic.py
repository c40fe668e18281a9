"""Quasi-static plate compression on the GPU (cm_qs_* with Newton-CG on the
backward kernels' Hessian-vector products) against the FP64 oracle's
minimiser of the same potential, along the same loading path.

Tolerance: the device stops at |f + p|_2 <= 1e-3 |p|_2 (projected residual,
float32 positions: the floor is about 5e-6 absolute, 3e-4 |p| at the
smallest compression), the oracle at a float64 gradient norm of 1e-10; the
plate force moves by well under the relative residual (measured 1e-5 to
2e-4), so the bar on the top-plate force is 2e-3 relative.  The plates
balance up to what the equilibrium test allows: Ft - Fb is the sum of the z
residuals (the elastic forces of a cell sum to zero), so |Ft - Fb| <=
sqrt(n) |r|_2 for n nodes.  At the first contact (2 % compression) the plate force of
a float32 state is resolved only to about 1 %: the residual floor of float32
positions leaves the state free to wander along the softest modes, which
change which nodes touch the plates; there the bar is 1e-2."""
import warnings

import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from oracle import quasistatic as oqs
from synth.configs import batch_from_cells, Cell
from synth.mesh import ellipsoid, sphere_mesh

pytestmark = pytest.mark.gpu
K = 100.0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _cells():
    """Ellipsoids with their shortest axis along the compression axis: a
    sphere between frictionless plates can roll at almost no energy cost
    (its discrete equilibria differ by orientation), an oblate cell cannot,
    so both solvers reach the same equilibrium."""
    thetas = [(1.0, 20.0, 0.5), (0.7, 30.0, 0.9), (1.5, 12.0, 0.1)]
    axes = [(1.2, 1.05, 0.8), (1.1, 1.3, 0.75), (1.25, 1.0, 0.85)]
    cells = []
    for k, (th, ax) in enumerate(zip(thetas, axes)):
        x, tets = sphere_mesh(300 + 100 * k, 5 + k)
        x = ellipsoid(x, np.array(ax))
        cells.append(Cell(x, tets, x.astype(np.float32), th))
    return batch_from_cells(cells)


def test_force_curve_against_oracle():
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    top0 = np.array([b.cell(c).x[:, 2].max() for c in range(b.n_cells)])
    bot = np.array([b.cell(c).x[:, 2].min() for c in range(b.n_cells)])
    delta = np.array([0.02, 0.05, 0.1, 0.2])
    tops = top0[None, :] - 2.0 * delta[:, None]
    qs = QuasiStaticCompression(cb, K)
    Ft, Fb, ok, y = qs.curve(cb.to_device(b.y), tops, bot)
    assert ok.all(), qs.stats
    print("newton / cg iterations:", qs.stats)
    worst = 0.0
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        yo = cell.x.copy()
        for s in range(len(delta)):
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", RuntimeWarning)
                yo, Fo, Fbo, g = oqs.equilibrium(m, yo, cell.theta, tops[s, c],
                                                 bot[c], K)
            err = abs(Ft[s, c] - Fo) / Fo
            worst = max(worst, err)
            assert err <= (1e-2 if delta[s] < 0.03 else 2e-3), (c, s, Ft[s, c], Fo)
            # plate balance: Ft - Fb = sum of the z residuals (the elastic
            # forces sum to zero), at most sqrt(n) |r|_2 by Cauchy-Schwarz
            n = b.node_off[c + 1] - b.node_off[c]
            assert abs(Ft[s, c] - Fb[s, c]) <= (np.sqrt(n) * qs.residuals[s, c]
                                                + 1e-6 * Ft[s, c])
    print("worst relative top-plate force difference:", worst)
    assert np.all(np.diff(Ft, axis=0) > 0)


def test_restart_from_equilibrium():
    """Solving again at the same plate position from an equilibrium takes at
    most a few Newton steps of float32 size and keeps the plate forces."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    top0 = np.array([b.cell(c).x[:, 2].max() for c in range(b.n_cells)])
    bot = np.array([b.cell(c).x[:, 2].min() for c in range(b.n_cells)])
    qs = QuasiStaticCompression(cb, K)
    Ft, _, ok, y = qs.curve(cb.to_device(b.y), (top0 - 0.1)[None, :], bot)
    assert ok.all()
    plate = torch.tensor(np.stack([top0 - 0.1, bot], axis=1), device=cb.device)
    n0 = qs.stats["newton"]
    y1 = y.clone()
    assert qs.equilibrate(y1, plate)
    assert qs.stats["newton"] - n0 <= 3
    assert (y1 - y).abs().max().item() <= 1e-5
    assert np.abs(qs.force[:, 0].cpu().numpy() - Ft[0]).max() <= 1e-4 * Ft[0].max()


def test_inexact_newton_matches_exact_solves():
    """The forcing term changes only how accurately each Newton system is
    solved, not the equilibrium test: eta_max = 0 (every CG solve to cg_tol)
    and the default inexact Newton steps give the same plate forces within
    the equilibrium tolerance.  eta_max outside [0, 1) is refused."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    top0 = np.array([b.cell(c).x[:, 2].max() for c in range(b.n_cells)])
    bot = np.array([b.cell(c).x[:, 2].min() for c in range(b.n_cells)])
    tops = top0[None, :] - 2.0 * np.array([0.05, 0.1, 0.2])[:, None]
    out = {}
    for eta in (0.0, 0.5):
        qs = QuasiStaticCompression(cb, K, eta_max=eta)
        Ft, Fb, ok, _ = qs.curve(cb.to_device(b.y), tops, bot)
        assert ok.all(), (eta, qs.stats)
        out[eta] = Ft
        print(f"eta_max {eta}: {qs.stats}")
    assert np.abs(out[0.5] - out[0.0]).max() <= 2e-3 * np.abs(out[0.0]).max()
    with pytest.raises(RuntimeError, match="eta_max"):
        QuasiStaticCompression(cb, K, eta_max=1.0).curve(
            cb.to_device(b.y), tops[:1], bot)


def _stiffness_blocks(x, tets, mu, kappa):
    """Per node, the summed diagonal 3x3 blocks V0 (mu |b|^2 I + (kappa +
    mu/3) b b^T) of the small-strain stiffness (b: the node's row of the
    tetrahedron's gradient operator; mu, kappa scalars or per tetrahedron),
    in float64."""
    D = np.zeros((len(x), 3, 3))
    mu = np.broadcast_to(np.asarray(mu, np.float64), (len(tets),))[:, None, None]
    kappa = np.broadcast_to(np.asarray(kappa, np.float64), (len(tets),))[:, None, None]
    e = x[tets[:, :3]] - x[tets[:, [3]]]
    Bt = np.linalg.inv(np.transpose(e, (0, 2, 1)))       # rows b_1, b_2, b_3
    V0 = np.abs(np.linalg.det(e)) / 6.0
    rows = np.concatenate([Bt, -Bt.sum(axis=1, keepdims=True)], axis=1)
    for a in range(4):
        b = rows[:, a, :]
        blk = V0[:, None, None] * (mu * (b * b).sum(1)[:, None, None] * np.eye(3)
                                   + (kappa + mu / 3.0) * b[:, :, None] * b[:, None, :])
        np.add.at(D, tets[:, a], blk)
    return D


def test_stiffness_blocks_and_preconditioned_cg():
    """cm_qs_stiffness against the blocks summed in float64 on the host; the
    preconditioned CG reaches the same plate forces as plain CG."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    kel = torch.empty(6 * b.n_nodes, dtype=torch.float32, device=cb.device)
    nat.check(nat.lib().cm_qs_stiffness(cb._h, _ptr(kel), _stream(None)))
    kh = kel.view(6, -1).cpu().numpy()
    perm = cb.new_to_old  # internal id -> input id
    got = np.zeros((b.n_nodes, 3, 3))
    ii = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for q, (i, j) in enumerate(ii):
        got[perm, i, j] = kh[q]
        got[perm, j, i] = kh[q]
    for c in range(b.n_cells):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        want = _stiffness_blocks(cell.x, cell.tets, cell.theta[0], cell.theta[1])
        err = np.abs(got[n0:n1] - want).max() / np.abs(want).max()
        assert err <= 1e-5, (c, err)
    top0 = np.array([b.cell(c).x[:, 2].max() for c in range(b.n_cells)])
    bot = np.array([b.cell(c).x[:, 2].min() for c in range(b.n_cells)])
    tops = top0[None, :] - 2.0 * np.array([0.05, 0.1, 0.2])[:, None]
    out = {}
    for pre in (False, True):
        qs = QuasiStaticCompression(cb, K, precondition=pre)
        Ft, _, ok, _ = qs.curve(cb.to_device(b.y), tops, bot)
        assert ok.all(), (pre, qs.stats)
        out[pre] = Ft
        print(f"precondition {pre}: {qs.stats}")
    assert np.abs(out[True] - out[False]).max() <= 2e-3 * np.abs(out[False]).max()


def test_stiffness_blocks_with_material_regions():
    """Every tetrahedron's block takes the (mu, kappa) of its region."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    from synth.configs import radial_regions
    b = _cells()
    reg = np.concatenate([radial_regions(b.cell(c).x, b.cell(c).tets)
                          for c in range(b.n_cells)])
    th = np.array([[1.0, 20.0, 0.5], [3.0, 5.0, 0.2], [0.4, 40.0, 0.9]] * b.n_cells)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets, regions=reg, n_regions=3)
    cb.set_params(th[:, 0], th[:, 1], th[:, 2])
    kel = torch.empty(6 * b.n_nodes, dtype=torch.float32, device=cb.device)
    nat.check(nat.lib().cm_qs_stiffness(cb._h, _ptr(kel), _stream(None)))
    kh = kel.view(6, -1).cpu().numpy()
    got = np.zeros((b.n_nodes, 3, 3))
    for q, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        got[cb.new_to_old, i, j] = kh[q]
        got[cb.new_to_old, j, i] = kh[q]
    for c in range(b.n_cells):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        r = reg[b.tet_off[c]:b.tet_off[c + 1]]
        want = _stiffness_blocks(cell.x, cell.tets, th[3 * c + r, 0], th[3 * c + r, 1])
        err = np.abs(got[n0:n1] - want).max() / np.abs(want).max()
        assert err <= 1e-5, (c, err)


@pytest.mark.parametrize("precondition", [True, False])
def test_cg_step_against_its_formula(precondition):
    """One cm_qs_cg_step on a cell of 1,500 nodes (operands held in
    registers) and one of 6,000 (more than 4 per thread of the 1,024-thread
    workgroup: operands streamed), against the iteration written out in
    float64 on the CPU from the same inputs: Ap = -ybar + penalty Hessian p,
    alpha = r.z / p.Ap, x += alpha p, r -= alpha Ap, z = M r, beta =
    r_new.z_new / r.z, p = z + beta p, and the stop test.  Float32 state:
    1e-5 of the largest value."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    xs, ts = zip(*[sphere_mesh(n, 40 + n) for n in (1500, 6000)])
    sizes = [len(x) for x in xs]
    assert sizes[0] <= 4096 < sizes[1]
    node_off = np.cumsum([0] + sizes)
    tet_off = np.cumsum([0] + [len(t) for t in ts])
    cb = CellBatch(node_off, tet_off, np.concatenate(xs), np.concatenate(ts))
    N, C = cb.n_nodes, cb.n_cells
    rng = np.random.default_rng(41)
    yh = np.concatenate(xs).astype(np.float32)
    ph, rh, xh = (rng.normal(size=(N, 3)).astype(np.float32) for _ in range(3))
    ybh = (-(2.0 * ph + 0.1 * rng.normal(size=(N, 3)))).astype(np.float32)
    diag = (1.0 + rng.uniform(size=(N, 3))).astype(np.float32)
    off = (0.1 * rng.uniform(-1, 1, size=(N, 3))).astype(np.float32)
    y, p, r, x, ybar = (cb.to_device(a) for a in (yh, ph, rh, xh, ybh))
    minv = torch.cat([cb.to_device(diag), cb.to_device(off)]) if precondition else None
    Ap = cb.empty_nodes()
    k, rel_tol, top, bot = 100.0, 1e-3, 0.7, -0.7
    plate = torch.tensor([[top, bot]] * C, dtype=torch.float64, device=cb.device)
    # host copies in the internal order (SoA; each cell's range preserved)
    Y, P, R, X, YB = (t.cpu().numpy().astype(np.float64).reshape(3, N)
                      for t in (y, p, r, x, ybar))
    M = minv.cpu().numpy().astype(np.float64).reshape(6, N) if precondition else None

    def mul(v):
        if M is None:
            return v.copy()
        xx, yy, zz, xy, xz, yz = M
        return np.stack([xx * v[0] + xy * v[1] + xz * v[2],
                         xy * v[0] + yy * v[1] + yz * v[2],
                         xz * v[0] + yz * v[1] + zz * v[2]])

    state = np.zeros((C, 16))
    Z0 = mul(R)
    for c in range(C):
        sl = slice(node_off[c], node_off[c + 1])
        state[c, 0] = (R[:, sl] * Z0[:, sl]).sum()
        state[c, 1] = [1e-30, 1e30][c]  # cell 1 stops, cell 0 does not
        state[c, 2] = 1.0
        state[c, 14] = 0.1
    st = torch.from_numpy(state).to(cb.device)
    nat.check(nat.lib().cm_qs_cg_step(
        cb._h, _ptr(y), _ptr(plate), k, rel_tol, _ptr(ybar), _ptr(x), _ptr(r),
        _ptr(p), _ptr(Ap), _ptr(st), _ptr(minv), _stream(None)))
    torch.cuda.synchronize()
    got = {n: t.cpu().numpy().astype(np.float64).reshape(3, N)
           for n, t in (("x", x), ("r", r), ("p", p))}
    sg = st.cpu().numpy()
    h = 2 * k * (np.maximum(Y[2] - top, 0) + np.maximum(bot - Y[2], 0))
    A = -YB
    A[2] += h * P[2]
    for c in range(C):
        sl = slice(node_off[c], node_off[c + 1])
        rs = state[c, 0]
        alpha = rs / (P[:, sl] * A[:, sl]).sum()
        xn = X[:, sl] + alpha * P[:, sl]
        rn = R[:, sl] - alpha * A[:, sl]
        zn = mul(np.pad(rn, ((0, 0), (node_off[c], N - node_off[c + 1]))))[:, sl]
        rzn = (rn * zn).sum()
        pn = zn + (rzn / rs) * P[:, sl]
        for name, want in (("x", xn), ("r", rn), ("p", pn)):
            err = np.abs(got[name][:, sl] - want).max() / np.abs(want).max()
            print(f"cell {c} ({sizes[c]} nodes) {name}: {err:.2e}", flush=True)
            assert err <= 1e-5, (c, name)
        assert abs(sg[c, 0] - rzn) <= 1e-5 * abs(rzn), c
        stop = (rn ** 2).sum() <= max(rel_tol, 0.1) ** 2 * state[c, 1]
        assert sg[c, 2] == (0.0 if stop else 1.0), c
