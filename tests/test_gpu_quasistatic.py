"""Quasi-static plate compression on the GPU (cm_qs_* with Newton-CG on the
backward kernels' Hessian-vector products) against the FP64 oracle's
minimiser of the same potential, along the same loading path, from first
contact to 80 % plate travel (the paper's compressions go past the force
upturn at about 40 % deformation, Sec. "Results" of the FluidFM comparison).

Tolerance: the device stops at |f + p|_2 <= 1e-3 |p|_2 (projected residual,
float32 positions: the floor is about 5e-6 absolute, 3e-4 |p| at the
smallest compression), the oracle at a float64 gradient norm of 1e-10; the
plate force moves by well under the relative residual (measured 3e-5 to
8e-4 from 5 % on), so the bar on the top-plate force is 2e-3 relative.  At
the first contact (2 %) the plate force of a float32 state is resolved only
to about 1 % (the residual floor of float32 positions leaves the state free
to wander along the softest modes, which changes the nodes that touch the
plates): there the bar is 1e-2.  The plates balance: at equilibrium the
elastic forces of a cell sum to zero, so the top and bottom plate forces
are equal; the bar on |Ft - Fb| / Ft is 5e-3 at first contact and 2e-3 from
5 % on (measured 3.5e-3 and 1.5e-3).  No tetrahedron may be inverted at any
equilibrium (the line search keeps the states on the side J > 0)."""
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


FRACTIONS = np.array([0.02, 0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8])


def _plates(b, fractions):
    top0 = np.array([b.cell(c).x[:, 2].max() for c in range(b.n_cells)])
    bot = np.array([b.cell(c).x[:, 2].min() for c in range(b.n_cells)])
    tops = top0[None, :] - np.asarray(fractions)[:, None] * (top0 - bot)[None, :]
    return tops, bot, top0 - bot


def test_force_curve_against_oracle():
    """Plate travel from 2 % to 80 % of each cell's height: the top-plate
    force against the oracle at every position, the plate balance, no
    inverted tetrahedron, the cells' own height compressed by at least 60 %,
    and the upturn (log-log slope between 40 % and 80 % well above the 3/2 of
    Hertz contact)."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    tops, bot, H = _plates(b, FRACTIONS)
    qs = QuasiStaticCompression(cb, K)
    y = cb.to_device(b.y)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    Ft, Fb, ok, heights = [], [], [], []
    plates = torch.tensor(np.stack([tops, np.broadcast_to(bot, tops.shape)], axis=2),
                          device=cb.device)
    for s in range(len(FRACTIONS)):
        if s > 0:
            from paper_2003_03130_amd import _native as nat
            from paper_2003_03130_amd.cells import _ptr, _stream
            nat.check(nat.lib().cm_qs_predict(cb._h, _ptr(plates[s - 1]),
                                              _ptr(plates[s]), _ptr(y), _stream(None)))
        ok.append(qs.equilibrate(y, plates[s]))
        Ft.append(qs.force[:, 0].cpu().numpy().copy())
        Fb.append(qs.force[:, 1].cpu().numpy().copy())
        cb.forces(y, n_inverted=ninv)
        assert int(ninv.sum().item()) == 0, (s, ninv)
        yh = cb.to_host(y)
        heights.append([np.ptp(yh[b.node_off[c]:b.node_off[c + 1], 2])
                        for c in range(b.n_cells)])
    Ft, Fb, heights = np.array(Ft), np.array(Fb), np.array(heights)
    assert all(ok), qs.stats
    print("newton / cg iterations:", qs.stats)
    worst = 0.0
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        yo = cell.y.astype(np.float64)
        for s in range(len(FRACTIONS)):
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", RuntimeWarning)
                yo, Fo, Fbo, g = oqs.equilibrium(m, yo, cell.theta, tops[s, c],
                                                 bot[c], K)
            first = FRACTIONS[s] < 0.03
            err = abs(Ft[s, c] - Fo) / Fo
            worst = max(worst, err)
            assert err <= (1e-2 if first else 2e-3), (c, s, Ft[s, c], Fo)
            bal = abs(Ft[s, c] - Fb[s, c]) / Ft[s, c]
            assert bal <= (5e-3 if first else 2e-3), (c, s, bal)
    print("worst relative top-plate force difference:", worst)
    assert np.all(np.diff(Ft, axis=0) > 0)
    compression = 1.0 - heights[-1] / H
    print("height compression at 80 % plate travel:", compression)
    assert np.all(compression >= 0.6)
    slope = np.log(Ft[-1] / Ft[5]) / np.log(FRACTIONS[-1] / FRACTIONS[5])
    print("log-log slope of F between 40 % and 80 %:", slope)
    assert np.all(slope > 2.5)


def test_w_sets_the_upturn():
    """One cell with mu = 1, kappa = 20 and w = 0.25, 0.5, 1 (the paper's
    fitted values): the forces agree at small compression (the small-strain
    limit depends on mu = mu1 + mu2 only, eq. elastic-moduli:mr) and spread
    past the upturn, the smaller w (more of the K invariant) the stiffer;
    every curve against the oracle."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    x, tets = sphere_mesh(300, 5)
    x = ellipsoid(x, np.array((1.2, 1.05, 0.8)))
    ws = (0.25, 0.5, 1.0)
    b = batch_from_cells([Cell(x, tets, x.astype(np.float32), (1.0, 20.0, w))
                          for w in ws])
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    fr = np.array([0.05, 0.2, 0.4, 0.6, 0.8])
    tops, bot, _ = _plates(b, fr)
    qs = QuasiStaticCompression(cb, K)
    Ft, _, ok, _ = qs.curve(cb.to_device(b.y), tops, bot)
    assert ok.all()
    m = oracle.OracleMesh(x, tets)
    for c, w in enumerate(ws):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            Fo, _ = oqs.force_curve(m, b.cell(c).y.astype(np.float64), (1.0, 20.0, w),
                                    tops[:, c], bot[c], K)
        err = np.abs(Ft[:, c] - Fo) / Fo
        print(f"w {w}: {Ft[:, c]} (oracle {Fo}), rel. difference {err.max():.2e}")
        assert err.max() <= 2e-3
    assert np.ptp(Ft[0]) <= 0.01 * Ft[0].mean()
    assert Ft[-1, 0] > Ft[-1, 1] > Ft[-1, 2]
    assert (Ft[-1, 0] - Ft[-1, 2]) > 0.3 * Ft[-1, 2]


def test_plate_force_gradient_against_oracle_differences():
    """dF_top/d(mu, kappa, w) from the adjoint of the equilibrium (one CG
    solve per plate position, then one backward pass) against central
    differences of the oracle's equilibrium force (h = 1e-4 relative);
    bar 2e-3 of the largest component (measured up to 5e-4 at 10 %)."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    fr = np.array([0.1, 0.4, 0.7])
    tops, bot, _ = _plates(b, fr)
    qs = QuasiStaticCompression(cb, K)
    _, _, ok, _ = qs.curve(cb.to_device(b.y), tops, bot, jacobian=True)
    assert ok.all()
    Jg = qs.jacobian
    print("adjoint CG iterations:", qs.stats.get("adjoint_cg"))
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        th = np.array(cell.theta)
        steps = np.array([1e-4 * th[0], 1e-4 * th[1], 1e-4])
        fd = np.zeros((len(fr), 3))
        for k in range(3):
            Fs = []
            for sgn in (1, -1):
                tt = th.copy()
                tt[k] += sgn * steps[k]
                with warnings.catch_warnings():
                    warnings.simplefilter("ignore", RuntimeWarning)
                    F, _ = oqs.force_curve(m, cell.y.astype(np.float64), tuple(tt),
                                           tops[:, c], bot[c], K)
                Fs.append(F)
            fd[:, k] = (Fs[0] - Fs[1]) / (2 * steps[k])
        for s in range(len(fr)):
            err = np.abs(Jg[s, c] - fd[s]).max() / np.abs(fd[s]).max()
            print(f"cell {c} at {fr[s]:.0%}: adjoint {Jg[s, c]}, differences "
                  f"{fd[s]}, {err:.1e}", flush=True)
            assert err <= 2e-3, (c, s)


def test_calibration_recovers_hidden_parameters():
    """Force-indentation curves of hidden (mu, kappa, w) to 80 % plate travel
    from the oracle; Levenberg-Marquardt from another start with the
    adjoint's derivatives lowers every cell's loss by orders of magnitude
    and brings (mu, w) to within 1 % and kappa to within 10 % of the hidden
    values."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.calibrate import fit_curves
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    theta_star = b.theta.copy()
    theta0 = theta_star * np.array([1.4, 0.6, 1.0])
    theta0[:, 2] = np.clip(1.0 - theta_star[:, 2] * 0.7, 0.05, 0.95)
    fr = np.array([0.05, 0.2, 0.4, 0.6, 0.8])
    tops, bot, _ = _plates(b, fr)
    target = np.zeros((len(fr), b.n_cells))
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            target[:, c], _ = oqs.force_curve(m, cell.y.astype(np.float64),
                                              cell.theta, tops[:, c], bot[c], K)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(theta0[:, 0], theta0[:, 1], theta0[:, 2])
    qs = QuasiStaticCompression(cb, K)
    res = fit_curves(qs, cb.to_device(b.y), tops, bot, target, theta0, iters=8,
                     log=print)
    losses = np.array([h["loss"] for h in res["history"]])
    print("loss per iteration:", losses.sum(axis=1))
    assert np.all(np.diff(losses, axis=0) <= 0)
    assert np.all(losses[-1] <= 1e-3 * losses[0])
    rel = np.abs(res["theta"] - theta_star) / np.abs(theta_star)
    print("fitted:", res["theta"], "hidden:", theta_star, "rel. error:", rel)
    assert np.all(rel[:, 0] <= 1e-2) and np.all(np.abs(res["theta"][:, 2] - theta_star[:, 2]) <= 1e-2)
    assert np.all(rel[:, 1] <= 1e-1)


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


def test_cg_iteration_in_one_call_equals_two_calls():
    """cm_qs_cg_iteration (the tile pass without its finalize, the shared
    nodes summed inside the CG kernel) gives bitwise the iterates of
    cm_forces_backward_cells + cm_qs_cg_step: same plate forces, same
    Newton and CG counts, same final positions; on cells held in registers
    and on one of more than 4,096 nodes (streamed)."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b0 = _cells()
    x, tets = sphere_mesh(6000, 77)
    x = ellipsoid(x, np.array((1.15, 1.1, 0.8)))
    cells = [b0.cell(c) for c in range(b0.n_cells)]
    cells.append(Cell(x, tets, x.astype(np.float32), (1.2, 15.0, 0.4)))
    b = batch_from_cells(cells)
    assert b.node_off[-1] - b.node_off[-2] > 4096
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    tops, bot, _ = _plates(b, [0.05, 0.3])
    out = {}
    for fused in (False, True):
        qs = QuasiStaticCompression(cb, K, fused_cg=fused)
        Ft, Fb, ok, y = qs.curve(cb.to_device(b.y), tops, bot, jacobian=True)
        torch.cuda.synchronize()
        assert ok.all()
        out[fused] = (Ft, Fb, y.cpu().numpy(), qs.jacobian, dict(qs.stats))
        print(f"fused {fused}: {qs.stats}")
    a, c = out[False], out[True]
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    assert np.array_equal(a[2], c[2]) and np.array_equal(a[3], c[3])
    assert a[4] == c[4]


def test_pipelined_checks_keep_the_iterates():
    """Convergence checks read a block of 8 CG iterations late give bitwise
    the iterates of the loop that waits after every block (the block queued
    behind the last one that mattered runs as no-ops): same plate forces,
    Newton and CG counts, parameter derivatives and final positions; on
    cells of the 2-node and 4-node register paths of the CG kernel and one
    streamed."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b0 = _cells()
    cells = [b0.cell(c) for c in range(b0.n_cells)]
    for n, seed, ax in ((3000, 78, (1.1, 1.2, 0.8)), (6000, 77, (1.15, 1.1, 0.8))):
        x, tets = sphere_mesh(n, seed)
        x = ellipsoid(x, np.array(ax))
        cells.append(Cell(x, tets, x.astype(np.float32), (1.2, 15.0, 0.4)))
    b = batch_from_cells(cells)
    sizes = np.diff(b.node_off)
    assert sizes.min() <= 2048 and ((sizes > 2048) & (sizes <= 4096)).any()
    assert sizes.max() > 4096
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    tops, bot, _ = _plates(b, [0.05, 0.3, 0.5])
    out = {}
    for pipe in (False, True):
        qs = QuasiStaticCompression(cb, K, pipelined_checks=pipe)
        Ft, Fb, ok, y = qs.curve(cb.to_device(b.y), tops, bot, jacobian=True)
        torch.cuda.synchronize()
        assert ok.all()
        out[pipe] = (Ft, Fb, y.cpu().numpy(), qs.jacobian, dict(qs.stats))
        print(f"pipelined {pipe}: {qs.stats}", flush=True)
    a, c = out[False], out[True]
    for k in range(4):
        assert np.array_equal(a[k], c[k]), k
    assert a[4] == c[4]


SPHERE_R = 0.66  # probe radius over particle radius in the paper's colloidal-probe comparison
SPHERE_FRACTIONS = np.array([0.05, 0.1, 0.2, 0.3, 0.4])


def _sphere_axes(b):
    return np.array([b.cell(c).y.astype(np.float64)[:, :2].mean(axis=0)
                     for c in range(b.n_cells)])


def test_sphere_indentation_against_oracle():
    """A sphere of radius 0.66 (the paper's probe-to-particle ratio) on each
    cell's axis indents it by 5 % to 40 % of its height: the sphere's force
    against the oracle at every position, the sphere/plate balance, the
    held centroid, no inverted tetrahedron, and a force below the flat
    plate's at the same travel."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    tops, bot, _ = _plates(b, SPHERE_FRACTIONS)
    axes = _sphere_axes(b)
    qs = QuasiStaticCompression(cb, K, sphere_radius=SPHERE_R, sphere_axis=axes)
    Ft, Fb, ok, y = qs.curve(cb.to_device(b.y), tops, bot)
    assert ok.all(), qs.stats
    print("sphere: newton / cg iterations:", qs.stats, flush=True)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    cb.forces(y, n_inverted=ninv)
    assert int(ninv.sum().item()) == 0
    cent = qs.cell_centroids(y).cpu().numpy()
    assert np.abs(cent - axes).max() <= 1e-5, cent - axes
    worst = 0.0
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            Fo, _ = oqs.force_curve(m, cell.y.astype(np.float64), cell.theta, tops[:, c],
                                    bot[c], K, sphere=(SPHERE_R, axes[c, 0], axes[c, 1]))
        for s in range(len(SPHERE_FRACTIONS)):
            first = s == 0
            err = abs(Ft[s, c] - Fo[s]) / Fo[s]
            worst = max(worst, err)
            assert err <= (1e-2 if first else 2e-3), (c, s, Ft[s, c], Fo[s])
            bal = abs(Ft[s, c] - Fb[s, c]) / Ft[s, c]
            assert bal <= (5e-3 if first else 2e-3), (c, s, bal)
    print("worst relative sphere force difference:", worst, flush=True)
    assert np.all(np.diff(Ft, axis=0) > 0)
    qp = QuasiStaticCompression(cb, K)
    Fp, _, okp, _ = qp.curve(cb.to_device(b.y), tops[-1:], bot)
    assert okp.all() and np.all(Ft[-1] < Fp[0])


def test_sphere_force_gradient_against_oracle_differences():
    """Under the sphere, dF/d(mu, kappa, w) from the adjoint of the
    equilibrium with the held centroid (the right-hand side and the CG
    projected like the Newton systems) against central differences of the
    oracle's equilibrium force (h = 1e-4 relative); bar 2e-3 of the largest
    component.  The sensitivity of the sphere's contact Hessian to the state
    needs equilibria to 1e-5 of the penalty force: at the default 1e-3 the
    residual left at 30 % indentation (4e-4) moved dF/dmu by 0.8 %."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    fr = np.array([0.1, 0.3])
    tops, bot, _ = _plates(b, fr)
    axes = _sphere_axes(b)
    qs = QuasiStaticCompression(cb, K, sphere_radius=SPHERE_R, sphere_axis=axes,
                                rel_tol=1e-5)
    _, _, ok, _ = qs.curve(cb.to_device(b.y), tops, bot, jacobian=True)
    assert ok.all()
    Jg = qs.jacobian
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        th = np.array(cell.theta)
        steps = np.array([1e-4 * th[0], 1e-4 * th[1], 1e-4])
        fd = np.zeros((len(fr), 3))
        for k in range(3):
            Fs = []
            for sgn in (1, -1):
                tt = th.copy()
                tt[k] += sgn * steps[k]
                with warnings.catch_warnings():
                    warnings.simplefilter("ignore", RuntimeWarning)
                    F, _ = oqs.force_curve(m, cell.y.astype(np.float64), tuple(tt), tops[:, c],
                                           bot[c], K, sphere=(SPHERE_R, axes[c, 0], axes[c, 1]))
                Fs.append(F)
            fd[:, k] = (Fs[0] - Fs[1]) / (2 * steps[k])
        for s in range(len(fr)):
            err = np.abs(Jg[s, c] - fd[s]).max() / np.abs(fd[s]).max()
            print(f"sphere, cell {c} at {fr[s]:.0%}: adjoint {Jg[s, c]}, differences "
                  f"{fd[s]}, {err:.1e}", flush=True)
            assert err <= 2e-3, (c, s)


def test_sphere_indentation_of_a_streamed_cell_against_oracle():
    """Under the sphere, cells of more than 2,048 nodes take the CG kernel's
    streaming path (its 2-node register variant covers the smaller ones): a
    2,409-node cell indented by 10 % and 25 % of its height against the
    oracle (bar 2e-3), its centroid held and the sphere and plate forces in
    balance."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    x, tets = sphere_mesh(2300, 41)
    x = ellipsoid(x, np.array((1.1, 1.2, 0.8)))
    theta = (1.2, 15.0, 0.4)
    b = batch_from_cells([Cell(x, tets, x.astype(np.float32), theta)])
    assert b.node_off[1] > 2048
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    tops, bot, _ = _plates(b, [0.1, 0.25])
    axes = _sphere_axes(b)
    qs = QuasiStaticCompression(cb, K, sphere_radius=SPHERE_R, sphere_axis=axes)
    Ft, Fb, ok, y = qs.curve(cb.to_device(b.y), tops, bot)
    assert ok.all(), qs.stats
    assert np.abs(qs.cell_centroids(y).cpu().numpy() - axes).max() <= 1e-5
    m = oracle.OracleMesh(x, tets)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        Fo, _ = oqs.force_curve(m, b.y.astype(np.float64), theta, tops[:, 0], bot[0], K,
                                sphere=(SPHERE_R, axes[0, 0], axes[0, 1]))
    err = np.abs(Ft[:, 0] - Fo) / Fo
    print("streamed sphere cell: device", Ft[:, 0], "oracle", Fo, "err", err, qs.stats, flush=True)
    assert err.max() <= 2e-3
    assert (np.abs(Ft[:, 0] - Fb[:, 0]) / Ft[:, 0]).max() <= 2e-3


def test_calibration_by_sphere_indentation():
    """The paper's AFM comparison fits the model to colloidal-probe curves:
    force curves of hidden (mu, kappa, w) under the sphere to 40 % of the
    height from the oracle, then Levenberg-Marquardt from another start with
    the sphere's adjoint derivatives (equilibria to 1e-5 of the penalty
    force, which the adjoint needs under the sphere).  The loss falls by
    orders of magnitude and mu is recovered to 1 %; kappa and w, which
    shallow sphere indentation constrains less than deep plate compression,
    to within 10 % and 0.05."""
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.calibrate import fit_curves
    from paper_2003_03130_amd.quasistatic import QuasiStaticCompression
    b = _cells()
    theta_star = b.theta.copy()
    theta0 = theta_star * np.array([1.4, 0.6, 1.0])
    theta0[:, 2] = np.clip(1.0 - theta_star[:, 2] * 0.7, 0.05, 0.95)
    fr = np.array([0.05, 0.1, 0.2, 0.3, 0.4])
    tops, bot, _ = _plates(b, fr)
    axes = _sphere_axes(b)
    target = np.zeros((len(fr), b.n_cells))
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            target[:, c], _ = oqs.force_curve(m, cell.y.astype(np.float64), cell.theta,
                                              tops[:, c], bot[c], K,
                                              sphere=(SPHERE_R, axes[c, 0], axes[c, 1]))
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(theta0[:, 0], theta0[:, 1], theta0[:, 2])
    qs = QuasiStaticCompression(cb, K, sphere_radius=SPHERE_R, sphere_axis=axes, rel_tol=1e-5)
    res = fit_curves(qs, cb.to_device(b.y), tops, bot, target, theta0, iters=8, log=print)
    losses = np.array([h["loss"] for h in res["history"]])
    print("sphere calibration, loss per iteration:", losses.sum(axis=1), flush=True)
    assert np.all(np.diff(losses, axis=0) <= 0)
    assert np.all(losses[-1] <= 1e-3 * losses[0])
    rel = np.abs(res["theta"] - theta_star) / np.abs(theta_star)
    print("fitted:", res["theta"], "hidden:", theta_star, "rel. error:", rel, flush=True)
    assert np.all(rel[:, 0] <= 1e-2)
    assert np.all(rel[:, 1] <= 1e-1)
    assert np.all(np.abs(res["theta"][:, 2] - theta_star[:, 2]) <= 5e-2)
