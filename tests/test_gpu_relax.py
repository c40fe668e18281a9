"""Plate compression on the GPU against the FP64 oracle's replay of the same
discrete scheme (a reading of the paper's unavailable supporting
information: the paper itself pins nothing here).

Tolerances (max-normalised over a run): plate forces, final positions and
the parameter gradient 1e-5, the bar of the single evaluation.  The float32
state carries a rounding of about 6e-8 relative per step against the float64
replay; over the 40 contracting steps of these runs the measured errors stay
near 1e-6.
"""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from synth.configs import (DRAG, K_PLATE, STOKES_DT, compression_batch,
                           cotangent, plate_schedule, random_theta)

pytestmark = pytest.mark.gpu
TRAJ_TOL, GRAD_TOL = 1e-5, 1e-5
MOB = STOKES_DT / DRAG


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _setup(n_steps=40, compression=0.1, checkpoint=10, n_cells=3, fused=True):
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.relax import PlateCompression
    b = compression_batch(n_cells, 300, 5000, n_meshes=2)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    top, bot = plate_schedule(n_steps, compression=compression)
    pc = PlateCompression(cb, top, bot, K_PLATE, MOB, checkpoint=checkpoint,
                          fused=fused)
    return b, cb, pc, top, bot


@pytest.mark.parametrize("fused", [True, False])
def test_trajectory_matches_oracle(fused):
    b, cb, pc, top, bot = _setup(fused=fused)
    pc.set_theta(b.theta)
    F, yN, _ = pc.forward(cb.to_device(b.y))
    Fh = F.cpu().numpy()
    yh = cb.to_host(yN)
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        Fo, yo = m.relax_forward(cell.y.astype(np.float64), cell.theta, top,
                                 bot, K_PLATE, MOB)
        ferr = np.abs(Fh[:, c] - Fo).max() / np.abs(Fo).max()
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        yerr = np.abs(yh[n0:n1] - yo).max() / np.abs(yo).max()
        print(f"cell {c}: plate force err {ferr:.2e}, final position err "
              f"{yerr:.2e}", flush=True)
        assert ferr <= TRAJ_TOL and yerr <= TRAJ_TOL


def _targets(b, top, bot):
    """Force curves of the hidden parameters, from the oracle (N, n_cells)."""
    out = []
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        Fo, _ = m.relax_forward(cell.y.astype(np.float64), cell.theta, top,
                                bot, K_PLATE, MOB)
        out.append(Fo)
    return np.stack(out, axis=1)


@pytest.mark.parametrize("fused", [True, False])
def test_bptt_gradient_matches_oracle_forward_mode(fused):
    import torch
    b, cb, pc, top, bot = _setup(fused=fused)
    Ft = _targets(b, top, bot)
    theta0 = b.info["theta0"]
    pc.set_theta(theta0)
    N = len(top)
    scale = 1.0 / (N * b.n_cells)
    loss, g, _ = pc.gradient(cb.to_device(b.y),
                             torch.from_numpy(Ft).to(cb.device), scale)
    g = g.cpu().numpy()
    L_or = 0.0
    for c in range(b.n_cells):
        cell = b.cell(c)
        m = oracle.OracleMesh(cell.x, cell.tets)
        Lc, gc, _ = m.relax_grad(cell.y.astype(np.float64), tuple(theta0[c]),
                                 top, bot, K_PLATE, MOB, Ft[:, c], scale)
        L_or += Lc
        err = np.abs(g[c] - gc).max() / np.abs(gc).max()
        print(f"cell {c}: grad gpu {g[c]} oracle {gc} err {err:.2e}", flush=True)
        assert err <= GRAD_TOL
    assert abs(loss - L_or) <= TRAJ_TOL * abs(L_or)


def test_checkpointing_is_exact():
    import torch
    b, cb, pc, top, bot = _setup(n_steps=30, checkpoint=7)
    Ft = torch.from_numpy(_targets(b, top, bot)).to(cb.device)
    pc.set_theta(b.info["theta0"])
    y0 = cb.to_device(b.y)
    l1, g1, F1 = pc.gradient(y0, Ft, 0.01)
    pc.checkpoint = 1  # every state kept, no recomputation
    l2, g2, F2 = pc.gradient(y0, Ft, 0.01)
    assert l1 == l2 and torch.equal(g1, g2) and torch.equal(F1, F2)


def test_plate_step_argument_errors():
    import torch
    from paper_2003_03130_amd import CellmechError
    from paper_2003_03130_amd import _native as nat
    b, cb, pc, top, bot = _setup(n_steps=2)
    y = cb.to_device(b.y)
    f = cb.empty_nodes()
    with pytest.raises(CellmechError) as ei:
        cb.plate_step(y, f, pc.plates[0], K_PLATE, MOB, y)
    assert ei.value.status == nat.CM_EINVAL
    with pytest.raises(CellmechError) as ei:
        cb.plate_step(y, f, pc.plates[0], -1.0, MOB, cb.empty_nodes())
    assert ei.value.status == nat.CM_EINVAL
    lam = torch.zeros_like(y)
    with pytest.raises(CellmechError) as ei:
        cb.plate_step_adjoint(y, lam, f, pc.plates[0], K_PLATE, MOB, lam)
    assert ei.value.status == nat.CM_EINVAL


def _one_step_both_routes(cb, y, lam_next, plate, F_target, k, m):
    """One forward and one reverse plate step by the fused calls and by the
    two-call route; returns the pairs of results."""
    import torch
    dev = cb.device
    yn_f, yn_t = cb.empty_nodes(), cb.empty_nodes()
    F_f = torch.empty(cb.n_cells, dtype=torch.float64, device=dev)
    F_t = torch.empty_like(F_f)
    E_f = torch.empty_like(F_f)
    ni_f = torch.empty(cb.n_cells, dtype=torch.int32, device=dev)
    cb.plate_forces_step(y, plate, k, m, yn_f, F_f, E_f, ni_f)
    ni_t = torch.empty_like(ni_f)
    f, E_t = cb.forces(y, n_inverted=ni_t)
    cb.plate_step(y, f, plate, k, m, yn_t, F_t)
    acc0 = torch.linspace(-1, 1, 3 * cb.n_mat, dtype=torch.float64, device=dev)
    acc_f, acc_t = acc0.clone(), acc0.clone()
    lam_f, lam_t = cb.empty_nodes(), cb.empty_nodes()
    cb.plate_backward_step(y, lam_next, plate, k, m, lam_f, F_t, F_target,
                           0.3, acc_f)
    ybar, tb = cb.backward(y, lam_next)
    cb.plate_step_adjoint(y, lam_next, ybar, plate, k, m, lam_t, F_t,
                          F_target, 0.3, tb, acc_t)
    torch.cuda.synchronize()
    return ((yn_f, yn_t), (F_f, F_t), (E_f, E_t), (ni_f, ni_t), (lam_f, lam_t),
            (acc_f, acc_t))


def _assert_routes_agree(pairs):
    """Both routes run the same per-node arithmetic (one inlined function):
    positions, adjoint state, energies, counts and the parameter accumulator
    bitwise equal.  The top-plate force sums the same float64 node terms in
    another order (tile shares instead of one workgroup per cell): equal to
    1e-12 relative (about 1e-16 per term times the number of terms)."""
    import torch
    (yf, yt), (Ff, Ft), (Ef, Et), (nf, nt), (lf, lt), (af, at) = pairs
    for a, b in ((yf, yt), (lf, lt)):
        d = (a - b).abs().max().item()
        print(f"max |fused - two-call| {d:.3e} of {b.abs().max().item():.3e}",
              flush=True)
        assert torch.equal(a, b)
    assert torch.equal(Ef, Et) and torch.equal(nf, nt)
    dF = ((Ff - Ft).abs().max() / Ft.abs().max()).item()
    print(f"plate force: max rel diff {dF:.2e}", flush=True)
    assert dF <= 1e-12
    assert torch.equal(af, at)


def test_fused_steps_equal_the_two_call_route():
    """cm_plate_forces_step / cm_plate_backward_step against cm_forces +
    cm_plate_step and cm_forces_backward + cm_plate_step_adjoint, on a state
    in contact with both plates (owned and shared nodes pressed), with and
    without the loss term."""
    import torch
    from synth.configs import cotangent
    b, cb, pc, top, bot = _setup(n_steps=2)
    pc.set_theta(b.info["theta0"])
    y = cb.to_device(b.y)
    yh = b.y
    zc = [(yh[b.node_off[c]:b.node_off[c + 1], 2].max(),
           yh[b.node_off[c]:b.node_off[c + 1], 2].min()) for c in range(b.n_cells)]
    # plates 10 % inside the cell's extent: many nodes in contact
    plate = torch.tensor([[zt - 0.1 * (zt - zb), zb + 0.1 * (zt - zb)]
                          for zt, zb in zc], dtype=torch.float64, device=cb.device)
    lam_next = cb.to_device(cotangent(b.n_nodes, 91))
    Ftgt = torch.linspace(0.5, 2.0, b.n_cells, dtype=torch.float64,
                          device=cb.device)
    for F_target in (Ftgt, None):
        pairs = _one_step_both_routes(cb, y, lam_next, plate, F_target,
                                      K_PLATE, MOB)
        assert (pairs[1][1] > 0).all()  # the top plate touches every cell
        _assert_routes_agree(pairs)


def test_fused_steps_with_regions_and_template():
    """The fused steps on a batch with three material regions per cell
    (thetabar accumulated per region) and on a template batch."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from synth.configs import cotangent, radial_regions, random_theta
    b = compression_batch(2, 300, 5000, n_meshes=2)
    reg = np.concatenate([
        radial_regions(b.x[b.node_off[c]:b.node_off[c + 1]],
                       b.tets[b.tet_off[c]:b.tet_off[c + 1]])
        for c in range(b.n_cells)])
    cbr = CellBatch(b.node_off, b.tet_off, b.x, b.tets, regions=reg, n_regions=3)
    rng = np.random.default_rng(93)
    th = np.array([random_theta(rng) for _ in range(2 * 3)])
    cbr.set_params(th[:, 0], th[:, 1], th[:, 2])
    c0 = b.cell(0)
    cbt = CellBatch.template(3, c0.x, c0.tets)
    tht = np.array([random_theta(rng) for _ in range(3)])
    cbt.set_params(tht[:, 0], tht[:, 1], tht[:, 2])
    for cb, yh in ((cbr, b.y), (cbt, np.tile(c0.y, (3, 1)))):
        y = cb.to_device(yh)
        z = yh[:, 2]
        plate = torch.tensor([[z.max() - 0.1 * np.ptp(z), z.min() + 0.1 * np.ptp(z)]]
                             * cb.n_cells, dtype=torch.float64, device=cb.device)
        lam_next = cb.to_device(cotangent(cb.n_nodes, 95))
        Ftgt = torch.ones(cb.n_cells, dtype=torch.float64, device=cb.device)
        _assert_routes_agree(_one_step_both_routes(cb, y, lam_next, plate, Ftgt,
                                                   K_PLATE, MOB))


def test_fused_step_argument_errors():
    import torch
    from paper_2003_03130_amd import CellmechError
    from paper_2003_03130_amd import _native as nat
    b, cb, pc, top, bot = _setup(n_steps=2)
    y = cb.to_device(b.y)
    lam = torch.zeros_like(y)
    with pytest.raises(CellmechError) as ei:
        cb.plate_forces_step(y, pc.plates[0], K_PLATE, MOB, cb.empty_nodes())
    assert ei.value.status == nat.CM_ESTATE  # no parameters yet
    pc.set_theta(b.theta)
    for call in (lambda: cb.plate_forces_step(y, pc.plates[0], K_PLATE, MOB, y),
                 lambda: cb.plate_forces_step(y, pc.plates[0], float("nan"), MOB,
                                              cb.empty_nodes()),
                 lambda: cb.plate_backward_step(y, lam, pc.plates[0], K_PLATE,
                                                MOB, lam),
                 lambda: cb.plate_backward_step(y, lam, pc.plates[0], K_PLATE,
                                                -MOB, cb.empty_nodes()),
                 lambda: cb.plate_backward_step(y, lam, pc.plates[0], K_PLATE,
                                                MOB, cb.empty_nodes(), None,
                                                pc.plates[0][:1])):
        with pytest.raises(CellmechError) as ei:
            call()
        assert ei.value.status == nat.CM_EINVAL


def test_fused_step_counts_nodes_of_no_tetrahedron():
    """A node in no tetrahedron has no slot in any tile: the fused step
    still moves it by the plate penalty and counts its plate force."""
    import torch
    from paper_2003_03130_amd import CellBatch
    b = compression_batch(2, 300, 5000, n_meshes=2)
    c0, c1 = b.cell(0), b.cell(1)
    z0 = c0.y[:, 2]
    extra = [[0.0, 0.0, z0.max() + 0.05]]  # above the top plate set below
    x = np.concatenate([c0.x, extra, c1.x])
    y = np.concatenate([c0.y, extra, c1.y]).astype(np.float32)
    n0 = len(c0.x) + 1
    tets = np.concatenate([c0.tets, c1.tets])
    cb = CellBatch([0, n0, n0 + len(c1.x)], [0, len(c0.tets), len(tets)], x,
                   tets)
    rng = np.random.default_rng(97)
    th = np.array([random_theta(rng) for _ in range(2)])
    cb.set_params(th[:, 0], th[:, 1], th[:, 2])
    yd = cb.to_device(y)
    plate = torch.tensor([[z0.max() - 0.1 * np.ptp(z0), z0.min() + 0.1 * np.ptp(z0)]] * 2,
                         dtype=torch.float64, device=cb.device)
    pairs = _one_step_both_routes(cb, yd, cb.to_device(cotangent(cb.n_nodes, 98)),
                                  plate, None, K_PLATE, MOB)
    _assert_routes_agree(pairs)
    yn = cb.to_host(pairs[0][0])
    assert yn[len(c0.x), 2] < y[len(c0.x), 2]  # pushed down by the top plate
