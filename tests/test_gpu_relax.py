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
                           plate_schedule)

pytestmark = pytest.mark.gpu
TRAJ_TOL, GRAD_TOL = 1e-5, 1e-5
MOB = STOKES_DT / DRAG


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _setup(n_steps=40, compression=0.1, checkpoint=10, n_cells=3):
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd.relax import PlateCompression
    b = compression_batch(n_cells, 300, 5000, n_meshes=2)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    top, bot = plate_schedule(n_steps, compression=compression)
    pc = PlateCompression(cb, top, bot, K_PLATE, MOB, checkpoint=checkpoint)
    return b, cb, pc, top, bot


def test_trajectory_matches_oracle():
    b, cb, pc, top, bot = _setup()
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


def test_bptt_gradient_matches_oracle_forward_mode():
    import torch
    b, cb, pc, top, bot = _setup()
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
