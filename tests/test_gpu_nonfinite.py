"""Non-finite inputs (cm_forces_checked): a NaN or an infinite coordinate
makes exactly the tetrahedra of that node non-finite; the per-cell count says
so, the other cells' results are bitwise those of a clean call, and every
kernel of the forward and backward passes runs to completion (the next calls
on the same handle work)."""
import numpy as np
import pytest

from gpu_util import require_gpu
from synth.configs import uneven_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_nonfinite_positions_are_flagged_per_cell():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=4, seed=95, tet_lo=1500, tet_hi=6000, ladder=3)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    y_clean = cb.to_device(b.y)
    ninv0 = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    f0, E0 = cb.forces(y_clean, n_inverted=ninv0)
    f1, E1, nf = cb.forces_checked(y_clean)
    torch.cuda.synchronize()
    assert torch.equal(f0, f1) and torch.equal(E0, E1)
    assert nf.cpu().numpy().tolist() == [0] * b.n_cells

    bad = b.y.copy()
    picks = {1: (17, 0, np.nan), 3: (5, 2, np.inf)}   # cell: (local node, axis, value)
    expect = [0] * b.n_cells
    for c, (node, ax, val) in picks.items():
        bad[b.node_off[c] + node, ax] = val
        tets = b.tets[b.tet_off[c]:b.tet_off[c + 1]]
        expect[c] = int((tets == node).any(axis=1).sum())
    y_bad = cb.to_device(bad)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    print("non-finite case: cells 1 (NaN) and 3 (inf)", flush=True)
    f2, E2, nf2 = cb.forces_checked(y_bad, n_inverted=ninv)
    torch.cuda.synchronize()
    assert nf2.cpu().numpy().tolist() == expect
    E2h, E0h = E2.cpu().numpy(), E0.cpu().numpy()
    fh2, fh0 = cb.to_host(f2), cb.to_host(f0)
    for c in range(b.n_cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        if expect[c]:
            assert not np.isfinite(E2h[c])
            assert not np.isfinite(fh2[n0:n1]).all()
        else:
            assert E2h[c] == E0h[c]
            assert np.array_equal(fh2[n0:n1], fh0[n0:n1])
    # NaN positions count as inverted (J > 0 fails), as a reading of J <= 0
    assert ninv.cpu().numpy()[1] >= expect[1]
    # the backward pass on the same input also runs to completion
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=cb.device)
    ybar, _ = cb.backward(y_bad, y_clean, None, thetabar=tb)
    torch.cuda.synchronize()
    assert np.isfinite(tb.cpu().numpy().reshape(-1, 3)[0]).all()
    # and the handle keeps working on clean input
    f3, E3, nf3 = cb.forces_checked(y_clean)
    torch.cuda.synchronize()
    assert torch.equal(f3, f0) and torch.equal(E3, E0)
    assert int(nf3.sum().item()) == 0
