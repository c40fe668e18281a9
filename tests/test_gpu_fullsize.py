"""Full-size parity: the 4,096-cell uneven workload (41,987,047 tetrahedra,
seed 3000) in the configuration the benchmark times — autotuned launch,
forward + backward captured as one graph and replayed — checked against the
FP64 oracle on 64 cells spread over the batch (the oracle evaluates them one
by one), plus properties that hold at any size: every replay is bitwise the
eager pass, every cell's forces balance (zero net force), no tetrahedron is
inverted.  Tolerances as everywhere: forces, ybar, thetabar max-normalised
1e-5, energy 1e-6 relative."""
import numpy as np
import pytest

import oracle
from gpu_util import force_rel_err, rel_err, require_gpu
from synth.configs import cotangent, uneven_batch

pytestmark = pytest.mark.gpu
TOL, E_TOL = 1e-5, 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.timeout(600)
def test_full_workload_graph_replay_against_oracle():
    import torch
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=4096, seed=3000)
    assert b.n_tets == 41987047 and b.n_cells == 4096
    print(f"workload: {b.n_cells} cells, {b.n_tets} tets", flush=True)
    cb = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    dev = cb.device
    y = cb.to_device(b.y)
    v = cotangent(b.n_nodes, 3001)
    fbar = cb.to_device(v)
    eb_h = np.random.default_rng(3002).uniform(0.0, 1.0, b.n_cells)
    ebar = torch.tensor(eb_h, dtype=torch.float64, device=dev)
    cb.autotune(y)
    print(f"launch {cb.get_launch()}", flush=True)
    f, ybar = cb.empty_nodes(), cb.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=dev)
    ninv = torch.empty(b.n_cells, dtype=torch.int32, device=dev)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=dev)
    # eager pass
    cb.forces(y, f, E, ninv)
    cb.backward(y, fbar, ebar, ybar, tb)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (f, E, ninv, ybar, tb)]
    # the benchmark's step: one captured graph, replayed
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cb.graph_capture(1, y, f, E, ninv, fbar, ebar, ybar, tb, stream=s)
    for rep in range(3):
        for t in (f, ybar):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        cb.graph_launch(stream=s)
        torch.cuda.synchronize()
        for got, want in zip((f, E, ninv, ybar, tb), eager):
            assert torch.equal(got, want), rep
    fh, yh = cb.to_host(f), cb.to_host(ybar)
    Eh, nh = E.cpu().numpy(), ninv.cpu().numpy()
    th = tb.cpu().numpy().reshape(-1, 3)
    assert nh.sum() == 0
    # zero net force per cell (any size)
    for c in range(b.n_cells):
        fc = fh[b.node_off[c]:b.node_off[c + 1]].astype(np.float64)
        assert np.abs(fc.sum(axis=0)).max() <= 1e-5 * np.abs(fc).sum(axis=0).max(), c
    # sampled cells against the oracle
    worst = np.zeros(4)
    for c in np.linspace(0, b.n_cells - 1, 64).astype(int):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        y64 = cell.y.astype(np.float64)
        fo, Eo, no = m.forces(y64, cell.theta)
        yo, to = m.backward(y64, cell.theta, v[n0:n1].astype(np.float64),
                            float(eb_h[c]))
        err = (force_rel_err(fh[n0:n1], fo), rel_err(Eh[c], Eo),
               force_rel_err(yh[n0:n1], yo), force_rel_err(th[c], to))
        worst = np.maximum(worst, err)
        assert nh[c] == no, c
        assert err[0] <= TOL and err[1] <= E_TOL, (c, err)
        assert err[2] <= TOL and err[3] <= TOL, (c, err)
    print("worst force, energy, ybar, thetabar:", worst.tolist(), flush=True)
