"""cm_forces_noalloc (scratch in a static device array, no allocation)
against cm_forces through the C ABI: two calls in a row, the second on a
smaller handle, each bitwise equal to cm_forces and within the parity bars of
the FP64 oracle; a replay under HIP graph capture; the size limit."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from synth.configs import small_sphere_case, uneven_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _call_noalloc(cb, y):
    import torch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    f = torch.full((3 * cb.n_nodes,), float("nan"), dtype=torch.float32,
                   device=cb.device)
    E = torch.full((cb.n_cells,), float("nan"), dtype=torch.float64,
                   device=cb.device)
    ninv = torch.full((cb.n_cells,), -1, dtype=torch.int32, device=cb.device)
    nat.check(nat.lib().cm_forces_noalloc(cb._h, _ptr(y), _ptr(f), _ptr(E),
                                          _ptr(ninv), _stream(None)))
    return f, E, ninv


def _check_against_forces_and_oracle(cb, cells, y, f, E, ninv):
    import torch
    f_ref, E_ref = cb.forces(y, n_inverted=(ni := torch.zeros(
        cb.n_cells, dtype=torch.int32, device=cb.device)))
    torch.cuda.synchronize()
    assert torch.equal(f, f_ref), "forces differ from cm_forces"
    assert torch.equal(E, E_ref), "energies differ from cm_forces"
    assert torch.equal(ninv, ni), "inverted counts differ from cm_forces"
    fh = cb.to_host(f)
    Eh = E.cpu().numpy()
    off = cb.node_off
    for c, cell in enumerate(cells):
        m = oracle.OracleMesh(cell.x, cell.tets)
        fo, Eo, _ = m.forces(cell.y.astype(np.float64), cell.theta)
        fg = fh[off[c]:off[c + 1]].astype(np.float64)
        assert np.abs(fg - fo).max() / np.abs(fo).max() <= 1e-5, c
        assert abs(Eh[c] - Eo) / abs(Eo) <= 1e-6, c


def test_noalloc_two_calls_second_smaller():
    from paper_2003_03130_amd import CellBatch
    b = uneven_batch(n_cells=12, seed=91, tet_lo=2000, tet_hi=20000, ladder=6)
    cells = [b.cell(c) for c in range(b.n_cells)]
    big = CellBatch(b.node_off, b.tet_off, b.x, b.tets)
    big.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    small_cell = small_sphere_case(1003)
    small = CellBatch.single(small_cell.x, small_cell.tets)
    small.set_params(*small_cell.theta)
    assert small.info["n_slots"] < big.info["n_slots"]
    yb = big.to_device(b.y)
    ys = small.to_device(small_cell.y)
    print(f"noalloc call 1: {big.n_cells} cells, {big.n_tets} tets, "
          f"{big.info['n_slots']} slots", flush=True)
    out1 = _call_noalloc(big, yb)
    _check_against_forces_and_oracle(big, cells, yb, *out1)
    print(f"noalloc call 2: 1 cell, {small.n_tets} tets, "
          f"{small.info['n_slots']} slots", flush=True)
    out2 = _call_noalloc(small, ys)
    _check_against_forces_and_oracle(small, [small_cell], ys, *out2)
    # the first handle again, after the smaller call reused the array
    out3 = _call_noalloc(big, yb)
    _check_against_forces_and_oracle(big, cells, yb, *out3)


def test_noalloc_under_graph_capture():
    """The call records into a graph (no allocation, no memset node);
    every replay, with eager work of the same handle in between, equals the
    eager call."""
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    c = small_sphere_case(1007)
    cb = CellBatch.single(c.x, c.tets)
    cb.set_params(*c.theta)
    y = cb.to_device(c.y)
    f_eager, E_eager, n_eager = _call_noalloc(cb, y)
    torch.cuda.synchronize()
    f = torch.empty_like(f_eager)
    E = torch.empty_like(E_eager)
    ninv = torch.empty_like(n_eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        nat.check(nat.lib().cm_forces_noalloc(cb._h, _ptr(y), _ptr(f), _ptr(E),
                                              _ptr(ninv), _stream(side)))
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        f.fill_(float("nan"))
        E.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(f, f_eager) and torch.equal(E, E_eager), rep
        assert torch.equal(ninv, n_eager), rep
        cb.forces(y)  # eager work of the same handle between replays
        torch.cuda.synchronize()


def test_noalloc_rejects_oversize_handle():
    import torch
    from paper_2003_03130_amd import CellBatch
    from paper_2003_03130_amd import _native as nat
    from paper_2003_03130_amd.cells import _ptr, _stream
    c = small_sphere_case(1001)
    n_cells = 1000
    cb = CellBatch.template(n_cells, c.x, c.tets, tile_tets=256)
    need = 12 * cb.info["n_slots"]
    assert need > 16 << 20, need
    cb.set_params(*c.theta)
    y = cb.to_device(np.tile(c.y, (n_cells, 1)))
    f = cb.empty_nodes()
    E = torch.empty(n_cells, dtype=torch.float64, device=cb.device)
    rc = nat.lib().cm_forces_noalloc(cb._h, _ptr(y), _ptr(f), _ptr(E), None,
                                     _stream(None))
    assert rc == nat.CM_EINVAL
    msg = nat.lib().cm_last_error().decode()
    assert "scratch" in msg and str(16 << 20) in msg
