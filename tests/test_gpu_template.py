"""Shared-mesh batches (cm_template_create) on the GPU: several copies of one
reference mesh, each with its own deformation and parameters.  The tet data
is stored once and the tiles of all copies are interleaved; forces, energies,
inverted counts, the adjoint and the parameter gradient must equal, bit for
bit, those of a batch that holds every copy in its own arrays, and match the
FP64 oracle to the parity tolerance of the single-mesh tests."""
import numpy as np
import pytest

import oracle
from gpu_util import force_rel_err, require_gpu
from synth.configs import cotangent, template_batch

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _pair(b, **kw):
    from paper_2003_03130_amd import CellBatch
    n, m = b.info["template_nodes"], b.info["template_tets"]
    tp = CellBatch.template(b.n_cells, b.x[:n], b.tets[:m], **kw)
    ds = CellBatch(b.node_off, b.tet_off, b.x, b.tets, **kw)
    for cb in (tp, ds):
        cb.set_params(b.theta[:, 0], b.theta[:, 1], b.theta[:, 2])
    return tp, ds


def _run(cb, b, v, eb):
    import torch
    y = cb.to_device(b.y)
    ninv = torch.zeros(b.n_cells, dtype=torch.int32, device=cb.device)
    f, E = cb.forces(y, n_inverted=ninv)
    yb, tb = cb.backward(y, cb.to_device(v), eb)
    torch.cuda.synchronize()
    return (cb.to_host(f), E.cpu().numpy(), ninv.cpu().numpy(),
            cb.to_host(yb), tb.cpu().numpy())


@pytest.mark.parametrize("n_cells,n_target,tile", [(5, 1000, 768),
                                                   (24, 400, 128),
                                                   (3, 4000, 4096)])
def test_template_equals_distinct_arrays(n_cells, n_target, tile):
    import torch
    b = template_batch(n_cells, n_target, seed=40 + n_cells)
    tp, ds = _pair(b, tile_tets=tile)
    assert tp.n_nodes == ds.n_nodes == b.n_nodes
    assert tp.n_tets == ds.n_tets == b.n_tets
    assert tp.info["n_chunks"] * n_cells == ds.info["n_chunks"]
    v = cotangent(b.n_nodes, 3)
    eb = torch.linspace(0.2, 1.0, n_cells, dtype=torch.float64, device=tp.device)
    got, want = _run(tp, b, v, eb), _run(ds, b, v, eb)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    # launch shapes do not change the bits (shapes whose LDS does not fit
    # are refused by the library and skipped)
    from paper_2003_03130_amd import CellmechError
    tried = 0
    for waves, bpcu in [(2, 0), (1, 2)]:
        try:
            tp.set_launch(waves, bpcu)
            again = _run(tp, b, v, eb)
        except CellmechError:
            continue
        tried += 1
        for g, w in zip(again, want):
            assert np.array_equal(g, w)
    assert tried >= 1


def test_template_against_oracle():
    import torch
    b = template_batch(4, 2000, seed=91)
    tp, _ = _pair(b)
    v = cotangent(b.n_nodes, 8)
    eb = torch.full((b.n_cells,), 0.7, dtype=torch.float64, device=tp.device)
    f, E, ninv, yb, tb = _run(tp, b, v, eb)
    tb = tb.reshape(-1, 3)
    for c in range(b.n_cells):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        yd = cell.y.astype(np.float64)
        fo, Eo, no = m.forces(yd, cell.theta)
        assert force_rel_err(f[n0:n1], fo) <= TOL
        assert abs(E[c] - Eo) <= TOL * abs(Eo)
        assert ninv[c] == no
        yo, to = m.backward(yd, cell.theta, v[n0:n1].astype(np.float64), 0.7)
        assert np.abs(yb[n0:n1] - yo).max() <= TOL * np.abs(yo).max()
        assert np.abs(tb[c] - to).max() <= TOL * np.abs(to).max()


def test_template_graph_replay_and_percell_rejected():
    import torch
    from paper_2003_03130_amd import CellmechError
    from paper_2003_03130_amd import _native as nat
    b = template_batch(6, 800, seed=17)
    tp, _ = _pair(b)
    y = tp.to_device(b.y)
    v = tp.to_device(cotangent(b.n_nodes, 2))
    eb = torch.full((b.n_cells,), 0.5, dtype=torch.float64, device=tp.device)
    fe, Ee = tp.forces(y)
    ye, te = tp.backward(y, v, eb)
    fe, Ee, ye, te = fe.clone(), Ee.clone(), ye.clone(), te.clone()
    f, yb = tp.empty_nodes(), tp.empty_nodes()
    E = torch.empty(b.n_cells, dtype=torch.float64, device=tp.device)
    tb = torch.empty(3 * b.n_cells, dtype=torch.float64, device=tp.device)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tp.graph_capture(1, y, f, E, None, v, eb, yb, tb, stream=s)
    for _ in range(3):
        for t in (f, E, yb, tb):
            t.zero_()
        torch.cuda.synchronize()
        tp.graph_launch(stream=s)
        s.synchronize()
        assert torch.equal(f, fe) and torch.equal(E, Ee)
        assert torch.equal(yb, ye) and torch.equal(tb, te)
        tp.forces(y)
        torch.cuda.synchronize()
    for call in (lambda: tp.forces(y, percell=True),
                 lambda: tp.backward(y, v, eb, percell=True)):
        with pytest.raises(CellmechError) as ei:
            call()
        assert ei.value.status == nat.CM_EINVAL


def test_template_backward_restricted_to_flagged_cells():
    """cm_forces_backward_cells on a shared-mesh batch (tiles interleaved by
    copy): flagged copies bitwise equal to the full backward, the others
    untouched."""
    import torch
    b = template_batch(6, 800, seed=93)
    tp, _ = _pair(b, tile_tets=128)
    y = tp.to_device(b.y)
    v = tp.to_device(cotangent(b.n_nodes, 94))
    eb = torch.linspace(-1.0, 1.0, b.n_cells, dtype=torch.float64, device=tp.device)
    y0, t0 = tp.backward(y, v, eb)
    y0, t0 = tp.to_host(y0), t0.cpu().numpy().reshape(b.n_cells, 3)
    sel = torch.tensor([0.0, 1.0, 1.0, 0.0, 0.0, 1.0], dtype=torch.float64,
                       device=tp.device)
    yb = torch.full_like(tp.empty_nodes(), 5.0)
    tb = torch.full((3 * b.n_cells,), 9.0, dtype=torch.float64, device=tp.device)
    tp.backward(y, v, eb, yb, tb, cells=sel)
    y1, t1 = tp.to_host(yb), tb.cpu().numpy().reshape(b.n_cells, 3)
    for c in range(b.n_cells):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        if sel[c] != 0:
            assert np.array_equal(y1[n0:n1], y0[n0:n1]) and np.array_equal(t1[c], t0[c])
        else:
            assert np.all(y1[n0:n1] == 5.0) and np.all(t1[c] == 9.0)
