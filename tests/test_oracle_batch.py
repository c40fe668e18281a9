"""The oracle's timing mode (forward + backward of a range of cells, OpenMP
over cells) runs the single-cell routines unchanged: its results equal those
of one call per cell bitwise, in the -O2 test build and, within rounding, in
the -O3 -march=native -fopenmp timing build on several threads."""
import os
import tempfile

import numpy as np

import oracle
from synth.configs import cotangent, uneven_batch


def _case():
    b = uneven_batch(n_cells=5, seed=17, tet_lo=500, tet_hi=3000, ladder=3)
    v = cotangent(b.n_nodes, 18)
    e = np.linspace(0.2, 1.0, b.n_cells)
    return b, v, e


def _per_cell(b, v, e):
    out = []
    for c in range(b.n_cells):
        cell = b.cell(c)
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        m = oracle.OracleMesh(cell.x, cell.tets)
        f, E, _ = m.forces(cell.y, cell.theta)
        yb, tb = m.backward(cell.y, cell.theta, v[n0:n1], e[c])
        out.append((f, E, yb, tb))
    return out


def test_batch_mode_equals_per_cell_calls():
    b, v, e = _case()
    ref = _per_cell(b, v, e)
    ob = oracle.OracleBatch(b.node_off, b.tet_off, b.x, b.tets)
    f, E, yb, tb = ob.fwd_bwd(b.y, b.theta, v, e)
    for c, (fo, Eo, yo, to) in enumerate(ref):
        n0, n1 = b.node_off[c], b.node_off[c + 1]
        assert np.array_equal(f[n0:n1], fo) and E[c] == Eo
        assert np.array_equal(yb[n0:n1], yo) and np.array_equal(tb[c], to)
    # a sub-range leaves the other cells' outputs at zero
    f2, E2, _, _ = ob.fwd_bwd(b.y, b.theta, v, e, 1, 3)
    assert np.array_equal(f2[b.node_off[1]:b.node_off[3]], f[b.node_off[1]:b.node_off[3]])
    assert E2[0] == 0.0 and E2[3] == 0.0 and E2[1] == E[1]


def test_timing_build_on_threads():
    b, v, e = _case()
    so = os.path.join(tempfile.mkdtemp(), "libcm_oracle_omp.so")
    oracle.build_timing(so)
    ob = oracle.OracleBatch(b.node_off, b.tet_off, b.x, b.tets, lib_path=so)
    assert ob.threads(3) == 3
    f, E, yb, tb = ob.fwd_bwd(b.y, b.theta, v, e)
    ref = oracle.OracleBatch(b.node_off, b.tet_off, b.x, b.tets).fwd_bwd(
        b.y, b.theta, v, e)
    for a, r in zip((f, E, yb, tb), ref):
        assert np.abs(a - r).max() <= 1e-12 * np.abs(r).max()
