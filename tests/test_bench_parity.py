"""The benchmark's every-cell parity gate (bench.parity_all_cells) on the CPU:
fed the oracle's own outputs it reports zero errors and passes; a force or
ybar error above 1e-5 in one cell, or a thetabar error above both 1e-5 and
twice the cell's float32-input sensitivity, fails it; a thetabar error below
that sensitivity bound passes."""
import os
import sys

import numpy as np
import pytest

import oracle
from synth.configs import cotangent, uneven_batch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture(scope="module")
def case(tmp_path_factory):
    b = uneven_batch(n_cells=6, seed=41, tet_lo=500, tet_hi=3000, ladder=3)
    so = str(tmp_path_factory.mktemp("oracle") / "cm_oracle_omp.so")
    oracle.build_timing(so)
    v = cotangent(b.n_nodes, 42)
    eb = np.linspace(0.2, 0.8, b.n_cells)
    ob = oracle.OracleBatch(b.node_off, b.tet_off, b.x, b.tets, lib_path=so)
    f, E, yb, tb = ob.fwd_bwd(b.y.astype(np.float64), b.theta, v.astype(np.float64), eb)
    return b, so, v, eb, (f, E, yb, tb)


def _run(case, f=None, E=None, yb=None, tb=None):
    b, so, v, eb, ref = case
    dev = tuple(x.copy() if y is None else y for x, y in zip(ref, (f, E, yb, tb)))
    return bench.parity_all_cells(b, dev, v, eb, so, threads=2)


def test_exact_outputs_pass(case):
    r = _run(case)
    assert r["ok"] and r["cells"] == 6
    assert r["force"] == r["ybar"] == r["energy"] == r["thetabar"] == 0.0
    assert r["thetabar_above_1e-5"] == []


def test_force_and_ybar_errors_fail(case):
    b, _, _, _, (f, E, yb, tb) = case
    n0, n1 = b.node_off[3], b.node_off[4]
    g = f.copy()
    g[n0:n1] += 2e-5 * np.abs(f[n0:n1]).max()
    r = _run(case, f=g)
    assert not r["ok"] and 1.9e-5 < r["force"] < 2.1e-5
    y2 = yb.copy()
    y2[n0] += 2e-5 * np.abs(yb[n0:n1]).max()
    assert not _run(case, yb=y2)["ok"]
    E2 = E.copy()
    E2[2] *= 1 + 2e-6
    assert not _run(case, E=E2)["ok"]


def test_thetabar_bar_is_the_float32_input_sensitivity(case):
    b, _, _, _, (f, E, yb, tb) = case
    base = _run(case, tb=tb.copy())
    assert base["ok"]
    # a thetabar error of 1e-3 of its largest component in cell 1: above 1e-5,
    # and above twice the cell's sensitivity (rounding B and V0 to float32
    # moves these cells' thetabar by far less than 5e-4)
    t2 = tb.copy()
    t2[1, 0] += 1e-3 * np.abs(tb[1]).max()
    r = _run(case, tb=t2)
    assert not r["ok"]
    (rec,) = r["thetabar_above_1e-5"]
    assert rec["cell"] == 1 and abs(rec["err"] - 1e-3) < 1e-6
    assert 2 * rec["float32_input_sensitivity"] < 1e-3
    # an error below twice the sensitivity but above 1e-5 passes
    s = rec["float32_input_sensitivity"]
    if 2 * s > 1.2e-5:
        t3 = tb.copy()
        t3[1, 0] += 1.5 * s * np.abs(tb[1]).max()
        assert _run(case, tb=t3)["ok"]
