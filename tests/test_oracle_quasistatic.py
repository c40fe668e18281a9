"""Pins of the FP64 quasi-static compression oracle (CPU).

The equilibria come from a library minimiser of Pi = E + plate potential;
they are checked against what does not depend on that solver: the plate
forces balance (E is translation invariant, so the net elastic force is
zero), the explicit plate-compression steps of the C oracle (independent
code for the penalty law and the plate force) leave an equilibrium in place
and report the same top-plate force, and the force grows with the
compression."""
import warnings

import numpy as np
import pytest

import oracle
from oracle import quasistatic as qs
from synth.mesh import sphere_mesh

THETA = (1.0, 20.0, 0.5)
K = 100.0


@pytest.fixture(scope="module")
def path():
    x, tets = sphere_mesh(300, 3)
    m = oracle.OracleMesh(x, tets)
    top0, bot = x[:, 2].max(), x[:, 2].min()
    tops = top0 - 2.0 * np.array([0.02, 0.05, 0.1])
    out, y = [], x.copy()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        for t in tops:
            y, Ft, Fb, g = qs.equilibrium(m, y, THETA, t, bot, K)
            out.append((t, y.copy(), Ft, Fb, g))
    return m, bot, out


def test_equilibria_balance_the_plates(path):
    _, _, out = path
    F = [o[2] for o in out]
    for t, y, Ft, Fb, g in out:
        assert g <= 1e-6 * Ft
        assert abs(Ft - Fb) <= 1e-6 * Ft
    assert F[0] > 0 and np.all(np.diff(F) > 0)


def test_equilibrium_is_a_fixed_point_of_the_plate_steps(path):
    m, bot, out = path
    for t, y, Ft, _, _ in out:
        F, yf = m.relax_forward(y, THETA, np.full(50, t), bot, K, 4e-3)
        assert np.abs(F - Ft).max() <= 1e-6 * Ft
        assert np.abs(yf - y).max() <= 1e-8
