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


# ---- sphere indenter (the colloidal-probe setup) ----------------------------

def _sphere_cloud(seed=11):
    """Nodes around the lowest point of a sphere of radius 0.7 (apex at
    z = 0.1), a third of them inside it."""
    rng = np.random.default_rng(seed)
    y = rng.uniform(-0.4, 0.4, size=(60, 3))
    y[:, 2] = rng.uniform(0.0, 0.3, size=60)
    return y, 0.1, (0.7, 0.05, -0.03)


def test_sphere_force_is_minus_the_gradient_of_its_potential():
    y, top, sph = _sphere_cloud()
    phi, p, F, _ = qs.sphere_terms(y, top, sph, K)
    assert (p != 0).any(axis=1).sum() >= 10
    h = 1e-6
    g = np.zeros_like(y)
    for i in range(len(y)):
        for a in range(3):
            yp, ym = y.copy(), y.copy()
            yp[i, a] += h
            ym[i, a] -= h
            g[i, a] = (qs.sphere_terms(yp, top, sph, K)[0] - qs.sphere_terms(ym, top, sph, K)[0]) / (2 * h)
    assert np.abs(-g - p).max() <= 1e-6 * np.abs(p).max()


def test_sphere_hessian_is_the_derivative_of_its_force():
    y, top, sph = _sphere_cloud(12)
    _, p, _, hv = qs.sphere_terms(y, top, sph, K)
    v = np.random.default_rng(5).standard_normal(y.shape)
    h = 1e-6
    pp = qs.sphere_terms(y + h * v, top, sph, K)[1]
    pm = qs.sphere_terms(y - h * v, top, sph, K)[1]
    dp = (pp - pm) / (2 * h)           # d p = -Hess(phi) v
    assert np.abs(dp + hv(v)).max() <= 1e-5 * np.abs(hv(v)).max()


def test_sphere_force_on_the_indenter_is_the_upward_sum_of_reactions():
    """The sphere's force equals the z-component of the nodes' penalty forces
    with the sign reversed (Newton's third law), computed independently of
    the direction field: the derivative of the potential along a rigid
    downward move of the sphere."""
    y, top, sph = _sphere_cloud(13)
    _, p, F, _ = qs.sphere_terms(y, top, sph, K)
    h = 1e-7
    dphi = (qs.sphere_terms(y, top - h, sph, K)[0] - qs.sphere_terms(y, top + h, sph, K)[0]) / (2 * h)
    # lowering the sphere by dt raises the stored energy by F dt
    assert F > 0 and abs(dphi - F) <= 1e-6 * F
    assert abs(F + p[:, 2].sum()) <= 1e-12 * F


def test_large_sphere_acts_like_the_top_plate():
    """A sphere of radius 1e5 over a cell of radius 1 differs from the flat
    plate at its lowest point by less than r^2 / (2 R) = 5e-6 in every
    node's penetration."""
    x, _ = sphere_mesh(300, 3)
    y = x.copy()
    top = x[:, 2].max() - 0.1
    cx, cy = x[:, 0].mean(), x[:, 1].mean()
    phi_p, p_p, _, Ft_p, _ = qs.plate_terms(y, top, -10.0, K)
    phi_s, p_s, Ft_s, _ = qs.sphere_terms(y, top, (1e5, cx, cy), K)
    assert abs(Ft_s - Ft_p) <= 1e-3 * Ft_p
    assert abs(phi_s - phi_p) <= 1e-3 * phi_p
    assert np.abs(p_s - p_p).max() <= 1e-3 * np.abs(p_p).max()


@pytest.fixture(scope="module")
def sphere_path():
    x, tets = sphere_mesh(300, 3)
    m = oracle.OracleMesh(x, tets)
    top0, bot = x[:, 2].max(), x[:, 2].min()
    sph = (0.66, x[:, 0].mean(), x[:, 1].mean())
    # from 5 % of the diameter: at 2 % the sphere holds a single node with a
    # force below the minimiser's absolute gradient tolerance
    tops = top0 - 2.0 * np.array([0.05, 0.1, 0.2])
    out, y = [], x.copy()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        for t in tops:
            y, Ft, Fb, g = qs.equilibrium(m, y, THETA, t, bot, K, gtol=1e-12, sphere=sph)
            out.append((t, y.copy(), Ft, Fb, g))
    return m, bot, sph, out


def test_sphere_equilibria_balance_the_indenter_and_the_plate(sphere_path):
    """Equilibria with the centroid held laterally: the indenter's and the
    plate's forces balance (E is translation invariant, so the net vertical
    elastic force is zero), the centroid has not moved, the force grows with
    the indentation."""
    m, _, sph, out = sphere_path
    F = [o[2] for o in out]
    for t, y, Ft, Fb, g in out:
        # the minimiser stops at |grad|_inf ~ 3e-9; summed over the ~10
        # contact nodes that bounds the balance at ~1e-6 of the smallest force
        assert g <= 1e-6 * Ft
        assert abs(Ft - Fb) <= 1e-5 * Ft
        assert np.abs(y[:, :2].mean(axis=0) - np.array(sph[1:])).max() <= 1e-12
    assert F[0] > 0 and np.all(np.diff(F) > 0)


def test_sphere_indents_less_than_the_plate_compresses(sphere_path):
    """At the same travel the sphere pushes on a smaller contact than the
    plate, so its force is smaller."""
    m, bot, sph, out = sphere_path
    t, _, Fs, _, _ = out[-1]
    y0 = out[0][1]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        _, Fp, _, _ = qs.equilibrium(m, y0, THETA, t, bot, K)
    assert 0 < Fs < Fp
