"""FP64 reference for quasi-static plate compression and sphere indentation
(test infrastructure only).

The cell rests on a bottom plate and a top plate is lowered, or a sphere
indents it from above (Sec. "Simulation setup", and the colloidal-probe
variant of Sec. "Validation with AFM experiments"); the repulsion that keeps
nodes out of the plates or the sphere is given in the paper's unavailable
supporting information, so the reading of the plate-compression tests is
used: the penalty force p_z = -k max(0, z - top)^2 + k max(0, bottom - z)^2
derives from the potential phi(z) = (k/3) [max(0, z - top)^3 +
max(0, bottom - z)^3].  The sphere (radius R, lowest point at height `top`,
axis (cx, cy), centre c = (cx, cy, top + R)) repels with the same law in the
penetration depth g = max(0, R - |y - c|): potential (k/3) g^3, force
k g^2 n on the node (n the unit vector from c to the node), and the force on
the sphere is the sum of the nodes' reactions, k g^2 (c_z - y_z) / |y - c|
upward.  A quasi-static state at indenter position `top` minimises Pi(y) =
E(y) + sum_nodes phi(y), i.e. f(y) + p(y) = 0.  Here Pi is minimised by a
library trust-region Newton method (scipy, Krylov subproblem) on the
oracle's energy, forces and Hessian-vector products; the top force is
F = k sum max(0, y_z - top)^2 for the plate and the bottom-plate force
k sum max(0, bottom - y_z)^2.  The energy density grows without bound as
J -> 0 from above, but with the real cube root it is finite again for J < 0,
so a finite step could jump over that barrier: states that invert more
tetrahedra than the start has are taken as inadmissible (Pi = +inf there,
which makes the trust region shrink).  Under the sphere, frictionless
contacts leave lateral sliding unstable (the contact normal tilts away from
the axis as the cell moves off it), so there the cell's centroid is held at
its lateral start position: Pi is minimised over positions shifted back to
that centroid, which removes the mean lateral components from the gradient
and the Hessian.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def plate_terms(y, top, bottom, k):
    """Penalty potential, force (N, 3), Hessian diagonal of the z entries,
    top and bottom plate forces."""
    z = y[:, 2]
    dt = np.maximum(z - top, 0.0)
    db = np.maximum(bottom - z, 0.0)
    phi = (k / 3.0) * (dt ** 3 + db ** 3).sum()
    p = np.zeros_like(y)
    p[:, 2] = k * (db * db - dt * dt)
    h = 2.0 * k * (dt + db)
    return phi, p, h, k * (dt * dt).sum(), k * (db * db).sum()


def sphere_terms(y, top, sphere, k):
    """Sphere indenter (R, cx, cy) with its lowest point at height top:
    penalty potential, force on the nodes (N, 3), the upward force on the
    sphere, and a function giving the potential's Hessian times v (N, 3):
    H v = 2 k g (n.v) n - k (g^2 / d) (v - (n.v) n), d = |y - c| (the
    potential (k/3) g^3 with g = R - d is differentiated twice)."""
    R, cx, cy = (float(v) for v in sphere)
    c = np.array([cx, cy, top + R])
    r = y - c
    d = np.sqrt((r * r).sum(axis=1))
    g = np.maximum(R - d, 0.0)
    inside = g > 0.0
    n = np.zeros_like(y)
    n[inside] = r[inside] / d[inside, None]
    phi = (k / 3.0) * (g ** 3).sum()
    p = (k * g * g)[:, None] * n
    F = (k * g * g * np.where(inside, (c[2] - y[:, 2]) / np.where(inside, d, 1.0), 0.0)).sum()

    def hess_v(v):
        nv = (n * v).sum(axis=1)
        gd = np.where(inside, g * g / np.where(inside, d, 1.0), 0.0)
        return (2.0 * k * g * nv)[:, None] * n - (k * gd)[:, None] * (v - nv[:, None] * n)
    return phi, p, F, hess_v


def contact_terms(y, top, bottom, k, sphere=None):
    """Penalty potential, force (N, 3), Hessian-vector function, top force
    (plate or sphere) and bottom-plate force; sphere = None: the top plate
    (plate_terms), else (R, cx, cy)."""
    phi, p, h, Ft, Fb = plate_terms(y, top, bottom, k)
    if sphere is None:
        def hess_v(v):
            out = np.zeros_like(v)
            out[:, 2] = h * v[:, 2]
            return out
        return phi, p, hess_v, Ft, Fb
    # the bottom plate alone from plate_terms, the sphere in place of the top
    z = y[:, 2]
    db = np.maximum(bottom - z, 0.0)
    phi_s, p_s, Fs, hv_s = sphere_terms(y, top, sphere, k)
    pb = np.zeros_like(y)
    pb[:, 2] = k * db * db

    def hess_v(v):
        out = hv_s(v)
        out[:, 2] += 2.0 * k * db * v[:, 2]
        return out
    return (k / 3.0) * (db ** 3).sum() + phi_s, pb + p_s, hess_v, Fs, k * (db * db).sum()


def equilibrium(mesh, y0, theta, top, bottom, k, gtol=1e-10, maxiter=500, sphere=None):
    """Minimiser of Pi from y0 for an OracleMesh (top plate, or the sphere
    indenter (R, cx, cy) with its lowest point at top, the centroid held
    laterally); returns (y, F_top, F_bottom, |grad Pi|_inf) (the gradient
    without its mean lateral part under the sphere, which the holding force
    takes)."""
    y0 = np.asarray(y0, np.float64)
    shape = y0.shape
    ninv0 = mesh.forces(y0, theta)[2]
    c0 = y0[:, :2].mean(axis=0)

    def place(v):
        # positions: v itself (plates), or v shifted to the held centroid
        y = v.reshape(shape)
        if sphere is None:
            return y
        y = y.copy()
        y[:, :2] += c0 - y[:, :2].mean(axis=0)
        return y

    def lateral_free(g):
        # the transpose of place's derivative: mean x, y components removed
        if sphere is None:
            return g
        g = g.copy()
        g[:, :2] -= g[:, :2].mean(axis=0)
        return g

    def fun(v):
        y = place(v)
        f, E, ninv = mesh.forces(y, theta)
        phi, p, _, _, _ = contact_terms(y, top, bottom, k, sphere)
        grad = lateral_free(-(f + p)).ravel()
        if ninv > ninv0:
            return np.inf, grad
        return E + phi, grad

    def hessp(v, d):
        y = place(v)
        dv = lateral_free(d.reshape(shape))
        Hf, _ = mesh.jvp(y, theta, v=dv)          # (df/dy) d = -Hess(E) d
        _, _, hess_v, _, _ = contact_terms(y, top, bottom, k, sphere)
        return lateral_free(-Hf + hess_v(dv)).ravel()

    res = minimize(fun, y0.ravel(), jac=True, hessp=hessp, method="trust-krylov",
                   options={"gtol": gtol, "maxiter": maxiter})
    y = place(res.x)
    f, _, _ = mesh.forces(y, theta)
    _, p, _, Ft, Fb = contact_terms(y, top, bottom, k, sphere)
    return y, Ft, Fb, float(np.abs(lateral_free(f + p)).max())


def force_curve(mesh, x, theta, tops, bottom, k, gtol=1e-10, sphere=None):
    """Quasi-static top forces (plate, or sphere indenter (R, cx, cy)) for
    decreasing heights `tops`, each solve started from the previous
    equilibrium."""
    y = np.asarray(x, np.float64).copy()
    F = []
    for t in tops:
        y, Ft, _, _ = equilibrium(mesh, y, theta, t, bottom, k, gtol, sphere=sphere)
        F.append(Ft)
    return np.array(F), y
