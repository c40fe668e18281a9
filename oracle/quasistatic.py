"""FP64 reference for quasi-static plate compression (test infrastructure
only).

The cell rests on a bottom plate and a top plate is lowered (Sec.
"Simulation setup"); the repulsion that keeps nodes out of the plates is
given in the paper's unavailable supporting information, so the reading of
the plate-compression tests is used: the penalty force
p_z = -k max(0, z - top)^2 + k max(0, bottom - z)^2 derives from the potential
phi(z) = (k/3) [max(0, z - top)^3 + max(0, bottom - z)^3].  A quasi-static
state at plate position `top` minimises Pi(y) = E(y) + sum_nodes phi(y_z),
i.e. f(y) + p(y) = 0.  Here Pi is minimised by a library trust-region Newton
method (scipy, Krylov subproblem) on the oracle's energy, forces and
Hessian-vector products; the top-plate force is F = k sum max(0, y_z - top)^2
and the bottom-plate force k sum max(0, bottom - y_z)^2.  The energy density
grows without bound as J -> 0 from above, but with the real cube root it is
finite again for J < 0, so a finite step could jump over that barrier:
states that invert more tetrahedra than the start has are taken as
inadmissible (Pi = +inf there, which makes the trust region shrink).
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


def equilibrium(mesh, y0, theta, top, bottom, k, gtol=1e-10, maxiter=500):
    """Minimiser of Pi from y0 for an OracleMesh; returns (y, F_top,
    F_bottom, |grad Pi|_inf)."""
    y0 = np.asarray(y0, np.float64)
    shape = y0.shape
    ninv0 = mesh.forces(y0, theta)[2]

    def fun(v):
        y = v.reshape(shape)
        f, E, ninv = mesh.forces(y, theta)
        phi, p, _, _, _ = plate_terms(y, top, bottom, k)
        if ninv > ninv0:
            return np.inf, -(f + p).ravel()
        return E + phi, -(f + p).ravel()

    def hessp(v, d):
        y = v.reshape(shape)
        dv = d.reshape(shape)
        Hf, _ = mesh.jvp(y, theta, v=dv)          # (df/dy) d = -Hess(E) d
        _, _, h, _, _ = plate_terms(y, top, bottom, k)
        out = -Hf
        out[:, 2] += h * dv[:, 2]
        return out.ravel()

    res = minimize(fun, y0.ravel(), jac=True, hessp=hessp, method="trust-krylov",
                   options={"gtol": gtol, "maxiter": maxiter})
    y = res.x.reshape(shape)
    f, _, _ = mesh.forces(y, theta)
    _, p, _, Ft, Fb = plate_terms(y, top, bottom, k)
    return y, Ft, Fb, float(np.abs(f + p).max())


def force_curve(mesh, x, theta, tops, bottom, k, gtol=1e-10):
    """Quasi-static top-plate forces for decreasing plate heights `tops`,
    each solve started from the previous equilibrium."""
    y = np.asarray(x, np.float64).copy()
    F = []
    for t in tops:
        y, Ft, _, _ = equilibrium(mesh, y, theta, t, bottom, k, gtol)
        F.append(Ft)
    return np.array(F), y
