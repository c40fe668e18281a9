"""Calibration of (mu, kappa, w) per cell from force-indentation curves.

The paper fits its model to measured compression curves (Sec. "Results" of
the FluidFM comparison: Young's modulus and w from the best fit, w setting
the force upturn at large deformation).  Here the curve of every cell is the
quasi-static top-plate force at a list of plate positions
(QuasiStaticCompression.curve), and its derivative with respect to the
parameters comes from the adjoint of the equilibrium at each position (one
extra CG solve on the device, QuasiStaticCompression.plate_force_gradient).
The fit is a Levenberg-Marquardt iteration per cell on relative residuals
r_s = (F_s - F*_s) / max(|F*_s|, floor), in the coordinates (log mu,
log kappa, w) with w kept in [0, 1] and every step limited to max_step in
each coordinate; all cells of the batch are evaluated together and accept
or reject their own steps (a cell whose equilibria did not all converge
rejects its step).  Every force and derivative
comes from the device library; this module only forms the 3 x 3 normal
equations of each cell.
"""
from __future__ import annotations

import numpy as np


def _to_params(z):
    return np.stack([np.exp(z[:, 0]), np.exp(z[:, 1]), np.clip(z[:, 2], 0.0, 1.0)],
                    axis=1)


def _to_coords(theta):
    return np.stack([np.log(theta[:, 0]), np.log(theta[:, 1]), theta[:, 2]], axis=1)


def fit_curves(qs, y0, tops, bottom, F_target, theta0, iters=6, lam=1e-3,
               floor=None, max_step=0.5, log=None):
    """Levenberg-Marquardt fit of every cell's (mu, kappa, w) to its target
    curve.  qs: QuasiStaticCompression on the batch; y0: start positions
    (device SoA); tops: (S,) or (S, n_cells) plate heights; bottom: scalar or
    (n_cells,); F_target: (S, n_cells); theta0: (n_cells, 3).  Returns a dict
    with the parameters, per-cell losses and the history of every iteration
    (loss per cell, parameters, accepted steps).  Requires one material slot
    per cell (no regions)."""
    cb = qs.cb
    if cb.n_mat != cb.n_cells:
        raise ValueError("fit_curves needs one material slot per cell")
    F_target = np.asarray(F_target, dtype=np.float64)
    scale = np.maximum(np.abs(F_target), floor if floor is not None
                       else 1e-3 * np.abs(F_target).max())
    z = _to_coords(np.asarray(theta0, dtype=np.float64))
    lam = np.full(cb.n_cells, float(lam))

    def evaluate(theta, jac):
        cb.set_params(theta[:, 0], theta[:, 1], theta[:, 2])
        Ft, _, _, _ = qs.curve(y0, tops, bottom, jacobian=jac)
        ok = qs.cell_converged.all(axis=0)
        r = (Ft - F_target) / scale
        J = None
        if jac:
            # d r_s / d(log mu, log kappa, w)
            J = qs.jacobian / scale[:, :, None]
            J = J * np.stack([theta[:, 0], theta[:, 1], np.ones(len(theta))],
                             axis=1)[None]
        return r, J, ok

    theta = _to_params(z)
    r, J, ok = evaluate(theta, True)
    loss = (r ** 2).sum(axis=0)
    hist = [{"loss": loss.copy(), "theta": theta.copy(), "accepted": None,
             "converged": ok.copy()}]
    for it in range(iters):
        # per cell: (J^T J + lam diag(J^T J)) dz = -J^T r
        JtJ = np.einsum("sci,scj->cij", J, J)
        g = np.einsum("sci,sc->ci", J, r)
        D = np.einsum("cii->ci", JtJ)
        A = JtJ + lam[:, None, None] * np.einsum("ci,ij->cij", D, np.eye(3))
        dz = -np.linalg.solve(A, g[:, :, None])[:, :, 0]
        dz = np.clip(dz, -max_step, max_step)
        z_try = z + dz
        z_try[:, 2] = np.clip(z_try[:, 2], 0.0, 1.0)
        theta_try = _to_params(z_try)
        r_t, J_t, ok_t = evaluate(theta_try, True)
        loss_t = (r_t ** 2).sum(axis=0)
        acc = (loss_t < loss) & ok_t
        z = np.where(acc[:, None], z_try, z)
        r = np.where(acc[None, :], r_t, r)
        J = np.where(acc[None, :, None], J_t, J)
        loss = np.where(acc, loss_t, loss)
        lam = np.where(acc, lam / 10.0, lam * 10.0)
        theta = _to_params(z)
        hist.append({"loss": loss.copy(), "theta": theta.copy(),
                     "accepted": acc.copy(), "converged": ok_t.copy()})
        if log:
            log(f"iteration {it + 1}: loss {loss.sum():.3e}, accepted "
                f"{int(acc.sum())}/{len(acc)}")
    # leave the handle at the fitted parameters
    cb.set_params(theta[:, 0], theta[:, 1], theta[:, 2])
    return {"theta": theta, "loss": loss, "history": hist}
