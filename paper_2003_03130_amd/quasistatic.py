"""Quasi-static plate compression of a batch of cells (force-indentation
curves): each plate position is brought to equilibrium by Newton steps whose
systems are solved per cell by conjugate gradients on the device (cm_qs_*;
Hessian-vector products from cm_forces_backward).  Python only orders the
calls and checks convergence flags between Newton steps."""
from __future__ import annotations

import numpy as np

from . import _native as nat
from .cells import _ptr, _stream


class QuasiStaticCompression:
    """batch: CellBatch with parameters set; k_plate: plate penalty;
    rel_tol / abs_tol: equilibrium when |f + p|_2 <= max(abs_tol,
    rel_tol |p|_2) per cell (p the plate forces) or when a Newton step
    moves no node by more than step_tol (the float32 floor of the residual);
    cg_tol: relative CG residual; cap: largest node move per Newton step."""

    def __init__(self, batch, k_plate, rel_tol=1e-3, abs_tol=1e-9,
                 step_tol=1e-6, cg_tol=1e-3, max_newton=40, max_cg=400,
                 cap=0.05):
        import torch
        self.cb = batch
        self.k = float(k_plate)
        self.rel_tol, self.abs_tol = float(rel_tol), float(abs_tol)
        self.step_tol = float(step_tol)
        self.cg_tol, self.cap = float(cg_tol), float(cap)
        self.max_newton, self.max_cg = int(max_newton), int(max_cg)
        dev = batch.device
        self._f = batch.empty_nodes()
        self._r = batch.empty_nodes()
        self._p = batch.empty_nodes()
        self._x = batch.empty_nodes()
        self._Ap = batch.empty_nodes()
        self._ybar = batch.empty_nodes()
        self._E = torch.empty(batch.n_cells, dtype=torch.float64, device=dev)
        self._tb = torch.empty(3 * batch.n_mat, dtype=torch.float64,
                               device=dev)
        self.state = torch.zeros(batch.n_cells, 8, dtype=torch.float64,
                                 device=dev)
        self.force = torch.zeros(batch.n_cells, 2, dtype=torch.float64,
                                 device=dev)
        self.stats = {"newton": 0, "cg": 0}

    def _residual(self, y, plate, restart=False):
        cb = self.cb
        cb.forces(y, self._f, self._E)
        nat.check(nat.lib().cm_qs_residual(
            cb._h, _ptr(y), _ptr(self._f), _ptr(plate), self.k, self.abs_tol,
            self.rel_tol, self.step_tol, int(restart), _ptr(self._r),
            _ptr(self._p), _ptr(self._x), _ptr(self.state), _ptr(self.force),
            _stream(None)))

    def equilibrate(self, y, plate):
        """Newton iterations at one plate position (plate: float64 device
        tensor (n_cells, 2) = top, bottom); y (device SoA) is updated in
        place.  Returns True when every cell met the tolerance."""
        cb = self.cb
        for it in range(self.max_newton):
            self._residual(y, plate, restart=(it == 0))
            if not bool((self.state[:, 2] > 0).any()):
                return True
            self.stats["newton"] += 1
            for j in range(self.max_cg):
                cb.backward(y, self._p, None, self._ybar, self._tb)
                nat.check(nat.lib().cm_qs_cg_step(
                    cb._h, _ptr(y), _ptr(plate), self.k, self.cg_tol,
                    _ptr(self._ybar), _ptr(self._x), _ptr(self._r),
                    _ptr(self._p), _ptr(self._Ap), _ptr(self.state),
                    _stream(None)))
                self.stats["cg"] += 1
                if j % 8 == 7 and not bool((self.state[:, 2] > 0).any()):
                    break
            nat.check(nat.lib().cm_qs_update(
                cb._h, _ptr(self._x), self.cap, _ptr(y), _ptr(self.state),
                _stream(None)))
        self._residual(y, plate)
        return not bool((self.state[:, 2] > 0).any())

    def curve(self, y0, tops, bottom):
        """Top-plate force of every cell at each plate height (tops: (S,) or
        (S, n_cells); bottom: scalar or (n_cells,)), starting from y0 and
        each position from the previous equilibrium (affine predictor).
        Returns (forces (S, n_cells) top, (S, n_cells) bottom, converged (S,),
        final positions)."""
        import torch
        cb = self.cb
        tops = np.asarray(tops, dtype=np.float64)
        if tops.ndim == 1:
            tops = np.repeat(tops[:, None], cb.n_cells, axis=1)
        bot = np.broadcast_to(np.asarray(bottom, np.float64), (cb.n_cells,))
        y = y0.clone()
        plates = torch.from_numpy(np.stack([tops, np.broadcast_to(
            bot, tops.shape)], axis=2).copy()).to(cb.device)
        Ft, Fb, ok = [], [], []
        for s in range(len(tops)):
            if s > 0:
                nat.check(nat.lib().cm_qs_predict(
                    cb._h, _ptr(plates[s - 1]), _ptr(plates[s]), _ptr(y),
                    _stream(None)))
            ok.append(self.equilibrate(y, plates[s]))
            Ft.append(self.force[:, 0].cpu().numpy().copy())
            Fb.append(self.force[:, 1].cpu().numpy().copy())
        return np.array(Ft), np.array(Fb), np.array(ok), y
