"""Quasi-static plate compression or sphere indentation of a batch of cells
(force-indentation curves): each plate or indenter position is brought to
equilibrium by Newton steps whose
systems are solved per cell by conjugate gradients on the device (cm_qs_*;
Hessian-vector products from cm_forces_backward), each step globalised by a
backtracking (Armijo) line search on the total potential and solved only as
accurately as the Newton residual's progress asks for (inexact Newton with
Eisenstat and Walker's forcing term, per cell on the device), the conjugate
gradients preconditioned by the inverse 3x3 node blocks of the small-strain
stiffness plus the penalty Hessian (block Jacobi).  Python only
orders the calls and checks convergence flags between Newton steps."""
from __future__ import annotations

import numpy as np

from . import _native as nat
from .cells import _ptr, _stream


class QuasiStaticCompression:
    """batch: CellBatch with parameters set; k_plate: plate penalty;
    rel_tol / abs_tol: equilibrium when |f + p|_2 <= max(abs_tol,
    rel_tol |p|_2, floor_factor rho) per cell (rel_tol None: 1e-3 under the
    plates, 1e-5 under a sphere, whose contact leaves soft tilting modes
    along which a residual of 1e-3 |p| moved the sphere's force by up to
    2 %; at 1e-5 it is within 3e-4 of the FP64 equilibrium; p the plate forces, rho the
    float32 floor of the residual, estimated at every plate position) or
    when a Newton step moves no node by more than step_tol; cg_tol: smallest
    relative CG residual; eta_max: largest forcing term of the inexact Newton
    steps (0: every CG solve to cg_tol); precondition: block-Jacobi CG;
    fused_cg: each CG iteration as one library call with its Hessian-vector
    product (cm_qs_cg_iteration) instead of two; pipelined_checks: the host
    reads the CG convergence check of a block of iterations only after the
    next block is queued (same iterates; False: it waits after every block);
    cap: largest node move per Newton step; armijo: sufficient decrease of
    the line search, which gives up below min_move; sphere_radius > 0: a
    sphere of that radius indents the cells instead of the top plate (its
    lowest point at the "top" height, its axis at sphere_axis (n_cells, 2),
    by default each cell's centroid at the first equilibrium; the centroids
    are held laterally, see cm_qs_set_indenter)."""

    def __init__(self, batch, k_plate, rel_tol=None, abs_tol=1e-9,
                 step_tol=1e-6, floor_factor=2.0, cg_tol=1e-3, max_newton=40,
                 max_cg=400, cap=0.05, armijo=1e-4, min_move=1e-7,
                 max_backtrack=12, eta_max=0.5, precondition=True,
                 fused_cg=True, pipelined_checks=True, sphere_radius=0.0,
                 sphere_axis=None):
        import torch
        self.cb = batch
        self.k = float(k_plate)
        if rel_tol is None:
            rel_tol = 1e-5 if float(sphere_radius) > 0.0 else 1e-3
        self.rel_tol, self.abs_tol = float(rel_tol), float(abs_tol)
        self.step_tol = float(step_tol)
        self.floor_factor = float(floor_factor)
        self.armijo, self.min_move = float(armijo), float(min_move)
        self.max_backtrack = int(max_backtrack)
        self.cg_tol, self.cap = float(cg_tol), float(cap)
        self.eta_max = float(eta_max)
        self.precondition = bool(precondition)
        # one call per CG iteration (cm_qs_cg_iteration) or the two-call
        # route (cm_forces_backward_cells + cm_qs_cg_step); bitwise equal
        self.fused_cg = bool(fused_cg)
        self.pipelined_checks = bool(pipelined_checks)
        self.sphere_radius = float(sphere_radius)
        self._sphere_axis = None if sphere_axis is None else torch.as_tensor(
            np.asarray(sphere_axis, dtype=np.float64).reshape(batch.n_cells, 2)).to(batch.device)
        if self.precondition:
            self._kel = torch.empty(6 * batch.n_nodes, dtype=torch.float32,
                                    device=batch.device)
            self._minv = torch.empty_like(self._kel)
        else:
            self._kel = self._minv = None
        self.max_newton, self.max_cg = int(max_newton), int(max_cg)
        dev = batch.device
        self._f = batch.empty_nodes()
        self._r = batch.empty_nodes()
        self._p = batch.empty_nodes()
        self._x = batch.empty_nodes()
        self._Ap = batch.empty_nodes()
        self._ybar = batch.empty_nodes()
        self._rn = batch.empty_nodes()
        self._yt = batch.empty_nodes()
        self._ft = batch.empty_nodes()
        self._Et = torch.empty(batch.n_cells, dtype=torch.float64, device=dev)
        # inverted tetrahedra at y and at the line-search trial: a trial may
        # not invert more than y has (the barrier at J = 0)
        self._ninv = torch.zeros(batch.n_cells, dtype=torch.int32, device=dev)
        self._ninv_t = torch.zeros(batch.n_cells, dtype=torch.int32, device=dev)
        self._E = torch.empty(batch.n_cells, dtype=torch.float64, device=dev)
        self._tb = torch.empty(3 * batch.n_mat, dtype=torch.float64,
                               device=dev)
        self.state = torch.zeros(batch.n_cells, 16, dtype=torch.float64,
                                 device=dev)
        self.force = torch.zeros(batch.n_cells, 2, dtype=torch.float64,
                                 device=dev)
        self.stats = {"newton": 0, "cg": 0, "trials": 0}
        self._flags, self._flag_i = None, 0  # pinned flags of _active_async

    def cell_centroids(self, y):
        """(n_cells, 2) float64 device tensor: every cell's mean x and y."""
        import torch
        cb = self.cb
        N = cb.n_nodes
        counts = torch.from_numpy(np.diff(cb.node_off)).to(cb.device)
        cell = torch.repeat_interleave(torch.arange(cb.n_cells, device=cb.device), counts)
        out = torch.zeros(cb.n_cells, 2, dtype=torch.float64, device=cb.device)
        out[:, 0].index_add_(0, cell, y[:N].double())
        out[:, 1].index_add_(0, cell, y[N:2 * N].double())
        return out / counts[:, None].double()

    def _set_contact(self, y):
        """Puts this solver's top contact on the handle, which holds one
        (plates, or the sphere with its axes)."""
        cb = self.cb
        if self.sphere_radius > 0.0:
            if self._sphere_axis is None:
                self._sphere_axis = self.cell_centroids(y).contiguous()
            nat.check(nat.lib().cm_qs_set_indenter(
                cb._h, self.sphere_radius, _ptr(self._sphere_axis), _stream(None)))
        else:
            nat.check(nat.lib().cm_qs_set_indenter(cb._h, 0.0, None, _stream(None)))

    def _residual(self, y, plate, restart=False):
        cb = self.cb
        cb.forces(y, self._f, self._E, self._ninv)
        nat.check(nat.lib().cm_qs_residual(
            cb._h, _ptr(y), _ptr(self._f), _ptr(self._E), _ptr(plate), self.k,
            self.abs_tol, self.rel_tol, self.step_tol, self.floor_factor,
            self.eta_max, int(restart), _ptr(self._r), _ptr(self._p), _ptr(self._x),
            _ptr(self._rn), _ptr(self.state), _ptr(self.force), _ptr(self._kel),
            _ptr(self._minv), _stream(None)))

    def _active(self, col):
        return bool((self.state[:, col] > 0).any())

    def _active_async(self, col):
        """Queues on the current stream a check whether any cell has state
        column col set, copied into pinned host memory; returns a function
        that waits for that copy alone and returns the answer."""
        import torch
        if self._flags is None:
            self._flags = [torch.zeros(1, dtype=torch.bool, pin_memory=True)
                           for _ in range(2)]
        buf = self._flags[self._flag_i]
        self._flag_i ^= 1
        buf.copy_((self.state[:, col] > 0).any().reshape(1), non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()

        def wait():
            ev.synchronize()
            return bool(buf[0])
        return wait

    def _cg_loop(self, y, plate, tol, max_iter, counter):
        """CG iterations for every cell still active (state column 2), in
        blocks of 8, until a block ends with no cell active, or max_iter.
        The check after a block runs on the device, and the host reads it
        only once the next block is queued, so the device does not wait for
        the host between blocks; the block queued behind the last one that
        mattered runs as no-ops (every kernel skips finished cells), so the
        iterates are those of a loop that stops right after that block, and
        the count leaves that block out."""
        cb = self.cb
        lib, st = nat.lib(), _stream(None)
        if self.fused_cg:
            args = (cb._h, _ptr(y), _ptr(plate), self.k, float(tol),
                    _ptr(self._ybar), _ptr(self._x), _ptr(self._r),
                    _ptr(self._p), _ptr(self._Ap), _ptr(self.state),
                    _ptr(self._minv), st)
            step = lib.cm_qs_cg_iteration

            def iteration():
                nat.check(step(*args))
        else:
            # Hessian-vector products only for the cells still in CG (state
            # column 2 as the cell flags; no parameter gradient), then one
            # CG iteration
            flags = self.state[:, 2]
            hvp_args = (cb._h, _ptr(y), _ptr(self._p), None, _ptr(flags),
                        flags.stride(0), _ptr(self._ybar), None, st)
            cg_args = (cb._h, _ptr(y), _ptr(plate), self.k, float(tol),
                       _ptr(self._ybar), _ptr(self._x), _ptr(self._r),
                       _ptr(self._p), _ptr(self._Ap), _ptr(self.state),
                       _ptr(self._minv), st)

            def iteration():
                nat.check(lib.cm_forces_backward_cells(*hvp_args))
                nat.check(lib.cm_qs_cg_step(*cg_args))
        pending, j = None, 0
        while j < max_iter:
            n = min(8, max_iter - j)
            for _ in range(n):
                iteration()
            j += n
            self.stats[counter] = self.stats.get(counter, 0) + n
            check = self._active_async(2)
            if not self.pipelined_checks:
                if not check():
                    break
                continue
            if pending is not None and not pending():
                self.stats[counter] -= n  # queued after the solve ended
                break
            pending = check

    def equilibrate(self, y, plate):
        """Newton iterations at one plate position (plate: float64 device
        tensor (n_cells, 2) = top, bottom); y (device SoA) is updated in
        place.  Returns True when every cell met the tolerance."""
        self._set_contact(y)
        cb = self.cb
        if self.precondition:  # for the current parameters
            nat.check(nat.lib().cm_qs_stiffness(cb._h, _ptr(self._kel),
                                                _stream(None)))
        # float32 floor of the residual at this plate position
        nat.check(nat.lib().cm_qs_noise(cb._h, _ptr(y), _ptr(self._Ap),
                                        _stream(None)))
        cb.backward(y, self._Ap, None, self._ybar, self._tb)
        nat.check(nat.lib().cm_qs_floor(
            cb._h, _ptr(y), _ptr(plate), self.k, _ptr(self._Ap),
            _ptr(self._ybar), _ptr(self.state), _stream(None)))
        for it in range(self.max_newton):
            self._residual(y, plate, restart=(it == 0))
            if not self._active(11):
                return True
            self.stats["newton"] += 1
            self._cg_loop(y, plate, self.cg_tol, self.max_cg, "cg")
            self._line_search(y, plate)
        self._residual(y, plate)
        return not self._active(11)

    def _line_search(self, y, plate):
        cb = self.cb
        nat.check(nat.lib().cm_qs_ls_start(
            cb._h, _ptr(self._x), _ptr(self._rn), self.cap, _ptr(y),
            _ptr(self._yt), _ptr(self.state), _stream(None)))
        for _ in range(self.max_backtrack):
            if not self._active(12):
                return
            cb.forces(self._yt, self._ft, self._Et, self._ninv_t)
            nat.check(nat.lib().cm_qs_ls_accept(
                cb._h, _ptr(self._x), _ptr(plate), self.k, _ptr(self._Et),
                self.armijo, self.min_move, _ptr(y), _ptr(self._yt),
                _ptr(self.state), _ptr(self._ninv_t), _ptr(self._ninv),
                _stream(None)))
            self.stats["trials"] += 1

    def plate_force_gradient(self, y, plate, weight=None, tol=1e-5):
        """dF_top/d(mu, kappa, w) per material slot at the equilibrium y of
        the plate position `plate` (implicit differentiation: one CG solve
        Hess(Pi) lam = weight dF_top/dy on the device, then thetabar =
        lam^T df/dtheta from cm_forces_backward).  Call it right after
        equilibrate() at that position (the preconditioner blocks of its
        last residual are used).  weight: float64 device tensor (n_cells,)
        or None (1).  Returns a float64 device tensor (n_mat, 3)."""
        self._set_contact(y)
        import torch
        cb = self.cb
        lib, st = nat.lib(), _stream(None)
        nat.check(lib.cm_qs_adjoint_rhs(
            cb._h, _ptr(y), _ptr(plate), self.k, _ptr(weight), _ptr(self._r),
            _ptr(self._p), _ptr(self._x), _ptr(self.state), _ptr(self._minv),
            st))
        self._cg_loop(y, plate, tol, 4 * self.max_cg, "adjoint_cg")
        tb = torch.empty(3 * cb.n_mat, dtype=torch.float64, device=cb.device)
        cb.backward(y, self._x, None, self._ybar, tb)
        return tb.view(-1, 3)

    def curve(self, y0, tops, bottom, jacobian=False, adjoint_tol=1e-5):
        """Top-plate force of every cell at each plate height (tops: (S,) or
        (S, n_cells); bottom: scalar or (n_cells,)), starting from y0 and
        each position from the previous equilibrium (affine predictor).
        Returns (forces (S, n_cells) top, (S, n_cells) bottom, converged (S,),
        final positions); self.residuals (S, n_cells) holds the final
        projected Newton residual norms |f + p|_2 and self.cell_converged
        (S, n_cells) which cells met the tolerance.  With jacobian=True,
        self.jacobian (S, n_mat, 3) holds dF_top/d(mu, kappa, w) at every
        plate position (plate_force_gradient after each equilibrium)."""
        import torch
        cb = self.cb
        tops = np.asarray(tops, dtype=np.float64)
        if tops.ndim == 1:
            tops = np.repeat(tops[:, None], cb.n_cells, axis=1)
        bot = np.broadcast_to(np.asarray(bottom, np.float64), (cb.n_cells,))
        y = y0.clone()
        plates = torch.from_numpy(np.stack([tops, np.broadcast_to(
            bot, tops.shape)], axis=2).copy()).to(cb.device)
        Ft, Fb, ok, res, jac, cok = [], [], [], [], [], []
        for s in range(len(tops)):
            if s > 0:
                nat.check(nat.lib().cm_qs_predict(
                    cb._h, _ptr(plates[s - 1]), _ptr(plates[s]), _ptr(y),
                    _stream(None)))
            ok.append(self.equilibrate(y, plates[s]))
            cok.append((self.state[:, 11] == 0).cpu().numpy())
            if jacobian:
                jac.append(self.plate_force_gradient(
                    y, plates[s], tol=adjoint_tol).cpu().numpy())
            Ft.append(self.force[:, 0].cpu().numpy().copy())
            Fb.append(self.force[:, 1].cpu().numpy().copy())
            res.append(self.state[:, 3].sqrt().cpu().numpy())
        self.residuals = np.array(res)
        self.cell_converged = np.array(cok)
        self.jacobian = np.array(jac) if jacobian else None
        return np.array(Ft), np.array(Fb), np.array(ok), y
