"""Plate compression of a batch of cells with checkpointed reverse-mode
gradients (backpropagation through time).

The paper compresses cells between a resting and a moving plate with a
repulsive force that keeps vertices out of the plates (Sec. "Simulation
setup"); its force law and time integration are in the unavailable
supporting information.  The reading used here (see cm_plate_step in
include/cellmech.h): overdamped explicit steps

    y_{n+1} = y_n + m (f(y_n; theta) + p(y_n; h_n)),   n = 0 .. N-1,

with a quadratic plate penalty p and the measured force on the top plate
F_n = k sum max(0, y_z - h_n)^2.  The calibration loss is
L = scale * sum_n sum_c (F_n,c - F*_n,c)^2.

Reverse mode: lam_N = 0 and, for n = N-1 .. 0,
    lam_n = lam_{n+1} + m ((df/dy)^T + dp/dy) lam_{n+1} + dL/dy_n,
    dL/dtheta += m (df/dtheta)^T lam_{n+1},
where (df/dy)^T lam and (df/dtheta)^T lam come from cm_forces_backward.  By
default every step is one fused call (cm_plate_forces_step,
cm_plate_backward_step: the force or adjoint pass applies the step in its
epilogue); fused=False runs the two-call route (cm_forces + cm_plate_step,
cm_forces_backward + cm_plate_step_adjoint).  Only
every `checkpoint`-th state is kept during the forward sweep, plus the states
of the last segment; every other segment is recomputed from its checkpoint
during the reverse sweep (the recomputation is bitwise identical, so the
gradient equals the one with every state stored; the plate forces of the
loss come from the forward sweep).
Every arithmetic step runs in libcellmech's kernels; this module only
orders the calls and owns the buffers.
"""
from __future__ import annotations

import numpy as np


class PlateCompression:
    """N-step plate compression of every cell of a CellBatch.

    top: top-plate heights, shape (N,) (same for every cell) or (N, n_cells);
    bottom: bottom-plate height (scalar or (n_cells,)); k_plate: penalty;
    mobility: time step over drag; checkpoint: states kept every that many
    steps during the forward sweep of gradient(); fused: one library call
    per step (else forces and plate step as two calls)."""

    def __init__(self, batch, top, bottom, k_plate, mobility, checkpoint=20,
                 fused=True):
        import torch
        self.cb = batch
        top = np.asarray(top, dtype=np.float64)
        if top.ndim == 1:
            top = np.repeat(top[:, None], batch.n_cells, axis=1)
        self.n_steps = top.shape[0]
        bottom = np.broadcast_to(np.asarray(bottom, dtype=np.float64),
                                 (batch.n_cells,))
        plates = np.empty((self.n_steps, batch.n_cells, 2))
        plates[:, :, 0] = top
        plates[:, :, 1] = bottom[None, :]
        dev = batch.device
        self.plates = torch.from_numpy(plates.reshape(self.n_steps, -1)).to(dev)
        self.k = float(k_plate)
        self.m = float(mobility)
        self.checkpoint = int(checkpoint)
        self.fused = bool(fused)
        if self.checkpoint < 1:
            raise ValueError("checkpoint must be >= 1")
        nn = 3 * batch.n_nodes
        self._f = torch.empty(nn, dtype=torch.float32, device=dev)
        self._ybar = torch.empty(nn, dtype=torch.float32, device=dev)
        self._tb = torch.empty(3 * batch.n_mat, dtype=torch.float64,
                               device=dev)
        self._E = torch.empty(batch.n_cells, dtype=torch.float64, device=dev)

    def set_theta(self, theta):
        """theta: (n_mat, 3) host array or float64 device tensor, one row
        per material slot (one per cell without regions)."""
        import torch
        if isinstance(theta, torch.Tensor):
            t = theta.to(self.cb.device, torch.float64)
            self.cb.set_params(t[:, 0], t[:, 1], t[:, 2])
        else:
            t = np.asarray(theta, dtype=np.float64).reshape(-1, 3)
            self.cb.set_params(t[:, 0], t[:, 1], t[:, 2])

    def _step(self, n, y, y_next, force):
        cb = self.cb
        if self.fused:
            cb.plate_forces_step(y, self.plates[n], self.k, self.m, y_next,
                                 force)
        else:
            cb.forces(y, self._f, self._E)
            cb.plate_step(y, self._f, self.plates[n], self.k, self.m, y_next,
                          force)

    def _adjoint(self, n, y_n, lam, lam_new, F, F_target, scale, tacc):
        cb = self.cb
        if self.fused:
            cb.plate_backward_step(y_n, lam, self.plates[n], self.k, self.m,
                                   lam_new, F[n], F_target[n], scale, tacc)
        else:
            cb.backward(y_n, lam, None, self._ybar, self._tb)
            cb.plate_step_adjoint(y_n, lam, self._ybar, self.plates[n],
                                  self.k, self.m, lam_new, F[n], F_target[n],
                                  scale, self._tb, tacc)

    def forward(self, y0, keep_every=None, tail=None):
        """Runs all steps from y0 (device SoA).  Returns (F (N, n_cells)
        float64 device tensor, final positions, kept states dict n -> y_n).
        tail = (n0, buffers): the states y_n, n >= n0, are also copied into
        buffers[n - n0]."""
        import torch
        N = self.n_steps
        F = torch.empty(N, self.cb.n_cells, dtype=torch.float64,
                        device=self.cb.device)
        y = y0.clone()
        nxt = torch.empty_like(y)
        kept = {}
        for n in range(N):
            if keep_every and n % keep_every == 0:
                kept[n] = y.clone()
            if tail is not None and n >= tail[0]:
                tail[1][n - tail[0]].copy_(y)
            self._step(n, y, nxt, F[n])
            y, nxt = nxt, y
        return F, y, kept

    def gradient(self, y0, F_target, scale):
        """Loss and dL/dtheta (n_mat, 3) by checkpointed reverse mode.
        F_target: (N, n_cells) float64 device tensor."""
        import torch
        N, C = self.n_steps, self.checkpoint
        cb = self.cb
        lam = torch.zeros(3 * cb.n_nodes, dtype=torch.float32, device=cb.device)
        seg_states = [torch.empty_like(lam) for _ in range(C)]
        # the forward sweep leaves the last segment's states in seg_states,
        # so only the earlier segments are recomputed
        last0 = ((N - 1) // C) * C
        F, _, kept = self.forward(y0, keep_every=C, tail=(last0, seg_states))
        loss = float(scale * ((F - F_target) ** 2).sum())
        lam_new = torch.empty_like(lam)
        tacc = torch.zeros(3 * cb.n_mat, dtype=torch.float64,
                           device=cb.device)
        for s0 in reversed(range(0, N, C)):
            s1 = min(N, s0 + C)
            if s0 != last0:
                # recompute the segment's states y_s0 .. y_{s1-1} from its
                # checkpoint (bitwise the states of the forward sweep; the
                # plate forces F_n come from the forward sweep)
                seg_states[0].copy_(kept[s0])
                for j in range(s1 - s0 - 1):
                    self._step(s0 + j, seg_states[j], seg_states[j + 1], None)
            for j in reversed(range(s1 - s0)):
                n = s0 + j
                self._adjoint(n, seg_states[j], lam, lam_new, F, F_target,
                              scale, tacc)
                lam, lam_new = lam_new, lam
        return loss, tacc.view(-1, 3), F
