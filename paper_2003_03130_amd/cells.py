"""Python handle over the C ABI: device memory and streams come from PyTorch,
every computation runs in libcellmech (HIP, gfx950)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as nat


def _ptr(a) -> ctypes.c_void_p:
    """Raw pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _options(order, tile_tets, degenerate_tol):
    o = nat.Options()
    nat.lib().cm_options_default(ctypes.byref(o))
    if order is not None:
        o.order = int(order)
    if tile_tets is not None:
        o.tile_tets = int(tile_tets)
    if degenerate_tol is not None:
        o.degenerate_tol = float(degenerate_tol)
    return o


def _regions(regions, n_regions, n_tets):
    """uint8 region id per tetrahedron and the region count (default:
    largest id + 1)."""
    reg = np.asarray(regions)
    if reg.shape != (n_tets,) or (reg.size and (reg.min() < 0 or reg.max() > 255)):
        raise ValueError("regions must be one id in [0, 255] per tetrahedron")
    reg = np.ascontiguousarray(reg, dtype=np.uint8)
    nr = int(n_regions) if n_regions is not None else int(reg.max()) + 1
    return reg, nr


def _host_inputs(node_off, tet_off, x, tets):
    node_off = np.ascontiguousarray(node_off, dtype=np.int64)
    tet_off = np.ascontiguousarray(tet_off, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
    return node_off, tet_off, x, tets


class CellBatch:
    """Reference meshes of one or more cells resident on the current GPU.

    ``node_off``/``tet_off`` are CSR offsets, ``x`` the (N, 3) float64
    reference positions and ``tets`` the (M, 4) cell-local vertex indices.
    Device node arrays are float32 structure-of-arrays (3 * N) in the internal
    node order; ``to_device``/``to_host`` convert from/to (N, 3) input order.
    """

    def __init__(self, node_off, tet_off, x, tets, order=None, tile_tets=None,
                 degenerate_tol=None, stream=None, regions=None,
                 n_regions=None):
        node_off, tet_off, x, tets = _host_inputs(node_off, tet_off, x, tets)
        self.n_cells = len(node_off) - 1
        opt = _options(order, tile_tets, degenerate_tol)
        h = ctypes.c_void_p()
        if regions is None:
            nat.check(nat.lib().cm_batch_create(
                self.n_cells, _ptr(node_off), _ptr(tet_off), _ptr(x),
                _ptr(tets), ctypes.byref(opt), _stream(stream),
                ctypes.byref(h)))
        else:
            reg, nr = _regions(regions, n_regions, len(tets))
            nat.check(nat.lib().cm_batch_create_regions(
                self.n_cells, _ptr(node_off), _ptr(tet_off), _ptr(x),
                _ptr(tets), _ptr(reg), nr, ctypes.byref(opt), _stream(stream),
                ctypes.byref(h)))
        self._finish(h, node_off, tet_off)
        self.is_template = False

    def _finish(self, h, node_off, tet_off):
        import torch
        self._h = h
        info = nat.Info()
        nat.check(nat.lib().cm_get_info(self._h, ctypes.byref(info)))
        self.info = info.as_dict()
        self.n_regions = int(info.n_regions)
        self.n_mat = self.n_cells * self.n_regions
        self.n_nodes = int(info.n_nodes)
        self.n_tets = int(info.n_tets)
        self.node_off = node_off
        self.tet_off = tet_off
        self.new_to_old = np.empty(self.n_nodes, dtype=np.int64)
        nat.check(nat.lib().cm_permutation(self._h, _ptr(self.new_to_old)))
        self.old_to_new = np.empty_like(self.new_to_old)
        self.old_to_new[self.new_to_old] = np.arange(self.n_nodes)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def tuned(cls, node_off, tet_off, x, tets, tile_candidates=None,
              cache_path=None, order=None, degenerate_tol=None, stream=None):
        """cm_batch_create_tuned: the tile size (and launch) chosen by timing
        every candidate; ``self.candidate_ms`` holds each candidate's time."""
        node_off, tet_off, x, tets = _host_inputs(node_off, tet_off, x, tets)
        opt = _options(order, None, degenerate_tol)
        cand = (None if tile_candidates is None else
                np.ascontiguousarray(tile_candidates, dtype=np.int32))
        n_cand = 5 if cand is None else len(cand)
        ms = np.full(n_cand, np.inf)
        h = ctypes.c_void_p()
        nat.check(nat.lib().cm_batch_create_tuned(
            len(node_off) - 1, _ptr(node_off), _ptr(tet_off), _ptr(x),
            _ptr(tets), ctypes.byref(opt), _ptr(cand), n_cand,
            cache_path.encode() if cache_path else None, _ptr(ms),
            _stream(stream), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.n_cells = len(node_off) - 1
        self._finish(h, node_off, tet_off)
        self.is_template = False
        self.candidate_ms = ms
        return self

    @classmethod
    def from_cells(cls, cells, **kw):
        node_off = np.concatenate([[0], np.cumsum([len(c.x) for c in cells])])
        tet_off = np.concatenate([[0], np.cumsum([len(c.tets) for c in cells])])
        return cls(node_off, tet_off, np.concatenate([c.x for c in cells]),
                   np.concatenate([c.tets for c in cells]), **kw)

    @classmethod
    def single(cls, x, tets, **kw):
        return cls([0, len(x)], [0, len(tets)], x, tets, **kw)

    @classmethod
    def template(cls, n_cells, x, tets, order=None, tile_tets=None,
                 degenerate_tol=None, stream=None, regions=None,
                 n_regions=None):
        """``n_cells`` copies of one reference mesh (cm_template_create).

        The tet data is stored once and shared; node arrays and parameters
        are per cell, cell c owning input rows [c n, (c + 1) n) of the
        (n_cells n, 3) arrays that ``to_device``/``to_host`` take.  Per-cell
        launches are not available on such a batch.
        """
        _, _, x, tets = _host_inputs([0], [0], x, tets)
        n, m = len(x), len(tets)
        opt = _options(order, tile_tets, degenerate_tol)
        h = ctypes.c_void_p()
        if regions is None:
            nat.check(nat.lib().cm_template_create(
                int(n_cells), n, m, _ptr(x), _ptr(tets), ctypes.byref(opt),
                _stream(stream), ctypes.byref(h)))
        else:
            reg, nr = _regions(regions, n_regions, m)
            nat.check(nat.lib().cm_template_create_regions(
                int(n_cells), n, m, _ptr(x), _ptr(tets), _ptr(reg), nr,
                ctypes.byref(opt), _stream(stream), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.n_cells = int(n_cells)
        self._finish(h, np.arange(n_cells + 1, dtype=np.int64) * n,
                     np.arange(n_cells + 1, dtype=np.int64) * m)
        self.is_template = True
        return self

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_h", None):
            nat.lib().cm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ layout
    def to_device(self, a_input_order):
        """(N, 3) array in input order -> float32 SoA (3N,) device tensor."""
        import torch
        a = np.asarray(a_input_order, dtype=np.float32).reshape(-1, 3)
        soa = np.ascontiguousarray(a[self.new_to_old].T).reshape(-1)
        return torch.from_numpy(soa).to(self.device)

    def to_host(self, t):
        """float32 SoA (3N,) device tensor -> (N, 3) numpy in input order."""
        soa = t.detach().float().cpu().numpy().reshape(3, -1)
        out = np.empty((self.n_nodes, 3), dtype=np.float32)
        out[self.new_to_old] = soa.T
        return out

    def empty_nodes(self):
        import torch
        return torch.empty(3 * self.n_nodes, dtype=torch.float32,
                           device=self.device)

    # ------------------------------------------------------------ params
    def set_params(self, mu, kappa, w, stream=None):
        """Host sequences (validated) or float64 device tensors with one
        value per material slot (cell c, region r at c * n_regions + r; an
        (n_cells, n_regions) array is taken in that order); host scalars
        broadcast."""
        import torch
        if isinstance(mu, torch.Tensor):
            tens = [t.to(self.device, torch.float64).contiguous().reshape(-1)
                    for t in (mu, kappa, w)]
            if any(t.numel() != self.n_mat for t in tens):
                raise ValueError(f"need {self.n_mat} values per parameter")
            self._param_keep = tens
            nat.check(nat.lib().cm_set_params(
                self._h, _ptr(tens[0]), _ptr(tens[1]), _ptr(tens[2]), 1,
                _stream(stream)))
        else:
            arr = []
            for v in (mu, kappa, w):
                v = np.asarray(v, dtype=np.float64)
                v = v.reshape(-1) if v.size == self.n_mat else v
                arr.append(np.ascontiguousarray(
                    np.broadcast_to(v, (self.n_mat,))))
            nat.check(nat.lib().cm_set_params(
                self._h, _ptr(arr[0]), _ptr(arr[1]), _ptr(arr[2]), 0,
                _stream(stream)))

    # ------------------------------------------------------------ compute
    def forces(self, y, f=None, energy=None, n_inverted=None, stream=None,
               percell=False):
        import torch
        if f is None:
            f = self.empty_nodes()
        if energy is None:
            energy = torch.empty(self.n_cells, dtype=torch.float64,
                                 device=self.device)
        fn = nat.lib().cm_forces_percell if percell else nat.lib().cm_forces
        nat.check(fn(self._h, _ptr(y), _ptr(f), _ptr(energy), _ptr(n_inverted),
                     _stream(stream)))
        return f, energy

    def forces_checked(self, y, f=None, energy=None, n_inverted=None,
                       stream=None):
        """cm_forces_checked: (f, energy, n_nonfinite) with n_nonfinite an
        int32 device tensor (n_cells,) counting each cell's tetrahedra with
        a non-finite energy or force."""
        import torch
        if f is None:
            f = self.empty_nodes()
        if energy is None:
            energy = torch.empty(self.n_cells, dtype=torch.float64,
                                 device=self.device)
        nonfin = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        nat.check(nat.lib().cm_forces_checked(
            self._h, _ptr(y), _ptr(f), _ptr(energy), _ptr(n_inverted),
            _ptr(nonfin), _stream(stream)))
        return f, energy, nonfin

    def backward(self, y, fbar=None, ebar=None, ybar=None, thetabar=None,
                 stream=None, percell=False, cells=None):
        """cells: optional float64 device tensor of shape (n_cells,) (a
        strided view such as a column of a state array is fine): only cells
        with a nonzero entry are evaluated, the others' ybar and thetabar
        entries are left unchanged (cm_forces_backward_cells)."""
        import torch
        if ybar is None:
            ybar = self.empty_nodes()
        if thetabar is None:
            thetabar = torch.empty(3 * self.n_mat, dtype=torch.float64,
                                   device=self.device)
        if cells is not None:
            if percell:
                raise ValueError("cells and percell cannot be combined")
            if (cells.dtype != torch.float64 or cells.dim() != 1
                    or cells.shape[0] != self.n_cells or not cells.is_cuda):
                raise ValueError("cells must be a float64 device tensor of "
                                 "shape (n_cells,)")
            nat.check(nat.lib().cm_forces_backward_cells(
                self._h, _ptr(y), _ptr(fbar), _ptr(ebar), _ptr(cells),
                cells.stride(0), _ptr(ybar), _ptr(thetabar), _stream(stream)))
            return ybar, thetabar
        fn = (nat.lib().cm_forces_backward_percell if percell
              else nat.lib().cm_forces_backward)
        nat.check(fn(self._h, _ptr(y), _ptr(fbar), _ptr(ebar), _ptr(ybar),
                     _ptr(thetabar), _stream(stream)))
        return ybar, thetabar

    def forces_and_backward(self, y, fbar=None, ebar=None, f=None, energy=None,
                            n_inverted=None, ybar=None, thetabar=None,
                            stream=None):
        """cm_forces_and_backward: forward and backward in one pass, for
        cotangents (fbar, ebar) given up front; returns (f, energy, ybar,
        thetabar), bitwise those of forces() followed by backward()."""
        import torch
        if f is None:
            f = self.empty_nodes()
        if energy is None:
            energy = torch.empty(self.n_cells, dtype=torch.float64,
                                 device=self.device)
        if ybar is None:
            ybar = self.empty_nodes()
        if thetabar is None:
            thetabar = torch.empty(3 * self.n_mat, dtype=torch.float64,
                                   device=self.device)
        nat.check(nat.lib().cm_forces_and_backward(
            self._h, _ptr(y), _ptr(f), _ptr(energy), _ptr(n_inverted),
            _ptr(fbar), _ptr(ebar), _ptr(ybar), _ptr(thetabar), _stream(stream)))
        return f, energy, ybar, thetabar

    # ------------------------------------------------------------ launch
    def set_launch(self, waves_per_block, blocks_per_cu):
        nat.check(nat.lib().cm_set_launch(self._h, waves_per_block,
                                          blocks_per_cu))

    def get_launch(self):
        w, b = ctypes.c_int32(), ctypes.c_int32()
        nat.check(nat.lib().cm_get_launch(self._h, ctypes.byref(w),
                                          ctypes.byref(b)))
        return w.value, b.value

    def autotune(self, y, cache_path=None, stream=None):
        nat.check(nat.lib().cm_autotune(
            self._h, _ptr(y), cache_path.encode() if cache_path else None,
            _stream(stream)))
        return self.get_launch()

    def plate_step(self, y, f, plate, k_plate, mobility, y_next, force=None,
                   stream=None):
        """y_next = y + m (f + plate penalty); force = per-cell top force."""
        nat.check(nat.lib().cm_plate_step(
            self._h, _ptr(y), _ptr(f), _ptr(plate), float(k_plate),
            float(mobility), _ptr(y_next), _ptr(force), _stream(stream)))

    def plate_step_adjoint(self, y, lam_next, ybar_el, plate, k_plate,
                           mobility, lam, F_meas=None, F_target=None,
                           scale=0.0, thetabar_el=None, thetabar_acc=None,
                           stream=None):
        nat.check(nat.lib().cm_plate_step_adjoint(
            self._h, _ptr(y), _ptr(lam_next), _ptr(ybar_el), _ptr(plate),
            float(k_plate), float(mobility), _ptr(F_meas), _ptr(F_target),
            float(scale), _ptr(thetabar_el), _ptr(thetabar_acc), _ptr(lam),
            _stream(stream)))

    def plate_forces_step(self, y, plate, k_plate, mobility, y_next,
                          force=None, energy=None, n_inverted=None,
                          stream=None):
        """One plate step with the elastic forces computed inside it
        (cm_plate_forces_step): y_next, and optionally the per-cell top
        force, energy and inverted count at y."""
        nat.check(nat.lib().cm_plate_forces_step(
            self._h, _ptr(y), _ptr(plate), float(k_plate), float(mobility),
            _ptr(y_next), _ptr(force), _ptr(energy), _ptr(n_inverted),
            _stream(stream)))

    def plate_backward_step(self, y, lam_next, plate, k_plate, mobility, lam,
                            F_meas=None, F_target=None, scale=0.0,
                            thetabar_acc=None, stream=None):
        """The reverse plate step with the adjoint of the forces computed
        inside it (cm_plate_backward_step)."""
        nat.check(nat.lib().cm_plate_backward_step(
            self._h, _ptr(y), _ptr(lam_next), _ptr(plate), float(k_plate),
            float(mobility), _ptr(F_meas), _ptr(F_target), float(scale),
            _ptr(thetabar_acc), _ptr(lam), _stream(stream)))

    SHAPE_FIELDS = ("volume", "com_x", "com_y", "com_z", "a1", "a2", "a3",
                    "D", "d_max", "strain")

    def shape(self, y, d_ref=None, out=None, stream=None):
        """Taylor deformation and cell strain per cell (cm_shape): a float64
        (n_cells, 10) device tensor with the columns of SHAPE_FIELDS."""
        import torch
        if out is None:
            out = torch.empty(self.n_cells, 10, dtype=torch.float64,
                              device=self.device)
        if d_ref is not None and not isinstance(d_ref, torch.Tensor):
            d_ref = torch.as_tensor(np.broadcast_to(
                np.asarray(d_ref, dtype=np.float64), (self.n_cells,)).copy(),
                device=self.device)
            self._dref_keep = d_ref
        nat.check(nat.lib().cm_shape(self._h, _ptr(y), _ptr(d_ref), _ptr(out),
                                     _stream(stream)))
        return out

    def profile_kernels(self, y, f, energy, fbar, ebar, ybar, thetabar,
                        reps=10, stream=None):
        """Average ms per launch of the forward tile, forward finalize,
        backward tile and backward finalize kernels and of the fused forward
        + backward tile and finalize kernels (HIP events)."""
        ms = np.zeros(6, dtype=np.float64)
        nat.check(nat.lib().cm_profile_kernels(
            self._h, _ptr(y), _ptr(f), _ptr(energy), _ptr(fbar), _ptr(ebar),
            _ptr(ybar), _ptr(thetabar), int(reps), _ptr(ms), _stream(stream)))
        return ms

    def graph_capture(self, mode, y, f, energy=None, n_inverted=None,
                      fbar=None, ebar=None, ybar=None, thetabar=None,
                      stream=None):
        nat.check(nat.lib().cm_graph_capture(
            self._h, int(mode), _ptr(y), _ptr(f), _ptr(energy),
            _ptr(n_inverted), _ptr(fbar), _ptr(ebar), _ptr(ybar),
            _ptr(thetabar), _stream(stream)))

    def graph_launch(self, stream=None):
        nat.check(nat.lib().cm_graph_launch(self._h, _stream(stream)))


class HostLayout:
    """The prepared tables of cm_layout_* (host only, no GPU needed)."""

    def __init__(self, node_off, tet_off, x, tets, order=None, tile_tets=None,
                 degenerate_tol=None, regions=None, n_regions=None):
        node_off, tet_off, x, tets = _host_inputs(node_off, tet_off, x, tets)
        opt = _options(order, tile_tets, degenerate_tol)
        h = ctypes.c_void_p()
        reg, nr = (None, 1) if regions is None else _regions(
            regions, n_regions, len(tets))
        nat.check(nat.lib().cm_layout_create_regions(
            len(node_off) - 1, _ptr(node_off), _ptr(tet_off), _ptr(x),
            _ptr(tets), _ptr(reg), nr, ctypes.byref(opt), ctypes.byref(h)))
        self.n_regions = nr
        self._load(h)
        self.is_template = False

    @classmethod
    def template(cls, n_cells, x, tets, order=None, tile_tets=None,
                 degenerate_tol=None):
        """Layout of ``n_cells`` copies of one mesh (cm_layout_create_template);
        ``cell_tile_off`` stays zero, the tiles of cell c being c + k n_cells."""
        _, _, x, tets = _host_inputs([0], [0], x, tets)
        opt = _options(order, tile_tets, degenerate_tol)
        h = ctypes.c_void_p()
        nat.check(nat.lib().cm_layout_create_template(
            int(n_cells), len(x), len(tets), _ptr(x), _ptr(tets),
            ctypes.byref(opt), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.n_regions = 1
        self._load(h)
        self.is_template = True
        return self

    def _load(self, h):
        try:
            sz = np.zeros(8, dtype=np.int64)
            nat.check(nat.lib().cm_layout_sizes(h, sz.ctypes.data_as(nat._p64)))
            (self.n_tiles, self.n_chunks, self.n_slots, self.n_shared,
             self.n_nodes, self.n_cells, self.max_tile_nodes,
             self.tile_tets) = (int(v) for v in sz)
            self.tiles = np.zeros((self.n_tiles, 8), dtype=np.int32)
            raw = np.zeros(self.n_chunks * 3072, dtype=np.uint8)
            self.slot_node = np.zeros(self.n_slots, dtype=np.int32)
            self.shared_node = np.zeros(self.n_shared, dtype=np.int32)
            self.shared_slot_ptr = np.zeros(self.n_shared + 1, dtype=np.int32)
            self.shared_slots = np.zeros(self.n_slots, dtype=np.int32)
            self.cell_tile_off = np.zeros(self.n_cells + 1, dtype=np.int32)
            self.cell_shared_off = np.zeros(self.n_cells + 1, dtype=np.int32)
            self.new_to_old = np.zeros(self.n_nodes, dtype=np.int64)
            nat.check(nat.lib().cm_layout_export(
                h, _ptr(self.tiles), _ptr(raw), _ptr(self.slot_node),
                _ptr(self.shared_node), _ptr(self.shared_slot_ptr),
                _ptr(self.shared_slots), _ptr(self.cell_tile_off),
                _ptr(self.cell_shared_off), _ptr(self.new_to_old)))
            nmat = self.n_cells * self.n_regions
            self.tile_mat = np.zeros(self.n_tiles, dtype=np.int32)
            self.mat_tile_first = np.zeros(nmat, dtype=np.int32)
            self.mat_tile_count = np.zeros(nmat, dtype=np.int32)
            nat.check(nat.lib().cm_layout_export_regions(
                h, _ptr(self.tile_mat), _ptr(self.mat_tile_first),
                _ptr(self.mat_tile_count)))
        finally:
            nat.lib().cm_layout_destroy(h)
        # three rows of 64 16-byte records per chunk: (idx01, idx23, V0, B0),
        # (B1..B4), (B5..B8)
        ch = raw.reshape(self.n_chunks, 3072)
        a = ch[:, :1024].view(np.uint32).reshape(self.n_chunks, 64, 4)
        idx = a[..., :2]
        self.local_idx = np.stack([idx[..., 0] & 0xFFFF, idx[..., 0] >> 16,
                                   idx[..., 1] & 0xFFFF, idx[..., 1] >> 16],
                                  axis=-1).astype(np.int64)
        self.empty = idx[..., 0] == 0xFFFFFFFF
        af = a.view(np.float32)
        rest = ch[:, 1024:].view(np.float32).reshape(self.n_chunks, 2, 64, 4)
        self.B = np.concatenate([af[..., 3:4], rest[:, 0], rest[:, 1]], axis=-1).reshape(
            self.n_chunks, 64, 3, 3)
        self.V0 = np.ascontiguousarray(af[..., 2])
