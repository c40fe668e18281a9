"""FP64 CPU reference for the Mooney-Rivlin tetrahedral force (test
infrastructure only).

The oracle is the plain C++ routine in ``cm_oracle.cpp`` compiled with g++ and
called through ctypes.  It shares no code with the device library.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the device path never does.

Routes (see the header of ``cm_oracle.cpp``):
  * ``forces``       O1, the paper's derivative table (eq. elastic-force-vertex-1)
  * ``forces_ad``    O2, dual-number AD of the energy definition
  * ``jvp``          directional derivative of O1 (Hessian-vector product and
                     parameter sensitivities)
  * ``backward``     reverse-mode cotangents of L(f, E)
  * ``jvp_nested``   second-order duals through O2 (cross-check of ``jvp``)
  * ``relax_forward`` / ``relax_grad``  plate compression with explicit
                     overdamped steps (a reading of the paper's unavailable
                     supporting information; parity unpinned by the paper)
                     and its parameter gradient by forward-mode duals
  * ``RegionMesh``   a cell whose tetrahedra belong to material regions with
                     their own parameters: the forces and the energy are sums
                     over tetrahedra (eq. elastic-force-vertex-0), so they are
                     the sums of the single-material results of each region's
                     tetrahedra
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cm_oracle.cpp")
_SO = os.path.join(_HERE, "libcm_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_d = ctypes.c_double

_libs = {}


def build(force: bool = True, src: str = _SRC, out: str = _SO) -> str:
    """Compile the oracle with g++ (no -ffast-math, IEEE FP64 semantics)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                        "-fno-fast-math", "-o", tmp, src], check=True)
        os.replace(tmp, out)
    return out


def build_timing(out: str, src: str = _SRC) -> str:
    """The same source built for the CPU-baseline timing mode: -O3 for the
    host it runs on, OpenMP over cells (still no -ffast-math)."""
    tmp = out + ".tmp"
    subprocess.run(["g++", "-O3", "-march=native", "-fopenmp", "-std=c++17",
                    "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, src],
                   check=True)
    os.replace(tmp, out)
    return out


def lib(path: str = None):
    """The ctypes handle of the oracle library (built on first use)."""
    path = path or _SO
    if path not in _libs:
        if path == _SO and not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(path)
        L.or_prepare.argtypes = [_i64, _i64, _dp, _ip, _dp, _dp, _dp]
        L.or_prepare.restype = ctypes.c_int
        common = [_i64, _i64, _dp, _ip, _dp, _dp, _dp]
        L.or_forces_table.argtypes = common + [_d, _d, _d, _dp, _dp, _lp]
        L.or_forces_table.restype = None
        L.or_forces_ad.argtypes = common + [_d, _d, _d, _dp, _dp]
        L.or_forces_ad.restype = None
        L.or_forces_jvp.argtypes = common + [_dp, _d, _d, _d, _dp, _dp, _dp]
        L.or_forces_jvp.restype = None
        L.or_backward.argtypes = common + [_d, _d, _d, _dp, _d, _dp, _dp]
        L.or_backward.restype = None
        L.or_forces_jvp_nested.argtypes = common + [_dp, _d, _d, _d, _dp]
        L.or_forces_jvp_nested.restype = None
        L.or_relax_forward.argtypes = common + [_d, _d, _d, ctypes.c_int,
                                                _dp, _d, _d, _d, _dp, _dp]
        L.or_relax_forward.restype = None
        L.or_relax_grad.argtypes = common + [_d, _d, _d, ctypes.c_int,
                                             _dp, _d, _d, _d, _dp, _d, _dp,
                                             _dp, _dp]
        L.or_relax_grad.restype = None
        L.or_energy_density.argtypes = [_dp, _d, _d, _d]
        L.or_energy_density.restype = ctypes.c_double
        L.or_stress_table.argtypes = [_dp, _d, _d, _d, _dp]
        L.or_stress_table.restype = None
        L.or_batch_fwd_bwd.argtypes = [_i64, _i64, _lp, _lp, _dp, _ip, _dp,
                                       _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                       _dp, _dp]
        L.or_batch_fwd_bwd.restype = None
        L.or_threads.argtypes = [ctypes.c_int]
        L.or_threads.restype = ctypes.c_int
        _libs[path] = L
    return _libs[path]


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class OracleMesh:
    """A reference mesh with its FP64 inverse edge matrices and volumes."""

    def __init__(self, x, tets, lib_path: str = None):
        self.L = lib(lib_path)
        self.x = _f64(x, (-1, 3))
        self.tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        self.n_nodes = self.x.shape[0]
        self.n_tets = self.tets.shape[0]
        self.B = np.empty((self.n_tets, 3, 3))
        self.V0 = np.empty(self.n_tets)
        self.detJ = np.empty(self.n_tets)
        rc = self.L.or_prepare(self.n_nodes, self.n_tets, _ptr(self.x),
                              _ptr(self.tets, _ip), _ptr(self.B),
                              _ptr(self.V0), _ptr(self.detJ))
        if rc == -1:
            raise ValueError("tetrahedron index out of range")
        if rc == -2:
            raise ValueError("degenerate tetrahedron (det J == 0)")

    def _args(self):
        return (self.n_nodes, self.n_tets, _ptr(self.x), _ptr(self.tets, _ip),
                _ptr(self.B), _ptr(self.V0))

    def _y(self, y):
        y = _f64(y, (-1, 3))
        assert y.shape[0] == self.n_nodes
        return y

    def forces(self, y, theta):
        """O1: (forces (N, 3), total energy, number of tets with J <= 0)."""
        y = self._y(y)
        f = np.empty_like(y)
        E = ctypes.c_double()
        ninv = ctypes.c_int64()
        mu, kappa, w = theta
        self.L.or_forces_table(*self._args(), _ptr(y), mu, kappa, w, _ptr(f),
                              ctypes.byref(E), ctypes.byref(ninv))
        return f, E.value, ninv.value

    def forces_ad(self, y, theta):
        """O2: (forces, total energy) by dual-number AD of the energy."""
        y = self._y(y)
        f = np.empty_like(y)
        E = ctypes.c_double()
        mu, kappa, w = theta
        self.L.or_forces_ad(*self._args(), _ptr(y), mu, kappa, w, _ptr(f),
                           ctypes.byref(E))
        return f, E.value

    def jvp(self, y, theta, v=None, dtheta=None):
        """d/de (f, E)(y + e v, theta + e dtheta) at e = 0."""
        y = self._y(y)
        df = np.empty_like(y)
        dE = ctypes.c_double()
        vv = _f64(v, (-1, 3)) if v is not None else None
        vp = _ptr(vv) if vv is not None else None
        dt = _f64(dtheta) if dtheta is not None else None
        mu, kappa, w = theta
        self.L.or_forces_jvp(*self._args(), _ptr(y), vp, mu, kappa, w,
                            _ptr(dt) if dt is not None else None, _ptr(df),
                            ctypes.byref(dE))
        return df, dE.value

    def backward(self, y, theta, fbar=None, ebar=0.0):
        """(ybar (N, 3), thetabar (3,) = dL/d(mu, kappa, w))."""
        y = self._y(y)
        ybar = np.empty_like(y)
        tb = np.empty(3)
        fb = _f64(fbar, (-1, 3)) if fbar is not None else None
        mu, kappa, w = theta
        self.L.or_backward(*self._args(), _ptr(y), mu, kappa, w,
                          _ptr(fb) if fb is not None else None, float(ebar),
                          _ptr(ybar), _ptr(tb))
        return ybar, tb

    def jvp_nested(self, y, theta, v):
        """d/de f(y + e v) by second-order duals through O2."""
        y = self._y(y)
        vv = _f64(v, (-1, 3))
        df = np.empty_like(y)
        mu, kappa, w = theta
        self.L.or_forces_jvp_nested(*self._args(), _ptr(y), _ptr(vv), mu,
                                   kappa, w, _ptr(df))
        return df


    def relax_forward(self, y0, theta, top, bottom, k_plate, mobility):
        """Plate compression (reading of the missing supporting information):
        per-step top-plate forces (N,) and final positions (N_nodes, 3)."""
        y0 = self._y(y0)
        top = _f64(top)
        F = np.empty(len(top))
        yf = np.empty_like(y0)
        mu, kappa, w = theta
        self.L.or_relax_forward(*self._args(), _ptr(y0), mu, kappa, w,
                                len(top), _ptr(top), float(bottom),
                                float(k_plate), float(mobility), _ptr(F),
                                _ptr(yf))
        return F, yf

    def relax_grad(self, y0, theta, top, bottom, k_plate, mobility, F_target,
                   scale):
        """(loss, dL/d(mu, kappa, w), F) by forward-mode duals through all
        steps, L = scale * sum_n (F_n - F_target[n])^2."""
        y0 = self._y(y0)
        top = _f64(top)
        Ft = _f64(F_target)
        F = np.empty(len(top))
        g = np.empty(3)
        loss = ctypes.c_double()
        mu, kappa, w = theta
        self.L.or_relax_grad(*self._args(), _ptr(y0), mu, kappa, w, len(top),
                             _ptr(top), float(bottom), float(k_plate),
                             float(mobility), _ptr(Ft), float(scale),
                             ctypes.byref(loss), _ptr(g), _ptr(F))
        return loss.value, g, F


class OracleBatch:
    """Cells of a batch (concatenated arrays as in the device library) with
    their FP64 inverse edge matrices and volumes, for the timing mode:
    forward and backward of a range of cells, OpenMP over cells."""

    def __init__(self, node_off, tet_off, x, tets, lib_path: str = None):
        self.L = lib(lib_path)
        self.node_off = np.ascontiguousarray(node_off, dtype=np.int64)
        self.tet_off = np.ascontiguousarray(tet_off, dtype=np.int64)
        self.x = _f64(x, (-1, 3))
        self.tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        self.n_cells = len(self.node_off) - 1
        m = len(self.tets)
        self.B = np.empty((m, 3, 3))
        self.V0 = np.empty(m)
        for c in range(self.n_cells):
            n0, n1 = self.node_off[c], self.node_off[c + 1]
            t0, t1 = self.tet_off[c], self.tet_off[c + 1]
            rc = self.L.or_prepare(n1 - n0, t1 - t0, _ptr(self.x[n0:n1]),
                                   _ptr(self.tets[t0:t1], _ip),
                                   _ptr(self.B[t0:t1]), _ptr(self.V0[t0:t1]),
                                   None)
            if rc != 0:
                raise ValueError(f"cell {c}: bad mesh ({rc})")

    def threads(self, n: int = 0) -> int:
        return int(self.L.or_threads(int(n)))

    def fwd_bwd(self, y, theta, fbar, ebar, c0=0, c1=None):
        """Forces, energies, ybar and thetabar of cells [c0, c1)."""
        c1 = self.n_cells if c1 is None else c1
        y, fbar = _f64(y, (-1, 3)), _f64(fbar, (-1, 3))
        theta, ebar = _f64(theta, (-1, 3)), _f64(ebar)
        f, ybar = np.zeros_like(y), np.zeros_like(y)
        E, tb = np.zeros(self.n_cells), np.zeros((self.n_cells, 3))
        self.L.or_batch_fwd_bwd(int(c0), int(c1), _ptr(self.node_off, _lp),
                                _ptr(self.tet_off, _lp), _ptr(self.x),
                                _ptr(self.tets, _ip), _ptr(self.B),
                                _ptr(self.V0), _ptr(y), _ptr(theta),
                                _ptr(fbar), _ptr(ebar), _ptr(f), _ptr(E),
                                _ptr(ybar), _ptr(tb))
        return f, E, ybar, tb


def energy_density(F, theta, lib_path: str = None) -> float:
    """U(F) from the definitions (eqs. invariantJ/I/K, strain energy)."""
    F = _f64(F, (9,))
    mu, kappa, w = theta
    return lib(lib_path).or_energy_density(_ptr(F), mu, kappa, w)


def stress_table(F, theta, lib_path: str = None) -> np.ndarray:
    """dU/dF (3, 3) from the derivative table."""
    F = _f64(F, (9,))
    P = np.empty(9)
    mu, kappa, w = theta
    lib(lib_path).or_stress_table(_ptr(F), mu, kappa, w, _ptr(P))
    return P.reshape(3, 3)


class RegionMesh:
    """One cell with per-tetrahedron material regions.  The paper's force
    evaluation is local to each tetrahedron, so parts of a cell can carry
    their own parameters (Sec. "Theory", after eq. elastic-force-vertex-1).
    Region r uses thetas[r] = (mu, kappa, w); results are the sums over the
    regions of OracleMesh results on that region's tetrahedra."""

    def __init__(self, x, tets, regions, n_regions, lib_path: str = None):
        regions = np.asarray(regions)
        self.n_regions = int(n_regions)
        self.parts = [OracleMesh(x, np.asarray(tets)[regions == r], lib_path)
                      if (regions == r).any() else None
                      for r in range(self.n_regions)]

    def forces(self, y, thetas):
        f, E, ninv = 0.0, 0.0, 0
        for part, th in zip(self.parts, thetas):
            if part is not None:
                fr, Er, nr = part.forces(y, tuple(th))
                f, E, ninv = f + fr, E + Er, ninv + nr
        return f, E, ninv

    def backward(self, y, thetas, fbar=None, ebar=0.0):
        """ybar summed over regions and thetabar (n_regions, 3); a region
        without tetrahedra has a zero gradient."""
        ybar, tb = 0.0, np.zeros((self.n_regions, 3))
        for r, (part, th) in enumerate(zip(self.parts, thetas)):
            if part is not None:
                yr, tr = part.backward(y, tuple(th), fbar, ebar)
                ybar, tb[r] = ybar + yr, tr
        return ybar, tb
