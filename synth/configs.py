"""Seeded workloads with the shapes of the paper's compression setups.

Every case is a set of cells.  A cell is a reference mesh (float64 positions,
int32 tetrahedra), deformed positions rounded to float32 (the storage format of
the device path, so that the oracle and the device evaluate the same input),
and Mooney-Rivlin parameters (mu, kappa, w) with mu1 = w*mu and
mu2 = (1-w)*mu (Sec. "Theory").

Deformations are an affine map ``A`` applied to the reference mesh plus
Gaussian node noise.  The paper compresses cells by up to 80 % (Introduction,
Sec. "Results"); noise keeps every tetrahedron's deformation gradient distinct
so that parity is not tested on a homogeneous field only.

Noise rule (a reading of the workload description; the literal per-node noise
of 0.01 R inverts tetrahedra on fine meshes): the noise amplitude is
``sigma = 0.05 * mean edge length`` and, while any tetrahedron has a volume
ratio J below ``0.25 * det A``, the noise on all four vertices of every such
tetrahedron is halved.  J here is the ratio of deformed to reference signed
volume, an input-quality gate; no energy is evaluated.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mesh import (_edge_matrices, ellipsoid, mean_edge_length, sphere_mesh,
                   unique_edges)

NOISE_FRAC = 0.05
J_FLOOR = 0.25


@dataclass
class Cell:
    x: np.ndarray          # (N, 3) float64 reference positions
    tets: np.ndarray       # (M, 4) int32, cell-local vertex indices
    y: np.ndarray          # (N, 3) float32 deformed positions
    theta: tuple           # (mu, kappa, w)
    A: np.ndarray = field(default=None)  # the affine map used (3, 3)
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(self.x.shape[0])

    @property
    def n_tets(self):
        return int(self.tets.shape[0])


@dataclass
class Batch:
    """Cells concatenated: node_off/tet_off are CSR offsets (n_cells + 1)."""
    node_off: np.ndarray   # int64
    tet_off: np.ndarray    # int64
    x: np.ndarray          # (sum N, 3) float64
    tets: np.ndarray       # (sum M, 4) int32, cell-local indices
    y: np.ndarray          # (sum N, 3) float32
    theta: np.ndarray      # (n_cells, 3) float64: mu, kappa, w
    info: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return int(len(self.node_off) - 1)

    @property
    def n_nodes(self):
        return int(self.node_off[-1])

    @property
    def n_tets(self):
        return int(self.tet_off[-1])

    def cell(self, c: int) -> Cell:
        n0, n1 = self.node_off[c], self.node_off[c + 1]
        t0, t1 = self.tet_off[c], self.tet_off[c + 1]
        return Cell(self.x[n0:n1], self.tets[t0:t1], self.y[n0:n1],
                    tuple(float(v) for v in self.theta[c]))


def batch_from_cells(cells) -> Batch:
    node_off = np.zeros(len(cells) + 1, dtype=np.int64)
    tet_off = np.zeros(len(cells) + 1, dtype=np.int64)
    node_off[1:] = np.cumsum([c.n_nodes for c in cells])
    tet_off[1:] = np.cumsum([c.n_tets for c in cells])
    return Batch(node_off, tet_off,
                 np.concatenate([c.x for c in cells]),
                 np.concatenate([c.tets for c in cells]).astype(np.int32),
                 np.concatenate([c.y for c in cells]).astype(np.float32),
                 np.array([c.theta for c in cells], dtype=np.float64))


def _det_edges(p, tets):
    """det[p1 - p4, p2 - p4, p3 - p4] per tet (scalar triple product)."""
    p4 = p[tets[:, 3]]
    a = p[tets[:, 0]] - p4
    b = p[tets[:, 1]] - p4
    c = p[tets[:, 2]] - p4
    return np.einsum("ij,ij->i", a, np.cross(b, c))


def volume_ratios(x, y, tets, ref_det=None):
    """det(deformed edge matrix) / det(reference edge matrix) per tet."""
    if ref_det is None:
        ref_det = _det_edges(x, tets)
    return _det_edges(y, tets) / ref_det


def deform(x, tets, A, rng, noise_frac=NOISE_FRAC, h_mean=None):
    """Affine map plus the shrinking node noise described in the module doc.

    Returns float64 deformed positions and a dict of statistics.
    """
    A = np.asarray(A, dtype=np.float64)
    if h_mean is None:
        h_mean = mean_edge_length(x, tets)
    sigma = noise_frac * h_mean
    eta = rng.normal(0.0, sigma, size=x.shape)
    base = x @ A.T
    floor = J_FLOOR * np.linalg.det(A)
    ref_det = _det_edges(x, tets)
    shrunk = np.zeros(len(x), dtype=bool)
    rounds = 0
    y = base + eta
    J = volume_ratios(x, y, tets, ref_det)
    while True:
        bad = J < floor
        if not bad.any():
            break
        nodes = np.unique(tets[bad].ravel())
        eta[nodes] *= 0.5
        shrunk[nodes] = True
        y = base + eta
        # only tets touching a changed node need a new ratio
        touched = np.flatnonzero(shrunk[tets].any(axis=1))
        J[touched] = volume_ratios(x, y, tets[touched], ref_det[touched])
        rounds += 1
        if rounds > 60:
            raise RuntimeError("noise rule did not converge")
    return y, {"sigma": sigma, "shrink_rounds": rounds,
               "shrunk_frac": float(shrunk.mean()), "min_J": float(J.min())}


def compression_shear_map(lam, gamma):
    """Compression to ``lam`` along z plus simple shear ``gamma`` (xz)."""
    return np.array([[1.0, 0.0, gamma], [0.0, 1.0, 0.0], [0.0, 0.0, lam]])


def random_theta(rng):
    """mu ~ U[0.5, 2], kappa/mu ~ U[5, 50], w ~ U[0, 1]."""
    mu = rng.uniform(0.5, 2.0)
    return (mu, mu * rng.uniform(5.0, 50.0), rng.uniform(0.0, 1.0))


def small_sphere_case(seed: int, noise=True) -> Cell:
    """~1,000 nodes / ~5,000 tets; uniaxial compression lam ~ U[0.2, 1];
    mu = 1, kappa = 10, w = 0.5."""
    x, tets = sphere_mesh(1000, seed)
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.2, 1.0)
    A = np.diag([1.0, 1.0, lam])
    if noise:
        y, info = deform(x, tets, A, rng)
    else:
        y, info = x @ A.T, {}
    info["lam"] = lam
    return Cell(x, tets, y.astype(np.float32), (1.0, 10.0, 0.5), A, info)


def paper_sphere_case(seed: int, n_target: int = 20000, noise=True) -> Cell:
    """~20,000 nodes / ~115,000 tets; compression s ~ U[0, 0.8] along z plus
    shear gamma ~ U[0, 0.5]; random (mu, kappa, w)."""
    x, tets = sphere_mesh(n_target, seed)
    rng = np.random.default_rng(seed)
    lam = 1.0 - rng.uniform(0.0, 0.8)
    gamma = rng.uniform(0.0, 0.5)
    A = compression_shear_map(lam, gamma)
    theta = random_theta(rng)
    if noise:
        y, info = deform(x, tets, A, rng)
    else:
        y, info = x @ A.T, {}
    info.update(lam=lam, gamma=gamma)
    return Cell(x, tets, y.astype(np.float32), theta, A, info)


def cotangent(n_nodes: int, seed: int) -> np.ndarray:
    """Seeded N(0, 1) cotangent for the force output (float32, (N, 3))."""
    return np.random.default_rng(seed).normal(
        0.0, 1.0, size=(n_nodes, 3)).astype(np.float32)


def mesh_ladder(n_entries, tet_lo, tet_hi, seed):
    """Sphere meshes whose tet counts span [tet_lo, tet_hi] geometrically."""
    targets = np.geomspace(tet_lo, tet_hi, n_entries)
    out = []
    for k, mt in enumerate(targets):
        # about 5.3 tets per node over this range
        x, tets = sphere_mesh(max(40, int(round(mt / 5.3))), seed + k)
        edges = unique_edges(tets)
        out.append((x, tets, edges))
    return out


def uneven_batch(n_cells=4096, seed=3000, tet_lo=500, tet_hi=20000,
                 ladder=64, axes_lo=0.7, axes_hi=1.3) -> Batch:
    """Cells of uneven size: ellipsoids with semi-axes ~ U[0.7, 1.3] R and
    tet counts ~ U[tet_lo, tet_hi], each with its own compression + shear,
    noise and (mu, kappa, w).  Meshes come from a ladder of ``ladder``
    resolutions; every cell gets its own reference geometry (the axes), so
    every cell's inverse edge matrices differ."""
    lad = mesh_ladder(ladder, tet_lo, tet_hi, seed + 1)
    lad_m = np.array([len(t) for _, t, _ in lad])
    ss = np.random.SeedSequence(seed)
    cells = []
    for child in ss.spawn(n_cells):
        rng = np.random.default_rng(child)
        target = rng.uniform(tet_lo, tet_hi)
        k = int(np.argmin(np.abs(lad_m - target)))
        x0, tets, edges = lad[k]
        axes = rng.uniform(axes_lo, axes_hi, size=3)
        x = ellipsoid(x0, axes)
        h = float(np.linalg.norm(x[edges[:, 0]] - x[edges[:, 1]], axis=1).mean())
        lam = 1.0 - rng.uniform(0.0, 0.8)
        gamma = rng.uniform(0.0, 0.5)
        A = compression_shear_map(lam, gamma)
        theta = random_theta(rng)
        y, info = deform(x, tets, A, rng, h_mean=h)
        cells.append(Cell(x, tets, y.astype(np.float32), theta, A, info))
    b = batch_from_cells(cells)
    b.info = {"ladder_tets": lad_m.tolist()}
    return b


def template_batch(n_cells, n_target, seed) -> Batch:
    """``n_cells`` copies of one sphere mesh (about ``n_target`` nodes), each
    with its own compression + shear, node noise and (mu, kappa, w), drawn as
    in uneven_batch.  The arrays hold every copy, so the same Batch feeds a
    shared-mesh handle (first copy) and a distinct-array handle (all)."""
    x, tets = sphere_mesh(n_target, seed)
    h = mean_edge_length(x, tets)
    ss = np.random.SeedSequence(seed + 1)
    cells = []
    for child in ss.spawn(n_cells):
        rng = np.random.default_rng(child)
        A = compression_shear_map(1.0 - rng.uniform(0.0, 0.8),
                                  rng.uniform(0.0, 0.5))
        theta = random_theta(rng)
        y, info = deform(x, tets, A, rng, h_mean=h)
        cells.append(Cell(x, tets, y.astype(np.float32), theta, A, info))
    b = batch_from_cells(cells)
    b.info = {"template_nodes": len(x), "template_tets": len(tets)}
    return b


def radial_regions(x, tets, r_nucleus=0.45, r_cortex=0.85):
    """Material region of every tetrahedron from the distance of its
    reference centroid to the cell's centre of mass (radius-normalised):
    1 = nucleus (< r_nucleus), 2 = cortex shell (> r_cortex), 0 = cytoplasm."""
    c = x[tets].mean(axis=1)
    c = c - x.mean(axis=0)
    r = np.linalg.norm(c, axis=1) / np.linalg.norm(x - x.mean(axis=0), axis=1).max()
    reg = np.zeros(len(tets), dtype=np.uint8)
    reg[r < r_nucleus] = 1
    reg[r > r_cortex] = 2
    return reg


# ---------------------------------------------------------------- plates
STOKES_DT = 1e-3      # time step of the compression runs
DRAG = 0.25           # uniform nodal drag; mobility = STOKES_DT / DRAG
K_PLATE = 100.0       # plate penalty in units of mu_ref / R^2 (mu_ref = 1)


def plate_schedule(n_steps, radius=1.0, compression=0.8):
    """Top-plate heights: linear from +R to R - 2 R compression over the
    steps (80 % of the diameter by default); the bottom plate rests at -R."""
    top = radius - 2.0 * radius * compression * np.arange(n_steps) / max(
        n_steps - 1, 1)
    return top, -radius


def oblate_batch(n_cells, n_target, seed, n_meshes=8):
    """Undeformed oblate ellipsoids for quasi-static compression: semi-axes
    U[1.05, 1.25] x U[1.0, 1.2] x U[0.75, 0.85] R (shortest on z, the
    compression axis, so the cell cannot roll between frictionless plates),
    meshes from ``n_meshes`` sphere seeds, theta drawn like random_theta."""
    meshes = [sphere_mesh(n_target, seed + 31 * k) for k in range(n_meshes)]
    rng = np.random.default_rng(seed)
    cells = []
    for c in range(n_cells):
        x0, tets = meshes[c % n_meshes]
        ax = np.array([rng.uniform(1.05, 1.25), rng.uniform(1.0, 1.2),
                       rng.uniform(0.75, 0.85)])
        x = ellipsoid(x0, ax)
        cells.append(Cell(x, tets.copy(), x.astype(np.float32),
                          random_theta(rng)))
    return batch_from_cells(cells)


def compression_batch(n_cells, n_target, seed, n_meshes=None):
    """Spheres (R = 1) for the plate-compression runs, each with a hidden
    parameter set theta* (seed) and a start theta0 (seed + 1), both drawn
    like random_theta.  Meshes come from ``n_meshes`` distinct seeds (all
    cells by default); every cell keeps its own arrays."""
    n_meshes = n_meshes or n_cells
    meshes = [sphere_mesh(n_target, seed + 17 * k) for k in range(n_meshes)]
    r_star = np.random.default_rng(seed)
    r_zero = np.random.default_rng(seed + 1)
    cells, th0 = [], []
    for c in range(n_cells):
        x, tets = meshes[c % n_meshes]
        cells.append(Cell(x.copy(), tets.copy(), x.astype(np.float32),
                          random_theta(r_star)))
        th0.append(random_theta(r_zero))
    b = batch_from_cells(cells)
    b.info = {"theta_star": b.theta.copy(),
              "theta0": np.array(th0, dtype=np.float64)}
    return b


def calibration_batch(n_cells, n_target, seed, n_meshes=8):
    """Oblate cells (as oblate_batch) for quasi-static calibration: the
    batch's theta is the hidden theta* (seed), info["theta0"] a start drawn
    the same way (seed + 1)."""
    b = oblate_batch(n_cells, n_target, seed, n_meshes=n_meshes)
    r0 = np.random.default_rng(seed + 1)
    b.info = {"theta_star": b.theta.copy(),
              "theta0": np.array([random_theta(r0) for _ in range(n_cells)],
                                 dtype=np.float64)}
    return b


def qs_fractions(n_steps=10, lo=0.08, hi=0.8):
    """Plate travel of the quasi-static calibration curves as fractions of
    each cell's reference height (8 % to 80 %)."""
    return np.linspace(lo, hi, n_steps)
