"""Writes relax_targets.npy: the top-plate force curves F*[n, c] of the
plate-compression workload (256 spheres of about 51k tetrahedra, 200
overdamped explicit steps, plates to 20 % compression; synth.configs
compression_batch, seed 5000) at each cell's hidden parameters theta*,
replayed by the FP64 oracle (or_relax_forward).  These are the calibration
targets of the benchmark's plate-compression leg and of the full-size GPU
test.  Calls only oracle/ and the seeded input generator.

usage: python tests/golden/make_relax_targets.py [n_workers]
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.configs import (DRAG, K_PLATE, STOKES_DT, compression_batch,  # noqa: E402
                           plate_schedule)

N_CELLS, N_TARGET, SEED, N_MESHES = 256, 9000, 5000, 8
N_STEPS, COMPRESSION = 200, 0.2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "relax_targets.npy")

_b = None


def _curve(c):
    cell = _b.cell(c)
    m = oracle.OracleMesh(cell.x, cell.tets)
    top, bot = plate_schedule(N_STEPS, compression=COMPRESSION)
    # the start state as the device holds it (float32 reference positions)
    F, _ = m.relax_forward(cell.y.astype(np.float64),
                           tuple(_b.info["theta_star"][c]), top, bot,
                           K_PLATE, STOKES_DT / DRAG)
    return c, F


def main():
    global _b
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    _b = compression_batch(N_CELLS, N_TARGET, SEED, n_meshes=N_MESHES)
    oracle.lib()  # built before the workers fork
    out = np.empty((N_STEPS, N_CELLS))
    with Pool(workers) as pool:
        for c, F in pool.imap_unordered(_curve, range(N_CELLS)):
            out[:, c] = F
            print(f"cell {c} done", flush=True)
    np.save(OUT, out)
    print(f"wrote {OUT}: {out.shape}")


if __name__ == "__main__":
    main()
