"""Writes qs_targets.npy: quasi-static force-indentation curves F*[s, c] of
the calibration workload (synth.configs calibration_batch(32, 2000, 7100):
oblate cells of about 2,000 nodes; plates closing from each cell's reference
extent by the fractions qs_fractions() = 8 % ... 80 % of its height) at the
hidden parameters theta*, computed by the FP64 oracle's minimiser of the
plate potential (oracle/quasistatic.py, each position from the previous
equilibrium).  Targets of the benchmark's calibration leg.  Calls only
oracle/ and the seeded input generator.

usage: python tests/golden/make_qs_targets.py [n_workers]
"""
import os
import sys
import warnings
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import quasistatic as oqs  # noqa: E402
from synth.configs import K_PLATE, calibration_batch, qs_fractions  # noqa: E402

N_CELLS, N_TARGET, SEED = 32, 2000, 7100
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qs_targets.npy")

_b = None


def _curve(c):
    cell = _b.cell(c)
    m = oracle.OracleMesh(cell.x, cell.tets)
    top0, bot = cell.x[:, 2].max(), cell.x[:, 2].min()
    tops = top0 - qs_fractions() * (top0 - bot)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", RuntimeWarning)
        F, _ = oqs.force_curve(m, cell.y.astype(np.float64),
                               tuple(_b.info["theta_star"][c]), tops, bot, K_PLATE)
    return c, F


def main():
    global _b
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    _b = calibration_batch(N_CELLS, N_TARGET, SEED)
    oracle.lib()
    out = np.empty((len(qs_fractions()), N_CELLS))
    with Pool(workers) as pool:
        for c, F in pool.imap_unordered(_curve, range(N_CELLS)):
            out[:, c] = F
            print(f"cell {c} done", flush=True)
    np.save(OUT, out)
    print(f"wrote {OUT}: {out.shape}")


if __name__ == "__main__":
    main()
