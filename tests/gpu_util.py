"""Helpers of the GPU tests: device checks and the parity metrics."""
import numpy as np
import pytest

import oracle


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03130_amd import _native
    _native.lib()  # raises if the HIP library is missing: no fallback


def force_rel_err(f_gpu, f_ref):
    """max_a |f_gpu - f_ref| / max_a |f_ref| over all components."""
    return float(np.abs(f_gpu.astype(np.float64) - f_ref).max()
                 / np.abs(f_ref).max())


def rel_err(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


def oracle_cell(cell, theta=None):
    m = oracle.OracleMesh(cell.x, cell.tets)
    return m, m.forces(cell.y.astype(np.float64), theta or cell.theta)


def run_cell(cell, **kw):
    """Forces, energy and inverted count of one cell on the GPU."""
    import torch
    from paper_2003_03130_amd import CellBatch
    cb = CellBatch.single(cell.x, cell.tets, **kw)
    cb.set_params(*cell.theta)
    y = cb.to_device(cell.y)
    ninv = torch.zeros(1, dtype=torch.int32, device=cb.device)
    f, E = cb.forces(y, n_inverted=ninv)
    torch.cuda.synchronize()
    return cb, cb.to_host(f), float(E.item()), int(ninv.item())
