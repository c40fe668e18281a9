"""Mooney-Rivlin tetrahedral cell forces on AMD Instinct MI355X (gfx950).

Hot path of Mueller et al., "A hyperelastic model for simulating cells in
flow" (arXiv 2003.03130): per-tetrahedron deformation gradient, invariants,
three-parameter Mooney-Rivlin energy and nodal forces f = -V0 dU/dy, plus
their exact adjoint.  All arithmetic runs in the HIP library libcellmech.so
(include/cellmech.h); this package marshals arguments and provides a
torch.autograd.Function and a checkpointed relaxation driver on top.
"""
from ._native import CellmechError, ORDER_INPUT, ORDER_MORTON, ORDER_RCM  # noqa: F401
from .cells import CellBatch, HostLayout  # noqa: F401


def moduli_from_young_poisson(E, nu):
    """Small-strain consistency of Sec. "Theory" (eq. elastic-moduli:mr):
    mu = E / (2 (1 + nu)), kappa = E / (3 (1 - 2 nu))."""
    return E / (2.0 * (1.0 + nu)), E / (3.0 * (1.0 - 2.0 * nu))
