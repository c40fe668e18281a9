"""Planted mistakes in the oracle must be caught by the pins.

Each mutant is a copy of ``oracle/cm_oracle.cpp`` with one plausible mistake
(a dropped term, a wrong sign, index or power, a transposed operand), compiled
with g++ into a temporary directory.  Every pin of ``tests/pins.py`` runs on
it; at least one must fail.  CPU only.
"""
import os

import pytest

import oracle
import pins

MUTANTS = [
    ("drop_kappa_term", "S g_J = dU_dI * dI_dJ + dU_dK * dK_dJ + dU_dJ;",
     "S g_J = dU_dI * dI_dJ + dU_dK * dK_dJ;"),
    ("sign_dK_dTC2", "S dK_dTC2 = -0.5 * Jm43;", "S dK_dTC2 = 0.5 * Jm43;"),
    ("transpose_B_in_dF_du", "dF += B[m][l] *", "dF += B[l][m] *"),
    ("transpose_Finv_in_dJ_dF", "S dJ_dF = J * Finv[l][i];",
     "S dJ_dF = J * Finv[i][l];"),
    ("wrong_power_J53", "S Jm53 = Jm43 * s;", "S Jm53 = Jm23 * s;"),
    ("reference_volume_factor", "*V0 = std::fabs(dJ) / 6.0;",
     "*V0 = std::fabs(dJ) / 2.0;"),
    ("vertex4_sign", "((m == a ? 1.0 : 0.0) - (a == 3 ? 1.0 : 0.0))",
     "((m == a ? 1.0 : 0.0) + (a == 3 ? 1.0 : 0.0))"),
    ("transpose_F_in_dTC2_dF", "4.0 * F[i][k] * C[k][l]",
     "4.0 * F[k][i] * C[k][l]"),
    ("mu_split_swapped", "double mu1 = w * mu, mu2 = (1.0 - w) * mu;",
     "double mu1 = (1.0 - w) * mu, mu2 = w * mu;"),
    ("wrong_origin_vertex", "A[i][k] = u[k][i] - u[3][i];",
     "A[i][k] = u[k][i] - u[0][i];"),
    ("missing_half_in_K", "S K = 0.5 * (TC * TC - TC2) * Jm43;",
     "S K = (TC * TC - TC2) * Jm43;"),
    ("dK_dJ_coefficient", "S dK_dJ = (-2.0 / 3.0) * (TC * TC - TC2) * Jm73;",
     "S dK_dJ = (-4.0 / 3.0) * (TC * TC - TC2) * Jm73;"),
    ("cube_root_of_abs", "inline double real_cbrt(double x) { return std::cbrt(x); }",
     "inline double real_cbrt(double x) { return std::cbrt(std::fabs(x)); }"),
    ("ybar_energy_sign", "ybar[q] -= ebar * f[q];", "ybar[q] += ebar * f[q];"),
    ("thetabar_w_not_tracked", "D mu1 = dw * dmu, mu2 = (1.0 - dw) * dmu;",
     "D mu1 = dw * dmu, mu2 = (1.0 - w) * dmu;"),
    ("plate_penalty_sign", "pz = pz - k * d * d;", "pz = pz + k * d * d;"),
    ("plate_step_uses_old_force_sign",
     "y[3 * a + 2] = z + mob * (f[3 * a + 2] + pz);",
     "y[3 * a + 2] = z - mob * (f[3 * a + 2] + pz);"),
    ("relax_gradient_factor", "g[k] += 2.0 * scale * r * F[n].d[k];",
     "g[k] += scale * r * F[n].d[k];"),
    ("left_instead_of_right_cauchy_green",
     "for (int m = 0; m < 3; ++m) s = s + F[m][k] * F[m][l];",
     "for (int m = 0; m < 3; ++m) s = s + F[k][m] * F[l][m];"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    with open(oracle._SRC) as fh:
        src = fh.read()
    assert old in src, f"mutation site of {name} not found"
    mutated = src.replace(old, new)
    path = os.path.join(tmp_path, f"mut_{name}.cpp")
    with open(path, "w") as fh:
        fh.write(mutated)
    so = oracle.build(force=True, src=path,
                      out=os.path.join(tmp_path, f"libmut_{name}.so"))
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(so)
        except (AssertionError, ValueError, FloatingPointError):
            caught.append(pin.__name__)
    assert caught, f"no pin detects the mutant {name}"
