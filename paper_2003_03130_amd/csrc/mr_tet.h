// Per-tetrahedron Mooney-Rivlin evaluation for gfx950.
//
// The paper evaluates f_i^a = -V0 dU/du_i^a with the chain rule of
// eq. elastic-force-vertex-1 and the derivative table that follows the
// Jacobian paragraph.  Collecting that chain rule gives the first
// Piola-Kirchhoff stress P = dU/dF in closed form:
//   P = mu1 J^-2/3 (F - T_C/3 F^-T)
//     + mu2 J^-4/3 (T_C F - F C - 2/3 I2 F^-T)
//     + kappa J (J - 1) F^-T,                 I2 = (T_C^2 - T_C2)/2,
// and, with dF_kl/du_i^a = delta_ki B_ml (delta_ma - delta_4a), the forces
//   [f^1 f^2 f^3] = -V0 P B^T,   f^4 = -(f^1 + f^2 + f^3).
// With cof F = J F^-T (division free) this is
//   P = c1 F + c2 (F C) + c3 cof F,
//   c1 = mu1 J^-2/3 + mu2 J^-4/3 T_C,  c2 = -mu2 J^-4/3,
//   c3 = -(mu1 J^-2/3 T_C + 2 mu2 J^-4/3 I2) / (3 J) + kappa (J - 1).
//
// Precision: the edge vectors y^k - y^4 and F = D_s B are formed in float64
// (the difference of two float32 positions is exact in float64, so F is the
// exact product of the float32 inputs up to one float64 rounding; a float32
// edge or product would amplify rounding by the condition number of the
// reference tetrahedron).  The invariants, the powers of J, the energy
// density and, in the forward pass, the coefficients c1..c3 are float64; the
// remaining 3x3 tensor algebra (F C, cof F, P B^T) is float32 (the backward
// pass forms its coefficient chain in float32 too, see tet_backward).
// J^-1/3 is the reciprocal of the real (sign-preserving) cube root: a
// float32 hardware log2/exp2 seed
// refined by one Newton step in float64.
// Every helper contracts a * b + c into a fused multiply-add only within
// one expression, as written (fp contract on): the rounding of each result
// is then fixed by the source alone, whatever code the helper is inlined
// into, so the separate passes and the fused forward + backward pass round
// identically.
#pragma once
#include <hip/hip_runtime.h>

namespace cm {

struct Material {
  double mu1, mu2, kappa;
};

// Real J^-1/3 (negative for J < 0, infinite/NaN for J = 0).
__device__ __forceinline__ double inv_cbrt(double J) {
#pragma clang fp contract(on)
  const float jf = (float)J;
  float s = __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(fabsf(jf)) * (1.0f / 3.0f));
  s = copysignf(s, jf);
  const double r = (double)s;
  // Newton step for g(r) = r^-3 - J: r <- r (4 - J r^3) / 3.
  return r * (4.0 - J * (r * r * r)) * (1.0 / 3.0);
}

// Scalar part shared by the forward and backward passes.
struct Scalars {
  double TC, J, r, r2, r4, I2;
};

// Float64 invariants of the float64 deformation gradient f; Cf receives
// C = F^T F rounded to float32 (C00 C11 C22 C01 C02 C12).
__device__ __forceinline__ void invariants(const double f[3][3], float Cf[6],
                                           Scalars& s) {
#pragma clang fp contract(on)
  const double C00 = f[0][0] * f[0][0] + f[1][0] * f[1][0] + f[2][0] * f[2][0];
  const double C11 = f[0][1] * f[0][1] + f[1][1] * f[1][1] + f[2][1] * f[2][1];
  const double C22 = f[0][2] * f[0][2] + f[1][2] * f[1][2] + f[2][2] * f[2][2];
  const double C01 = f[0][0] * f[0][1] + f[1][0] * f[1][1] + f[2][0] * f[2][1];
  const double C02 = f[0][0] * f[0][2] + f[1][0] * f[1][2] + f[2][0] * f[2][2];
  const double C12 = f[0][1] * f[0][2] + f[1][1] * f[1][2] + f[2][1] * f[2][2];
  Cf[0] = (float)C00; Cf[1] = (float)C11; Cf[2] = (float)C22;
  Cf[3] = (float)C01; Cf[4] = (float)C02; Cf[5] = (float)C12;
  s.TC = C00 + C11 + C22;
  s.J = f[0][0] * (f[1][1] * f[2][2] - f[1][2] * f[2][1]) -
        f[0][1] * (f[1][0] * f[2][2] - f[1][2] * f[2][0]) +
        f[0][2] * (f[1][0] * f[2][1] - f[1][1] * f[2][0]);
  s.r = inv_cbrt(s.J);
  s.r2 = s.r * s.r;
  s.r4 = s.r2 * s.r2;
  // I2 = (T_C^2 - T_C2) / 2, the sum of the principal 2x2 minors of C
  s.I2 = C00 * C11 + C00 * C22 + C11 * C22 - C01 * C01 - C02 * C02 - C12 * C12;
}

// Cofactor matrix cof F = det(F) F^-T (columns are cross products of the
// other two columns of F).
__device__ __forceinline__ void cofactor(const float F[3][3], float K[3][3]) {
#pragma clang fp contract(on)
  K[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  K[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  K[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  K[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  K[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  K[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  K[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  K[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  K[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
}

// F C with C symmetric stored as C00 C11 C22 C01 C02 C12.
__device__ __forceinline__ void times_sym(const float F[3][3], const float C[6],
                                          float R[3][3]) {
#pragma clang fp contract(on)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    R[i][0] = F[i][0] * C[0] + F[i][1] * C[3] + F[i][2] * C[4];
    R[i][1] = F[i][0] * C[3] + F[i][1] * C[1] + F[i][2] * C[5];
    R[i][2] = F[i][0] * C[4] + F[i][1] * C[5] + F[i][2] * C[2];
  }
}

// F = D_s B in float64 from the float32 vertex positions p0..p3 (columns of
// D_s are the edges y^k - y^4, exact in float64); f32 receives F rounded.
__device__ __forceinline__ void deformation_gradient(
    const float4& p0, const float4& p1, const float4& p2, const float4& p3,
    const float B[9], double F[3][3], float f32[3][3]) {
#pragma clang fp contract(on)
  const double e[3][3] = {
      {(double)p0.x - (double)p3.x, (double)p0.y - (double)p3.y, (double)p0.z - (double)p3.z},
      {(double)p1.x - (double)p3.x, (double)p1.y - (double)p3.y, (double)p1.z - (double)p3.z},
      {(double)p2.x - (double)p3.x, (double)p2.y - (double)p3.y, (double)p2.z - (double)p3.z}};
  double b[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) b[m] = (double)B[m];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      F[i][j] = e[0][i] * b[j] + e[1][i] * b[3 + j] + e[2][i] * b[6 + j];
      f32[i][j] = (float)F[i][j];
    }
}

// Direction dF = D_v B (float32) from the float32 cotangents v0..v3.
__device__ __forceinline__ void direction_gradient(
    const float4& v0, const float4& v1, const float4& v2, const float4& v3,
    const float B[9], float D[3][3]) {
#pragma clang fp contract(on)
  const float e[3][3] = {{v0.x - v3.x, v0.y - v3.y, v0.z - v3.z},
                         {v1.x - v3.x, v1.y - v3.y, v1.z - v3.z},
                         {v2.x - v3.x, v2.y - v3.y, v2.z - v3.z}};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      D[i][j] = e[0][i] * B[j] + e[1][i] * B[3 + j] + e[2][i] * B[6 + j];
}

// Stress and forces from F (float32 copy), C and the float64 scalars: h[k][i]
// on vertices k = 0..2 (vertex 3 takes the negative sum) and the
// tetrahedron's energy V0 U (float64).
__device__ __forceinline__ void stress_forces(const float F[3][3], const float Cf[6],
                                              const Scalars& s, const float B[9],
                                              float V0, const Material& m,
                                              float h[3][3], double& vU) {
#pragma clang fp contract(on)
  const double Jm1 = s.J - 1.0;
  const double U = 0.5 * m.mu1 * (s.TC * s.r2 - 3.0) +
                   0.5 * m.mu2 * (s.I2 * s.r4 - 3.0) + 0.5 * m.kappa * Jm1 * Jm1;
  vU = (double)V0 * U;
  const double a = m.mu1 * s.r2, b = m.mu2 * s.r4;
  const double c1 = a + b * s.TC;
  const double c2 = -b;
  const double c3 = -(a * s.TC + 2.0 * b * s.I2) * (1.0 / 3.0) * (s.r2 * s.r) +
                    m.kappa * Jm1;
  const double nv = -(double)V0;
  const float s1 = (float)(nv * c1), s2 = (float)(nv * c2), s3 = (float)(nv * c3);
  // P = F (s1 I + s2 C) + s3 cof F
  const float M[6] = {fmaf(s2, Cf[0], s1), fmaf(s2, Cf[1], s1), fmaf(s2, Cf[2], s1),
                      s2 * Cf[3], s2 * Cf[4], s2 * Cf[5]};
  float K[3][3], P[3][3];
  times_sym(F, M, P);
  cofactor(F, K);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P[i][j] = fmaf(s3, K[i][j], P[i][j]);
  // h[k][i] = (P B^T)_ik, already scaled by -V0
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      h[k][i] = P[i][0] * B[3 * k] + P[i][1] * B[3 * k + 1] + P[i][2] * B[3 * k + 2];
}

// Forward: forces h[k][i] on vertices k = 0..2 (vertex 3 takes the negative
// sum) and the tetrahedron's energy V0 U (float64).
__device__ __forceinline__ void tet_forward(const float4& p0, const float4& p1,
                                            const float4& p2, const float4& p3,
                                            const float B[9], float V0,
                                            const Material& m, float h[3][3],
                                            double& vU, bool& inverted) {
#pragma clang fp contract(on)
  double Fd[3][3];
  float F[3][3], Cf[6];
  deformation_gradient(p0, p1, p2, p3, B, Fd, F);
  Scalars s;
  invariants(Fd, Cf, s);
  inverted = !(s.J > 0.0);
  stress_forces(F, Cf, s, B, V0, m, h, vU);
}

// d(cof F) along dF: the columns of cof F are cross products of the other
// two columns of F (cyclic), so each derivative column is a sum of two
// cross products.
__device__ __forceinline__ void cofactor_dir(const float F[3][3],
                                             const float D[3][3],
                                             float R[3][3]) {
#pragma clang fp contract(on)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    // cross(D[:,a], F[:,b]) + cross(F[:,a], D[:,b])
    R[0][c] = D[1][a] * F[2][b] - D[2][a] * F[1][b] + F[1][a] * D[2][b] - F[2][a] * D[1][b];
    R[1][c] = D[2][a] * F[0][b] - D[0][a] * F[2][b] + F[2][a] * D[0][b] - F[0][a] * D[2][b];
    R[2][c] = D[0][a] * F[1][b] - D[1][a] * F[0][b] + F[0][a] * D[1][b] - F[1][a] * D[0][b];
  }
}

// Backward of one tetrahedron for a loss L(f, E) (adjoint_terms takes F, dF,
// C, cof F and the float64 scalars; tet_backward forms them first):
//   dF = D_fbar B is the direction of the Hessian-vector product (the forces
//   are -grad E, so (df/dy)^T fbar = d/de f(y + e fbar));
//   h[k][i] = (-V0 (dP[dF] - ebar P) B^T)_ik, the contribution to ybar of
//   vertices k = 0..2 (vertex 3 takes the negative sum);
//   dL/d(mu1, mu2, kappa) of this tetrahedron is V0 (-gp + ebar ge / 2):
//   P is linear in (mu1, mu2, kappa), P = mu1 P_I + mu2 P_K + kappa P_J, so
//   gp = (<P_I, dF>, <P_K, dF>, (J - 1) <cof F, dF>) and
//   ge = (I - 3, K - 3, (J - 1)^2) (twice the energy parts).
// F and the invariants are float64 as in the forward pass; the stress
// coefficients and their derivatives along dF are float32, formed from
// float32 copies of the float64 invariants (J - 1 included): that chain has
// no cancellation beyond the one P itself carries, and float32 there keeps
// float64 off most of the pass.  gp and ge stay float64 (the deviatoric
// parts of gp, I - 3 and K - 3 cancel down to the order of the strain).
// GRAD = false: the Hessian-vector product alone (no energy cotangent, no
// parameter gradient): ebar is taken as 0 and gp, ge are not formed.
template <bool GRAD>
__device__ __forceinline__ void adjoint_terms(const float F[3][3], const float dF[3][3],
                                              const float Cf[6], const float K[3][3],
                                              const Scalars& s, const float B[9],
                                              float V0, const Material& m, double ebar,
                                              float h[3][3], double gp[3], double ge[3]) {
#pragma clang fp contract(on)
  // dC = dF^T F + F^T dF (symmetric): diagonal dC_jj = 2 u_j with
  // u_j = <F e_j, dF e_j>; off-diagonal 01 02 12
  float u[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    u[j] = dF[0][j] * F[0][j] + dF[1][j] * F[1][j] + dF[2][j] * F[2][j];
  const float dC01 = dF[0][0] * F[0][1] + dF[1][0] * F[1][1] + dF[2][0] * F[2][1] +
                     F[0][0] * dF[0][1] + F[1][0] * dF[1][1] + F[2][0] * dF[2][1];
  const float dC02 = dF[0][0] * F[0][2] + dF[1][0] * F[1][2] + dF[2][0] * F[2][2] +
                     F[0][0] * dF[0][2] + F[1][0] * dF[1][2] + F[2][0] * dF[2][2];
  const float dC12 = dF[0][1] * F[0][2] + dF[1][1] * F[1][2] + dF[2][1] * F[2][2] +
                     F[0][1] * dF[0][2] + F[1][1] * dF[1][2] + F[2][1] * dF[2][2];
  // <F, dF> = tr(dC)/2, <F C, dF> = <C, F^T dF> = <C, dC>/2, <cof F, dF> = dJ
  const float fF = u[0] + u[1] + u[2];
  const float fFC = Cf[0] * u[0] + Cf[1] * u[1] + Cf[2] * u[2] +
                    Cf[3] * dC01 + Cf[4] * dC02 + Cf[5] * dC12;
  float fK = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) fK = fmaf(K[i][j], dF[i][j], fK);
  // float32 copies of the float64 scalars
  const double Jm1d = s.J - 1.0;
  const float TC = (float)s.TC, I2 = (float)s.I2, r2 = (float)s.r2, r4 = (float)s.r4;
  const float r3 = (float)(s.r2 * s.r);  // 1/J
  const float Jm1 = (float)Jm1d;
  // directional derivatives of tr C, tr C^2, J and I2 = (trC^2 - trC2)/2;
  // with t = dJ / J: d J^-2/3 = -(2/3) J^-2/3 t, d J^-4/3 = -(4/3) J^-4/3 t
  const float dTC = 2.f * fF;
  const float dJ = fK;
  const float dI2 = 2.f * (TC * fF - fFC);
  const float tq = r3 * dJ;
  const float a = (float)m.mu1 * r2, b = (float)m.mu2 * r4, ka = (float)m.kappa;
  const float da = (-2.f / 3.f) * a * tq, db = (-4.f / 3.f) * b * tq;
  const float c1 = a + b * TC, dc1 = da + db * TC + b * dTC;
  const float c2 = -b, dc2 = -db;
  const float q = -(a * TC + 2.f * b * I2) * (1.f / 3.f);
  const float dq = -(da * TC + a * dTC + 2.f * (db * I2 + b * dI2)) * (1.f / 3.f);
  const float c3 = q * r3 + ka * Jm1;
  const float dc3 = r3 * (dq - q * tq) + ka * dJ;
  const float nv = -V0;
  const float eb = GRAD ? (float)ebar : 0.f;
  const float s1 = nv * (dc1 - eb * c1), t1 = nv * c1;
  const float s2 = nv * (dc2 - eb * c2), t2 = nv * c2;
  const float s3 = nv * (dc3 - eb * c3), t3 = nv * c3;

  // -V0 (dP - ebar P) with P = c1 F + c2 F C + c3 cof F:
  //   s1 F + t1 dF + s2 F C + t2 (dF C + F dC) + s3 cof F + t3 d(cof F)
  //   = F (s1 I + s2 C + t2 dC) + dF (t1 I + t2 C) + s3 cof F + t3 d(cof F)
  const float t2x2 = 2.f * t2;
  const float M[6] = {fmaf(t2x2, u[0], fmaf(s2, Cf[0], s1)),
                      fmaf(t2x2, u[1], fmaf(s2, Cf[1], s1)),
                      fmaf(t2x2, u[2], fmaf(s2, Cf[2], s1)),
                      fmaf(t2, dC01, s2 * Cf[3]), fmaf(t2, dC02, s2 * Cf[4]),
                      fmaf(t2, dC12, s2 * Cf[5])};
  const float Nm[6] = {fmaf(t2, Cf[0], t1), fmaf(t2, Cf[1], t1), fmaf(t2, Cf[2], t1),
                       t2 * Cf[3], t2 * Cf[4], t2 * Cf[5]};
  float dK[3][3];
  cofactor_dir(F, dF, dK);
  const int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  float Q[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Q[i][j] = F[i][0] * M[sym[0][j]] + F[i][1] * M[sym[1][j]] + F[i][2] * M[sym[2][j]] +
                dF[i][0] * Nm[sym[0][j]] + dF[i][1] * Nm[sym[1][j]] +
                dF[i][2] * Nm[sym[2][j]] + s3 * K[i][j] + t3 * dK[i][j];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      h[k][i] = Q[i][0] * B[3 * k] + Q[i][1] * B[3 * k + 1] + Q[i][2] * B[3 * k + 2];

  // parameter gradient: per unit V0, the directional derivatives p of the
  // energy parts along dF and the energy parts e themselves, so that
  // g = V0 (-p + ebar e / 2) is formed once per tile
  if constexpr (GRAD) {
    // gp[0] and gp[1] are deviatoric projections: <F, dF> and the TC dJ / 3J
    // term cancel down to the order of the strain, so they are formed in
    // float64 from the float64 invariants (a float32 copy of TC or 1/J would
    // enter amplified by 1/strain)
    const double fFd = (double)fF, dJd = (double)dJ;
    const double tqd = (s.r2 * s.r) * dJd;
    gp[0] = s.r2 * (fFd - s.TC * tqd * (1.0 / 3.0));
    gp[1] = s.r4 * (s.TC * fFd - (double)fFC - (2.0 / 3.0) * s.I2 * tqd);
    gp[2] = Jm1d * dJd;
    ge[0] = s.TC * s.r2 - 3.0;
    ge[1] = s.I2 * s.r4 - 3.0;
    ge[2] = Jm1d * Jm1d;
  }
}

template <bool GRAD>
__device__ __forceinline__ void tet_backward(
    const float4& p0, const float4& p1, const float4& p2, const float4& p3,
    const float4& v0, const float4& v1, const float4& v2, const float4& v3,
    const float B[9], float V0, const Material& m, double ebar, float h[3][3],
    double gp[3], double ge[3]) {
#pragma clang fp contract(on)
  double Fd[3][3];
  float F[3][3], dF[3][3], Cf[6], K[3][3];
  deformation_gradient(p0, p1, p2, p3, B, Fd, F);
  direction_gradient(v0, v1, v2, v3, B, dF);
  Scalars s;
  invariants(Fd, Cf, s);
  cofactor(F, K);
  adjoint_terms<GRAD>(F, dF, Cf, K, s, B, V0, m, ebar, h, gp, ge);
}

}  // namespace cm
