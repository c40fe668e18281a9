// FP64 reference ("oracle") for the per-tetrahedron Mooney-Rivlin force of
// Mueller et al., "A hyperelastic model for simulating cells in flow"
// (arXiv 2003.03130).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
// CPU reference the device path is checked against.  It shares no code with
// the device library; only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load it.
//
// What it computes, for every tetrahedron t of a mesh with reference vertex
// positions x and deformed positions y (Sec. "Tetrahedralized cell model"):
//   u = y - x                                   (eq. vertex-displacement)
//   A_ik = u_i^k - u_i^4                         (eq. matrix-A)
//   J_ik = x_i^k - x_i^4,  B = J^{-1}            (Jacobian paragraph)
//   F = I + A B                                  (eq. displacement-derivative)
//   C = F^T F, T_C = tr C, T_C2 = tr(C^2)
//   J = det F, I = T_C J^{-2/3},
//   K = 1/2 (T_C^2 - T_C2) J^{-4/3}              (eqs. invariantJ/I/K)
//   U = mu1/2 (I-3) + mu2/2 (K-3) + kappa/2 (J-1)^2
//                                                (eq. strain-energy-density:mr)
//   mu1 = w mu, mu2 = (1-w) mu                   (Sec. "Theory", last eq.)
//   f_i^a = -V0 dU/du_i^a                        (eq. elastic-force-vertex-0)
// and the node force is the sum over the tetrahedra that share the node; the
// total energy is E = sum_t V0_t U_t, so f = -grad_y E.
//
// Readings where the paper is silent:
//  * V0 = |det J| / 6 (the reference volume of the tetrahedron).
//  * J <= 0: J^{-1/3} is taken as 1 / cbrt(J) with the sign-preserving real
//    cube root, so every power J^{-p/3} is the real power of the real root.
//    Such tetrahedra are counted.
//
// Three independent routes are provided:
//  O1  table path: the chain rule of eq. elastic-force-vertex-1 assembled from
//      the twelve derivative entries listed after the Jacobian paragraph.
//  O2  forward-mode automatic differentiation of U(F(y)) with 12-component
//      dual numbers; it never uses the derivative table.
//  JVP the O1 routine run on 1-component dual numbers: the directional
//      derivative of the forces (a Hessian-vector product of E, up to sign)
//      and of forces/energy with respect to (mu, kappa, w).
//  A second-order check of the Hessian-vector product runs O2 on nested duals.
//
// Plate compression (time-stepped relaxation): the paper compresses cells
// between two plates with a repulsive force that keeps vertices out of the
// plates (Sec. "Simulation setup") and defers the force law and the time
// integration to its supporting information, which is not available.  The
// reading implemented here (parity unpinned by the paper):
//   y_{n+1} = y_n + m (f(y_n) + p(y_n; h_n)),       n = 0 .. N-1,
//   p_z = -k max(0, y_z - h_n)^2 + k max(0, b - y_z)^2 (x, y components 0),
//   F_n = k sum_vertices max(0, y_z - h_n)^2        (force on the top plate),
// with top-plate heights h_n, bottom plate b, penalty k and mobility m.
// Its gradient with respect to (mu, kappa, w) is taken by forward-mode dual
// numbers through all steps (independent of any reverse-mode scheme).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- dual numbers
template <class T, int N>
struct Dual {
  T v;
  T d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = T(0); }
  Dual(double c) : v(c) { for (int i = 0; i < N; ++i) d[i] = T(0); }
};

template <class T, int N>
Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, double c) { return a + Dual<T, N>(c); }
template <class T, int N> Dual<T, N> operator+(double c, const Dual<T, N>& a) { return Dual<T, N>(c) + a; }
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, double c) { return a - Dual<T, N>(c); }
template <class T, int N> Dual<T, N> operator-(double c, const Dual<T, N>& a) { return Dual<T, N>(c) - a; }
template <class T, int N> Dual<T, N> operator*(const Dual<T, N>& a, double c) { return a * Dual<T, N>(c); }
template <class T, int N> Dual<T, N> operator*(double c, const Dual<T, N>& a) { return Dual<T, N>(c) * a; }
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, double c) { return a / Dual<T, N>(c); }
template <class T, int N> Dual<T, N> operator/(double c, const Dual<T, N>& a) { return Dual<T, N>(c) / a; }

// Real (sign-preserving) cube root and its derivative d cbrt(x) = dx / (3 cbrt(x)^2).
inline double real_cbrt(double x) { return std::cbrt(x); }
template <class T, int N>
Dual<T, N> real_cbrt(const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = real_cbrt(a.v);
  T den = T(3.0) * r.v * r.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / den;
  return r;
}

inline double value_of(double a) { return a; }
template <class T, int N> double value_of(const Dual<T, N>& a) { return value_of(a.v); }

// ------------------------------------------------------------- 3x3 helpers
template <class S>
S det3(const S M[3][3]) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
       - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
       + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// adj(M) with M adj(M) = det(M) I.
template <class S>
void adjugate3(const S M[3][3], S R[3][3]) {
  R[0][0] = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  R[0][1] = M[0][2] * M[2][1] - M[0][1] * M[2][2];
  R[0][2] = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  R[1][0] = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  R[1][1] = M[0][0] * M[2][2] - M[0][2] * M[2][0];
  R[1][2] = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  R[2][0] = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  R[2][1] = M[0][1] * M[2][0] - M[0][0] * M[2][1];
  R[2][2] = M[0][0] * M[1][1] - M[0][1] * M[1][0];
}

// Reference data of one tetrahedron: Jacobian J_ik = x_i^k - x_i^4
// (columns k = 1..3 are the tetrahedral coordinate directions),
// B = J^{-1}, V0 = |det J| / 6.  Returns det J.
double reference_tet(const double x[4][3], double B[3][3], double* V0) {
  double Jm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Jm[i][k] = x[k][i] - x[3][i];
  double dJ = det3(Jm);
  double adj[3][3];
  adjugate3(Jm, adj);
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) B[k][j] = adj[k][j] / dJ;
  *V0 = std::fabs(dJ) / 6.0;
  return dJ;
}

// --------------------------------------------------------------- O1: table
// Forces on the 4 vertices of one tetrahedron and its energy density, by the
// chain rule of eq. elastic-force-vertex-1 with the tabulated derivatives.
// S is double or a dual number (positions and parameters may carry tangents).
template <class S>
void o1_tet(const S y[4][3], const double x[4][3], const double B[3][3],
            double V0, const S& mu1, const S& mu2, const S& kappa,
            S f[4][3], S* U_out, S* J_out) {
  // vertex displacements u^a = y^a - x^a
  S u[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) u[a][i] = y[a][i] - x[a][i];
  // A_ik = u_i^k - u_i^4
  S A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) A[i][k] = u[k][i] - u[3][i];
  // F_ij = delta_ij + A_ik B_kj
  S F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S s(i == j ? 1.0 : 0.0);
      for (int k = 0; k < 3; ++k) s = s + A[i][k] * B[k][j];
      F[i][j] = s;
    }
  // C = F^T F
  S C[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      S s(0.0);
      for (int m = 0; m < 3; ++m) s = s + F[m][k] * F[m][l];
      C[k][l] = s;
    }
  S TC = C[0][0] + C[1][1] + C[2][2];
  S TC2(0.0);  // tr(C^2) = C_kl C_lk
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) TC2 = TC2 + C[k][l] * C[l][k];
  S J = det3(F);
  S s = 1.0 / real_cbrt(J);          // J^{-1/3}
  S Jm23 = s * s;                     // J^{-2/3}
  S Jm43 = Jm23 * Jm23;               // J^{-4/3}
  S Jm53 = Jm43 * s;                  // J^{-5/3}
  S Jm73 = Jm53 * Jm23;               // J^{-7/3}
  S I = TC * Jm23;
  S K = 0.5 * (TC * TC - TC2) * Jm43;
  *U_out = 0.5 * mu1 * (I - 3.0) + 0.5 * mu2 * (K - 3.0)
         + 0.5 * kappa * (J - 1.0) * (J - 1.0);
  *J_out = J;

  // The tabulated derivatives.
  S dU_dI = 0.5 * mu1;
  S dI_dTC = Jm23;
  S dU_dK = 0.5 * mu2;
  S dK_dTC = TC * Jm43;
  S dI_dJ = (-2.0 / 3.0) * TC * Jm53;
  S dK_dJ = (-2.0 / 3.0) * (TC * TC - TC2) * Jm73;
  S dU_dJ = kappa * (J - 1.0);
  S dK_dTC2 = -0.5 * Jm43;
  S Finv[3][3];
  {
    S adj[3][3];
    adjugate3(F, adj);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Finv[a][b] = adj[a][b] / J;
  }
  // dT_C/dF_il = 2 F_il; dJ/dF_il = J F^{-1}_li; dT_C2/dF_il = 4 F_ik C_kl.
  S g_TC = dU_dI * dI_dTC + dU_dK * dK_dTC;
  S g_J = dU_dI * dI_dJ + dU_dK * dK_dJ + dU_dJ;
  S g_TC2 = dU_dK * dK_dTC2;
  S P[3][3];  // the bracket of eq. elastic-force-vertex-1, i.e. dU/dF_il
  for (int i = 0; i < 3; ++i)
    for (int l = 0; l < 3; ++l) {
      S dTC_dF = 2.0 * F[i][l];
      S dJ_dF = J * Finv[l][i];
      S dTC2_dF(0.0);
      for (int k = 0; k < 3; ++k) dTC2_dF = dTC2_dF + 4.0 * F[i][k] * C[k][l];
      P[i][l] = g_TC * dTC_dF + g_J * dJ_dF + g_TC2 * dTC2_dF;
    }
  // dF_kl/du_i^a = delta_ki B_ml (delta_ma - delta_4a), vertices a = 1..4,
  // m = 1..3, so f_i^a = -V0 sum_kl P_kl delta_ki sum_m B_ml (delta_ma - delta_4a).
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      S acc(0.0);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          if (k != i) continue;
          double dF = 0.0;
          for (int m = 0; m < 3; ++m)
            dF += B[m][l] * ((m == a ? 1.0 : 0.0) - (a == 3 ? 1.0 : 0.0));
          acc = acc + P[k][l] * dF;
        }
      f[a][i] = -V0 * acc;
    }
}

// ------------------------------------------------------ O2: dual-number AD
// U(F(y)) from the definitions only (eqs. invariantJ/I/K, strain energy),
// with F = D_s B built from the deformed edge vectors (equal to I + A B).
template <class S>
S energy_density_of_F(const S F[3][3], const S& mu1, const S& mu2,
                      const S& kappa) {
  S C[3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      S s(0.0);
      for (int m = 0; m < 3; ++m) s = s + F[m][k] * F[m][l];
      C[k][l] = s;
    }
  S TC = C[0][0] + C[1][1] + C[2][2];
  S TC2(0.0);
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) TC2 = TC2 + C[k][l] * C[l][k];
  S J = det3(F);
  S r = real_cbrt(J);
  S I = TC / (r * r);
  S K = 0.5 * (TC * TC - TC2) / (r * r * r * r);
  return 0.5 * mu1 * (I - 3.0) + 0.5 * mu2 * (K - 3.0)
       + 0.5 * kappa * (J - 1.0) * (J - 1.0);
}

template <class S>
void deformation_gradient_from_positions(const S y[4][3], const double B[3][3],
                                         S F[3][3]) {
  S Ds[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Ds[i][k] = y[k][i] - y[3][i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S s(0.0);
      for (int k = 0; k < 3; ++k) s = s + Ds[i][k] * B[k][j];
      F[i][j] = s;
    }
}

// f = -V0 dU/dy over the 12 vertex coordinates, for a base scalar T
// (double, or Dual<double,1> for the nested second-order check).
template <class T>
void o2_tet(const T yv[4][3], const double B[3][3], double V0, const T& mu1,
            const T& mu2, const T& kappa, T f[4][3], T* U_out) {
  typedef Dual<T, 12> D;
  D y[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      y[a][i] = D(0.0);
      y[a][i].v = yv[a][i];
      y[a][i].d[3 * a + i] = T(1.0);
    }
  D m1(0.0), m2(0.0), ka(0.0);
  m1.v = mu1; m2.v = mu2; ka.v = kappa;
  D F[3][3];
  deformation_gradient_from_positions(y, B, F);
  D U = energy_density_of_F(F, m1, m2, ka);
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) f[a][i] = -V0 * U.d[3 * a + i];
  *U_out = U.v;
}

// ------------------------------------------------------------ mesh drivers
struct View {
  int64_t n_nodes, n_tets;
  const double* x;
  const int32_t* tets;
  const double* B;    // 9 per tet, B[k][j] row-major
  const double* V0;
};

void gather_ref(const View& m, int64_t t, double x[4][3], double B[3][3]) {
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) x[a][i] = m.x[3 * (int64_t)m.tets[4 * t + a] + i];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) B[k][j] = m.B[9 * t + 3 * k + j];
}

bool check_indices(int64_t n_nodes, int64_t n_tets, const int32_t* tets) {
  for (int64_t q = 0; q < 4 * n_tets; ++q)
    if (tets[q] < 0 || tets[q] >= n_nodes) return false;
  return true;
}

// O1 over a whole mesh for any scalar type S (positions and parameters may
// carry tangents); forces accumulated in tetrahedron order.
template <class S>
void o1_mesh(const View& m, const S* y, const S& mu1, const S& mu2,
             const S& kappa, S* f) {
  for (int64_t q = 0; q < 3 * m.n_nodes; ++q) f[q] = S(0.0);
  for (int64_t t = 0; t < m.n_tets; ++t) {
    double xt[4][3], Bt[3][3];
    gather_ref(m, t, xt, Bt);
    S yt[4][3], ft[4][3], U, J;
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) yt[a][i] = y[3 * (int64_t)m.tets[4 * t + a] + i];
    o1_tet<S>(yt, xt, Bt, m.V0[t], mu1, mu2, kappa, ft, &U, &J);
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) {
        S& dst = f[3 * (int64_t)m.tets[4 * t + a] + i];
        dst = dst + ft[a][i];
      }
  }
}

// The plate-compression run for scalar type S; returns F_n in F (n_steps).
template <class S>
void relax_run(const View& m, std::vector<S>& y, const S& mu1, const S& mu2,
               const S& kappa, int n_steps, const double* top, double bottom,
               double k, double mob, S* F) {
  std::vector<S> f(3 * m.n_nodes);
  for (int n = 0; n < n_steps; ++n) {
    o1_mesh<S>(m, y.data(), mu1, mu2, kappa, f.data());
    S Fn(0.0);
    for (int64_t a = 0; a < m.n_nodes; ++a) {
      S& z = y[3 * a + 2];
      S pz(0.0);
      if (value_of(z) > top[n]) {
        S d = z - top[n];
        pz = pz - k * d * d;
        Fn = Fn + k * d * d;
      }
      if (value_of(z) < bottom) {
        S d = bottom - z;
        pz = pz + k * d * d;
      }
      // y_{n+1} = y_n + m (f + p), computed from the old state
      y[3 * a] = y[3 * a] + mob * f[3 * a];
      y[3 * a + 1] = y[3 * a + 1] + mob * f[3 * a + 1];
      y[3 * a + 2] = z + mob * (f[3 * a + 2] + pz);
    }
    F[n] = Fn;
  }
}

}  // namespace

extern "C" {

// Reference inverse edge matrices and volumes, FP64.  Returns 0, or -1 on an
// index out of range, or -2 if some tetrahedron has det J == 0.
int or_prepare(int64_t n_nodes, int64_t n_tets, const double* x,
               const int32_t* tets, double* B, double* V0, double* detJ) {
  if (!check_indices(n_nodes, n_tets, tets)) return -1;
  for (int64_t t = 0; t < n_tets; ++t) {
    double xt[4][3], Bt[3][3];
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) xt[a][i] = x[3 * (int64_t)tets[4 * t + a] + i];
    double d = reference_tet(xt, Bt, &V0[t]);
    if (detJ) detJ[t] = d;
    if (d == 0.0) return -2;
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j) B[9 * t + 3 * k + j] = Bt[k][j];
  }
  return 0;
}

// O1 forces (N x 3, overwritten) and total energy; counts tets with J <= 0.
// Node sums are accumulated in tetrahedron order.
void or_forces_table(int64_t n_nodes, int64_t n_tets, const double* x,
                     const int32_t* tets, const double* B, const double* V0,
                     const double* y, double mu, double kappa, double w,
                     double* f, double* energy, int64_t* n_inverted) {
  View m{n_nodes, n_tets, x, tets, B, V0};
  std::memset(f, 0, sizeof(double) * 3 * n_nodes);
  double mu1 = w * mu, mu2 = (1.0 - w) * mu;
  double E = 0.0;
  int64_t ninv = 0;
  for (int64_t t = 0; t < n_tets; ++t) {
    double xt[4][3], Bt[3][3], yt[4][3], ft[4][3], U, J;
    gather_ref(m, t, xt, Bt);
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) yt[a][i] = y[3 * (int64_t)tets[4 * t + a] + i];
    o1_tet<double>(yt, xt, Bt, V0[t], mu1, mu2, kappa, ft, &U, &J);
    if (!(J > 0.0)) ++ninv;
    E += V0[t] * U;
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) f[3 * (int64_t)tets[4 * t + a] + i] += ft[a][i];
  }
  *energy = E;
  if (n_inverted) *n_inverted = ninv;
}

// O2 forces and energy by dual-number AD of the energy (no derivative table).
void or_forces_ad(int64_t n_nodes, int64_t n_tets, const double* x,
                  const int32_t* tets, const double* B, const double* V0,
                  const double* y, double mu, double kappa, double w,
                  double* f, double* energy) {
  View m{n_nodes, n_tets, x, tets, B, V0};
  std::memset(f, 0, sizeof(double) * 3 * n_nodes);
  double mu1 = w * mu, mu2 = (1.0 - w) * mu;
  double E = 0.0;
  for (int64_t t = 0; t < n_tets; ++t) {
    double xt[4][3], Bt[3][3], yt[4][3], ft[4][3], U;
    gather_ref(m, t, xt, Bt);
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) yt[a][i] = y[3 * (int64_t)tets[4 * t + a] + i];
    o2_tet<double>(yt, Bt, V0[t], mu1, mu2, kappa, ft, &U);
    E += V0[t] * U;
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) f[3 * (int64_t)tets[4 * t + a] + i] += ft[a][i];
  }
  *energy = E;
}

// Directional derivative of the O1 forces and energy:
//   df = d/de f(y + e v; theta + e dtheta) at e = 0, likewise dE.
// v (N x 3) and dtheta (3: dmu, dkappa, dw) may be null (zero direction).
void or_forces_jvp(int64_t n_nodes, int64_t n_tets, const double* x,
                   const int32_t* tets, const double* B, const double* V0,
                   const double* y, const double* v, double mu, double kappa,
                   double w, const double* dtheta, double* df, double* dE) {
  typedef Dual<double, 1> D;
  View m{n_nodes, n_tets, x, tets, B, V0};
  std::memset(df, 0, sizeof(double) * 3 * n_nodes);
  D dmu(mu), dka(kappa), dw(w);
  if (dtheta) { dmu.d[0] = dtheta[0]; dka.d[0] = dtheta[1]; dw.d[0] = dtheta[2]; }
  D mu1 = dw * dmu, mu2 = (1.0 - dw) * dmu;
  double E_t = 0.0;
  for (int64_t t = 0; t < n_tets; ++t) {
    double xt[4][3], Bt[3][3];
    D yt[4][3], ft[4][3], U, J;
    gather_ref(m, t, xt, Bt);
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) {
        int64_t g = 3 * (int64_t)tets[4 * t + a] + i;
        yt[a][i] = D(y[g]);
        yt[a][i].d[0] = v ? v[g] : 0.0;
      }
    o1_tet<D>(yt, xt, Bt, V0[t], mu1, mu2, dka, ft, &U, &J);
    E_t += V0[t] * U.d[0];
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) df[3 * (int64_t)tets[4 * t + a] + i] += ft[a][i].d[0];
  }
  if (dE) *dE = E_t;
}

// Reverse-mode cotangents of L(f, E) with dL/df = fbar (nullable = 0) and
// dL/dE = ebar:
//   ybar = (df/dy)^T fbar + ebar dE/dy = (df/dy) fbar - ebar f
//          (df/dy = -Hessian(E) is symmetric),
//   thetabar_k = fbar . df/dtheta_k + ebar dE/dtheta_k, theta = (mu, kappa, w).
void or_backward(int64_t n_nodes, int64_t n_tets, const double* x,
                 const int32_t* tets, const double* B, const double* V0,
                 const double* y, double mu, double kappa, double w,
                 const double* fbar, double ebar, double* ybar,
                 double* thetabar) {
  std::vector<double> f(3 * n_nodes), df(3 * n_nodes);
  double E, dE;
  or_forces_table(n_nodes, n_tets, x, tets, B, V0, y, mu, kappa, w, f.data(),
                  &E, nullptr);
  if (fbar)
    or_forces_jvp(n_nodes, n_tets, x, tets, B, V0, y, fbar, mu, kappa, w,
                  nullptr, ybar, &dE);
  else
    std::memset(ybar, 0, sizeof(double) * 3 * n_nodes);
  for (int64_t q = 0; q < 3 * n_nodes; ++q) ybar[q] -= ebar * f[q];
  for (int k = 0; k < 3; ++k) {
    double e[3] = {0.0, 0.0, 0.0};
    e[k] = 1.0;
    or_forces_jvp(n_nodes, n_tets, x, tets, B, V0, y, nullptr, mu, kappa, w,
                  e, df.data(), &dE);
    double acc = ebar * dE;
    if (fbar)
      for (int64_t q = 0; q < 3 * n_nodes; ++q) acc += fbar[q] * df[q];
    thetabar[k] = acc;
  }
}

// Second-order cross-check: d/de f(y + e v) by running O2 on nested duals.
void or_forces_jvp_nested(int64_t n_nodes, int64_t n_tets, const double* x,
                          const int32_t* tets, const double* B,
                          const double* V0, const double* y, const double* v,
                          double mu, double kappa, double w, double* df) {
  typedef Dual<double, 1> T;
  (void)x;
  std::memset(df, 0, sizeof(double) * 3 * n_nodes);
  T mu1(w * mu), mu2((1.0 - w) * mu), ka(kappa);
  for (int64_t t = 0; t < n_tets; ++t) {
    double Bt[3][3];
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j) Bt[k][j] = B[9 * t + 3 * k + j];
    T yt[4][3], ft[4][3], U;
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) {
        int64_t g = 3 * (int64_t)tets[4 * t + a] + i;
        yt[a][i] = T(y[g]);
        yt[a][i].d[0] = v[g];
      }
    o2_tet<T>(yt, Bt, V0[t], mu1, mu2, ka, ft, &U);
    for (int a = 0; a < 4; ++a)
      for (int i = 0; i < 3; ++i) df[3 * (int64_t)tets[4 * t + a] + i] += ft[a][i].d[0];
  }
}

// Energy density U(F) from the definitions (used by the physics pins).
double or_energy_density(const double* F9, double mu, double kappa, double w) {
  double F[3][3];
  for (int i = 0; i < 9; ++i) F[i / 3][i % 3] = F9[i];
  double mu1 = w * mu, mu2 = (1.0 - w) * mu, ka = kappa;
  return energy_density_of_F<double>(F, mu1, mu2, ka);
}

// dU/dF assembled from the derivative table (the O1 bracket) for a given F,
// obtained by running O1 on the unit right tetrahedron x^k = e_k, x^4 = 0
// (there B = I, V0 = 1/6 and the forces on vertices 1..3 are -P/6 by column).
void or_stress_table(const double* F9, double mu, double kappa, double w,
                     double* P9) {
  double x[4][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 0, 0}};
  double B[3][3], V0;
  reference_tet(x, B, &V0);
  double y[4][3];
  for (int a = 0; a < 4; ++a)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int j = 0; j < 3; ++j) s += F9[3 * i + j] * x[a][j];
      y[a][i] = s;
    }
  double f[4][3], U, J;
  o1_tet<double>(y, x, B, V0, w * mu, (1.0 - w) * mu, kappa, f, &U, &J);
  // f_i^a = -V0 P_il B_al for a = 1..3 and B = I: P_ia = -f_i^a / V0.
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) P9[3 * i + a] = -f[a][i] / V0;
}

// Plate compression of one cell (see the header): F_out[n] for n < n_steps
// and the final positions (y_final, nullable).
void or_relax_forward(int64_t n_nodes, int64_t n_tets, const double* x,
                      const int32_t* tets, const double* B, const double* V0,
                      const double* y0, double mu, double kappa, double w,
                      int n_steps, const double* top, double bottom,
                      double k_plate, double mobility, double* F_out,
                      double* y_final) {
  View m{n_nodes, n_tets, x, tets, B, V0};
  std::vector<double> y(y0, y0 + 3 * n_nodes);
  relax_run<double>(m, y, w * mu, (1.0 - w) * mu, kappa, n_steps, top, bottom,
                    k_plate, mobility, F_out);
  if (y_final) std::memcpy(y_final, y.data(), sizeof(double) * 3 * n_nodes);
}

// Loss L = scale * sum_n (F_n - F_target[n])^2 of the plate compression and
// dL/d(mu, kappa, w) by forward-mode duals (three tangents) through all
// steps.  F_out (nullable) receives F_n.
void or_relax_grad(int64_t n_nodes, int64_t n_tets, const double* x,
                   const int32_t* tets, const double* B, const double* V0,
                   const double* y0, double mu, double kappa, double w,
                   int n_steps, const double* top, double bottom,
                   double k_plate, double mobility, const double* F_target,
                   double scale, double* loss, double* dtheta, double* F_out) {
  typedef Dual<double, 3> D;
  View m{n_nodes, n_tets, x, tets, B, V0};
  std::vector<D> y(3 * n_nodes);
  for (int64_t q = 0; q < 3 * n_nodes; ++q) y[q] = D(y0[q]);
  D dmu(mu), dka(kappa), dw(w);
  dmu.d[0] = 1.0;
  dka.d[1] = 1.0;
  dw.d[2] = 1.0;
  std::vector<D> F(n_steps);
  relax_run<D>(m, y, dw * dmu, (1.0 - dw) * dmu, dka, n_steps, top, bottom,
               k_plate, mobility, F.data());
  double L = 0.0, g[3] = {0.0, 0.0, 0.0};
  for (int n = 0; n < n_steps; ++n) {
    const double r = F[n].v - F_target[n];
    L += scale * r * r;
    for (int k = 0; k < 3; ++k) g[k] += 2.0 * scale * r * F[n].d[k];
    if (F_out) F_out[n] = F[n].v;
  }
  *loss = L;
  for (int k = 0; k < 3; ++k) dtheta[k] = g[k];
}

// Timing mode of the CPU baseline: the forward (O1) and the backward of every
// cell c in [c0, c1) of a batch, the cells distributed over OpenMP threads
// (a build with -fopenmp; without it the loop runs on one thread).  Per-cell
// arrays are concatenated: node_off / tet_off are CSR offsets (n_cells + 1),
// tets are cell-local, B / V0 come from or_prepare on each cell, theta holds
// (mu, kappa, w) per cell; f, ybar (3 per node), energy (1 per cell) and
// thetabar (3 per cell) are outputs.  Each cell runs or_forces_table and
// or_backward unchanged.
void or_batch_fwd_bwd(int64_t c0, int64_t c1, const int64_t* node_off,
                      const int64_t* tet_off, const double* x,
                      const int32_t* tets, const double* B, const double* V0,
                      const double* y, const double* theta, const double* fbar,
                      const double* ebar, double* f, double* energy,
                      double* ybar, double* thetabar) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t n0 = node_off[c], n = node_off[c + 1] - n0;
    const int64_t t0 = tet_off[c], m = tet_off[c + 1] - t0;
    const double* th = theta + 3 * c;
    or_forces_table(n, m, x + 3 * n0, tets + 4 * t0, B + 9 * t0, V0 + t0,
                    y + 3 * n0, th[0], th[1], th[2], f + 3 * n0, energy + c,
                    nullptr);
    or_backward(n, m, x + 3 * n0, tets + 4 * t0, B + 9 * t0, V0 + t0,
                y + 3 * n0, th[0], th[1], th[2], fbar + 3 * n0, ebar[c],
                ybar + 3 * n0, thetabar + 3 * c);
  }
}

// Threads of the timing mode: sets the OpenMP thread count when n > 0 and
// returns the count in effect (1 without OpenMP).
int or_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // extern "C"
