// lbmhd_oracle.cpp -- plain FP64 CPU oracle for the 2D lattice Boltzmann MHD
// update with a local Smagorinsky-MHD closure (Flint & Vahala, "Lattice
// Boltzmann Large Eddy Simulation Model of MHD", arXiv:1607.08675).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
// reference the GPU library is checked against.  Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
// no code, header, table or constant with the GPU library: every lattice
// quantity below is built here from the paper's definitions.
//
// What it follows, step by step (paper section / equation):
//   * lattices: D2Q9 velocities c_i and D2Q5 velocities C_k (Sec. 3, the
//     explicit component lists after the T_m matrix);
//   * equilibria f_i^eq(rho,u,B) and g_k^eq(u,B) (Sec. 1.2 / Sec. 3, the
//     D2Q9 and D2Q5 relaxation distributions);
//   * moment transform M = T f with the nine rows of eq. FluidTMatrix, T_m of
//     eq. MagTMatrix (Sec. 3);
//   * collision in moment space with diagonal rates s_i and a single magnetic
//     rate s_m (Sec. 3, text after the velocity lists), moments 0..2 being the
//     collision invariants;
//   * rates from the transport coefficients nu = 1/(3 s_3) - 1/6 = 1/(3 s_4) - 1/6
//     and eta = 1/(3 s_m) - 1/6 (Sec. 4.3);
//   * the Smagorinsky closures nu_T = C_Sv Delta^2 |S| and eta_T = C_Sb Delta^2 |j|
//     (eqs. SmagorinskyClosure, SmagorinskyMHDClosureV/B), with the
//     strain read from the site's own non-equilibrium second moments (the
//     Sec. 1.2 relation between sum_i c_a c_b f^(1) and the strain) and the
//     current read from the non-equilibrium first moments of g;
//   * the cross-helicity closure (les = 4, or 6 together with the kinetic
//     closure; eqs. CHClosureV/B): nu_t = C_Sv Delta^2 |S^v : S^b|^(1/2) and
//     eta_t = C_Sb Delta^2 sgn(j . omega) |j . omega|^(1/2), where S^v is the
//     strain of u, S^b the symmetrised gradient of B and omega the vorticity;
//   * collide-then-stream with unit time step (the discrete LB update of
//     Sec. 1.2): f_i(x + c_i, t+1) = f_i*(x, t).
//
//   * kinetic LES closure (les = 2, or 3 together with the Smagorinsky
//     closure; Sec. 4.1): the relaxation targets are the
//     filtered equilibrium moments M^eq(filtered conserved moments) + the
//     Delta^2 terms, obtained by applying the filter-width expansion of
//     products (eq. FilterExampleSmall) and of ratios (eq. FilterExampleLarge)
//     to every quadratic term of eqs. KinMomentEq and MagMomentEq, as the paper
//     does for M_3 in eq. DeltaEqEx; linear terms are unchanged.
//
// Readings where the paper is silent or garbled:
//   * weights w = (4/9, 1/9 x4, 1/36 x4), w' = (1/3, 1/6 x4): the only ones
//     for which T f^eq reproduces the printed equilibrium moment table
//     (eq. KinMomentEq) and T_m g^eq reproduces eq. MagMomentEq;
//   * the equilibrium magnetic moments are read with u, not rho*u (the form
//     printed for the D2Q5 equilibrium and for the final induction equation);
//   * closure: tau = tau0 + 3 nu_T solved self-consistently with the strain
//     estimated from pre-collision non-equilibrium moments relaxed with that
//     same tau, giving tau = (tau0 + sqrt(tau0^2 + 18 C_S Delta^2 Q / rho)) / 2
//     with Q = sqrt((M4 - M4eq)^2 + 4 (M3 - M3eq)^2); likewise
//     tau_m = (tau_m0 + sqrt(tau_m0^2 + 36 C_S Delta^2 |A|)) / 2 with
//     A = (N_y1 - N_y1^eq) - (N_x2 - N_x2^eq), with C_Sv in tau and C_Sb
//     in tau_m (cs and csb of the parameters);
//   * derivative of |.| and of the norm Q is taken as 0 where the argument is
//     exactly 0 (tangent-linear mode only);
//   * kinetic closure: the lattice sites carry the filtered fields, and the
//     gradients in the Delta^2 terms are the isotropic D2Q9 differences
//     d_a X(x) = 3 sum_i w_i c_ia X(x + c_i) of the pre-collision rho, rho u, B;
//     the relaxation times stay tau0 and tau_m0;
//   * cross-helicity closure: S^v from the non-equilibrium M3, M4 as for the
//     Smagorinsky closure; S^b and j from the non-equilibrium first-moment
//     tensor of g, Lambda_ab = sum_k C_ka g_kb ~ -(tau_m / 3) d_a B_b (its
//     equilibrium is antisymmetric, so the symmetric part carries d_a B_b
//     alone); only the traceless parts of S^v and S^b enter the contraction;
//     omega = d_x u_y - d_y u_x with d_a u_b = (d_a j_b - u_b d_a rho) / rho
//     from the isotropic lattice differences of the pre-collision rho and j;
//     tau = tau0 + 3 nu_t and tau_m = tau_m0 + 3 eta_t solved self-consistently
//     (each a cubic in the square root of the relaxation time, largest root);
//     where backscatter (eta_t < 0) would make the total resistivity
//     eta + eta_t negative, it is clipped at zero, tau_m = 1/2.
//
// State layout: 19 planes of nx*ny doubles, [plane][y][x] with x fastest.
// Planes 0..8 hold f_0..f_8, planes 9..13 hold the x component of g_0..g_4,
// planes 14..18 the y component.  The state is the pre-collision population
// at integer time t (the paper's update order).

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <utility>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- lattices
// D2Q9 and D2Q5 velocity components exactly as listed in Sec. 3.
const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const int MX[5] = {0, 1, 0, -1, 0};
const int MY[5] = {0, 0, 1, 0, -1};

double weight9(int i) {
  int c2 = CX[i] * CX[i] + CY[i] * CY[i];
  return c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
}
double weight5(int k) {
  int c2 = MX[k] * MX[k] + MY[k] * MY[k];
  return c2 == 0 ? 1.0 / 3.0 : 1.0 / 6.0;
}

// Row r of the fluid transform T (eq. FluidTMatrix), as the polynomial in
// (c_x, c_y) the paper gives for that row.
double trow(int r, int i) {
  double cx = CX[i], cy = CY[i];
  double cx2 = cx * cx, cy2 = cy * cy;
  switch (r) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cx * cy;
    case 4: return cx2 - cy2;
    case 5: return 3.0 * cx * cy2 - 2.0 * cx;
    case 6: return 3.0 * cy * cx2 - 2.0 * cy;
    case 7: return 4.0 - 9.0 * (cx2 + cy2 - 2.0 * cx2 * cy2);
    case 8: return 4.0 - 4.0 * (cx2 + cy2) + 3.0 * cx2 * cy2;
  }
  return 0.0;
}
// Row r of the magnetic transform T_m (eq. MagTMatrix).
double tmrow(int r, int k) {
  double cx = MX[k], cy = MY[k];
  switch (r) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cx * cx;
    case 4: return cy * cy;
  }
  return 0.0;
}

struct Tables {
  double T[9][9];
  double Tinv[9][9];
  double Tm[5][5];
  double Tminv[5][5];
  Tables() {
    for (int r = 0; r < 9; ++r)
      for (int i = 0; i < 9; ++i) T[r][i] = trow(r, i);
    for (int r = 0; r < 5; ++r)
      for (int k = 0; k < 5; ++k) Tm[r][k] = tmrow(r, k);
    // T_m^-1 by Gauss-Jordan elimination with partial pivoting.
    double a[5][10];
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 10; ++c) a[r][c] = c < 5 ? Tm[r][c] : (c - 5 == r ? 1.0 : 0.0);
    for (int c = 0; c < 5; ++c) {
      int piv = c;
      for (int r = c + 1; r < 5; ++r)
        if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
      for (int k = 0; k < 10; ++k) std::swap(a[c][k], a[piv][k]);
      const double d = a[c][c];
      for (int k = 0; k < 10; ++k) a[c][k] /= d;
      for (int r = 0; r < 5; ++r)
        if (r != c) {
          const double m = a[r][c];
          for (int k = 0; k < 10; ++k) a[r][k] -= m * a[c][k];
        }
    }
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) Tminv[r][c] = a[r][5 + c];
    // The rows of T are mutually orthogonal (checked by the tests), so
    // T^-1 = T^T diag(1 / |row|^2).
    for (int r = 0; r < 9; ++r) {
      double n2 = 0.0;
      for (int i = 0; i < 9; ++i) n2 += T[r][i] * T[r][i];
      for (int i = 0; i < 9; ++i) Tinv[i][r] = T[r][i] / n2;
    }
  }
};
const Tables& tables() {
  static const Tables t;
  return t;
}

// ------------------------------------------------------------ dual numbers
// Forward-mode dual number with ND tangent directions: the tangent-linear
// reference.  Only the operations the update uses are defined.
constexpr int ND = 16;
struct Dual {
  double v;
  double d[ND];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }
};
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) {
  Dual r(a.v * b);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b;
  return r;
}
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }

inline double root(double x) { return std::sqrt(x); }
inline Dual root(const Dual& x) {
  Dual r(std::sqrt(x.v));
  double g = r.v > 0.0 ? 0.5 / r.v : 0.0;  // kink reading at exactly 0
  for (int k = 0; k < ND; ++k) r.d[k] = g * x.d[k];
  return r;
}
inline double magnitude(double x) { return std::fabs(x); }
inline Dual magnitude(const Dual& x) {
  Dual r(std::fabs(x.v));
  double g = x.v > 0.0 ? 1.0 : (x.v < 0.0 ? -1.0 : 0.0);
  for (int k = 0; k < ND; ++k) r.d[k] = g * x.d[k];
  return r;
}

}  // namespace

// ---------------------------------------------------------------- interface
extern "C" {

typedef struct {
  int32_t nx, ny;
  double nu, eta;          // shear viscosity and resistivity, lattice units
  double s5, s6, s7, s8;   // rates of the non-hydrodynamic moments
  int32_t les;             // bit 0: Smagorinsky-MHD closure; bit 1: kinetic
                           // closure (filtered equilibria); bit 2: cross-
                           // helicity closure (not with bit 0); 0: none
  double cs, csb;          // closure constants: C_Sv (fluid) and C_Sb (field)
  double delta;            // filter width Delta
} orc_params;

enum { ORC_NPOP = 19, ORC_NDIAG = 14, ORC_ND = ND };

}  // extern "C"

namespace {

template <class R>
void equilibrium(R rho, R ux, R uy, R bx, R by, R feq[9], R geq[10]) {
  // D2Q9 equilibrium with the Maxwell-stress terms, and the D2Q5 vector
  // equilibrium (Sec. 3, the two relaxation distributions).
  R u2 = ux * ux + uy * uy;
  R b2 = bx * bx + by * by;
  for (int i = 0; i < 9; ++i) {
    double w = weight9(i);
    R cu = ux * double(CX[i]) + uy * double(CY[i]);
    R cb = bx * double(CX[i]) + by * double(CY[i]);
    double c2 = double(CX[i] * CX[i] + CY[i] * CY[i]);
    feq[i] = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2) +
             4.5 * w * (0.5 * b2 * c2 - cb * cb);
  }
  for (int k = 0; k < 5; ++k) {
    double w = weight5(k);
    R cu = ux * double(MX[k]) + uy * double(MY[k]);
    R cb = bx * double(MX[k]) + by * double(MY[k]);
    geq[k] = w * (bx + 3.0 * (cu * bx - cb * ux));
    geq[5 + k] = w * (by + 3.0 * (cu * by - cb * uy));
  }
}

template <class R>
void moment_equilibria(R rho, R jx, R jy, R bx, R by, R meq[9], R neq[10]) {
  // Equilibrium moments of eq. KinMomentEq (written with rho u as printed)
  // and eq. MagMomentEq (read with u = (rho u) / rho).
  R jsq = (jx * jx + jy * jy) / rho;
  meq[0] = rho;
  meq[1] = jx;
  meq[2] = jy;
  meq[3] = jx * jy / rho - bx * by;
  meq[4] = (jx * jx - jy * jy) / rho - bx * bx + by * by;
  meq[5] = -jx;
  meq[6] = -jy;
  meq[7] = -3.0 * jsq;
  meq[8] = (5.0 / 3.0) * rho - 3.0 * jsq;
  R ux = jx / rho, uy = jy / rho;
  R b[2] = {bx, by};
  R u[2] = {ux, uy};
  for (int a = 0; a < 2; ++a) {
    neq[5 * a + 0] = b[a];
    neq[5 * a + 1] = ux * b[a] - u[a] * bx;
    neq[5 * a + 2] = uy * b[a] - u[a] * by;
    neq[5 * a + 3] = b[a] / 3.0;
    neq[5 * a + 4] = b[a] / 3.0;
  }
}

// Filter-width expansion of a filtered product (eq. FilterExampleSmall):
// (XY)bar - Xbar Ybar = Delta^2 / 12 d_b X d_b Y + O(Delta^4).
template <class R>
R filtered_product_term(double d2, const R dX[2], const R dY[2]) {
  return (d2 / 12.0) * (dX[0] * dY[0] + dX[1] * dY[1]);
}

// Filter-width expansion of a filtered ratio (eq. FilterExampleLarge):
// (XY/Z)bar - Xbar Ybar / Zbar = Delta^2 / (12 Z) [ d_b X d_b Y
//   - (d_b Z / Z) (X d_b Y + Y d_b X - X Y d_b Z / Z) ] + O(Delta^4).
template <class R>
R filtered_ratio_term(double d2, R X, R Y, R Z, const R dX[2], const R dY[2], const R dZ[2]) {
  R acc = 0.0;
  for (int b = 0; b < 2; ++b)
    acc = acc + dX[b] * dY[b] - (dZ[b] / Z) * (X * dY[b] + Y * dX[b] - X * Y * dZ[b] / Z);
  return (d2 / 12.0) / Z * acc;
}

// Delta^2 parts of the filtered equilibrium moments: each quadratic term of
// eqs. KinMomentEq and MagMomentEq (rho u written as j, u = j / rho) replaced
// by its expansion; the linear terms have none.  grad holds d_x, d_y of
// (rho, j_x, j_y, B_x, B_y).
template <class R>
void filtered_moment_corrections(double d2, R rho, R jx, R jy, R bx, R by, const R grad[10],
                                 R dmeq[9], R dneq[10]) {
  const R* gr = grad + 0;
  const R* gjx = grad + 2;
  const R* gjy = grad + 4;
  const R* gbx = grad + 6;
  const R* gby = grad + 8;
  for (int i = 0; i < 9; ++i) dmeq[i] = 0.0;
  for (int i = 0; i < 10; ++i) dneq[i] = 0.0;
  const R jxjx = filtered_ratio_term(d2, jx, jx, rho, gjx, gjx, gr);
  const R jyjy = filtered_ratio_term(d2, jy, jy, rho, gjy, gjy, gr);
  // M_3 = jx jy / rho - Bx By
  dmeq[3] = filtered_ratio_term(d2, jx, jy, rho, gjx, gjy, gr) - filtered_product_term(d2, gbx, gby);
  // M_4 = (jx^2 - jy^2) / rho - Bx^2 + By^2
  dmeq[4] = jxjx - jyjy - filtered_product_term(d2, gbx, gbx) + filtered_product_term(d2, gby, gby);
  // M_7 = -3 (jx^2 + jy^2) / rho,  M_8 = 5 rho / 3 - 3 (jx^2 + jy^2) / rho
  dmeq[7] = -3.0 * (jxjx + jyjy);
  dmeq[8] = -3.0 * (jxjx + jyjy);
  // N_a1 = u_x B_a - u_a B_x,  N_a2 = u_y B_a - u_a B_y
  const R b[2] = {bx, by};
  const R j[2] = {jx, jy};
  const R* gb[2] = {gbx, gby};
  const R* gj[2] = {gjx, gjy};
  for (int a = 0; a < 2; ++a) {
    dneq[5 * a + 1] = filtered_ratio_term(d2, jx, b[a], rho, gjx, gb[a], gr) -
                      filtered_ratio_term(d2, j[a], bx, rho, gj[a], gbx, gr);
    dneq[5 * a + 2] = filtered_ratio_term(d2, jy, b[a], rho, gjy, gb[a], gr) -
                      filtered_ratio_term(d2, j[a], by, rho, gj[a], gby, gr);
  }
}

// Largest real root of t^3 - p t - q = 0 for p > 0: the trigonometric form
// where the cubic has three real roots, Cardano's formula where it has one
// (q > 2 (p/3)^(3/2)).  Returns -1 when no root is positive (q below
// -2 (p/3)^(3/2)).
double largest_cubic_root(double p, double q) {
  const double r = std::sqrt(p / 3.0);
  const double h = q / (2.0 * r * r * r);
  if (h > 1.0) {
    const double d = std::sqrt(0.25 * q * q - r * r * r * r * r * r);
    return std::cbrt(0.5 * q + d) + std::cbrt(0.5 * q - d);
  }
  if (h < -1.0) return -1.0;
  return 2.0 * r * std::cos(std::acos(h) / 3.0);
}

// The same root in R: one Newton step from the FP64 root t keeps its value and
// gives dual numbers the implicit-function derivative (t dp + dq) / (3 t^2 - p).
template <class R>
R cubic_root_in(R p, R q, double t) {
  return t - (t * t * t - p * t - q) / (3.0 * t * t - p);
}

inline double sign_of(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

struct Rates {
  double tau0, taum0;   // constant relaxation times 1/s_3 and 1/s_m
  double s[9];          // s_0..s_8; s_3, s_4 replaced by the closure
};

Rates make_rates(const orc_params& p) {
  Rates r;
  // nu = 1/(3 s_3) - 1/6 and eta = 1/(3 s_m) - 1/6 (Sec. 4.3).
  r.tau0 = 3.0 * p.nu + 0.5;
  r.taum0 = 3.0 * p.eta + 0.5;
  r.s[0] = r.s[1] = r.s[2] = 0.0;  // invariants: M - M^eq vanishes there
  r.s[3] = r.s[4] = 1.0 / r.tau0;
  r.s[5] = p.s5;
  r.s[6] = p.s6;
  r.s[7] = p.s7;
  r.s[8] = p.s8;
  return r;
}

// One collision at one site.  f[9] and g[10] are overwritten with the
// post-collision populations.  tau_out / taum_out receive the relaxation
// times actually used.
template <class R>
void collide_site(const orc_params& p, const Rates& rt, R cs, R csb, R f[9], R g[10],
                  double* tau_out, double* taum_out, const R* grad = nullptr) {
  const Tables& tb = tables();
  // Conserved moments (Sec. 3, text after the kinetic equations).
  R rho = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho = rho + f[i];
    jx = jx + double(CX[i]) * f[i];
    jy = jy + double(CY[i]) * f[i];
  }
  for (int k = 0; k < 5; ++k) {
    bx = bx + g[k];
    by = by + g[5 + k];
  }
  // Moments M = T f, N = T_m g.
  R M[9], N[10];
  for (int r = 0; r < 9; ++r) {
    R acc = 0.0;
    for (int i = 0; i < 9; ++i) acc = acc + tb.T[r][i] * f[i];
    M[r] = acc;
  }
  for (int a = 0; a < 2; ++a)
    for (int r = 0; r < 5; ++r) {
      R acc = 0.0;
      for (int k = 0; k < 5; ++k) acc = acc + tb.Tm[r][k] * g[5 * a + k];
      N[5 * a + r] = acc;
    }
  R meq[9], neq[10];
  moment_equilibria(rho, jx, jy, bx, by, meq, neq);

  // Kinetic LES closure: relax toward the filtered equilibrium moments.
  R dneq[10];
  for (int q = 0; q < 10; ++q) dneq[q] = 0.0;
  if (p.les & 2) {
    R dmeq[9];
    filtered_moment_corrections(p.delta * p.delta, rho, jx, jy, bx, by, grad, dmeq, dneq);
    for (int r = 0; r < 9; ++r) meq[r] = meq[r] + dmeq[r];
    for (int q = 0; q < 10; ++q) neq[q] = neq[q] + dneq[q];
  }

  // Smagorinsky closure.  With the kinetic closure as well (les = 3) the
  // non-equilibrium moments are taken relative to the filtered equilibrium:
  // the paper's first-order moment M3^(1) is the strain term plus M3^(Delta).
  R tau = rt.tau0, taum = rt.taum0;
  if (p.les & 1) {
    double d2 = p.delta * p.delta;
    // Fluid: |S| = 3 Q / (2 rho tau) from the non-equilibrium M3, M4;
    // tau = tau0 + 3 C_S Delta^2 |S| solved for tau.
    R n3 = M[3] - meq[3], n4 = M[4] - meq[4];
    R Q = root(n4 * n4 + 4.0 * n3 * n3);
    tau = 0.5 * (rt.tau0 + root(rt.tau0 * rt.tau0 + 18.0 * d2 * cs * Q / rho));
    // Magnetic: j_z = -3 A / tau_m from the antisymmetric part of the
    // non-equilibrium first-moment tensor of g; tau_m = tau_m0 + 3 C_S Delta^2 |j|.
    R A = (N[5 + 1] - neq[5 + 1]) - (N[0 + 2] - neq[0 + 2]);
    taum = 0.5 * (rt.taum0 + root(rt.taum0 * rt.taum0 + 36.0 * d2 * csb * magnitude(A)));
  }
  // Cross-helicity closure (eqs. CHClosureV/B): C_Sv in nu_t, C_Sb in eta_t.
  if (p.les & 4) {
    double d2 = p.delta * p.delta;
    // Traceless strains: S^v_xx - S^v_yy = -3 n4 / (2 rho tau), S^v_xy =
    // -3 n3 / (2 rho tau); S^b_xx - S^b_yy = -3 (L_xx - L_yy) / tau_m,
    // S^b_xy = -3 (L_xy + L_yx) / (2 tau_m), L = non-equilibrium Lambda.
    // For traceless symmetric 2x2 tensors S^v : S^b = (1/2) (S^v_xx - S^v_yy)
    // (S^b_xx - S^b_yy) + 2 S^v_xy S^b_xy = 9 P / (4 rho tau tau_m) with
    // P = n4 (L_xx - L_yy) + 2 n3 (L_xy + L_yx).
    R n3 = M[3] - meq[3], n4 = M[4] - meq[4];
    R dL = (N[0 + 1] - neq[0 + 1]) - (N[5 + 2] - neq[5 + 2]);
    R sL = (N[5 + 1] - neq[5 + 1]) + (N[0 + 2] - neq[0 + 2]);
    R P = n4 * dL + 2.0 * n3 * sL;
    // j_z = -3 A / tau_m (as for the Smagorinsky closure) and the vorticity
    // from the lattice gradients: grad = (d_x rho, d_y rho, d_x j_x, d_y j_x,
    // d_x j_y, d_y j_y, ...).
    R A = (N[5 + 1] - neq[5 + 1]) - (N[0 + 2] - neq[0 + 2]);
    R ux = jx / rho, uy = jy / rho;
    R omega = ((grad[4] - uy * grad[0]) - (grad[3] - ux * grad[1])) / rho;
    // tau_m = tau_m0 + 3 eta_t with j . omega = -3 A omega / tau_m: for
    // t = sqrt(tau_m), t^3 - tau_m0 t - qb = 0 with
    // qb = -3 sqrt(3) C_S Delta^2 sgn(A omega) |A omega|^(1/2).
    R X = A * omega;
    R qb = -3.0 * std::sqrt(3.0) * d2 * csb * sign_of(value(X)) * root(magnitude(X));
    const double tm = largest_cubic_root(rt.taum0, value(qb));
    if (tm < std::sqrt(0.5)) {
      taum = R(0.5);  // eta + eta_t clipped at zero
    } else {
      R t = cubic_root_in(R(rt.taum0), qb, tm);
      taum = t * t;
    }
    // tau = tau0 + 3 nu_t, nu_t = C_S Delta^2 (9 |P| / (4 rho tau tau_m))^(1/2):
    // for t = sqrt(tau), t^3 - tau0 t - qv = 0, qv = (9/2) C_S Delta^2 (|P| / (rho tau_m))^(1/2).
    R qv = 4.5 * d2 * cs * root(magnitude(P) / (rho * taum));
    R t = cubic_root_in(R(rt.tau0), qv, largest_cubic_root(rt.tau0, value(qv)));
    tau = t * t;
  }
  if (tau_out) *tau_out = value(tau);
  if (taum_out) *taum_out = value(taum);

  // Relax in moment space: M*_r = M_r - s_r (M_r - M_r^eq).
  R s[9];
  for (int r = 0; r < 9; ++r) s[r] = R(rt.s[r]);
  s[3] = 1.0 / tau;
  s[4] = 1.0 / tau;
  R Mstar[9];
  for (int r = 0; r < 9; ++r) Mstar[r] = M[r] - s[r] * (M[r] - meq[r]);
  // Back to distribution space: f* = T^-1 M*.
  for (int i = 0; i < 9; ++i) {
    R acc = 0.0;
    for (int r = 0; r < 9; ++r) acc = acc + tb.Tinv[i][r] * Mstar[r];
    f[i] = acc;
  }
  // Magnetic: single relaxation toward g^eq(u, B) (plus, for the kinetic
  // closure, T_m^-1 of the Delta^2 parts of the equilibrium moments).
  R feq_unused[9], geq[10];
  equilibrium(rho, jx / rho, jy / rho, bx, by, feq_unused, geq);
  if (p.les & 2)
    for (int a = 0; a < 2; ++a)
      for (int k = 0; k < 5; ++k) {
        R acc = 0.0;
        for (int r = 0; r < 5; ++r) acc = acc + tb.Tminv[k][r] * dneq[5 * a + r];
        geq[5 * a + k] = geq[5 * a + k] + acc;
      }
  R sm = 1.0 / taum;
  for (int q = 0; q < 10; ++q) g[q] = g[q] - sm * (g[q] - geq[q]);
}

inline int64_t wrap(int64_t a, int64_t n) { return ((a % n) + n) % n; }

bool valid(const orc_params* p) {
  return p && p->nx >= 2 && p->ny >= 2 && p->nu > 0.0 && p->eta > 0.0 && p->les >= 0 &&
         p->les <= 6 && !((p->les & 1) && (p->les & 4));
}

// d_x and d_y of (rho, j_x, j_y, B_x, B_y) at every site: the isotropic D2Q9
// difference d_a X(x) = 3 sum_i w_i c_ia X(x + c_i), periodic.  grad is 10
// planes of n.
template <class R>
void lattice_gradients(const orc_params& p, const R* st, std::vector<R>& grad) {
  const int64_t nx = p.nx, ny = p.ny, n = nx * ny;
  std::vector<R> mac(5 * n);
  for (int64_t s = 0; s < n; ++s) {
    R rho = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
    for (int i = 0; i < 9; ++i) {
      rho = rho + st[i * n + s];
      jx = jx + double(CX[i]) * st[i * n + s];
      jy = jy + double(CY[i]) * st[i * n + s];
    }
    for (int k = 0; k < 5; ++k) {
      bx = bx + st[(9 + k) * n + s];
      by = by + st[(14 + k) * n + s];
    }
    mac[s] = rho;
    mac[n + s] = jx;
    mac[2 * n + s] = jy;
    mac[3 * n + s] = bx;
    mac[4 * n + s] = by;
  }
  grad.assign(10 * n, R(0.0));
  for (int64_t y = 0; y < ny; ++y)
    for (int64_t x = 0; x < nx; ++x) {
      const int64_t s = y * nx + x;
      for (int i = 1; i < 9; ++i) {
        const int64_t t = wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx);
        for (int m = 0; m < 5; ++m) {
          grad[(2 * m) * n + s] = grad[(2 * m) * n + s] + 3.0 * weight9(i) * double(CX[i]) * mac[m * n + t];
          grad[(2 * m + 1) * n + s] =
              grad[(2 * m + 1) * n + s] + 3.0 * weight9(i) * double(CY[i]) * mac[m * n + t];
        }
      }
    }
}

template <class R>
void collide_all(const orc_params& p, R* st, R cs, R csb, double* tau_out, double* taum_out) {
  const int64_t n = int64_t(p.nx) * p.ny;
  const Rates rt = make_rates(p);
  std::vector<R> grad;
  const bool stencil = (p.les & 6) != 0;
  if (stencil) lattice_gradients(p, st, grad);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; ++s) {
    R f[9], g[10], gs[10];
    for (int i = 0; i < 9; ++i) f[i] = st[i * n + s];
    for (int q = 0; q < 10; ++q) g[q] = st[(9 + q) * n + s];
    if (stencil)
      for (int m = 0; m < 10; ++m) gs[m] = grad[m * n + s];
    collide_site(p, rt, cs, csb, f, g, tau_out ? tau_out + s : nullptr,
                 taum_out ? taum_out + s : nullptr, stencil ? gs : nullptr);
    for (int i = 0; i < 9; ++i) st[i * n + s] = f[i];
    for (int q = 0; q < 10; ++q) st[(9 + q) * n + s] = g[q];
  }
}

// Streaming: population i at x moves to x + c_i (periodic).
template <class R>
void stream_all(const orc_params& p, const R* in, R* out) {
  const int64_t nx = p.nx, ny = p.ny, n = nx * ny;
#pragma omp parallel for schedule(static)
  for (int64_t y = 0; y < ny; ++y)
    for (int64_t x = 0; x < nx; ++x) {
      for (int i = 0; i < 9; ++i) {
        int64_t xd = wrap(x + CX[i], nx), yd = wrap(y + CY[i], ny);
        out[i * n + yd * nx + xd] = in[i * n + y * nx + x];
      }
      for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 5; ++k) {
          int64_t xd = wrap(x + MX[k], nx), yd = wrap(y + MY[k], ny);
          int plane = 9 + 5 * a + k;
          out[plane * n + yd * nx + xd] = in[plane * n + y * nx + x];
        }
    }
}

template <class R>
void init_all(const orc_params& p, const R* rho, const R* ux, const R* uy, const R* bx,
              const R* by, R* st) {
  const int64_t n = int64_t(p.nx) * p.ny;
  for (int64_t s = 0; s < n; ++s) {
    R feq[9], geq[10];
    equilibrium(rho[s], ux[s], uy[s], bx[s], by[s], feq, geq);
    for (int i = 0; i < 9; ++i) st[i * n + s] = feq[i];
    for (int q = 0; q < 10; ++q) st[(9 + q) * n + s] = geq[q];
  }
}

// Total energy sum_x (|rho u|^2 / (2 rho) + |B|^2 / 2).
template <class R>
R energy_all(const orc_params& p, const R* st) {
  const int64_t n = int64_t(p.nx) * p.ny;
  R e = 0.0;
  for (int64_t s = 0; s < n; ++s) {
    R rho = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
    for (int i = 0; i < 9; ++i) {
      R f = st[i * n + s];
      rho = rho + f;
      jx = jx + double(CX[i]) * f;
      jy = jy + double(CY[i]) * f;
    }
    for (int k = 0; k < 5; ++k) {
      bx = bx + st[(9 + k) * n + s];
      by = by + st[(14 + k) * n + s];
    }
    e = e + (jx * jx + jy * jy) / (2.0 * rho) + 0.5 * (bx * bx + by * by);
  }
  return e;
}

}  // namespace

extern "C" {

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Lattice vectors and weights, as doubles.
void orc_lattice(double cx[9], double cy[9], double w[9], double mcx[5], double mcy[5],
                 double wm[5]) {
  for (int i = 0; i < 9; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    w[i] = weight9(i);
  }
  for (int k = 0; k < 5; ++k) {
    mcx[k] = MX[k];
    mcy[k] = MY[k];
    wm[k] = weight5(k);
  }
}

// T (9x9), T^-1 (9x9) and T_m (5x5), row-major.
void orc_matrices(double T[81], double Tinv[81], double Tm[25]) {
  const Tables& tb = tables();
  for (int r = 0; r < 9; ++r)
    for (int i = 0; i < 9; ++i) {
      T[9 * r + i] = tb.T[r][i];
      Tinv[9 * r + i] = tb.Tinv[r][i];
    }
  for (int r = 0; r < 5; ++r)
    for (int k = 0; k < 5; ++k) Tm[5 * r + k] = tb.Tm[r][k];
}

void orc_equilibrium(double rho, double ux, double uy, double bx, double by, double feq[9],
                     double geq[10]) {
  equilibrium<double>(rho, ux, uy, bx, by, feq, geq);
}

void orc_moment_equilibria(double rho, double jx, double jy, double bx, double by,
                           double meq[9], double neq[10]) {
  moment_equilibria<double>(rho, jx, jy, bx, by, meq, neq);
}

// f = f^eq(rho, u, B), g = g^eq(u, B) at every site.
int orc_init(const orc_params* p, const double* rho, const double* ux, const double* uy,
             const double* bx, const double* by, double* state) {
  if (!valid(p)) return -1;
  init_all<double>(*p, rho, ux, uy, bx, by, state);
  return 0;
}

// Collision at every site, in place.  tau / taum (nullable, nx*ny each)
// receive the relaxation times used.
int orc_collide(const orc_params* p, double* state, double* tau, double* taum) {
  if (!valid(p)) return -1;
  collide_all<double>(*p, state, p->cs, p->csb, tau, taum);
  return 0;
}

int orc_stream(const orc_params* p, const double* in, double* out) {
  if (!valid(p)) return -1;
  stream_all<double>(*p, in, out);
  return 0;
}

// nsteps applications of collide-then-stream, in place.
int orc_run(const orc_params* p, double* state, int64_t nsteps) {
  if (!valid(p) || nsteps < 0) return -1;
  const int64_t n = int64_t(p->nx) * p->ny;
  std::vector<double> tmp(size_t(ORC_NPOP) * n);
  for (int64_t t = 0; t < nsteps; ++t) {
    collide_all<double>(*p, state, p->cs, p->csb, nullptr, nullptr);
    stream_all<double>(*p, state, tmp.data());
    std::memcpy(state, tmp.data(), sizeof(double) * tmp.size());
  }
  return 0;
}

// rho, u = (rho u) / rho, B at every site.
int orc_macro(const orc_params* p, const double* st, double* rho, double* ux, double* uy,
              double* bx, double* by) {
  if (!valid(p)) return -1;
  const int64_t n = int64_t(p->nx) * p->ny;
  for (int64_t s = 0; s < n; ++s) {
    double r = 0.0, jx = 0.0, jy = 0.0, b0 = 0.0, b1 = 0.0;
    for (int i = 0; i < 9; ++i) {
      r += st[i * n + s];
      jx += CX[i] * st[i * n + s];
      jy += CY[i] * st[i * n + s];
    }
    for (int k = 0; k < 5; ++k) {
      b0 += st[(9 + k) * n + s];
      b1 += st[(14 + k) * n + s];
    }
    rho[s] = r;
    ux[s] = jx / r;
    uy[s] = jy / r;
    bx[s] = b0;
    by[s] = b1;
  }
  return 0;
}

// Global diagnostics, accumulated in order over sites:
//  0 mass sum(rho)           1,2 momentum sum(rho u)      3,4 flux sum(B)
//  5 kinetic energy sum(|rho u|^2 / (2 rho))   6 magnetic energy sum(|B|^2 / 2)
//  7 cross helicity sum(u . B)                  8 max |d_x B_x + d_y B_y|
//  9 enstrophy sum(w^2 / 2), w = d_x u_y - d_y u_x
// 10 sum(j^2 / 2), j = d_x B_y - d_y B_x
// 11 number of sites holding a non-finite population   12 max |u|
// 13 max |d_x B_x + d_y B_y| / max |j|  (0 if j vanishes)
// d_x a = (a(x+1) - a(x-1)) / 2, periodic.
int orc_diag(const orc_params* p, const double* st, double out[ORC_NDIAG]) {
  if (!valid(p)) return -1;
  const int64_t nx = p->nx, ny = p->ny, n = nx * ny;
  std::vector<double> rho(n), ux(n), uy(n), bx(n), by(n);
  orc_macro(p, st, rho.data(), ux.data(), uy.data(), bx.data(), by.data());
  for (int q = 0; q < ORC_NDIAG; ++q) out[q] = 0.0;
  double maxdiv = 0.0, maxj = 0.0, maxu = 0.0;
  int64_t bad = 0;
  for (int64_t y = 0; y < ny; ++y)
    for (int64_t x = 0; x < nx; ++x) {
      int64_t s = y * nx + x;
      int64_t e = y * nx + wrap(x + 1, nx), w = y * nx + wrap(x - 1, nx);
      int64_t nn = wrap(y + 1, ny) * nx + x, so = wrap(y - 1, ny) * nx + x;
      bool finite = true;
      for (int q = 0; q < ORC_NPOP; ++q)
        if (!std::isfinite(st[q * n + s])) finite = false;
      if (!finite) ++bad;
      double jx = rho[s] * ux[s], jy = rho[s] * uy[s];
      out[0] += rho[s];
      out[1] += jx;
      out[2] += jy;
      out[3] += bx[s];
      out[4] += by[s];
      out[5] += (jx * jx + jy * jy) / (2.0 * rho[s]);
      out[6] += 0.5 * (bx[s] * bx[s] + by[s] * by[s]);
      out[7] += ux[s] * bx[s] + uy[s] * by[s];
      double div = 0.5 * (bx[e] - bx[w]) + 0.5 * (by[nn] - by[so]);
      double om = 0.5 * (uy[e] - uy[w]) - 0.5 * (ux[nn] - ux[so]);
      double jz = 0.5 * (by[e] - by[w]) - 0.5 * (bx[nn] - bx[so]);
      if (std::fabs(div) > maxdiv) maxdiv = std::fabs(div);
      if (std::fabs(jz) > maxj) maxj = std::fabs(jz);
      out[9] += 0.5 * om * om;
      out[10] += 0.5 * jz * jz;
      double um = std::sqrt(ux[s] * ux[s] + uy[s] * uy[s]);
      if (um > maxu) maxu = um;
    }
  out[8] = maxdiv;
  out[11] = double(bad);
  out[12] = maxu;
  out[13] = maxj > 0.0 ? maxdiv / maxj : 0.0;
  return 0;
}

// T_m^-1 (5x5, row-major).
void orc_tm_inverse(double out[25]) {
  const Tables& tb = tables();
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) out[5 * r + c] = tb.Tminv[r][c];
}

// The two filter-width expansion terms at one point: out[0] = the product
// term of eq. FilterExampleSmall, out[1] = the ratio term of eq.
// FilterExampleLarge, for values X, Y, Z and gradients dX, dY, dZ (x, y).
void orc_filter_terms(double d2, double X, double Y, double Z, const double dX[2],
                      const double dY[2], const double dZ[2], double out[2]) {
  out[0] = filtered_product_term<double>(d2, dX, dY);
  out[1] = filtered_ratio_term<double>(d2, X, Y, Z, dX, dY, dZ);
}

// Delta^2 parts of the filtered equilibrium moments at one site (kinetic
// closure), from rho, j, B and grad = d_x, d_y of (rho, j_x, j_y, B_x, B_y).
void orc_filtered_moment_corrections(double d2, double rho, double jx, double jy, double bx,
                                     double by, const double grad[10], double dmeq[9],
                                     double dneq[10]) {
  filtered_moment_corrections<double>(d2, rho, jx, jy, bx, by, grad, dmeq, dneq);
}

// Lattice gradients used by the kinetic closure: 10 planes of nx*ny.
int orc_gradients(const orc_params* p, const double* st, double* grad) {
  if (!valid(p)) return -1;
  std::vector<double> g;
  lattice_gradients<double>(*p, st, g);
  std::memcpy(grad, g.data(), sizeof(double) * g.size());
  return 0;
}

double orc_energy(const orc_params* p, const double* st) {
  if (!valid(p)) return NAN;
  return energy_all<double>(*p, st);
}

// ---------------------------------------------------------- tangent-linear
// Tangent of one collision at every site: state (19*n) is advanced in place,
// dstate (ndir planes of 19*n, direction-major) carries the tangents, and
// dcs[2 * ndir] are the tangents of (C_Sv, C_Sb) per direction.
int orc_tl_collide(const orc_params* p, double* state, double* dstate, const double* dcs,
                   int ndir) {
  if (!valid(p) || ndir < 1 || ndir > ND) return -1;
  const int64_t n = int64_t(p->nx) * p->ny, m = int64_t(ORC_NPOP) * n;
  std::vector<Dual> st(m);
  for (int64_t q = 0; q < m; ++q) {
    st[q].v = state[q];
    for (int k = 0; k < ndir; ++k) st[q].d[k] = dstate[k * m + q];
  }
  Dual cs(p->cs), csb(p->csb);
  for (int k = 0; k < ndir; ++k) {
    cs.d[k] = dcs ? dcs[2 * k] : 0.0;
    csb.d[k] = dcs ? dcs[2 * k + 1] : 0.0;
  }
  collide_all<Dual>(*p, st.data(), cs, csb, nullptr, nullptr);
  for (int64_t q = 0; q < m; ++q) {
    state[q] = st[q].v;
    for (int k = 0; k < ndir; ++k) dstate[k * m + q] = st[q].d[k];
  }
  return 0;
}

// Directional derivatives of the final total energy J(u0, B0, C_Sv, C_Sb)
// after nsteps, starting from equilibrium with rho0 fixed.  dfields holds ndir
// blocks of 4 planes (du_x, du_y, dB_x, dB_y), each nx*ny; dcs[2 * ndir] the
// tangents of (C_Sv, C_Sb) per direction.
// Writes J and dJ[k] = <grad J, v_k>.
int orc_tl_energy(const orc_params* p, const double* rho, const double* ux, const double* uy,
                  const double* bx, const double* by, const double* dfields, const double* dcs,
                  int ndir, int64_t nsteps, double* J, double* dJ) {
  if (!valid(p) || ndir < 1 || ndir > ND || nsteps < 0) return -1;
  const int64_t n = int64_t(p->nx) * p->ny;
  std::vector<Dual> r(n), u(n), v(n), a(n), b(n);
  for (int64_t s = 0; s < n; ++s) {
    r[s] = Dual(rho[s]);
    u[s] = Dual(ux[s]);
    v[s] = Dual(uy[s]);
    a[s] = Dual(bx[s]);
    b[s] = Dual(by[s]);
    for (int k = 0; k < ndir; ++k) {
      const double* d = dfields + int64_t(k) * 4 * n;
      u[s].d[k] = d[0 * n + s];
      v[s].d[k] = d[1 * n + s];
      a[s].d[k] = d[2 * n + s];
      b[s].d[k] = d[3 * n + s];
    }
  }
  std::vector<Dual> st(size_t(ORC_NPOP) * n), tmp(size_t(ORC_NPOP) * n);
  init_all<Dual>(*p, r.data(), u.data(), v.data(), a.data(), b.data(), st.data());
  Dual cs(p->cs), csb(p->csb);
  for (int k = 0; k < ndir; ++k) {
    cs.d[k] = dcs ? dcs[2 * k] : 0.0;
    csb.d[k] = dcs ? dcs[2 * k + 1] : 0.0;
  }
  for (int64_t t = 0; t < nsteps; ++t) {
    collide_all<Dual>(*p, st.data(), cs, csb, nullptr, nullptr);
    stream_all<Dual>(*p, st.data(), tmp.data());
    st.swap(tmp);
  }
  Dual e = energy_all<Dual>(*p, st.data());
  *J = e.v;
  for (int k = 0; k < ndir; ++k) dJ[k] = e.d[k];
  return 0;
}

}  // extern "C"
