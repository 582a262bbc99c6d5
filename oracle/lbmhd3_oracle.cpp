// lbmhd3_oracle.cpp -- plain FP64 CPU oracle for the three-dimensional
// extension of the lattice Boltzmann MHD update with the Smagorinsky-MHD
// closure (Flint & Vahala, arXiv:1607.08675; the paper works in 2D and states
// that the model extends to 3D with more lattice velocities, Sec. 3 and
// Sec. 5, without giving the 3D lattice).
//
// TEST INFRASTRUCTURE ONLY.  Slow, obviously correct reference for the GPU
// library's 3D path.  Only the test suite, the smoke check and the CPU
// baseline of the benchmark may load it.  It shares no code, header or
// constant with the GPU library or with the 2D oracle.
//
// The 3D model, each choice a reading of the paper's 2D construction:
//   * f on D3Q27 = D2Q9 x D1Q3 (the tensor-product lattice whose z sums give
//     the paper's D2Q9 and weights 4/9, 1/9, 1/36), weights 8/27, 2/27, 1/54,
//     1/216, c_s^2 = 1/3;
//   * f^eq_i = w_i [rho + 3 c_i.j + (9/2) (c_i c_i - I/3) : (j j / rho
//     + |B|^2 I / 2 - B B)], the second-order Hermite form whose 2D version is
//     the paper's D2Q9 equilibrium with the Maxwell stress (Sec. 3);
//   * g on the six unit vectors +-x, +-y, +-z with weight 1/6 each (no rest
//     vector): its z sums give the paper's D2Q5 weights 1/3, 1/6, and the
//     same magnetic 'sound speed' 1/3, so tau_m0 = 3 eta + 1/2 as in 2D;
//     g^eq_kb = (1/6) [B_b + 3 (C_k.u B_b - C_k.B u_b)] (Sec. 3's D2Q5 form);
//   * single-relaxation collisions f* = f - (f - f^eq) / tau and
//     g* = g - (g - g^eq) / tau_m: the paper's moment-space collision gives the
//     BGK update of Sec. 1.2 when every rate equals 1/tau, and no 3D moment
//     basis is given;
//   * or (mrt = 1) a moment-space collision for f (Sec. 3): the moments are
//     the products p_r(c_x, c_y) q_k(c_z) of the paper's nine D2Q9 rows
//     (eq. FluidTMatrix) with q_0 = 1, q_1 = c_z, q_2 = 3 c_z^2 - 1, the
//     tensor-product basis of D3Q27 = D2Q9 x D1Q3; f* = f - T^-1 S T (f - f^eq).
//     Rates: the k = 0 block (the z sums) takes the paper's 2D rates (shear
//     1/tau for rows 3, 4, s5 for rows 5, 6, s7, s8), so for fields invariant
//     along z the z sums follow the paper's 2D update exactly at any rates;
//     the shears xz, yz (k = 1, rows 1, 2) take 1/tau, the z normal stress
//     (k = 2, row 0) szz, every other moment that varies along c_z the ghost
//     rate sg; rows 0 (k = 0, 1) are conserved.  With every rate 1/tau this
//     is the BGK update.  The basis singles out z: the update is covariant
//     under the cube's rotations only when the rates of rotated moments agree
//     (for instance all 1/tau);
//   * Smagorinsky closure per site exactly as in 2D: with Pi' the traceless
//     part of Pi^neq = sum_i c_i c_i (f_i - f^eq_i) and Q = sqrt(2 Pi':Pi'),
//     |S| = 3 Q / (2 rho tau) and tau = (tau0 + sqrt(tau0^2 + 18 C_Sv Delta^2 Q
//     / rho)) / 2; with A = eps : Lambda^neq (Lambda_ab = sum_k C_ka g_kb,
//     Lambda^neq_ab ~ -(tau_m / 3) d_a B_b), |j| = 3 |A| / tau_m and
//     tau_m = (tau_m0 + sqrt(tau_m0^2 + 36 C_Sb Delta^2 |A|)) / 2;
//   * collide-then-stream with unit time step, periodic in x, y, z.
//
// State layout: 45 planes of nx*ny*nz doubles, [plane][z][y][x], x fastest.
// Planes 0..26 hold f in the velocity order of C27 below (opposite velocities
// adjacent after the rest velocity); planes 27..32 the x component of g for
// the six vectors of C6, 33..38 the y component, 39..44 the z component.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const int C27[27][3] = {
    {0, 0, 0},                                                    // rest
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},   // faces
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},                             // xy edges
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},                             // xz edges
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},                             // yz edges
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},                            // corners
    {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};
const int C6[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
const int NP = 45;

// D1Q3 weights (2/3, 1/6, 1/6) multiplied over the three axes.
double weight27(int i) {
  double w = 1.0;
  for (int a = 0; a < 3; ++a) w *= C27[i][a] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
  return w;
}

struct P3 {
  int nx, ny, nz;
  double nu, eta;
  int les;
  double cs, csb, delta;
  int mrt;
  double s5, s7, s8, sg, szz;
};

// Row r of the paper's D2Q9 moment transform (eq. FluidTMatrix) as a
// polynomial in (c_x, c_y), and the three D1Q3 rows in c_z.
double prow(int r, double cx, double cy) {
  const double x2 = cx * cx, y2 = cy * cy;
  switch (r) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cx * cy;
    case 4: return x2 - y2;
    case 5: return 3.0 * cx * y2 - 2.0 * cx;
    case 6: return 3.0 * cy * x2 - 2.0 * cy;
    case 7: return 4.0 - 9.0 * (x2 + y2 - 2.0 * x2 * y2);
    default: return 4.0 - 4.0 * (x2 + y2) + 3.0 * x2 * y2;
  }
}
double qrow(int k, double cz) { return k == 0 ? 1.0 : (k == 1 ? cz : 3.0 * cz * cz - 1.0); }

// T (27 x 27, row 3 r + k = p_r q_k) and its inverse by Gauss-Jordan
// elimination with partial pivoting, computed once.
struct Basis27 {
  double T[27][27], Ti[27][27];
  Basis27() {
    double A[27][54];
    for (int m = 0; m < 27; ++m)
      for (int i = 0; i < 27; ++i) {
        T[m][i] = prow(m / 3, C27[i][0], C27[i][1]) * qrow(m % 3, C27[i][2]);
        A[m][i] = T[m][i];
        A[m][27 + i] = m == i ? 1.0 : 0.0;
      }
    for (int c = 0; c < 27; ++c) {
      int piv = c;
      for (int r = c + 1; r < 27; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      for (int j = 0; j < 54; ++j) std::swap(A[c][j], A[piv][j]);
      const double d = A[c][c];
      for (int j = 0; j < 54; ++j) A[c][j] /= d;
      for (int r = 0; r < 27; ++r)
        if (r != c) {
          const double f = A[r][c];
          for (int j = 0; j < 54; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int i = 0; i < 27; ++i)
      for (int m = 0; m < 27; ++m) Ti[i][m] = A[i][27 + m];
  }
};
const Basis27& basis27() {
  static const Basis27 b;
  return b;
}

// Rate of moment m = 3 r + k (see the header): sv = 1/tau.
double rate27(const P3& p, int m, double sv) {
  const int r = m / 3, k = m % 3;
  if (k == 0) {
    const double s2d[9] = {0.0, 0.0, 0.0, sv, sv, p.s5, p.s5, p.s7, p.s8};
    return s2d[r];
  }
  if (k == 1) return r == 0 ? 0.0 : (r <= 2 ? sv : p.sg);
  return r == 0 ? p.szz : p.sg;
}

void equilibrium(double rho, const double u[3], const double B[3], double feq[27],
                 double geq[18]) {
  double j[3] = {rho * u[0], rho * u[1], rho * u[2]};
  double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  // Pi' = j j / rho + |B|^2 I / 2 - B B
  double Pi[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Pi[a][b] = j[a] * j[b] / rho + (a == b ? 0.5 * b2 : 0.0) - B[a] * B[b];
  for (int i = 0; i < 27; ++i) {
    double cj = 0.0, qp = 0.0;
    for (int a = 0; a < 3; ++a) cj += C27[i][a] * j[a];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        qp += (C27[i][a] * C27[i][b] - (a == b ? 1.0 / 3.0 : 0.0)) * Pi[a][b];
    feq[i] = weight27(i) * (rho + 3.0 * cj + 4.5 * qp);
  }
  for (int k = 0; k < 6; ++k) {
    double cu = 0.0, cb = 0.0;
    for (int a = 0; a < 3; ++a) {
      cu += C6[k][a] * u[a];
      cb += C6[k][a] * B[a];
    }
    for (int b = 0; b < 3; ++b) geq[6 * b + k] = (B[b] + 3.0 * (cu * B[b] - cb * u[b])) / 6.0;
  }
}

// One collision at one site: f[27], g[18] (component-major) overwritten.
void collide_site(const P3& p, double f[27], double g[18], double* tau_out, double* taum_out) {
  double rho = 0.0, j[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  for (int i = 0; i < 27; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += C27[i][a] * f[i];
  }
  for (int b = 0; b < 3; ++b)
    for (int k = 0; k < 6; ++k) B[b] += g[6 * b + k];
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double feq[27], geq[18];
  equilibrium(rho, u, B, feq, geq);
  const double tau0 = 3.0 * p.nu + 0.5, taum0 = 3.0 * p.eta + 0.5;
  double tau = tau0, taum = taum0;
  if (p.les) {
    const double d2 = p.delta * p.delta;
    double Pn[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < 27; ++i)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Pn[a][b] += C27[i][a] * C27[i][b] * (f[i] - feq[i]);
    const double tr = (Pn[0][0] + Pn[1][1] + Pn[2][2]) / 3.0;
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double t = Pn[a][b] - (a == b ? tr : 0.0);
        ss += t * t;
      }
    const double Q = std::sqrt(2.0 * ss);
    tau = 0.5 * (tau0 + std::sqrt(tau0 * tau0 + 18.0 * d2 * p.cs * Q / rho));
    double L[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += C6[k][a] * (g[6 * b + k] - geq[6 * b + k]);
        L[a][b] = acc;
      }
    // A_c = eps_cab L_ab
    const double A[3] = {L[1][2] - L[2][1], L[2][0] - L[0][2], L[0][1] - L[1][0]};
    const double An = std::sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    taum = 0.5 * (taum0 + std::sqrt(taum0 * taum0 + 36.0 * d2 * p.csb * An));
  }
  if (tau_out) *tau_out = tau;
  if (taum_out) *taum_out = taum;
  if (p.mrt) {
    const Basis27& b = basis27();
    double rel[27];
    for (int m = 0; m < 27; ++m) {
      double nm = 0.0;
      for (int i = 0; i < 27; ++i) nm += b.T[m][i] * (f[i] - feq[i]);
      rel[m] = rate27(p, m, 1.0 / tau) * nm;
    }
    for (int i = 0; i < 27; ++i) {
      double df = 0.0;
      for (int m = 0; m < 27; ++m) df += b.Ti[i][m] * rel[m];
      f[i] -= df;
    }
  } else {
    for (int i = 0; i < 27; ++i) f[i] -= (f[i] - feq[i]) / tau;
  }
  for (int q = 0; q < 18; ++q) g[q] -= (g[q] - geq[q]) / taum;
}

inline int64_t wrap(int64_t a, int64_t n) { return ((a % n) + n) % n; }

bool valid(const P3* p) {
  auto rate = [](double s) { return s > 0.0 && s < 2.0; };
  return p && p->nx >= 1 && p->ny >= 1 && p->nz >= 1 && p->nu > 0.0 && p->eta > 0.0 &&
         (p->les == 0 || p->les == 1) && (p->mrt == 0 || p->mrt == 1) &&
         (p->mrt == 0 || (rate(p->s5) && rate(p->s7) && rate(p->s8) && rate(p->sg) &&
                          rate(p->szz)));
}

int64_t sites(const P3& p) { return int64_t(p.nx) * p.ny * p.nz; }

void collide_all(const P3& p, double* st, double* tau, double* taum) {
  const int64_t n = sites(p);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < n; ++s) {
    double f[27], g[18];
    for (int i = 0; i < 27; ++i) f[i] = st[i * n + s];
    for (int q = 0; q < 18; ++q) g[q] = st[(27 + q) * n + s];
    collide_site(p, f, g, tau ? tau + s : nullptr, taum ? taum + s : nullptr);
    for (int i = 0; i < 27; ++i) st[i * n + s] = f[i];
    for (int q = 0; q < 18; ++q) st[(27 + q) * n + s] = g[q];
  }
}

// population of velocity c at x moves to x + c
void stream_all(const P3& p, const double* in, double* out) {
  const int64_t nx = p.nx, ny = p.ny, nz = p.nz, n = sites(p);
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t s = (z * ny + y) * nx + x;
        for (int q = 0; q < NP; ++q) {
          const int* c = q < 27 ? C27[q] : C6[(q - 27) % 6];
          const int64_t d = (wrap(z + c[2], nz) * ny + wrap(y + c[1], ny)) * nx + wrap(x + c[0], nx);
          out[q * n + d] = in[q * n + s];
        }
      }
}

void moments(const double* st, int64_t n, int64_t s, double* rho, double j[3], double B[3]) {
  *rho = 0.0;
  j[0] = j[1] = j[2] = B[0] = B[1] = B[2] = 0.0;
  for (int i = 0; i < 27; ++i) {
    *rho += st[i * n + s];
    for (int a = 0; a < 3; ++a) j[a] += C27[i][a] * st[i * n + s];
  }
  for (int b = 0; b < 3; ++b)
    for (int k = 0; k < 6; ++k) B[b] += st[(27 + 6 * b + k) * n + s];
}

}  // namespace

extern "C" {

typedef struct {
  int32_t nx, ny, nz;
  double nu, eta;
  int32_t les;          // 0: fixed rates; 1: Smagorinsky-MHD closure
  double cs, csb;       // closure constants C_Sv and C_Sb
  double delta;         // filter width
  int32_t mrt;          // 0: single relaxation; 1: moment-space collision for f
  double s5, s7, s8;    // rates of the paper's 2D rows 5 and 6, 7, 8 (k = 0)
  double sg, szz;       // the other moments that vary along c_z; the z normal stress
} orc3_params;

int orc3_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// velocities (27 x 3 and 6 x 3, as doubles) and weights
void orc3_lattice(double c27[81], double w27[27], double c6[18], double w6[6]) {
  for (int i = 0; i < 27; ++i) {
    for (int a = 0; a < 3; ++a) c27[3 * i + a] = C27[i][a];
    w27[i] = weight27(i);
  }
  for (int k = 0; k < 6; ++k) {
    for (int a = 0; a < 3; ++a) c6[3 * k + a] = C6[k][a];
    w6[k] = 1.0 / 6.0;
  }
}

void orc3_equilibrium(double rho, const double u[3], const double B[3], double feq[27],
                      double geq[18]) {
  equilibrium(rho, u, B, feq, geq);
}

static P3 unpack(const orc3_params* q) {
  return P3{q->nx, q->ny, q->nz, q->nu, q->eta, q->les, q->cs, q->csb, q->delta,
            q->mrt, q->s5, q->s7, q->s8, q->sg, q->szz};
}

int orc3_init(const orc3_params* q, const double* rho, const double* ux, const double* uy,
              const double* uz, const double* bx, const double* by, const double* bz,
              double* st) {
  const P3 p = unpack(q);
  if (!valid(&p)) return -1;
  const int64_t n = sites(p);
  for (int64_t s = 0; s < n; ++s) {
    const double u[3] = {ux[s], uy[s], uz[s]}, B[3] = {bx[s], by[s], bz[s]};
    double feq[27], geq[18];
    equilibrium(rho[s], u, B, feq, geq);
    for (int i = 0; i < 27; ++i) st[i * n + s] = feq[i];
    for (int k = 0; k < 18; ++k) st[(27 + k) * n + s] = geq[k];
  }
  return 0;
}

int orc3_collide(const orc3_params* q, double* st, double* tau, double* taum) {
  const P3 p = unpack(q);
  if (!valid(&p)) return -1;
  collide_all(p, st, tau, taum);
  return 0;
}

int orc3_stream(const orc3_params* q, const double* in, double* out) {
  const P3 p = unpack(q);
  if (!valid(&p)) return -1;
  stream_all(p, in, out);
  return 0;
}

int orc3_run(const orc3_params* q, double* st, int64_t nsteps) {
  const P3 p = unpack(q);
  if (!valid(&p) || nsteps < 0) return -1;
  std::vector<double> tmp(size_t(NP) * sites(p));
  for (int64_t t = 0; t < nsteps; ++t) {
    collide_all(p, st, nullptr, nullptr);
    stream_all(p, st, tmp.data());
    std::memcpy(st, tmp.data(), tmp.size() * sizeof(double));
  }
  return 0;
}

// rho, u (3 planes), B (3 planes) of the state
int orc3_macro(const orc3_params* q, const double* st, double* rho, double* u, double* B) {
  const P3 p = unpack(q);
  if (!valid(&p)) return -1;
  const int64_t n = sites(p);
  for (int64_t s = 0; s < n; ++s) {
    double r, j[3], b[3];
    moments(st, n, s, &r, j, b);
    rho[s] = r;
    for (int a = 0; a < 3; ++a) {
      u[a * n + s] = j[a] / r;
      B[a * n + s] = b[a];
    }
  }
  return 0;
}

// mass, momentum (3), flux (3), e_kin, e_mag, max |div B| (centred), max |u|,
// non-finite count
int orc3_diag(const orc3_params* q, const double* st, double out[12]) {
  const P3 p = unpack(q);
  if (!valid(&p)) return -1;
  const int64_t nx = p.nx, ny = p.ny, nz = p.nz, n = sites(p);
  std::vector<double> Bf(3 * n);
  for (int i = 0; i < 12; ++i) out[i] = 0.0;
  for (int64_t s = 0; s < n; ++s) {
    double r, j[3], b[3];
    moments(st, n, s, &r, j, b);
    out[0] += r;
    for (int a = 0; a < 3; ++a) {
      out[1 + a] += j[a];
      out[4 + a] += b[a];
      Bf[a * n + s] = b[a];
    }
    out[7] += (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / (2.0 * r);
    out[8] += 0.5 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    out[10] = std::fmax(out[10], std::sqrt(j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / r);
    if (!std::isfinite(r)) out[11] += 1.0;
  }
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        auto at = [&](int a, int64_t xx, int64_t yy, int64_t zz) {
          return Bf[a * n + (wrap(zz, nz) * ny + wrap(yy, ny)) * nx + wrap(xx, nx)];
        };
        const double div = 0.5 * (at(0, x + 1, y, z) - at(0, x - 1, y, z)) +
                           0.5 * (at(1, x, y + 1, z) - at(1, x, y - 1, z)) +
                           0.5 * (at(2, x, y, z + 1) - at(2, x, y, z - 1));
        out[9] = std::fmax(out[9], std::fabs(div));
      }
  return 0;
}

}  // extern "C"
