// Drives every entry point of the two FP64 oracles on small, ragged lattices
// so that a build with AddressSanitizer and UndefinedBehaviorSanitizer sees
// each loop and stencil at least once.  Checks the invariants that need no
// reference values (return codes, finiteness, conservation of mass and field
// by the collision) and prints "ok" on success.  Test infrastructure only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
typedef struct {
  int32_t nx, ny;
  double nu, eta;
  double s5, s6, s7, s8;
  int32_t les;
  double cs, csb;
  double delta;
} orc_params;
typedef struct {
  int32_t nx, ny, nz;
  double nu, eta;
  int32_t les;
  double cs, csb, delta;
  int32_t mrt;
  double s5, s7, s8, sg, szz;
} orc3_params;

void orc_lattice(double*, double*, double*, double*, double*, double*);
void orc_matrices(double*, double*, double*);
void orc_equilibrium(double, double, double, double, double, double*, double*);
void orc_moment_equilibria(double, double, double, double, double, double*, double*);
int orc_init(const orc_params*, const double*, const double*, const double*, const double*,
             const double*, double*);
int orc_collide(const orc_params*, double*, double*, double*);
int orc_stream(const orc_params*, const double*, double*);
int orc_run(const orc_params*, double*, int64_t);
int orc_macro(const orc_params*, const double*, double*, double*, double*, double*, double*);
int orc_diag(const orc_params*, const double*, double*);
void orc_tm_inverse(double*);
void orc_filter_terms(double, double, double, double, const double*, const double*,
                      const double*, double*);
void orc_filtered_moment_corrections(double, double, double, double, double, double,
                                     const double*, double*, double*);
int orc_gradients(const orc_params*, const double*, double*);
double orc_energy(const orc_params*, const double*);
int orc_tl_collide(const orc_params*, double*, double*, const double*, int);
int orc_tl_energy(const orc_params*, const double*, const double*, const double*, const double*,
                  const double*, const double*, const double*, int, int64_t, double*, double*);

void orc3_lattice(double*, double*, double*, double*);
void orc3_equilibrium(double, const double*, const double*, double*, double*);
int orc3_init(const orc3_params*, const double*, const double*, const double*, const double*,
              const double*, const double*, const double*, double*);
int orc3_collide(const orc3_params*, double*, double*, double*);
int orc3_stream(const orc3_params*, const double*, double*);
int orc3_run(const orc3_params*, double*, int64_t);
int orc3_macro(const orc3_params*, const double*, double*, double*, double*);
int orc3_diag(const orc3_params*, const double*, double*);
}

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAILED %s at line %d\n", #c, __LINE__);         \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static bool finite_all(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// smooth periodic fields with a little of everything
static void fields2(int nx, int ny, std::vector<double> (&f)[5]) {
  const double tp = 6.283185307179586;
  for (auto& a : f) a.assign(size_t(nx) * ny, 0.0);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const double X = tp * x / nx, Y = tp * y / ny;
      const size_t s = size_t(y) * nx + x;
      f[0][s] = 1.0 + 0.01 * std::cos(X + Y);
      f[1][s] = -0.05 * std::sin(Y) + 0.01 * std::cos(2 * X);
      f[2][s] = 0.05 * std::sin(X);
      f[3][s] = -0.05 * std::sin(Y);
      f[4][s] = 0.05 * std::sin(2 * X) + 0.01 * std::cos(Y);
    }
}

static void check2(int nx, int ny, int les) {
  orc_params p{nx, ny, 0.01, 0.02, 1.0, 1.0, 1.2, 1.1, les, 0.1, 0.08, 1.0};
  const size_t n = size_t(nx) * ny;
  std::vector<double> f[5];
  fields2(nx, ny, f);
  std::vector<double> st(19 * n), tmp(19 * n), tau(n), taum(n);
  CHECK(orc_init(&p, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(),
                 st.data()) == 0);
  std::vector<double> m0[5], m1[5];
  for (int k = 0; k < 5; ++k) m0[k].resize(n), m1[k].resize(n);
  CHECK(orc_macro(&p, st.data(), m0[0].data(), m0[1].data(), m0[2].data(), m0[3].data(),
                  m0[4].data()) == 0);
  CHECK(orc_collide(&p, st.data(), tau.data(), taum.data()) == 0);
  CHECK(orc_macro(&p, st.data(), m1[0].data(), m1[1].data(), m1[2].data(), m1[3].data(),
                  m1[4].data()) == 0);
  for (size_t s = 0; s < n; ++s) {   // the collision keeps rho and B at every site
    CHECK(std::fabs(m1[0][s] - m0[0][s]) < 1e-13);
    CHECK(std::fabs(m1[3][s] - m0[3][s]) < 1e-13);
    CHECK(std::fabs(m1[4][s] - m0[4][s]) < 1e-13);
    CHECK(tau[s] >= 0.5 && taum[s] >= 0.5);
  }
  CHECK(orc_stream(&p, st.data(), tmp.data()) == 0);
  CHECK(orc_run(&p, tmp.data(), 3) == 0);
  CHECK(finite_all(tmp));
  std::vector<double> dg(14), grad(10 * n);
  CHECK(orc_diag(&p, tmp.data(), dg.data()) == 0);
  CHECK(finite_all(dg));
  CHECK(orc_gradients(&p, tmp.data(), grad.data()) == 0);
  CHECK(finite_all(grad));
  CHECK(std::isfinite(orc_energy(&p, tmp.data())));
  // tangents: two directions, one of them along both closure constants
  std::vector<double> dst(2 * 19 * n), dcs{0.0, 0.0, 1.0, 1.0};
  for (size_t q = 0; q < 19 * n; ++q) dst[q] = 1e-3 * std::sin(0.37 * double(q));
  std::vector<double> st2 = tmp;
  CHECK(orc_tl_collide(&p, st2.data(), dst.data(), dcs.data(), 2) == 0);
  CHECK(finite_all(dst));
  std::vector<double> dfields(2 * 4 * n);
  for (size_t q = 0; q < dfields.size(); ++q) dfields[q] = 1e-2 * std::cos(0.11 * double(q));
  double J = 0.0, dJ[2] = {0.0, 0.0};
  CHECK(orc_tl_energy(&p, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(),
                      dfields.data(), dcs.data(), 2, 2, &J, dJ) == 0);
  CHECK(std::isfinite(J) && std::isfinite(dJ[0]) && std::isfinite(dJ[1]));
}

static void check3(int nx, int ny, int nz, int les, int mrt) {
  orc3_params p{nx, ny, nz, 0.02, 0.03, les, 0.1, 0.05, 1.0, mrt, 1.3, 0.7, 1.6, 1.1, 0.9};
  const size_t n = size_t(nx) * ny * nz;
  std::vector<double> f[7];
  for (auto& a : f) a.assign(n, 0.0);
  for (size_t s = 0; s < n; ++s) {
    f[0][s] = 1.0;
    for (int k = 1; k < 7; ++k) f[k][s] = 0.02 * std::sin(0.7 * double(s) + k);
  }
  std::vector<double> st(45 * n), tmp(45 * n), tau(n), taum(n);
  CHECK(orc3_init(&p, f[0].data(), f[1].data(), f[2].data(), f[3].data(), f[4].data(),
                  f[5].data(), f[6].data(), st.data()) == 0);
  std::vector<double> r0(n), u0(3 * n), b0(3 * n), r1(n), u1(3 * n), b1(3 * n);
  CHECK(orc3_macro(&p, st.data(), r0.data(), u0.data(), b0.data()) == 0);
  CHECK(orc3_collide(&p, st.data(), tau.data(), taum.data()) == 0);
  CHECK(orc3_macro(&p, st.data(), r1.data(), u1.data(), b1.data()) == 0);
  for (size_t s = 0; s < n; ++s) CHECK(std::fabs(r1[s] - r0[s]) < 1e-13);
  for (size_t s = 0; s < 3 * n; ++s) CHECK(std::fabs(b1[s] - b0[s]) < 1e-13);
  CHECK(orc3_stream(&p, st.data(), tmp.data()) == 0);
  CHECK(orc3_run(&p, tmp.data(), 2) == 0);
  CHECK(finite_all(tmp));
  std::vector<double> dg(12);
  CHECK(orc3_diag(&p, tmp.data(), dg.data()) == 0);
  CHECK(finite_all(dg));
}

int main() {
  double a[81], b[81], c[27], d[27], e[25], w[27], cc[18], ww[6];
  orc_lattice(a, b, c, d, e, w);
  orc_matrices(a, b, e);
  orc_tm_inverse(e);
  double feq[9], geq[10], meq[9], neq[10];
  orc_equilibrium(1.0, 0.1, -0.05, 0.02, 0.03, feq, geq);
  orc_moment_equilibria(1.0, 0.1, -0.05, 0.02, 0.03, meq, neq);
  const double g2[2] = {0.1, 0.2}, g3[2] = {-0.1, 0.3}, g4[2] = {0.05, 0.0};
  double out[2];
  orc_filter_terms(1.0, 1.0, 0.1, 0.2, g2, g3, g4, out);
  double grad[10];
  for (int k = 0; k < 10; ++k) grad[k] = 0.01 * (k + 1);
  orc_filtered_moment_corrections(1.0, 1.0, 0.1, 0.05, 0.02, 0.03, grad, meq, neq);
  orc3_lattice(a, w, cc, ww);
  const double u3[3] = {0.1, -0.05, 0.02}, b3[3] = {0.03, 0.01, -0.02};
  double feq3[27], geq3[18];
  orc3_equilibrium(1.0, u3, b3, feq3, geq3);
  // invalid parameters are refused, not read past
  orc_params bad{1, 4, 0.01, 0.01, 1.0, 1.0, 1.0, 1.0, 0, 0.1, 0.1, 1.0};
  std::vector<double> st(19 * 4);
  CHECK(orc_run(&bad, st.data(), 1) != 0);
  orc_params bad2{4, 4, 0.01, 0.01, 1.0, 1.0, 1.0, 1.0, 5, 0.1, 0.1, 1.0};
  std::vector<double> st2(19 * 16);
  CHECK(orc_run(&bad2, st2.data(), 1) != 0);
  const int sizes[][2] = {{2, 2}, {5, 3}, {7, 4}, {3, 9}};
  for (auto& sz : sizes)
    for (int les : {0, 1, 2, 3, 4, 6}) check2(sz[0], sz[1], les);
  const int sizes3[][3] = {{2, 2, 2}, {3, 4, 5}, {5, 2, 3}};
  for (auto& sz : sizes3)
    for (int les : {0, 1})
      for (int mrt : {0, 1}) check3(sz[0], sz[1], sz[2], les, mrt);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
