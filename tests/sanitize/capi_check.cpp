// Host-side paths of the C ABI (parameter validation, sizes, calls refused
// before bind, error strings) driven without a GPU, for a build whose host
// code runs under AddressSanitizer and UndefinedBehaviorSanitizer.  Prints
// "ok" on success.  Test infrastructure only.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <limits>

#include "lbmhd.h"
#include "lbmhd3.h"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAILED %s at line %d\n", #c, __LINE__);         \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static lbmhd_params base() {
  lbmhd_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = 64;
  p.ny = 48;
  p.nu = 0.01;
  p.eta = 0.02;
  p.s5 = p.s6 = 1.0;
  p.s7 = 1.1;
  p.s8 = 0.9;
  p.les = 1;
  p.cs = p.cs_b = 0.1;
  p.delta = 1.0;
  p.storage = LBMHD_FP32;
  p.inplace = 0;
  return p;
}

static void expect_rejected(const lbmhd_params& p) {
  lbmhd_t* h = nullptr;
  CHECK(lbmhd_create(&p, &h) == LBMHD_ERR_INVALID_ARG);
  CHECK(h == nullptr);
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  lbmhd_params p;
  p = base(); p.nx = 1; expect_rejected(p);
  p = base(); p.ny = 0; expect_rejected(p);
  p = base(); p.nu = 0.0; expect_rejected(p);
  p = base(); p.eta = nan; expect_rejected(p);
  p = base(); p.s5 = 2.0; expect_rejected(p);
  p = base(); p.s5 = 1.1; p.s6 = 1.2; expect_rejected(p);
  p = base(); p.les = 5; expect_rejected(p);
  p = base(); p.les = -1; expect_rejected(p);
  p = base(); p.cs = -0.1; expect_rejected(p);
  p = base(); p.cs_b = inf; expect_rejected(p);
  p = base(); p.delta = 0.0; expect_rejected(p);
  p = base(); p.inplace = 1; p.les = 4; expect_rejected(p);
  p = base(); p.storage = 7; expect_rejected(p);
  p = base(); p.nx = 70000; p.ny = 70000; expect_rejected(p);
  CHECK(lbmhd_create(nullptr, nullptr) != LBMHD_OK);

  for (int storage : {LBMHD_FP32, LBMHD_FP16})
    for (int inplace : {0, 1}) {
      p = base();
      p.nx = 100;
      p.ny = 36;
      p.storage = storage;
      p.inplace = inplace;
      lbmhd_t* h = nullptr;
      CHECK(lbmhd_create(&p, &h) == LBMHD_OK && h != nullptr);
      size_t lat = 0, ws = 0, adj = 0, acc = 0;
      CHECK(lbmhd_sizes(h, &lat, &ws, &adj, &acc) == LBMHD_OK);
      CHECK(lat > 0 && ws > 0 && adj > 0 && acc > 0);
      CHECK(lbmhd_sizes(h, nullptr, nullptr, nullptr, nullptr) == LBMHD_OK);
      int64_t pitch = 0, plane = 0, apitch = 0, aplane = 0;
      CHECK(lbmhd_layout(h, &pitch, &plane, &apitch, &aplane) == LBMHD_OK);
      CHECK(pitch >= p.nx && plane >= pitch * p.ny && apitch >= p.nx && aplane >= apitch * p.ny);
      CHECK(lat == size_t(19 * plane) * (p.storage == LBMHD_FP32 ? 4 : 2));
      CHECK(adj == size_t(19 * aplane) * 4);
      CHECK(lbmhd_layout(h, nullptr, nullptr, nullptr, nullptr) == LBMHD_OK);
      CHECK(lbmhd_layout(nullptr, &pitch, nullptr, nullptr, nullptr) == LBMHD_ERR_INVALID_ARG);
      CHECK(lbmhd_step(h, 1) == LBMHD_ERR_NOT_BOUND);
      CHECK(std::strlen(lbmhd_last_error(h)) > 0);
      lbmhd_diag_t d;
      CHECK(lbmhd_diag(h, &d) == LBMHD_ERR_NOT_BOUND);
      CHECK(lbmhd_run(h, 10, 5, nullptr, &d, 2) == LBMHD_ERR_NOT_BOUND);
      CHECK(lbmhd_run(h, -1, 5, nullptr, nullptr, 0) == LBMHD_ERR_NOT_BOUND);
      CHECK(lbmhd_bind(h, nullptr, 0, nullptr, 0, nullptr, 0, nullptr) == LBMHD_ERR_INVALID_ARG);
      int64_t step = -1;
      CHECK(lbmhd_get_step(h, &step) == LBMHD_OK && step == 0);
      CHECK(lbmhd_destroy(h) == LBMHD_OK);
    }
  CHECK(lbmhd_destroy(nullptr) == LBMHD_OK);
  for (int code = -6; code <= 0; ++code) CHECK(lbmhd_strerror(code) != nullptr);

  lbmhd3_params q;
  std::memset(&q, 0, sizeof(q));
  q.nx = 16; q.ny = 8; q.nz = 4; q.nu = 0.01; q.eta = 0.02; q.les = 1;
  q.cs = q.cs_b = 0.1; q.delta = 1.0;
  lbmhd3_t* h3 = nullptr;
  CHECK(lbmhd3_create(&q, &h3) == LBMHD_OK && h3 != nullptr);
  size_t lat3 = 0, ws3 = 0;
  CHECK(lbmhd3_sizes(h3, &lat3, &ws3) == LBMHD_OK && lat3 > 0 && ws3 > 0);
  CHECK(lbmhd3_step(h3, 1) == LBMHD_ERR_NOT_BOUND);
  CHECK(std::strlen(lbmhd3_last_error(h3)) > 0);
  CHECK(lbmhd3_destroy(h3) == LBMHD_OK);
  CHECK(lbmhd3_destroy(nullptr) == LBMHD_OK);
  lbmhd3_params bad = q;
  bad.nz = 0;
  h3 = nullptr;
  CHECK(lbmhd3_create(&bad, &h3) == LBMHD_ERR_INVALID_ARG && h3 == nullptr);
  bad = q;
  bad.nx = 1 << 14; bad.ny = 1 << 14; bad.nz = 8;
  CHECK(lbmhd3_create(&bad, &h3) == LBMHD_ERR_INVALID_ARG && h3 == nullptr);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
