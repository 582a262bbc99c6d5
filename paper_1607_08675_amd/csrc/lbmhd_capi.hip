// lbmhd_capi.hip -- host side of the C ABI declared in include/lbmhd.h:
// parameter validation, the handle, buffer binding and kernel sequencing.
// No exception crosses the interface; every HIP status is checked and kept.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "lbmhd_impl.h"

struct lbmhd {
  lbmhd_params p;
  lbk::Geom geo;   // state lattice
  lbk::Geom geoa;  // FP32 adjoint lattice
  lbk::Rates rates;
  size_t lattice_bytes = 0, workspace_bytes = 0, adj_lattice_bytes = 0, adj_acc_bytes = 0;
  void* lat[2] = {nullptr, nullptr};
  double* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = 0;  // index of the lattice holding the current state
  bool reversed = false;  // in-place mode: the lattice is in the reversed layout
  int64_t step = 0;
  // lbmhd_run: the stream its diagnostics passes run on, the events that
  // order them against the bound stream, and which bound lattices a pass
  // enqueued there may still be reading
  hipStream_t side = nullptr;
  hipEvent_t ev_state = nullptr, ev_diag = nullptr;
  bool reading[2] = {false, false};
  std::string err;
};

namespace {

constexpr size_t kAlign = 256;

// The eddy closure in effect: 0 none, 1 Smagorinsky-MHD, 2 cross-helicity
// (C_S = 0 makes the eddy closures the identity, tau = tau0: skip them).
int eddy_of(const lbmhd_t* h) {
  const int les = h->p.les;
  const bool on = h->p.cs > 0.0 || h->p.cs_b > 0.0;
  return (les & 1) && on ? 1 : ((les & 4) && on ? 2 : 0);
}

// Whether the update reads the neighbours' moments (kinetic closure, or the
// cross-helicity closure's vorticity).
bool reads_neighbours(const lbmhd_t* h) { return (h->p.les & 2) || eddy_of(h) == 2; }

// One step src -> dst with the handle's closure.
hipError_t launch_one_step(const lbmhd_t* h, const void* src, void* dst) {
  const int eddy = eddy_of(h);
  if (reads_neighbours(h))
    return lbk::launch_step_nb(h->p.storage, eddy, (h->p.les & 2) != 0, src, dst, h->geo,
                               h->rates, h->p.delta, h->stream);
  return lbk::launch_step(h->p.storage, eddy == 1, src, dst, h->geo, h->rates, h->stream);
}

// Two steps src -> dst in one pass (mid: also the state between them).
hipError_t launch_two_steps(const lbmhd_t* h, const void* src, void* dst, void* mid) {
  const int eddy = eddy_of(h);
  if (reads_neighbours(h))
    return lbk::launch_step_nb2(h->p.storage, eddy, (h->p.les & 2) != 0, src, dst, mid, h->geo,
                                h->rates, h->p.delta, h->stream);
  return lbk::launch_step2(h->p.storage, eddy == 1, src, dst, mid, h->geo, h->rates, h->stream);
}

// Steps that one kernel pass of lbmhd_step covers: 3 (FP32 only), 2 or 1.
// Automatic: where the multi-step kernels fill the chip, triples for FP32
// (measured faster than pairs from 1024^2 to 8192^2) and pairs for FP16; the
// closures that read the neighbours' moments take pairs with FP32 storage (at
// 4096^2, 1.9x single steps for the kinetic closure, 1.65x for the
// cross-helicity one, 1.15x for both together; with FP16 storage pairs
// measured no faster than single steps).
int pass_steps(const lbmhd_t* h) {
  const int spp = h->p.steps_per_pass;
  if (h->p.inplace || spp == 1) return 1;
  if (reads_neighbours(h)) {
    if (spp >= 2) return 2;
    return h->p.storage == LBMHD_FP32 && lbk::step_nb2_pays(h->geo) ? 2 : 1;
  }
  const bool fp32 = h->p.storage == LBMHD_FP32;
  if (spp == 3) return fp32 ? 3 : 2;
  if (spp == 2) return 2;
  if (!lbk::step2_pays(h->p.storage, h->geo)) return 1;
  return fp32 ? 3 : 2;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int fail(lbmhd_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(lbmhd_t* h, hipError_t e, const char* where) {
  return fail(h, LBMHD_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Rows are padded to whole 256-byte blocks, and successive planes are spaced
// by their ny rows plus a gap of kPlaneGap bytes.  Without the gap the planes
// of a square power-of-two lattice lie a large power of two apart (2^26 bytes
// at 4096^2 FP32), so the 19 populations of a site differ only in high address
// bits; with it the kernels that read or write all planes of a row at once ran
// 1-4% faster on MI355X, the paired reverse step 14%, with identical results.
constexpr size_t kPlaneGap = 768;

lbk::Geom make_geom(int nx, int ny, size_t esize) {
  lbk::Geom g;
  g.nx = nx;
  g.ny = ny;
  g.pitch = int(round_up(size_t(nx) * esize, kAlign) / esize);
  g.plane = (long long)g.pitch * ny + (long long)(kPlaneGap / esize);
  return g;
}

bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

// Workspace (doubles): per-block partials of the reductions, then 32 result
// slots ([0, 16) diagnostics, [16] the C_Sv sum, [17] the mismatch, [18] the
// C_Sb sum).
size_t workspace_doubles() { return size_t(lbk::kDiagBlocks) * lbk::kDiagSlots + 32; }
double* ws_out(lbmhd_t* h) { return h->ws + size_t(lbk::kDiagBlocks) * lbk::kDiagSlots; }

int need_bound(lbmhd_t* h) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  if (!h->bound) return fail(h, LBMHD_ERR_NOT_BOUND, "lbmhd_bind() has not succeeded");
  return LBMHD_OK;
}

// The bound lattice holding the current state in the natural layout: an
// in-place lattice left in the reversed layout by an odd number of steps is
// turned back first (one in-place pass).
int current(lbmhd_t* h, const void** out) {
  if (h->p.inplace && h->reversed) {
    hipError_t e = lbk::launch_unswap_aa(h->p.storage, h->lat[0], h->geo, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "layout launch");
    h->reversed = false;
  }
  *out = h->lat[h->cur];
  return LBMHD_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

// A caller-supplied state that is the bound in-place lattice must be read in
// the natural layout: turn that lattice back first if it is reversed.
int natural(lbmhd_t* h, const void* state) {
  if (h->p.inplace && h->reversed && state &&
      overlap(state, h->lattice_bytes, h->lat[0], h->lattice_bytes)) {
    const void* st = nullptr;
    return current(h, &st);
  }
  return LBMHD_OK;
}

// One reverse step (state x, lam_next -> lam_prev) with the kernels of the
// handle's closure.
hipError_t adj_one(lbmhd_t* h, const void* x, const float* from, float* to, double* acc) {
  const double d2 = h->p.delta * h->p.delta;
  const bool smag = (h->p.les & 1) != 0;
  if (h->p.les & 2)
    return lbk::launch_adj_step_kin(h->p.storage, smag, x, from, to, acc, h->geo, h->geoa,
                                    h->rates, d2, h->stream);
  return lbk::launch_adj_step(h->p.storage, smag, x, from, to, acc, h->geo, h->geoa, h->rates,
                              d2, h->stream);
}

// Whether reverse steps can go in pairs from one stored state (closures that
// read no neighbours).
bool adj_pairs_ok(const lbmhd_t* h) { return (h->p.les & 6) == 0; }

// Two reverse steps (state x_t, lam_{t+2} -> lam_t); x_{t+1} is recomputed with
// the forward collision lbmhd_step uses.
hipError_t adj_two(lbmhd_t* h, const void* x, const float* from, float* to, double* acc) {
  const double d2 = h->p.delta * h->p.delta;
  return lbk::launch_adj_step2(h->p.storage, eddy_of(h) == 1, (h->p.les & 1) != 0, x, from, to,
                               acc, h->geo, h->geoa, h->rates, d2, h->stream);
}

// Reverse sweep over n steps taken in pairs: state(t) is x_t for the even t
// (and for t = n - 1 when n is odd, whose reverse step goes first, alone).
// lam holds lam_n on entry and lam_0 on return.
template <class StateAt>
int sweep_pairs(lbmhd_t* h, int64_t n, StateAt state, float* lam, float* tmp, double* acc) {
  // the last launch must write lam
  float* from = lam;
  float* to = tmp;
  if ((n / 2 + n % 2) % 2) {
    hipError_t e = lbk::launch_copy(lam, tmp, h->adj_lattice_bytes, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy launch");
    from = tmp;
    to = lam;
  }
  int64_t t = n;
  if (n % 2) {
    hipError_t e = adj_one(h, state(n - 1), from, to, acc);
    if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
    std::swap(from, to);
    --t;
  }
  for (; t >= 2; t -= 2) {
    hipError_t e = adj_two(h, state(t - 2), from, to, acc);
    if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
    std::swap(from, to);
  }
  return LBMHD_OK;
}

// Run the diagnostics kernels on `lat` with the block partials at `part` and
// the results at `res` (the workspace unless given), and copy the 16 results
// to host.
int run_diag(lbmhd_t* h, const void* lat, double out[lbk::kDiagSlots],
             double* part = nullptr, double* res = nullptr) {
  if (!part) {
    part = h->ws;
    res = ws_out(h);
  }
  hipError_t e = lbk::launch_diag(h->p.storage, lat, part, res, h->geo, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics launch");
  e = hipMemcpyAsync(out, res, sizeof(double) * lbk::kDiagSlots, hipMemcpyDeviceToHost,
                     h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics synchronise");
  return LBMHD_OK;
}

// Diagnostics results (16 doubles) into the public struct; nonzero
// non-finite count -> LBMHD_ERR_NONFINITE.
int fill_diag(lbmhd_t* h, const double v[lbk::kDiagSlots], lbmhd_diag_t* out) {
  out->mass = v[0];
  out->mom_x = v[1];
  out->mom_y = v[2];
  out->flux_x = v[3];
  out->flux_y = v[4];
  out->e_kin = v[5];
  out->e_mag = v[6];
  out->cross_helicity = v[7];
  out->enstrophy = v[8];
  out->current_sq = v[9];
  out->nonfinite = int64_t(v[10]);
  out->max_abs_divB = v[11];
  out->max_u = v[12];
  out->step = h->step;
  if (out->nonfinite > 0)
    return fail(h, LBMHD_ERR_NONFINITE,
                std::to_string(out->nonfinite) + " sites hold non-finite populations");
  return LBMHD_OK;
}

// ------------------------------------------------ static diagnostics scratch
// lbmhd_diag_noalloc keeps the reductions' block partials (at most
// kDiagBlocks x kDiagSlots doubles) and the result slots (kDiagSlots doubles)
// here instead of in the bound workspace.  Each GPU holds its own copy; host
// code never uses the array's name as an address, only the per-device
// address from hipGetSymbolAddress.
constexpr size_t kScratchParts = size_t(lbk::kDiagBlocks);
constexpr size_t kScratchDoubles = kScratchParts * lbk::kDiagSlots + lbk::kDiagSlots;
static_assert(kScratchDoubles * sizeof(double) == 524416, "documented scratch size");
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the GPU of the handle's stream, looked up
// (with that GPU current) on the first call for that GPU.
int scratch_address(lbmhd_t* h, double** out) {
  int dev = -1;
  // the null stream belongs to the current device
  hipError_t e = h->stream ? hipStreamGetDevice(h->stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(h, e, "stream device query");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(h, LBMHD_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(h, e, "current device query");
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess)
      return hip_fail(h, e, "device switch");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    hipError_t e2 = cur != dev ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return hip_fail(h, e, "scratch address lookup");
    if (e2 != hipSuccess) return hip_fail(h, e2, "device switch back");
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return LBMHD_OK;
}

}  // namespace

extern "C" {

const char* lbmhd_strerror(int code) {
  switch (code) {
    case LBMHD_OK: return "ok";
    case LBMHD_ERR_INVALID_ARG: return "invalid argument";
    case LBMHD_ERR_NOT_BOUND: return "device buffers not bound";
    case LBMHD_ERR_HIP: return "HIP runtime error";
    case LBMHD_ERR_NONFINITE: return "non-finite populations";
    case LBMHD_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* lbmhd_last_error(const lbmhd_t* h) { return h ? h->err.c_str() : ""; }

int lbmhd_create(const lbmhd_params* p, lbmhd_t** out) {
  if (!p || !out) return LBMHD_ERR_INVALID_ARG;
  *out = nullptr;
  if (p->nx < 2 || p->ny < 2) return LBMHD_ERR_INVALID_ARG;
  if (!(p->nu > 0.0) || !(p->eta > 0.0) || !isfinite(p->nu) || !isfinite(p->eta))
    return LBMHD_ERR_INVALID_ARG;
  if (!rate_ok(p->s5) || !rate_ok(p->s6) || !rate_ok(p->s7) || !rate_ok(p->s8))
    return LBMHD_ERR_INVALID_ARG;
  if (p->s5 != p->s6) return LBMHD_ERR_INVALID_ARG;
  if (p->les < 0 || p->les > 6 || ((p->les & 1) && (p->les & 4))) return LBMHD_ERR_INVALID_ARG;
  if (!(p->cs >= 0.0) || !isfinite(p->cs) || !(p->cs_b >= 0.0) || !isfinite(p->cs_b) ||
      !(p->delta > 0.0) || !isfinite(p->delta))
    return LBMHD_ERR_INVALID_ARG;
  if (p->storage != LBMHD_FP32 && p->storage != LBMHD_FP16) return LBMHD_ERR_INVALID_ARG;
  // the in-place update keeps every site's reads and writes within its own
  // locations; closures that read the neighbours' populations cannot
  if (p->inplace != 0 && p->inplace != 1) return LBMHD_ERR_INVALID_ARG;
  if (p->inplace && (p->les & 6)) return LBMHD_ERR_INVALID_ARG;
  if (p->steps_per_pass < 0 || p->steps_per_pass > 3) return LBMHD_ERR_INVALID_ARG;
  // cross-helicity closure: as tau_m0 = 3 eta + 1/2 approaches 3/2, the clip
  // of the magnetic relaxation time approaches a double root of its cubic,
  // where the kernel's Newton steps converge only linearly; up to
  // tau_m0 = 5/4 six steps land within 1e-6 of the root (measured)
  if ((p->les & 4) && 3.0 * p->eta + 0.5 > 1.25) return LBMHD_ERR_UNSUPPORTED;
  const size_t esize = p->storage == LBMHD_FP32 ? 4 : 2;
  lbk::Geom g = make_geom(p->nx, p->ny, esize);
  lbk::Geom ga = make_geom(p->nx, p->ny, 4);
  // in-plane byte offsets are 32-bit unsigned in the kernels (FP32 adjoint
  // planes are the largest)
  if ((unsigned long long)ga.plane * 4ull >= (1ull << 32)) return LBMHD_ERR_INVALID_ARG;

  lbmhd_t* h = new (std::nothrow) lbmhd;
  if (!h) return LBMHD_ERR_INVALID_ARG;
  h->p = *p;
  h->geo = g;
  h->geoa = ga;
  const double tau0 = 3.0 * p->nu + 0.5, taum0 = 3.0 * p->eta + 0.5;
  const double d2 = p->delta * p->delta;
  lbk::Rates& r = h->rates;
  r.s3q = float(0.25 / tau0);
  r.s5q = float(p->s5 / 12.0);
  r.s7q = float(p->s7 / 180.0);
  r.s8q = float(p->s8 / 20.0);
  r.sm = float(1.0 / taum0);
  r.tau0 = float(tau0);
  r.tau0sq = float(tau0 * tau0);
  r.taum0 = float(taum0);
  r.taum0sq = float(taum0 * taum0);
  r.cf = float(18.0 * p->cs * d2);
  r.cm = float(36.0 * p->cs_b * d2);
  r.tau0d = 2.0f * r.tau0;
  r.tau0dsq = 4.0f * r.tau0sq;
  r.cf4 = 4.0f * r.cf;
  r.taum0h = 0.5f * r.taum0;
  r.taum0hsq = 0.25f * r.taum0sq;
  r.cmq = 0.25f * r.cm;
  r.stau0 = float(std::sqrt(tau0));
  r.staum0 = float(std::sqrt(taum0));
  r.kv = float(4.5 * p->cs * d2);
  r.kb = float(3.0 * std::sqrt(3.0) * p->cs_b * d2);
  // the largest root of t^3 - tau_m0 t - q is below t* = max(sqrt(1/2),
  // sqrt(tau_m0 / 3)) (or absent) exactly when q < t*^3 - tau_m0 t*
  const double ts = std::max(std::sqrt(0.5), std::sqrt(taum0 / 3.0));
  r.qclip = float(ts * ts * ts - taum0 * ts);
  h->lattice_bytes = size_t(lbk::kNPop) * size_t(g.plane) * esize;
  h->adj_lattice_bytes = size_t(lbk::kNPop) * size_t(ga.plane) * 4;
  h->workspace_bytes = round_up(workspace_doubles() * sizeof(double), kAlign);
  h->adj_acc_bytes = round_up(2 * size_t(lbk::adj_step_blocks(g)) * sizeof(double), kAlign);
  *out = h;
  return LBMHD_OK;
}

int lbmhd_destroy(lbmhd_t* h) {
  if (h && h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h && h->ev_state) (void)hipEventDestroy(h->ev_state);
  if (h && h->ev_diag) (void)hipEventDestroy(h->ev_diag);
  delete h;
  return LBMHD_OK;
}

int lbmhd_sizes(const lbmhd_t* h, size_t* lattice, size_t* workspace, size_t* adj_lattice,
                size_t* adj_acc) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  if (lattice) *lattice = h->lattice_bytes;
  if (workspace) *workspace = h->workspace_bytes;
  if (adj_lattice) *adj_lattice = h->adj_lattice_bytes;
  if (adj_acc) *adj_acc = h->adj_acc_bytes;
  return LBMHD_OK;
}

int lbmhd_layout(const lbmhd_t* h, int64_t* pitch, int64_t* plane, int64_t* adj_pitch,
                 int64_t* adj_plane) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  if (pitch) *pitch = h->geo.pitch;
  if (plane) *plane = h->geo.plane;
  if (adj_pitch) *adj_pitch = h->geoa.pitch;
  if (adj_plane) *adj_plane = h->geoa.plane;
  return LBMHD_OK;
}

int lbmhd_bind(lbmhd_t* h, void* lat_a, size_t lat_a_bytes, void* lat_b, size_t lat_b_bytes,
               void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  h->bound = false;
  if (h->p.inplace) {  // one lattice: lat_b is not used
    lat_b = nullptr;
    lat_b_bytes = 0;
  }
  if (!lat_a || (!lat_b && !h->p.inplace) || !workspace)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null buffer passed to lbmhd_bind");
  if (lat_a_bytes < h->lattice_bytes || (!h->p.inplace && lat_b_bytes < h->lattice_bytes) ||
      workspace_bytes < h->workspace_bytes)
    return fail(h, LBMHD_ERR_INVALID_ARG, "buffer smaller than lbmhd_sizes() requires");
  if (!aligned(lat_a) || (lat_b && !aligned(lat_b)) || !aligned(workspace))
    return fail(h, LBMHD_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
  if (overlap(lat_a, h->lattice_bytes, workspace, h->workspace_bytes) ||
      (lat_b && (overlap(lat_a, h->lattice_bytes, lat_b, h->lattice_bytes) ||
                 overlap(lat_b, h->lattice_bytes, workspace, h->workspace_bytes))))
    return fail(h, LBMHD_ERR_INVALID_ARG, "bound buffers overlap");
  h->lat[0] = lat_a;
  h->lat[1] = lat_b;
  h->ws = static_cast<double*>(workspace);
  h->stream = static_cast<hipStream_t>(stream);
  h->cur = 0;
  h->reversed = false;
  h->step = 0;
  h->bound = true;
  return LBMHD_OK;
}

int lbmhd_init_fields(lbmhd_t* h, const double* rho, const double* ux, const double* uy,
                      const double* bx, const double* by) {
  if (int rc = need_bound(h)) return rc;
  if (!rho || !ux || !uy || !bx || !by) return fail(h, LBMHD_ERR_INVALID_ARG, "null field");
  hipError_t e = lbk::launch_init(h->p.storage, rho, ux, uy, bx, by, h->lat[0], h->geo,
                                    h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "init launch");
  h->cur = 0;
  h->reversed = false;
  h->step = 0;
  return LBMHD_OK;
}

int lbmhd_steps_per_pass(const lbmhd_t* h, int32_t* out) {
  if (!h || !out) return LBMHD_ERR_INVALID_ARG;
  *out = pass_steps(h);
  return LBMHD_OK;
}

// Before a pass writes bound lattice i: if a diagnostics pass of lbmhd_run
// may still read it, the bound stream waits for the last one enqueued (the
// side stream runs them in order, so that covers every earlier one too).
int before_write(lbmhd_t* h, int i) {
  if (!h->reading[i]) return LBMHD_OK;
  h->reading[0] = h->reading[1] = false;
  hipError_t e = hipStreamWaitEvent(h->stream, h->ev_diag, 0);
  return e == hipSuccess ? LBMHD_OK : hip_fail(h, e, "diagnostics wait");
}

int lbmhd_step(lbmhd_t* h, int64_t nsteps) {
  if (int rc = need_bound(h)) return rc;
  if (nsteps < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "negative step count");
  const bool les = (h->p.les & 1) && (h->p.cs > 0.0 || h->p.cs_b > 0.0);
  int64_t t = 0;
  const int ps = pass_steps(h);
  if (ps == 3) {
    // a remainder of two steps is one pair, of one step a single step: a
    // triple and a single step took 5-8% less time than two pairs from 2048^2
    // to 8192^2 on MI355X (as long at 1024^2)
    for (; t + 3 <= nsteps; t += 3) {
      if (int rc = before_write(h, 1 - h->cur)) return rc;
      hipError_t e = lbk::launch_step_t3(les, h->lat[h->cur], h->lat[1 - h->cur], nullptr,
                                         nullptr, h->geo, h->rates, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "step launch");
      h->cur = 1 - h->cur;
      h->step += 3;
    }
  }
  if (ps >= 2) {
    for (; t + 2 <= nsteps; t += 2) {
      if (int rc = before_write(h, 1 - h->cur)) return rc;
      hipError_t e = launch_two_steps(h, h->lat[h->cur], h->lat[1 - h->cur], nullptr);
      if (e != hipSuccess) return hip_fail(h, e, "step launch");
      h->cur = 1 - h->cur;
      h->step += 2;
    }
  }
  for (; t < nsteps; ++t) {
    if (int rc = before_write(h, h->p.inplace ? 0 : 1 - h->cur)) return rc;
    hipError_t e;
    if (h->p.inplace) {
      e = lbk::launch_step_aa(h->p.storage, les, h->reversed ? 1 : 0, h->lat[0], h->geo,
                              h->rates, h->stream);
      h->reversed = !h->reversed;
    } else {
      e = launch_one_step(h, h->lat[h->cur], h->lat[1 - h->cur]);
      h->cur = 1 - h->cur;
    }
    if (e != hipSuccess) return hip_fail(h, e, "step launch");
    ++h->step;
  }
  return LBMHD_OK;
}

int lbmhd_step_between(lbmhd_t* h, const void* src, void* dst) {
  if (int rc = need_bound(h)) return rc;
  if (!src || !dst || !aligned(src) || !aligned(dst))
    return fail(h, LBMHD_ERR_INVALID_ARG, "null or unaligned lattice");
  if (overlap(src, h->lattice_bytes, dst, h->lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "src and dst overlap");
  for (const void* b : {(const void*)h->lat[0], (const void*)h->lat[1]})
    if (b && overlap(dst, h->lattice_bytes, b, h->lattice_bytes))
      return fail(h, LBMHD_ERR_INVALID_ARG, "dst overlaps a bound lattice");
  if (int rc = natural(h, src)) return rc;
  hipError_t e = launch_one_step(h, src, dst);
  if (e != hipSuccess) return hip_fail(h, e, "step launch");
  return LBMHD_OK;
}

int lbmhd_step_store(lbmhd_t* h, const void* src, void* store, size_t stride, int64_t n) {
  if (int rc = need_bound(h)) return rc;
  if (n < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "negative step count");
  if (n == 0) return LBMHD_OK;
  if (!src || !store || !aligned(src) || !aligned(store))
    return fail(h, LBMHD_ERR_INVALID_ARG, "null or unaligned lattice");
  if (stride < h->lattice_bytes || stride % kAlign != 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "stride below the lattice size or not 256-aligned");
  if (size_t(n - 1) > (SIZE_MAX - h->lattice_bytes) / stride)
    return fail(h, LBMHD_ERR_INVALID_ARG, "store range overflows");
  const size_t span = size_t(n - 1) * stride + h->lattice_bytes;
  if (overlap(src, h->lattice_bytes, store, span))
    return fail(h, LBMHD_ERR_INVALID_ARG, "store overlaps src");
  for (const void* b : {(const void*)h->lat[0], (const void*)h->lat[1], (const void*)h->ws})
    if (b && overlap(store, span, b, b == h->ws ? h->workspace_bytes : h->lattice_bytes))
      return fail(h, LBMHD_ERR_INVALID_ARG, "store overlaps a bound buffer");
  if (int rc = natural(h, src)) return rc;
  const char* prev = static_cast<const char*>(src);
  char* out = static_cast<char*>(store);
  int64_t t = 0;
  const bool les = (h->p.les & 1) && (h->p.cs > 0.0 || h->p.cs_b > 0.0);
  // triples (FP32) that also store both intermediate states; a remainder of
  // one step goes with the last triple as two pairs
  if (pass_steps(h) == 3) {
    int64_t triples = n / 3;
    if (n % 3 == 1 && triples > 0) --triples;
    for (; t < 3 * triples; t += 3) {
      hipError_t e = lbk::launch_step_t3(les, prev, out + 2 * stride, out, out + stride, h->geo,
                                         h->rates, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "step launch");
      prev = out + 2 * stride;
      out += 3 * stride;
    }
  }
  // pairs of steps in one pass that stores the intermediate state too; in
  // automatic mode for FP32 only (with FP16 the extra store made the pass
  // slower than two single steps: 75 against 64 us per step at 2048^2)
  if (pass_steps(h) >= 2 && (h->p.storage == LBMHD_FP32 || h->p.steps_per_pass >= 2)) {
    for (; t + 2 <= n; t += 2) {
      hipError_t e = launch_two_steps(h, prev, out + stride, out);
      if (e != hipSuccess) return hip_fail(h, e, "step launch");
      prev = out + stride;
      out += 2 * stride;
    }
  }
  for (; t < n; ++t) {
    hipError_t e = launch_one_step(h, prev, out);
    if (e != hipSuccess) return hip_fail(h, e, "step launch");
    prev = out;
    out += stride;
  }
  return LBMHD_OK;
}

int lbmhd_step_store_pairs(lbmhd_t* h, const void* src, void* store, size_t stride,
                           int64_t npairs) {
  if (int rc = need_bound(h)) return rc;
  if (npairs < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "negative pair count");
  if (npairs == 0) return LBMHD_OK;
  if (!src || !store || !aligned(src) || !aligned(store))
    return fail(h, LBMHD_ERR_INVALID_ARG, "null or unaligned lattice");
  if (stride < h->lattice_bytes || stride % kAlign != 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "stride below the lattice size or not 256-aligned");
  if (size_t(npairs - 1) > (SIZE_MAX - h->lattice_bytes) / stride)
    return fail(h, LBMHD_ERR_INVALID_ARG, "store range overflows");
  const size_t span = size_t(npairs - 1) * stride + h->lattice_bytes;
  if (overlap(src, h->lattice_bytes, store, span))
    return fail(h, LBMHD_ERR_INVALID_ARG, "store overlaps src");
  for (const void* b : {(const void*)h->lat[0], (const void*)h->lat[1], (const void*)h->ws})
    if (b && overlap(store, span, b, b == h->ws ? h->workspace_bytes : h->lattice_bytes))
      return fail(h, LBMHD_ERR_INVALID_ARG, "store overlaps a bound buffer");
  if (int rc = natural(h, src)) return rc;
  const char* prev = static_cast<const char*>(src);
  char* out = static_cast<char*>(store);
  for (int64_t k = 0; k < npairs; ++k) {
    hipError_t e = launch_two_steps(h, prev, out, nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "step launch");
    prev = out;
    out += stride;
  }
  return LBMHD_OK;
}

int lbmhd_macro(lbmhd_t* h, double* rho, double* ux, double* uy, double* bx, double* by) {
  if (int rc = need_bound(h)) return rc;
  if (!rho || !ux || !uy || !bx || !by) return fail(h, LBMHD_ERR_INVALID_ARG, "null field");
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  hipError_t e = lbk::launch_macro(h->p.storage, st, rho, ux, uy, bx, by, h->geo, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "macro launch");
  return LBMHD_OK;
}

int lbmhd_macro_box(lbmhd_t* h, int32_t w, double* rho, double* ux, double* uy, double* bx,
                    double* by) {
  if (int rc = need_bound(h)) return rc;
  if (!rho || !ux || !uy || !bx || !by) return fail(h, LBMHD_ERR_INVALID_ARG, "null field");
  if (w < 1 || h->p.nx % w != 0 || h->p.ny % w != 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "box width must divide nx and ny");
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  hipError_t e = lbk::launch_macro_box(h->p.storage, st, w, rho, ux, uy, bx, by, h->geo,
                                       h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "box macro launch");
  return LBMHD_OK;
}

int lbmhd_mismatch(lbmhd_t* h, const void* state, const double* ux_t, const double* uy_t,
                   const double* bx_t, const double* by_t, double* L) {
  if (int rc = need_bound(h)) return rc;
  if (!ux_t || !uy_t || !bx_t || !by_t || !L)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null target or output");
  double* part = h->ws;  // the partials area of the reductions
  double* dev = ws_out(h) + lbk::kDiagSlots + 1;
  if (!state) {
    if (int rc = current(h, &state)) return rc;
  } else if (int rc = natural(h, state)) {
    return rc;
  }
  hipError_t e = lbk::launch_mismatch(h->p.storage, state, ux_t, uy_t, bx_t, by_t, part, dev,
                                      h->geo, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "mismatch launch");
  e = hipMemcpyAsync(L, dev, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "mismatch copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "mismatch synchronise");
  return LBMHD_OK;
}

int lbmhd_diag(lbmhd_t* h, lbmhd_diag_t* out) {
  if (int rc = need_bound(h)) return rc;
  if (!out) return fail(h, LBMHD_ERR_INVALID_ARG, "null output");
  double v[lbk::kDiagSlots];
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  if (int rc = run_diag(h, st, v)) return rc;
  return fill_diag(h, v, out);
}

// The diagnostics of the state just reached, enqueued without waiting on the
// host: results to dev (16 doubles).  With two lattices the pass runs on the
// side stream after the bound stream's work so far, and the lattice it reads
// is marked so that the next pass that writes it waits for it; an in-place
// lattice (whose next pass rewrites it) is read on the bound stream.
int enqueue_diag(lbmhd_t* h, double* dev) {
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  hipError_t e;
  if (h->p.inplace) {
    e = lbk::launch_diag(h->p.storage, st, h->ws, dev, h->geo, h->stream);
    return e == hipSuccess ? LBMHD_OK : hip_fail(h, e, "diagnostics launch");
  }
  if ((e = hipEventRecord(h->ev_state, h->stream)) != hipSuccess ||
      (e = hipStreamWaitEvent(h->side, h->ev_state, 0)) != hipSuccess)
    return hip_fail(h, e, "diagnostics ordering");
  // whatever of the pass got enqueued, later writes of the lattice wait for it
  const hipError_t el = lbk::launch_diag(h->p.storage, st, h->ws, dev, h->geo, h->side);
  if ((e = hipEventRecord(h->ev_diag, h->side)) != hipSuccess)
    return hip_fail(h, e, "diagnostics ordering");
  h->reading[h->cur] = true;
  return el == hipSuccess ? LBMHD_OK : hip_fail(h, el, "diagnostics launch");
}

int lbmhd_run(lbmhd_t* h, int64_t nsteps, int64_t every, double* dev, lbmhd_diag_t* out,
              int64_t nout) {
  if (int rc = need_bound(h)) return rc;
  if (nsteps < 0 || every < 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "negative step count or interval");
  if (every == 0 || nsteps < every) return lbmhd_step(h, nsteps);
  const int64_t nd = nsteps / every;
  if (!dev || !out || nout < nd)
    return fail(h, LBMHD_ERR_INVALID_ARG, "diagnostics buffers missing or too small");
  const size_t dev_bytes = size_t(nd) * lbk::kDiagSlots * sizeof(double);
  if (reinterpret_cast<uintptr_t>(dev) % alignof(double) != 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "unaligned diagnostics buffer");
  for (const void* b : {(const void*)h->lat[0], (const void*)h->lat[1]})
    if (b && overlap(dev, dev_bytes, b, h->lattice_bytes))
      return fail(h, LBMHD_ERR_INVALID_ARG, "diagnostics buffer overlaps a bound lattice");
  if (overlap(dev, dev_bytes, h->ws, h->workspace_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "diagnostics buffer overlaps the workspace");
  // an interval that lbmhd_step ends with a single step (FP32 storage, a
  // closure without neighbour terms) takes that step and the diagnostics of
  // its result in one pass on the bound stream
  const int ps = pass_steps(h);
  const bool fuse = !h->p.inplace && h->p.storage == LBMHD_FP32 && !reads_neighbours(h) &&
                    (ps == 1 || every % ps == 1);
  if (!h->p.inplace && !fuse && !h->side) {
    hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_state, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_diag, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(h, e, "diagnostics stream");
  }
  std::vector<int64_t> at(size_t(nd), 0);
  int rc = LBMHD_OK;
  for (int64_t k = 0; k < nd && rc == LBMHD_OK; ++k) {
    if (fuse) {
      rc = lbmhd_step(h, every - 1);
      // the pass writes the workspace partials and the other lattice
      if (rc == LBMHD_OK) rc = before_write(h, 0);
      if (rc == LBMHD_OK) rc = before_write(h, 1);
      if (rc == LBMHD_OK) {
        hipError_t e = lbk::launch_step_diag(eddy_of(h) == 1, h->lat[h->cur], h->lat[1 - h->cur],
                                             h->ws, dev + k * lbk::kDiagSlots, h->geo, h->rates,
                                             h->stream);
        if (e != hipSuccess) {
          rc = hip_fail(h, e, "step and diagnostics launch");
        } else {
          h->cur = 1 - h->cur;
          ++h->step;
        }
      }
    } else {
      rc = lbmhd_step(h, every);
      if (rc == LBMHD_OK) rc = enqueue_diag(h, dev + k * lbk::kDiagSlots);
    }
    at[size_t(k)] = h->step;
  }
  if (rc == LBMHD_OK) rc = lbmhd_step(h, nsteps - nd * every);
  // later work on the bound stream (and the copy below) follows every pass
  if (h->reading[0] || h->reading[1]) {
    h->reading[0] = h->reading[1] = false;
    hipError_t e = hipStreamWaitEvent(h->stream, h->ev_diag, 0);
    if (e != hipSuccess && rc == LBMHD_OK) rc = hip_fail(h, e, "diagnostics wait");
  }
  if (rc != LBMHD_OK) return rc;
  std::vector<double> v(size_t(nd) * lbk::kDiagSlots);
  hipError_t e = hipMemcpyAsync(v.data(), dev, dev_bytes, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics copy");
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess)
    return hip_fail(h, e, "diagnostics synchronise");
  const int64_t now = h->step;
  for (int64_t k = 0; k < nd; ++k) {
    h->step = at[size_t(k)];
    const int r = fill_diag(h, v.data() + k * lbk::kDiagSlots, out + k);
    if (r != LBMHD_OK && rc == LBMHD_OK) rc = r;
  }
  h->step = now;
  return rc;
}

int lbmhd_diag_noalloc(lbmhd_t* h, lbmhd_diag_t* out) {
  if (int rc = need_bound(h)) return rc;
  if (!out) return fail(h, LBMHD_ERR_INVALID_ARG, "null output");
  if (size_t(lbk::diag_partials(h->geo)) > kScratchParts)
    return fail(h, LBMHD_ERR_UNSUPPORTED, "more reduction partials than the static scratch holds");
  double* s = nullptr;
  if (int rc = scratch_address(h, &s)) return rc;
  double v[lbk::kDiagSlots];
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  if (int rc = run_diag(h, st, v, s, s + kScratchParts * lbk::kDiagSlots)) return rc;
  return fill_diag(h, v, out);
}

int lbmhd_get_populations(lbmhd_t* h, double* out) {
  if (int rc = need_bound(h)) return rc;
  if (!out) return fail(h, LBMHD_ERR_INVALID_ARG, "null output");
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  hipError_t e = lbk::launch_decode(h->p.storage, st, out, h->geo, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "decode launch");
  return LBMHD_OK;
}

int lbmhd_set_populations(lbmhd_t* h, const double* in, int64_t step) {
  if (int rc = need_bound(h)) return rc;
  if (!in || step < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "null input or negative step");
  hipError_t e = lbk::launch_encode(h->p.storage, in, h->lat[0], h->geo, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "encode launch");
  h->cur = 0;
  h->reversed = false;
  h->step = step;
  return LBMHD_OK;
}

int lbmhd_save_state(lbmhd_t* h, void* dst) {
  if (int rc = need_bound(h)) return rc;
  if (!dst || !aligned(dst)) return fail(h, LBMHD_ERR_INVALID_ARG, "null or unaligned dst");
  const void* st = nullptr;
  if (int rc = current(h, &st)) return rc;
  hipError_t e = lbk::launch_copy(st, dst, h->lattice_bytes, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "copy launch");
  return LBMHD_OK;
}

int lbmhd_load_state(lbmhd_t* h, const void* src, int64_t step) {
  if (int rc = need_bound(h)) return rc;
  if (!src || !aligned(src) || step < 0)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null or unaligned src, or negative step");
  // src may be the bound lattice itself (then nothing moves) but not a range
  // that partly overlaps it
  if (src != h->lat[0] && overlap(src, h->lattice_bytes, h->lat[0], h->lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "src partly overlaps the bound lattice");
  // an in-place lattice left reversed by an odd step count is read naturally
  if (int rc = natural(h, src)) return rc;
  if (src != h->lat[0]) {
    hipError_t e = lbk::launch_copy(src, h->lat[0], h->lattice_bytes, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy launch");
  }
  h->cur = 0;
  h->reversed = false;
  h->step = step;
  return LBMHD_OK;
}

int lbmhd_get_step(const lbmhd_t* h, int64_t* step) {
  if (!h || !step) return LBMHD_ERR_INVALID_ARG;
  *step = h->step;
  return LBMHD_OK;
}

int lbmhd_current_state(const lbmhd_t* h, const void** out) {
  if (!h || !out) return LBMHD_ERR_INVALID_ARG;
  if (!h->lat[0]) return LBMHD_ERR_NOT_BOUND;
  *out = h->p.inplace ? h->lat[0] : h->lat[h->cur];
  return LBMHD_OK;
}

int lbmhd_energy(lbmhd_t* h, const void* state, double* J) {
  if (int rc = need_bound(h)) return rc;
  if (!J) return fail(h, LBMHD_ERR_INVALID_ARG, "null output");
  double v[lbk::kDiagSlots];
  if (!state) {
    if (int rc = current(h, &state)) return rc;
  } else if (int rc = natural(h, state)) {
    return rc;
  }
  if (int rc = run_diag(h, state, v)) return rc;
  *J = v[5] + v[6];
  return LBMHD_OK;
}

int lbmhd_adj_seed_energy(lbmhd_t* h, const void* state, float* lam) {
  if (int rc = need_bound(h)) return rc;
  if (!state || !lam) return fail(h, LBMHD_ERR_INVALID_ARG, "null state or lambda");
  if (int rc = natural(h, state)) return rc;
  hipError_t e = lbk::launch_adj_seed(h->p.storage, state, lam, h->geo, h->geoa, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint seed launch");
  return LBMHD_OK;
}

int lbmhd_adj_seed_mismatch(lbmhd_t* h, const void* state, const double* ux_t,
                            const double* uy_t, const double* bx_t, const double* by_t,
                            double scale, float* lam) {
  if (int rc = need_bound(h)) return rc;
  if (!state || !ux_t || !uy_t || !bx_t || !by_t || !lam)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  if (int rc = natural(h, state)) return rc;
  hipError_t e = lbk::launch_adj_seed_mismatch(h->p.storage, state, ux_t, uy_t, bx_t, by_t, scale,
                                               lam, h->geo, h->geoa, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "mismatch seed launch");
  return LBMHD_OK;
}

int lbmhd_adj_step(lbmhd_t* h, const void* state_n, const float* lam_next, float* lam_prev,
                   double* acc) {
  if (int rc = need_bound(h)) return rc;
  if (h->p.les & 4)
    return fail(h, LBMHD_ERR_UNSUPPORTED,
                "the adjoint of the cross-helicity closure is not provided");
  if (!state_n || !lam_next || !lam_prev || !acc)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  if (overlap(lam_next, h->adj_lattice_bytes, lam_prev, h->adj_lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "lam_prev overlaps lam_next");
  if (int rc = natural(h, state_n)) return rc;
  hipError_t e = adj_one(h, state_n, lam_next, lam_prev, acc);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
  return LBMHD_OK;
}

int lbmhd_adj_sweep(lbmhd_t* h, const void* src, const void* store, size_t stride, int64_t n,
                    float* lam, float* tmp, double* acc) {
  if (int rc = need_bound(h)) return rc;
  if (h->p.les & 4)
    return fail(h, LBMHD_ERR_UNSUPPORTED,
                "the adjoint of the cross-helicity closure is not provided");
  if (n < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "negative step count");
  if (n == 0) return LBMHD_OK;
  if (!src || !lam || !tmp || !acc || (n > 1 && !store))
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  if (n > 1 && (stride < h->lattice_bytes || stride % kAlign != 0))
    return fail(h, LBMHD_ERR_INVALID_ARG, "stride below the lattice size or not 256-aligned");
  if (overlap(lam, h->adj_lattice_bytes, tmp, h->adj_lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "tmp overlaps lam");
  if (int rc = natural(h, src)) return rc;
  if (adj_pairs_ok(h) && lbk::adj_step2_pays(h->geo)) {
    const char* base = static_cast<const char*>(store);
    return sweep_pairs(h, n, [&](int64_t t) -> const void* {
      return t == 0 ? src : base + size_t(t - 1) * stride;
    }, lam, tmp, acc);
  }
  // the last step must write lam: with an odd count the sweep starts from tmp
  float* from = lam;
  float* to = tmp;
  if (n % 2) {
    hipError_t e = lbk::launch_copy(lam, tmp, h->adj_lattice_bytes, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy launch");
    from = tmp;
    to = lam;
  }
  for (int64_t t = n - 1; t >= 0; --t) {
    const void* x = t == 0 ? src : static_cast<const char*>(store) + size_t(t - 1) * stride;
    hipError_t e = adj_one(h, x, from, to, acc);
    if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
    std::swap(from, to);
  }
  return LBMHD_OK;
}

int lbmhd_adj_step2(lbmhd_t* h, const void* state_t, const float* lam_next, float* lam_prev,
                    double* acc) {
  if (int rc = need_bound(h)) return rc;
  if (!adj_pairs_ok(h))
    return fail(h, LBMHD_ERR_UNSUPPORTED,
                "paired reverse steps are provided for les = 0 and 1 only");
  if (!state_t || !lam_next || !lam_prev || !acc)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  if (overlap(lam_next, h->adj_lattice_bytes, lam_prev, h->adj_lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "lam_prev overlaps lam_next");
  if (int rc = natural(h, state_t)) return rc;
  hipError_t e = adj_two(h, state_t, lam_next, lam_prev, acc);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint step launch");
  return LBMHD_OK;
}

int lbmhd_adj_sweep_pairs(lbmhd_t* h, const void* src, const void* store, size_t stride,
                          int64_t n, float* lam, float* tmp, double* acc) {
  if (int rc = need_bound(h)) return rc;
  if (!adj_pairs_ok(h))
    return fail(h, LBMHD_ERR_UNSUPPORTED,
                "paired reverse steps are provided for les = 0 and 1 only");
  if (n < 0) return fail(h, LBMHD_ERR_INVALID_ARG, "negative step count");
  if (n == 0) return LBMHD_OK;
  if (!src || !lam || !tmp || !acc || (n > 2 && !store))
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  if (n > 2 && (stride < h->lattice_bytes || stride % kAlign != 0))
    return fail(h, LBMHD_ERR_INVALID_ARG, "stride below the lattice size or not 256-aligned");
  if (overlap(lam, h->adj_lattice_bytes, tmp, h->adj_lattice_bytes))
    return fail(h, LBMHD_ERR_INVALID_ARG, "tmp overlaps lam");
  if (int rc = natural(h, src)) return rc;
  const char* base = static_cast<const char*>(store);
  return sweep_pairs(h, n, [&](int64_t t) -> const void* {
    return t == 0 ? src : base + size_t(t / 2 - 1) * stride;
  }, lam, tmp, acc);
}

int lbmhd_adj_acc_total(lbmhd_t* h, const double* acc, double* out) {
  if (int rc = need_bound(h)) return rc;
  if (!acc || !out) return fail(h, LBMHD_ERR_INVALID_ARG, "null argument");
  // workspace tail: [16] the C_Sv sum, [17] the mismatch, [18] the C_Sb sum
  double* dev = ws_out(h) + lbk::kDiagSlots;
  const long long nb = lbk::adj_step_blocks(h->geo);
  hipError_t e = lbk::launch_sum(acc, nb, dev, h->stream);
  if (e == hipSuccess) e = lbk::launch_sum(acc + nb, nb, dev + 2, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sum launch");
  e = hipMemcpyAsync(out, dev, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out + 1, dev + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sum copy");
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "sum synchronise");
  return LBMHD_OK;
}

int lbmhd_adj_fields(lbmhd_t* h, const float* lam0, const double* rho0, const double* ux0,
                     const double* uy0, const double* bx0, const double* by0, double* g_ux,
                     double* g_uy, double* g_bx, double* g_by) {
  if (int rc = need_bound(h)) return rc;
  if (!lam0 || !rho0 || !ux0 || !uy0 || !bx0 || !by0 || !g_ux || !g_uy || !g_bx || !g_by)
    return fail(h, LBMHD_ERR_INVALID_ARG, "null adjoint argument");
  hipError_t e = lbk::launch_adj_fields(lam0, rho0, ux0, uy0, bx0, by0, g_ux, g_uy, g_bx, g_by,
                                          h->geoa, h->p.nx, h->p.ny, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "adjoint fields launch");
  return LBMHD_OK;
}

}  // extern "C"
