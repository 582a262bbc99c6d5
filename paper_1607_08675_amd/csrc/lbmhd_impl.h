// lbmhd_impl.h -- internal declarations shared by the kernels and the C ABI
// of the gfx950 lattice Boltzmann MHD library (not installed, not part of
// the public interface in include/lbmhd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbmhd.h"

namespace lbk {

// Device layout of one lattice: 19 planes, each ny rows of `pitch` elements
// (pitch >= nx, a multiple of 256 bytes), plane stride `plane` elements.
struct Geom {
  int nx, ny;
  int pitch;
  long long plane;
};

// Collision constants, precomputed on the host in FP64 and rounded once.
struct Rates {
  float s3q;      // s_3 / 4 with s_3 = s_4 = 1 / tau0 (fixed-rate case)
  float s5q;      // s_5 / 12 (= s_6 / 12)
  float s7q;      // s_7 / 180
  float s8q;      // s_8 / 20
  float sm;       // s_m = 1 / tau_m0 (fixed-rate case)
  float tau0;     // 3 nu + 1/2
  float tau0sq;   // tau0^2
  float taum0;    // 3 eta + 1/2
  float taum0sq;  // tau_m0^2
  float cf;       // 18 C_S Delta^2
  float cm;       // 36 C_S Delta^2
  // the same constants scaled by powers of two (exact), as the forward
  // collision uses them: 1 / (4 tau) = 1 / (tau0d + sqrt(tau0dsq + cf4 Q / rho)),
  // 1 / tau_m = 1 / (taum0h + sqrt(taum0hsq + cmq |A|))
  float tau0d;    // 2 tau0
  float tau0dsq;  // 4 tau0^2
  float cf4;      // 4 cf
  float taum0h;   // tau_m0 / 2
  float taum0hsq; // tau_m0^2 / 4
  float cmq;      // cm / 4
  // cross-helicity closure: sqrt(tau) and sqrt(tau_m) are the largest roots
  // of t^3 - p t - q = 0 (p = tau0, tau_m0)
  float stau0;    // sqrt(tau0)
  float staum0;   // sqrt(tau_m0)
  float kv;       // (9/2) C_S Delta^2:  q_v = kv (|P| / (rho tau_m))^(1/2)
  float kb;       // 3 sqrt(3) C_S Delta^2:  q_b = -kb sgn(X) |X|^(1/2)
  float qclip;    // q_b below which the root lies under max(sqrt(1/2), sqrt(tau_m0/3))
};

constexpr int kNPop = 19;
constexpr int kDiagSlots = 16;   // doubles per diagnostics partial
constexpr int kDiagBlocks = 4096; // partials in the workspace (one per reducing block)

// Forward step: dst = C(S(src)).
hipError_t launch_step(int storage, bool les, const void* src, void* dst, const Geom& g,
                       const Rates& r, hipStream_t s);
// Two forward steps in one pass: dst = C(S(C(S(src)))), equal to two
// launch_step calls; with mid != nullptr the intermediate state C(S(src)) is
// stored there as well.  src, dst and mid must not overlap.
hipError_t launch_step2(int storage, bool les, const void* src, void* dst, void* mid,
                        const Geom& g, const Rates& r, hipStream_t s);
// Three forward steps in one pass, FP32 storage only: dst = (C S)^3 src,
// equal to three launch_step calls; with mid1, mid2 != nullptr the states
// after one and two steps are stored there too.  The buffers do not overlap.
hipError_t launch_step_t3(bool les, const void* src, void* dst, void* mid1, void* mid2,
                          const Geom& g, const Rates& r, hipStream_t s);
// Whether launch_step2 beats two launch_step calls on this lattice: it needs
// enough blocks to fill the chip (measured crossover: 1024^2 FP32, 2048^2 FP16).
bool step2_pays(int storage, const Geom& g);
// In-place step on one lattice (AA pattern): phase 0 takes the natural
// layout to the reversed one, phase 1 back; launch_unswap_aa turns a
// reversed layout into the natural one in place.
hipError_t launch_step_aa(int storage, bool les, int phase, void* lat, const Geom& g,
                          const Rates& r, hipStream_t s);
hipError_t launch_unswap_aa(int storage, void* lat, const Geom& g, hipStream_t s);
// Forward step that needs the neighbours' rho, j, B (lattice gradients):
// the kinetic closure (kin: filtered equilibria, filter width delta) and/or
// the eddy closure `eddy` (0 none, 1 Smagorinsky, 2 cross-helicity).
hipError_t launch_step_nb(int storage, int eddy, bool kin, const void* src, void* dst,
                          const Geom& g, const Rates& r, double delta, hipStream_t s);
// Two such steps in one pass: dst = C(S(C(S(src)))), equal to two
// launch_step_nb calls bit for bit; with mid != nullptr the intermediate state
// is stored there as well.  src, dst and mid must not overlap.
hipError_t launch_step_nb2(int storage, int eddy, bool kin, const void* src, void* dst,
                           void* mid, const Geom& g, const Rates& r, double delta, hipStream_t s);
// Whether launch_step_nb2 beats two launch_step_nb calls on this lattice.
bool step_nb2_pays(const Geom& g);
// Equilibrium initialisation from FP64 fields.
hipError_t launch_init(int storage, const double* rho, const double* ux, const double* uy,
                       const double* bx, const double* by, void* lat, const Geom& g,
                       hipStream_t s);
// Plain populations <-> encoded lattice.
hipError_t launch_decode(int storage, const void* lat, double* out, const Geom& g, hipStream_t s);
hipError_t launch_encode(int storage, const double* in, void* lat, const Geom& g, hipStream_t s);
// Macroscopic fields of an encoded lattice (no streaming).
hipError_t launch_macro(int storage, const void* lat, double* rho, double* ux, double* uy,
                        double* bx, double* by, const Geom& g, hipStream_t s);
// Byte copy (vector loads/stores) for checkpoints.
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// Diagnostics in one pass over the lattice: per-block partials (at most
// kDiagBlocks x kDiagSlots doubles at part) folded into out_dev[0 .. 12].
hipError_t launch_diag(int storage, const void* lat, double* part, double* out_dev,
                       const Geom& g, hipStream_t s);
// One step src -> dst of FP32 storage (the plain or the Smagorinsky-MHD
// update) fused with the diagnostics of dst, results as launch_diag's.
hipError_t launch_step_diag(bool les, const void* src, void* dst, double* part, double* out_dev,
                            const Geom& g, const Rates& r, hipStream_t s);
// Number of block partials launch_diag writes for this lattice (<= kDiagBlocks).
int diag_partials(const Geom& g);

// Box-averaged macroscopic fields (w x w blocks).
hipError_t launch_macro_box(int storage, const void* lat, int w, double* rho, double* ux,
                            double* uy, double* bx, double* by, const Geom& g, hipStream_t s);
// Mismatch to target fields: per-block partials (at most kDiagBlocks doubles at part)
// folded into out_dev[0].
hipError_t launch_mismatch(int storage, const void* lat, const double* ux_t, const double* uy_t,
                           const double* bx_t, const double* by_t, double* part, double* out_dev,
                           const Geom& g, hipStream_t s);

// Adjoint.
hipError_t launch_adj_seed(int storage, const void* lat, float* lam, const Geom& g,
                           const Geom& ga, hipStream_t s);
hipError_t launch_adj_seed_mismatch(int storage, const void* lat, const double* ux_t,
                                    const double* uy_t, const double* bx_t, const double* by_t,
                                    double scale, float* lam, const Geom& g, const Geom& ga,
                                    hipStream_t s);
hipError_t launch_adj_step(int storage, bool les, const void* state, const float* lam_next,
                           float* lam_prev, double* acc, const Geom& g, const Geom& ga,
                           const Rates& r, double delta2, hipStream_t s);
int adj_step_blocks(const Geom& g);
// Two reverse steps in one pass: lam_prev = R_t(R_{t+1}(lam_next)) from the
// state x_t alone (x_{t+1} is recomputed on chip), equal to two
// launch_adj_step calls with the stored x_{t+1} and x_t; the closure-constant
// derivatives of both steps are added to acc (block slots b and
// adj_step_blocks(g) + b).  Closures that read no neighbours: les_fwd, the
// forward step takes the Smagorinsky-MHD collision (as launch_step's les);
// les, the reverse steps differentiate it (les_fwd implies les).
hipError_t launch_adj_step2(int storage, bool les_fwd, bool les, const void* state,
                            const float* lam_next, float* lam_prev, double* acc, const Geom& g,
                            const Geom& ga, const Rates& r, double delta2, hipStream_t s);
// Whether launch_adj_step2 fills the chip on this lattice.
bool adj_step2_pays(const Geom& g);
// The same reverse step for the kinetic closure (les = 2, or 3 with the
// Smagorinsky-MHD closure): one walk over strips of rows, the gradient
// adjoints of the neighbours kept on chip.
hipError_t launch_adj_step_kin(int storage, bool les, const void* state, const float* lam_next,
                               float* lam_prev, double* acc, const Geom& g, const Geom& ga,
                               const Rates& r, double delta2, hipStream_t s);
hipError_t launch_sum(const double* in, long long n, double* out_dev, hipStream_t s);
hipError_t launch_adj_fields(const float* lam0, const double* rho0, const double* ux0,
                             const double* uy0, const double* bx0, const double* by0,
                             double* gux, double* guy, double* gbx, double* gby, const Geom& ga,
                             int nx, int ny, hipStream_t s);

}  // namespace lbk
