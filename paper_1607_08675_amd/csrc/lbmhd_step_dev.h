// lbmhd_step_dev.h -- device building blocks of the forward step shared by
// the forward kernels (lbmhd_kernels.hip) and the adjoint kernels
// (lbmhd_adjoint.hip): storage codecs, lattice tables, plane accesses, the
// collision, the pull gather of one row and the tables of the row-walking
// multi-step kernels.  Internal to the library; everything lives in an
// anonymous namespace, so each translation unit that includes it compiles its
// own copy of the same source, and the kernels of both round identically.
#pragma once

#include <math.h>

#include "lbmhd_impl.h"

namespace lbk {
namespace {
// ------------------------------------------------------------ storage codec
template <int ST>
struct Codec;
template <>
struct Codec<LBMHD_FP32> {
  using T = float;
  __device__ static __forceinline__ float dec(float v) { return v; }
  __device__ static __forceinline__ float enc(float v) { return v; }
};
template <>
struct Codec<LBMHD_FP16> {
  using T = _Float16;
  // deviation = half * 2^-10; scaling by a power of two is exact, the only
  // rounding is the RNE conversion of the FP32 value to half.  The empty asm
  // statements pin the FP32 values on both sides.  Without them the compiler
  // may fuse the conversion with the multiply-add that produced v
  // (v_fma_mix*), rounding straight to half; and on decoding, it may fuse the
  // exact scale of a decoded value into the add that consumes it, where
  // a * b + dec(h) could otherwise have fused a * b, a choice that depends
  // on the surrounding code.  Either way two kernels computing the same
  // update would differ in rare last bits.
  __device__ static __forceinline__ float dec(_Float16 v) {
    float f = float(v) * 0x1p-10f;
    asm("" : "+v"(f));
    return f;
  }
  __device__ static __forceinline__ _Float16 enc(float v) {
    asm("" : "+v"(v));
    return _Float16(v * 0x1p10f);
  }
};

// FP16 storage as the plain and Smagorinsky-MHD kernels hold it: the
// collision runs on the stored values themselves, i.e. on deviations in units
// of 2^-10 (collide<..., SC = true> folds the scale into its constants), so
// decoding and encoding are bare conversions.  Every operand is then 2^10
// (products of two: 2^20) times its unscaled counterpart, exactly, and the
// stored halves are the same as with the scale applied around the collision.
constexpr int kFP16S = 2;
template <>
struct Codec<kFP16S> {
  using T = _Float16;
  __device__ static __forceinline__ float dec(_Float16 v) {
    float f = float(v);
    asm("" : "+v"(f));
    return f;
  }
  __device__ static __forceinline__ _Float16 enc(float v) {
    asm("" : "+v"(v));
    return _Float16(v);
  }
};

// V consecutive stored elements moved as one vector access.
template <typename T, int V>
struct Vec;
template <>
struct Vec<float, 1> {
  typedef float type;
};
template <>
struct Vec<_Float16, 1> {
  typedef _Float16 type;
};
template <>
struct Vec<_Float16, 2> {
  typedef _Float16 type __attribute__((ext_vector_type(2)));
};

// D2Q9 / D2Q5 lattice (Sec. 3 velocity lists) and the weights under which the
// equilibria reproduce the printed moment tables.
__device__ constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kMx[5] = {0, 1, 0, -1, 0};
__device__ constexpr int kMy[5] = {0, 0, 1, 0, -1};
__device__ constexpr double kW[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__device__ constexpr double kWm[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
// Element `off` of a plane: the plane base is uniform across the wavefront and
// the byte offset fits 32 bits (checked at lbmhd_create), so the compiler emits
// scalar-base + 32-bit-offset global accesses instead of 64-bit lane addresses.
template <typename VT, typename T>
__device__ __forceinline__ VT ld_plane(const T* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const VT*>(reinterpret_cast<const char*>(base) + off * unsigned(sizeof(T)));
}
template <typename VT, typename T>
__device__ __forceinline__ void st_plane_nt(T* __restrict__ base, unsigned off, VT v) {
  __builtin_nontemporal_store(
      v, reinterpret_cast<VT*>(reinterpret_cast<char*>(base) + off * unsigned(sizeof(T))));
}

// velocity (c_x, c_y) of the population held by each of the 19 planes
__device__ constexpr int kPlaneCx[kNPop] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0,
                                            1, 0, -1, 0, 0, 1,  0, -1, 0};
__device__ constexpr int kPlaneCy[kNPop] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0,
                                            0, 1, 0, -1, 0, 0, 1,  0, -1};
constexpr int kStepThreads = 256;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ------------------------------------------------------------ the collision
// One collision in deviation variables.  f[9] = f_i - w_i and g[10] (g_x,
// then g_y) in, post-collision values out.
//  M = T f with the rows of eq. FluidTMatrix; the equilibrium moments of
//  eq. KinMomentEq (w carries rho = 1, so T(f - w) differs from T f only in
//  M_0 and M_8, by 1 and 5/3); f* = f - T^-1 diag(s) (M - M^eq) with
//  T^-1 = T^T diag(1/9, 1/6, 1/6, 1/4, 1/4, 1/12, 1/12, 1/180, 1/20)
//  expanded by hand; g* = g - s_m (g - g^eq) with g^eq of Sec. 3.
//  With LES the shear rate and the magnetic rate follow the Smagorinsky-MHD
//  closure: tau = (tau0 + sqrt(tau0^2 + 18 C_S Delta^2 Q / rho)) / 2 with
//  Q = sqrt((M4 - M4eq)^2 + 4 (M3 - M3eq)^2) (|S| = 3 Q / (2 rho tau)), and
//  tau_m = (tau_m0 + sqrt(tau_m0^2 + 36 C_S Delta^2 |A|)) / 2 with A the
//  antisymmetric non-equilibrium first moment of g (j = -3 A / tau_m).
//  With EDDY = 2 the cross-helicity closure (eqs. CHClosureV/B) sets them:
//  nu_t = C_S Delta^2 |S^v : S^b|^(1/2), eta_t = C_S Delta^2 sgn(j w) |j w|^(1/2),
//  with S^v from M3, M4 as above, S^b and j from the non-equilibrium
//  first-moment tensor L_ab = sum_k C_ka g_kb ~ -(tau_m / 3) d_a B_b, and the
//  vorticity w from the neighbours (NbTerms).  For traceless strains
//  S^v : S^b = 9 P / (4 rho tau tau_m), P = n4 (L_xx - L_yy) + 2 n3 (L_xy + L_yx),
//  and j w = -3 A w / tau_m, so sqrt(tau_m) and sqrt(tau) are the largest
//  roots of t^3 - tau_m0 t - q_b and t^3 - tau0 t - q_v with
//  q_b = -3 sqrt(3) C_S Delta^2 sgn(A w) |A w|^(1/2) and
//  q_v = (9/2) C_S Delta^2 (|P| / (rho tau_m))^(1/2).  Where backscatter would
//  make eta + eta_t negative, tau_m = 1/2.
// Terms that need the neighbours: Delta^2 parts of the filtered equilibrium
// moments (kinetic closure), added to M3^eq, M4^eq, M7^eq = M8^eq and to the
// u x B term E of g^eq (N_y1^eq = E, N_x2^eq = -E); the vorticity w.
struct NbTerms {
  float m3, m4, m78, e, w;
};

// Largest root t of t^3 - p t - q = 0 (p > 0, sp = sqrt(p)), returned as
// t^2 = p + d (2 sp + d), d = t - sp: Newton steps on the convex, increasing
// h(d) = d (2 p + 3 sp d + d^2) - q from an upper bound of the root
// (min(q / (2 p), q^(1/3)) for q > 0, 0 otherwise), so the iterates fall
// monotonically.  For q >= 0 six steps reach FP32 resolution at every p
// (measured to p = 20).  For q < 0 the caller clips first, so the root is at
// least t* = max(sqrt(1/2), sqrt(p / 3)), a simple root for p < 3/2; but as p
// nears 3/2 the clip nears the cubic's double root at sqrt(p / 3), where
// Newton converges only linearly.  Six steps land within 1e-6 of the root
// up to p = 5/4 (measured: 8.8e-4 at p = 1.4), and lbmhd_create refuses the
// closure beyond.  The steps stop early once a step has left d unchanged in
// every lane of the wavefront: the step is a fixed map of d, so every later
// step would leave it unchanged too, and the result is that of six steps.
__device__ __forceinline__ float cubic_root_sq(float p, float sp, float q) {
#pragma clang fp contract(off)
  float d = q > 0.0f ? fminf(q * (0.5f * frcp(p)), cbrtf(q)) : 0.0f;
  for (int i = 0; i < 6; ++i) {
    const float h = fmaf(d, fmaf(d, 3.0f * sp + d, 2.0f * p), -q);
    const float hp = fmaf(d, fmaf(3.0f, d, 6.0f * sp), 2.0f * p);
    const float dn = fmaf(-h, frcp(hp), d);
    const bool fixed = dn == d;
    d = dn;
    if (__all(fixed)) break;
  }
  return fmaf(d, 2.0f * sp + d, p);
}

// Every multiply-add of the collision is written out: fmaf where one
// rounding is wanted, a separate product where two.  The compiler may not
// contract anything else (fp contract off), so each kernel that inlines the
// collision -- one or two sites per thread, halo columns, several steps per
// pass, in place -- rounds it identically and their results agree bit for bit.
// With SC the populations are in units of 2^-10 (scaled FP16 storage): each
// product of two scaled quantities carries an extra 2^10, taken out by the
// factor kS = 2^-10 folded into the constant of the operation that consumes it
// (exact), so the result is 2^10 times the unscaled one bit for bit.
template <int EDDY, bool KIN = false, bool SC = false>
__device__ __forceinline__ void collide(float (&f)[9], float (&g)[10], const Rates& r,
                                        const NbTerms& kc = NbTerms{0.f, 0.f, 0.f, 0.f, 0.f}) {
#pragma clang fp contract(off)
  static_assert(!SC || (!KIN && EDDY < 2), "scaled populations: plain and Smagorinsky only");
  constexpr float kS = SC ? 0x1p-10f : 1.0f;
  const float a13 = f[1] + f[3], a24 = f[2] + f[4];
  const float d13 = f[1] - f[3], d24 = f[2] - f[4];
  const float s57 = f[5] + f[7], s68 = f[6] + f[8];
  const float d57 = f[5] - f[7], d68 = f[6] - f[8];
  const float dd = s57 + s68;
  const float sa = a13 + a24;
  const float f0dd = f[0] + dd;
  const float drho = f0dd + sa;
  const float rho = SC ? fmaf(kS, drho, 1.0f) : 1.0f + drho;
  const float jx = (d13 + d57) - d68;
  const float jy = (d24 + d57) + d68;
  const float M3 = s57 - s68;
  const float M4 = a13 - a24;
  const float M5 = fmaf(-3.0f, d13, jx);
  const float M6 = fmaf(-3.0f, d24, jy);
  const float M7 = fmaf(-5.0f, sa, 4.0f * f0dd);   // 4 f0 - 5 (a13 + a24) + 4 dd
  const float M8 = fmaf(4.0f, f[0], -dd);

  const float ir = frcp(rho);
  const float ux = jx * ir, uy = jy * ir;
  const float Bx = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
  const float By = ((g[5] + g[6]) + (g[7] + g[8])) + g[9];
  const float jyuy = jy * uy;
  const float jj = fmaf(jx, ux, jyuy);                       // |j|^2 / rho
  const float Byy = By * By;
  float n3 = fmaf(-kS, fmaf(-Bx, By, jx * uy), M3);          // M3 - (jx uy - Bx By)
  float n4 = fmaf(-kS, fmaf(jx, ux, -jyuy) - fmaf(Bx, Bx, -Byy), M4);
  const float n5 = M5 + jx;
  const float n6 = M6 + jy;
  float n7 = fmaf(3.0f * kS, jj, M7);
  float n8 = fmaf(3.0f * kS, jj, fmaf(-5.0f / 3.0f, drho, M8));
  float E = fmaf(ux, By, -(uy * Bx));                          // scaled: 2^20 E
  if (KIN) {
    // relax toward the filtered equilibria; with the Smagorinsky closure as
    // well, Q and A below are then measured from the filtered equilibria
    n3 -= kc.m3;
    n4 -= kc.m4;
    n7 -= kc.m78;
    n8 -= kc.m78;
    E += kc.e;
  }

  float s3q, sm;
  if (EDDY == 1) {
    // s3q = 1 / (4 tau) = 1 / (2 tau0 + sqrt(4 tau0^2 + 4 cf Q / rho)) with
    // the powers of two folded into the constants (exact)
    const float Q = fsqrt(fmaf(n4, n4, 4.0f * (n3 * n3)));
    s3q = frcp(r.tau0d + fsqrt(fmaf((r.cf4 * kS) * Q, ir, r.tau0dsq)));
    const float A = fmaf(-2.0f * kS, E, (g[6] - g[8]) - (g[2] - g[4]));
    // sm = 1 / tau_m = 1 / (tau_m0 / 2 + sqrt(tau_m0^2 / 4 + cm |A| / 4))
    sm = frcp(r.taum0h + fsqrt(fmaf(r.cmq * kS, fabsf(A), r.taum0hsq)));
  } else if (EDDY == 2) {
    const float lxy = g[6] - g[8], lyx = g[2] - g[4];
    const float P = fmaf(n4, (g[1] - g[3]) - (g[7] - g[9]), 2.0f * (n3 * (lxy + lyx)));
    const float X = fmaf(-2.0f, E, lxy - lyx) * kc.w;
    const float qb = -r.kb * copysignf(fsqrt(fabsf(X)), X);
    const float taum = qb < r.qclip ? 0.5f : fmaxf(0.5f, cubic_root_sq(r.taum0, r.staum0, qb));
    const float qv = r.kv * fsqrt(fabsf(P) * ir * frcp(taum));
    s3q = 0.25f * frcp(cubic_root_sq(r.tau0, r.stau0, qv));
    sm = frcp(taum);
  } else {
    s3q = r.s3q;
    sm = r.sm;
  }
  const float r3 = s3q * n3, r4 = s3q * n4;
  const float r5 = r.s5q * n5, r6 = r.s5q * n6;
  const float r7 = r.s7q * n7, r8 = r.s8q * n8;
  const float c58 = fmaf(4.0f, r7, -r8);
  f[0] = fmaf(-4.0f, r7 + r8, f[0]);
  f[1] -= fmaf(-5.0f, r7, fmaf(-2.0f, r5, r4));
  f[2] -= fmaf(-5.0f, r7, fmaf(-2.0f, r6, -r4));
  f[3] -= fmaf(-5.0f, r7, fmaf(2.0f, r5, r4));
  f[4] -= fmaf(-5.0f, r7, fmaf(2.0f, r6, -r4));
  const float p56 = r5 + r6, m56 = r5 - r6;
  f[5] -= (r3 + p56) + c58;
  f[6] -= c58 - (r3 + m56);
  f[7] -= (r3 - p56) + c58;
  f[8] -= (m56 - r3) + c58;

  // g^eq of the four moving directions is B/6 +- E/2; the rest direction takes
  // the remainder B - 4 (B/6) so that sum_k g^eq = B holds in FP32 as well
  // (6 * fl(1/6) != 1 would otherwise feed a systematic drift into B).
  const float bx6 = Bx * (1.0f / 6.0f), by6 = By * (1.0f / 6.0f);
  const float msm = -sm;
  g[0] = fmaf(msm, g[0] - fmaf(-4.0f, bx6, Bx), g[0]);
  g[1] = fmaf(msm, g[1] - bx6, g[1]);
  g[2] = fmaf(msm, g[2] - fmaf(-0.5f * kS, E, bx6), g[2]);
  g[3] = fmaf(msm, g[3] - bx6, g[3]);
  g[4] = fmaf(msm, g[4] - fmaf(0.5f * kS, E, bx6), g[4]);
  g[5] = fmaf(msm, g[5] - fmaf(-4.0f, by6, By), g[5]);
  g[6] = fmaf(msm, g[6] - fmaf(0.5f * kS, E, by6), g[6]);
  g[7] = fmaf(msm, g[7] - by6, g[7]);
  g[8] = fmaf(msm, g[8] - fmaf(-0.5f * kS, E, by6), g[8]);
  g[9] = fmaf(msm, g[9] - by6, g[9]);
}

// --------------------------------------------------------------- the step
// Pre-collision values of the V consecutive sites x .. x + V - 1 of one row:
// pre_q(x) = src_q(x - c_q), periodic.  xl and xr are the columns left of x
// and right of x + V - 1 (wrapped); row[c_y + 1] is the source row of a plane
// with velocity c_y.  A plane that streams along x is read as the aligned
// vector of the sites plus one edge element.  V > 1 requires nx % V == 0.
template <int ST, int V>
__device__ __forceinline__ void gather_row(const typename Codec<ST>::T* __restrict__ src,
                                           long long P, int x, int xl, int xr,
                                           const unsigned (&row)[3], float (&v)[kNPop][V]) {
  using C = Codec<ST>;
  using T = typename C::T;
  using VT = typename Vec<T, V>::type;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    const T* __restrict__ base = src + q * P;
    const unsigned r = row[kPlaneCy[q] + 1];
    if (V == 1 || kPlaneCx[q] == 0) {
      const int xs = kPlaneCx[q] == 0 ? x : (kPlaneCx[q] == 1 ? xl : xr);
      const VT a = ld_plane<VT>(base, r + unsigned(xs));
      if constexpr (V == 1) {
        v[q][0] = C::dec(a);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) v[q][j] = C::dec(a[j]);
      }
    } else if constexpr (V > 1) {
      const VT a = ld_plane<VT>(base, r + unsigned(x));
      const float e = C::dec(ld_plane<T>(base, r + unsigned(kPlaneCx[q] == 1 ? xl : xr)));
#pragma unroll
      for (int j = 0; j < V; ++j) {
        if (kPlaneCx[q] == 1)
          v[q][j] = j == 0 ? e : C::dec(a[j > 0 ? j - 1 : 0]);
        else
          v[q][j] = j == V - 1 ? e : C::dec(a[j < V - 1 ? j + 1 : 0]);
      }
    }
  }
}

// One collision of each of the V sites in v (planes in the storage order).
template <int V, bool LES, bool SC = false>
__device__ __forceinline__ void collide_sites(float (&v)[kNPop][V], const Rates& rt) {
#pragma unroll
  for (int j = 0; j < V; ++j) {
    float f[9], g[10];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = v[i][j];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = v[9 + k][j];
    collide<LES ? 1 : 0, false, SC>(f, g, rt);
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i][j] = f[i];
#pragma unroll
    for (int k = 0; k < 10; ++k) v[9 + k][j] = g[k];
  }
}

// Encode and store the V sites of v at element `off` of every plane.
template <int ST, int V>
__device__ __forceinline__ void store_row(typename Codec<ST>::T* __restrict__ dst, long long P,
                                          unsigned off, const float (&v)[kNPop][V]) {
  using C = Codec<ST>;
  using VT = typename Vec<typename C::T, V>::type;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    VT w;
    if constexpr (V == 1) {
      w = C::enc(v[q][0]);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) w[j] = C::enc(v[q][j]);
    }
    st_plane_nt<VT>(dst + q * P, off, w);
  }
}

// ----------------------------------------------- row walks over strips

// Row-walking kernels hand the planes that move along x to the neighbouring
// columns through LDS, grouped by c_y.
// LDS group of each plane with c_x != 0 (0: c_y = +1, 1: c_y = 0, 2: c_y = -1)
// and its index in the group; -1 for the register-held planes (c_x = 0).
__device__ constexpr int kT2Group[kNPop] = {-1, 1, -1, 1, -1, 0, 0, 2, 2, -1,
                                            1, -1, 1, -1, -1, 1, -1, 1, -1};
__device__ constexpr int kT2Index[kNPop] = {0, 0, 0, 1, 0, 0, 1, 0, 1, 0,
                                            2, 0, 3, 0, 0, 4, 0, 5, 0};
// index of a c_x = 0 plane among the three of its c_y: {0, 9, 14} (c_y = 0),
// {2, 11, 16} (c_y = +1), {4, 13, 18} (c_y = -1)
__device__ constexpr int kT2Reg[kNPop] = {0, -1, 0, -1, 0, -1, -1, -1, -1, 1,
                                          -1, 1, -1, 1, 2, -1, 2, -1, 2};

// Row offsets of the gather for row r (-ny <= r < 2 ny, wrapped once): the source
// row of a plane with velocity c_y is r - c_y, indexed by c_y + 1.
__device__ __forceinline__ void t2_rows(int r, const Geom& geo, unsigned (&row)[3]) {
  r = r < 0 ? r + geo.ny : (r >= geo.ny ? r - geo.ny : r);
  const int rm = r == 0 ? geo.ny - 1 : r - 1;
  const int rp = r == geo.ny - 1 ? 0 : r + 1;
  row[0] = unsigned(rp) * geo.pitch;
  row[1] = unsigned(r) * geo.pitch;
  row[2] = unsigned(rm) * geo.pitch;
}

// Row-walking kernels with three levels: 256-column tiles plus a fifth wave
// for the halo columns.
constexpr int kT3Cols = 256;
constexpr int kT3Threads = kT3Cols + 64;
constexpr int kT3Rows = 10;   // planes with c_x != 0

// LDS row of plane q (c_x != 0): the c_y = +1 planes, then c_y = 0, then c_y = -1.
__device__ __forceinline__ int t3_row(int q) {
  const int g = kT2Group[q], i = kT2Index[q];
  return g == 0 ? i : (g == 1 ? 2 + i : 8 + i);
}

}  // namespace
}  // namespace lbk
