// lbmhd3.hip -- the three-dimensional LB-MHD update on gfx950 and its C ABI
// (include/lbmhd3.h).  The model: D3Q27 populations f with the second-order
// equilibrium including the Maxwell stress, six magnetic vector populations g,
// single-relaxation collisions and the per-site Smagorinsky-MHD closure of
// the 2D update (Flint & Vahala, arXiv:1607.08675, Sec. 1.1 and Sec. 3,
// extended to 3D as the paper states it extends).
//
// One thread updates one site: it gathers the 45 post-collision populations
// of the neighbours (pull streaming, all loads issued first), collides in
// registers and writes 45 values to the other lattice.  HBM-bound: 45 x e
// bytes read + 45 x e bytes written per site, e = 4 (FP32 storage) or 2
// (FP16).  Stored values are the deviations f - w (g as is), in FP32 or as
// half(2^10 (f - w)) rounded to nearest even; the collision runs in FP32.
// Plane element offsets are 32-bit byte offsets from a wavefront-uniform
// plane base (create checks that a plane stays below 4 GiB).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <type_traits>

#include "lbmhd3.h"

namespace lbk3 {
namespace {

constexpr int kQ = 27;        // D3Q27
constexpr int kNPop = 45;     // 27 + 3 x 6
constexpr int kThreads = 256; // sites per block (one x segment of one row)

// velocity of each of the 45 planes (planes 27..44: the six magnetic vectors
// for the x, then y, then z component)
__device__ constexpr int kCx[kNPop] = {
    0, 1, -1, 0, 0,  0, 0,  1, -1, 1, -1, 1, -1, 1, -1, 0,  0,  0, 0,  1, -1, 1,  -1,
    1, -1, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, 0, 0, 0,  0, 1, -1, 0, 0, 0,  0};
__device__ constexpr int kCy[kNPop] = {
    0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
    -1, 1, 1, -1, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 0, 0};
__device__ constexpr int kCz[kNPop] = {
    0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1,
    1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1};

// D1Q3 weights multiplied over the axes: 8/27, 2/27, 1/54, 1/216
__host__ __device__ constexpr double weight27(int cx, int cy, int cz) {
  return (cx == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (cy == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
         (cz == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
}

struct Geom3 {
  int nx, ny, nz;
  unsigned pitch;    // elements per padded row
  long long plane;   // elements per plane (nz * ny * pitch)
};

struct Rates3 {
  float itau0, itaum0;    // fixed-rate case
  float tau0, tau0sq, taum0, taum0sq;
  float cf, cm;           // 18 C_Sv Delta^2, 36 C_Sb Delta^2
  float s5, s7, s8, sg, szz;   // moment-space collision rates
};

// The paper's D2Q9 velocity order (rows of eq. FluidTMatrix act on it) and
// 180 times the inverse of its nine rows: column r maps a moment back to the
// nine populations.
__device__ constexpr int kX2[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kY2[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr float kT2inv180[9][9] = {
    {20, 0, 0, 0, 0, 0, 0, 4, 36},       {20, 30, 0, 0, 45, -30, 0, -5, 0},
    {20, 0, 30, 0, -45, 0, -30, -5, 0},  {20, -30, 0, 0, 45, 30, 0, -5, 0},
    {20, 0, -30, 0, -45, 0, 30, -5, 0},  {20, 30, 30, 45, 0, 15, 15, 4, -9},
    {20, -30, 30, -45, 0, -15, 15, 4, -9}, {20, -30, -30, 45, 0, -15, -15, 4, -9},
    {20, 30, -30, -45, 0, 15, -15, 4, -9}};

// Row r of the paper's D2Q9 transform at velocity (cx, cy) (compile time).
__host__ __device__ constexpr float prow2(int r, int cx, int cy) {
  return r == 0   ? 1.0f
         : r == 1 ? float(cx)
         : r == 2 ? float(cy)
         : r == 3 ? float(cx * cy)
         : r == 4 ? float(cx * cx - cy * cy)
         : r == 5 ? float(3 * cx * cy * cy - 2 * cx)
         : r == 6 ? float(3 * cy * cx * cx - 2 * cy)
         : r == 7 ? float(4 - 9 * (cx * cx + cy * cy - 2 * cx * cx * cy * cy))
                  : float(4 - 4 * (cx * cx + cy * cy) + 3 * cx * cx * cy * cy);
}

// f* = f - T^-1 S T (f - f^eq) in the tensor-product basis p_r q_k (see
// lbmhd3_params): nq = f - f^eq in, the amount to subtract from f out.
// T = T2 (x) T1 factorises: the c_z transform (q = 1, c_z, 3 c_z^2 - 1) of
// each of the nine (c_x, c_y) columns, the paper's nine rows on each of the
// three results, the rates, and back (T1^-1: w_z q_k / |q_k|^2 with
// |q|^2 = 1, 1/3, 2 under the D1Q3 weights).
__device__ __forceinline__ void mrt_relax(float (&nq)[kQ], float sv, const Rates3& r) {
  float a[3][9];
#pragma unroll
  for (int j = 0; j < 9; ++j) a[0][j] = a[1][j] = a[2][j] = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
#pragma unroll
    for (int j = 0; j < 9; ++j)
      if (kCx[i] == kX2[j] && kCy[i] == kY2[j]) {
        a[0][j] += nq[i];
        if (kCz[i]) {
          a[1][j] += float(kCz[i]) * nq[i];
          a[2][j] += 2.0f * nq[i];
        } else {
          a[2][j] -= nq[i];
        }
      }
  }
  float b[3][9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float rel[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      float mom = 0.0f;
#pragma unroll
      for (int j = 0; j < 9; ++j)
        if (prow2(m, kX2[j], kY2[j]) != 0.0f) mom += prow2(m, kX2[j], kY2[j]) * a[k][j];
      float s;
      if (k == 0)
        s = m < 3 ? 0.0f : (m < 5 ? sv : (m < 7 ? r.s5 : (m == 7 ? r.s7 : r.s8)));
      else if (k == 1)
        s = m == 0 ? 0.0f : (m < 3 ? sv : r.sg);
      else
        s = m == 0 ? r.szz : r.sg;
      rel[m] = (1.0f / 180.0f) * (s * mom);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int m = 0; m < 9; ++m)
        if (kT2inv180[j][m] != 0.0f) acc += kT2inv180[j][m] * rel[m];
      b[k][j] = acc;
    }
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
#pragma unroll
    for (int j = 0; j < 9; ++j)
      if (kCx[i] == kX2[j] && kCy[i] == kY2[j])
        nq[i] = kCz[i] == 0 ? (2.0f / 3.0f) * b[0][j] - (1.0f / 3.0f) * b[2][j]
                            : (1.0f / 6.0f) * (b[0][j] + b[2][j]) + float(kCz[i]) * 0.5f * b[1][j];
  }
}

// Storage codecs: FP32 deviations, or FP16 deviations scaled by 2^10 (the
// scaling is exact; the conversion to half rounds to nearest even).  The
// empty asm keeps the FP32 value, so the conversion is not fused with the
// multiply-add that produced it.
template <int ST>
struct Codec3;
template <>
struct Codec3<LBMHD_FP32> {
  using T = float;
  __device__ static __forceinline__ float dec(float v) { return v; }
  __device__ static __forceinline__ float enc(float v) { return v; }
};
template <>
struct Codec3<LBMHD_FP16> {
  using T = _Float16;
  __device__ static __forceinline__ float dec(_Float16 v) { return float(v) * 0x1p-10f; }
  __device__ static __forceinline__ _Float16 enc(float v) {
    asm("" : "+v"(v));
    return _Float16(v * 0x1p10f);
  }
};

template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off * unsigned(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st_nt(T* __restrict__ base, unsigned off, T v) {
  __builtin_nontemporal_store(
      v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off * unsigned(sizeof(T))));
}

// One collision at one site.  d[27] = f - w (deviations), g[18] (x, y, z
// components of the six vectors) in, post-collision values out.
template <bool LES, bool MRT>
__device__ __forceinline__ void collide3(float (&d)[kQ], float (&g)[18], const Rates3& r) {
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
  float pxx = 0.0f, pyy = 0.0f, pzz = 0.0f, pxy = 0.0f, pxz = 0.0f, pyz = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    drho += d[i];
    if (kCx[i]) jx += kCx[i] * d[i];
    if (kCy[i]) jy += kCy[i] * d[i];
    if (kCz[i]) jz += kCz[i] * d[i];
    if (LES) {
      if (kCx[i]) pxx += d[i];
      if (kCy[i]) pyy += d[i];
      if (kCz[i]) pzz += d[i];
      if (kCx[i] * kCy[i]) pxy += kCx[i] * kCy[i] * d[i];
      if (kCx[i] * kCz[i]) pxz += kCx[i] * kCz[i] * d[i];
      if (kCy[i] * kCz[i]) pyz += kCy[i] * kCz[i] * d[i];
    }
  }
  const float rho = 1.0f + drho;
  const float ir = 1.0f / rho;
  const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const float Bx = ((g[0] + g[1]) + (g[2] + g[3])) + (g[4] + g[5]);
  const float By = ((g[6] + g[7]) + (g[8] + g[9])) + (g[10] + g[11]);
  const float Bz = ((g[12] + g[13]) + (g[14] + g[15])) + (g[16] + g[17]);
  const float hb2 = 0.5f * ((Bx * Bx + By * By) + Bz * Bz);
  // Pi' = j j / rho + |B|^2 I / 2 - B B
  const float qxx = jx * ux + hb2 - Bx * Bx, qyy = jy * uy + hb2 - By * By;
  const float qzz = jz * uz + hb2 - Bz * Bz;
  const float qxy = jx * uy - Bx * By, qxz = jx * uz - Bx * Bz, qyz = jy * uz - By * Bz;
  const float qtr = (1.0f / 3.0f) * ((qxx + qyy) + qzz);
  float itau = r.itau0, itaum = r.itaum0;
  if (LES) {
    // Pi^neq = sum c c (f - f^eq) = sum c c d - (drho / 3) I - Pi'
    const float t = (1.0f / 3.0f) * drho;
    float nxx = pxx - t - qxx, nyy = pyy - t - qyy, nzz = pzz - t - qzz;
    const float nxy = pxy - qxy, nxz = pxz - qxz, nyz = pyz - qyz;
    const float tr = (1.0f / 3.0f) * ((nxx + nyy) + nzz);
    nxx -= tr;
    nyy -= tr;
    nzz -= tr;
    const float Q = sqrtf(2.0f * (((nxx * nxx + nyy * nyy) + nzz * nzz) +
                                  2.0f * ((nxy * nxy + nxz * nxz) + nyz * nyz)));
    itau = 2.0f / (r.tau0 + sqrtf(r.tau0sq + r.cf * Q * ir));
    // Lambda_ab = sum_k C_ka g_kb with g[6 b + k], k = +x, -x, +y, -y, +z, -z;
    // A = eps : Lambda^neq, the equilibrium part of eps : Lambda being 2 u x B
    const float lyz = g[14] - g[15], lzy = g[10] - g[11];  // L_yz, L_zy
    const float lzx = g[4] - g[5], lxz = g[12] - g[13];    // L_zx, L_xz
    const float lxy = g[6] - g[7], lyx = g[2] - g[3];      // L_xy, L_yx
    const float Ax = (lyz - lzy) - 2.0f * (uy * Bz - uz * By);
    const float Ay = (lzx - lxz) - 2.0f * (uz * Bx - ux * Bz);
    const float Az = (lxy - lyx) - 2.0f * (ux * By - uy * Bx);
    const float An = sqrtf((Ax * Ax + Ay * Ay) + Az * Az);
    itaum = 2.0f / (r.taum0 + sqrtf(r.taum0sq + r.cm * An));
  }
  // f^eq_i - w_i = w_i (drho + 3 c.j + (9/2) (c.Pi'.c - tr Pi' / 3)).  The
  // weights are rounded to FP32, so sum_i f^eq = rho and sum_i c_i f^eq = j
  // hold only to rounding, with the same sign step after step; the remainders
  // go to the rest and face populations so that the collision conserves mass
  // and momentum up to unbiased rounding (measured in FP32 emulation of a 24^3
  // vortex: 4.5x smaller velocity error after 200 steps).
  float deq[kQ];
  float sm = 0.0f, sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float w = float(weight27(kCx[i], kCy[i], kCz[i]));
    float cj = 0.0f, cqc = 0.0f;
    if (kCx[i]) cj += kCx[i] * jx;
    if (kCy[i]) cj += kCy[i] * jy;
    if (kCz[i]) cj += kCz[i] * jz;
    if (kCx[i]) cqc += qxx;
    if (kCy[i]) cqc += qyy;
    if (kCz[i]) cqc += qzz;
    if (kCx[i] * kCy[i]) cqc += 2.0f * kCx[i] * kCy[i] * qxy;
    if (kCx[i] * kCz[i]) cqc += 2.0f * kCx[i] * kCz[i] * qxz;
    if (kCy[i] * kCz[i]) cqc += 2.0f * kCy[i] * kCz[i] * qyz;
    deq[i] = w * ((drho + 3.0f * cj) + 4.5f * (cqc - qtr));
    sm += deq[i];
    if (kCx[i]) sx += kCx[i] * deq[i];
    if (kCy[i]) sy += kCy[i] * deq[i];
    if (kCz[i]) sz += kCz[i] * deq[i];
  }
  const float rx = 0.5f * (jx - sx), ry = 0.5f * (jy - sy), rz = 0.5f * (jz - sz);
  deq[0] += drho - sm;
  deq[1] += rx;
  deq[2] -= rx;
  deq[3] += ry;
  deq[4] -= ry;
  deq[5] += rz;
  deq[6] -= rz;
  if (MRT) {
    float nq[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) nq[i] = d[i] - deq[i];
    mrt_relax(nq, itau, r);
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] -= nq[i];
  } else {
#pragma unroll
    for (int i = 0; i < kQ; ++i) d[i] -= itau * (d[i] - deq[i]);
  }
  // g^eq_kb = (B_b + 3 (C_k.u B_b - C_k.B u_b)) / 6 for C_k = +-e_a:
  // +-(u_a B_b - B_a u_b) / 2 around B_b / 6.  The +-z pair takes the
  // remainder (B_b - 4 (B_b / 6)) / 2 so that sum_k g^eq = B holds in FP32
  // (6 fl(1/6) != 1 would otherwise drive a steady drift of B).
  const float B[3] = {Bx, By, Bz}, U[3] = {ux, uy, uz};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const float b6 = B[b] * (1.0f / 6.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float base = a == 2 ? 0.5f * (B[b] - 4.0f * b6) : b6;
      const float e = 0.5f * (U[a] * B[b] - B[a] * U[b]);
      g[6 * b + 2 * a] -= itaum * (g[6 * b + 2 * a] - (base + e));
      g[6 * b + 2 * a + 1] -= itaum * (g[6 * b + 2 * a + 1] - (base - e));
    }
  }
}

// Thread t of block b updates site x = (b mod tiles_x) * 256 + t of row
// (y, z), b / tiles_x = z * ny + y.
template <int ST, bool LES, bool MRT>
__global__ __launch_bounds__(kThreads) void k_step3(const typename Codec3<ST>::T* __restrict__ src,
                                                    typename Codec3<ST>::T* __restrict__ dst,
                                                    Geom3 g, Rates3 r, int tiles_x) {
  using C = Codec3<ST>;
  const int x = (int(blockIdx.x) % tiles_x) * kThreads + int(threadIdx.x);
  const int row = int(blockIdx.x) / tiles_x;
  const int y = row % g.ny, z = row / g.ny;
  if (x >= g.nx) return;
  const int xs[3] = {x == g.nx - 1 ? 0 : x + 1, x, x == 0 ? g.nx - 1 : x - 1};   // x - c, c = -1, 0, 1
  const int ys[3] = {y == g.ny - 1 ? 0 : y + 1, y, y == 0 ? g.ny - 1 : y - 1};
  const int zs[3] = {z == g.nz - 1 ? 0 : z + 1, z, z == 0 ? g.nz - 1 : z - 1};
  float v[kNPop];
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    const unsigned off = (unsigned(zs[kCz[q] + 1]) * unsigned(g.ny) + unsigned(ys[kCy[q] + 1])) *
                             g.pitch + unsigned(xs[kCx[q] + 1]);
    v[q] = C::dec(ld(src + q * g.plane, off));
  }
  float d[kQ], gg[18];
#pragma unroll
  for (int i = 0; i < kQ; ++i) d[i] = v[i];
#pragma unroll
  for (int k = 0; k < 18; ++k) gg[k] = v[kQ + k];
  collide3<LES, MRT>(d, gg, r);
  const unsigned o = (unsigned(z) * unsigned(g.ny) + unsigned(y)) * g.pitch + unsigned(x);
#pragma unroll
  for (int i = 0; i < kQ; ++i) st_nt(dst + i * g.plane, o, C::enc(d[i]));
#pragma unroll
  for (int k = 0; k < 18; ++k) st_nt(dst + (kQ + k) * g.plane, o, C::enc(gg[k]));
}

__device__ __forceinline__ long long site_index(const Geom3& g, long long s, unsigned* off) {
  const long long x = s % g.nx, yz = s / g.nx;
  const long long y = yz % g.ny, z = yz / g.ny;
  *off = (unsigned(z) * unsigned(g.ny) + unsigned(y)) * g.pitch + unsigned(x);
  return s;
}

// Equilibria of FP64 fields, stored as deviations.
template <int ST>
__global__ __launch_bounds__(256) void k_init3(const double* __restrict__ rho,
                                               const double* __restrict__ ux,
                                               const double* __restrict__ uy,
                                               const double* __restrict__ uz,
                                               const double* __restrict__ bx,
                                               const double* __restrict__ by,
                                               const double* __restrict__ bz,
                                               typename Codec3<ST>::T* __restrict__ lat,
                                               Geom3 g) {
  using C = Codec3<ST>;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  unsigned o;
  site_index(g, s, &o);
  const double r = rho[s], U[3] = {ux[s], uy[s], uz[s]}, B[3] = {bx[s], by[s], bz[s]};
  const double j[3] = {r * U[0], r * U[1], r * U[2]};
  const double hb2 = 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  double P[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) P[a][b] = j[a] * U[b] + (a == b ? hb2 : 0.0) - B[a] * B[b];
  const double tr = (P[0][0] + P[1][1] + P[2][2]) / 3.0;
  for (int i = 0; i < kQ; ++i) {
    const int c[3] = {kCx[i], kCy[i], kCz[i]};
    double cj = 0.0, cqc = 0.0;
    for (int a = 0; a < 3; ++a) {
      cj += c[a] * j[a];
      for (int b = 0; b < 3; ++b) cqc += c[a] * c[b] * P[a][b];
    }
    const double w = weight27(c[0], c[1], c[2]);
    lat[i * g.plane + o] = C::enc(float(w * ((r - 1.0) + 3.0 * cj + 4.5 * (cqc - tr))));
  }
  for (int b = 0; b < 3; ++b)
    for (int k = 0; k < 6; ++k) {
      const int q = kQ + 6 * b + k;
      const int c[3] = {kCx[q], kCy[q], kCz[q]};
      const double cu = c[0] * U[0] + c[1] * U[1] + c[2] * U[2];
      const double cb = c[0] * B[0] + c[1] * B[1] + c[2] * B[2];
      lat[q * g.plane + o] = C::enc(float((B[b] + 3.0 * (cu * B[b] - cb * U[b])) / 6.0));
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_decode3(const typename Codec3<ST>::T* __restrict__ lat,
                                                 double* __restrict__ out, Geom3 g) {
  using C = Codec3<ST>;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  unsigned o;
  site_index(g, s, &o);
  for (int q = 0; q < kNPop; ++q) {
    const double w = q < kQ ? weight27(kCx[q], kCy[q], kCz[q]) : 0.0;
    out[q * n + s] = w + double(C::dec(lat[q * g.plane + o]));
  }
}

template <int ST>
__global__ __launch_bounds__(256) void k_encode3(const double* __restrict__ in,
                                                 typename Codec3<ST>::T* __restrict__ lat,
                                                 Geom3 g) {
  using C = Codec3<ST>;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  unsigned o;
  site_index(g, s, &o);
  for (int q = 0; q < kNPop; ++q) {
    const double w = q < kQ ? weight27(kCx[q], kCy[q], kCz[q]) : 0.0;
    lat[q * g.plane + o] = C::enc(float(in[q * n + s] - w));
  }
}

// rho, u, B of the state in FP64 (7 fields of n)
template <int ST>
__global__ __launch_bounds__(256) void k_macro3(const typename Codec3<ST>::T* __restrict__ lat,
                                                double* __restrict__ rho, double* __restrict__ u,
                                                double* __restrict__ B, Geom3 g) {
  using C = Codec3<ST>;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  unsigned o;
  site_index(g, s, &o);
  double dr = 0.0, j[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < kQ; ++i) {
    const double v = C::dec(lat[i * g.plane + o]);
    dr += v;
    j[0] += kCx[i] * v;
    j[1] += kCy[i] * v;
    j[2] += kCz[i] * v;
  }
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 6; ++k) b[c] += C::dec(lat[(kQ + 6 * c + k) * g.plane + o]);
  const double r = 1.0 + dr;
  rho[s] = r;
  for (int c = 0; c < 3; ++c) {
    u[c * n + s] = j[c] / r;
    B[c * n + s] = b[c];
  }
}

// Reduction over the macro fields: sums (mass, momentum 3, flux 3, e_kin,
// e_mag, non-finite count), maxima (|div B| centred, |u|); one partial row of
// 12 doubles per block.
constexpr int kRed = 12;
__global__ __launch_bounds__(256) void k_reduce3(const double* __restrict__ ws,
                                                 double* __restrict__ part, Geom3 g) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const double* rho = ws;
  const double* u = ws + n;
  const double* B = ws + 4 * n;
  double v[kRed];
  for (int q = 0; q < kRed; ++q) v[q] = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const long long x = s % g.nx, yz = s / g.nx, y = yz % g.ny, z = yz / g.ny;
    const long long xp = (x + 1) % g.nx, xm = (x + g.nx - 1) % g.nx;
    const long long yp = (y + 1) % g.ny, ym = (y + g.ny - 1) % g.ny;
    const long long zp = (z + 1) % g.nz, zm = (z + g.nz - 1) % g.nz;
    auto at = [&](long long xx, long long yy, long long zz) { return (zz * g.ny + yy) * g.nx + xx; };
    const double r = rho[s];
    double uu = 0.0, bb = 0.0;
    for (int c = 0; c < 3; ++c) {
      v[1 + c] += r * u[c * n + s];
      v[4 + c] += B[c * n + s];
      uu += u[c * n + s] * u[c * n + s];
      bb += B[c * n + s] * B[c * n + s];
    }
    v[0] += r;
    v[7] += 0.5 * r * uu;
    v[8] += 0.5 * bb;
    v[9] += isfinite(r) ? 0.0 : 1.0;
    const double div = 0.5 * (B[at(xp, y, z)] - B[at(xm, y, z)]) +
                       0.5 * (B[n + at(x, yp, z)] - B[n + at(x, ym, z)]) +
                       0.5 * (B[2 * n + at(x, y, zp)] - B[2 * n + at(x, y, zm)]);
    v[10] = fmax(v[10], fabs(div));
    v[11] = fmax(v[11], sqrt(uu));
  }
  __shared__ double sh[kRed][256];
  const int t = threadIdx.x;
  for (int q = 0; q < kRed; ++q) sh[q][t] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      for (int q = 0; q < 10; ++q) sh[q][t] += sh[q][t + w];
      for (int q = 10; q < kRed; ++q) sh[q][t] = fmax(sh[q][t], sh[q][t + w]);
    }
    __syncthreads();
  }
  if (t < kRed) part[(long long)blockIdx.x * kRed + t] = sh[t][0];
}

__global__ __launch_bounds__(256) void k_final3(const double* __restrict__ part, int nparts,
                                                double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t >= kRed) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) {
    const double x = part[(long long)b * kRed + t];
    acc = t < 10 ? acc + x : fmax(acc, x);
  }
  out[t] = acc;
}

constexpr int kReduceBlocks = 1024;

}  // namespace
}  // namespace lbk3

struct lbmhd3 {
  lbmhd3_params p;
  lbk3::Geom3 geo;
  lbk3::Rates3 rates;
  size_t lattice_bytes = 0, workspace_bytes = 0;
  void* lat[2] = {nullptr, nullptr};
  double* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int cur = 0;
  int64_t step = 0;
  std::string err;
};

namespace {

constexpr size_t kAlign3 = 256;

int fail3(lbmhd3_t* h, int code, const std::string& m) {
  if (h) h->err = m;
  return code;
}
int hip_fail3(lbmhd3_t* h, hipError_t e, const char* where) {
  return fail3(h, LBMHD_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}
int need3(lbmhd3_t* h) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  if (!h->bound) return fail3(h, LBMHD_ERR_NOT_BOUND, "lbmhd3_bind() has not succeeded");
  return LBMHD_OK;
}
bool aligned3(const void* p) { return reinterpret_cast<uintptr_t>(p) % kAlign3 == 0; }
bool overlap3(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}
long long sites3(const lbmhd3_t* h) {
  return (long long)h->geo.nx * h->geo.ny * h->geo.nz;
}
unsigned blocks3(long long n) { return unsigned((n + 255) / 256); }
// workspace: 7 macro fields of n doubles, reduction partials, 16 results
size_t ws_doubles3(long long n) {
  return 7 * size_t(n) + size_t(lbk3::kReduceBlocks) * lbk3::kRed + 16;
}
// rho, u (3 fields), B (3 fields) of the current state, FP64 device fields
void launch_macro3(lbmhd3_t* h, double* rho, double* u, double* B) {
  const dim3 grid(blocks3(sites3(h)));
  if (h->p.storage == LBMHD_FP32)
    hipLaunchKernelGGL(lbk3::k_macro3<LBMHD_FP32>, grid, dim3(256), 0, h->stream,
                       static_cast<const float*>(h->lat[h->cur]), rho, u, B, h->geo);
  else
    hipLaunchKernelGGL(lbk3::k_macro3<LBMHD_FP16>, grid, dim3(256), 0, h->stream,
                       static_cast<const _Float16*>(h->lat[h->cur]), rho, u, B, h->geo);
}

}  // namespace

extern "C" {

int lbmhd3_create(const lbmhd3_params* p, lbmhd3_t** out) {
  if (!out) return LBMHD_ERR_INVALID_ARG;
  *out = nullptr;
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return LBMHD_ERR_INVALID_ARG;
  if (!(p->nu > 0.0) || !(p->eta > 0.0) || !std::isfinite(p->nu) || !std::isfinite(p->eta))
    return LBMHD_ERR_INVALID_ARG;
  if (p->les != 0 && p->les != 1) return LBMHD_ERR_INVALID_ARG;
  if (p->storage != LBMHD_FP32 && p->storage != LBMHD_FP16) return LBMHD_ERR_INVALID_ARG;
  if (p->mrt != 0 && p->mrt != 1) return LBMHD_ERR_INVALID_ARG;
  if (p->mrt) {
    for (double s : {p->s5, p->s7, p->s8, p->sg, p->szz})
      if (!(s > 0.0 && s < 2.0)) return LBMHD_ERR_INVALID_ARG;
  }
  const size_t esize = p->storage == LBMHD_FP32 ? 4 : 2;
  if (!(p->cs >= 0.0) || !(p->cs_b >= 0.0) || !std::isfinite(p->cs) || !std::isfinite(p->cs_b) ||
      !(p->delta > 0.0) || !std::isfinite(p->delta))
    return LBMHD_ERR_INVALID_ARG;
  lbk3::Geom3 g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.pitch = unsigned((size_t(p->nx) * esize + kAlign3 - 1) / kAlign3 * kAlign3 / esize);
  // planes spaced by their rows plus a gap of three 256-byte blocks, as in 2D
  // (at 256^3 FP32 they would otherwise lie 2^26 bytes apart)
  g.plane = (long long)g.pitch * p->ny * p->nz + (long long)(768 / esize);
  // in-plane byte offsets are 32-bit in the step kernel
  if ((unsigned long long)g.plane * esize >= (1ull << 32)) return LBMHD_ERR_INVALID_ARG;
  lbmhd3_t* h = new (std::nothrow) lbmhd3;
  if (!h) return LBMHD_ERR_INVALID_ARG;
  h->p = *p;
  h->geo = g;
  const double tau0 = 3.0 * p->nu + 0.5, taum0 = 3.0 * p->eta + 0.5, d2 = p->delta * p->delta;
  h->rates = lbk3::Rates3{float(1.0 / tau0), float(1.0 / taum0), float(tau0), float(tau0 * tau0),
                          float(taum0), float(taum0 * taum0), float(18.0 * p->cs * d2),
                          float(36.0 * p->cs_b * d2), float(p->s5), float(p->s7),
                          float(p->s8), float(p->sg), float(p->szz)};
  h->lattice_bytes = size_t(lbk3::kNPop) * size_t(g.plane) * esize;
  h->workspace_bytes =
      (ws_doubles3((long long)p->nx * p->ny * p->nz) * sizeof(double) + kAlign3 - 1) / kAlign3 *
      kAlign3;
  *out = h;
  return LBMHD_OK;
}

int lbmhd3_destroy(lbmhd3_t* h) {
  delete h;
  return LBMHD_OK;
}

int lbmhd3_sizes(const lbmhd3_t* h, size_t* lattice, size_t* workspace) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  if (lattice) *lattice = h->lattice_bytes;
  if (workspace) *workspace = h->workspace_bytes;
  return LBMHD_OK;
}

int lbmhd3_bind(lbmhd3_t* h, void* lat_a, size_t lat_a_bytes, void* lat_b, size_t lat_b_bytes,
                void* workspace, size_t workspace_bytes, void* stream) {
  if (!h) return LBMHD_ERR_INVALID_ARG;
  h->bound = false;
  if (!lat_a || !lat_b || !workspace)
    return fail3(h, LBMHD_ERR_INVALID_ARG, "null buffer passed to lbmhd3_bind");
  if (lat_a_bytes < h->lattice_bytes || lat_b_bytes < h->lattice_bytes ||
      workspace_bytes < h->workspace_bytes)
    return fail3(h, LBMHD_ERR_INVALID_ARG, "buffer smaller than lbmhd3_sizes() requires");
  if (!aligned3(lat_a) || !aligned3(lat_b) || !aligned3(workspace))
    return fail3(h, LBMHD_ERR_INVALID_ARG, "buffers must be 256-byte aligned");
  if (overlap3(lat_a, h->lattice_bytes, lat_b, h->lattice_bytes) ||
      overlap3(lat_a, h->lattice_bytes, workspace, h->workspace_bytes) ||
      overlap3(lat_b, h->lattice_bytes, workspace, h->workspace_bytes))
    return fail3(h, LBMHD_ERR_INVALID_ARG, "bound buffers overlap");
  h->lat[0] = lat_a;
  h->lat[1] = lat_b;
  h->ws = static_cast<double*>(workspace);
  h->stream = static_cast<hipStream_t>(stream);
  h->cur = 0;
  h->step = 0;
  h->bound = true;
  return LBMHD_OK;
}

int lbmhd3_init_fields(lbmhd3_t* h, const double* rho, const double* ux, const double* uy,
                       const double* uz, const double* bx, const double* by, const double* bz) {
  if (int rc = need3(h)) return rc;
  if (!rho || !ux || !uy || !uz || !bx || !by || !bz)
    return fail3(h, LBMHD_ERR_INVALID_ARG, "null field");
  if (h->p.storage == LBMHD_FP32)
    hipLaunchKernelGGL(lbk3::k_init3<LBMHD_FP32>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, rho, ux, uy, uz, bx, by, bz, static_cast<float*>(h->lat[0]),
                       h->geo);
  else
    hipLaunchKernelGGL(lbk3::k_init3<LBMHD_FP16>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, rho, ux, uy, uz, bx, by, bz,
                       static_cast<_Float16*>(h->lat[0]), h->geo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(h, e, "init launch");
  h->cur = 0;
  h->step = 0;
  return LBMHD_OK;
}

int lbmhd3_step(lbmhd3_t* h, int64_t nsteps) {
  if (int rc = need3(h)) return rc;
  if (nsteps < 0) return fail3(h, LBMHD_ERR_INVALID_ARG, "negative step count");
  const bool les = h->p.les && (h->p.cs > 0.0 || h->p.cs_b > 0.0);
  const int tiles_x = (h->geo.nx + lbk3::kThreads - 1) / lbk3::kThreads;
  const dim3 grid(unsigned(tiles_x) * unsigned(h->geo.ny) * unsigned(h->geo.nz));
  for (int64_t t = 0; t < nsteps; ++t) {
    const void* src = h->lat[h->cur];
    void* dst = h->lat[1 - h->cur];
    auto go = [&](auto st_tag, auto les_tag, auto mrt_tag) {
      constexpr int ST = decltype(st_tag)::value;
      using T = typename lbk3::Codec3<ST>::T;
      hipLaunchKernelGGL((lbk3::k_step3<ST, decltype(les_tag)::value, decltype(mrt_tag)::value>),
                         grid, dim3(lbk3::kThreads), 0, h->stream, static_cast<const T*>(src),
                         static_cast<T*>(dst), h->geo, h->rates, tiles_x);
    };
    using F32 = std::integral_constant<int, LBMHD_FP32>;
    using F16 = std::integral_constant<int, LBMHD_FP16>;
    using Y = std::true_type;
    using N = std::false_type;
    const bool fp32 = h->p.storage == LBMHD_FP32, mrt = h->p.mrt != 0;
    if (fp32 && les && mrt) go(F32{}, Y{}, Y{});
    else if (fp32 && les) go(F32{}, Y{}, N{});
    else if (fp32 && mrt) go(F32{}, N{}, Y{});
    else if (fp32) go(F32{}, N{}, N{});
    else if (les && mrt) go(F16{}, Y{}, Y{});
    else if (les) go(F16{}, Y{}, N{});
    else if (mrt) go(F16{}, N{}, Y{});
    else go(F16{}, N{}, N{});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail3(h, e, "step launch");
    h->cur = 1 - h->cur;
    ++h->step;
  }
  return LBMHD_OK;
}

int lbmhd3_macro(lbmhd3_t* h, double* rho, double* u, double* B) {
  if (int rc = need3(h)) return rc;
  if (!rho || !u || !B) return fail3(h, LBMHD_ERR_INVALID_ARG, "null field");
  launch_macro3(h, rho, u, B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(h, e, "macro launch");
  return LBMHD_OK;
}

int lbmhd3_diag(lbmhd3_t* h, lbmhd3_diag_t* out) {
  if (int rc = need3(h)) return rc;
  if (!out) return fail3(h, LBMHD_ERR_INVALID_ARG, "null output");
  const long long n = sites3(h);
  double* part = h->ws + 7 * n;
  double* res = part + size_t(lbk3::kReduceBlocks) * lbk3::kRed;
  launch_macro3(h, h->ws, h->ws + n, h->ws + 4 * n);
  const int nb = int(std::min<long long>(lbk3::kReduceBlocks, blocks3(n)));
  hipLaunchKernelGGL(lbk3::k_reduce3, dim3(nb), dim3(256), 0, h->stream, h->ws, part, h->geo);
  hipLaunchKernelGGL(lbk3::k_final3, dim3(1), dim3(256), 0, h->stream, part, nb, res);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(h, e, "diagnostics launch");
  double v[lbk3::kRed];
  e = hipMemcpyAsync(v, res, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail3(h, e, "diagnostics copy");
  out->mass = v[0];
  out->mom_x = v[1];
  out->mom_y = v[2];
  out->mom_z = v[3];
  out->flux_x = v[4];
  out->flux_y = v[5];
  out->flux_z = v[6];
  out->e_kin = v[7];
  out->e_mag = v[8];
  out->nonfinite = int64_t(v[9]);
  out->max_abs_divB = v[10];
  out->max_u = v[11];
  out->step = h->step;
  if (out->nonfinite > 0)
    return fail3(h, LBMHD_ERR_NONFINITE,
                 std::to_string(out->nonfinite) + " sites hold non-finite populations");
  return LBMHD_OK;
}

int lbmhd3_get_populations(lbmhd3_t* h, double* out) {
  if (int rc = need3(h)) return rc;
  if (!out) return fail3(h, LBMHD_ERR_INVALID_ARG, "null output");
  if (h->p.storage == LBMHD_FP32)
    hipLaunchKernelGGL(lbk3::k_decode3<LBMHD_FP32>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, static_cast<const float*>(h->lat[h->cur]), out, h->geo);
  else
    hipLaunchKernelGGL(lbk3::k_decode3<LBMHD_FP16>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, static_cast<const _Float16*>(h->lat[h->cur]), out, h->geo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(h, e, "decode launch");
  return LBMHD_OK;
}

int lbmhd3_set_populations(lbmhd3_t* h, const double* in, int64_t step) {
  if (int rc = need3(h)) return rc;
  if (!in || step < 0) return fail3(h, LBMHD_ERR_INVALID_ARG, "null input or negative step");
  if (h->p.storage == LBMHD_FP32)
    hipLaunchKernelGGL(lbk3::k_encode3<LBMHD_FP32>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, in, static_cast<float*>(h->lat[0]), h->geo);
  else
    hipLaunchKernelGGL(lbk3::k_encode3<LBMHD_FP16>, dim3(blocks3(sites3(h))), dim3(256), 0,
                       h->stream, in, static_cast<_Float16*>(h->lat[0]), h->geo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(h, e, "encode launch");
  h->cur = 0;
  h->step = step;
  return LBMHD_OK;
}

const char* lbmhd3_last_error(const lbmhd3_t* h) { return h ? h->err.c_str() : ""; }

}  // extern "C"
