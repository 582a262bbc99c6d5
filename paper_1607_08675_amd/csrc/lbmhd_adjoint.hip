// lbmhd_adjoint.hip -- reverse-mode (adjoint) kernels of the lattice
// Boltzmann MHD step on gfx950.
//
// The forward step is x_{n+1}(x) = C(pre(x)), pre_i(x) = x_n,i(x - c_i): a
// periodic gather S followed by the per-site collision C (moment-space MRT
// for f, single-rate relaxation for g, Smagorinsky-MHD relaxation times).
// Its transpose is lam_n = S^T J_C(pre)^T lam_{n+1}.  Adjoint lattices are
// kept in streamed position: plane i at site x + c_i holds dJ/dx_i(x), the
// sensitivity of population i stored where that population arrives after
// the next streaming (nu = S lam, nu_i(y) = lam_i(y - c_i)).  The reverse step
// then is nu_n = J_C(pre)^T S^T nu_{n+1}: every site recomputes the collision
// from the gathered x_n, gathers its own lam_{n+1,i}(x) = nu_{n+1,i}(x + c_i),
// applies the hand-derived transposed Jacobian and stores nu_n at x.  All
// shifted accesses are loads; every store is aligned (a scatter of shifted
// stores leaves partial cache lines at tile edges and measured 15% slower).
// The derivatives with respect to the closure constants C_Sv (eddy
// viscosity) and C_Sb (eddy resistivity) are accumulated per thread block in
// FP64, each into a slot owned by that block.
//
// Reverse-mode rules follow the forward collision operation by operation;
// the kinks of |A| and of the norm Q take derivative 0 at exactly 0.
#include <math.h>

#include <type_traits>

#include "lbmhd_impl.h"
#include "lbmhd_step_dev.h"

#ifndef LBMHD_ADJ_TX
#define LBMHD_ADJ_TX 256
#endif

namespace lbk {
namespace {

// Decoded deviations of a stored state, as the forward step decodes them
// (FP16: the stored half times 2^-10).
template <int ST>
using Dec = Codec<ST>;

// One element of a plane with a uniform base and a 32-bit element offset.
template <typename T>
__device__ __forceinline__ T ld_elem(const T* __restrict__ base, unsigned off) {
  return ld_plane<T>(base, off);
}

struct AdjConsts {
  float dcf;  // d(18 C_Sv Delta^2) / dC_Sv
  float dcm;  // d(36 C_Sb Delta^2) / dC_Sb
};

// Contributions of one site to dJ/dC_Sv and dJ/dC_Sb.
struct CsGrad {
  float v, b;
};

// Filter-width parts of the kinetic closure's equilibrium moments (added to
// M3^eq, M4^eq, M7^eq = M8^eq and to the u x B term E of g^eq), or their
// adjoints.
struct KinTerms {
  float m3, m4, m78, e;
};

// lam (19 values, in: adjoint of the post-collision populations; out:
// adjoint of the pre-collision populations) for the collision at the
// pre-collision state f[9], g[10] (deviation variables).  Returns the
// site's contributions to dJ/dC_Sv and dJ/dC_Sb.  With KIN the equilibria
// carry the kinetic closure's terms kc (held fixed here: their dependence on
// the site's own and its neighbours' moments is taken by the caller from the
// adjoints written to *kcb).
template <bool LES, bool KIN = false>
__device__ __forceinline__ CsGrad collide_adjoint(const float (&f)[9], const float (&g)[10],
                                                 float (&lf)[9], float (&lg)[10],
                                                 const Rates& r, const AdjConsts& ac,
                                                 const KinTerms& kc = KinTerms{0.f, 0.f, 0.f, 0.f},
                                                 KinTerms* kcb = nullptr) {
  // Every multiply-add is written out and no other contraction is allowed,
  // so each kernel that inlines this function rounds it identically (two
  // reverse steps in one pass equal two single ones bit for bit).
#pragma clang fp contract(off)
  // ---- forward recompute of what the reverse sweep needs (the forward
  // collision's quantities)
  const float a13 = f[1] + f[3], a24 = f[2] + f[4];
  const float d13 = f[1] - f[3], d24 = f[2] - f[4];
  const float s57 = f[5] + f[7], s68 = f[6] + f[8];
  const float d57 = f[5] - f[7], d68 = f[6] - f[8];
  const float dd = s57 + s68;
  const float drho = f[0] + a13 + a24 + dd;
  const float rho = 1.0f + drho;
  const float jx = d13 + d57 - d68;
  const float jy = d24 + d57 + d68;
  const float M3 = s57 - s68;
  const float M4 = a13 - a24;
  const float ir = frcp(rho);
  const float ux = jx * ir, uy = jy * ir;
  const float Bx = (g[0] + g[1]) + (g[2] + g[3]) + g[4];
  const float By = (g[5] + g[6]) + (g[7] + g[8]) + g[9];
  float n3 = M3 - fmaf(jx, uy, -(Bx * By));
  float n4 = M4 - (fmaf(jx, ux, -(jy * uy)) - fmaf(Bx, Bx, -(By * By)));
  float E = fmaf(ux, By, -(uy * Bx));
  if (KIN) {
    n3 -= kc.m3;
    n4 -= kc.m4;
    E += kc.e;
  }
  float s3q, sm, Q = 0.0f, Rr = 1.0f, tau = 1.0f, A = 0.0f, Rm = 1.0f, taum = 1.0f;
  if (LES) {
    Q = fsqrt(fmaf(n4, n4, 4.0f * (n3 * n3)));
    Rr = fsqrt(fmaf(r.cf * Q, ir, r.tau0sq));
    tau = 0.5f * (r.tau0 + Rr);
    s3q = 0.25f * frcp(tau);
    A = fmaf(-2.0f, E, (g[6] - g[8]) - (g[2] - g[4]));
    Rm = fsqrt(fmaf(r.cm, fabsf(A), r.taum0sq));
    taum = 0.5f * (r.taum0 + Rm);
    sm = frcp(taum);
  } else {
    s3q = r.s3q;
    sm = r.sm;
  }
  const float bx6 = Bx * (1.0f / 6.0f), by6 = By * (1.0f / 6.0f), he = 0.5f * E;
  const float geq[10] = {fmaf(-4.0f, bx6, Bx), bx6, bx6 - he, bx6, bx6 + he,
                         fmaf(-4.0f, by6, By), by6 + he, by6, by6 - he, by6};

  // ---- reverse
  // f* = f - K r, K_ij = T_ji:  rbar_j = -(T lam*_f)_j, j = 3..8.
  const float la13 = lf[1] + lf[3], la24 = lf[2] + lf[4];
  const float ld13 = lf[1] - lf[3], ld24 = lf[2] - lf[4];
  const float ls57 = lf[5] + lf[7], ls68 = lf[6] + lf[8];
  const float ld57 = lf[5] - lf[7], ld68 = lf[6] - lf[8];
  const float ldd = ls57 + ls68;
  const float ljx = ld13 + ld57 - ld68, ljy = ld24 + ld57 + ld68;
  const float rb3 = -(ls57 - ls68);
  const float rb4 = -(la13 - la24);
  const float rb5 = -fmaf(-3.0f, ld13, ljx);
  const float rb6 = -fmaf(-3.0f, ld24, ljy);
  const float rb7 = -fmaf(4.0f, lf[0], fmaf(-5.0f, la13 + la24, 4.0f * ldd));
  const float rb8 = -fmaf(4.0f, lf[0], -ldd);
  float nb3 = s3q * rb3, nb4 = s3q * rb4;
  const float nb5 = r.s5q * rb5, nb6 = r.s5q * rb6;
  const float nb7 = r.s7q * rb7, nb8 = r.s8q * rb8;
  const float s3qb = fmaf(n3, rb3, n4 * rb4);

  // g* = g - sm (g - geq)
  float smb = 0.0f, geqb[10], lgo[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    smb = fmaf(-lg[q], g[q] - geq[q], smb);
    geqb[q] = sm * lg[q];
    lgo[q] = fmaf(-sm, lg[q], lg[q]);
  }
  float Bxb = fmaf(1.0f / 3.0f, geqb[0], (1.0f / 6.0f) * (geqb[1] + geqb[2] + geqb[3] + geqb[4]));
  float Byb = fmaf(1.0f / 3.0f, geqb[5], (1.0f / 6.0f) * (geqb[6] + geqb[7] + geqb[8] + geqb[9]));
  float Eb = 0.5f * (-geqb[2] + geqb[4] + geqb[6] - geqb[8]);

  CsGrad dcs{0.0f, 0.0f};
  float irb = 0.0f;
  if (LES) {
    // sm = 1 / taum, taum = (taum0 + Rm) / 2, Rm = sqrt(taum0^2 + cm |A|)
    const float taumb = -smb * sm * sm;
    const float amb = 0.5f * taumb * 0.5f * frcp(Rm);
    const float absAb = r.cm * amb;
    const float Ab = A > 0.0f ? absAb : (A < 0.0f ? -absAb : 0.0f);
    dcs.b = fmaf(ac.dcm * fabsf(A), amb, dcs.b);
    lgo[6] += Ab;
    lgo[8] -= Ab;
    lgo[2] -= Ab;
    lgo[4] += Ab;
    Eb = fmaf(-2.0f, Ab, Eb);
    // s3q = 1 / (4 tau), tau = (tau0 + Rr) / 2, Rr = sqrt(tau0^2 + cf Q ir)
    const float itau = frcp(tau);
    const float taub = -0.25f * s3qb * itau * itau;
    const float ab = 0.5f * taub * 0.5f * frcp(Rr);
    const float Qb = r.cf * ir * ab;
    irb = fmaf(r.cf * Q, ab, irb);
    dcs.v = fmaf(ac.dcf * Q * ir, ab, dcs.v);
    if (Q > 0.0f) {
      const float iQ = frcp(Q);
      nb4 = fmaf(Qb * n4, iQ, nb4);
      nb3 = fmaf(4.0f * Qb * n3, iQ, nb3);
    }
  }
  if (KIN) {
    kcb->m3 = -nb3;
    kcb->m4 = -nb4;
    kcb->m78 = -(nb7 + nb8);
    kcb->e = Eb;
  }
  // E = ux By - uy Bx (+ e)
  float uxb = Eb * By, uyb = -Eb * Bx;
  Byb = fmaf(Eb, ux, Byb);
  Bxb = fmaf(-Eb, uy, Bxb);
  // n3 = M3 - jx jy ir + Bx By
  float jxb = -nb3 * jy * ir, jyb = -nb3 * jx * ir;
  irb = fmaf(-nb3 * jx, jy, irb);
  Bxb = fmaf(nb3, By, Bxb);
  Byb = fmaf(nb3, Bx, Byb);
  // n4 = M4 - (jx^2 - jy^2) ir + Bx^2 - By^2
  jxb = fmaf(-2.0f * nb4 * jx, ir, jxb);
  jyb = fmaf(2.0f * nb4 * jy, ir, jyb);
  irb = fmaf(-nb4, fmaf(jx, jx, -(jy * jy)), irb);
  Bxb = fmaf(2.0f * nb4, Bx, Bxb);
  Byb = fmaf(-2.0f * nb4, By, Byb);
  // n5 = M5 + jx, n6 = M6 + jy
  jxb += nb5;
  jyb += nb6;
  // n7, n8 through jj = (jx^2 + jy^2) ir and drho
  const float jjb = 3.0f * (nb7 + nb8);
  float drhob = -(5.0f / 3.0f) * nb8;
  jxb = fmaf(2.0f * jjb * jx, ir, jxb);
  jyb = fmaf(2.0f * jjb * jy, ir, jyb);
  irb = fmaf(jjb, fmaf(jx, jx, jy * jy), irb);
  // ux = jx ir, uy = jy ir
  jxb = fmaf(uxb, ir, jxb);
  jyb = fmaf(uyb, ir, jyb);
  irb = fmaf(uxb, jx, fmaf(uyb, jy, irb));
  // ir = 1 / (1 + drho)
  drhob = fmaf(-irb * ir, ir, drhob);
  // moments M3..M8 = T_r f; drho = sum f; j = sum c f
  const float Mb3 = nb3, Mb4 = nb4, Mb5 = nb5, Mb6 = nb6, Mb7 = nb7, Mb8 = nb8;
  lf[0] += fmaf(4.0f, Mb7 + Mb8, drhob);
  lf[1] += fmaf(-5.0f, Mb7, fmaf(-2.0f, Mb5, drhob + jxb + Mb4));
  lf[2] += fmaf(-5.0f, Mb7, fmaf(-2.0f, Mb6, drhob + jyb - Mb4));
  lf[3] += fmaf(-5.0f, Mb7, fmaf(2.0f, Mb5, drhob - jxb + Mb4));
  lf[4] += fmaf(-5.0f, Mb7, fmaf(2.0f, Mb6, drhob - jyb - Mb4));
  const float c58 = fmaf(4.0f, Mb7, -Mb8);
  lf[5] += drhob + jxb + jyb + Mb3 + Mb5 + Mb6 + c58;
  lf[6] += drhob - jxb + jyb - Mb3 - Mb5 + Mb6 + c58;
  lf[7] += drhob - jxb - jyb + Mb3 - Mb5 - Mb6 + c58;
  lf[8] += drhob + jxb - jyb - Mb3 + Mb5 - Mb6 + c58;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    lg[k] = lgo[k] + Bxb;
    lg[5 + k] = lgo[5 + k] + Byb;
  }
  return dcs;
}

template <int ST, bool LES>
__global__ __launch_bounds__(LBMHD_ADJ_TX) void k_adj_step(
    const typename Dec<ST>::T* __restrict__ st, const float* __restrict__ lam_next,
    float* __restrict__ lam_prev, double* __restrict__ acc, Geom geo, Geom ga, Rates rt,
    AdjConsts ac, int tiles_x) {
  using D = Dec<ST>;
  const int b = int(blockIdx.x);
  const int x = (b % tiles_x) * LBMHD_ADJ_TX + int(threadIdx.x);
  const int y = b / tiles_x;
  CsGrad dcs{0.0f, 0.0f};
  if (x < geo.nx) {
    const int xm = x == 0 ? geo.nx - 1 : x - 1;
    const int xp = x == geo.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? geo.ny - 1 : y - 1;
    const int yp = y == geo.ny - 1 ? 0 : y + 1;
    // offsets of x - c_i in the state layout and of x + c_i in the adjoint
    // layout
    const unsigned r0 = unsigned(y) * geo.pitch, rm = unsigned(ym) * geo.pitch,
                   rp = unsigned(yp) * geo.pitch;
    const unsigned o[9] = {r0 + x,  r0 + xm, rm + x,  r0 + xp, rp + x,
                           rm + xm, rm + xp, rp + xp, rp + xm};
    const unsigned a0 = unsigned(y) * ga.pitch, am = unsigned(ym) * ga.pitch,
                   ap = unsigned(yp) * ga.pitch;
    const unsigned on[9] = {a0 + x,  a0 + xp, ap + x,  a0 + xm, am + x,
                            ap + xp, ap + xm, am + xm, am + xp};
    const long long P = geo.plane, PA = ga.plane;
    float f[9], g[10], lf[9], lg[10];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = D::dec(ld_elem(st + i * P, o[i]));
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      g[k] = D::dec(ld_elem(st + (9 + k) * P, o[k]));
      g[5 + k] = D::dec(ld_elem(st + (14 + k) * P, o[k]));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) lf[i] = ld_elem(lam_next + i * PA, on[i]);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      lg[k] = ld_elem(lam_next + (9 + k) * PA, on[k]);
      lg[5 + k] = ld_elem(lam_next + (14 + k) * PA, on[k]);
    }
    dcs = collide_adjoint<LES>(f, g, lf, lg, rt, ac);
    const unsigned oc = a0 + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) st_plane_nt(lam_prev + i * PA, oc, lf[i]);
#pragma unroll
    for (int q = 0; q < 10; ++q) st_plane_nt(lam_prev + (9 + q) * PA, oc, lg[q]);
  }
  if (LES) {
    // acc[b] gains the block's dJ/dC_Sv, acc[gridDim.x + b] its dJ/dC_Sb
    __shared__ double sh[2][LBMHD_ADJ_TX];
    sh[0][threadIdx.x] = double(dcs.v);
    sh[1][threadIdx.x] = double(dcs.b);
    __syncthreads();
    for (int w = LBMHD_ADJ_TX / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
        sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      acc[blockIdx.x] += sh[0][0];
      acc[gridDim.x + blockIdx.x] += sh[1][0];
    }
  }
}

// Offsets of x + c_i (i = 0..8, D2Q9 order; the five D2Q5 vectors are the
// first five) in the adjoint layout: where the adjoint of population i at x
// is kept.
__device__ __forceinline__ void streamed_offsets(const Geom& ga, int x, int y, unsigned (&on)[9]) {
  const int xm = x == 0 ? ga.nx - 1 : x - 1;
  const int xp = x == ga.nx - 1 ? 0 : x + 1;
  const unsigned a0 = unsigned(y) * ga.pitch,
                 am = unsigned(y == 0 ? ga.ny - 1 : y - 1) * ga.pitch,
                 ap = unsigned(y == ga.ny - 1 ? 0 : y + 1) * ga.pitch;
  on[0] = a0 + x;
  on[1] = a0 + xp;
  on[2] = ap + x;
  on[3] = a0 + xm;
  on[4] = am + x;
  on[5] = ap + xp;
  on[6] = ap + xm;
  on[7] = am + xm;
  on[8] = am + xp;
}

// lam = dJ/dx for J = sum |rho u|^2 / (2 rho) + |B|^2 / 2:
// dJ/df_i = c_i . u - |u|^2 / 2, dJ/dg = B.
template <int ST>
__global__ void k_adj_seed(const typename Dec<ST>::T* __restrict__ st, float* __restrict__ lam,
                           Geom geo, Geom ga) {
  using D = Dec<ST>;
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  const long long o = (long long)y * geo.pitch + x;
  double v[kNPop];
#pragma unroll
  for (int q = 0; q < kNPop; ++q) v[q] = double(D::dec(st[q * geo.plane + o]));
  double dr = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dr += v[i];
    jx += kCx[i] * v[i];
    jy += kCy[i] * v[i];
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    bx += v[9 + k];
    by += v[14 + k];
  }
  const double rho = 1.0 + dr, ux = jx / rho, uy = jy / rho, h = 0.5 * (ux * ux + uy * uy);
  unsigned on[9];
  streamed_offsets(ga, x, y, on);
#pragma unroll
  for (int i = 0; i < 9; ++i) lam[i * ga.plane + on[i]] = float(kCx[i] * ux + kCy[i] * uy - h);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    lam[(9 + k) * ga.plane + on[k]] = float(bx);
    lam[(14 + k) * ga.plane + on[k]] = float(by);
  }
}

// lam = scale * dL/dx for L = sum |u - u_t|^2 + |B - B_t|^2:
// dL/df_i = 2 (u - u_t) . (c_i - u) / rho, dL/dg = 2 (B - B_t).
template <int ST>
__global__ void k_adj_seed_mismatch(const typename Dec<ST>::T* __restrict__ st,
                                    const double* __restrict__ ux_t,
                                    const double* __restrict__ uy_t,
                                    const double* __restrict__ bx_t,
                                    const double* __restrict__ by_t, double scale,
                                    float* __restrict__ lam, Geom geo, Geom ga) {
  using D = Dec<ST>;
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  const long long o = (long long)y * geo.pitch + x;
  double v[kNPop];
#pragma unroll
  for (int q = 0; q < kNPop; ++q) v[q] = double(D::dec(st[q * geo.plane + o]));
  double dr = 0.0, jx = 0.0, jy = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dr += v[i];
    jx += kCx[i] * v[i];
    jy += kCy[i] * v[i];
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    bx += v[9 + k];
    by += v[14 + k];
  }
  const double rho = 1.0 + dr, ux = jx / rho, uy = jy / rho;
  const double eu = 2.0 * scale * (ux - ux_t[s]) / rho, ev = 2.0 * scale * (uy - uy_t[s]) / rho;
  unsigned on[9];
  streamed_offsets(ga, x, y, on);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    lam[i * ga.plane + on[i]] = float(eu * (kCx[i] - ux) + ev * (kCy[i] - uy));
  const double gx = 2.0 * scale * (bx - bx_t[s]), gy = 2.0 * scale * (by - by_t[s]);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    lam[(9 + k) * ga.plane + on[k]] = float(gx);
    lam[(14 + k) * ga.plane + on[k]] = float(gy);
  }
}

// Pull lam0 (streamed position) back through x_0 = (f^eq(rho0, u0, B0),
// g^eq(u0, B0)).
__global__ void k_adj_fields(const float* __restrict__ lam, const double* __restrict__ rho0,
                             const double* __restrict__ ux0, const double* __restrict__ uy0,
                             const double* __restrict__ bx0, const double* __restrict__ by0,
                             double* __restrict__ gux, double* __restrict__ guy,
                             double* __restrict__ gbx, double* __restrict__ gby, Geom ga,
                             int nx, int ny) {
  const long long n = (long long)nx * ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / nx), x = int(s % nx);
  unsigned on[9];
  streamed_offsets(ga, x, y, on);
  const double rho = rho0[s], ux = ux0[s], uy = uy0[s], bx = bx0[s], by = by0[s];
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double l = double(lam[i * ga.plane + on[i]]);
    const double cx = kCx[i], cy = kCy[i], w = kW[i];
    const double cu = cx * ux + cy * uy, cb = cx * bx + cy * by, c2 = cx * cx + cy * cy;
    // f^eq_i = w rho (1 + 3 cu + 4.5 cu^2 - 1.5 u^2) + 4.5 w (B^2 c^2 / 2 - cb^2)
    a += l * w * rho * (3.0 * cx + 9.0 * cu * cx - 3.0 * ux);
    b += l * w * rho * (3.0 * cy + 9.0 * cu * cy - 3.0 * uy);
    c += l * 4.5 * w * (bx * c2 - 2.0 * cb * cx);
    d += l * 4.5 * w * (by * c2 - 2.0 * cb * cy);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double lx = double(lam[(9 + k) * ga.plane + on[k]]);
    const double ly = double(lam[(14 + k) * ga.plane + on[k]]);
    const double cx = kMx[k], cy = kMy[k], w = kWm[k];
    const double cu = cx * ux + cy * uy, cb = cx * bx + cy * by;
    // g^eq_x = w (B_x + 3 (cu B_x - cb u_x)), g^eq_y = w (B_y + 3 (cu B_y - cb u_y))
    a += lx * w * 3.0 * (cx * bx - cb) + ly * w * 3.0 * cx * by;
    b += lx * w * 3.0 * cy * bx + ly * w * 3.0 * (cy * by - cb);
    c += lx * w * (1.0 + 3.0 * (cu - cx * ux)) + ly * w * 3.0 * (-cx * uy);
    d += lx * w * 3.0 * (-cy * ux) + ly * w * (1.0 + 3.0 * (cu - cy * uy));
  }
  gux[s] = a;
  guy[s] = b;
  gbx[s] = c;
  gby[s] = d;
}

// ------------------------------------------------------ kinetic closure
// The kinetic closure's equilibrium terms depend on the gradients of
// rho - 1, j, B over the eight neighbours (isotropic D2Q9 difference
// d_a X = 3 sum_i w_i c_ia X(x + c_i)) and on the site's own moments, all of
// the gathered pre-collision state.  The reverse step has two parts per site.
// Part A: recompute the forward terms, apply the transposed collision
// Jacobian with those terms held fixed, and carry the adjoints of the terms
// back to the site's own moments (added to its populations) and to the ten
// gradient components.  Part B: add the transposed stencil of the
// neighbours' gradient adjoints to the site's moment adjoints and map them
// onto its populations.  One kernel walks strips of rows and takes both
// (k_adj_kin below).

// The closure's terms from the gradients gx, gy and the site's moments v of
// (rho - 1, j_x, j_y, B_x, B_y); c12 = Delta^2 / 12.  Same operations as the
// forward step.
__device__ __forceinline__ KinTerms kin_terms(const float (&gx)[5], const float (&gy)[5],
                                              const float (&v)[5], float c12) {
  const float ir = frcp(1.0f + v[0]);
  const float grx = gx[0] * ir, gry = gy[0] * ir;
  float hx[4], hy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hx[k] = gx[k + 1] - v[k + 1] * grx;
    hy[k] = gy[k + 1] - v[k + 1] * gry;
  }
  const float cr = c12 * ir;
  const float jxjx = cr * (hx[0] * hx[0] + hy[0] * hy[0]);
  const float jyjy = cr * (hx[1] * hx[1] + hy[1] * hy[1]);
  KinTerms k;
  k.m3 = cr * (hx[0] * hx[1] + hy[0] * hy[1]) - c12 * (gx[3] * gx[4] + gy[3] * gy[4]);
  k.m4 = (jxjx - jyjy) - c12 * ((gx[3] * gx[3] + gy[3] * gy[3]) - (gx[4] * gx[4] + gy[4] * gy[4]));
  k.m78 = -3.0f * (jxjx + jyjy);
  k.e = cr * ((hx[0] * hx[3] + hy[0] * hy[3]) - (hx[1] * hx[2] + hy[1] * hy[2]));
  return k;
}

// Adjoint of kin_terms: from the adjoints b of the four terms, the adjoints of
// the gradients (gxb, gyb) and of the site's moments (vb).
__device__ __forceinline__ void kin_terms_adjoint(const float (&gx)[5], const float (&gy)[5],
                                                  const float (&v)[5], float c12,
                                                  const KinTerms& b, float (&gxb)[5],
                                                  float (&gyb)[5], float (&vb)[5]) {
  const float ir = frcp(1.0f + v[0]);
  const float grx = gx[0] * ir, gry = gy[0] * ir;
  float hx[4], hy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hx[k] = gx[k + 1] - v[k + 1] * grx;
    hy[k] = gy[k + 1] - v[k + 1] * gry;
  }
  const float cr = c12 * ir;
  // jxjx enters m4 and m78, jyjy enters m4 (with a minus) and m78
  const float jxjxb = b.m4 - 3.0f * b.m78, jyjyb = -b.m4 - 3.0f * b.m78;
  const float crb = b.m3 * (hx[0] * hx[1] + hy[0] * hy[1]) +
                    b.e * ((hx[0] * hx[3] + hy[0] * hy[3]) - (hx[1] * hx[2] + hy[1] * hy[2])) +
                    jxjxb * (hx[0] * hx[0] + hy[0] * hy[0]) +
                    jyjyb * (hx[1] * hx[1] + hy[1] * hy[1]);
  const float hxb[4] = {cr * (b.m3 * hx[1] + b.e * hx[3] + 2.0f * jxjxb * hx[0]),
                        cr * (b.m3 * hx[0] - b.e * hx[2] + 2.0f * jyjyb * hx[1]),
                        -cr * b.e * hx[1], cr * b.e * hx[0]};
  const float hyb[4] = {cr * (b.m3 * hy[1] + b.e * hy[3] + 2.0f * jxjxb * hy[0]),
                        cr * (b.m3 * hy[0] - b.e * hy[2] + 2.0f * jyjyb * hy[1]),
                        -cr * b.e * hy[1], cr * b.e * hy[0]};
#pragma unroll
  for (int k = 0; k < 5; ++k) gxb[k] = gyb[k] = vb[k] = 0.0f;
  // the product terms B B use the plain gradients
  gxb[3] = -c12 * (b.m3 * gx[4] + 2.0f * b.m4 * gx[3]);
  gxb[4] = -c12 * (b.m3 * gx[3] - 2.0f * b.m4 * gx[4]);
  gyb[3] = -c12 * (b.m3 * gy[4] + 2.0f * b.m4 * gy[3]);
  gyb[4] = -c12 * (b.m3 * gy[3] - 2.0f * b.m4 * gy[4]);
  // h_k = g_(k+1) - v_(k+1) g_0 ir
  float grxb = 0.0f, gryb = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    gxb[k + 1] += hxb[k];
    gyb[k + 1] += hyb[k];
    vb[k + 1] -= hxb[k] * grx + hyb[k] * gry;
    grxb -= hxb[k] * v[k + 1];
    gryb -= hyb[k] * v[k + 1];
  }
  gxb[0] += grxb * ir;
  gyb[0] += gryb * ir;
  const float irb = grxb * gx[0] + gryb * gy[0] + c12 * crb;
  vb[0] -= irb * ir * ir;
}

// Adjoints of (rho - 1, j_x, j_y, B_x, B_y) added to the populations they are
// sums of.
__device__ __forceinline__ void add_moment_adjoints(const float (&m)[5], float (&lf)[9],
                                                    float (&lg)[10]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) lf[i] += m[0] + kCx[i] * m[1] + kCy[i] * m[2];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    lg[k] += m[3];
    lg[5 + k] += m[4];
  }
}

// Both parts in one walk.  A block owns a tile of kT3Cols columns and a strip
// of `rows` rows: pass t gathers row y0 + t (its moments go to a 3-row LDS
// ring with two halo columns on each side), applies part A to row
// a = y0 - 1 + t on the tile's columns and one halo column on each side (the
// ten gradient adjoints go to a second 3-row LDS ring), and part B to row
// a - 1, whose part-A adjoint the thread carried from the last pass in
// registers; lam_prev is written once (with FP32 states the gather of pass
// t + 1 is issued during pass t).  The fifth wave owns the halo columns
// (lanes 0 .. 3: x0 - 2, x0 - 1, x0 + wt, x0 + wt + 1; part A on the inner
// two).  Two barriers per pass.  HBM bytes per site: the state gather, the
// lam_next gather and the lam_prev store, plus four halo rows of gathers and
// two of part A per strip.  The closure-constant derivatives are summed per
// block over the sites it owns (slots b and nslots + b of acc).
template <int ST, bool LES>
__global__ __launch_bounds__(kT3Threads) void k_adj_kin(
    const typename Dec<ST>::T* __restrict__ st, const float* __restrict__ lam_next,
    float* __restrict__ lam_prev, double* __restrict__ acc, Geom geo, Geom ga, Rates rt,
    AdjConsts ac, float c12, int tiles_x, int rows, int nslots) {
  using D = Dec<ST>;
  __shared__ float mac[3][5][kT3Cols + 4];    // moments: column lc + 2
  __shared__ float gbr[3][10][kT3Cols + 2];   // gradient adjoints: column lc + 1
  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane, PA = ga.plane;
  const int tile = int(blockIdx.x) % tiles_x, strip = int(blockIdx.x) / tiles_x;
  const int x0 = tile * kT3Cols, y0 = strip * rows;
  const int wt = min(kT3Cols, nx - x0), h = min(rows, ny - y0);
  const int tid = int(threadIdx.x);
  // the thread's column lc: its own (threads 0 .. kT3Cols - 1) or a halo one
  int lc = tid;
  bool hasm = tid < wt;   // gathers the column's populations and moments
  if (tid >= kT3Cols) {
    const int k = tid - kT3Cols;
    hasm = k < 4;
    lc = k == 0 ? -2 : (k == 1 ? -1 : (k == 2 ? wt : wt + 1));
  }
  const bool hasa = hasm && lc >= -1 && lc <= wt;   // part A
  const bool own = hasm && lc >= 0 && lc < wt;      // part B and lam_prev
  const int mc = lc + 2, gc = lc + 1;
  int x = (x0 + lc) % nx;
  if (x < 0) x += nx;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  // gathered pre-collision populations of row yy (any integer, periodic) at
  // this thread's column: x_n(. - c_q)
  auto gather = [&](int yy, float (&p)[19]) {
    yy %= ny;
    if (yy < 0) yy += ny;
    const int ym = yy == 0 ? ny - 1 : yy - 1, yp = yy == ny - 1 ? 0 : yy + 1;
    const unsigned r0 = unsigned(yy) * geo.pitch, rm = unsigned(ym) * geo.pitch,
                   rp = unsigned(yp) * geo.pitch;
    const unsigned o[9] = {r0 + x, r0 + xm, rm + x, r0 + xp, rp + x,
                           rm + xm, rm + xp, rp + xp, rp + xm};
#pragma unroll
    for (int i = 0; i < 9; ++i) p[i] = D::dec(ld_elem(st + i * P, o[i]));
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      p[9 + k] = D::dec(ld_elem(st + (9 + k) * P, o[k]));
      p[14 + k] = D::dec(ld_elem(st + (14 + k) * P, o[k]));
    }
  };
  auto moments = [&](const float (&p)[19], int slot) {
    mac[slot][0][mc] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7])) + p[8];
    mac[slot][1][mc] = (p[1] - p[3]) + (p[5] - p[7]) - (p[6] - p[8]);
    mac[slot][2][mc] = (p[2] - p[4]) + (p[5] - p[7]) + (p[6] - p[8]);
    mac[slot][3][mc] = (p[9] + p[10]) + (p[11] + p[12]) + p[13];
    mac[slot][4][mc] = (p[14] + p[15]) + (p[16] + p[17]) + p[18];
  };
  CsGrad dcs{0.0f, 0.0f};
  // With FP32 states the next pass's gather is issued right after the first
  // barrier and flies during parts A and B (1.03 / 1.18 ms per step at 4096^2
  // with les = 2 / 3, against 1.31 / 1.30 gathering at the start of each
  // pass); with FP16 states that ran slower (1.50 against 1.19 ms).
  constexpr bool kPf = ST == LBMHD_FP32;
  float cur[19], nxt[19], nx2[19];
  float clf[9], clg[10];   // part-A adjoint of the last pass's row (own columns)
#pragma unroll
  for (int i = 0; i < 9; ++i) clf[i] = 0.0f;
#pragma unroll
  for (int q = 0; q < 10; ++q) clg[q] = 0.0f;
  if (hasm) {
    gather(y0 - 2, nxt);
    moments(nxt, 0);
    gather(y0 - 1, cur);
    moments(cur, 1);
    if (kPf) gather(y0, nxt);
  }
  for (int t = 0; t < h + 2; ++t) {
    const int a = y0 - 1 + t;
    const int sm = t % 3, s0 = (t + 1) % 3, sp = (t + 2) % 3;
    if (hasm) {
      if (!kPf) gather(a + 1, nxt);
      moments(nxt, sp);
    }
    __syncthreads();
    if (kPf && hasm && t + 1 < h + 2) gather(a + 2, nx2);
    // part A at row a
    float lf[9], lg[10];
    if (hasa) {
      const int c = mc;
      float gx[5], gy[5], v[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const float e = mac[s0][k][c + 1], w = mac[s0][k][c - 1];
        const float nn = mac[sp][k][c], ss = mac[sm][k][c];
        const float ne = mac[sp][k][c + 1], nw = mac[sp][k][c - 1];
        const float se = mac[sm][k][c + 1], sw = mac[sm][k][c - 1];
        gx[k] = (1.0f / 3.0f) * (e - w) + (1.0f / 12.0f) * ((ne - nw) + (se - sw));
        gy[k] = (1.0f / 3.0f) * (nn - ss) + (1.0f / 12.0f) * ((ne + nw) - (se + sw));
        v[k] = mac[s0][k][c];
      }
      const KinTerms kc = kin_terms(gx, gy, v, c12);
      // lam_{n+1} of this site's populations, kept at x + c_i
      int ya = a % ny;
      if (ya < 0) ya += ny;
      const int ym = ya == 0 ? ny - 1 : ya - 1, yp = ya == ny - 1 ? 0 : ya + 1;
      const unsigned a0 = unsigned(ya) * ga.pitch, am = unsigned(ym) * ga.pitch,
                     ap = unsigned(yp) * ga.pitch;
      const unsigned on[9] = {a0 + x, a0 + xp, ap + x, a0 + xm, am + x,
                              ap + xp, ap + xm, am + xm, am + xp};
      float f[9], g[10];
#pragma unroll
      for (int i = 0; i < 9; ++i) lf[i] = ld_elem(lam_next + i * PA, on[i]);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        lg[k] = ld_elem(lam_next + (9 + k) * PA, on[k]);
        lg[5 + k] = ld_elem(lam_next + (14 + k) * PA, on[k]);
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = cur[i];
#pragma unroll
      for (int q = 0; q < 10; ++q) g[q] = cur[9 + q];
      KinTerms kcb;
      const CsGrad d = collide_adjoint<LES, true>(f, g, lf, lg, rt, ac, kc, &kcb);
      if (own && t >= 1 && t <= h) {
        dcs.v += d.v;
        dcs.b += d.b;
      }
      float gxb[5], gyb[5], vb[5];
      kin_terms_adjoint(gx, gy, v, c12, kcb, gxb, gyb, vb);
      add_moment_adjoints(vb, lf, lg);
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        gbr[sm][k][gc] = gxb[k];
        gbr[sm][5 + k][gc] = gyb[k];
      }
    }
    __syncthreads();
    // part B at row a - 1: rows a - 2, a - 1, a of the gradient adjoints are
    // in the slots of passes t - 2, t - 1, t
    if (own && t >= 2) {
      const int rm = (t - 2) % 3, r0 = (t - 1) % 3, rp = t % 3;
      const int c = gc;
      float eta[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        // d/d(d_x X_k) in plane k, d/d(d_y X_k) in plane 5 + k
        eta[k] = (1.0f / 3.0f) * ((gbr[r0][k][c - 1] - gbr[r0][k][c + 1]) +
                                  (gbr[rm][5 + k][c] - gbr[rp][5 + k][c])) +
                 (1.0f / 12.0f) * ((gbr[rm][k][c - 1] + gbr[rm][5 + k][c - 1]) +
                                   (gbr[rm][5 + k][c + 1] - gbr[rm][k][c + 1]) +
                                   (gbr[rp][k][c - 1] - gbr[rp][5 + k][c - 1]) -
                                   (gbr[rp][k][c + 1] + gbr[rp][5 + k][c + 1]));
      }
      add_moment_adjoints(eta, clf, clg);
      int yb = (a - 1) % ny;
      if (yb < 0) yb += ny;
      const unsigned oc = unsigned(yb) * ga.pitch + unsigned(x);
#pragma unroll
      for (int i = 0; i < 9; ++i) st_plane_nt(lam_prev + i * PA, oc, clf[i]);
#pragma unroll
      for (int q = 0; q < 10; ++q) st_plane_nt(lam_prev + (9 + q) * PA, oc, clg[q]);
    }
    if (own) {
#pragma unroll
      for (int i = 0; i < 9; ++i) clf[i] = lf[i];
#pragma unroll
      for (int q = 0; q < 10; ++q) clg[q] = lg[q];
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
      cur[q] = nxt[q];
      if (kPf) nxt[q] = nx2[q];
    }
  }
  if (LES) {
    // the block's sums into acc[b] (C_Sv) and acc[nslots + b] (C_Sb), reduced
    // in the (now idle) moment buffer
    __syncthreads();
    float* red = &mac[0][0][0];
    static_assert(3 * 5 * (kT3Cols + 4) >= 2 * kT3Threads, "moment buffer too small");
    red[tid] = dcs.v;
    red[kT3Threads + tid] = dcs.b;
    __syncthreads();
    if (tid == 0) {
      double sv = 0.0, sb = 0.0;
      for (int i = 0; i < kT3Threads; ++i) {
        sv += double(red[i]);
        sb += double(red[kT3Threads + i]);
      }
      acc[blockIdx.x] += sv;
      acc[nslots + blockIdx.x] += sb;
    }
  }
}

// ------------------------------------------- two reverse steps in one pass
// lam_t = R_t(R_{t+1}(lam_{t+2})) in the streamed placement, R_n being the
// reverse step at state x_n (k_adj_step), with x_{t+1} = C(S(x_t)) recomputed
// on chip from the stored x_t: one stored state serves two reverse steps, so
// a sweep needs every other state only.  R_n at site x reads x_n at x - c_i
// (its pre-collision gather) and lam_{n+1} at x + c_i, so lam_t at x needs
// lam_{t+1} one site out, hence x_{t+1} and lam_{t+2} two sites out and x_t
// three.  A block owns a tile of kT3Cols columns and a strip of `rows` rows
// and walks upward; pass t, with a = y0 - 2 + t:
//   A. gathers row a of x_t (columns x0 - 2 .. x0 + wt + 1) and collides it
//      with the forward collision: row a of x_{t+1}, passed through the
//      storage codec as the forward step stores it; the planes that move along
//      x go to the LDS row l1, the others stay in registers;
//   B. reverse step t + 1 at row a - 1 (columns x0 - 1 .. x0 + wt): the
//      pre-collision values of x_{t+1} from l1 and the registers, as in the
//      forward three-step kernel, and lam_{t+2} at x + c_i from HBM; the
//      result goes to l2 and the registers;
//   C. reverse step t at row a - 2 (the tile's own columns): x_t gathered
//      again (rows read in the last three passes, served by the caches) and
//      lam_{t+1} at x + c_i from l2 and the registers -- the hand-over runs
//      the other way than the forward one: a plane with c_y = +1 is read in
//      the pass that writes it, c_y = 0 one pass later, c_y = -1 two; the
//      result is stored.
// Two barriers per pass; a fifth wave owns the four halo columns.  Both
// reverse steps apply collide_adjoint to the values k_adj_step would read
// (the recomputed state equals the stored one bit for bit), and the
// closure-constant derivatives of both steps are summed per block over the
// sites the block owns (slots b and nslots + b of acc).  LESF: the forward
// step's collision takes the Smagorinsky-MHD closure (as lbmhd_step chooses
// it: not with C_S = 0); LESA: the reverse steps differentiate it.  HBM bytes per site
// for two reverse steps: x_t, lam_{t+2} and lam_t once each, plus the
// strips' halo rows and the tiles' halo columns.
template <int ST, bool LESF, bool LESA>
__global__ __launch_bounds__(kT3Threads) void k_adj_step2(
    const typename Codec<ST>::T* __restrict__ st, const float* __restrict__ lam_next,
    float* __restrict__ lam_prev, double* __restrict__ acc, Geom geo, Geom ga, Rates rt,
    AdjConsts ac, int tiles_x, int rows, int nslots) {
  // the forward recompute runs on the stored values as the forward step
  // does (FP16: in units of 2^-10); the reverse steps see deviations
  constexpr int SF = ST == LBMHD_FP32 ? LBMHD_FP32 : kFP16S;
  using CF = Codec<SF>;
  using CA = Codec<ST>;
  __shared__ float l1[kT3Rows][kT3Cols + 4];   // x_{t+1}: column lc + 2
  __shared__ float l2[kT3Rows][kT3Cols + 2];   // lam_{t+1}: column lc + 1
  __shared__ double red[2][kT3Threads];
  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane, PA = ga.plane;
  const int tile = int(blockIdx.x) % tiles_x, strip = int(blockIdx.x) / tiles_x;
  const int x0 = tile * kT3Cols, y0 = strip * rows;
  const int wt = min(kT3Cols, nx - x0), h = min(rows, ny - y0);
  // the thread's column: its own (threads 0 .. kT3Cols - 1) or a halo column
  // (lanes 0 .. 3 of the fifth wave: x0 - 2, x0 - 1, x0 + wt, x0 + wt + 1)
  const int tid = int(threadIdx.x);
  int lc = tid;
  bool has = tid < wt;
  if (tid >= kT3Cols) {
    const int k = tid - kT3Cols;
    has = k < 4;
    lc = k == 0 ? -2 : (k == 1 ? -1 : (k == 2 ? wt : wt + 1));
  }
  const bool up2 = has && lc >= -1 && lc <= wt;   // takes reverse step t + 1
  const bool up3 = has && lc >= 0 && lc < wt;     // takes reverse step t
  // LDS columns read in stages B and C: lc - c_x + c1 and lc + c_x + c2 (fixed
  // in-bounds columns for the threads that take no such step)
  const int c1 = up2 ? lc + 2 : 2;
  const int c2 = up3 ? lc + 1 : 1;
  int xc = (x0 + lc) % nx;
  if (xc < 0) xc += nx;
  const int xl = xc == 0 ? nx - 1 : xc - 1;
  const int xr = xc == nx - 1 ? 0 : xc + 1;

  // x_{t+1} of earlier passes for this thread's column (as in k_step_t3's
  // first level): z, the c_x = 0 planes by c_y; x, the c_x != 0 planes
  // already taken from column lc - c_x (6 with c_y = 0, 2 with c_y = +1)
  float z1c[3], z1u1[3], z1u2[3], x1c[6], x1u1[2], x1u2[2];
  // lam_{t+1} of earlier passes: w, the c_x = 0 planes (c_y = 0 one pass
  // back, c_y = -1 two); y, the c_x != 0 planes taken from column lc + c_x
  float w2c[3], w2d1[3], w2d2[3], y2c[6], y2d1[2], y2d2[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) z1c[k] = z1u1[k] = z1u2[k] = w2c[k] = w2d1[k] = w2d2[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) x1c[k] = y2c[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 2; ++k) x1u1[k] = x1u2[k] = y2d1[k] = y2d2[k] = 0.0f;
  double dv = 0.0, db = 0.0;
  for (int t = 0; t < h + 4; ++t) {
    // A. row a = y0 - 2 + t of x_{t+1}
    float n1c[3], n1u[3], n1d[3];
    if (has) {
      unsigned row[3];
      t2_rows(y0 - 2 + t, geo, row);
      float v[kNPop][1];
      gather_row<SF, 1>(st, P, xc, xl, xr, row, v);
      collide_sites<1, LESF, SF == kFP16S>(v, rt);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const float e = CA::dec(CF::enc(v[q][0]));
        const int k = kT2Reg[q];
        if (kT2Group[q] >= 0)
          l1[t3_row(q)][lc + 2] = e;
        else if (kPlaneCy[q] == 0)
          n1c[k] = e;
        else if (kPlaneCy[q] == 1)
          n1u[k] = e;
        else
          n1d[k] = e;
      }
    }
    __syncthreads();
    // B. reverse step t + 1 at row b = y0 - 3 + t (from pass 2 on); the l1 row
    // of this pass is read in every pass, before the next one overwrites it
    float n2c[3], n2u[3], n2d[3];
    const bool do2 = t >= 2 && up2;
    {
      float e[kT3Rows];
#pragma unroll
      for (int q = 0; q < kNPop; ++q)
        if (kT2Group[q] >= 0) e[t3_row(q)] = l1[t3_row(q)][c1 - kPlaneCx[q]];
      float pre[kNPop];
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
        if (g >= 0)
          pre[q] = g == 0 ? x1u2[i] : (g == 1 ? x1c[i] : e[t3_row(q)]);
        else
          pre[q] = kPlaneCy[q] == 0 ? z1c[k] : (kPlaneCy[q] == 1 ? z1u2[k] : n1d[k]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        x1u2[i] = x1u1[i];
        x1u1[i] = e[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) x1c[i] = e[2 + i];
      if (do2) {
        const int b = y0 - 3 + t;
        unsigned ra[3];
        t2_rows(b, ga, ra);
        // lam_{t+2} at x + c_i: row b + c_y is ra[1 - c_y]; each element is read
        // once per strip (non-temporal: the x_t rows stage C gathers again
        // stay in the caches; 5% faster at 4096^2)
        float lam[kNPop];
#pragma unroll
        for (int q = 0; q < kNPop; ++q) {
          const int cx = kPlaneCx[q];
          const unsigned col = unsigned(cx == 0 ? xc : (cx == 1 ? xr : xl));
          lam[q] = __builtin_nontemporal_load(lam_next + q * PA + (ra[1 - kPlaneCy[q]] + col));
        }
        float f[9], g[10], lf[9], lg[10];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          f[i] = pre[i];
          lf[i] = lam[i];
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) {
          g[k] = pre[9 + k];
          lg[k] = lam[9 + k];
        }
        const CsGrad d = collide_adjoint<LESA>(f, g, lf, lg, rt, ac);
        if (LESA && up3 && b >= y0 && b < y0 + h) {
          dv += double(d.v);
          db += double(d.b);
        }
#pragma unroll
        for (int q = 0; q < kNPop; ++q) {
          const float val = q < 9 ? lf[q] : lg[q - 9];
          const int k = kT2Reg[q];
          if (kT2Group[q] >= 0)
            l2[t3_row(q)][lc + 1] = val;
          else if (kPlaneCy[q] == 0)
            n2c[k] = val;
          else if (kPlaneCy[q] == 1)
            n2u[k] = val;
          else
            n2d[k] = val;
        }
      }
    }
    __syncthreads();
    // C. reverse step t at row c = y0 - 4 + t (from pass 4 on), stored; the
    // l2 row of this pass is read in every pass, as above
    {
      float e[kT3Rows];
#pragma unroll
      for (int q = 0; q < kNPop; ++q)
        if (kT2Group[q] >= 0) e[t3_row(q)] = l2[t3_row(q)][c2 + kPlaneCx[q]];
      if (t >= 4 && up3) {
        const int c = y0 - 4 + t;
        float lam[kNPop];
#pragma unroll
        for (int q = 0; q < kNPop; ++q) {
          const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
          if (g >= 0)
            lam[q] = g == 0 ? e[t3_row(q)] : (g == 1 ? y2c[i] : y2d2[i]);
          else
            lam[q] = kPlaneCy[q] == 1 ? n2u[k] : (kPlaneCy[q] == 0 ? w2c[k] : w2d2[k]);
        }
        unsigned row[3];
        t2_rows(c, geo, row);
        float v[kNPop][1];
        gather_row<ST, 1>(st, P, xc, xl, xr, row, v);
        float f[9], g[10], lf[9], lg[10];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          f[i] = v[i][0];
          lf[i] = lam[i];
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) {
          g[k] = v[9 + k][0];
          lg[k] = lam[9 + k];
        }
        const CsGrad d = collide_adjoint<LESA>(f, g, lf, lg, rt, ac);
        if (LESA) {
          dv += double(d.v);
          db += double(d.b);
        }
        const unsigned oc = unsigned(c) * ga.pitch + unsigned(xc);
#pragma unroll
        for (int i = 0; i < 9; ++i) st_plane_nt(lam_prev + i * PA, oc, lf[i]);
#pragma unroll
        for (int q = 0; q < 10; ++q) st_plane_nt(lam_prev + (9 + q) * PA, oc, lg[q]);
      }
      // group 0 (c_y = +1) was used above from this pass; keep group 1 one
      // pass and group 2 two
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        y2d2[i] = y2d1[i];
        y2d1[i] = e[8 + i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) y2c[i] = e[2 + i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      z1u2[k] = z1u1[k];
      z1u1[k] = has ? n1u[k] : 0.0f;
      z1c[k] = has ? n1c[k] : 0.0f;
      w2d2[k] = w2d1[k];
      w2d1[k] = do2 ? n2d[k] : 0.0f;
      w2c[k] = do2 ? n2c[k] : 0.0f;
    }
  }
  if (LESA) {
    red[0][tid] = dv;
    red[1][tid] = db;
    __syncthreads();
    if (tid < kT3Threads - kT3Cols) {
      red[0][tid] += red[0][kT3Cols + tid];
      red[1][tid] += red[1][kT3Cols + tid];
    }
    __syncthreads();
    for (int w = kT3Cols / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      acc[blockIdx.x] += red[0][0];
      acc[nslots + blockIdx.x] += red[1][0];
    }
  }
}

}  // namespace

int adj_step_blocks(const Geom& g) {
  return ((g.nx + LBMHD_ADJ_TX - 1) / LBMHD_ADJ_TX) * g.ny;
}

hipError_t launch_adj_step(int storage, bool les, const void* state, const float* lam_next,
                           float* lam_prev, double* acc, const Geom& g, const Geom& ga,
                           const Rates& r, double delta2, hipStream_t s) {
  const int tiles_x = (g.nx + LBMHD_ADJ_TX - 1) / LBMHD_ADJ_TX;
  const dim3 grid(unsigned(adj_step_blocks(g))), block(LBMHD_ADJ_TX);
  // cf = 18 C_Sv Delta^2 and cm = 36 C_Sb Delta^2 are linear in their constants.
  const AdjConsts ac{float(18.0 * delta2), float(36.0 * delta2)};
  if (storage == LBMHD_FP32) {
    auto* st = static_cast<const float*>(state);
    if (les)
      hipLaunchKernelGGL((k_adj_step<LBMHD_FP32, true>), grid, block, 0, s, st, lam_next,
                         lam_prev, acc, g, ga, r, ac, tiles_x);
    else
      hipLaunchKernelGGL((k_adj_step<LBMHD_FP32, false>), grid, block, 0, s, st, lam_next,
                         lam_prev, acc, g, ga, r, ac, tiles_x);
  } else {
    auto* st = static_cast<const _Float16*>(state);
    if (les)
      hipLaunchKernelGGL((k_adj_step<LBMHD_FP16, true>), grid, block, 0, s, st, lam_next,
                         lam_prev, acc, g, ga, r, ac, tiles_x);
    else
      hipLaunchKernelGGL((k_adj_step<LBMHD_FP16, false>), grid, block, 0, s, st, lam_next,
                         lam_prev, acc, g, ga, r, ac, tiles_x);
  }
  return hipGetLastError();
}

// Strip height of the two-reverse-step kernel (halo overhead 4 / rows): as
// for the forward three-step kernel, about 512 blocks up to 128-row strips,
// 32-row strips beyond.
static int adj_step2_rows(const Geom& g) {
  const long long tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const long long rows = tiles_x * g.ny / 512;
  return int(rows < 8 ? 8 : (rows > 128 ? 32 : rows));
}

template <int ST, bool LESF, bool LESA>
void launch_adj_step2_t(const void* state, const float* lam_next, float* lam_prev, double* acc,
                        const Geom& g, const Geom& ga, const Rates& r, const AdjConsts& ac,
                        hipStream_t s) {
  const int rows = adj_step2_rows(g);
  const int tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const int strips = (g.ny + rows - 1) / rows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kT3Threads);
  hipLaunchKernelGGL((k_adj_step2<ST, LESF, LESA>), grid, block, 0, s,
                     static_cast<const typename Codec<ST>::T*>(state), lam_next, lam_prev, acc, g,
                     ga, r, ac, tiles_x, rows, adj_step_blocks(g));
}

hipError_t launch_adj_step2(int storage, bool les_fwd, bool les, const void* state,
                            const float* lam_next, float* lam_prev, double* acc, const Geom& g,
                            const Geom& ga, const Rates& r, double delta2, hipStream_t s) {
  if (les_fwd && !les) return hipErrorInvalidValue;
  const AdjConsts ac{float(18.0 * delta2), float(36.0 * delta2)};
  auto go = [&](auto fp32) {
    constexpr int ST = decltype(fp32)::value ? LBMHD_FP32 : LBMHD_FP16;
    if (les_fwd)
      launch_adj_step2_t<ST, true, true>(state, lam_next, lam_prev, acc, g, ga, r, ac, s);
    else if (les)
      launch_adj_step2_t<ST, false, true>(state, lam_next, lam_prev, acc, g, ga, r, ac, s);
    else
      launch_adj_step2_t<ST, false, false>(state, lam_next, lam_prev, acc, g, ga, r, ac, s);
  };
  if (storage == LBMHD_FP32)
    go(std::true_type{});
  else
    go(std::false_type{});
  return hipGetLastError();
}

bool adj_step2_pays(const Geom& g) {
  const long long tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  return tiles_x * ((g.ny + 7) / 8) >= 512;
}

// Strip height of the kinetic reverse step: about 512 blocks (two per CU; two
// halo rows of part A and four of gathers per strip), 8 to 256 rows.  At 4096^2
// (128-row strips) that took 1.31 ms per step, against 1.60 with 384 blocks,
// 1.65 with 768 or 1536 and 2.16 with 256.
static int adj_kin_rows(const Geom& g) {
  const long long tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const long long rows = (tiles_x * g.ny + 511) / 512;
  return int(rows < 8 ? 8 : (rows > 256 ? 256 : rows));
}

hipError_t launch_adj_step_kin(int storage, bool les, const void* state, const float* lam_next,
                               float* lam_prev, double* acc, const Geom& g, const Geom& ga,
                               const Rates& r, double delta2, hipStream_t s) {
  const int tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const int rows = adj_kin_rows(g);
  const int strips = (g.ny + rows - 1) / rows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kT3Threads);
  const AdjConsts ac{float(18.0 * delta2), float(36.0 * delta2)};
  const float c12 = float(delta2 / 12.0);
  const int nslots = adj_step_blocks(g);
  auto go = [&](auto fp32) {
    constexpr int ST = decltype(fp32)::value ? LBMHD_FP32 : LBMHD_FP16;
    auto* st = static_cast<const typename Dec<ST>::T*>(state);
    if (les)
      hipLaunchKernelGGL((k_adj_kin<ST, true>), grid, block, 0, s, st, lam_next, lam_prev, acc,
                         g, ga, r, ac, c12, tiles_x, rows, nslots);
    else
      hipLaunchKernelGGL((k_adj_kin<ST, false>), grid, block, 0, s, st, lam_next, lam_prev, acc,
                         g, ga, r, ac, c12, tiles_x, rows, nslots);
  };
  if (storage == LBMHD_FP32)
    go(std::true_type{});
  else
    go(std::false_type{});
  return hipGetLastError();
}

hipError_t launch_adj_seed(int storage, const void* lat, float* lam, const Geom& g,
                           const Geom& ga, hipStream_t s) {
  const unsigned nb = unsigned(((long long)g.nx * g.ny + 255) / 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_adj_seed<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float*>(lat), lam, g, ga);
  else
    hipLaunchKernelGGL(k_adj_seed<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), lam, g, ga);
  return hipGetLastError();
}

hipError_t launch_adj_seed_mismatch(int storage, const void* lat, const double* ux_t,
                                    const double* uy_t, const double* bx_t, const double* by_t,
                                    double scale, float* lam, const Geom& g, const Geom& ga,
                                    hipStream_t s) {
  const unsigned nb = unsigned(((long long)g.nx * g.ny + 255) / 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_adj_seed_mismatch<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float*>(lat), ux_t, uy_t, bx_t, by_t, scale, lam, g, ga);
  else
    hipLaunchKernelGGL(k_adj_seed_mismatch<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), ux_t, uy_t, bx_t, by_t, scale, lam, g,
                       ga);
  return hipGetLastError();
}

hipError_t launch_adj_fields(const float* lam0, const double* rho0, const double* ux0,
                             const double* uy0, const double* bx0, const double* by0,
                             double* gux, double* guy, double* gbx, double* gby, const Geom& ga,
                             int nx, int ny, hipStream_t s) {
  const unsigned nb = unsigned(((long long)nx * ny + 255) / 256);
  hipLaunchKernelGGL(k_adj_fields, dim3(nb), dim3(256), 0, s, lam0, rho0, ux0, uy0, bx0, by0,
                     gux, guy, gbx, gby, ga, nx, ny);
  return hipGetLastError();
}

}  // namespace lbk
