// lbmhd_kernels.hip -- gfx950 kernels of the lattice Boltzmann MHD update
// (Flint & Vahala, arXiv:1607.08675): fused pull-stream + moment-space
// collision, equilibrium initialisation, encode/decode, macroscopic fields
// and FP64 diagnostics.
//
// Data layout in HBM (one lattice): 19 planes [plane][y][pitch], x fastest.
// Planes 0..8 = f_0..f_8 (D2Q9), 9..13 = g_x,0..4, 14..18 = g_y,0..4 (D2Q5),
// velocities in the order of Sec. 3.  Every plane stores the deviation from
// the rest state (f_i - w_i, g unchanged): this keeps the low-order bits of
// rho u = sum c_i f_i that a plain f_i would spend on the large w_i.
//
// The step is HBM-bound: 19 loads + 19 stores per site against ~200 FP32
// operations, so the kernel is laid out for bandwidth, not for matrix cores.
// A thread owns V consecutive sites of one row (V = 1 for FP32 storage, V = 2
// for FP16 so that every lane moves 4-byte words); a 256-thread block owns
// 256 V consecutive sites.  All 19 gathers are issued before any arithmetic;
// a plane that streams along x is read with the aligned vector of the
// thread's own sites plus one edge element, the +-1 shifts being served by
// the caches; stores are aligned and non-temporal.  Blocks run in plain row
// order (a remap giving each XCD a contiguous band of tiles measured slower).
#include <math.h>

#include "lbmhd_impl.h"
#include "lbmhd_step_dev.h"

namespace lbk {
namespace {

// dst(x) = C(pre(x)),  pre_i(x) = src_i(x - c_i) (periodic pull; Sec. 1.2
// streaming written as a gather).  Thread t of block b updates sites
// x0 .. x0 + V - 1 of row y, x0 = (b mod tiles_x) * 256 V + t V, y = b / tiles_x.
// V > 1 requires nx % V == 0.
template <int ST, int V, bool LES>
__global__ __launch_bounds__(kStepThreads) void k_step(
    const typename Codec<ST>::T* __restrict__ src, typename Codec<ST>::T* __restrict__ dst,
    Geom geo, Rates rt, int tiles_x) {
  const int x0 = ((int(blockIdx.x) % tiles_x) * kStepThreads + int(threadIdx.x)) * V;
  const int y = int(blockIdx.x) / tiles_x;
  if (x0 >= geo.nx) return;
  const int xl = x0 == 0 ? geo.nx - 1 : x0 - 1;       // source of c_x = +1 planes
  const int xr = x0 + V == geo.nx ? 0 : x0 + V;       // source of c_x = -1 planes
  const int ym = y == 0 ? geo.ny - 1 : y - 1;
  const int yp = y == geo.ny - 1 ? 0 : y + 1;
  // source row of a plane with velocity c_y: y - c_y, indexed by c_y + 1
  const unsigned row[3] = {unsigned(yp) * geo.pitch, unsigned(y) * geo.pitch,
                           unsigned(ym) * geo.pitch};
  float v[kNPop][V];
  gather_row<ST, V>(src, geo.plane, x0, xl, xr, row, v);
  collide_sites<V, LES, ST == kFP16S>(v, rt);
  store_row<ST, V>(dst, geo.plane, row[1] + unsigned(x0), v);
}

// ------------------------------------------- two steps in one pass over HBM
// dst = C(S(C(S(src)))) for the closures that read no neighbours (plain and
// Smagorinsky-MHD): temporal blocking.  A block of kT2Threads threads owns a
// tile of W = kT2Threads V columns and a strip of `rows` rows of the output
// and walks the strip upward.  Pass t first updates row r = y0 - 1 + t from
// src (gathered as in k_step) on the tile's columns and on one halo column on
// each side, then updates row r - 1 a second time from those results: its
// pre-collision value of plane q is the first update's post-collision value
// at x - c_q.  The intermediate state never reaches HBM.  Planes that move
// along x are handed to the neighbouring columns through LDS, grouped by c_y:
// a plane with c_y = +1 is read two passes after it is written, c_y = 0 one
// pass after, c_y = -1 in the same pass, hence rings of 4, 3 and 2 row slots,
// which lets one barrier per pass order every write before its reads and
// every read before the slot is written again.  Planes with c_x = 0 stay in
// the thread's registers for the same number of passes.  The intermediate
// values pass through the storage codec, so that the result equals two
// k_step launches bit for bit (the collision spells out its fused
// multiply-adds, so the halo sites' single-site copy of it rounds as the
// paired one does).  HBM bytes per site for two steps: one
// read and one write of the lattice, plus halo re-reads of 2 / rows of the
// rows and 4 / W of the columns.
constexpr int kT2Threads = 256;
// LDS rings: 2 planes x 4 slots + 6 x 3 + 2 x 2 plane-rows
constexpr int kT2SlotsA = 4, kT2SlotsB = 3, kT2SlotsC = 2;
constexpr int kT2Slots = 2 * kT2SlotsA + 6 * kT2SlotsB + 2 * kT2SlotsC;
constexpr int kT2BaseB = 2 * kT2SlotsA, kT2BaseC = kT2BaseB + 6 * kT2SlotsB;
// MID: also store the intermediate state (after the first update) to mid;
// each block writes the rows and columns it owns, so every site once.
template <int ST, int V, bool LES, bool MID>
__global__ __launch_bounds__(kT2Threads) void k_step2(
    const typename Codec<ST>::T* __restrict__ src, typename Codec<ST>::T* __restrict__ dst,
    typename Codec<ST>::T* __restrict__ mid, Geom geo, Rates rt, int tiles_x, int rows,
    bool xcd_map) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int W = kT2Threads * V;
  __shared__ T lds[kT2Slots][W + 2];   // LDS column s holds local column s - 1
  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane;
  // blocks go round-robin to the eight XCDs: with xcd_map (strips % 8 == 0)
  // each XCD gets whole strips, so that the halo lines that neighbouring
  // tiles share meet in one L2
  int tile, strip;
  if (xcd_map) {
    const int k = int(blockIdx.x) >> 3;
    strip = (int(blockIdx.x) & 7) + 8 * (k / tiles_x);
    tile = k % tiles_x;
  } else {
    tile = int(blockIdx.x) % tiles_x;
    strip = int(blockIdx.x) / tiles_x;
  }
  const int x0 = tile * W;
  const int y0 = strip * rows;
  const int wt = min(W, nx - x0);          // columns of this tile
  const int h = min(rows, ny - y0);        // output rows of this strip
  const int lc = int(threadIdx.x) * V;     // first local column of the thread
  const bool active = lc < wt;
  const int x = x0 + lc;
  const int xl = x == 0 ? nx - 1 : x - 1;
  const int xr = x + V >= nx ? x + V - nx : x + V;
  // threads 0 and 1 also update the halo columns x0 - 1 and x0 + wt (wrapped)
  const bool halo = threadIdx.x < 2;
  const int hx = threadIdx.x == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + wt == nx ? 0 : x0 + wt);
  const int hs = threadIdx.x == 0 ? 0 : wt + 1;
  const int hxl = hx == 0 ? nx - 1 : hx - 1;
  const int hxr = hx == nx - 1 ? 0 : hx + 1;

  // c_x = 0 planes of earlier passes: c_y = 0 from the last pass (zc), c_y = +1
  // from the last two (zu1, zu2)
  float zc[3][V], zu1[3][V], zu2[3][V];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < V; ++j) zc[k][j] = zu1[k][j] = zu2[k][j] = 0.0f;
  int sA = 0, sB = 0;   // t mod kT2SlotsA, t mod kT2SlotsB
  for (int t = 0; t < h + 2; ++t) {
    const int sC = t & 1;
    // first update of row y0 - 1 + t; c_x = 0 planes kept by c_y (nc: 0, nu: +1, nd: -1)
    float nc[3][V], nu[3][V], nd[3][V];
    unsigned row[3];
    t2_rows(y0 - 1 + t, geo, row);
    if (active) {
      float v[kNPop][V];
      gather_row<ST, V>(src, P, x, xl, xr, row, v);
      collide_sites<V, LES, ST == kFP16S>(v, rt);
      if (MID && t >= 1 && t <= h) store_row<ST, V>(mid, P, row[1] + unsigned(x), v);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const T e = C::enc(v[q][j]);
          const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
          if (g == 0)
            lds[sA * 2 + i][lc + j + 1] = e;
          else if (g == 1)
            lds[kT2BaseB + sB * 6 + i][lc + j + 1] = e;
          else if (g == 2)
            lds[kT2BaseC + sC * 2 + i][lc + j + 1] = e;
          else if (kPlaneCy[q] == 0)
            nc[k][j] = C::dec(e);
          else if (kPlaneCy[q] == 1)
            nu[k][j] = C::dec(e);
          else
            nd[k][j] = C::dec(e);
        }
      }
    }
    if (halo) {
      float v[kNPop][1];
      gather_row<ST, 1>(src, P, hx, hxl, hxr, row, v);
      collide_sites<1, LES, ST == kFP16S>(v, rt);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const T e = C::enc(v[q][0]);
        const int g = kT2Group[q], i = kT2Index[q];
        if (g == 0)
          lds[sA * 2 + i][hs] = e;
        else if (g == 1)
          lds[kT2BaseB + sB * 6 + i][hs] = e;
        else if (g == 2)
          lds[kT2BaseC + sC * 2 + i][hs] = e;
      }
    }
    __syncthreads();
    // second update of row y0 - 2 + t (from pass 2 on)
    if (t >= 2 && active) {
      const int sB1 = sB == 0 ? kT2SlotsB - 1 : sB - 1;            // (t - 1) mod slots
      const int sA2 = sA >= 2 ? sA - 2 : sA + kT2SlotsA - 2;       // (t - 2) mod slots
      float v[kNPop][V];
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
          const int sx = lc + j - kPlaneCx[q] + 1;
          if (g == 0)
            v[q][j] = C::dec(lds[sA2 * 2 + i][sx]);
          else if (g == 1)
            v[q][j] = C::dec(lds[kT2BaseB + sB1 * 6 + i][sx]);
          else if (g == 2)
            v[q][j] = C::dec(lds[kT2BaseC + sC * 2 + i][sx]);
          else if (kPlaneCy[q] == 0)
            v[q][j] = zc[k][j];
          else if (kPlaneCy[q] == 1)
            v[q][j] = zu2[k][j];
          else
            v[q][j] = nd[k][j];
        }
      }
      collide_sites<V, LES, ST == kFP16S>(v, rt);
      store_row<ST, V>(dst, P, unsigned(y0 + t - 2) * geo.pitch + unsigned(x), v);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        zu2[k][j] = zu1[k][j];
        zu1[k][j] = active ? nu[k][j] : 0.0f;
        zc[k][j] = active ? nc[k][j] : 0.0f;
      }
    sA = sA == kT2SlotsA - 1 ? 0 : sA + 1;
    sB = sB == kT2SlotsB - 1 ? 0 : sB + 1;
  }
}

// ----------------------------------------- three steps in one pass (FP32)
// The two-step scheme one level deeper: dst = (C S)^3 src for FP32 storage
// and the closures without neighbour terms.  A block owns a tile of kT3Cols
// columns and a strip of `rows` output rows; pass t takes row y0 - 2 + t
// through the first update (from HBM), row y0 - 3 + t through the second
// (from level 1) and row y0 - 4 + t through the third (from level 2, to
// HBM).  The first update also covers two halo columns on each side and the
// second one on each side; a fifth wave owns those four halo columns, so
// that every thread keeps the values of its own column in registers and no
// wave collides more than three times per pass.  Planes with c_x != 0 cross
// to the neighbouring column through one LDS row per plane and level: the
// consumer reads it right after the barrier that publishes it (two barriers
// per pass, after the first and after the second update), and carries the
// c_y = 0 values one pass and the c_y = +1 values two passes in registers,
// as it does for its own c_x = 0 planes.  So each LDS row is rewritten on
// the next pass and a level is 10 plane-rows.  HBM bytes per site for three
// steps: one read and one write of the lattice, plus halo re-reads of
// 4 / rows of the rows and 8 / kT3Cols of the columns.
// MID: also store the states after the first and the second update to mid1
// and mid2 (each block the rows and columns it owns, so every site once).
template <bool LES, bool MID>
__global__ __launch_bounds__(kT3Threads) void k_step_t3(const float* __restrict__ src,
                                                        float* __restrict__ dst,
                                                        float* __restrict__ mid1,
                                                        float* __restrict__ mid2, Geom geo,
                                                        Rates rt, int tiles_x, int rows,
                                                        bool xcd_map) {
  __shared__ float l1[kT3Rows][kT3Cols + 4];   // first update: column lc + 2
  __shared__ float l2[kT3Rows][kT3Cols + 2];   // second update: column lc + 1
  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane;
  int tile, strip;
  if (xcd_map) {   // whole strips per XCD, as in k_step2
    const int k = int(blockIdx.x) >> 3;
    strip = (int(blockIdx.x) & 7) + 8 * (k / tiles_x);
    tile = k % tiles_x;
  } else {
    tile = int(blockIdx.x) % tiles_x;
    strip = int(blockIdx.x) / tiles_x;
  }
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
  const bool up2 = has && lc >= -1 && lc <= wt;   // takes the second update
  const bool up3 = has && lc >= 0 && lc < wt;     // takes the third update
  // LDS columns read for the second and third updates: lc - c_x + c1 and
  // lc - c_x + c2.  Threads that take no such update read columns 1 .. 3 or
  // 0 .. 2 instead (in bounds, never used), so the reads need no branch.
  const int c1 = up2 ? lc + 2 : 2;
  const int c2 = up3 ? lc + 1 : 1;
  int xc = (x0 + lc) % nx;
  if (xc < 0) xc += nx;
  const int xl = xc == 0 ? nx - 1 : xc - 1;
  const int xr = xc == nx - 1 ? 0 : xc + 1;

  // Inputs of earlier passes, per level, for this thread's column: c_y = 0
  // planes from the last pass, c_y = +1 planes from the last two; z: the
  // c_x = 0 planes (3 per c_y), x: the c_x != 0 ones (6 with c_y = 0, 2 with
  // c_y = +1), already taken from column lc - c_x.
  float z1c[3], z1u1[3], z1u2[3], z2c[3], z2u1[3], z2u2[3];
  float x1c[6], x1u1[2], x1u2[2], x2c[6], x2u1[2], x2u2[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) z1c[k] = z1u1[k] = z1u2[k] = z2c[k] = z2u1[k] = z2u2[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) x1c[k] = x2c[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 2; ++k) x1u1[k] = x1u2[k] = x2u1[k] = x2u2[k] = 0.0f;
  for (int t = 0; t < h + 4; ++t) {
    // first update of row y0 - 2 + t
    float n1c[3], n1u[3], n1d[3];
    if (has) {
      unsigned row[3];
      t2_rows(y0 - 2 + t, geo, row);
      float v[kNPop][1];
      gather_row<LBMHD_FP32, 1>(src, P, xc, xl, xr, row, v);
      collide_sites<1, LES>(v, rt);
      if (MID && up3 && t >= 2 && t <= h + 1)
        store_row<LBMHD_FP32, 1>(mid1, P, row[1] + unsigned(xc), v);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const int k = kT2Reg[q];
        if (kT2Group[q] >= 0)
          l1[t3_row(q)][lc + 2] = v[q][0];
        else if (kPlaneCy[q] == 0)
          n1c[k] = v[q][0];
        else if (kPlaneCy[q] == 1)
          n1u[k] = v[q][0];
        else
          n1d[k] = v[q][0];
      }
    }
    __syncthreads();
    // second update of row y0 - 3 + t (from pass 2 on); the level-1 row of
    // this pass is read in every pass, before the next one overwrites it
    float n2c[3], n2u[3], n2d[3];
    const bool do2 = t >= 2 && up2;
    {
      float e[kT3Rows];
#pragma unroll
      for (int q = 0; q < kNPop; ++q)
        if (kT2Group[q] >= 0) e[t3_row(q)] = l1[t3_row(q)][c1 - kPlaneCx[q]];
      float v[kNPop][1];
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
        if (g >= 0)
          v[q][0] = g == 0 ? x1u2[i] : (g == 1 ? x1c[i] : e[t3_row(q)]);
        else
          v[q][0] = kPlaneCy[q] == 0 ? z1c[k] : (kPlaneCy[q] == 1 ? z1u2[k] : n1d[k]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        x1u2[i] = x1u1[i];
        x1u1[i] = e[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) x1c[i] = e[2 + i];
      if (do2) {
        collide_sites<1, LES>(v, rt);
        if (MID && up3 && t >= 3 && t <= h + 2)
          store_row<LBMHD_FP32, 1>(mid2, P, unsigned(y0 - 3 + t) * geo.pitch + unsigned(xc), v);
#pragma unroll
        for (int q = 0; q < kNPop; ++q) {
          const int k = kT2Reg[q];
          if (kT2Group[q] >= 0)
            l2[t3_row(q)][lc + 1] = v[q][0];
          else if (kPlaneCy[q] == 0)
            n2c[k] = v[q][0];
          else if (kPlaneCy[q] == 1)
            n2u[k] = v[q][0];
          else
            n2d[k] = v[q][0];
        }
      }
    }
    __syncthreads();
    // third update of row y0 - 4 + t (from pass 4 on), stored; the level-2
    // row of this pass is read in every pass, as above
    {
      float e[kT3Rows];
#pragma unroll
      for (int q = 0; q < kNPop; ++q)
        if (kT2Group[q] >= 0) e[t3_row(q)] = l2[t3_row(q)][c2 - kPlaneCx[q]];
      if (t >= 4 && up3) {
        float v[kNPop][1];
#pragma unroll
        for (int q = 0; q < kNPop; ++q) {
          const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
          if (g >= 0)
            v[q][0] = g == 0 ? x2u2[i] : (g == 1 ? x2c[i] : e[t3_row(q)]);
          else
            v[q][0] = kPlaneCy[q] == 0 ? z2c[k] : (kPlaneCy[q] == 1 ? z2u2[k] : n2d[k]);
        }
        collide_sites<1, LES>(v, rt);
        store_row<LBMHD_FP32, 1>(dst, P, unsigned(y0 - 4 + t) * geo.pitch + unsigned(xc), v);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        x2u2[i] = x2u1[i];
        x2u1[i] = e[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) x2c[i] = e[2 + i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      z1u2[k] = z1u1[k];
      z1u1[k] = has ? n1u[k] : 0.0f;
      z1c[k] = has ? n1c[k] : 0.0f;
      z2u2[k] = z2u1[k];
      z2u1[k] = do2 ? n2u[k] : 0.0f;
      z2c[k] = do2 ? n2c[k] : 0.0f;
    }
  }
}

// --------------------------------------------- steps with lattice gradients
// Same update as k_step for the closures that need the neighbours: the
// kinetic closure (KIN) relaxes toward the filtered equilibria, whose Delta^2
// parts need gradients of rho, j, B; the cross-helicity closure (EDDY = 2)
// needs the vorticity.  The gradients are those of the pre-collision
// (gathered) neighbours, by the isotropic D2Q9 difference
// d_a X = 3 sum_i w_i c_ia X(x + c_i).  A block of kKinThreads threads owns
// as many columns and a strip of kKinRows rows.  It walks the strip row by
// row: it gathers row y+1 (each population is read once), writes that row's
// rho - 1, j (and B for KIN) into a rolling 3-row LDS buffer with one halo
// column on each side, and then collides row y, whose populations it
// gathered on the previous pass.
#ifndef LBMHD_KIN_ROWS
#define LBMHD_KIN_ROWS 16
#endif
#ifndef LBMHD_KIN_THREADS
#define LBMHD_KIN_THREADS 512
#endif
constexpr int kKinRows = LBMHD_KIN_ROWS;
constexpr int kKinThreads = LBMHD_KIN_THREADS;
constexpr int kKinCols = kKinThreads + 2;

// Encoded populations of the pre-collision state at (x, y): pre_q(x) =
// src_q(x - c_q), periodic.  The loads are only issued here; decoding happens
// where the values are used, so they can stay in flight meanwhile.
template <int ST>
__device__ __forceinline__ void load_site(const typename Codec<ST>::T* __restrict__ src,
                                          const Geom& geo, int x, int y,
                                          typename Codec<ST>::T (&p)[kNPop]) {
  const int xm = x == 0 ? geo.nx - 1 : x - 1;
  const int xp = x == geo.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? geo.ny - 1 : y - 1;
  const int yp = y == geo.ny - 1 ? 0 : y + 1;
  const unsigned row[3] = {unsigned(yp) * geo.pitch, unsigned(y) * geo.pitch,
                           unsigned(ym) * geo.pitch};
  const long long P = geo.plane;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    const int xs = kPlaneCx[q] == 0 ? x : (kPlaneCx[q] == 1 ? xm : xp);
    p[q] = ld_plane<typename Codec<ST>::T>(src + q * P, row[kPlaneCy[q] + 1] + unsigned(xs));
  }
}

// rho - 1, j_x, j_y, B_x, B_y of gathered populations (deviation variables).
__device__ __forceinline__ void site_moments(const float (&p)[kNPop], float (&m)[5]) {
  m[0] = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7])) + p[8];
  m[1] = (p[1] - p[3]) + (p[5] - p[7]) - (p[6] - p[8]);
  m[2] = (p[2] - p[4]) + (p[5] - p[7]) + (p[6] - p[8]);
  m[3] = (p[9] + p[10]) + (p[11] + p[12]) + p[13];
  m[4] = (p[14] + p[15]) + (p[16] + p[17]) + p[18];
}

// Terms of the closures with lattice gradients at one site, from the
// pre-collision rho - 1, j (and B for KIN) of the site and its eight
// neighbours: rows rm (y - 1), r0 (y) and rp (y + 1) of a moment buffer whose
// fields lie `fs` floats apart, the site at column c.  Isotropic D2Q9
// gradient: d_x = (E - W)/3 + (NE - NW + SE - SW)/12, d_y likewise.
// h_X = grad X - X grad(rho) / rho (= rho grad(X / rho)); ratio terms
// (X Y / rho) of the kinetic closure use it, product terms (B B) the plain
// gradients:
//   R(X, Y) = Delta^2 / (12 rho) h_X . h_Y,  S(X, Y) = Delta^2 / 12 grad X . grad Y;
// the vorticity is d_x u_y - d_y u_x = (h_jy,x - h_jx,y) / rho.  Every
// multiply-add is written out (no other contraction), so each kernel that
// evaluates the terms rounds them identically.
template <int EDDY, bool KIN>
__device__ __forceinline__ NbTerms nb_terms(const float* __restrict__ rm,
                                            const float* __restrict__ r0,
                                            const float* __restrict__ rp, int fs, int c,
                                            float c12) {
#pragma clang fp contract(off)
  constexpr int NF = KIN ? 5 : 3;
  float gx[NF], gy[NF], v[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int o = k * fs + c;
    const float e = r0[o + 1], w = r0[o - 1];
    const float nn = rp[o], ss = rm[o];
    const float ne = rp[o + 1], nw = rp[o - 1];
    const float se = rm[o + 1], sw = rm[o - 1];
    gx[k] = fmaf(1.0f / 3.0f, e - w, (1.0f / 12.0f) * ((ne - nw) + (se - sw)));
    gy[k] = fmaf(1.0f / 3.0f, nn - ss, (1.0f / 12.0f) * ((ne + nw) - (se + sw)));
    v[k] = r0[o];
  }
  const float ir = frcp(1.0f + v[0]);
  const float grx = gx[0] * ir, gry = gy[0] * ir;
  float hx[NF - 1], hy[NF - 1];
#pragma unroll
  for (int k = 0; k < NF - 1; ++k) {
    hx[k] = fmaf(-v[k + 1], grx, gx[k + 1]);
    hy[k] = fmaf(-v[k + 1], gry, gy[k + 1]);
  }
  NbTerms kc{0.f, 0.f, 0.f, 0.f, 0.f};
  if constexpr (KIN) {
    const float cr = c12 * ir;
    const float jxjx = cr * fmaf(hx[0], hx[0], hy[0] * hy[0]);
    const float jyjy = cr * fmaf(hx[1], hx[1], hy[1] * hy[1]);
    kc.m3 = fmaf(cr, fmaf(hx[0], hx[1], hy[0] * hy[1]), -(c12 * fmaf(gx[3], gx[4], gy[3] * gy[4])));
    kc.m4 = fmaf(-c12, fmaf(gx[3], gx[3], gy[3] * gy[3]) - fmaf(gx[4], gx[4], gy[4] * gy[4]),
                 jxjx - jyjy);
    kc.m78 = -3.0f * (jxjx + jyjy);
    kc.e = cr * (fmaf(hx[0], hx[3], hy[0] * hy[3]) - fmaf(hx[1], hx[2], hy[1] * hy[2]));
  }
  if constexpr (EDDY == 2) kc.w = (hx[1] - hy[0]) * ir;
  return kc;
}

template <int ST, int EDDY, bool KIN>
__global__ __launch_bounds__(kKinThreads) void k_step_nb(
    const typename Codec<ST>::T* __restrict__ src, typename Codec<ST>::T* __restrict__ dst,
    Geom geo, Rates rt, float c12, int tiles_x) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int NF = KIN ? 5 : 3;   // staged fields: rho - 1, j (, B)
  __shared__ float mac[3][NF][kKinCols];
  const int tx = int(threadIdx.x);
  const int xt = (int(blockIdx.x) % tiles_x) * kKinThreads;
  const int y0 = (int(blockIdx.x) / tiles_x) * kKinRows;
  const int y1 = min(y0 + kKinRows, geo.ny);
  const int x = xt + tx;
  const bool active = x < geo.nx;
  const int xc = x % geo.nx;                                   // column staged by this thread
  const int xh = tx == 0 ? (xt == 0 ? geo.nx - 1 : xt - 1)     // halo column (threads 0, 1)
                         : (xt + kKinThreads) % geo.nx;
  const int ch = tx == 0 ? 0 : kKinCols - 1;
  // Rows are loaded one pass ahead of their use: the loads of row y + 2 (and,
  // in threads 0 and 1, of a halo column) are issued before row y collides,
  // and row y + 1, loaded on the previous pass, is decoded and its moments
  // written to LDS slot `slot` (rows wrap periodically).
  T raw[kNPop], rawh[kNPop];
  auto issue = [&](int yy) {
    yy = yy < 0 ? yy + geo.ny : (yy >= geo.ny ? yy - geo.ny : yy);
    load_site<ST>(src, geo, xc, yy, raw);
    if (tx < 2) load_site<ST>(src, geo, xh, yy, rawh);
  };
  auto commit = [&](int slot, float (&p)[kNPop]) {
#pragma unroll
    for (int q = 0; q < kNPop; ++q) p[q] = C::dec(raw[q]);
    float m[5];
    site_moments(p, m);
#pragma unroll
    for (int k = 0; k < NF; ++k) mac[slot][k][tx + 1] = m[k];
    if (tx < 2) {
      float ph[kNPop], mh[5];
#pragma unroll
      for (int q = 0; q < kNPop; ++q) ph[q] = C::dec(rawh[q]);
      site_moments(ph, mh);
#pragma unroll
      for (int k = 0; k < NF; ++k) mac[slot][k][ch] = mh[k];
    }
  };
  float cur[kNPop], nxt[kNPop];
  issue(y0 - 1);                                  // row y0 - 1: moments only
  commit(0, nxt);
  issue(y0);
  commit(1, cur);
  issue(y0 + 1);
  const long long P = geo.plane;
  for (int y = y0; y < y1; ++y) {
    const int sm = (y - y0) % 3, s0 = (y - y0 + 1) % 3, sp = (y - y0 + 2) % 3;
    commit(sp, nxt);
    if (y + 2 <= y1) issue(y + 2);
    __syncthreads();
    if (active) {
      const NbTerms kc =
          nb_terms<EDDY, KIN>(&mac[sm][0][0], &mac[s0][0][0], &mac[sp][0][0], kKinCols, tx + 1, c12);
      float f[9], g[10];
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = cur[i];
#pragma unroll
      for (int k = 0; k < 10; ++k) g[k] = cur[9 + k];
      collide<EDDY, KIN>(f, g, rt, kc);
      const unsigned od = unsigned(y) * geo.pitch + unsigned(x);
#pragma unroll
      for (int i = 0; i < 9; ++i) st_plane_nt<T>(dst + i * P, od, C::enc(f[i]));
#pragma unroll
      for (int k = 0; k < 10; ++k) st_plane_nt<T>(dst + (9 + k) * P, od, C::enc(g[k]));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kNPop; ++q) cur[q] = nxt[q];
  }
}

// ------------------------ two steps per pass with lattice gradients
// dst = (C S)^2 src for the closures that need the neighbours' moments
// (kinetic, cross-helicity).  The second update at a site needs the first
// update's output two sites out (its own gather reaches one site, the
// gradients of the gathered moments one more), and the first update needs the
// input three sites out for its moments and four for their gathers.  A block
// owns a tile of kNb2Cols columns and a strip of `rows` output rows and walks
// upward; pass t, with a = y0 - 3 + t:
//   1. gathers row a from HBM (columns x0 - 3 .. x0 + wt + 2) and writes its
//      moments to ring m1 (3 rows);
//   2. first update of row a - 1 (columns x0 - 2 .. x0 + wt + 1), with the
//      gradients of rows a - 2 .. a of m1; the planes moving along x go to the
//      neighbouring columns through one LDS row per plane (y1), the others
//      stay in the thread's registers;
//   3. second gather of row a - 2 (columns x0 - 1 .. x0 + wt): each thread
//      reads the y1 values it needs right after the barrier that publishes
//      them and carries them on in registers (c_y = 0 planes one pass, c_y = +1
//      two), as the three-step kernel does; their moments go to ring m2;
//   4. second update of row a - 3 (the tile's own columns), with the
//      gradients of rows a - 4 .. a - 2 of m2, stored.
// Three barriers per pass, between the stages.  A fifth wave owns the six
// halo columns.  The first update's output passes through the storage codec,
// so the result equals two k_step_nb launches bit for bit.  MID: also store
// the intermediate state (each block the rows and columns it owns).  HBM
// bytes per site for two steps: one read and one write of the lattice, plus
// halo re-reads of 6 / rows of the rows and 6 / kNb2Cols of the columns.
constexpr int kNb2Cols = 256;
constexpr int kNb2Threads = kNb2Cols + 64;

// Compiled for at least four waves per SIMD (at most 128 VGPRs): with the
// compiler's own choice the pass measured 1.2x slower for the kinetic and the
// cross-helicity closure and 1.5x slower for both together (135 VGPRs), at
// 4096^2, with bit-identical results.
template <int ST, int EDDY, bool KIN, bool MID>
__global__ __launch_bounds__(kNb2Threads) __attribute__((amdgpu_waves_per_eu(4))) void k_step_nb2(
    const typename Codec<ST>::T* __restrict__ src, typename Codec<ST>::T* __restrict__ dst,
    typename Codec<ST>::T* __restrict__ mid, Geom geo, Rates rt, float c12, int tiles_x,
    int rows, bool xcd_map) {
  using C = Codec<ST>;
  using T = typename C::T;
  constexpr int NF = KIN ? 5 : 3;        // staged fields: rho - 1, j (, B)
  constexpr int W = kNb2Cols;
  __shared__ float m1[3][NF][W + 6];     // LDS column lc + 3
  __shared__ T y1[kT3Rows][W + 4];       // LDS column lc + 2
  __shared__ float m2[3][NF][W + 2];     // LDS column lc + 1
  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane;
  int tile, strip;
  if (xcd_map) {   // whole strips per XCD, as in k_step2
    const int k = int(blockIdx.x) >> 3;
    strip = (int(blockIdx.x) & 7) + 8 * (k / tiles_x);
    tile = k % tiles_x;
  } else {
    tile = int(blockIdx.x) % tiles_x;
    strip = int(blockIdx.x) / tiles_x;
  }
  const int x0 = tile * W, y0 = strip * rows;
  const int wt = min(W, nx - x0), h = min(rows, ny - y0);
  // the thread's column: its own (threads 0 .. W - 1) or a halo column
  // (lanes 0 .. 5 of the fifth wave: x0 - 3 .. x0 - 1, x0 + wt .. x0 + wt + 2)
  const int tid = int(threadIdx.x);
  int lc = tid;
  bool has = tid < wt;
  if (tid >= W) {
    const int k = tid - W;
    has = k < 6;
    lc = k < 3 ? k - 3 : wt + (k - 3);
  }
  const bool up2 = has && lc >= -2 && lc <= wt + 1;   // takes the first update
  const bool up3 = has && lc >= -1 && lc <= wt;       // takes the second gather
  const bool up4 = has && lc >= 0 && lc < wt;         // takes the second update
  // y1 column read for the second gather: lc + 2 - c_x (a fixed in-bounds
  // column for the threads that take no second gather)
  const int c3 = up3 ? lc + 2 : 2;
  int xc = (x0 + lc) % nx;
  if (xc < 0) xc += nx;
  const int xl = xc == 0 ? nx - 1 : xc - 1;
  const int xr = xc == nx - 1 ? 0 : xc + 1;

  float p1c[kNPop], p2c[kNPop];        // gathers of the previous pass (rows a - 1, a - 3)
  float z1c[3], z1u1[3], z1u2[3];      // y1, planes with c_x = 0, by c_y and pass
  float x1c[6], x1u1[2], x1u2[2];      // y1, planes with c_x != 0, taken from lc - c_x
#pragma unroll
  for (int q = 0; q < kNPop; ++q) p1c[q] = p2c[q] = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) z1c[k] = z1u1[k] = z1u2[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) x1c[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 2; ++k) x1u1[k] = x1u2[k] = 0.0f;
  // Kinetic closure with FP32 states: the next pass's first gather is issued
  // right after this pass's first barrier and flies during stages 2 to 4
  // (66.5k against 62.4k MLUPS at 4096^2, 62.8k against 57.9k with les = 3,
  // same results); the cross-helicity closure's registers spill with it
  // (29.7k against 54.6k).
  constexpr bool kPf = ST == LBMHD_FP32 && EDDY != 2;
  float pf[kNPop][1];
  // rows y0 - 3 .. y0 + h + 2: more than one period on a lattice two rows high
  auto gather_at = [&](int r, float (&v)[kNPop][1]) {
    int a = r % ny;
    if (a < 0) a += ny;
    unsigned row[3];
    t2_rows(a, geo, row);
    gather_row<ST, 1>(src, P, xc, xl, xr, row, v);
  };
  if (kPf && has) gather_at(y0 - 3, pf);
  for (int t = 0; t < h + 6; ++t) {
    const int s0 = t % 3;                         // ring slot of this pass
    const int s1 = s0 == 0 ? 2 : s0 - 1;          // (t - 1) mod 3
    const int s2 = s1 == 0 ? 2 : s1 - 1;          // (t - 2) mod 3
    // 1. gather row a = y0 - 3 + t and stage its moments
    float p1n[kNPop];
    if (has) {
      float v[kNPop][1];
      if (kPf) {
#pragma unroll
        for (int q = 0; q < kNPop; ++q) v[q][0] = pf[q][0];
      } else {
        gather_at(y0 - 3 + t, v);
      }
#pragma unroll
      for (int q = 0; q < kNPop; ++q) p1n[q] = v[q][0];
      float m[5];
      site_moments(p1n, m);
#pragma unroll
      for (int k = 0; k < NF; ++k) m1[s0][k][lc + 3] = m[k];
    }
    __syncthreads();
    if (kPf && has && t + 1 < h + 6) gather_at(y0 - 2 + t, pf);
    // 2. first update of row a - 1 (from pass 2 on)
    float n2c[3], n2u[3], n2d[3];
    const bool do2 = up2 && t >= 2;
    if (do2) {
      const NbTerms kc =
          nb_terms<EDDY, KIN>(&m1[s2][0][0], &m1[s1][0][0], &m1[s0][0][0], W + 6, lc + 3, c12);
      float f[9], g[10];
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = p1c[i];
#pragma unroll
      for (int k = 0; k < 10; ++k) g[k] = p1c[9 + k];
      collide<EDDY, KIN>(f, g, rt, kc);
      float v[kNPop];
#pragma unroll
      for (int i = 0; i < 9; ++i) v[i] = f[i];
#pragma unroll
      for (int k = 0; k < 10; ++k) v[9 + k] = g[k];
      const int r1 = y0 - 4 + t;                  // row a - 1
      if (MID && lc >= 0 && lc < wt && r1 >= y0 && r1 < y0 + h) {
        const unsigned od = unsigned(r1) * geo.pitch + unsigned(xc);
#pragma unroll
        for (int q = 0; q < kNPop; ++q) st_plane_nt<T>(mid + q * P, od, C::enc(v[q]));
      }
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const T e = C::enc(v[q]);
        const int k = kT2Reg[q];
        if (kT2Group[q] >= 0)
          y1[t3_row(q)][lc + 2] = e;
        else if (kPlaneCy[q] == 0)
          n2c[k] = C::dec(e);
        else if (kPlaneCy[q] == 1)
          n2u[k] = C::dec(e);
        else
          n2d[k] = C::dec(e);
      }
    }
    __syncthreads();
    // 3. second gather of row a - 2 (from pass 4 on); the y1 row of this pass
    // is read in every pass, before the next one overwrites it
    float p2n[kNPop];
    const bool do3 = up3 && t >= 4;
    {
      float e[kT3Rows];
#pragma unroll
      for (int q = 0; q < kNPop; ++q)
        if (kT2Group[q] >= 0) e[t3_row(q)] = C::dec(y1[t3_row(q)][c3 - kPlaneCx[q]]);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) {
        const int g = kT2Group[q], i = kT2Index[q], k = kT2Reg[q];
        if (g >= 0)
          p2n[q] = g == 0 ? x1u2[i] : (g == 1 ? x1c[i] : e[t3_row(q)]);
        else
          p2n[q] = kPlaneCy[q] == 0 ? z1c[k] : (kPlaneCy[q] == 1 ? z1u2[k] : n2d[k]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        x1u2[i] = x1u1[i];
        x1u1[i] = e[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) x1c[i] = e[2 + i];
      if (do3) {
        float m[5];
        site_moments(p2n, m);
#pragma unroll
        for (int k = 0; k < NF; ++k) m2[s0][k][lc + 1] = m[k];
      }
    }
    __syncthreads();
    // 4. second update of row a - 3 (from pass 6 on), stored
    if (up4 && t >= 6) {
      const NbTerms kc =
          nb_terms<EDDY, KIN>(&m2[s2][0][0], &m2[s1][0][0], &m2[s0][0][0], W + 2, lc + 1, c12);
      float f[9], g[10];
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = p2c[i];
#pragma unroll
      for (int k = 0; k < 10; ++k) g[k] = p2c[9 + k];
      collide<EDDY, KIN>(f, g, rt, kc);
      const unsigned od = unsigned(y0 - 6 + t) * geo.pitch + unsigned(xc);
#pragma unroll
      for (int i = 0; i < 9; ++i) st_plane_nt<T>(dst + i * P, od, C::enc(f[i]));
#pragma unroll
      for (int k = 0; k < 10; ++k) st_plane_nt<T>(dst + (9 + k) * P, od, C::enc(g[k]));
    }
#pragma unroll
    for (int q = 0; q < kNPop; ++q) {
      p1c[q] = has ? p1n[q] : 0.0f;
      p2c[q] = do3 ? p2n[q] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      z1u2[k] = z1u1[k];
      z1u1[k] = do2 ? n2u[k] : 0.0f;
      z1c[k] = do2 ? n2c[k] : 0.0f;
    }
  }
}

// ------------------------------------------------------ in-place (AA) step
// One lattice updated in place by two alternating steps.  Layout N (natural,
// as for k_step): slot q at x holds the post-collision f*_q(x).  Layout R
// (reversed): slot opp(q) at x + c_q holds f*_q(x).
//   PHASE 0, N -> R: pre_q(x) = N_q(x - c_q), the pull gather of k_step;
//     collide; f*_q(x) is stored in slot opp(q) at x + c_q.
//   PHASE 1, R -> N: pre_q(x) = R_opp(q)(x), all local; collide; f*_q(x) is
//     stored in slot q at x.
// In both phases the locations whose values a thread uses and the locations
// it writes are the same set, and no two threads share one, so no thread
// reads a value another thread writes in the same launch.  (With V = 2 the
// paired loads of x-moving planes also fetch one neighbour element that is
// not used; x-moving planes are stored element by element.)
__device__ constexpr int kPlaneOpp[kNPop] = {0,  3,  4,  1,  2,  7,  8,  5,  6, 9,
                                             12, 13, 10, 11, 14, 17, 18, 15, 16};

template <int ST, int V, bool LES, int PHASE>
__global__ __launch_bounds__(kStepThreads) void k_step_aa(typename Codec<ST>::T* __restrict__ lat,
                                                          Geom geo, Rates rt, int tiles_x) {
  using C = Codec<ST>;
  using T = typename C::T;
  using VT = typename Vec<T, V>::type;
  const int x0 = ((int(blockIdx.x) % tiles_x) * kStepThreads + int(threadIdx.x)) * V;
  const int y = int(blockIdx.x) / tiles_x;
  if (x0 >= geo.nx) return;
  const int xl = x0 == 0 ? geo.nx - 1 : x0 - 1;
  const int xr = x0 + V == geo.nx ? 0 : x0 + V;
  const int ym = y == 0 ? geo.ny - 1 : y - 1;
  const int yp = y == geo.ny - 1 ? 0 : y + 1;
  // row[c + 1] is the row of y - c
  const unsigned row[3] = {unsigned(yp) * geo.pitch, unsigned(y) * geo.pitch,
                           unsigned(ym) * geo.pitch};
  const long long P = geo.plane;
  float v[kNPop][V];
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    if (PHASE == 1) {
      const VT a = ld_plane<VT>(lat + kPlaneOpp[q] * P, row[1] + unsigned(x0));
      if constexpr (V == 1) {
        v[q][0] = C::dec(a);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) v[q][j] = C::dec(a[j]);
      }
    } else {
      const T* __restrict__ base = lat + q * P;
      const unsigned r = row[kPlaneCy[q] + 1];
      if (V == 1 || kPlaneCx[q] == 0) {
        const int xs = kPlaneCx[q] == 0 ? x0 : (kPlaneCx[q] == 1 ? xl : xr);
        const VT a = ld_plane<VT>(base, r + unsigned(xs));
        if constexpr (V == 1) {
          v[q][0] = C::dec(a);
        } else {
#pragma unroll
          for (int j = 0; j < V; ++j) v[q][j] = C::dec(a[j]);
        }
      } else if constexpr (V > 1) {
        const VT a = ld_plane<VT>(base, r + unsigned(x0));
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
  float out[kNPop][V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    float f[9], g[10];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = v[i][j];
#pragma unroll
    for (int k = 0; k < 10; ++k) g[k] = v[9 + k][j];
    collide<LES ? 1 : 0, false, ST == kFP16S>(f, g, rt);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i][j] = f[i];
#pragma unroll
    for (int k = 0; k < 10; ++k) out[9 + k][j] = g[k];
  }
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    if (PHASE == 1 || kPlaneCx[q] == 0) {
      // local store (PHASE 1), or the unshifted x of a plane moving along y only
      T* __restrict__ base = lat + (PHASE == 1 ? q : kPlaneOpp[q]) * P;
      const unsigned r = PHASE == 1 ? row[1] : row[1 - kPlaneCy[q]];
      VT w;
      if constexpr (V == 1) {
        w = C::enc(out[q][0]);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) w[j] = C::enc(out[q][j]);
      }
      st_plane_nt<VT>(base, r + unsigned(x0), w);
    } else {
      // f*_q(x0 + j) goes to x0 + j + c_x: one element at a time
      T* __restrict__ base = lat + kPlaneOpp[q] * P;
      const unsigned r = row[1 - kPlaneCy[q]];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        int xd = x0 + j + kPlaneCx[q];
        xd = xd < 0 ? geo.nx - 1 : (xd >= geo.nx ? xd - geo.nx : xd);
        st_plane_nt<T>(base, r + unsigned(xd), C::enc(out[q][j]));
      }
    }
  }
}

// Layout R -> N in place: for each plane q of one direction of every
// opposite pair (the other is opp(q)), swap slot q at x with slot opp(q) at
// x + c_q.  Each pair of locations belongs to exactly one (x, q), so the
// swaps are independent.  One workgroup per row.
template <int ST>
__global__ __launch_bounds__(256) void k_unswap_aa(typename Codec<ST>::T* __restrict__ lat,
                                                   Geom geo) {
  using T = typename Codec<ST>::T;
  constexpr int kHalf[8] = {1, 2, 5, 6, 10, 11, 15, 16};
  const int y = int(blockIdx.x);
  const long long P = geo.plane;
  for (int x = int(threadIdx.x); x < geo.nx; x += int(blockDim.x)) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int q = kHalf[h];
      int xd = x + kPlaneCx[q], yd = y + kPlaneCy[q];
      xd = xd < 0 ? geo.nx - 1 : (xd >= geo.nx ? 0 : xd);
      yd = yd < 0 ? geo.ny - 1 : (yd >= geo.ny ? 0 : yd);
      T* a = lat + q * P + (long long)y * geo.pitch + x;
      T* b = lat + kPlaneOpp[q] * P + (long long)yd * geo.pitch + xd;
      const T t = *a;
      *a = *b;
      *b = t;
    }
  }
}

// ------------------------------------------------------- initialisation etc.
// f^eq - w and g^eq of Sec. 3 in FP64 at one site.
__device__ __forceinline__ void equilibrium_dev(double rho, double ux, double uy, double bx,
                                                double by, double (&df)[9], double (&gq)[10]) {
  const double u2 = ux * ux + uy * uy, b2 = bx * bx + by * by;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cu = kCx[i] * ux + kCy[i] * uy;
    const double cb = kCx[i] * bx + kCy[i] * by;
    const double c2 = double(kCx[i] * kCx[i] + kCy[i] * kCy[i]);
    df[i] = kW[i] * (rho - 1.0) + kW[i] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * u2) +
            4.5 * kW[i] * (0.5 * b2 * c2 - cb * cb);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double cu = kMx[k] * ux + kMy[k] * uy;
    const double cb = kMx[k] * bx + kMy[k] * by;
    gq[k] = kWm[k] * (bx + 3.0 * (cu * bx - cb * ux));
    gq[5 + k] = kWm[k] * (by + 3.0 * (cu * by - cb * uy));
  }
}

template <int ST>
__global__ void k_init(const double* __restrict__ rho, const double* __restrict__ ux,
                       const double* __restrict__ uy, const double* __restrict__ bx,
                       const double* __restrict__ by, typename Codec<ST>::T* __restrict__ lat,
                       Geom geo) {
  using C = Codec<ST>;
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  double df[9], gq[10];
  equilibrium_dev(rho[s], ux[s], uy[s], bx[s], by[s], df, gq);
  const long long o = (long long)y * geo.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) lat[i * geo.plane + o] = C::enc(float(df[i]));
#pragma unroll
  for (int q = 0; q < 10; ++q) lat[(9 + q) * geo.plane + o] = C::enc(float(gq[q]));
}

template <int ST>
__global__ void k_decode(const typename Codec<ST>::T* __restrict__ lat, double* __restrict__ out,
                         Geom geo) {
  using C = Codec<ST>;
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  const long long o = (long long)y * geo.pitch + x;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    const double w = q < 9 ? kW[q] : 0.0;
    out[q * n + s] = w + double(C::dec(lat[q * geo.plane + o]));
  }
}

template <int ST>
__global__ void k_encode(const double* __restrict__ in, typename Codec<ST>::T* __restrict__ lat,
                         Geom geo) {
  using C = Codec<ST>;
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  const long long o = (long long)y * geo.pitch + x;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    const double w = q < 9 ? kW[q] : 0.0;
    lat[q * geo.plane + o] = C::enc(float(in[q * n + s] - w));
  }
}

// Macroscopic fields (FP64) of the stored state at one site; returns false if
// any population is not finite.
template <int ST>
__device__ __forceinline__ bool macro_site(const typename Codec<ST>::T* __restrict__ lat,
                                           const Geom& geo, long long o, double& rho,
                                           double& ux, double& uy, double& bx, double& by) {
  using C = Codec<ST>;
  float v[kNPop];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < kNPop; ++q) {
    v[q] = C::dec(lat[q * geo.plane + o]);
    ok = ok && isfinite(v[q]);
  }
  double dr = 0.0, jx = 0.0, jy = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    dr += double(v[i]);
    jx += kCx[i] * double(v[i]);
    jy += kCy[i] * double(v[i]);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    b0 += double(v[9 + k]);
    b1 += double(v[14 + k]);
  }
  rho = 1.0 + dr;
  ux = jx / rho;
  uy = jy / rho;
  bx = b0;
  by = b1;
  return ok;
}

template <int ST>
__global__ void k_macro(const typename Codec<ST>::T* __restrict__ lat, double* __restrict__ rho,
                        double* __restrict__ ux, double* __restrict__ uy,
                        double* __restrict__ bx, double* __restrict__ by, Geom geo) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int y = int(s / geo.nx), x = int(s % geo.nx);
  double r, a, b, c, d;
  macro_site<ST>(lat, geo, (long long)y * geo.pitch + x, r, a, b, c, d);
  rho[s] = r;
  ux[s] = a;
  uy[s] = b;
  bx[s] = c;
  by[s] = d;
}

template <int ST>
__global__ void k_macro_box(const typename Codec<ST>::T* __restrict__ lat, int w,
                            double* __restrict__ rho, double* __restrict__ ux,
                            double* __restrict__ uy, double* __restrict__ bx,
                            double* __restrict__ by, Geom geo) {
  const int cnx = geo.nx / w, cny = geo.ny / w;
  const long long n = (long long)cnx * cny;
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int cy = int(s / cnx), cx = int(s % cnx);
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int dy = 0; dy < w; ++dy)
    for (int dx = 0; dx < w; ++dx) {
      double v[5];
      macro_site<ST>(lat, geo, (long long)(cy * w + dy) * geo.pitch + (cx * w + dx), v[0], v[1],
                     v[2], v[3], v[4]);
#pragma unroll
      for (int q = 0; q < 5; ++q) a[q] += v[q];
    }
  const double iw = 1.0 / (double(w) * w);
  rho[s] = a[0] * iw;
  ux[s] = a[1] * iw;
  uy[s] = a[2] * iw;
  bx[s] = a[3] * iw;
  by[s] = a[4] * iw;
}

// Per-block partial sums of |u - u_t|^2 + |B - B_t|^2 (grid-stride over sites).
template <int ST>
__global__ __launch_bounds__(256) void k_mismatch(const typename Codec<ST>::T* __restrict__ lat,
                                                  const double* __restrict__ ux_t,
                                                  const double* __restrict__ uy_t,
                                                  const double* __restrict__ bx_t,
                                                  const double* __restrict__ by_t,
                                                  double* __restrict__ part, Geom geo) {
  __shared__ double sh[256];
  const long long n = (long long)geo.nx * geo.ny;
  double acc = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = int(s / geo.nx), x = int(s % geo.nx);
    double r, u, v, b0, b1;
    macro_site<ST>(lat, geo, (long long)y * geo.pitch + x, r, u, v, b0, b1);
    const double du = u - ux_t[s], dv = v - uy_t[s], d0 = b0 - bx_t[s], d1 = b1 - by_t[s];
    acc += du * du + dv * dv + d0 * d0 + d1 * d1;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n16) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------------------ diagnostics
enum {
  kSumMass = 0, kSumMx, kSumMy, kSumBx, kSumBy, kSumEk, kSumEm, kSumHc, kSumOm, kSumJ2,
  kSumBad, kNSum,          // slots 0..10 are sums
  kMaxDiv = kNSum, kMaxU,  // slots 11, 12 are maxima
  kNRed
};

template <int NT>
__device__ void block_reduce(double (&v)[kNRed], double* __restrict__ out) {
  __shared__ double sh[kNRed][NT];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kNRed; ++q) sh[q][t] = v[q];
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < kNSum; ++q) sh[q][t] += sh[q][t + w];
#pragma unroll
      for (int q = kNSum; q < kNRed; ++q) sh[q][t] = fmax(sh[q][t], sh[q][t + w]);
    }
    __syncthreads();
  }
  if (t < kNRed) out[t] = t == kMaxU ? sqrt(sh[t][0]) : sh[t][0];
}

// One pass over the lattice: a block of kDiagThreads threads owns as many
// columns and walks strips of kDiagRows rows (tile t, strip r: unit
// r * tiles_x + t; a block takes units blockIdx.x, + gridDim.x, ...).  Per row
// it loads the populations of row y + 1 (no streaming: the moments of the
// current state), forms rho, u, B in FP64 into a rolling 3-row LDS buffer with
// one halo column on each side, and then accumulates row y: the sums and
// maxima of the site's own fields and the centred differences
// d_x a = (a(x + 1) - a(x - 1)) / 2 of div B, w = d_x u_y - d_y u_x and
// j = d_x B_y - d_y B_x.  A site with a non-finite population has rho = NaN.
// Each block writes one partial (sums, maxima) to part[blockIdx.x], with the
// largest |u|^2 in the slot of max |u|: the final fold takes its square root
// (a correctly rounded square root is monotone, so the root of the largest
// square is the largest root).
constexpr int kDiagThreads = 256;
constexpr int kDiagRows = 64;   // 8-11% faster than 16 rows (fewer halo rows)

constexpr int kDiagNC = kDiagThreads + 2;
typedef double DiagRing[3][5][kDiagNC];   // rho, ux, uy, Bx, By of three rows

// The moments of one site from its stored populations (deviations f - w in
// the storage order, decoded by C) into column col of ring slot `slot`: rho
// (NaN when a population is not finite), u = j / rho and B.  Contraction is
// off here and in the two functions below, so that every kernel inlining
// them forms the diagnostics identically.
template <class C>
__device__ __forceinline__ void diag_moments(const typename C::T (&p)[kNPop], DiagRing& mac,
                                             int slot, int col) {
#pragma clang fp contract(off)
  bool ok = true;
  double dr = 0.0, jx = 0.0, jy = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float f = C::dec(p[i]);
    ok = ok && isfinite(f);
    dr += double(f);
    jx += kCx[i] * double(f);
    jy += kCy[i] * double(f);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const float gx = C::dec(p[9 + k]), gy = C::dec(p[14 + k]);
    ok = ok && isfinite(gx) && isfinite(gy);
    b0 += double(gx);
    b1 += double(gy);
  }
  const double r = 1.0 + dr;
  const double ir = 1.0 / r;
  mac[slot][0][col] = ok ? r : __builtin_nan("");
  mac[slot][1][col] = jx * ir;
  mac[slot][2][col] = jy * ir;
  mac[slot][3][col] = b0;
  mac[slot][4][col] = b1;
}

// Adds the site in ring column c of the middle row (slot s0; sm below, sp
// above) to the thread's sums and maxima.
__device__ __forceinline__ void diag_accumulate(double (&v)[kNRed], const DiagRing& mac, int sm,
                                                int s0, int sp, int c) {
#pragma clang fp contract(off)
  const double r = mac[s0][0][c], ux = mac[s0][1][c], uy = mac[s0][2][c];
  const double b0 = mac[s0][3][c], b1 = mac[s0][4][c];
  const double jx = r * ux, jy = r * uy;
  v[kSumMass] += r;
  v[kSumMx] += jx;
  v[kSumMy] += jy;
  v[kSumBx] += b0;
  v[kSumBy] += b1;
  v[kSumEk] += 0.5 * (jx * ux + jy * uy);   // |j|^2 / (2 rho)
  v[kSumEm] += 0.5 * (b0 * b0 + b1 * b1);
  v[kSumHc] += ux * b0 + uy * b1;
  const double div = 0.5 * (mac[s0][3][c + 1] - mac[s0][3][c - 1]) +
                     0.5 * (mac[sp][4][c] - mac[sm][4][c]);
  const double om = 0.5 * (mac[s0][2][c + 1] - mac[s0][2][c - 1]) -
                    0.5 * (mac[sp][1][c] - mac[sm][1][c]);
  const double jz = 0.5 * (mac[s0][4][c + 1] - mac[s0][4][c - 1]) -
                    0.5 * (mac[sp][3][c] - mac[sm][3][c]);
  v[kSumOm] += 0.5 * om * om;
  v[kSumJ2] += 0.5 * jz * jz;
  v[kSumBad] += isfinite(r) ? 0.0 : 1.0;
  v[kMaxDiv] = fmax(v[kMaxDiv], fabs(div));
  v[kMaxU] = fmax(v[kMaxU], ux * ux + uy * uy);   // |u|^2: rooted in the fold
}

// The block's sums and maxima into part[blockIdx.x], reduced in the (idle)
// ring.
__device__ __forceinline__ void diag_partial(const double (&v)[kNRed], DiagRing& mac,
                                             double* __restrict__ part) {
#pragma clang fp contract(off)
  static_assert(3 * 5 * kDiagNC >= kNRed * kDiagThreads, "ring too small to reduce in");
  const int tx = int(threadIdx.x);
  double* red = &mac[0][0][0];
#pragma unroll
  for (int q = 0; q < kNRed; ++q) red[q * kDiagThreads + tx] = v[q];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if (tx < w) {
#pragma unroll
      for (int q = 0; q < kNSum; ++q) red[q * kDiagThreads + tx] += red[q * kDiagThreads + tx + w];
#pragma unroll
      for (int q = kNSum; q < kNRed; ++q)
        red[q * kDiagThreads + tx] = fmax(red[q * kDiagThreads + tx], red[q * kDiagThreads + tx + w]);
    }
    __syncthreads();
  }
  if (tx < kNRed) part[(long long)blockIdx.x * kDiagSlots + tx] = red[tx * kDiagThreads];
}

template <int ST>
__global__ __launch_bounds__(kDiagThreads) void k_diag(const typename Codec<ST>::T* __restrict__ lat,
                                                       double* __restrict__ part, Geom geo,
                                                       int tiles_x, int units) {
  using C = Codec<ST>;
  using T = typename C::T;
  __shared__ DiagRing mac;
  const int tx = int(threadIdx.x);
  double v[kNRed];
#pragma unroll
  for (int q = 0; q < kNRed; ++q) v[q] = 0.0;
  for (int u = int(blockIdx.x); u < units; u += int(gridDim.x)) {
    const int xt = (u % tiles_x) * kDiagThreads;
    const int y0 = (u / tiles_x) * kDiagRows;
    const int y1 = min(y0 + kDiagRows, geo.ny);
    const int x = xt + tx;
    const bool active = x < geo.nx;
    const int xc = x % geo.nx;   // past the last column: its periodic images
    const int xh = tx == 0 ? (xt == 0 ? geo.nx - 1 : xt - 1) : (xt + kDiagThreads) % geo.nx;
    const int ch = tx == 0 ? 0 : kDiagNC - 1;
    T raw[kNPop], rawh[kNPop];
    auto load = [&](int xx, int yy, T (&p)[kNPop]) {
      const unsigned o = unsigned(yy) * geo.pitch + unsigned(xx);
#pragma unroll
      for (int q = 0; q < kNPop; ++q) p[q] = ld_plane<T>(lat + q * geo.plane, o);
    };
    auto issue = [&](int yy) {
      yy = yy < 0 ? yy + geo.ny : (yy >= geo.ny ? yy - geo.ny : yy);
      load(xc, yy, raw);
      if (tx < 2) load(xh, yy, rawh);
    };
    auto commit = [&](int slot) {
      diag_moments<C>(raw, mac, slot, tx + 1);
      if (tx < 2) diag_moments<C>(rawh, mac, slot, ch);
    };
    issue(y0 - 1);
    commit(0);
    issue(y0);
    commit(1);
    issue(y0 + 1);
    for (int y = y0; y < y1; ++y) {
      const int sm = (y - y0) % 3, s0 = (y - y0 + 1) % 3, sp = (y - y0 + 2) % 3;
      commit(sp);
      if (y + 2 <= y1) issue(y + 2);
      __syncthreads();
      if (active) diag_accumulate(v, mac, sm, s0, sp, tx + 1);
      __syncthreads();
    }
  }
  diag_partial(v, mac, part);
}

// One step src -> dst (as k_step, FP32 storage) fused with the diagnostics
// of dst (as k_diag): the same tiles, strips, units and accumulation order, so
// the partials equal those of k_diag on the stored result bit for bit.  Each
// block computes the new state of its strip's rows and of the row above and
// below (not stored), on its tile's columns and one halo column on each side
// (threads 0 and 1, not stored), gathering the next row while it accumulates
// the current one; only the strip's own rows and columns are written.
template <bool LES>
__global__ __launch_bounds__(kDiagThreads) void k_step_diag(const float* __restrict__ src,
                                                            float* __restrict__ dst,
                                                            double* __restrict__ part, Geom geo,
                                                            Rates rt, int tiles_x, int units) {
  __shared__ DiagRing mac;
  const int tx = int(threadIdx.x);
  const long long P = geo.plane;
  double v[kNRed];
#pragma unroll
  for (int q = 0; q < kNRed; ++q) v[q] = 0.0;
  for (int u = int(blockIdx.x); u < units; u += int(gridDim.x)) {
    const int xt = (u % tiles_x) * kDiagThreads;
    const int y0 = (u / tiles_x) * kDiagRows;
    const int y1 = min(y0 + kDiagRows, geo.ny);
    const int x = xt + tx;
    const bool active = x < geo.nx;
    const int xc = x % geo.nx;   // past the last column: its periodic images
    const int xh = tx == 0 ? (xt == 0 ? geo.nx - 1 : xt - 1) : (xt + kDiagThreads) % geo.nx;
    const int ch = tx == 0 ? 0 : kDiagNC - 1;
    const int xcl = xc == 0 ? geo.nx - 1 : xc - 1, xcr = xc == geo.nx - 1 ? 0 : xc + 1;
    const int xhl = xh == 0 ? geo.nx - 1 : xh - 1, xhr = xh == geo.nx - 1 ? 0 : xh + 1;
    float f[kNPop][1], fh[kNPop][1];   // the gathered row in flight
    auto gather = [&](int r) {
      unsigned row[3];
      t2_rows(r, geo, row);
      gather_row<LBMHD_FP32, 1>(src, P, xc, xcl, xcr, row, f);
      if (tx < 2) gather_row<LBMHD_FP32, 1>(src, P, xh, xhl, xhr, row, fh);
    };
    auto moments = [&](const float (&w)[kNPop][1], int slot, int col) {
      float e[kNPop];   // FP32 storage: the values stored are the collided ones
#pragma unroll
      for (int q = 0; q < kNPop; ++q) e[q] = w[q][0];
      diag_moments<Codec<LBMHD_FP32>>(e, mac, slot, col);
    };
    // collide the gathered row r, store it if it is one of the strip's rows,
    // and put its moments into ring slot `slot`
    auto finish = [&](int r, int slot) {
      collide_sites<1, LES, false>(f, rt);
      if (active && r >= y0 && r < y1)
        store_row<LBMHD_FP32, 1>(dst, P, unsigned(r) * geo.pitch + unsigned(x), f);
      moments(f, slot, tx + 1);
      if (tx < 2) {
        collide_sites<1, LES, false>(fh, rt);
        moments(fh, slot, ch);
      }
    };
    gather(y0 - 1);
    finish(y0 - 1, 0);
    gather(y0);
    finish(y0, 1);
    gather(y0 + 1);
    for (int y = y0; y < y1; ++y) {
      const int sm = (y - y0) % 3, s0 = (y - y0 + 1) % 3, sp = (y - y0 + 2) % 3;
      finish(y + 1, sp);
      if (y + 2 <= y1) gather(y + 2);
      __syncthreads();
      if (active) diag_accumulate(v, mac, sm, s0, sp, tx + 1);
      __syncthreads();
    }
  }
  diag_partial(v, mac, part);
}

// Pass 3: one block folds the partials.
__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out) {
  double v[kNRed];
#pragma unroll
  for (int q = 0; q < kNRed; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < kNSum; ++q) v[q] += part[(long long)b * kDiagSlots + q];
#pragma unroll
    for (int q = kNSum; q < kNRed; ++q) v[q] = fmax(v[q], part[(long long)b * kDiagSlots + q]);
  }
  block_reduce<256>(v, out);
}

__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ in, long long n,
                                             double* __restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a += in[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

inline unsigned blocks_for(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

// ----------------------------------------------------------------- launchers
template <int ST, int V>
void launch_step_v(bool les, const void* src, void* dst, const Geom& g, const Rates& r,
                   hipStream_t s) {
  using T = typename Codec<ST>::T;
  const int tiles_x = (g.nx / V + kStepThreads - 1) / kStepThreads;
  const dim3 grid(unsigned(tiles_x) * unsigned(g.ny)), block(kStepThreads);
  auto* a = static_cast<const T*>(src);
  auto* b = static_cast<T*>(dst);
  if (les)
    hipLaunchKernelGGL((k_step<ST, V, true>), grid, block, 0, s, a, b, g, r, tiles_x);
  else
    hipLaunchKernelGGL((k_step<ST, V, false>), grid, block, 0, s, a, b, g, r, tiles_x);
}

// Strip height of the two-step kernel, measured on MI355X: FP32 runs best
// with about 512 blocks (2048^2: 32 rows, 4096^2: 128), FP16 with about 4096
// (8192^2: 32 rows, 4096^2 and 2048^2: 8); halo overhead 2 / rows.
static int step2_rows(const Geom& g, int storage, int V) {
  const bool fp16 = storage != LBMHD_FP32;   // LBMHD_FP16 or its scaled tag
  const long long tiles_x = (g.nx + kT2Threads * V - 1) / (kT2Threads * V);
  const long long rows = tiles_x * g.ny / (fp16 ? 4096 : 512);
  const long long hi = fp16 ? 32 : 128;
  return int(rows < 8 ? 8 : (rows > hi ? hi : rows));
}

template <int ST, int V>
void launch_step2_v(bool les, const void* src, void* dst, void* mid, const Geom& g,
                    const Rates& r, hipStream_t s) {
  using T = typename Codec<ST>::T;
  const int rows = step2_rows(g, ST, V);
  const int tiles_x = (g.nx + kT2Threads * V - 1) / (kT2Threads * V);
  const int strips = (g.ny + rows - 1) / rows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kT2Threads);
  const bool xcd_map = strips % 8 == 0;
  auto* a = static_cast<const T*>(src);
  auto* b = static_cast<T*>(dst);
  auto* m = static_cast<T*>(mid);
  if (les && m)
    hipLaunchKernelGGL((k_step2<ST, V, true, true>), grid, block, 0, s, a, b, m, g, r, tiles_x,
                       rows, xcd_map);
  else if (les)
    hipLaunchKernelGGL((k_step2<ST, V, true, false>), grid, block, 0, s, a, b, m, g, r, tiles_x,
                       rows, xcd_map);
  else if (m)
    hipLaunchKernelGGL((k_step2<ST, V, false, true>), grid, block, 0, s, a, b, m, g, r, tiles_x,
                       rows, xcd_map);
  else
    hipLaunchKernelGGL((k_step2<ST, V, false, false>), grid, block, 0, s, a, b, m, g, r,
                       tiles_x, rows, xcd_map);
}

template <int ST, int EDDY, bool KIN>
void launch_step_nb_t(const void* src, void* dst, const Geom& g, const Rates& r, float c12,
                      hipStream_t s) {
  using T = typename Codec<ST>::T;
  const int tiles_x = (g.nx + kKinThreads - 1) / kKinThreads;
  const int strips = (g.ny + kKinRows - 1) / kKinRows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kKinThreads);
  hipLaunchKernelGGL((k_step_nb<ST, EDDY, KIN>), grid, block, 0, s, static_cast<const T*>(src),
                     static_cast<T*>(dst), g, r, c12, tiles_x);
}

template <int ST>
hipError_t launch_step_nb_s(int eddy, bool kin, const void* src, void* dst, const Geom& g,
                            const Rates& r, float c12, hipStream_t s) {
  if (kin && eddy == 0)
    launch_step_nb_t<ST, 0, true>(src, dst, g, r, c12, s);
  else if (kin && eddy == 1)
    launch_step_nb_t<ST, 1, true>(src, dst, g, r, c12, s);
  else if (kin && eddy == 2)
    launch_step_nb_t<ST, 2, true>(src, dst, g, r, c12, s);
  else if (!kin && eddy == 2)
    launch_step_nb_t<ST, 2, false>(src, dst, g, r, c12, s);
  else
    return hipErrorInvalidValue;   // no neighbour terms: the plain step applies
  return hipGetLastError();
}

// Strip height of the two-step kernel with lattice gradients (halo overhead
// 6 / rows): as for the three-step kernel, about 512 blocks up to 128-row
// strips, 32-row strips beyond.
static int step_nb2_rows(const Geom& g) {
  const long long tiles_x = (g.nx + kNb2Cols - 1) / kNb2Cols;
  const long long rows = tiles_x * g.ny / 512;
  return int(rows < 8 ? 8 : (rows > 128 ? 32 : rows));
}

template <int ST, int EDDY, bool KIN>
void launch_step_nb2_t(const void* src, void* dst, void* mid, const Geom& g, const Rates& r,
                       float c12, hipStream_t s) {
  using T = typename Codec<ST>::T;
  const int rows = step_nb2_rows(g);
  const int tiles_x = (g.nx + kNb2Cols - 1) / kNb2Cols;
  const int strips = (g.ny + rows - 1) / rows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kNb2Threads);
  const bool xcd_map = strips % 8 == 0;
  auto* a = static_cast<const T*>(src);
  auto* b = static_cast<T*>(dst);
  auto* m = static_cast<T*>(mid);
  if (m)
    hipLaunchKernelGGL((k_step_nb2<ST, EDDY, KIN, true>), grid, block, 0, s, a, b, m, g, r, c12,
                       tiles_x, rows, xcd_map);
  else
    hipLaunchKernelGGL((k_step_nb2<ST, EDDY, KIN, false>), grid, block, 0, s, a, b, m, g, r, c12,
                       tiles_x, rows, xcd_map);
}

template <int ST>
hipError_t launch_step_nb2_s(int eddy, bool kin, const void* src, void* dst, void* mid,
                             const Geom& g, const Rates& r, float c12, hipStream_t s) {
  if (kin && eddy == 0)
    launch_step_nb2_t<ST, 0, true>(src, dst, mid, g, r, c12, s);
  else if (kin && eddy == 1)
    launch_step_nb2_t<ST, 1, true>(src, dst, mid, g, r, c12, s);
  else if (kin && eddy == 2)
    launch_step_nb2_t<ST, 2, true>(src, dst, mid, g, r, c12, s);
  else if (!kin && eddy == 2)
    launch_step_nb2_t<ST, 2, false>(src, dst, mid, g, r, c12, s);
  else
    return hipErrorInvalidValue;   // no neighbour terms: the plain kernels apply
  return hipGetLastError();
}

hipError_t launch_step_nb2(int storage, int eddy, bool kin, const void* src, void* dst,
                           void* mid, const Geom& g, const Rates& r, double delta,
                           hipStream_t s) {
  const float c12 = float(delta * delta / 12.0);
  if (storage == LBMHD_FP32)
    return launch_step_nb2_s<LBMHD_FP32>(eddy, kin, src, dst, mid, g, r, c12, s);
  return launch_step_nb2_s<LBMHD_FP16>(eddy, kin, src, dst, mid, g, r, c12, s);
}

bool step_nb2_pays(const Geom& g) {
  const long long tiles_x = (g.nx + kNb2Cols - 1) / kNb2Cols;
  return tiles_x * ((g.ny + 7) / 8) >= 512;
}

hipError_t launch_step_nb(int storage, int eddy, bool kin, const void* src, void* dst,
                          const Geom& g, const Rates& r, double delta, hipStream_t s) {
  const float c12 = float(delta * delta / 12.0);
  if (storage == LBMHD_FP32) return launch_step_nb_s<LBMHD_FP32>(eddy, kin, src, dst, g, r, c12, s);
  return launch_step_nb_s<LBMHD_FP16>(eddy, kin, src, dst, g, r, c12, s);
}

hipError_t launch_step(int storage, bool les, const void* src, void* dst, const Geom& g,
                       const Rates& r, hipStream_t s) {
  if (storage == LBMHD_FP32)
    launch_step_v<LBMHD_FP32, 1>(les, src, dst, g, r, s);
  else if (g.nx % 2 == 0)
    launch_step_v<kFP16S, 2>(les, src, dst, g, r, s);
  else
    launch_step_v<kFP16S, 1>(les, src, dst, g, r, s);
  return hipGetLastError();
}

bool step2_pays(int storage, const Geom& g) {
  const int V = storage == LBMHD_FP16 && g.nx % 2 == 0 ? 2 : 1;
  const long long tiles_x = (g.nx + kT2Threads * V - 1) / (kT2Threads * V);
  return tiles_x * ((g.ny + 7) / 8) >= 512;
}

// Strip height of the three-step kernel (halo overhead 4 / rows), measured:
// about 512 blocks, which all run at once (registers admit four per CU), up
// to 128-row strips (2048^2: 32 rows, 4096^2: 128; 64-row strips there, 1024
// blocks, were slower); on larger lattices 32-row strips (8192^2: 16-row
// strips as fast, 64 and 8 rows 3% and 8% slower).
static int step_t3_rows(const Geom& g) {
  const long long tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const long long rows = tiles_x * g.ny / 512;
  return int(rows < 8 ? 8 : (rows > 128 ? 32 : rows));
}

hipError_t launch_step_t3(bool les, const void* src, void* dst, void* mid1, void* mid2,
                          const Geom& g, const Rates& r, hipStream_t s) {
  const int rows = step_t3_rows(g);
  const int tiles_x = (g.nx + kT3Cols - 1) / kT3Cols;
  const int strips = (g.ny + rows - 1) / rows;
  const dim3 grid(unsigned(tiles_x) * unsigned(strips)), block(kT3Threads);
  const bool xcd_map = strips % 8 == 0;
  auto* a = static_cast<const float*>(src);
  auto* b = static_cast<float*>(dst);
  auto* m1 = static_cast<float*>(mid1);
  auto* m2 = static_cast<float*>(mid2);
  if (m1 && les)
    hipLaunchKernelGGL((k_step_t3<true, true>), grid, block, 0, s, a, b, m1, m2, g, r, tiles_x,
                       rows, xcd_map);
  else if (m1)
    hipLaunchKernelGGL((k_step_t3<false, true>), grid, block, 0, s, a, b, m1, m2, g, r, tiles_x,
                       rows, xcd_map);
  else if (les)
    hipLaunchKernelGGL((k_step_t3<true, false>), grid, block, 0, s, a, b, m1, m2, g, r, tiles_x,
                       rows, xcd_map);
  else
    hipLaunchKernelGGL((k_step_t3<false, false>), grid, block, 0, s, a, b, m1, m2, g, r,
                       tiles_x, rows, xcd_map);
  return hipGetLastError();
}

hipError_t launch_step2(int storage, bool les, const void* src, void* dst, void* mid,
                        const Geom& g, const Rates& r, hipStream_t s) {
  if (storage == LBMHD_FP32)
    launch_step2_v<LBMHD_FP32, 1>(les, src, dst, mid, g, r, s);
  else if (g.nx % 2 == 0)
    launch_step2_v<kFP16S, 2>(les, src, dst, mid, g, r, s);
  else
    launch_step2_v<kFP16S, 1>(les, src, dst, mid, g, r, s);
  return hipGetLastError();
}

template <int ST, int V, int PHASE>
void launch_step_aa_v(bool les, void* lat, const Geom& g, const Rates& r, hipStream_t s) {
  using T = typename Codec<ST>::T;
  const int tiles_x = (g.nx / V + kStepThreads - 1) / kStepThreads;
  const dim3 grid(unsigned(tiles_x) * unsigned(g.ny)), block(kStepThreads);
  auto* a = static_cast<T*>(lat);
  if (les)
    hipLaunchKernelGGL((k_step_aa<ST, V, true, PHASE>), grid, block, 0, s, a, g, r, tiles_x);
  else
    hipLaunchKernelGGL((k_step_aa<ST, V, false, PHASE>), grid, block, 0, s, a, g, r, tiles_x);
}

// Both steps keep the widths of k_step: 1 FP32 or 2 FP16 sites per thread
// (16-byte vectors in the local step measured slower: 0.534 against 0.482
// ms per FP32 step at 4096^2, the register cost halving the occupancy).
template <int ST, int V>
void launch_step_aa_p(bool les, int phase, void* lat, const Geom& g, const Rates& r,
                      hipStream_t s) {
  if (phase == 0)
    launch_step_aa_v<ST, V, 0>(les, lat, g, r, s);
  else
    launch_step_aa_v<ST, V, 1>(les, lat, g, r, s);
}

hipError_t launch_step_aa(int storage, bool les, int phase, void* lat, const Geom& g,
                          const Rates& r, hipStream_t s) {
  if (storage == LBMHD_FP32)
    launch_step_aa_p<LBMHD_FP32, 1>(les, phase, lat, g, r, s);
  else if (g.nx % 2 == 0)
    launch_step_aa_p<kFP16S, 2>(les, phase, lat, g, r, s);
  else
    launch_step_aa_p<kFP16S, 1>(les, phase, lat, g, r, s);
  return hipGetLastError();
}

hipError_t launch_unswap_aa(int storage, void* lat, const Geom& g, hipStream_t s) {
  const unsigned nb = unsigned(g.ny);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_unswap_aa<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<float*>(lat), g);
  else
    hipLaunchKernelGGL(k_unswap_aa<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<_Float16*>(lat), g);
  return hipGetLastError();
}

hipError_t launch_init(int storage, const double* rho, const double* ux, const double* uy,
                       const double* bx, const double* by, void* lat, const Geom& g,
                       hipStream_t s) {
  const unsigned nb = blocks_for((long long)g.nx * g.ny, 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_init<LBMHD_FP32>, dim3(nb), dim3(256), 0, s, rho, ux, uy, bx, by,
                       static_cast<float*>(lat), g);
  else
    hipLaunchKernelGGL(k_init<LBMHD_FP16>, dim3(nb), dim3(256), 0, s, rho, ux, uy, bx, by,
                       static_cast<_Float16*>(lat), g);
  return hipGetLastError();
}

hipError_t launch_decode(int storage, const void* lat, double* out, const Geom& g,
                         hipStream_t s) {
  const unsigned nb = blocks_for((long long)g.nx * g.ny, 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_decode<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float*>(lat), out, g);
  else
    hipLaunchKernelGGL(k_decode<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), out, g);
  return hipGetLastError();
}

hipError_t launch_encode(int storage, const double* in, void* lat, const Geom& g,
                         hipStream_t s) {
  const unsigned nb = blocks_for((long long)g.nx * g.ny, 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_encode<LBMHD_FP32>, dim3(nb), dim3(256), 0, s, in,
                       static_cast<float*>(lat), g);
  else
    hipLaunchKernelGGL(k_encode<LBMHD_FP16>, dim3(nb), dim3(256), 0, s, in,
                       static_cast<_Float16*>(lat), g);
  return hipGetLastError();
}

hipError_t launch_macro(int storage, const void* lat, double* rho, double* ux, double* uy,
                        double* bx, double* by, const Geom& g, hipStream_t s) {
  const unsigned nb = blocks_for((long long)g.nx * g.ny, 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_macro<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float*>(lat), rho, ux, uy, bx, by, g);
  else
    hipLaunchKernelGGL(k_macro<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), rho, ux, uy, bx, by, g);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const long long n16 = (long long)(bytes / 16);
  const unsigned nb = unsigned(n16 < 256LL * 4096 ? blocks_for(n16, 256) : 4096u);
  if (n16 > 0)
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

int diag_partials(const Geom& g) {
  const int tiles_x = (g.nx + kDiagThreads - 1) / kDiagThreads;
  const long long units = (long long)tiles_x * ((g.ny + kDiagRows - 1) / kDiagRows);
  return int(std::min<long long>(kDiagBlocks, units));
}

hipError_t launch_diag(int storage, const void* lat, double* part, double* out_dev,
                       const Geom& g, hipStream_t s) {
  const int tiles_x = (g.nx + kDiagThreads - 1) / kDiagThreads;
  const long long units = (long long)tiles_x * ((g.ny + kDiagRows - 1) / kDiagRows);
  const int nparts = diag_partials(g);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_diag<LBMHD_FP32>, dim3(nparts), dim3(kDiagThreads), 0, s,
                       static_cast<const float*>(lat), part, g, tiles_x, int(units));
  else
    hipLaunchKernelGGL(k_diag<LBMHD_FP16>, dim3(nparts), dim3(kDiagThreads), 0, s,
                       static_cast<const _Float16*>(lat), part, g, tiles_x, int(units));
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, out_dev);
  return hipGetLastError();
}

hipError_t launch_step_diag(bool les, const void* src, void* dst, double* part, double* out_dev,
                            const Geom& g, const Rates& r, hipStream_t s) {
  const int tiles_x = (g.nx + kDiagThreads - 1) / kDiagThreads;
  const long long units = (long long)tiles_x * ((g.ny + kDiagRows - 1) / kDiagRows);
  const int nparts = diag_partials(g);
  auto* a = static_cast<const float*>(src);
  auto* b = static_cast<float*>(dst);
  if (les)
    hipLaunchKernelGGL(k_step_diag<true>, dim3(nparts), dim3(kDiagThreads), 0, s, a, b, part, g, r,
                       tiles_x, int(units));
  else
    hipLaunchKernelGGL(k_step_diag<false>, dim3(nparts), dim3(kDiagThreads), 0, s, a, b, part, g,
                       r, tiles_x, int(units));
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, out_dev);
  return hipGetLastError();
}

hipError_t launch_macro_box(int storage, const void* lat, int w, double* rho, double* ux,
                            double* uy, double* bx, double* by, const Geom& g, hipStream_t s) {
  const unsigned nb = blocks_for((long long)(g.nx / w) * (g.ny / w), 256);
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_macro_box<LBMHD_FP32>, dim3(nb), dim3(256), 0, s,
                       static_cast<const float*>(lat), w, rho, ux, uy, bx, by, g);
  else
    hipLaunchKernelGGL(k_macro_box<LBMHD_FP16>, dim3(nb), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), w, rho, ux, uy, bx, by, g);
  return hipGetLastError();
}

hipError_t launch_mismatch(int storage, const void* lat, const double* ux_t, const double* uy_t,
                           const double* bx_t, const double* by_t, double* part, double* out_dev,
                           const Geom& g, hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  const int nparts = int(std::min<long long>(kDiagBlocks, blocks_for(n, 256)));
  if (storage == LBMHD_FP32)
    hipLaunchKernelGGL(k_mismatch<LBMHD_FP32>, dim3(nparts), dim3(256), 0, s,
                       static_cast<const float*>(lat), ux_t, uy_t, bx_t, by_t, part, g);
  else
    hipLaunchKernelGGL(k_mismatch<LBMHD_FP16>, dim3(nparts), dim3(256), 0, s,
                       static_cast<const _Float16*>(lat), ux_t, uy_t, bx_t, by_t, part, g);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, part, (long long)nparts, out_dev);
  return hipGetLastError();
}

hipError_t launch_sum(const double* in, long long n, double* out_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, in, n, out_dev);
  return hipGetLastError();
}

}  // namespace lbk
