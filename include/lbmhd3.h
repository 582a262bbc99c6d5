/* lbmhd3.h -- C ABI of the three-dimensional LB-MHD update on MI355X (gfx950).
 *
 * Flint & Vahala, arXiv:1607.08675, work in 2D and state that the model
 * extends to 3D with more lattice velocities (Sec. 3, Sec. 5).  This is that
 * extension, built the way the 2D update is built:
 *  - f on D3Q27, the tensor product of the D1Q3 lattice (weights 8/27, 2/27,
 *    1/54, 1/216, whose sums over c_z are the paper's D2Q9 weights), with the
 *    second-order equilibrium
 *      f_i^eq = w_i [rho + 3 c_i.j + (9/2)(c_i c_i - I/3) : (j j / rho + |B|^2 I / 2 - B B)]
 *    (the 3D form of the paper's D2Q9 equilibrium with the Maxwell stress);
 *  - the magnetic vector populations g_kb on the six unit vectors +-x, +-y,
 *    +-z, weight 1/6 each (sums over C_z give the paper's D2Q5 weights),
 *    g_kb^eq = (B_b + 3 (C_k.u B_b - C_k.B u_b)) / 6;
 *  - single-relaxation collisions with tau0 = 3 nu + 1/2 and
 *    tau_m0 = 3 eta + 1/2 (the paper's moment-space collision with all rates
 *    equal; no 3D moment basis is given);
 *  - optionally the per-site Smagorinsky-MHD closure of the 2D update
 *    (eqs. SmagorinskyClosure, SmagorinskyMHDClosureV/B): Q = sqrt(2 Pi':Pi'),
 *    Pi' the traceless non-equilibrium stress, tau = (tau0 + sqrt(tau0^2 +
 *    18 C_Sv Delta^2 Q / rho)) / 2; A = eps : Lambda^neq, Lambda_ab =
 *    sum_k C_ka g_kb, tau_m = (tau_m0 + sqrt(tau_m0^2 + 36 C_Sb Delta^2 |A|)) / 2.
 * Fields that do not depend on one coordinate (and have no velocity or field
 * along it) evolve exactly as the paper's 2D update at equal rates.
 *
 * Conventions as in lbmhd.h (status codes LBMHD_*, caller-owned device
 * memory, one handle per stream, asynchronous calls unless stated).  Fields
 * are float64 device arrays of nx*ny*nz in [z][y][x] order, x fastest.
 * Population arrays are float64, 45 planes of nx*ny*nz: planes 0..26 the
 * D3Q27 populations with velocities
 *   (0,0,0), (1,0,0), (-1,0,0), (0,1,0), (0,-1,0), (0,0,1), (0,0,-1),
 *   (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 *   (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1), (1,1,1), (-1,-1,-1),
 *   (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1);
 * planes 27..32 the x component of g for C = +x, -x, +y, -y, +z, -z,
 * 33..38 the y component, 39..44 the z component.  The state is the
 * post-collision population at the current step (the step gathers from the
 * neighbours, then collides).  The lattice holds the encoded deviations f - w
 * and g (FP32, or FP16 scaled by 2^10, as `storage` selects) in 45 planes of
 * [z][y][row pitch padded to 256 bytes], successive planes spaced by their
 * rows plus a gap of 768 bytes (never read or written).
 */
#ifndef LBMHD3_H
#define LBMHD3_H

#include <stddef.h>
#include <stdint.h>

#include "lbmhd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmhd3 lbmhd3_t;

typedef struct {
  int32_t nx, ny, nz;     /* periodic lattice, each >= 1; one plane (nz * ny *
                             padded row) must stay below 4 GiB */
  double nu, eta;         /* viscosity and resistivity in lattice units, > 0 */
  int32_t les;            /* 0: fixed rates; 1: Smagorinsky-MHD closure */
  double cs, cs_b;        /* closure constants C_Sv, C_Sb >= 0 */
  double delta;           /* filter width Delta > 0 */
  int32_t storage;        /* LBMHD_FP32: deviations f - w (g as is) in FP32;
                             LBMHD_FP16: half(2^10 (f - w)), round to nearest
                             even (the 2D encodings); arithmetic in FP32 */
  int32_t mrt;            /* 0: single relaxation f* = f - (f - f^eq) / tau;
                             1: moment-space collision (Sec. 3) in the
                             tensor-product basis p_r(c_x, c_y) q_k(c_z) of
                             the paper's nine D2Q9 rows (eq. FluidTMatrix)
                             and q = 1, c_z, 3 c_z^2 - 1: the z sums (k = 0)
                             relax with the paper's 2D rates (shear 1/tau,
                             s5 for rows 5 and 6, s7, s8), so fields
                             invariant along z follow the 2D model exactly;
                             the shears xz, yz take 1/tau, the z normal
                             stress szz, every other moment varying along c_z
                             sg.  The basis singles out z. */
  double s5, s7, s8;      /* rates in (0, 2) of the 2D rows 5 and 6, 7, 8 */
  double sg, szz;         /* rates in (0, 2) (mrt = 1; ignored otherwise) */
} lbmhd3_params;

typedef struct {
  double mass, mom_x, mom_y, mom_z, flux_x, flux_y, flux_z;
  double e_kin, e_mag;    /* sum |rho u|^2 / (2 rho), sum |B|^2 / 2 */
  double max_abs_divB;    /* centred differences */
  double max_u;
  int64_t nonfinite;      /* sites with non-finite density */
  int64_t step;
} lbmhd3_diag_t;

/* Validate parameters and create a handle (host memory only).  Errors:
 * LBMHD_ERR_INVALID_ARG. */
int lbmhd3_create(const lbmhd3_params* p, lbmhd3_t** out);
/* Release the handle (not the caller's buffers).  NULL is accepted. */
int lbmhd3_destroy(lbmhd3_t* h);
/* Byte sizes of one lattice (two are bound) and of the workspace. */
int lbmhd3_sizes(const lbmhd3_t* h, size_t* lattice, size_t* workspace);
/* Attach two lattices, the workspace (device, 256-byte aligned, not
 * overlapping) and the HIP stream.  Errors: LBMHD_ERR_INVALID_ARG. */
int lbmhd3_bind(lbmhd3_t* h, void* lat_a, size_t lat_a_bytes, void* lat_b, size_t lat_b_bytes,
                void* workspace, size_t workspace_bytes, void* stream);
/* State = equilibria of the given device fields; step counter 0. */
int lbmhd3_init_fields(lbmhd3_t* h, const double* rho, const double* ux, const double* uy,
                       const double* uz, const double* bx, const double* by, const double* bz);
/* nsteps >= 0 steps, one kernel launch each. */
int lbmhd3_step(lbmhd3_t* h, int64_t nsteps);
/* rho (1 field), u (3 consecutive fields), B (3 consecutive fields), device. */
int lbmhd3_macro(lbmhd3_t* h, double* rho, double* u, double* B);
/* FP64 reductions of the current state; synchronises.  Returns
 * LBMHD_ERR_NONFINITE (after filling out) when a density is not finite. */
int lbmhd3_diag(lbmhd3_t* h, lbmhd3_diag_t* out);
/* Decode the state into 45 float64 planes (device), or load them (then the
 * step counter is `step`). */
int lbmhd3_get_populations(lbmhd3_t* h, double* out);
int lbmhd3_set_populations(lbmhd3_t* h, const double* in, int64_t step);
/* Text of the last failure on the handle. */
const char* lbmhd3_last_error(const lbmhd3_t* h);

#ifdef __cplusplus
}
#endif

#endif /* LBMHD3_H */
