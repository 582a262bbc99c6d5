/*
 * lbmhd.h -- C ABI of the MI355X (gfx950) lattice Boltzmann MHD library.
 *
 * The library advances the 2D lattice Boltzmann MHD model of Flint & Vahala,
 * "Lattice Boltzmann Large Eddy Simulation Model of MHD" (arXiv:1607.08675):
 * a D2Q9 density distribution f relaxed by a multi-relaxation-time collision
 * in the moment basis T of Sec. 3 (eq. FluidTMatrix), and a D2Q5 vector
 * distribution g for the magnetic field relaxed by a single rate s_m
 * (Sec. 3, eq. MagTMatrix), on a doubly periodic nx x ny lattice, with unit
 * time step and the collide/stream split of Sec. 1.2 and Sec. 3.  Optionally
 * the relaxation times carry the Smagorinsky-MHD eddy viscosity and eddy
 * resistivity (Sec. 1.1, eqs. SmagorinskyClosure, SmagorinskyMHDClosureV/B),
 * computed per site from the site's own non-equilibrium moments; the paper's
 * kinetic closure (Sec. 4.1, filtered equilibria) and the cross-helicity
 * closure (eqs. CHClosureV/B) are selected the same way (lbmhd_params.les).
 * The library also runs the update in place on one lattice, and provides its
 * discrete adjoint (reverse step, seeds, pull-back to the initial fields) for
 * the gradients of a final-time functional.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All functions return an int status: LBMHD_OK (0) or a negative
 *    LBMHD_ERR_* code.  No C++ exception crosses this interface.  The text of
 *    the last failure on a handle is available from lbmhd_last_error().
 *  - "device" pointers are HIP device memory owned by the caller (for example
 *    torch tensors); the library never frees caller memory and never
 *    allocates device memory after lbmhd_bind().
 *  - Field arrays ("fields") are float64, nx*ny elements, row-major [y][x]
 *    with x fastest and no padding.  Site (x, y) sits at x_i = 2 pi x / nx,
 *    y_j = 2 pi y / ny of the periodic box.
 *  - Population arrays ("populations") are float64, 19 planes of nx*ny in the
 *    same [y][x] order: planes 0..8 = f_0..f_8 with the D2Q9 velocities
 *    c_x = {0,1,0,-1,0,1,-1,-1,1}, c_y = {0,0,1,0,-1,1,1,-1,-1}; planes 9..13
 *    = x component of g_0..g_4 and 14..18 = y component, with the D2Q5
 *    velocities C_x = {0,1,0,-1,0}, C_y = {0,0,1,0,-1} (Sec. 3).
 *  - The state after n steps is the post-collision population at time n:
 *    each step gathers (streams) from the neighbours and then collides at the
 *    site.  Its density, momentum and B equal those of the pre-collision
 *    population at time n of the paper's collide-then-stream ordering, since
 *    the collision conserves them (Sec. 3, collision invariants).
 *  - All work is enqueued on the stream given to lbmhd_bind(); functions
 *    documented as "asynchronous" return before the GPU finishes.
 *  - A handle is not thread-safe; use one handle per stream.
 */
#ifndef LBMHD_H
#define LBMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBMHD_OK = 0,
  LBMHD_ERR_INVALID_ARG = -1, /* bad parameter, null or undersized buffer */
  LBMHD_ERR_NOT_BOUND = -2,   /* lbmhd_bind() has not succeeded yet */
  LBMHD_ERR_HIP = -3,         /* a HIP runtime call failed (text kept) */
  LBMHD_ERR_NONFINITE = -4,   /* lbmhd_diag() found NaN/Inf populations */
  LBMHD_ERR_UNSUPPORTED = -5  /* valid request the library does not offer */
};

/* Population storage in HBM.  Both store the deviation of each population
 * from its value in the rest state (f_i - w_i with the D2Q9 weights
 * w = 4/9, 1/9, 1/36; g unchanged since the rest state has B = 0).  FP16
 * stores round-to-nearest-even half(deviation * 2^10).  Collision arithmetic
 * is FP32 in both cases. */
enum { LBMHD_FP32 = 0, LBMHD_FP16 = 1 };

typedef struct lbmhd lbmhd_t;

typedef struct {
  int32_t nx, ny;         /* periodic lattice, each >= 2 */
  double nu, eta;         /* shear viscosity and resistivity in lattice
                             units, > 0; tau0 = 3 nu + 1/2 = 1/s_3 = 1/s_4 and
                             tau_m0 = 3 eta + 1/2 = 1/s_m (Sec. 4.3) */
  double s5, s6, s7, s8;  /* rates of the non-hydrodynamic moments M5..M8
                             (Sec. 3), each in (0, 2); s5 must equal s6 */
  int32_t les;            /* bit mask: 0, 1, 2, 3, 4 or 6.
                             0: rates fixed, plain equilibria;
                             bit 0 (1): Smagorinsky-MHD closure (Sec. 1.1):
                                per-site relaxation times from the site's own
                                non-equilibrium moments;
                             bit 1 (2): kinetic closure (Sec. 4.1): relaxation
                                toward the filtered equilibrium moments
                                M^eq + Delta^2 M^(Delta) of the filter-width
                                expansions (eqs. FilterExampleSmall,
                                FilterExampleLarge, DeltaEqEx), with gradients
                                of the neighbours' rho, j, B by the isotropic
                                D2Q9 difference 3 sum_i w_i c_i X(x + c_i);
                             3: both, the Smagorinsky estimate of |S| and |j|
                                then measured from the filtered equilibria;
                             bit 2 (4): cross-helicity closure (eqs.
                                CHClosureV/B): nu_t = C_S Delta^2 |S^v:S^b|^(1/2),
                                eta_t = C_S Delta^2 sgn(j.w) |j.w|^(1/2) with
                                backscatter (eta_t < 0) clipped where
                                eta + eta_t would be negative (tau_m = 1/2);
                                S^v, S^b, j from the site's non-equilibrium
                                moments, the vorticity w from the neighbours;
                                self-consistent tau, tau_m (cubic roots);
                             6: kinetic and cross-helicity closures together.
                             Bits 0 and 2 exclude each other.  Bit 2 needs
                             tau_m0 <= 5/4 (eta <= 1/4): as tau_m0 nears 3/2
                             the clip of tau_m nears a double root of its
                             cubic, where the kernel's Newton solution
                             converges only linearly. */
  double cs, cs_b;        /* closure constants C_Sv >= 0 of the eddy viscosity
                             and C_Sb >= 0 of the eddy resistivity (eqs.
                             SmagorinskyMHDClosureV/B, CHClosureV/B) */
  double delta;           /* filter width Delta > 0 in lattice units */
  int32_t storage;        /* LBMHD_FP32 or LBMHD_FP16 */
  int32_t inplace;        /* 0: two lattices, each step writes the other one;
                             1: one lattice updated in place (AA pattern: the
                             steps alternate between a pull-gather /
                             push-scatter step into reversed slots and a fully
                             local step back, the same bytes per step as the
                             two-lattice update).  Not with les = 2, 3, 4, 6
                             (those read the neighbours' populations).  Calls
                             that read the state, or take a state argument
                             that is the bound lattice itself, first return
                             a reversed lattice to the natural layout. */
  int32_t steps_per_pass; /* How many steps lbmhd_step takes per pass over
                             the lattice when two lattices are bound, the
                             intermediate states staying on chip.  Closures
                             that read no neighbours (les = 0 or 1): 0
                             (automatic) takes triples of steps with FP32
                             storage and pairs with FP16 when the lattice is
                             large enough for that to pay (at least 512 tiles
                             of 8 rows by 256 FP32 or 512 FP16 columns, e.g.
                             1024^2 FP32, 2048^2 FP16); 3 always takes
                             triples with FP32 (pairs with FP16); 2 always
                             takes pairs.  Closures that read the neighbours'
                             moments (les = 2, 3, 4, 6): 0 takes pairs with
                             FP32 storage from 512 tiles of 8 rows by 256
                             columns on (else single steps), 2 and 3 always
                             take pairs.  1 takes single steps.  After the
                             triples a remainder of two steps is one pair and
                             of one a single step; after pairs a single step
                             runs only when one is left.  Other values
                             are rejected.  The
                             result is bit for bit that of single steps, in
                             FP32 and FP16 storage (every kernel rounds the
                             collision and the gradient terms identically:
                             their fused multiply-adds are spelled out and
                             no other contraction is allowed). */
} lbmhd_params;

/* Global diagnostics of the current state, accumulated in FP64.
 * Differences are centred: d_x a = (a(x+1) - a(x-1)) / 2, periodic. */
typedef struct {
  double mass;            /* sum rho */
  double mom_x, mom_y;    /* sum rho u */
  double flux_x, flux_y;  /* sum B */
  double e_kin;           /* sum |rho u|^2 / (2 rho) */
  double e_mag;           /* sum |B|^2 / 2 */
  double cross_helicity;  /* sum u . B */
  double max_abs_divB;    /* max |d_x B_x + d_y B_y| */
  double enstrophy;       /* sum w^2 / 2, w = d_x u_y - d_y u_x */
  double current_sq;      /* sum j^2 / 2, j = d_x B_y - d_y B_x */
  double max_u;           /* max |u| */
  int64_t nonfinite;      /* sites holding a NaN or Inf population */
  int64_t step;           /* steps taken since the last (re)initialisation */
} lbmhd_diag_t;

/* Text for a status code.  Never NULL; static storage. */
const char* lbmhd_strerror(int code);

/* Text of the most recent failure on h ("" if none).  Owned by h; valid
 * until the next call on h. */
const char* lbmhd_last_error(const lbmhd_t* h);

/* Validate p and create a host-side handle.  Allocates no device memory.
 * Errors: LBMHD_ERR_INVALID_ARG if p is out of range (nx, ny < 2; nu, eta
 * <= 0; a rate outside (0, 2); s5 != s6; cs < 0; delta <= 0; unknown
 * storage; one FP32 plane of ny rows of padded nx reaching 4 GiB, since
 * in-plane byte offsets are 32-bit); LBMHD_ERR_UNSUPPORTED for the
 * cross-helicity closure (les bit 2) with eta > 1/4. */
int lbmhd_create(const lbmhd_params* p, lbmhd_t** out);

/* Release the handle (not the caller's buffers).  NULL is accepted. */
int lbmhd_destroy(lbmhd_t* h);

/* Byte sizes the caller must allocate in device memory:
 *   lattice    -- one encoded population lattice (two are bound, one in place);
 *   workspace  -- scratch used by diagnostics, energy and reductions (block
 *                 partials and results, the same at any lattice size);
 *   adj_lattice -- one FP32 adjoint lattice (lambda), for the adjoint calls;
 *   adj_acc    -- the FP64 accumulator array of lbmhd_adj_step.
 * Any output pointer may be NULL. */
int lbmhd_sizes(const lbmhd_t* h, size_t* lattice, size_t* workspace, size_t* adj_lattice,
                size_t* adj_acc);

/* Layout of an encoded lattice and of an adjoint lattice, in elements (FP32
 * or FP16 as `storage` selects for a state, FP32 for an adjoint lattice):
 * population q of site (x, y) is element q * plane + y * pitch + x of a
 * state, and q * adj_plane + y * adj_pitch + x of an adjoint lattice.  Rows
 * are padded to whole 256-byte blocks, and successive planes are spaced by
 * their ny rows plus a gap of 768 bytes, so that the 19 populations of a site
 * are not a large power of two apart (the kernels moving a row of every
 * plane at once run faster); the row padding and the gaps are never read or
 * written.  lattice = 19 * plane * element size, adj_lattice = 19 *
 * adj_plane * 4.  Any output pointer may be NULL.  Errors:
 * LBMHD_ERR_INVALID_ARG (h NULL). */
int lbmhd_layout(const lbmhd_t* h, int64_t* pitch, int64_t* plane, int64_t* adj_pitch,
                 int64_t* adj_plane);

/* Attach caller-owned device buffers and the HIP stream (a hipStream_t, or
 * NULL for the null stream).  lat_a and lat_b must each hold `lattice`
 * bytes and workspace `workspace` bytes (lbmhd_sizes), 256-byte aligned, and
 * must not overlap; with inplace = 1 only lat_a is used (lat_b may be NULL).
 * The stored sizes are checked against the requirement.
 * Does not initialise the state.  Errors: LBMHD_ERR_INVALID_ARG. */
int lbmhd_bind(lbmhd_t* h, void* lat_a, size_t lat_a_bytes, void* lat_b, size_t lat_b_bytes,
               void* workspace, size_t workspace_bytes, void* stream);

/* Set every site to the equilibria f^eq(rho, u, B) and g^eq(u, B) of Sec. 3
 * (the D2Q9 and D2Q5 relaxation distributions) computed in FP64, then encode
 * to storage.  rho, ux, uy, bx, by: device fields.  Resets the step count to
 * 0.  Asynchronous.  Errors: LBMHD_ERR_NOT_BOUND, LBMHD_ERR_INVALID_ARG,
 * LBMHD_ERR_HIP. */
int lbmhd_init_fields(lbmhd_t* h, const double* rho, const double* ux, const double* uy,
                      const double* bx, const double* by);

/* Advance nsteps >= 0 steps of stream + collide (Sec. 1.2 update with the
 * moment-space collision of Sec. 3; closures as selected by les), ping-ponging
 * the two bound lattices (or updating the one lattice in place).  Each kernel
 * launch fuses streaming and collision of one, two or three steps as
 * steps_per_pass selects (the same result, bit for bit).  Asynchronous. */
int lbmhd_step(lbmhd_t* h, int64_t nsteps);

/* Steps that one pass over the lattice covers when lbmhd_step advances a
 * multiple of that many steps on this handle: 3 or 2 where steps_per_pass
 * (and, for 0, the lattice size) selects the three- or two-step kernel for
 * this storage, closure and layout, else 1.  Host only.  Errors:
 * LBMHD_ERR_INVALID_ARG for NULL arguments. */
int lbmhd_steps_per_pass(const lbmhd_t* h, int32_t* out);

/* One step from the encoded lattice src into dst (device, `lattice` bytes
 * each, 256-byte aligned; dst overlaps neither src nor the bound buffers, src
 * may be a bound lattice), same update as lbmhd_step.  Leaves the handle's
 * current state and step count untouched; used to recompute stored states
 * for the adjoint.  Asynchronous. */
int lbmhd_step_between(lbmhd_t* h, const void* src, void* dst);

/* n >= 0 steps from the encoded lattice src, keeping every state: state t
 * (t = 1 .. n) is written to store + (t - 1) * stride bytes (device; stride a
 * multiple of 256 and >= `lattice` bytes).  The same update as lbmhd_step,
 * launched from the library in one call: where lbmhd_step takes several
 * steps per pass, consecutive steps go in triples (FP32) or pairs here (with
 * FP16 storage only when steps_per_pass is 2 or more), a pass that reads
 * state t - 1 once and writes all the states it computes (four lattice
 * transfers for three steps, three for two, instead of two per step).  The handle's current state and step count are untouched.  The
 * store range overlaps neither src nor the bound buffers.  Used to keep the
 * whole trajectory for the adjoint when it fits in device memory.
 * Asynchronous. */
int lbmhd_step_store(lbmhd_t* h, const void* src, void* store, size_t stride, int64_t n);

/* npairs >= 0 pairs of steps from the encoded lattice src, keeping every
 * other state: state 2k (k = 1 .. npairs) is written to store + (k - 1) *
 * stride bytes (device; stride a multiple of 256 and >= `lattice` bytes), the
 * odd states are never written.  Each pair is one pass over the lattice (the
 * two-step kernels of lbmhd_step), so the result equals 2 npairs single
 * steps bit for bit.  The handle's current state and step count are
 * untouched; the store range overlaps neither src nor the bound buffers.
 * Used to recompute a checkpoint segment for lbmhd_adj_sweep_pairs, which
 * needs only these states.  Asynchronous.  Errors as lbmhd_step_store. */
int lbmhd_step_store_pairs(lbmhd_t* h, const void* src, void* store, size_t stride,
                           int64_t npairs);

/* Macroscopic fields of the current state: rho = sum f, u = (sum c f) / rho,
 * B = sum g (Sec. 3).  Outputs: device fields.  Asynchronous. */
int lbmhd_macro(lbmhd_t* h, double* rho, double* ux, double* uy, double* bx, double* by);

/* Box-filtered macroscopic fields of the current state: rho, u, B of each
 * site (as lbmhd_macro) averaged over w x w blocks of sites (a width-w box
 * filter sampled on the coarse grid; w >= 1 must divide nx and ny).  Outputs:
 * device fields of (nx / w) x (ny / w), row-major.  Asynchronous. */
int lbmhd_macro_box(lbmhd_t* h, int32_t w, double* rho, double* ux, double* uy, double* bx,
                    double* by);

/* L2 mismatch L = sum_x |u - u_t|^2 + |B - B_t|^2 of the encoded lattice
 * `state` (device, `lattice` bytes; NULL = current state) against target
 * fields u_t, B_t (device fields, nx*ny), accumulated in FP64 and written to
 * *L (host).  Synchronises the bound stream. */
int lbmhd_mismatch(lbmhd_t* h, const void* state, const double* ux_t, const double* uy_t,
                   const double* bx_t, const double* by_t, double* L);

/* FP64 global diagnostics of the current state into *out (host memory).
 * Synchronises the bound stream.  Returns LBMHD_ERR_NONFINITE (with *out
 * filled) when any population is NaN or Inf. */
int lbmhd_diag(lbmhd_t* h, lbmhd_diag_t* out);

/* nsteps >= 0 steps of the update (Sec. 3), as lbmhd_step, with the
 * diagnostics of lbmhd_diag taken after steps every, 2 every, ... (those
 * <= nsteps) and no wait on the host between them.  With two bound lattices
 * each diagnostics pass runs on a second stream of the handle (one HIP stream
 * and two events, created at the first such call, no device memory): it
 * starts after the bound stream's work so far and overlaps the next kernel
 * pass, which only reads that state; a pass that would overwrite a state still
 * being read waits for it on the bound stream.  Where lbmhd_step would end an
 * interval with a single step (FP32 storage, les = 0 or 1: e.g. intervals of
 * 3k + 1 steps taken in triples), that step and the diagnostics of its result
 * are one pass on the bound stream instead.  An in-place lattice takes its
 * diagnostics on the bound stream.  The reductions' block partials use the
 * bound workspace.
 *   dev   -- device memory, 8-byte aligned, of at least nout * 16 doubles,
 *            overlapping no bound buffer; diagnostics k is left in doubles
 *            16k .. 16k + 12 in the order mass, mom_x, mom_y, flux_x,
 *            flux_y, e_kin, e_mag, cross_helicity, enstrophy, current_sq,
 *            nonfinite, max_abs_divB, max_u, the rest unspecified;
 *   out   -- host array of nout >= nsteps / every results, with step set.
 * Results equal those of lbmhd_diag at the same steps bit for bit (the same
 * kernels and reduction order).  When at least one diagnostics pass is taken,
 * the call synchronises the bound stream once, at the end, and returns
 * LBMHD_ERR_NONFINITE (every result filled) when any pass found NaN or Inf
 * populations; with every = 0 or nsteps < every it is lbmhd_step (dev and out
 * unused, asynchronous).  Errors: LBMHD_ERR_INVALID_ARG for negative nsteps or
 * every, NULL or undersized dev / out, or dev unaligned or overlapping a bound
 * buffer; LBMHD_ERR_NOT_BOUND, LBMHD_ERR_HIP.  Calls on one handle from
 * several threads race. */
int lbmhd_run(lbmhd_t* h, int64_t nsteps, int64_t every, double* dev, lbmhd_diag_t* out,
              int64_t nout);

/* Decode the current state to plain populations (device, 19*nx*ny float64):
 * f_i = w_i + deviation.  Asynchronous. */
int lbmhd_get_populations(lbmhd_t* h, double* out);

/* Encode plain populations (device, 19*nx*ny float64) as the current state
 * and set the step count.  The deviation from the rest state is formed in
 * FP64 and rounded to FP32 (then, for FP16 storage, to half of 2^10 times
 * it).  Asynchronous. */
int lbmhd_set_populations(lbmhd_t* h, const double* in, int64_t step);

/* Copy the current encoded lattice (`lattice` bytes) to / from caller device
 * memory, bit-exact; used for checkpoints.  load sets the step count.  src may
 * be the state buffer the handle reports (lbmhd_current_state), also of an
 * in-place lattice left in the reversed layout, which load turns back first;
 * a src that partly overlaps the first bound lattice is refused
 * (LBMHD_ERR_INVALID_ARG).  Asynchronous. */
int lbmhd_save_state(lbmhd_t* h, void* dst);
int lbmhd_load_state(lbmhd_t* h, const void* src, int64_t step);

/* Steps taken since the last (re)initialisation (host value). */
int lbmhd_get_step(const lbmhd_t* h, int64_t* step);

/* Device address of the bound lattice that holds the current state (which of
 * the two lattices depends on how many kernel passes the steps took; the one
 * lattice in place, whose layout is reversed after an odd step count until a
 * call that reads the state restores it).  For reading the state in place
 * without a copy; the library owns what it writes there.  Host only.
 * Errors: LBMHD_ERR_NOT_BOUND, LBMHD_ERR_INVALID_ARG for NULL arguments. */
int lbmhd_current_state(const lbmhd_t* h, const void** out);

/* Total energy J = sum (|rho u|^2 / (2 rho) + |B|^2 / 2) of an encoded
 * lattice `state` (device, `lattice` bytes; NULL = current state), in FP64,
 * written to *J (host).  Synchronises the bound stream. */
int lbmhd_energy(lbmhd_t* h, const void* state, double* J);

/* ---------------------------------------------------------------------
 * Adjoint (reverse mode) of the step.  The step maps an encoded lattice x_n
 * to x_{n+1} = C(S(x_n)) (S: periodic gather, C: per-site collision with
 * the closure).  Adjoint lattices are FP32, adj_lattice bytes, 19 planes in
 * the same padded layout as an FP32 state; they hold dJ/d(population) in
 * streamed position: plane i at site x + c_i (periodic; the D2Q5 planes of
 * vector k at x + C_k) holds dJ/dx_i(x), the sensitivity to population i of
 * site x kept where that population arrives in the next streaming.  With
 * this placement the reverse step gathers and stores aligned.  Storage
 * rounding is treated as the identity (its derivative is zero almost
 * everywhere).
 * ------------------------------------------------------------------- */

/* lam = dJ/dx (streamed position) for the total energy J of `state` (see
 * lbmhd_energy): dJ/df_i = c_i . u - |u|^2 / 2, dJ/dg_k = B.  Asynchronous. */
int lbmhd_adj_seed_energy(lbmhd_t* h, const void* state, float* lam);

/* lam = scale * dL/dx (streamed position) for the mismatch L of lbmhd_mismatch evaluated on
 * `state`: dL/df_i = 2 (u - u_t) . (c_i - u) / rho, dL/dg_k = 2 (B - B_t).
 * Asynchronous. */
int lbmhd_adj_seed_mismatch(lbmhd_t* h, const void* state, const double* ux_t,
                            const double* uy_t, const double* bx_t, const double* by_t,
                            double scale, float* lam);

/* The adjoint calls below cover les = 0, 1, 2 and 3.  With the kinetic
 * closure (les = 2, 3) the equilibrium terms depend on the neighbours'
 * moments, whose adjoints go back through the transposed gradient stencil;
 * one pass over strips of rows keeps those adjoints on chip.  With
 * the cross-helicity closure (les = 4, 6) lbmhd_adj_step and lbmhd_adj_sweep
 * return LBMHD_ERR_UNSUPPORTED. */

/* One reverse step: lam_prev = (dx_{n+1}/dx_n)^T lam_next (both in streamed
 * position), where state_n is the encoded lattice x_n (device, `lattice` bytes).  acc (device, adj_acc
 * bytes, FP64) holds two arrays of slots, one slot per thread block in each:
 * the first gains lam_next . d x_{n+1} / d C_Sv, the second
 * lam_next . d x_{n+1} / d C_Sb.  Slots are only ever added to, so zero acc
 * once before a backward sweep.  lam_prev must not alias lam_next.
 * Asynchronous. */
int lbmhd_adj_step(lbmhd_t* h, const void* state_n, const float* lam_next, float* lam_prev,
                   double* acc);

/* Reverse sweep over n >= 0 steps in one call: with x_0 = src and x_t at
 * store + (t - 1) * stride for t = 1 .. n - 1 (the layout lbmhd_step_store
 * writes), and lam holding lam_n (streamed position) on entry, apply
 * lbmhd_adj_step for t = n - 1 down to 0 and leave lam_0 in lam.  tmp is a
 * second adjoint lattice used as scratch (not overlapping lam); acc gains the
 * closure-constant sums as in lbmhd_adj_step.  Without neighbour terms
 * (les = 0, 1) and from 512 tiles of 8 rows by 256 columns on, the steps go
 * in pairs as in lbmhd_adj_sweep_pairs (the same lam_0 bit for bit, reading
 * the even states only).  Asynchronous.  Errors as lbmhd_adj_step. */
int lbmhd_adj_sweep(lbmhd_t* h, const void* src, const void* store, size_t stride, int64_t n,
                    float* lam, float* tmp, double* acc);

/* Two reverse steps in one pass over the lattice: lam_prev = (dx_{t+2} /
 * dx_t)^T lam_next from the encoded state_t = x_t alone; x_{t+1} =
 * C(S(x_t)) is recomputed on the device with the collision lbmhd_step
 * applies, so lam_prev equals lbmhd_adj_step(x_{t+1}, lam_next, tmp)
 * followed by lbmhd_adj_step(x_t, tmp, lam_prev) bit for bit, and acc gains
 * the same closure-constant sums up to the order of their additions.
 * Closures without neighbour terms (les = 0, 1); LBMHD_ERR_UNSUPPORTED for
 * les = 2, 3, 4, 6.  Other errors as lbmhd_adj_step.  Asynchronous. */
int lbmhd_adj_step2(lbmhd_t* h, const void* state_t, const float* lam_next, float* lam_prev,
                    double* acc);

/* Reverse sweep over n >= 0 steps of a trajectory kept every other state
 * (the layout lbmhd_step_store_pairs writes): x_0 = src and x_t at store +
 * (t / 2 - 1) * stride for the even t = 2 .. n - 1.  The reverse steps go in
 * pairs (lbmhd_adj_step2 from x_t for t = n - 2, n - 4, ...), after a single
 * lbmhd_adj_step from x_{n-1} first when n is odd; lam holds lam_n on entry
 * and lam_0 on return, tmp is scratch, acc gains the closure-constant sums.
 * Errors as lbmhd_adj_step2.  Asynchronous. */
int lbmhd_adj_sweep_pairs(lbmhd_t* h, const void* src, const void* store, size_t stride,
                          int64_t n, float* lam, float* tmp, double* acc);

/* Sum the two slot arrays of acc into out[0] (C_Sv) and out[1] (C_Sb), host,
 * in FP64.  Synchronises. */
int lbmhd_adj_acc_total(lbmhd_t* h, const double* acc, double* out);

/* Pull an adjoint lattice (streamed position) back through the initial equilibria: with
 * x_0 = encode(f^eq(rho0, u0, B0), g^eq(u0, B0)), write
 * dJ/du_x, dJ/du_y, dJ/dB_x, dJ/dB_y (device fields) from lam0 and the
 * initial fields (device fields).  Asynchronous. */
int lbmhd_adj_fields(lbmhd_t* h, const float* lam0, const double* rho0, const double* ux0,
                     const double* uy0, const double* bx0, const double* by0, double* g_ux,
                     double* g_uy, double* g_bx, double* g_by);

/* lbmhd_diag without the bound workspace, for callers that cannot allocate
 * device memory at the point of the call (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same kernels, same
 * results, same return codes and synchronisation as lbmhd_diag; the
 * reductions' block partials and result slots live instead in a static
 * device array of the library, 524,416 bytes on each GPU it runs on, held
 * until the process ends (at most 4096 partials of 16 doubles plus 16
 * result doubles, which every lattice size fits: the reducing blocks stride
 * over the lattice).  Its device address is looked up once per GPU, for the
 * device of the bound stream.  Calls on one GPU share that array: calls
 * that overlap in time on one GPU (on different streams or threads) race
 * and must be ordered by the caller.  Allocates nothing. */
int lbmhd_diag_noalloc(lbmhd_t* h, lbmhd_diag_t* out);

#ifdef __cplusplus
}
#endif

#endif /* LBMHD_H */
