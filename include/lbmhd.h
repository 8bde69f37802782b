/*
 * lbmhd.h -- C ABI of the MI355X (gfx950) filtered lattice-Boltzmann MHD engine.
 *
 * Method: Flint & Vahala, "A large eddy lattice Boltzmann simulation of
 * magnetohydrodynamic turbulence" (arXiv 1705.09807).  One timestep is the
 * collide-stream operator split of Sec. 2 (kinetic equations LBKinEqn and
 * LBMagEqn): moments, filtered equilibrium moments with the Delta^2/12
 * subgrid closure of Sec. 2.1 / Sec. 3 (density gradients dropped),
 * collision of the D2Q9 scalar f in moment space (FluidTMatrix, MRT rates),
 * SRT collision of the vector distribution g (D2Q5 here), streaming in
 * population space.  Periodic nx x ny lattice, lattice units.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: 0 (LBM_OK) or a negative LBM_E* code.  Nothing throws
 *    across the ABI.  On error, lbm_last_error() returns a message (thread
 *    local) and the context is left unchanged unless stated otherwise.
 *  - Ownership: the caller allocates and frees every device buffer (state,
 *    work, outputs).  The library never allocates or frees device memory.
 *    lbm_ctx is a host object owned by the library, released by lbm_destroy.
 *  - Streams: every call runs on the hipStream_t given to lbm_create and is
 *    asynchronous with respect to the host, except lbm_diagnostics, which
 *    synchronises that stream.
 *  - Device pointers must be 256-byte aligned.
 *  - Natural layout: a field array is [plane][y][x], x fastest, dense
 *    (row pitch nx, plane stride nx*ny).  Populations are ordered
 *    f_0..f_8, g_x0..g_x4, g_y0..g_y4 (19 planes), with the D2Q9
 *    velocities c_x = {0,1,0,-1,0,1,-1,-1,1}, c_y = {0,0,1,0,-1,1,1,-1,-1}
 *    of Sec. 2 (g uses the first five); with mag_lattice = LBM_MAG_D2Q9
 *    f_0..f_8, g_x0..g_x8, g_y0..g_y8 (27 planes, g on all nine).  "State
 *    at time t" means the post-streaming populations the next collision
 *    consumes.
 *  - Threading: a context is used by one host thread at a time.
 */
#ifndef LBMHD_H
#define LBMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)      /* bad parameter, null / misaligned pointer, size */
#define LBM_ESTATE (-2)      /* call out of order (e.g. step before init)      */
#define LBM_EHIP (-3)        /* HIP runtime error; message in lbm_last_error   */
#define LBM_ENONFINITE (-4)  /* diagnostics found NaN/Inf populations          */

/* Storage precision of the populations (arithmetic: FP64 for LBM_FP64, FP32
 * otherwise).  LBM_FP32, LBM_FP16 and LBM_BF16 store deviations from a rest
 * state, f_i - w_i rho0 and g_i - w'_i B_ref (lbm_params rho0, bref_x,
 * bref_y), so the small dynamic part keeps its digits; LBM_FP16 stores them
 * scaled by 2^8 (clear of the FP16 subnormal range); LBM_FP64 stores f_i and
 * g_i themselves (exact state round trips).  All conversions round to
 * nearest even. */
#define LBM_FP64 0
#define LBM_FP32 1
#define LBM_FP16 2
#define LBM_BF16 3

/* Gradients used by the closure.  The LOCAL variants (fused and synchronous
 * in-place schedules) take the strain rate from the non-equilibrium parts of
 * M3 and M4 and grad B from those of the first moments of g (first-order
 * Chapman-Enskog of the pre-collision populations, divergence-free strain),
 * and use the named stencil only for the vorticity D_x m_y - D_y m_x
 * (Sec. 3: not every derivative is available locally on D2Q9). */
#define LBM_STENCIL_ISO9 0      /* (a_E-a_W)/3 + (a_NE+a_SE-a_NW-a_SW)/12 */
#define LBM_STENCIL_CENTRAL5 1  /* (a_E-a_W)/2                             */
#define LBM_STENCIL_LOCAL_ISO9 2
#define LBM_STENCIL_LOCAL_CENTRAL5 3

/* Memory schedule of the timestep. */
#define LBM_SCHED_FUSED 0  /* two population buffers, one fused sweep per step */
#define LBM_SCHED_AA 1     /* one buffer updated in place (AA pattern); with the
                              closure on, a moment sweep precedes the collide sweep */
#define LBM_SCHED_AA_LAGGED 2  /* in place, one sweep per step: the closure
                              differentiates the moments of the previous step
                              (written by the previous sweep into a second set of
                              moment planes) instead of the current ones.  A
                              different result from the synchronous closure: the
                              gradients lag by one step.  The first step after
                              lbm_init_kh_jet, lbm_set_state or
                              lbm_init_from_moments is synchronous, so a run
                              resumed from a saved state is not bit-identical to
                              an uninterrupted one. */

/* Subgrid closure of the LES (Delta > 0). */
#define LBM_CLOSURE_ANALYTIC 0  /* the Delta^2/12 closure of Sec. 2.1 / Sec. 3      */
#define LBM_CLOSURE_LEARNED 1   /* analytic plus a learned per-cell correction
                                   (lbmhd_learned.h); LBM_SCHED_FUSED only        */
#define LBM_CLOSURE_FULL 2      /* the closure before Sec. 3's simplification: the
                                   filtered-density terms of FilterExampleLarge
                                   (Z = rho) kept in the Reynolds and induction
                                   products; LBM_SCHED_FUSED with LBM_STENCIL_ISO9
                                   or LBM_STENCIL_CENTRAL5 only                   */

/* Lattice of the vector distribution g. */
#define LBM_MAG_D2Q5 0  /* the first five D2Q9 velocities, weights (1/3, 1/6 x4)   */
#define LBM_MAG_D2Q9 1  /* all nine (Sec. 2's own choice, MagTMatrix / MagMomentEq;
                           with one rate s_m the moment-space collision equals
                           relaxation of g to the D2Q9 geq); LBM_SCHED_FUSED,
                           LBM_CLOSURE_ANALYTIC or _FULL, a stencil gradient and
                           FP64 or FP32 storage only                              */

typedef struct lbm_ctx lbm_ctx;

/* Run parameters, lattice units.  Rates follow Sec. 2: s3 = s4 = 2/(6 nu + 1)
 * (from nu = 1/(3 s) - 1/6), s_m = 2/(6 eta + 1); s0..s2 = 0 (conserved). */
typedef struct {
  int32_t nx, ny;          /* periodic grid, each >= 4 and <= 32768          */
  double nu, eta;          /* > 0, giving rates in (0, 2)                     */
  double s5, s6, s7, s8;   /* MRT ghost rates in (0, 2); <= 0 means "= s3",
                              i.e. the single-relaxation-time runs of Sec. 3 */
  double delta;            /* filter width Delta >= 0; 0 = unfiltered (DNS)   */
  double closure_scale;    /* multiplies Delta^2/12; 1 = as printed in Sec. 3 */
  int32_t grad_stencil;    /* LBM_STENCIL_*                                   */
  int32_t dtype;           /* LBM_FP64, LBM_FP32, LBM_FP16 or LBM_BF16        */
  int32_t schedule;        /* LBM_SCHED_*                                     */
  int32_t closure;         /* LBM_CLOSURE_*                                   */
  int32_t mag_lattice;     /* LBM_MAG_*                                       */
  int32_t reserved;        /* must be 0                                       */
  double rho0;             /* reference density of the FP32 deviations, > 0   */
  double bref_x, bref_y;   /* reference field of the FP32 g deviations (finite;
                              the run's mean field, e.g. (B0, 0) for the jet) */
} lbm_params;

/* Double-shear-layer Kelvin-Helmholtz jet: u_x = U0 [tanh((y - L/4)/d)
 * - tanh((y - 3L/4)/d) - 1] with L = ny, d = delta_over_L * ny;
 * u_y = pert_amp_over_U0 * U0 * sin(2 pi x / nx) + noise_amp * xi(x, y);
 * B = (B0, 0); rho = rho0.  xi is uniform on [-1, 1): output number
 * (y*nx + x + 1) of SplitMix64 (Steele, Lea & Flood 2014) started at `seed`,
 * top 53 bits scaled by 2^-53, mapped by 2u - 1.  Populations start at the
 * unfiltered equilibria feq / geq of Sec. 2. */
typedef struct {
  double U0, delta_over_L, B0, rho0, pert_amp_over_U0, noise_amp;
  uint64_t seed;
} lbm_kh_params;

/* The magnetized Kelvin-Helmholtz jet of Sec. 4:
 * u_y = U0 sech^2(2 pi k d / nx) + pert U0 sin(2 pi k x / nx), u_x = pert U0 sin(2 pi k y / ny),
 * B_x = pert B0 sin(2 pi k y / ny), B_y = B0 + pert B0 sin(2 pi k x / nx), rho = rho0,
 * with d = min(x, nx - x) (the printed profile sech^2(8 pi x / L) centred on
 * x = 0 of the periodic box) and the mean field along the jet.  The paper:
 * U0 = 4.88e-2, B0 = 0.005 U0, pert = 0.01, k = 4, nu = eta = 1e-3 at 1024^2
 * (Re = U0 L / nu = 50k, scaled with the grid).  Populations start at the
 * unfiltered equilibria feq / geq. */
typedef struct {
  double U0, B0, pert, rho0;
  int32_t k;               /* >= 1 */
  int32_t reserved;        /* must be 0 */
} lbm_sech2_params;

/* Scalar diagnostics, FP64 on the device.  Domain means: e_kin = <|m|^2/(2 rho)>,
 * e_mag = <|B|^2/2>, enstrophy = <w^2/2> with w = D_x u_y - D_y u_x,
 * j2 = <J_z^2> with J_z = D_x B_y - D_y B_x; D = central differences.
 * divb = D_x B_x + D_y B_y as max |.| and rms.  Raw sums of rho, m, B. */
typedef struct {
  int64_t t;
  double mass, mom_x, mom_y, bsum_x, bsum_y;
  double e_kin, e_mag, enstrophy, j2, divb_max, divb_rms;
  int64_t nonfinite;       /* cells with a non-finite population */
} lbm_diag;

/* Bytes of the caller-owned device buffers for these parameters (0 if the
 * parameters are invalid).  The state holds the populations in the storage
 * precision, one buffer (AA) or two (fused, the second starting 4 KB past
 * the 64 KB boundary that follows the first), each ny lattice rows of P
 * population rows (P = 19, or 27 with D2Q9 g) padded to a multiple of 64
 * elements, rounded up to 256 elements: the populations of a lattice row
 * are stored together (an internal layout: state IO uses the natural layout
 * above).  The work buffer holds moment planes and reduction partials (and,
 * with the learned closure, the packed network, a 16-byte input vector per
 * cell and the 4 FP32 correction planes). */
size_t lbm_state_bytes(const lbm_params* p);
size_t lbm_work_bytes(const lbm_params* p);

/* Validate p, derive the rates and bind the buffers and stream.  No device
 * work is enqueued.  state_dev / work_dev: >= lbm_*_bytes(p) bytes, 256-byte
 * aligned, caller owned, alive until lbm_destroy.  hip_stream: a
 * hipStream_t (NULL = the null stream).  The state is uninitialised until
 * lbm_init_kh_jet or lbm_set_state. */
int lbm_create(lbm_ctx** out, const lbm_params* p, void* state_dev, void* work_dev,
               void* hip_stream);

/* Write the Kelvin-Helmholtz initial state (see lbm_kh_params); t = 0. */
int lbm_init_kh_jet(lbm_ctx* ctx, const lbm_kh_params* kh);

/* Write the magnetized jet of Sec. 4 (see lbm_sech2_params); t = 0. */
int lbm_init_sech2_jet(lbm_ctx* ctx, const lbm_sech2_params* jet);

/* Replace the state by the unfiltered equilibria feq / geq (Sec. 2) of given
 * fields: mom_dev = 5 FP64 planes rho (> 0), m_x = rho u_x, m_y, B_x, B_y in
 * natural layout (e.g. filtered and subsampled DNS fields); time := t >= 0. */
int lbm_init_from_moments(lbm_ctx* ctx, const double* mom_dev, int64_t t);

/* Advance n >= 0 timesteps of Sec. 2 / Sec. 3 (collide in moment space,
 * stream).  Gradients of the closure are taken from the moments of the state
 * at the start of each step (synchronous). */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Current time t. */
int lbm_get_time(const lbm_ctx* ctx, int64_t* t_out);

/* Macroscopic fields of the state at time t into out_dev: 5 FP64 planes
 * rho, m_x = rho u_x, m_y, B_x, B_y (natural layout, 5*nx*ny doubles,
 * caller owned).  Sec. 2: rho = sum f_i, rho u = sum c_i f_i, B = sum g_i. */
int lbm_moments(lbm_ctx* ctx, double* out_dev);

/* Copy the populations of the state at time t to out_dev as P FP64 planes
 * in natural layout (P*nx*ny doubles, caller owned), P = 19 (D2Q5 g) or 27
 * (D2Q9 g). */
int lbm_get_state(lbm_ctx* ctx, double* out_dev);

/* Replace the state by P (19 or 27) FP64 planes in natural layout (rounded
 * to the storage precision) and set the time to t >= 0. */
int lbm_set_state(lbm_ctx* ctx, const double* in_dev, int64_t t);

/* Compute the diagnostics of the state at time t into *out_host (host
 * memory); synchronises the stream.  Returns LBM_ENONFINITE, with *out_host
 * filled, when a population is NaN or infinite. */
int lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out_host);

/* Release the context (not the caller's buffers).  NULL is accepted. */
int lbm_destroy(lbm_ctx* ctx);

/* Static description of an error code; the calling thread's last error. */
const char* lbm_strerror(int code);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMHD_H */
