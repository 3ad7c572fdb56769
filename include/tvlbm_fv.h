/*
 * tvlbm_fv.h -- C ABI of the finite-volume TVLBM update on one MI355X.
 *
 * The paper's own discretisation (Sbragaglia & Sugiyama, arXiv 1004.5059):
 * explicit Euler in time of df_l/dt = Omega_l - c_l . grad f_l, eq.(FVLB),
 * on a rectangular mesh, uniform in x (spacing dx) with spacings dy_j in y
 * (Sec. III), with
 *   - the second-order 9-point stencils of Sec. III for c . grad f and for
 *     the collision term Omega_l = -(f_l - feq_l)/tau;
 *   - optional diffuse-scattering wall points at the first and last mesh
 *     row: incoming populations (c.n <= 0, n the inward normal) advance
 *     with the one-sided stencils of Sec. VII, eq.(FVLB2); outgoing ones
 *     are re-emitted with the flux-weighted wall Maxwellian,
 *     eq.(IMPOSITION), from the new incoming normal flux;
 *   - the Hermite equilibrium of Sec. II / Appendix A on the same
 *     tensor-product Gauss-Hermite sets as include/tvlbm.h (c_l = xi_l).
 * Periodic in x or with zero-gradient ends; periodic in y or walled.
 *
 * Conventions as in include/tvlbm.h: return TVLBM_OK or a negative
 * TVLBM_E* code, TVLBM_F32 / TVLBM_F64, device buffers caller-owned,
 * populations [q][ny][ld] as deviations from the rest weights internally
 * (the public outputs are f itself), work on the given stream.
 */
#ifndef TVLBM_FV_H
#define TVLBM_FV_H

#include <stdint.h>

#include "tvlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tvlbm_fv tvlbm_fv;

typedef struct tvlbm_fv_desc {
  int32_t n_gh;        /* Gauss-Hermite points per axis: 3, 4 or 6          */
  int32_t eq_order;    /* 2, 3 or 4 (with n_gh 3, 4, 6), or 5 with n_gh 6   */
                       /* (Appendix A's fifth order; the 6-point rule      */
                       /* integrates its moments exactly)                  */
  int32_t dtype;       /* TVLBM_F32 | TVLBM_F64                             */
  int32_t compensated; /* FP32: compensated moment sums (1) or plain (0)    */
  int32_t nx, ny;      /* mesh points; walls need ny >= 3                   */
  int64_t ld;          /* row pitch in elements (>= nx), 0 = round up to 64 */
  double dx;           /* x spacing                                         */
  double dt;           /* time step                                         */
  double tau;          /* relaxation time (time units), > 0 if collide      */
  int32_t collide;     /* 0: no collision term                              */
  int32_t y_bc;        /* TVLBM_BC_PERIODIC | TVLBM_BC_DIFFUSE_WALLS        */
  double wall_lo_ux, wall_lo_T; /* wall at the first row: x velocity, T      */
  double wall_hi_ux, wall_hi_T; /* wall at the last row                      */
  const double *dy;    /* host: spacing after each mesh row, ny entries     */
                       /* (periodic; the last closes the period) or ny-1    */
                       /* (walls); NULL = all dx                            */
  void *f_a, *f_b;     /* device, q*ny*ld elements of dtype each            */
  void *omega;         /* device scratch for Omega, q*ny*ld elements        */
  void *stream;        /* hipStream_t or NULL                               */
} tvlbm_fv_desc;

/* EINVAL on bad sizes, spacings, dt, tau, pitch or null/shared buffers;
 * EUNSUPPORTED for other lattices or population blocks of 4 GiB or more. */
int tvlbm_fv_init(const tvlbm_fv_desc *desc, tvlbm_fv **fv);
int tvlbm_fv_destroy(tvlbm_fv *fv);
/* f = feq(rho, u, T) + noise (Sec. II; device [ny][nx] fields of dtype,
 * noise [q][ny][nx] or NULL), then eq.(IMPOSITION) at the walls */
int tvlbm_fv_set_fields(tvlbm_fv *fv, const void *rho, const void *ux, const void *uy,
                        const void *T, const void *noise);
/* nsteps steps of length dt (asynchronous) */
int tvlbm_fv_step(tvlbm_fv *fv, int32_t nsteps);
/* f at every mesh point, device [q][ny][nx] */
int tvlbm_fv_populations(tvlbm_fv *fv, void *out);
/* fields (device [ny][nx] each, any may be NULL) and FP64 totals (host,
 * may be NULL): mass, x/y momentum, energy summed with weights
 * dx * (dy_{j-1} + dy_j)/2 (half cells at walls).  Synchronises. */
int tvlbm_fv_moments(tvlbm_fv *fv, void *rho, void *ux, void *uy, void *T, double *totals);
int tvlbm_fv_step_count(const tvlbm_fv *fv, int64_t *k);

/* How a step runs on the GPU.  fused = 1 (the default): one pass that reads
 * the populations once and writes them once; each wavefront marches down
 * seg_rows rows of a 62-column strip, the 9-point stencils of Sec. III and
 * Sec. VII evaluated in their separable (1-D x 1-D) form.  fused = 0: two
 * passes, Omega of every point into the omega scratch array, then the
 * stencil update.  fused = 2 (FP32 with n_gh 3 or 4 only, else
 * EUNSUPPORTED): one pass with the four wavefronts of a workgroup sharing
 * a segment of seg_rows rows (rows interleaved, neighbour contributions
 * exchanged through LDS), for longer segments at the same parallelism.
 * All compute the same update; they differ by rounding only (the fused
 * passes sum the stencil terms in another order).
 * seg_rows: 1 .. 65536 rows per wavefront (0 keeps the current value,
 * default 6); prefetch: 1 loads row r+1 while row r is processed (default 0).
 * EINVAL on a null handle or argument, or values out of range. */
typedef struct tvlbm_fv_schedule {
  int32_t fused;
  int32_t seg_rows;
  int32_t prefetch;
} tvlbm_fv_schedule;
int tvlbm_fv_set_schedule(tvlbm_fv *fv, const tvlbm_fv_schedule *s);

/* Non-unit Prandtl number, eq.(FINAL) / eq.(OMEGAFVLB), and the
 * pressure-rescaled relaxation times of Sec. IX.  tau_g > 0 (finite) adds
 * to the collision term
 *   -(1/tau_g) feq_l / (rho T^2) Pi : (c_l - u)(c_l - u),
 *   Pi_ij = sum_l (f_l - feq_l)(c_l - u)_i (c_l - u)_j,
 * which gives the viscosity eta = c_v rho T tau tau_g / (2 tau + tau_g)
 * (c_v = D/2) and leaves the conductivity c_P rho T tau, i.e. Prandtl
 * number c_v tau_g / (2 tau + tau_g) in two dimensions.  The sign is the one
 * that makes this viscosity hold: the printed plus sign would let Pi grow
 * for tau_g < 2 tau.  tau_g <= 0 or infinite: single relaxation (default).
 * pressure_scaled = 1: tau -> tau / p and tau_g -> tau_g / p with the local
 * p = rho T.  No effect without collisions.  Applies to later steps.
 * EINVAL on a null handle, NaN or a flag other than 0 / 1. */
int tvlbm_fv_set_prandtl(tvlbm_fv *fv, double tau_g, int32_t pressure_scaled);

/* Wall model of the wall rows (no effect when periodic in y).
 * TVLBM_FV_WALL_DIFFUSE (default): eq.(IMPOSITION) with the fixed wall
 *   equilibrium (wall_*_ux, wall_*_T of the descriptor); the flow slips and
 *   the temperature jumps at the wall by amounts of order tau.
 * TVLBM_FV_WALL_SLIP_FREE: Sec. IX / Appendix B: at every wall point and
 *   step the wall equilibrium (u_eq, T_eq) is solved for, so that after the
 *   flux-weighted re-emission the point's own x velocity and temperature
 *   are the descriptor's wall values.  Newton's method on Appendix B's two
 *   conditions (its derivatives plus the change of the point's density with
 *   the emitted populations, which the printed ones leave out), in FP64:
 *   6 iterations from the wall values after set_fields or a change
 *   of model, then 3 from each point's root of the previous step, kept on the
 *   device); one extra launch per step.
 * Applies to later steps and to tvlbm_fv_set_fields.  EINVAL on a null
 * handle or another value. */
#define TVLBM_FV_WALL_DIFFUSE 0
#define TVLBM_FV_WALL_SLIP_FREE 1
int tvlbm_fv_set_wall_model(tvlbm_fv *fv, int32_t model);

/* x ends.  TVLBM_FV_X_PERIODIC (default), or TVLBM_FV_X_ZERO_GRADIENT: the
 * adiabatic ends of Sec. VI, every population copied across each end
 * (f(-dx) = f(0) and beyond the last point the last point).  Applies to
 * later steps.  EINVAL on a null handle or another value. */
#define TVLBM_FV_X_PERIODIC 0
#define TVLBM_FV_X_ZERO_GRADIENT 1
int tvlbm_fv_set_x_ends(tvlbm_fv *fv, int32_t mode);
int tvlbm_fv_get_schedule(const tvlbm_fv *fv, tvlbm_fv_schedule *s);

#ifdef __cplusplus
}
#endif
#endif /* TVLBM_FV_H */
