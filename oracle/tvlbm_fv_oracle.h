/*
 * tvlbm_fv_oracle.h -- plain FP64 CPU oracle of the paper's finite-volume
 * TVLBM update, eq.(FVLB), with the diffuse-scattering wall nodes of
 * eq.(FVLB2) and eq.(IMPOSITION).
 *
 * TEST INFRASTRUCTURE ONLY, like tvlbm_oracle.h (whose lattice and
 * equilibrium it uses); nothing in the product library includes or calls it.
 *
 * Grid: mesh points (i, j), i = 0..nx-1 periodic in x with spacing dx,
 * j = 0..ny-1 with spacings dy[j] = y_{j+1} - y_j (Sec. III: rectangular
 * elements, non-uniform in y).  Periodic in y: ny spacings (dy[ny-1] closes
 * the period).  With walls: ny-1 spacings and the wall nodes j = 0 (inward
 * normal +y) and j = ny-1 (inward normal -y).
 *
 * One step (time lapse dt, relaxation time tau, velocities c_l = xi_l):
 *   every mesh point:  Omega_l = -(f_l - feq_l(rho, u, T)) / tau;
 *   interior points, all l:   eq.(FVLB) with the second-order 9-point
 *     stencils of Sec. III for c.grad f and Omega;
 *   wall points, populations with c.n <= 0:  eq.(FVLB2) with the one-sided
 *     6-point stencils of Sec. VII;
 *   wall points, populations with c.n > 0:  eq.(IMPOSITION) from the new
 *     incoming populations (the state is kept "imposed" after every step).
 * Populations are f[l][j][i], l = a*n + b as in tvlbm_oracle.h.
 */
#ifndef TVLBM_FV_ORACLE_H
#define TVLBM_FV_ORACLE_H

#include "tvlbm_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny;
  double dx, dt, tau;
  int collide;               /* 0 = no collision term                       */
  int walls;                 /* 0 = periodic in y, 1 = wall nodes           */
  double ulo, Tlo, uhi, Thi; /* wall equilibria (x velocity, temperature)   */
  double *dy;                /* spacings after each mesh point (see above)  */
  double emit_lo[ORC_QMAX];  /* feq_l(wall) / sum_out |c.n| feq(wall)       */
  double emit_hi[ORC_QMAX];
  double tau_g;              /* > 0: the non-unit-Prandtl term of eq.(FINAL) */
  int pscale;                /* 1: tau -> tau / p, tau_g -> tau_g / p, p = rho T */
  int slip_free;             /* 1: wall equilibria from Newton-Raphson (App. B) */
  int x_open;                /* 1: zero-gradient x ends, f(-dx) = f(0),
                                f(L_x) = f(L_x - dx) (Sec. VI); 0: periodic */
  int nr_last;               /* iterations of the last wall-node solve          */
} orc_fv_grid;

/* dy: ny (periodic) or ny-1 (walls) spacings, NULL = all dx.  0 or < 0. */
int orc_fv_init(const orc_lattice *L, orc_fv_grid *G, int nx, int ny, double dx,
                const double *dy, double dt, double tau, int collide, int walls,
                double ulo, double Tlo, double uhi, double Thi);
void orc_fv_free(orc_fv_grid *G);
/* Collision of eq.(OMEGAFVLB): tau_g > 0 adds
 *   -(1/tau_g) feq_l / (rho T^2) Pi : (c_l - u)(c_l - u)
 * (sign: see the collision term in the .c file),
 *   Pi_ij = sum_l (f_l - feq_l)(c_l - u)_i (c_l - u)_j   (eq.(FINAL));
 * tau_g <= 0 leaves single relaxation.  pscale: both relaxation times are
 * divided by the local pressure p = rho T (Sec. IX). */
void orc_fv_set_prandtl(orc_fv_grid *G, double tau_g, int pscale);
/* Wall model.  0: eq.(IMPOSITION) with the fixed wall equilibrium (ulo, Tlo)
 * / (uhi, Thi).  1: slip-free walls, eq.(IMPOSITION2) read with the flux
 * weights of eq.(IMPOSITION): at every wall point and step the wall
 * equilibrium (u_eq, T_eq) is found by the Newton-Raphson iteration of
 * Appendix B so that after re-emission the point's own x velocity and
 * temperature are the prescribed wall values (F1 = F2 = 0). */
void orc_fv_set_wall_model(orc_fv_grid *G, int slip_free);
/* x ends: 0 periodic, 1 zero gradient (adiabatic) for every population */
void orc_fv_set_x_ends(orc_fv_grid *G, int x_open);
/* eq.(IMPOSITION) at both wall rows, in place (no-op when periodic) */
void orc_fv_impose(const orc_lattice *L, const orc_fv_grid *G, double *f);
/* f = feq(fields) + noise (noise may be NULL), then imposed */
void orc_fv_set_fields(const orc_lattice *L, const orc_fv_grid *G, const double *rho,
                       const double *ux, const double *uy, const double *T,
                       const double *noise, double *f);
void orc_fv_step(const orc_lattice *L, const orc_fv_grid *G, const double *f, double *out);
void orc_fv_run(const orc_lattice *L, const orc_fv_grid *G, double *f, int nsteps);
/* height of the dual cell of row j: (dy_{j-1} + dy_j)/2 (half cells at walls) */
double orc_fv_dual(const orc_fv_grid *G, int j);
/* mass, x/y momentum, energy summed with weights dx * dual(j) */
void orc_fv_totals(const orc_lattice *L, const orc_fv_grid *G, const double *f, double tot[4]);

#ifdef __cplusplus
}
#endif
#endif /* TVLBM_FV_ORACLE_H */
