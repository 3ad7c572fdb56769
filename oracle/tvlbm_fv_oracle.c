/*
 * tvlbm_fv_oracle.c -- FP64 CPU oracle of the finite-volume TVLBM update
 * (eq.(FVLB), eq.(FVLB2), eq.(IMPOSITION)).  TEST INFRASTRUCTURE ONLY.
 * See tvlbm_fv_oracle.h for the grid and the step.
 */
#include "tvlbm_fv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int wrapi(int i, int n) { return ((i % n) + n) % n; }

int orc_fv_init(const orc_lattice *L, orc_fv_grid *G, int nx, int ny, double dx,
                const double *dy, double dt, double tau, int collide, int walls,
                double ulo, double Tlo, double uhi, double Thi) {
  memset(G, 0, sizeof *G);
  if (nx < 2 || ny < (walls ? 3 : 2) || !(dx > 0.0) || !(dt > 0.0)) return -1;
  if (collide && !(tau > 0.0)) return -1;
  G->nx = nx; G->ny = ny; G->dx = dx; G->dt = dt; G->tau = tau;
  G->collide = collide; G->walls = walls;
  G->ulo = ulo; G->Tlo = Tlo; G->uhi = uhi; G->Thi = Thi;
  const int ns = walls ? ny - 1 : ny;
  G->dy = (double *)malloc(sizeof(double) * ns);
  if (!G->dy) return -2;
  for (int j = 0; j < ns; ++j) {
    G->dy[j] = dy ? dy[j] : dx;
    if (!(G->dy[j] > 0.0)) return -1;
  }
  if (walls) {
    /* eq.(IMPOSITION): outgoing l (c.n > 0) receives the incoming normal
     * flux times feq_l(wall) / sum_{c.n > 0} |c.n| feq(wall) */
    double flo[ORC_QMAX], fhi[ORC_QMAX], zlo = 0.0, zhi = 0.0;
    orc_feq(L, 1.0, ulo, 0.0, Tlo, flo);
    orc_feq(L, 1.0, uhi, 0.0, Thi, fhi);
    for (int l = 0; l < L->q; ++l) {
      const double cy = L->xi[l][1];
      if (cy > 0.0) zlo += cy * flo[l];
      if (cy < 0.0) zhi += -cy * fhi[l];
    }
    for (int l = 0; l < L->q; ++l) {
      const double cy = L->xi[l][1];
      G->emit_lo[l] = cy > 0.0 ? flo[l] / zlo : 0.0;
      G->emit_hi[l] = cy < 0.0 ? fhi[l] / zhi : 0.0;
    }
  }
  return 0;
}

void orc_fv_set_prandtl(orc_fv_grid *G, double tau_g, int pscale) {
  G->tau_g = tau_g;
  G->pscale = pscale;
}

void orc_fv_free(orc_fv_grid *G) {
  free(G->dy);
  G->dy = NULL;
}

double orc_fv_dual(const orc_fv_grid *G, int j) {
  const int ny = G->ny;
  if (!G->walls) return 0.5 * (G->dy[wrapi(j - 1, ny)] + G->dy[j]);
  if (j == 0) return 0.5 * G->dy[0];
  if (j == ny - 1) return 0.5 * G->dy[ny - 2];
  return 0.5 * (G->dy[j - 1] + G->dy[j]);
}

/* incoming normal flux at a wall point and the re-emitted populations */
static void impose_point(const orc_lattice *L, const orc_fv_grid *G, double *f, long plane,
                         long o, int top) {
  double s = 0.0;
  for (int l = 0; l < L->q; ++l) {
    const double cn = top ? -L->xi[l][1] : L->xi[l][1];  /* c . n, n inward */
    if (cn <= 0.0) s += -cn * f[l * plane + o];
  }
  for (int l = 0; l < L->q; ++l) {
    const double cn = top ? -L->xi[l][1] : L->xi[l][1];
    if (cn > 0.0) f[l * plane + o] = s * (top ? G->emit_hi[l] : G->emit_lo[l]);
  }
}

void orc_fv_impose(const orc_lattice *L, const orc_fv_grid *G, double *f) {
  if (!G->walls) return;
  const long plane = (long)G->nx * G->ny;
  for (int i = 0; i < G->nx; ++i) {
    impose_point(L, G, f, plane, i, 0);
    impose_point(L, G, f, plane, (long)(G->ny - 1) * G->nx + i, 1);
  }
}

void orc_fv_set_fields(const orc_lattice *L, const orc_fv_grid *G, const double *rho,
                       const double *ux, const double *uy, const double *T,
                       const double *noise, double *f) {
  const long plane = (long)G->nx * G->ny;
  double feq[ORC_QMAX];
  for (long c = 0; c < plane; ++c) {
    orc_feq(L, rho[c], ux[c], uy[c], T[c], feq);
    for (int l = 0; l < L->q; ++l) f[l * plane + c] = feq[l] + (noise ? noise[l * plane + c] : 0.0);
  }
  orc_fv_impose(L, G, f);
}

/* Omega_l = -(f_l - feq_l)/tau at every mesh point */
static void collision_term(const orc_lattice *L, const orc_fv_grid *G, const double *f,
                           double *om) {
  const long plane = (long)G->nx * G->ny;
  #pragma omp parallel for schedule(static)
  for (long c = 0; c < plane; ++c) {
    if (!G->collide) {
      for (int l = 0; l < L->q; ++l) om[l * plane + c] = 0.0;
      continue;
    }
    double r, vx, vy, T, feq[ORC_QMAX];
    orc_moments(L, f + c, plane, &r, &vx, &vy, &T);
    orc_feq(L, r, vx, vy, T, feq);
    /* pressure-rescaled relaxation times: tau / p, tau_g / p */
    const double ps = G->pscale ? r * T : 1.0;
    for (int l = 0; l < L->q; ++l) om[l * plane + c] = -ps * (f[l * plane + c] - feq[l]) / G->tau;
    if (G->tau_g > 0.0) {
      /* eq.(FINAL): Pi from the non-equilibrium part, central velocities.
       * The term enters with a minus sign: contracted with (c-u)(c-u) it
       * changes Pi at the rate -2 Pi / tau_g, so that the stress relaxes at
       * 1/tau + 2/tau_g and the viscosity is the paper's
       * c_v rho T tau tau_g / (2 tau + tau_g); the printed plus sign would
       * make the stress grow whenever tau_g < 2 tau. */
      double pxx = 0.0, pxy = 0.0, pyy = 0.0;
      for (int l = 0; l < L->q; ++l) {
        const double ne = f[l * plane + c] - feq[l];
        const double X = L->xi[l][0] - vx, Y = L->xi[l][1] - vy;
        pxx += ne * X * X;
        pxy += ne * X * Y;
        pyy += ne * Y * Y;
      }
      for (int l = 0; l < L->q; ++l) {
        const double X = L->xi[l][0] - vx, Y = L->xi[l][1] - vy;
        const double contr = pxx * X * X + 2.0 * pxy * X * Y + pyy * Y * Y;
        om[l * plane + c] -= ps / G->tau_g * feq[l] / (r * T * T) * contr;
      }
    }
  }
}

void orc_fv_step(const orc_lattice *L, const orc_fv_grid *G, const double *f, double *out) {
  const int nx = G->nx, ny = G->ny;
  const long plane = (long)nx * ny;
  double *om = (double *)malloc(sizeof(double) * plane * L->q);
  collision_term(L, G, f, om);
  #pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    const int wall_lo = G->walls && j == 0, wall_hi = G->walls && j == ny - 1;
    for (int i = 0; i < nx; ++i) {
      const int ip = wrapi(i + 1, nx), im = wrapi(i - 1, nx);
      for (int l = 0; l < L->q; ++l) {
        const double cx = L->xi[l][0], cy = L->xi[l][1];
        const double *F = f + l * plane, *W = om + l * plane;
        const long o = (long)j * nx + i;
        double dfx, dfy, omb;
        if (!wall_lo && !wall_hi) {
          /* interior point, Sec. III: neighbours 1 (+x), 2 (+y), 3 (-x),
           * 4 (-y), 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y) */
          const int jp = G->walls ? j + 1 : wrapi(j + 1, ny);
          const int jm = G->walls ? j - 1 : wrapi(j - 1, ny);
          const double dym = G->walls ? G->dy[j - 1] : G->dy[wrapi(j - 1, ny)];
          const double f1 = F[(long)j * nx + ip], f2 = F[(long)jp * nx + i];
          const double f3 = F[(long)j * nx + im], f4 = F[(long)jm * nx + i];
          const double f5 = F[(long)jp * nx + ip], f6 = F[(long)jp * nx + im];
          const double f7 = F[(long)jm * nx + im], f8 = F[(long)jm * nx + ip];
          dfx = (2.0 / (G->dx + G->dx)) *
                (3.0 / 8.0 * f1 - 3.0 / 8.0 * f3 + 1.0 / 16.0 * f5 - 1.0 / 16.0 * f6 -
                 1.0 / 16.0 * f7 + 1.0 / 16.0 * f8);
          dfy = (2.0 / (G->dy[j] + dym)) *
                (3.0 / 8.0 * f2 - 3.0 / 8.0 * f4 + 1.0 / 16.0 * f5 + 1.0 / 16.0 * f6 -
                 1.0 / 16.0 * f7 - 1.0 / 16.0 * f8);
          omb = 9.0 / 16.0 * W[o] +
                3.0 / 32.0 * (W[(long)j * nx + ip] + W[(long)jp * nx + i] + W[(long)j * nx + im] +
                              W[(long)jm * nx + i]) +
                1.0 / 64.0 * (W[(long)jp * nx + ip] + W[(long)jp * nx + im] +
                              W[(long)jm * nx + im] + W[(long)jm * nx + ip]);
        } else {
          /* wall point, Sec. VII: only the incoming populations advance;
           * neighbour 2 is the next mesh point into the fluid, 5 and 6 its
           * x neighbours (+x, -x).  The y derivative is one-sided. */
          const double cn = wall_hi ? -cy : cy;
          if (cn > 0.0) continue;  /* re-emitted below */
          const int j2 = wall_hi ? ny - 2 : 1;
          const double h = wall_hi ? G->dy[ny - 2] : G->dy[0];
          const double f0 = F[o], f1 = F[(long)j * nx + ip], f3 = F[(long)j * nx + im];
          const double f2 = F[(long)j2 * nx + i], f5 = F[(long)j2 * nx + ip],
                       f6 = F[(long)j2 * nx + im];
          dfx = (2.0 / (G->dx + G->dx)) *
                (3.0 / 8.0 * f1 - 3.0 / 8.0 * f3 + 1.0 / 8.0 * f5 - 1.0 / 8.0 * f6);
          /* derivative along the inward normal, then its sign for +y */
          const double dn = (2.0 / h) * (3.0 / 8.0 * f2 - 3.0 / 8.0 * f0 + 1.0 / 16.0 * f5 +
                                         1.0 / 16.0 * f6 - 1.0 / 16.0 * f1 - 1.0 / 16.0 * f3);
          dfy = wall_hi ? -dn : dn;
          omb = 9.0 / 16.0 * W[o] + 3.0 / 32.0 * W[(long)j * nx + ip] +
                3.0 / 16.0 * W[(long)j2 * nx + i] + 3.0 / 32.0 * W[(long)j * nx + im] +
                1.0 / 32.0 * W[(long)j2 * nx + ip] + 1.0 / 32.0 * W[(long)j2 * nx + im];
        }
        out[l * plane + o] = F[o] + G->dt * (omb - (cx * dfx + cy * dfy));
      }
    }
  }
  free(om);
  orc_fv_impose(L, G, out);
}

void orc_fv_run(const orc_lattice *L, const orc_fv_grid *G, double *f, int nsteps) {
  const long n = (long)G->nx * G->ny * L->q;
  double *tmp = (double *)malloc(sizeof(double) * n);
  for (int s = 0; s < nsteps; ++s) {
    orc_fv_step(L, G, f, tmp);
    memcpy(f, tmp, sizeof(double) * n);
  }
  free(tmp);
}

void orc_fv_totals(const orc_lattice *L, const orc_fv_grid *G, const double *f, double tot[4]) {
  const long plane = (long)G->nx * G->ny;
  tot[0] = tot[1] = tot[2] = tot[3] = 0.0;
  for (int j = 0; j < G->ny; ++j) {
    const double v = G->dx * orc_fv_dual(G, j);
    for (int i = 0; i < G->nx; ++i)
      for (int l = 0; l < L->q; ++l) {
        const double fl = f[l * plane + (long)j * G->nx + i];
        const double cx = L->xi[l][0], cy = L->xi[l][1];
        tot[0] += v * fl;
        tot[1] += v * cx * fl;
        tot[2] += v * cy * fl;
        tot[3] += v * 0.5 * (cx * cx + cy * cy) * fl;
      }
  }
}
