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

void orc_fv_set_wall_model(orc_fv_grid *G, int slip_free) { G->slip_free = slip_free; }
void orc_fv_set_x_ends(orc_fv_grid *G, int x_open) { G->x_open = x_open; }

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

/* Slip-free re-emission at one wall point (Appendix B).  Unknowns: the wall
 * equilibrium (ue, Te), started from the prescribed (uw, Tw).  With m the
 * incoming flux and Z(ue, Te) = sum_out |c.n| feq, the outgoing populations
 * are (m / Z) feq(ue, Te); the point then has
 *   F1 = rho uw - sum_l f_l c_x,   F2 = 2 rho Tw + rho uw^2 - sum_l f_l c^2.
 * Corrections: (Z / m) J^-1 (F1, F2) with J = [[A', B'], [C', D']], where
 * A..D are the flux-normalised derivatives printed in Appendix B and the
 * primes add the change of the point's density rho with the emitted
 * populations, A' = A - uw R_u, C' = C - (2 Tw + uw^2) R_u (R_u like A with
 * c_x replaced by 1; likewise B', D' with R_T): that is Newton's method on
 * the same F1, F2 (the printed coefficients omit the rho terms, which with
 * the flux-weighted emission makes the iteration oscillate and converge only
 * linearly).  Derivatives of feq by central differences.  Iterated until the
 * correction is below 1e-15 (at most 50 times); returns the count. */
static int impose_point_nr(const orc_lattice *L, double *f, long plane, long o, int top, double uw,
                           double Tw) {
  const int q = L->q;
  double cn[ORC_QMAX];
  double m = 0.0, rin = 0.0, jin = 0.0, ein = 0.0;
  for (int l = 0; l < q; ++l) {
    cn[l] = top ? -L->xi[l][1] : L->xi[l][1];
    if (cn[l] <= 0.0) {
      const double fl = f[l * plane + o];
      const double c2 = L->xi[l][0] * L->xi[l][0] + L->xi[l][1] * L->xi[l][1];
      m += -cn[l] * fl;
      rin += fl;
      jin += fl * L->xi[l][0];
      ein += fl * c2;
    }
  }
  double ue = uw, Te = Tw, fe[ORC_QMAX];
  int it = 0;
  while (it < 50) {
    const double h = 1e-6;
    double fu1[ORC_QMAX], fu0[ORC_QMAX], fT1[ORC_QMAX], fT0[ORC_QMAX];
    orc_feq(L, 1.0, ue, 0.0, Te, fe);
    orc_feq(L, 1.0, ue + h, 0.0, Te, fu1);
    orc_feq(L, 1.0, ue - h, 0.0, Te, fu0);
    orc_feq(L, 1.0, ue, 0.0, Te + h, fT1);
    orc_feq(L, 1.0, ue, 0.0, Te - h, fT0);
    double Z = 0.0, So = 0.0, Sx = 0.0, S2 = 0.0;
    double Zu = 0.0, Zt = 0.0, Ou = 0.0, Ot = 0.0, Xu = 0.0, Xt = 0.0, Eu = 0.0, Et = 0.0;
    for (int l = 0; l < q; ++l) {
      if (cn[l] <= 0.0) continue;
      const double cx = L->xi[l][0];
      const double c2 = cx * cx + L->xi[l][1] * L->xi[l][1];
      const double du = (fu1[l] - fu0[l]) / (2.0 * h), dT = (fT1[l] - fT0[l]) / (2.0 * h);
      Z += cn[l] * fe[l];
      So += fe[l];
      Sx += cx * fe[l];
      S2 += c2 * fe[l];
      Zu += cn[l] * du;
      Zt += cn[l] * dT;
      Ou += du;
      Ot += dT;
      Xu += cx * du;
      Xt += cx * dT;
      Eu += c2 * du;
      Et += c2 * dT;
    }
    const double s = m / Z;
    const double rho = rin + s * So, jx = jin + s * Sx, e2 = ein + s * S2;
    const double F1 = rho * uw - jx;
    const double F2 = 2.0 * rho * Tw + rho * uw * uw - e2;
    /* Appendix B's coefficients and the density terms */
    const double A = Xu - Zu * Sx / Z, B = Xt - Zt * Sx / Z;
    const double C = Eu - Zu * S2 / Z, D = Et - Zt * S2 / Z;
    const double Ru = Ou - Zu * So / Z, Rt = Ot - Zt * So / Z;
    const double w2 = 2.0 * Tw + uw * uw;
    const double A1 = A - uw * Ru, B1 = B - uw * Rt, C1 = C - w2 * Ru, D1 = D - w2 * Rt;
    const double k = Z / ((A1 * D1 - B1 * C1) * m);
    const double dU = k * (D1 * F1 - B1 * F2), dT = k * (-C1 * F1 + A1 * F2);
    ue += dU;
    Te += dT;
    ++it;
    if (fabs(dU) + fabs(dT) < 1e-15) break;
  }
  orc_feq(L, 1.0, ue, 0.0, Te, fe);
  double Z = 0.0;
  for (int l = 0; l < q; ++l)
    if (cn[l] > 0.0) Z += cn[l] * fe[l];
  for (int l = 0; l < q; ++l)
    if (cn[l] > 0.0) f[l * plane + o] = m / Z * fe[l];
  return it;
}

void orc_fv_impose(const orc_lattice *L, const orc_fv_grid *G, double *f) {
  if (!G->walls) return;
  const long plane = (long)G->nx * G->ny;
  int itmax = 0;
  for (int i = 0; i < G->nx; ++i) {
    const long olo = i, ohi = (long)(G->ny - 1) * G->nx + i;
    if (G->slip_free) {
      const int a = impose_point_nr(L, f, plane, olo, 0, G->ulo, G->Tlo);
      const int b = impose_point_nr(L, f, plane, ohi, 1, G->uhi, G->Thi);
      if (a > itmax) itmax = a;
      if (b > itmax) itmax = b;
    } else {
      impose_point(L, G, f, plane, olo, 0);
      impose_point(L, G, f, plane, ohi, 1);
    }
  }
  ((orc_fv_grid *)G)->nr_last = itmax;
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
      /* x neighbours: periodic, or the end point itself beyond a
       * zero-gradient end */
      const int ip = G->x_open ? (i + 1 < nx ? i + 1 : nx - 1) : wrapi(i + 1, nx);
      const int im = G->x_open ? (i > 0 ? i - 1 : 0) : wrapi(i - 1, nx);
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
