/*
 * tvlbm_oracle.c -- plain FP64 CPU oracle of the TVLBM step.
 *
 * TEST INFRASTRUCTURE ONLY (see tvlbm_oracle.h).  Built with
 * -O2 -ffp-contract=off so that every multiply and add rounds separately, as
 * written.  It is deliberately slow and literal: no blocking, no fusion, no
 * reordering beyond what the definitions below state.
 *
 * Pins (tests/test_oracle_*.py) tie each function to something other than
 * itself: Gauss-Hermite closed forms and moment identities, equilibrium
 * moment identities and the tensor form of the Hermite expansion, exact
 * conservation, the equilibrium fixed point, integer shifts against a plain
 * array roll, the Fourier symbol of the remap, and the linearised shear-wave
 * eigenvalue.  Non-uniform rows: the Fourier symbol of a shift by s/h rows
 * on rows of height h, remap matrices derived by hand on a two-height mesh,
 * the lengths that cross a wall and the emitted interval on that mesh.
 * Totals: closed-form totals of row-wise equilibria on rows of different
 * heights.  A NumPy mini-oracle (mini.py) agrees step by step.  The wall
 * re-emission rule itself (which equilibrium the incident mass is emitted
 * with) is pinned only by mass balance and the rest-state fixed point
 * (parity unpinned for its values).
 */
#include "tvlbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define D 2.0 /* space dimension */

/* ------------------------------------------------------------------------ */
/* 1-D Gauss-Hermite rule by the Golub-Welsch construction.                 */
/*                                                                          */
/* The probabilists' Hermite polynomials obey He_{k+1} = x He_k - k He_{k-1}; */
/* their Jacobi matrix is symmetric tridiagonal with zero diagonal and      */
/* off-diagonal sqrt(k).  Its eigenvalues are the nodes; the squared first  */
/* component of each normalised eigenvector is the weight (normalised to a   */
/* unit total).  The eigenproblem is solved with cyclic Jacobi rotations,   */
/* the nodes are polished by Newton on He_n, and the weights are evaluated  */
/* from the normalised eigenvector in closed form: for a node x the        */
/* eigenvector is (p_0(x), ..., p_{n-1}(x)) with p_k = He_k / sqrt(k!), so */
/* its squared first component after normalisation is 1 / sum_k p_k(x)^2.   */
/* ------------------------------------------------------------------------ */
static void hermite_he(int n, double x, double *he_n, double *he_nm1) {
  double a = 1.0, b = x; /* He_0, He_1 */
  if (n == 0) { *he_n = 1.0; *he_nm1 = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double c = x * b - (double)k * a;
    a = b;
    b = c;
  }
  *he_n = b;
  *he_nm1 = a;
}

int orc_gauss_hermite(int n, double *x, double *w) {
  if (n < 1 || n > ORC_NMAX) return -1;
  double A[ORC_NMAX][ORC_NMAX], V[ORC_NMAX][ORC_NMAX];
  memset(A, 0, sizeof A);
  memset(V, 0, sizeof V);
  for (int i = 0; i < n; ++i) V[i][i] = 1.0;
  for (int k = 1; k < n; ++k) A[k - 1][k] = A[k][k - 1] = sqrt((double)k);
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int r = p + 1; r < n; ++r) off += A[p][r] * A[p][r];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p) {
      for (int r = p + 1; r < n; ++r) {
        if (fabs(A[p][r]) < 1e-300) continue;
        double theta = (A[r][r] - A[p][p]) / (2.0 * A[p][r]);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) { /* columns p, r of A*P */
          double akp = A[k][p], akr = A[k][r];
          A[k][p] = c * akp - s * akr;
          A[k][r] = s * akp + c * akr;
        }
        for (int k = 0; k < n; ++k) { /* rows p, r of P^T*(A*P) */
          double apk = A[p][k], ark = A[r][k];
          A[p][k] = c * apk - s * ark;
          A[r][k] = s * apk + c * ark;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k][p], vkr = V[k][r];
          V[k][p] = c * vkp - s * vkr;
          V[k][r] = s * vkp + c * vkr;
        }
      }
    }
  }
  double nodes[ORC_NMAX];
  for (int i = 0; i < n; ++i) nodes[i] = A[i][i];
  /* ascending order (selection sort, n <= 8) */
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k)
      if (nodes[k] < nodes[i]) { double t = nodes[i]; nodes[i] = nodes[k]; nodes[k] = t; }
  for (int i = 0; i < n; ++i) {
    double xi = nodes[i];
    for (int it = 0; it < 3; ++it) { /* Newton on He_n, He_n' = n He_{n-1} */
      double hn, hnm1;
      hermite_he(n, xi, &hn, &hnm1);
      if (hnm1 != 0.0) xi -= hn / ((double)n * hnm1);
    }
    if (n % 2 == 1 && i == n / 2) xi = 0.0; /* odd rules contain the origin */
    double pk_prev = 1.0, pk = xi, sum = 1.0; /* He_0^2/0! */
    for (int k = 1; k < n; ++k) {
      double fact = 1.0;
      for (int m = 2; m <= k; ++m) fact *= (double)m;
      sum += pk * pk / fact;
      double nxt = xi * pk - (double)k * pk_prev;
      pk_prev = pk;
      pk = nxt;
    }
    x[i] = xi;
    w[i] = 1.0 / sum;
  }
  /* symmetrise: the rule is symmetric about 0 */
  for (int i = 0; i < n / 2; ++i) {
    double xa = 0.5 * (x[n - 1 - i] - x[i]);
    double wa = 0.5 * (w[n - 1 - i] + w[i]);
    x[i] = -xa; x[n - 1 - i] = xa;
    w[i] = wa; w[n - 1 - i] = wa;
  }
  return 0;
}

/* snap a displacement to the nearest integer when within 4 ulp of it */
static double snap(double s) {
  double r = nearbyint(s);
  double ulp = nextafter(fabs(s), INFINITY) - fabs(s);
  return (fabs(s - r) <= 4.0 * ulp) ? r : s;
}

int orc_lattice_gh(int n, int order, double cfl, int cfl_norm, orc_lattice *L) {
  if (n < 2 || n > ORC_NMAX || order < 2 || order > 5 || !(cfl > 0.0)) return -1;
  memset(L, 0, sizeof *L);
  L->n = n;
  L->q = n * n;
  L->order = order;
  if (orc_gauss_hermite(n, L->x, L->wx)) return -1;
  double xmax = L->x[n - 1];
  double cmax = (cfl_norm == 0) ? sqrt(2.0) * xmax : xmax;
  L->lambda = cfl / cmax;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      int l = a * n + b;
      L->xi[l][0] = L->x[a];
      L->xi[l][1] = L->x[b];
      L->w[l] = L->wx[a] * L->wx[b];
      L->s[l][0] = snap(L->lambda * L->x[a]);
      L->s[l][1] = snap(L->lambda * L->x[b]);
      if (fabs(L->s[l][0]) > 1.0 || fabs(L->s[l][1]) > 1.0) return -1;
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium: Hermite expansion of Sec. II written in the scalar form of   */
/* Appendix A (orders 2 to 5).  The density multiplies every order (the     */
/* appendix prints it only in the fifth-order term).                        */
/*   u_l = u . xi_l,  u2 = |u|^2,  c2 = |xi_l|^2,  th = T - 1                */
/* ------------------------------------------------------------------------ */
void orc_feq(const orc_lattice *L, double rho, double ux, double uy, double T,
             double *feq) {
  double u2 = ux * ux + uy * uy;
  double th = T - 1.0;
  for (int l = 0; l < L->q; ++l) {
    double ul = ux * L->xi[l][0] + uy * L->xi[l][1];
    double c2 = L->xi[l][0] * L->xi[l][0] + L->xi[l][1] * L->xi[l][1];
    double sum = 1.0 + ul;
    /* order 2 */
    sum += 0.5 * (ul * ul - u2 + th * (c2 - D));
    if (L->order >= 3)
      sum += (ul / 6.0) * (ul * ul - 3.0 * u2 + 3.0 * th * (c2 - D - 2.0));
    if (L->order >= 4) {
      sum += (ul * ul * ul * ul - 6.0 * ul * ul * u2 + 3.0 * u2 * u2) / 24.0;
      sum += (th / 4.0) * ((c2 - D - 2.0) * (ul * ul - u2) - 2.0 * ul * ul);
      sum += (th * th / 8.0) * (c2 * c2 - 2.0 * (D + 2.0) * c2 + D * (D + 2.0));
    }
    if (L->order >= 5) {
      const double ul3 = ul * ul * ul;
      sum += (ul3 * ul * ul - 10.0 * u2 * ul3 + 15.0 * u2 * u2 * ul) / 120.0;
      sum += (th / 12.0) * (c2 * ul3 - (D + 6.0) * ul3 - 3.0 * c2 * ul * u2 + (3.0 * D + 12.0) * u2 * ul);
      sum += (th * th / 8.0) * (ul * c2 * c2 - (2.0 * D + 8.0) * c2 * ul + (D * D + 6.0 * D + 8.0) * ul);
    }
    feq[l] = L->w[l] * rho * sum;
  }
}

/* Moments of Sec. II: rho = sum f, rho u = sum xi f,
 * rho T = (1/D) sum |xi - u|^2 f  (central form). */
void orc_moments(const orc_lattice *L, const double *f, long stride,
                 double *rho, double *ux, double *uy, double *T) {
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int l = 0; l < L->q; ++l) {
    double fl = f[(long)l * stride];
    r += fl;
    jx += L->xi[l][0] * fl;
    jy += L->xi[l][1] * fl;
  }
  double vx = jx / r, vy = jy / r;
  double e = 0.0;
  for (int l = 0; l < L->q; ++l) {
    double dx = L->xi[l][0] - vx, dy = L->xi[l][1] - vy;
    e += (dx * dx + dy * dy) * f[(long)l * stride];
  }
  *rho = r;
  *ux = vx;
  *uy = vy;
  *T = e / (D * r);
}

/* ------------------------------------------------------------------------ */
/* Grid: row boundaries and the exact 1-D overlap lengths of shifted rows.   */
/* ------------------------------------------------------------------------ */
static double overlap(double a0, double a1, double b0, double b1) {
  double lo = a0 > b0 ? a0 : b0;
  double hi = a1 < b1 ? a1 : b1;
  return hi > lo ? hi - lo : 0.0;
}

/* overlap of the unit source column offset by o cells and shifted by sx with
 * the unit target column [0,1] */
static double wx_tap(double sx, int o) {
  return overlap((double)o + sx, (double)(o + 1) + sx, 0.0, 1.0);
}

void orc_grid_free(orc_grid *G) {
  free(G->y); free(G->dy); free(G->yk_start); free(G->yk_src); free(G->yk_len);
  free(G->blo); free(G->ahi); free(G->glo); free(G->ghi);
  memset(G, 0, sizeof *G);
}

int orc_grid_init(const orc_lattice *L, orc_grid *G, int nx, int ny,
                  const double *dy, double tau, int collide, int walls,
                  double ulo, double Tlo, double uhi, double Thi) {
  memset(G, 0, sizeof *G);
  if (nx < 1 || ny < 2) return -1;
  G->nx = nx; G->ny = ny; G->tau = tau; G->collide = collide; G->walls = walls;
  G->ulo = ulo; G->Tlo = Tlo; G->uhi = uhi; G->Thi = Thi;
  int q = L->q;
  G->y = malloc(sizeof(double) * (ny + 1));
  G->dy = malloc(sizeof(double) * ny);
  G->y[0] = 0.0;
  for (int j = 0; j < ny; ++j) {
    G->dy[j] = dy ? dy[j] : 1.0;
    if (!(G->dy[j] > 0.0)) return -1;
    G->y[j + 1] = G->y[j] + G->dy[j];
  }
  double H = G->y[ny];
  /* y-overlaps, CSR by (l, target row k), source rows ascending */
  long cap = (long)q * ny * 8 + 16;
  G->yk_start = malloc(sizeof(int) * ((long)q * (ny + 1)));
  G->yk_src = malloc(sizeof(int) * cap);
  G->yk_len = malloc(sizeof(double) * cap);
  long nnz = 0;
  for (int l = 0; l < q; ++l) {
    double sy = L->s[l][1];
    for (int k = 0; k < ny; ++k) {
      G->yk_start[(long)l * (ny + 1) + k] = (int)nnz;
      for (int j = 0; j < ny; ++j) {
        /* source interval relative to the target row's lower edge */
        double a0 = (G->y[j] - G->y[k]) + sy, a1 = (G->y[j + 1] - G->y[k]) + sy;
        double len = overlap(a0, a1, 0.0, G->dy[k]);
        if (!walls) { /* periodic images */
          len += overlap(a0 - H, a1 - H, 0.0, G->dy[k]);
          len += overlap(a0 + H, a1 + H, 0.0, G->dy[k]);
        }
        if (len > 0.0) {
          if (nnz >= cap) return -1;
          G->yk_src[nnz] = j;
          G->yk_len[nnz] = len;
          ++nnz;
        }
      }
    }
    G->yk_start[(long)l * (ny + 1) + ny] = (int)nnz;
  }
  G->blo = calloc((size_t)q * ny, sizeof(double));
  G->ahi = calloc((size_t)q * ny, sizeof(double));
  G->glo = calloc((size_t)q * ny, sizeof(double));
  G->ghi = calloc((size_t)q * ny, sizeof(double));
  if (walls) {
    const double BIG = 1e300;
    for (int l = 0; l < q; ++l) {
      double sy = L->s[l][1];
      for (int j = 0; j < ny; ++j) {
        /* part of the shifted row j below y = 0 / above y = H */
        G->blo[(long)l * ny + j] = overlap(G->y[j] + sy, G->y[j + 1] + sy, -BIG, 0.0);
        G->ahi[(long)l * ny + j] = overlap((G->y[j] - H) + sy, (G->y[j + 1] - H) + sy, 0.0, BIG);
        /* ghost intervals: the wall emits into [0, sy] (bottom, sy > 0) and
         * into [H - |sy|, H] (top, sy < 0) */
        if (sy > 0.0)
          G->glo[(long)l * ny + j] = overlap(-G->y[j], sy - G->y[j], 0.0, G->dy[j]);
        if (sy < 0.0)
          G->ghi[(long)l * ny + j] = overlap((H - G->y[j]) + sy, H - G->y[j], 0.0, G->dy[j]);
      }
    }
    orc_feq(L, 1.0, ulo, 0.0, Tlo, G->fw_lo);
    orc_feq(L, 1.0, uhi, 0.0, Thi, G->fw_hi);
    G->zlo = 0.0;
    G->zhi = 0.0;
    for (int l = 0; l < q; ++l) {
      double sy = L->s[l][1];
      if (sy > 0.0) G->zlo += sy * G->fw_lo[l];
      if (sy < 0.0) G->zhi += -sy * G->fw_hi[l];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial state and collision                                              */
/* ------------------------------------------------------------------------ */
void orc_set_fields(const orc_lattice *L, const orc_grid *G,
                    const double *rho, const double *ux, const double *uy,
                    const double *T, const double *noise, double *f) {
  long nc = (long)G->nx * G->ny;
  for (long c = 0; c < nc; ++c) {
    double feq[ORC_QMAX];
    orc_feq(L, rho[c], ux[c], uy[c], T[c], feq);
    for (int l = 0; l < L->q; ++l)
      f[(long)l * nc + c] = feq[l] + (noise ? noise[(long)l * nc + c] : 0.0);
  }
}

/* BGK collision, eq.(lb) integrated explicitly over one step with tau in
 * steps: f* = f - (f - feq)/tau. */
void orc_collide(const orc_lattice *L, const orc_grid *G, const double *f,
                 double *fstar) {
  long nc = (long)G->nx * G->ny;
  int q = L->q;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    if (!G->collide) {
      for (int l = 0; l < q; ++l) fstar[(long)l * nc + c] = f[(long)l * nc + c];
      continue;
    }
    double rho, ux, uy, T, feq[ORC_QMAX];
    orc_moments(L, f + c, nc, &rho, &ux, &uy, &T);
    orc_feq(L, rho, ux, uy, T, feq);
    for (int l = 0; l < q; ++l) {
      double fl = f[(long)l * nc + c];
      fstar[(long)l * nc + c] = fl - (fl - feq[l]) / G->tau;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Volumetric streaming with diffuse walls                                  */
/* ------------------------------------------------------------------------ */
static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* x-part of the remap of row values v[] into column i; wx[o+2] holds the
 * overlap of source column i+o, o = -2..2 */
static void xtaps(double sx, double *wx) {
  for (int o = -2; o <= 2; ++o) wx[o + 2] = wx_tap(sx, o);
}
static double xpull(const double *v, int i, int nx, const double *wx) {
  double acc = 0.0;
  for (int o = -2; o <= 2; ++o) {
    if (wx[o + 2] == 0.0) continue;
    acc += wx[o + 2] * v[wrap(i + o, nx)];
  }
  return acc;
}

/* Mass (per unit column width) carried below y = 0 / above y = H by the
 * shifted source cells, assigned to the column where it lands. */
void orc_wall_incident(const orc_lattice *L, const orc_grid *G,
                       const double *fstar, double *mlo, double *mhi) {
  int nx = G->nx, ny = G->ny, q = L->q;
  long nc = (long)nx * ny;
  for (int i = 0; i < nx; ++i) {
    double lo = 0.0, hi = 0.0;
    for (int l = 0; l < q; ++l) {
      for (int j = 0; j < ny; ++j) {
        double b = G->blo[(long)l * ny + j], a = G->ahi[(long)l * ny + j];
        if (b == 0.0 && a == 0.0) continue;
        double wx[5];
        xtaps(L->s[l][0], wx);
        double x = xpull(fstar + (long)l * nc + (long)j * nx, i, nx, wx);
        lo += b * x;
        hi += a * x;
      }
    }
    mlo[i] = lo;
    mhi[i] = hi;
  }
}

void orc_wall_emitted(const orc_lattice *L, const orc_grid *G,
                      const double *fstar, double *elo, double *ehi) {
  int nx = G->nx, ny = G->ny, q = L->q;
  double *mlo = malloc(sizeof(double) * nx), *mhi = malloc(sizeof(double) * nx);
  orc_wall_incident(L, G, fstar, mlo, mhi);
  for (int i = 0; i < nx; ++i) {
    double lo = 0.0, hi = 0.0;
    for (int l = 0; l < q; ++l) {
      double glen = 0.0, hlen = 0.0;
      for (int k = 0; k < ny; ++k) {
        glen += G->glo[(long)l * ny + k];
        hlen += G->ghi[(long)l * ny + k];
      }
      if (glen > 0.0) lo += glen * (mlo[i] * G->fw_lo[l] / G->zlo);
      if (hlen > 0.0) hi += hlen * (mhi[i] * G->fw_hi[l] / G->zhi);
    }
    elo[i] = lo;
    ehi[i] = hi;
  }
  free(mlo);
  free(mhi);
}

void orc_stream(const orc_lattice *L, const orc_grid *G, const double *fstar,
                double *fout) {
  int nx = G->nx, ny = G->ny, q = L->q;
  long nc = (long)nx * ny;
  double *mlo = NULL, *mhi = NULL;
  if (G->walls) {
    mlo = malloc(sizeof(double) * nx);
    mhi = malloc(sizeof(double) * nx);
    orc_wall_incident(L, G, fstar, mlo, mhi);
  }
#pragma omp parallel for schedule(static)
  for (int l = 0; l < q; ++l) {
    double wx[5];
    xtaps(L->s[l][0], wx);
    double *glo_row = malloc(sizeof(double) * nx), *ghi_row = malloc(sizeof(double) * nx);
    if (G->walls) {
      for (int i = 0; i < nx; ++i) {
        /* re-emitted ghost populations, eq.(IMPOSITION): the incident mass
         * redistributed with the flux-weighted wall Maxwellian */
        glo_row[i] = (L->s[l][1] > 0.0) ? mlo[i] * G->fw_lo[l] / G->zlo : 0.0;
        ghi_row[i] = (L->s[l][1] < 0.0) ? mhi[i] * G->fw_hi[l] / G->zhi : 0.0;
      }
    }
    for (int k = 0; k < ny; ++k) {
      int e0 = G->yk_start[(long)l * (ny + 1) + k], e1 = G->yk_start[(long)l * (ny + 1) + k + 1];
      double gl = G->walls ? G->glo[(long)l * ny + k] : 0.0;
      double gh = G->walls ? G->ghi[(long)l * ny + k] : 0.0;
      for (int i = 0; i < nx; ++i) {
        double acc = 0.0;
        for (int e = e0; e < e1; ++e) {
          int j = G->yk_src[e];
          acc += G->yk_len[e] * xpull(fstar + (long)l * nc + (long)j * nx, i, nx, wx);
        }
        if (gl > 0.0) acc += gl * xpull(glo_row, i, nx, wx);
        if (gh > 0.0) acc += gh * xpull(ghi_row, i, nx, wx);
        fout[(long)l * nc + (long)k * nx + i] = acc / G->dy[k];
      }
    }
    free(glo_row);
    free(ghi_row);
  }
  free(mlo);
  free(mhi);
}

void orc_step(const orc_lattice *L, const orc_grid *G, const double *f,
              double *fout, double *work) {
  orc_collide(L, G, f, work);
  orc_stream(L, G, work, fout);
}

void orc_run(const orc_lattice *L, const orc_grid *G, double *f, int nsteps) {
  long n = (long)L->q * G->nx * G->ny;
  double *work = malloc(sizeof(double) * n), *tmp = malloc(sizeof(double) * n);
  for (int s = 0; s < nsteps; ++s) {
    orc_step(L, G, f, tmp, work);
    memcpy(f, tmp, sizeof(double) * n);
  }
  free(work);
  free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */
void orc_fields(const orc_lattice *L, const orc_grid *G, const double *f,
                double *fields) {
  long nc = (long)G->nx * G->ny;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < nc; ++c) {
    double r, ux, uy, T;
    orc_moments(L, f + c, nc, &r, &ux, &uy, &T);
    fields[c] = r;
    fields[nc + c] = ux;
    fields[2 * nc + c] = uy;
    fields[3 * nc + c] = T;
  }
}

void orc_totals(const orc_lattice *L, const orc_grid *G, const double *f,
                double *totals) {
  int nx = G->nx, ny = G->ny;
  long nc = (long)nx * ny;
  double M = 0.0, Px = 0.0, Py = 0.0, E = 0.0;
  for (int l = 0; l < L->q; ++l) {
    double c2 = L->xi[l][0] * L->xi[l][0] + L->xi[l][1] * L->xi[l][1];
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        double m = f[(long)l * nc + (long)j * nx + i] * G->dy[j];
        M += m;
        Px += L->xi[l][0] * m;
        Py += L->xi[l][1] * m;
        E += 0.5 * c2 * m;
      }
    }
  }
  totals[0] = M;
  totals[1] = Px;
  totals[2] = Py;
  totals[3] = E;
}

double orc_residual(const double *q, const double *qprev, long n, int K) {
  double num = 0.0, den = 0.0;
  for (long i = 0; i < n; ++i) {
    double d = q[i] - qprev[i];
    num += d * d;
    den += q[i] * q[i];
  }
  return sqrt(num) / ((double)K * sqrt(den));
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops that follow (n >= 1); for timing only. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
