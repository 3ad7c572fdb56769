/*
 * tvlbm_oracle.h -- plain FP64 CPU oracle of one TVLBM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * with the HIP path.
 *
 * What it computes (Sbragaglia & Sugiyama, "Volumetric formulation of lattice
 * Boltzmann models with energy conservation"):
 *   - macroscopic moments rho, u, T of the populations (Sec. II, the moment
 *     definitions and the central form of the temperature);
 *   - the Hermite-expanded equilibrium of Sec. II in the explicit scalar
 *     form of Appendix A, orders 2..4;
 *   - single-relaxation BGK collision, eq.(lb), in the explicit form
 *     f* = f - (f - feq)/tau with tau counted in time steps;
 *   - volumetric streaming: each population's cell, shifted by its lattice
 *     displacement s_l = lambda * xi_l, is split over the cells it covers in
 *     proportion to the exact overlap area (the volumetric scheme the paper
 *     builds on, Sec. I); rows may have non-uniform heights (the rectangular
 *     meshes of Sec. III);
 *   - diffuse-scattering walls whose re-emitted populations follow the
 *     flux-weighted wall Maxwellian of eq.(IMPOSITION) (Sec. VII);
 *   - FP64 totals of mass, momentum and energy, and the K-interval residual.
 *
 * Layout: populations are stored f[l][j][i] with l = a*n + b (a = x node
 * index, b = y node index, both ascending), j = row, i = column, pitch nx.
 */
#ifndef TVLBM_ORACLE_H
#define TVLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_QMAX 64
#define ORC_NMAX 8

typedef struct {
  int n;                     /* Gauss-Hermite points per axis              */
  int q;                     /* n*n populations                            */
  int order;                 /* Hermite order of the equilibrium (2..4)    */
  double x[ORC_NMAX];        /* 1-D nodes, ascending                       */
  double wx[ORC_NMAX];       /* 1-D weights, sum 1                         */
  double xi[ORC_QMAX][2];    /* 2-D velocities (Hermite units)             */
  double w[ORC_QMAX];        /* 2-D weights                                */
  double lambda;             /* cells per step per unit velocity           */
  double s[ORC_QMAX][2];     /* displacement per step, in cells            */
} orc_lattice;

/* cfl_norm: 0 = Euclidean |xi| of the fastest velocity, 1 = per component */
int orc_lattice_gh(int n, int order, double cfl, int cfl_norm, orc_lattice *L);

/* 1-D Gauss-Hermite rule (probabilists' weight, normalised to sum 1). */
int orc_gauss_hermite(int n, double *x, double *w);

void orc_feq(const orc_lattice *L, double rho, double ux, double uy, double T,
             double *feq);
void orc_moments(const orc_lattice *L, const double *f, long stride,
                 double *rho, double *ux, double *uy, double *T);

typedef struct {
  int nx, ny;
  double tau;
  int collide;               /* 0 = pure streaming                         */
  int walls;                 /* 0 = periodic in y, 1 = diffuse walls       */
  double ulo, Tlo, uhi, Thi; /* wall equilibria (x velocity, temperature)  */
  /* derived by orc_grid_init */
  double *y;                 /* ny+1 row boundaries, y[0] = 0              */
  double *dy;                /* ny row heights                             */
  int *yk_start;             /* q*(ny+1): CSR start per (l, target row)    */
  int *yk_src;               /* source rows                                */
  double *yk_len;            /* overlap lengths                            */
  double *blo, *ahi;         /* q*ny: length of shifted row below 0/above H */
  double *glo, *ghi;         /* q*ny: ghost-interval overlap per target row */
  double zlo, zhi;           /* flux normalisations of the wall Maxwellians */
  double fw_lo[ORC_QMAX], fw_hi[ORC_QMAX];
} orc_grid;

/* dy: ny row heights (NULL = all 1).  Returns 0 or a negative error. */
int orc_grid_init(const orc_lattice *L, orc_grid *G, int nx, int ny,
                  const double *dy, double tau, int collide, int walls,
                  double ulo, double Tlo, double uhi, double Thi);
void orc_grid_free(orc_grid *G);

/* f = feq(rho,u,T) (+ noise if not NULL); fields are [ny][nx]. */
void orc_set_fields(const orc_lattice *L, const orc_grid *G,
                    const double *rho, const double *ux, const double *uy,
                    const double *T, const double *noise, double *f);
/* post-collision populations f* = C(f), per cell. */
void orc_collide(const orc_lattice *L, const orc_grid *G, const double *f,
                 double *fstar);
/* volumetric streaming of post-collision populations (with walls). */
void orc_stream(const orc_lattice *L, const orc_grid *G, const double *fstar,
                double *fout);
/* one full step f^{k+1} = S(C(f^k)); work has q*nx*ny doubles. */
void orc_step(const orc_lattice *L, const orc_grid *G, const double *f,
              double *fout, double *work);
/* nsteps steps, in place on f. */
void orc_run(const orc_lattice *L, const orc_grid *G, double *f, int nsteps);
/* fields [4][ny][nx] = rho, ux, uy, T */
void orc_fields(const orc_lattice *L, const orc_grid *G, const double *f,
                double *fields);
/* totals[4] = M, Px, Py, E (cell areas dx=1, dy_j) */
void orc_totals(const orc_lattice *L, const orc_grid *G, const double *f,
                double *totals);
/* incident wall mass per column (lo, hi) of post-collision populations. */
void orc_wall_incident(const orc_lattice *L, const orc_grid *G,
                       const double *fstar, double *mlo, double *mhi);
/* emitted mass per ghost column (lo, hi) for the same populations. */
void orc_wall_emitted(const orc_lattice *L, const orc_grid *G,
                      const double *fstar, double *elo, double *ehi);
/* residual ||q - qprev||_2 / (K ||q||_2) over stacked fields, n values. */
double orc_residual(const double *q, const double *qprev, long n, int K);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
