/*
 * tvlbm.h -- C ABI of the MI355X (gfx950) TVLBM library.
 *
 * The library advances the thermal volumetric lattice Boltzmann model of
 * Sbragaglia & Sugiyama ("Volumetric formulation of lattice Boltzmann models
 * with energy conservation") on a rectangular grid:
 *
 *   one step = BGK collision toward the Hermite-expanded equilibrium in
 *   (rho, u, T) (Sec. II, eq.(lb), Appendix A), then volumetric streaming:
 *   every population's cell, displaced by s_l = lambda * xi_l cells, is split
 *   over the (at most four) cells it covers in proportion to the exact
 *   overlap area (the volumetric scheme the paper builds on, Sec. I), so mass,
 *   momentum and energy are conserved with off-lattice Gauss-Hermite
 *   velocities.  Optional diffuse walls in y follow eq.(IMPOSITION)
 *   (Sec. VII); optional non-uniform row heights follow the rectangular
 *   meshes of Sec. III.
 *
 * Conventions shared by every entry point
 *   - All functions return TVLBM_OK (0) or a negative TVLBM_E* code;
 *     tvlbm_strerror() names a code, tvlbm_last_error() gives detail.
 *   - Device pointers are borrowed: the caller allocates and frees them and
 *     keeps them alive for the life of the context.  The library owns its
 *     context, host tables and small internal device buffers (reduction
 *     partials, flags, residual snapshots).
 *   - Work is enqueued on the stream given at init (NULL = default stream)
 *     and is asynchronous, except for calls that return host values, which
 *     synchronise that stream.  A context is not thread-safe.
 *   - Velocity numbering: l = a*n + b, a = x node index, b = y node index,
 *     both ascending; xi_l = (x_a, x_b), w_l = w_a w_b (tensor-product
 *     Gauss-Hermite rule, probabilists' weight, sum w = 1).
 *   - Population arrays are structure-of-arrays [q][ny][pitch], x fastest.
 *   - Macroscopic fields are [ny][nx] arrays in the context's dtype.
 *   - State after k steps: f^k, the post-stream, pre-collision populations
 *     (a step is collide, then stream).  The two caller-provided buffers
 *     f_a/f_b hold, internally, post-collision populations minus the lattice
 *     weights (deviation storage); read results through the entry points
 *     below, not from those buffers.
 */
#ifndef TVLBM_H
#define TVLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TVLBM_OK 0
#define TVLBM_EINVAL (-1)        /* bad argument                          */
#define TVLBM_EHIP (-2)          /* a HIP runtime call failed             */
#define TVLBM_ENOMEM (-3)        /* internal allocation failed            */
#define TVLBM_ENONFINITE (-4)    /* rho <= 0, T <= 0 or a non-finite value */
#define TVLBM_EUNSUPPORTED (-5)  /* lattice/order/dtype not built         */
#define TVLBM_ENOTCONVERGED (-6) /* step limit reached before tolerance   */
#define TVLBM_EIO (-7)           /* checkpoint file error                 */

enum { TVLBM_F32 = 0, TVLBM_F64 = 1 };
enum { TVLBM_CFL_EUCLID = 0, TVLBM_CFL_COMPONENT = 1 };
enum { TVLBM_BC_PERIODIC = 0, TVLBM_BC_DIFFUSE_WALLS = 1 };

typedef struct tvlbm_ctx tvlbm_ctx;

typedef struct tvlbm_desc {
  int32_t n_gh;        /* Gauss-Hermite points per axis: 3, 4 or 6 (q = n_gh^2)   */
  int32_t eq_order;    /* Hermite order of the equilibrium: (3,2) (4,3) (6,4)     */
  int32_t dtype;       /* TVLBM_F32 or TVLBM_F64 (storage and arithmetic)         */
  int32_t nx, ny;      /* cells; nx >= 2, ny >= 2                                 */
  int32_t cfl_norm;    /* TVLBM_CFL_EUCLID: cfl = lambda*max|xi_l| (2-norm);      */
                       /* TVLBM_CFL_COMPONENT: cfl = lambda*max|x_a|              */
  int64_t ld;          /* row pitch of f_a/f_b in elements (>= nx); 0 = nx        */
                       /* rounded up to a multiple of 64                          */
  double tau;          /* BGK relaxation time in steps, > 0.5                     */
  double cfl;          /* largest displacement per step, in cells (<= 1 per axis) */
  int32_t collide;     /* 1 normally; 0 = pure streaming                          */
  int32_t y_bc;        /* TVLBM_BC_PERIODIC or TVLBM_BC_DIFFUSE_WALLS             */
  int32_t compensated; /* F32 only: 1 = compensated moment sums, 0 = plain sums   */
  int32_t reserved;    /* must be 0                                               */
  double wall_lo_ux, wall_lo_T; /* wall at y = 0: x velocity, temperature         */
  double wall_hi_ux, wall_hi_T; /* wall at y = H                                  */
  const double *dy;    /* host, ny row heights in cells (x spacing is 1);         */
                       /* NULL = unit rows.  EUNSUPPORTED if a row would need     */
                       /* more than four source rows (Sec. III meshes)            */
  void *f_a, *f_b;     /* device, each q*ny*ld elements of dtype, caller-owned    */
  void *stream;        /* hipStream_t, or NULL for the default stream             */
} tvlbm_desc;

/* Create a context: validates the descriptor, builds the Gauss-Hermite
 * velocity set, displacements and overlap tables, allocates small internal
 * device buffers.  Populations are undefined until tvlbm_set_fields or
 * tvlbm_set_populations.  EINVAL / EUNSUPPORTED / EHIP / ENOMEM. */
int tvlbm_init(const tvlbm_desc *desc, tvlbm_ctx **ctx);
int tvlbm_destroy(tvlbm_ctx *ctx);

/* f^0 = feq(rho, u, T) (Sec. II, Appendix A) + noise, and step counter 0.
 * rho/ux/uy/T: device [ny][nx]; noise: device [q][ny][nx] or NULL. */
int tvlbm_set_fields(tvlbm_ctx *ctx, const void *rho, const void *ux,
                     const void *uy, const void *T, const void *noise);
/* f^0 = f (device [q][ny][nx], absolute populations), step counter 0. */
int tvlbm_set_populations(tvlbm_ctx *ctx, const void *f);

/* Advance nsteps >= 0 steps (asynchronous); see tvlbm_set_variant for the
 * launches a two-step variant makes. */
int tvlbm_step(tvlbm_ctx *ctx, int32_t nsteps);

/* f^k (absolute, pre-collision) into device [q][ny][nx]; asynchronous. */
int tvlbm_populations(tvlbm_ctx *ctx, void *f_out);
/* C(f^k), the post-collision populations, into device [q][ny][nx]. */
int tvlbm_post_collision(tvlbm_ctx *ctx, void *g_out);

/* Moments of f^k: rho, u, T (Sec. II, central form of T) into the device
 * [ny][nx] arrays given (each may be NULL), and the FP64 totals
 * M = sum f dA, P = sum xi f dA, E = 1/2 sum |xi|^2 f dA into totals[4]
 * (host, may be NULL).  Synchronises.  ENONFINITE if any cell has rho <= 0,
 * T <= 0 or a non-finite moment. */
int tvlbm_moments(tvlbm_ctx *ctx, void *rho, void *ux, void *uy, void *T,
                  double totals[4]);

/* For callers that cannot allocate device memory (code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
 * moments of tvlbm_moments without any allocation and without a host
 * synchronisation.  Enqueues on the context's stream only kernels (no
 * memset, no copy), so the call can be captured.
 *   fields: device [4][ny][nx] in the context's dtype (rho, ux, uy, T), or
 *           NULL;
 *   totals: device double[4] (M, Px, Py, E in FP64, as tvlbm_moments), or
 *           NULL;
 *   flag:   device int32, set to 1 if any cell has rho <= 0, T <= 0 or a
 *           non-finite moment and to 0 otherwise, or NULL.
 * Outputs are caller-owned and valid once the stream reaches the call.
 * The per-block partial sums live in a static 2 MiB device array of the
 * library, one per GPU, resolved at tvlbm_init: grids needing more than
 * 65536 partial blocks (more than 67,108,864 cells with uniform rows, at
 * 1024 cells per block; 16,777,216 with non-uniform rows, at 256) are
 * rejected with EINVAL before anything is enqueued.  Calls that overlap on one GPU (several contexts or streams
 * at once) race on that array.  EINVAL also if the current device is not the
 * context's, or the populations are not set.  If the last launch was a
 * two-step one, the call first enqueues the step and the copy kernel that
 * form g^{k-1} (see tvlbm_set_variant).  A captured call reads the buffer
 * that holds the state when it is captured (the two buffers swap at every
 * launch of tvlbm_step): replay it when the context is back in that
 * buffer, e.g. in a graph that also holds the steps, advancing an even
 * number of launches. */
int tvlbm_moments_static(tvlbm_ctx *ctx, void *fields, double *totals, int32_t *flag);

/* Residual r = ||q^k - q^m||_2 / ((k - m) ||q^k||_2), q = stacked
 * (rho, ux, uy, T) over all cells, where m is the step of the previous call
 * (r = +inf on the first call or if no step was taken).  Synchronises. */
int tvlbm_residual(tvlbm_ctx *ctx, double *r);

/* Run until the residual over k_interval steps is below tol, or max_steps.
 * steps_done/r_final (host, may be NULL).  ENOTCONVERGED at the limit.
 * FP32: at every residual check that does not stop the solve, the deviation
 * mass of the state (tallied exactly, in 2^-32 fixed point) is compared
 * with the solve's starting mass and the deficit is added back to the
 * post-collision state as a uniform density increment at rest, delta w_l
 * per cell: FP32 rounding of the collision moves the mass by up to ~1e-9
 * of it per step where T != 1, which would otherwise add up over a long
 * solve.  FP64 runs are left as stepped. */
int tvlbm_solve(tvlbm_ctx *ctx, int64_t max_steps, double tol,
                int32_t k_interval, int64_t *steps_done, double *r_final);

/* Step counter k. */
int tvlbm_step_count(const tvlbm_ctx *ctx, int64_t *k);

/* Lattice tables (host arrays): xi[2q] (Hermite units), w[q],
 * shift[2q] (cells per step, as used by the kernels), lambda. */
int tvlbm_lattice(const tvlbm_ctx *ctx, double *xi, double *w, double *shift,
                  double *lambda);
/* The same tables without a context (host only, no device call): the
 * tensor product of the n_gh-point Gauss-Hermite rule (Sec. II, Appendix A)
 * that tvlbm_init would build for (n_gh, eq_order, cfl, cfl_norm).  Any
 * output may be NULL; xi and shift hold 2 n_gh^2 values, w n_gh^2.
 * EUNSUPPORTED for lattices the kernels do not implement. */
int tvlbm_lattice_table(int32_t n_gh, int32_t eq_order, double cfl, int32_t cfl_norm,
                        double *xi, double *w, double *shift, double *lambda);

/* Checkpoint: a TVLBM_CKPT_HEADER_BYTES header, then the raw state (g^k,
 * then the other buffer, q*ny*ld elements each).  The header (format 2,
 * magic "TVLBMCK2") records every descriptor field that fixes a step's
 * arithmetic: n_gh, eq_order, dtype, nx, ny, y_bc, collide, cfl_norm,
 * compensated (as used: 0 for F64), ld (as used), tau, cfl, the wall
 * velocities and temperatures (recorded as 0 for periodic grids) and an
 * FNV-1a 64-bit hash of the row heights (0 for unit rows), plus the step
 * count.  tvlbm_load restores the state and step count and returns EIO,
 * naming the first differing field in tvlbm_last_error, unless the
 * context's header would be identical (format-1 files are refused). */
#define TVLBM_CKPT_HEADER_BYTES 128
int tvlbm_save(tvlbm_ctx *ctx, const char *path);
int tvlbm_load(tvlbm_ctx *ctx, const char *path);
/* Host only (no device work): the header tvlbm_save would write for a
 * context built from desc at step `step` (out: host, >= out_bytes =
 * TVLBM_CKPT_HEADER_BYTES), and the check tvlbm_load applies to a header
 * read from a file (EIO on any difference; *step, may be NULL, gets the
 * stored step count). */
int tvlbm_ckpt_header(const tvlbm_desc *desc, int64_t step, void *out, int64_t out_bytes);
int tvlbm_ckpt_check(const void *header, int64_t bytes, const tvlbm_desc *desc, int64_t *step);

/* Launch-shape variant of the fused step kernel (rows per wavefront and
 * waves per workgroup); all variants compute identical results, bit for
 * bit.  0 = the default.  tvlbm_num_variants gives the count.  Some
 * variants advance two steps per launch (g^{k+2} from g^k in one sweep,
 * Sec. II's collide-and-stream map applied twice, each population read and
 * written once per two steps) on the grids that kernel covers (uniform
 * rows, periodic or with walls; FP32 with n_gh 3, 4 or 6, FP64 with n_gh 3
 * or 4); elsewhere they run variant 0.
 * tvlbm_step(ctx, n) with such a variant makes floor(n/2) two-step
 * launches and, for odd n, one single step.  After a two-step launch the
 * library has not formed g^{k-1} (from which the populations, moments,
 * residual and checkpoint of step k are taken); the next call that needs it
 * forms it first, with one step into a third population buffer of the
 * library and a copy kernel, bitwise what single steps would have left.
 * Selecting such a variant allocates that buffer (q*ny*ld elements of the
 * context's dtype; ENOMEM if it cannot), so no later call allocates. */
int tvlbm_num_variants(void);
int tvlbm_set_variant(tvlbm_ctx *ctx, int32_t variant);
/* Steps the step kernel advances per launch with the current variant on
 * this grid: 1 or 2, written to *k (host).  EINVAL for NULL arguments. */
int tvlbm_steps_per_launch(const tvlbm_ctx *ctx, int32_t *k);

/* Measurement helper, not part of the method: copies `bytes` (a multiple of
 * 16; src and dst 16-byte aligned, not overlapping) from src to dst on the
 * stream with a grid-stride 16-byte load/store kernel.  Timed on buffers
 * larger than the 256 MB Infinity Cache it gives the HBM read + write rate a
 * streaming kernel reaches on this GPU.  EINVAL on bad arguments. */
int tvlbm_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

const char *tvlbm_strerror(int code);
const char *tvlbm_last_error(const tvlbm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batched steady solves: many independent channels (diffuse walls in y,
 * periodic in x, uniform rows) of different sizes, relaxation times and wall
 * states advanced together, by default two steps per launch.  One persistent grid-stride kernel walks a
 * device-resident work list of (instance, column strip, row segments); every
 * k_interval steps a per-instance residual (same definition as
 * tvlbm_residual) retires the instances below tol and the work list is
 * compacted on the device.  A chunk of k_interval steps plus the residual and
 * compaction is captured once as a HIP graph and replayed; the host reads one
 * counter per replay.
 * ------------------------------------------------------------------------ */
typedef struct tvlbm_batch tvlbm_batch;

typedef struct tvlbm_inst {
  int32_t nx, ny;               /* cells                                     */
  double tau;                   /* relaxation time in steps, > 0.5           */
  double wall_lo_ux, wall_lo_T; /* wall at y = 0                             */
  double wall_hi_ux, wall_hi_T; /* wall at y = H                             */
} tvlbm_inst;

typedef struct tvlbm_batch_desc {
  int32_t n_gh, eq_order, dtype, compensated; /* as in tvlbm_desc            */
  double cfl;
  int32_t cfl_norm;
  int32_t n_inst;
  const tvlbm_inst *inst;       /* host, n_inst entries                      */
  void *arena_a, *arena_b;      /* device, tvlbm_batch_sizes() pop elements  */
  void *stream;                 /* hipStream_t; must not be the null stream  */
} tvlbm_batch_desc;

/* Element counts of one population arena (pop_elems) and of one packed
 * field array (field_elems = sum over instances of 4*nx*ny; instance b's
 * fields [4][ny][nx] = rho, ux, uy, T follow those of instance b-1). */
int tvlbm_batch_sizes(const tvlbm_batch_desc *desc, int64_t *pop_elems,
                      int64_t *field_elems);
int tvlbm_batch_init(const tvlbm_batch_desc *desc, tvlbm_batch **b);
int tvlbm_batch_destroy(tvlbm_batch *b);
/* f^0 = feq(fields) per instance; fields: device, packed as above. */
int tvlbm_batch_set_fields(tvlbm_batch *b, const void *fields);
/* Run every instance until its residual over k_interval (even, >= 2) steps
 * is below tol or it has taken max_steps.  FP32: as tvlbm_solve, the
 * starting mass of every instance that goes on is put back at each check.  steps_out (host, n_inst) gets the
 * steps each instance took, r_out (host, n_inst, may be NULL) its last
 * residual.  Synchronises.  ENOTCONVERGED if any instance hit max_steps.
 * An instance whose state goes non-finite stops at the next check with a
 * NaN residual and the others run on to their own ends; the call then
 * returns ENONFINITE, with steps_out and r_out filled for every instance. */
int tvlbm_batch_run(tvlbm_batch *b, int64_t max_steps, double tol,
                    int32_t k_interval, int64_t *steps_out, double *r_out);
/* Fields of every instance's current state into fields_out (device, packed);
 * synchronises; ENONFINITE as tvlbm_moments (fields_out is written first,
 * so the finite instances' fields are still usable). */
int tvlbm_batch_fields(tvlbm_batch *b, void *fields_out);
/* Launch shape for instances with nx <= max_nx (size class): wavefront strip
 * width (16, 32 or 64 columns) and rows per lane segment.  Results do not
 * depend on the shape. */
int tvlbm_batch_set_shape(tvlbm_batch *b, int32_t max_nx, int32_t width,
                          int32_t rows);

/* Launch tuning of a batched run; results do not depend on it. */
typedef struct tvlbm_batch_tuning {
  int32_t prefetch;    /* 1: step kernel with software-pipelined row loads;  */
                       /* 0: without (fewer registers, more waves resident)  */
  int32_t tail_active; /* > 0: once at most this many instances are still    */
                       /* unconverged, every remaining instance is cut into   */
                       /* items of the tail shape below; 0: never             */
  int32_t tail_width;  /* 16, 32 or 64 columns                               */
  int32_t tail_rows;   /* rows per lane segment, 1..255                      */
  int32_t two_step;    /* 1: two steps per launch (each population read and  */
                       /* written once per two steps) when the lattice has    */
                       /* that kernel (n_gh 3 or 4, or 6 in FP32) and         */
                       /* k_interval >= 4; each k_interval chunk ends with    */
                       /* 4 single steps (2 if k_interval = 2 mod 4); 0: one  */
                       /* step per launch                                     */
  int32_t two_rows;    /* two-step kernel: rows per segment, 1..255 (the tail */
                       /* work list uses tail_rows)                           */
} tvlbm_batch_tuning;
/* Defaults: prefetch 1, tail_active 0, tail shape 64 x 1, two_step 1,
 * two_rows 8.  EINVAL on values outside the ranges above.  Synchronises the
 * batch's stream. */
int tvlbm_batch_set_tuning(tvlbm_batch *b, const tvlbm_batch_tuning *t);
int tvlbm_batch_get_tuning(const tvlbm_batch *b, tvlbm_batch_tuning *t);

#ifdef __cplusplus
}
#endif
#endif /* TVLBM_H */
