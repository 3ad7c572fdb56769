// tvlbm_api.cpp -- the C ABI of include/tvlbm.h: context set-up, tables,
// launch geometry, residual, checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/tvlbm.h"
#include "tvlbm_core.h"
#include "tvlbm_launch.h"
#include "tvlbm_tables.h"

using namespace tvlbm;

namespace {

struct Variant {
  int width;  // columns per wavefront strip
  int rows;   // rows per lane segment
};
// Launch shapes of the fused step; all compute identical results.
const Variant kVariants[] = {{64, 4}, {64, 2}, {64, 8}, {64, 16}, {64, 1},
                             {32, 4}, {32, 8}, {16, 8}, {16, 16}};
const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Geometry {
  int tiles_x, n_tiles, nblocks;
};

Geometry geometry(int nx, int ny, const Variant& v) {
  Geometry g;
  const int spb = 4 * (64 / v.width);
  const int64_t nseg = ceil_div(ny, v.rows);
  g.tiles_x = (int)ceil_div(nx, v.width);
  g.n_tiles = (int)(g.tiles_x * ceil_div(nseg, spb));
  g.nblocks = (int)(ceil_div(g.n_tiles, 8) * 8);
  return g;
}

}  // namespace

struct tvlbm_ctx {
  tvlbm_desc d{};
  HostLattice hl;
  bool f64 = false, comp = true;
  int64_t ld = 0, plane = 0;
  hipStream_t st = nullptr;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;          // buf[cur] holds g^k; buf[cur^1] holds g^{k-1} (or f^0)
  int64_t step = 0;
  bool initialised = false;
  int variant = 0;
  double* d_part = nullptr;
  int part_cap = 0;
  double* d_tot = nullptr;
  int32_t* d_flag = nullptr;
  void* d_fld[2] = {nullptr, nullptr};
  int fld_cur = 0;
  bool fld_valid = false;
  int64_t fld_step = 0;
  Lat<float> latf{};
  Lat<double> latd{};
  Inst<float> instf{};
  Inst<double> instd{};
  std::string err;
};

static int fail(tvlbm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(c, expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((c), TVLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

template <typename R>
static void fill_lat(const HostLattice& H, Lat<R>& L) {
  std::memset(&L, 0, sizeof L);
  const int n = H.n;
  for (int a = 0; a < n; ++a) {
    // round the pull fraction to the dtype's unit-interval grid so that
    // (1 - p) + p == 1 exactly in that dtype
    const double ulp = std::is_same<R, float>::value ? 0x1p-24 : 0x1p-53;
    const double p = std::nearbyint(H.p[a] / ulp) * ulp;
    L.p[a] = (R)p;
    L.qm[a] = (R)(1.0 - p);
    L.x[a] = (R)H.x[a];
    L.x2[a] = (R)(H.x[a] * H.x[a]);
    L.xd[a] = H.x[a];
  }
  double sw = 0.0;
  for (int l = 0; l < H.q; ++l) {
    const double c2 = H.xi[2 * l] * H.xi[2 * l] + H.xi[2 * l + 1] * H.xi[2 * l + 1];
    L.w[l] = (R)H.w[l];
    L.wd[l] = H.w[l];
    L.cD[l] = (R)(c2 - 2.0);
    L.c4[l] = (R)((c2 * c2 - 8.0 * c2 + 8.0) / 8.0);
    sw += H.w[l];
  }
  L.sumw = sw;
}

// Per-instance constants: relaxation and the wall ghost coefficients.
// Bottom wall (y = 0): incident populations move down (x_b < 0); the
// re-emitted ones (x_b > 0) carry ghost values
//   g_l = (C + m) feqw_l / Z,  Z = sum_{x_b>0} p_b feqw_b-row,
//   C = sum_{x_b<0} p_b w_b  (rest-state part of the incident mass),
// i.e. the flux-weighted wall Maxwellian of eq.(IMPOSITION) with |c.n| dt
// equal to the displacement p_b.  In deviation form g_l - w_l =
// kap_l + phi_l m with phi_l = feqw_l / Z and kap_l = C phi_l - w_l.
template <typename R>
static void fill_inst(const HostLattice& H, double tau, int collide, int walls, double ulo,
                      double Tlo, double uhi, double Thi, int nx, int ny, int64_t ld, int64_t off,
                      int64_t fld, Inst<R>& P) {
  std::memset(&P, 0, sizeof P);
  P.off = off;
  P.ld = ld;
  P.plane = (int64_t)ny * ld;
  P.fld = fld;
  P.nx = nx;
  P.ny = ny;
  P.walls = walls;
  const double om = collide ? 1.0 / tau : 0.0;
  P.omo = (R)(1.0 - om);
  for (int l = 0; l < H.q; ++l) P.oww[l] = (R)(om * H.w[l]);
  if (walls) {
    const int n = H.n;
    double fl[36], fh[36];
    host_feq(H, 1.0, ulo, 0.0, Tlo, fl);
    host_feq(H, 1.0, uhi, 0.0, Thi, fh);
    double zlo = 0.0, zhi = 0.0, clo = 0.0, chi = 0.0;
    for (int b = 0; b < n; ++b) {
      for (int a = 0; a < n; ++a) {
        const int l = a * n + b;
        if (H.x[b] > 0) { zlo += H.p[b] * fl[l]; chi += H.p[b] * H.w[l]; }
        if (H.x[b] < 0) { zhi += H.p[b] * fh[l]; clo += H.p[b] * H.w[l]; }
      }
    }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const int l = a * n + b;
        if (H.x[b] > 0) {
          const double phi = fl[l] / zlo;
          P.phi_lo[l] = (R)phi;
          P.kap_lo[l] = (R)(clo * phi - H.w[l]);
        }
        if (H.x[b] < 0) {
          const double phi = fh[l] / zhi;
          P.phi_hi[l] = (R)phi;
          P.kap_hi[l] = (R)(chi * phi - H.w[l]);
        }
      }
  }
}

template <typename R>
static Lat<R>& lat_of(tvlbm_ctx* c);
template <>
Lat<float>& lat_of<float>(tvlbm_ctx* c) { return c->latf; }
template <>
Lat<double>& lat_of<double>(tvlbm_ctx* c) { return c->latd; }
template <typename R>
static Inst<R>& inst_of(tvlbm_ctx* c);
template <>
Inst<float>& inst_of<float>(tvlbm_ctx* c) { return c->instf; }
template <>
Inst<double>& inst_of<double>(tvlbm_ctx* c) { return c->instd; }

// Launch the fused kernel in a mode.  src is a population buffer (pitch ld).
template <typename R>
static int run_march(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst, void* fields,
                     bool want_totals) {
  const Variant v = kVariants[c->variant];
  const Geometry g = geometry(c->d.nx, c->d.ny, v);
  MarchArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.lat = lat_of<R>(c);
  A.inst = inst_of<R>(c);
  A.width = v.width;
  A.rows = v.rows;
  A.aux = aux;
  A.tiles_x = g.tiles_x;
  A.n_tiles = g.n_tiles;
  A.src = (const R*)src;
  A.dst = (R*)dst;
  A.fields = (R*)fields;
  A.partials = c->d_part;
  A.flag = c->d_flag;
  if (want_totals && g.nblocks > c->part_cap) return fail(c, TVLBM_EINVAL, "partials too small");
  HIPCHK(c, launch_march(c->hl.n, c->comp, mode, A, g.nblocks, c->st));
  if (want_totals) HIPCHK(c, launch_reduce(c->d_part, g.nblocks, 4, c->d_tot, c->st));
  return TVLBM_OK;
}

template <typename R>
static int run_march_any(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst,
                         void* fields, bool want_totals) {
  return run_march<R>(c, mode, aux, src, dst, fields, want_totals);
}

static int march(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst, void* fields,
                 bool want_totals) {
  return c->f64 ? run_march_any<double>(c, mode, aux, src, dst, fields, want_totals)
                : run_march_any<float>(c, mode, aux, src, dst, fields, want_totals);
}

static size_t esize(const tvlbm_ctx* c) { return c->f64 ? 8 : 4; }

extern "C" {

const char* tvlbm_strerror(int code) {
  switch (code) {
    case TVLBM_OK: return "ok";
    case TVLBM_EINVAL: return "invalid argument";
    case TVLBM_EHIP: return "HIP runtime error";
    case TVLBM_ENOMEM: return "out of memory";
    case TVLBM_ENONFINITE: return "non-finite or non-positive moment";
    case TVLBM_EUNSUPPORTED: return "unsupported configuration";
    case TVLBM_ENOTCONVERGED: return "not converged";
    case TVLBM_EIO: return "checkpoint i/o error";
  }
  return "unknown error";
}

const char* tvlbm_last_error(const tvlbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

int tvlbm_num_variants(void) { return kNumVariants; }

int tvlbm_init(const tvlbm_desc* d, tvlbm_ctx** out) {
  if (!d || !out) return TVLBM_EINVAL;
  *out = nullptr;
  tvlbm_ctx* c = new (std::nothrow) tvlbm_ctx();
  if (!c) return TVLBM_ENOMEM;
  auto bad = [&](int code, const char* m) {
    delete c;
    (void)m;
    return code;
  };
  if (d->dtype != TVLBM_F32 && d->dtype != TVLBM_F64) return bad(TVLBM_EINVAL, "dtype");
  if (d->nx < 2 || d->ny < 2) return bad(TVLBM_EINVAL, "size");
  if (d->y_bc != TVLBM_BC_PERIODIC && d->y_bc != TVLBM_BC_DIFFUSE_WALLS) return bad(TVLBM_EINVAL, "y_bc");
  if (d->collide && !(d->tau > 0.5)) return bad(TVLBM_EINVAL, "tau");
  if (!d->f_a || !d->f_b || d->f_a == d->f_b) return bad(TVLBM_EINVAL, "buffers");
  if (d->reserved != 0) return bad(TVLBM_EINVAL, "reserved");
  if (d->dy) {
    for (int j = 0; j < d->ny; ++j)
      if (d->dy[j] != 1.0) return bad(TVLBM_EUNSUPPORTED, "non-uniform rows");
  }
  c->d = *d;
  c->d.dy = nullptr;
  if (!build_lattice(d->n_gh, d->eq_order, d->cfl, d->cfl_norm, &c->hl))
    return bad(TVLBM_EUNSUPPORTED, "lattice");
  c->f64 = d->dtype == TVLBM_F64;
  c->comp = c->f64 ? false : (d->compensated != 0);
  c->ld = d->ld ? d->ld : ceil_div(d->nx, 64) * 64;
  if (c->ld < d->nx) return bad(TVLBM_EINVAL, "ld");
  c->plane = (int64_t)d->ny * c->ld;
  c->st = (hipStream_t)d->stream;
  c->buf[0] = d->f_a;
  c->buf[1] = d->f_b;
  const int walls = d->y_bc == TVLBM_BC_DIFFUSE_WALLS;
  fill_lat(c->hl, c->latf);
  fill_lat(c->hl, c->latd);
  fill_inst(c->hl, d->tau, d->collide, walls, d->wall_lo_ux, d->wall_lo_T, d->wall_hi_ux,
            d->wall_hi_T, d->nx, d->ny, c->ld, 0, 0, c->instf);
  fill_inst(c->hl, d->tau, d->collide, walls, d->wall_lo_ux, d->wall_lo_T, d->wall_hi_ux,
            d->wall_hi_T, d->nx, d->ny, c->ld, 0, 0, c->instd);
  int cap = 1024;  // also covers the residual reduction (<= 1024 blocks)
  for (int v = 0; v < kNumVariants; ++v) cap = std::max(cap, geometry(d->nx, d->ny, kVariants[v]).nblocks);
  c->part_cap = cap;
  const size_t fbytes = (size_t)4 * d->nx * d->ny * esize(c);
  if (hipMalloc(&c->d_part, sizeof(double) * 4 * (size_t)cap) != hipSuccess ||
      hipMalloc(&c->d_tot, sizeof(double) * 4) != hipSuccess ||
      hipMalloc(&c->d_flag, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_fld[0], fbytes) != hipSuccess || hipMalloc(&c->d_fld[1], fbytes) != hipSuccess) {
    hipFree(c->d_part); hipFree(c->d_tot); hipFree(c->d_flag);
    hipFree(c->d_fld[0]); hipFree(c->d_fld[1]);
    return bad(TVLBM_ENOMEM, "scratch");
  }
  if (hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->st) != hipSuccess) {
    tvlbm_destroy(c);
    return TVLBM_EHIP;
  }
  *out = c;
  return TVLBM_OK;
}

int tvlbm_destroy(tvlbm_ctx* c) {
  if (!c) return TVLBM_EINVAL;
  if (c->st) hipStreamSynchronize(c->st); else hipDeviceSynchronize();
  hipFree(c->d_part);
  hipFree(c->d_tot);
  hipFree(c->d_flag);
  hipFree(c->d_fld[0]);
  hipFree(c->d_fld[1]);
  delete c;
  return TVLBM_OK;
}

static int set_common(tvlbm_ctx* c, const void* rho, const void* ux, const void* uy, const void* T,
                      const void* noise, const void* fabs) {
  // f^0 goes to buf[1], g^0 = C(f^0) to buf[0]
  if (c->f64) {
    InitArgs<double> A;
    std::memset(&A, 0, sizeof A);
    A.lat = c->latd; A.inst = c->instd;
    A.rho = (const double*)rho; A.ux = (const double*)ux; A.uy = (const double*)uy; A.T = (const double*)T;
    A.noise = (const double*)noise; A.fabs = (const double*)fabs;
    A.f0 = (double*)c->buf[1]; A.g0 = (double*)c->buf[0];
    HIPCHK(c, launch_init(c->hl.n, false, A, c->st));
  } else {
    InitArgs<float> A;
    std::memset(&A, 0, sizeof A);
    A.lat = c->latf; A.inst = c->instf;
    A.rho = (const float*)rho; A.ux = (const float*)ux; A.uy = (const float*)uy; A.T = (const float*)T;
    A.noise = (const float*)noise; A.fabs = (const float*)fabs;
    A.f0 = (float*)c->buf[1]; A.g0 = (float*)c->buf[0];
    HIPCHK(c, launch_init(c->hl.n, c->comp, A, c->st));
  }
  c->cur = 0;
  c->step = 0;
  c->initialised = true;
  c->fld_valid = false;
  return TVLBM_OK;
}

int tvlbm_set_fields(tvlbm_ctx* c, const void* rho, const void* ux, const void* uy, const void* T,
                     const void* noise) {
  if (!c || !rho || !ux || !uy || !T) return fail(c, TVLBM_EINVAL, "null field");
  return set_common(c, rho, ux, uy, T, noise, nullptr);
}

int tvlbm_set_populations(tvlbm_ctx* c, const void* f) {
  if (!c || !f) return fail(c, TVLBM_EINVAL, "null populations");
  return set_common(c, nullptr, nullptr, nullptr, nullptr, nullptr, f);
}

int tvlbm_step(tvlbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return fail(c, TVLBM_EINVAL, "nsteps");
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  for (int32_t s = 0; s < nsteps; ++s) {
    int rc = march(c, MODE_STEP, 0, c->buf[c->cur], c->buf[c->cur ^ 1], nullptr, false);
    if (rc) return rc;
    c->cur ^= 1;
    ++c->step;
  }
  return TVLBM_OK;
}

// f^k = S(g^{k-1}) from buf[cur^1]; at k = 0 buf[cur^1] holds f^0 itself.
static int aux_from_state(tvlbm_ctx* c, int aux, void* dst, void* fields, bool totals) {
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  if (c->step == 0) aux |= AUX_IDENTITY;
  return march(c, MODE_AUX, aux, c->buf[c->cur ^ 1], dst, fields, totals);
}

int tvlbm_populations(tvlbm_ctx* c, void* f_out) {
  if (!c || !f_out) return fail(c, TVLBM_EINVAL, "null output");
  return aux_from_state(c, AUX_POPS, f_out, nullptr, false);
}

int tvlbm_post_collision(tvlbm_ctx* c, void* g_out) {
  if (!c || !g_out) return fail(c, TVLBM_EINVAL, "null output");
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  return march(c, MODE_AUX, AUX_POPS | AUX_IDENTITY, c->buf[c->cur], g_out, nullptr, false);
}

static int read_flag_and_reset(tvlbm_ctx* c, int32_t* flag) {
  HIPCHK(c, hipMemcpyAsync(flag, c->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (*flag) HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->st));
  return TVLBM_OK;
}

int tvlbm_moments(tvlbm_ctx* c, void* rho, void* ux, void* uy, void* T, double totals[4]) {
  if (!c) return TVLBM_EINVAL;
  void* fld = c->d_fld[c->fld_cur ^ 1];  // scratch slot; the residual snapshot stays intact
  int rc = aux_from_state(c, AUX_FIELDS, nullptr, fld, true);
  if (rc) return rc;
  const size_t plane = (size_t)c->d.nx * c->d.ny * esize(c);
  void* outs[4] = {rho, ux, uy, T};
  for (int k = 0; k < 4; ++k)
    if (outs[k])
      HIPCHK(c, hipMemcpyAsync(outs[k], (char*)fld + k * plane, plane, hipMemcpyDeviceToDevice, c->st));
  double t[4];
  HIPCHK(c, hipMemcpyAsync(t, c->d_tot, sizeof t, hipMemcpyDeviceToHost, c->st));
  int32_t flag = 0;
  rc = read_flag_and_reset(c, &flag);
  if (rc) return rc;
  if (totals) std::memcpy(totals, t, sizeof t);
  if (flag) return fail(c, TVLBM_ENONFINITE, "rho <= 0, T <= 0 or non-finite moment");
  return TVLBM_OK;
}

int tvlbm_residual(tvlbm_ctx* c, double* r) {
  if (!c || !r) return fail(c, TVLBM_EINVAL, "null");
  const int slot = c->fld_cur ^ 1;
  int rc = aux_from_state(c, AUX_FIELDS, nullptr, c->d_fld[slot], true);
  if (rc) return rc;
  double res = std::numeric_limits<double>::infinity();
  const int64_t nval = (int64_t)4 * c->d.nx * c->d.ny;
  if (c->fld_valid && c->step > c->fld_step) {
    const int nblk = (int)std::min<int64_t>(1024, ceil_div(nval, 256));
    if (nblk * 4 > c->part_cap * 4) return fail(c, TVLBM_EINVAL, "partials");
    if (c->f64)
      HIPCHK(c, launch_resid((const double*)c->d_fld[slot], (const double*)c->d_fld[c->fld_cur], nval,
                             c->d_part, nblk, c->st));
    else
      HIPCHK(c, launch_resid((const float*)c->d_fld[slot], (const float*)c->d_fld[c->fld_cur], nval,
                             c->d_part, nblk, c->st));
    HIPCHK(c, launch_reduce(c->d_part, nblk, 2, c->d_tot, c->st));
    double ab[2];
    HIPCHK(c, hipMemcpyAsync(ab, c->d_tot, sizeof ab, hipMemcpyDeviceToHost, c->st));
    int32_t flag = 0;
    rc = read_flag_and_reset(c, &flag);
    if (rc) return rc;
    if (flag) return fail(c, TVLBM_ENONFINITE, "non-finite state");
    res = std::sqrt(ab[0]) / ((double)(c->step - c->fld_step) * std::sqrt(ab[1]));
  } else {
    int32_t flag = 0;
    rc = read_flag_and_reset(c, &flag);
    if (rc) return rc;
    if (flag) return fail(c, TVLBM_ENONFINITE, "non-finite state");
  }
  c->fld_cur = slot;
  c->fld_valid = true;
  c->fld_step = c->step;
  *r = res;
  return TVLBM_OK;
}

int tvlbm_solve(tvlbm_ctx* c, int64_t max_steps, double tol, int32_t k_interval,
                int64_t* steps_done, double* r_final) {
  if (!c || k_interval < 1 || max_steps < 0) return fail(c, TVLBM_EINVAL, "solve args");
  double r = std::numeric_limits<double>::infinity();
  int rc = tvlbm_residual(c, &r);  // snapshot of the starting state
  if (rc) return rc;
  const int64_t start = c->step;
  while (c->step - start < max_steps) {
    const int32_t k = (int32_t)std::min<int64_t>(k_interval, max_steps - (c->step - start));
    rc = tvlbm_step(c, k);
    if (rc) return rc;
    rc = tvlbm_residual(c, &r);
    if (rc) return rc;
    if (r < tol) break;
  }
  if (steps_done) *steps_done = c->step - start;
  if (r_final) *r_final = r;
  return r < tol ? TVLBM_OK : TVLBM_ENOTCONVERGED;
}

int tvlbm_step_count(const tvlbm_ctx* c, int64_t* k) {
  if (!c || !k) return TVLBM_EINVAL;
  *k = c->step;
  return TVLBM_OK;
}

int tvlbm_lattice(const tvlbm_ctx* c, double* xi, double* w, double* shift, double* lambda) {
  if (!c) return TVLBM_EINVAL;
  const int q = c->hl.q;
  if (xi) std::memcpy(xi, c->hl.xi, sizeof(double) * 2 * q);
  if (w) std::memcpy(w, c->hl.w, sizeof(double) * q);
  if (shift) std::memcpy(shift, c->hl.shift, sizeof(double) * 2 * q);
  if (lambda) *lambda = c->hl.lambda;
  return TVLBM_OK;
}

int tvlbm_set_variant(tvlbm_ctx* c, int32_t v) {
  if (!c || v < 0 || v >= kNumVariants) return fail(c, TVLBM_EINVAL, "variant");
  c->variant = v;
  return TVLBM_OK;
}

struct CkptHeader {
  char magic[8];
  int32_t version, n_gh, eq_order, dtype, nx, ny, y_bc, collide;
  int64_t ld, step;
  double tau, cfl;
};

int tvlbm_save(tvlbm_ctx* c, const char* path) {
  if (!c || !path) return TVLBM_EINVAL;
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "TVLBMCK1", 8);
  h.version = 1; h.n_gh = c->d.n_gh; h.eq_order = c->d.eq_order; h.dtype = c->d.dtype;
  h.nx = c->d.nx; h.ny = c->d.ny; h.y_bc = c->d.y_bc; h.collide = c->d.collide;
  h.ld = c->ld; h.step = c->step; h.tau = c->d.tau; h.cfl = c->d.cfl;
  const size_t bytes = (size_t)c->hl.q * c->plane * esize(c);
  std::vector<char> host(bytes);
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(c, TVLBM_EIO, "open for write");
  bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
  for (int k = 0; k < 2 && ok; ++k) {
    if (hipMemcpyAsync(host.data(), c->buf[c->cur ^ k], bytes, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
      std::fclose(fp);
      return fail(c, TVLBM_EHIP, "copy out");
    }
    ok = std::fwrite(host.data(), 1, bytes, fp) == bytes;
  }
  ok = (std::fclose(fp) == 0) && ok;
  return ok ? TVLBM_OK : fail(c, TVLBM_EIO, "write");
}

int tvlbm_load(tvlbm_ctx* c, const char* path) {
  if (!c || !path) return TVLBM_EINVAL;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(c, TVLBM_EIO, "open for read");
  CkptHeader h;
  if (std::fread(&h, sizeof h, 1, fp) != 1 || std::memcmp(h.magic, "TVLBMCK1", 8) != 0 || h.version != 1 ||
      h.n_gh != c->d.n_gh || h.eq_order != c->d.eq_order || h.dtype != c->d.dtype || h.nx != c->d.nx ||
      h.ny != c->d.ny || h.ld != c->ld || h.y_bc != c->d.y_bc || h.tau != c->d.tau || h.cfl != c->d.cfl ||
      h.collide != c->d.collide) {
    std::fclose(fp);
    return fail(c, TVLBM_EIO, "checkpoint does not match this context");
  }
  const size_t bytes = (size_t)c->hl.q * c->plane * esize(c);
  std::vector<char> host(bytes);
  for (int k = 0; k < 2; ++k) {
    if (std::fread(host.data(), 1, bytes, fp) != bytes) {
      std::fclose(fp);
      return fail(c, TVLBM_EIO, "short read");
    }
    if (hipMemcpyAsync(c->buf[k == 0 ? 0 : 1], host.data(), bytes, hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
      std::fclose(fp);
      return fail(c, TVLBM_EHIP, "copy in");
    }
  }
  std::fclose(fp);
  c->cur = 0;
  c->step = h.step;
  c->initialised = true;
  c->fld_valid = false;
  return TVLBM_OK;
}

}  // extern "C"
