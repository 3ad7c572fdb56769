// tvlbm_fv_api.cpp -- C ABI of include/tvlbm_fv.h: mesh set-up, wall
// re-emission constants and the two-launch finite-volume step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/tvlbm_fv.h"
#include "tvlbm_core.h"
#include "tvlbm_fv_launch.h"
#include "tvlbm_hostlat.h"
#include "tvlbm_launch.h"
#include "tvlbm_tables.h"

using namespace tvlbm;

struct tvlbm_fv {
  tvlbm_fv_desc d{};
  HostLattice hl;
  bool f64 = false, comp = true;
  int64_t ld = 0, plane = 0;
  hipStream_t st = nullptr;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buf[cur] holds the state
  int64_t step = 0;
  std::vector<double> cyh, volh;  // host copies (double)
  void* d_cy = nullptr;           // [ny] in dtype
  double* d_vol = nullptr;        // [ny]
  double* d_part = nullptr;       // block partials of the totals
  double* d_tot = nullptr;        // 4 totals
  void* d_wtab = nullptr;         // [4][QMAX] wall constants in dtype
  int nblocks = 0;
  FvArgs<float> af{};
  FvArgs<double> ad{};
  tvlbm_fv_schedule sched{1, 6, 0};
  double tau_g = 0.0;  // > 0: non-unit-Prandtl term
  int pscale = 0;      // relaxation times divided by the local pressure
  int slip_free = 0;   // wall model: 0 fixed wall equilibrium, 1 Newton-iterated
  int x_open = 0;      // x ends: 0 periodic, 1 zero gradient
  bool nr_cold = true; // the stored wall roots are not valid yet
  double* d_wpar = nullptr;  // [2][nx][2] last wall-equilibrium roots
};

namespace {

// Wall re-emission, eq.(IMPOSITION), in deviations: an outgoing population
// (c.n > 0, n the inward normal) becomes d_l = kap_l + phi_l m with m the
// incoming normal flux of the deviations, phi_l = feq_l(wall) / Z,
// Z = sum_{c.n > 0} |c.n| feq(wall), kap_l = C phi_l - w_l and
// C = sum_{c.n <= 0} |c.n| w (the rest-state part of the incoming flux).
template <typename R>
void wall_constants(const HostLattice& H, double uw, double Tw, int top, R* kap, R* phi) {
  double feq[36];
  host_feq(H, 1.0, uw, 0.0, Tw, feq);
  double z = 0.0, cin = 0.0;
  for (int l = 0; l < H.q; ++l) {
    const double cn = top ? -H.xi[2 * l + 1] : H.xi[2 * l + 1];
    if (cn > 0.0) z += cn * feq[l];
    else cin += -cn * H.w[l];
  }
  for (int l = 0; l < QMAX; ++l) { kap[l] = R(0); phi[l] = R(0); }
  for (int l = 0; l < H.q; ++l) {
    const double cn = top ? -H.xi[2 * l + 1] : H.xi[2 * l + 1];
    if (cn > 0.0) {
      const double p = feq[l] / z;
      phi[l] = (R)p;
      kap[l] = (R)(cin * p - H.w[l]);
    }
  }
}

template <typename R>
void fill_args(tvlbm_fv* v, FvArgs<R>& A) {
  std::memset(&A, 0, sizeof A);
  fill_lat(v->hl, A.lat);
  A.nx = v->d.nx;
  A.ny = v->d.ny;
  A.walls = v->d.y_bc == TVLBM_BC_DIFFUSE_WALLS;
  A.x_open = v->x_open;
  A.collide = v->d.collide != 0;
  A.ld = v->ld;
  A.plane = v->plane;
  A.dt = (R)v->d.dt;
  A.inv_tau = v->d.collide ? (R)(1.0 / v->d.tau) : R(0);
  A.inv_dx = (R)(2.0 / (v->d.dx + v->d.dx));
  A.cy = (const R*)v->d_cy;
  A.vol = v->d_vol;
  A.strips = (v->d.nx + 61) / 62;
  A.seg_rows = v->sched.seg_rows;
  A.segs = (v->d.ny + A.seg_rows - 1) / A.seg_rows;
  A.prefetch = v->sched.prefetch;
  A.wtab = (const double*)v->d_wtab;
  A.tau_ratio = (v->d.collide && v->tau_g > 0.0) ? (R)(v->d.tau / v->tau_g) : R(0);
  A.pscale = v->d.collide ? v->pscale : 0;
  A.slip_free = v->slip_free;
  A.wall_u[0] = v->d.wall_lo_ux;
  A.wall_T[0] = v->d.wall_lo_T;
  A.wall_u[1] = v->d.wall_hi_ux;
  A.wall_T[1] = v->d.wall_hi_T;
  A.wpar = v->d_wpar;
  A.nr_warm = 0;
  if (A.walls) {
    wall_constants<R>(v->hl, v->d.wall_lo_ux, v->d.wall_lo_T, 0, A.kap_lo, A.phi_lo);
    wall_constants<R>(v->hl, v->d.wall_hi_ux, v->d.wall_hi_T, 1, A.kap_hi, A.phi_hi);
  }
}

bool upload_wall_table(tvlbm_fv* v) {
  double t[4 * QMAX];
  wall_constants<double>(v->hl, v->d.wall_lo_ux, v->d.wall_lo_T, 0, t, t + QMAX);
  wall_constants<double>(v->hl, v->d.wall_hi_ux, v->d.wall_hi_T, 1, t + 2 * QMAX, t + 3 * QMAX);
  return hipMemcpy(v->d_wtab, t, sizeof t, hipMemcpyHostToDevice) == hipSuccess;
}

template <typename R>
FvArgs<R>& args_of(tvlbm_fv* v);
template <>
FvArgs<float>& args_of<float>(tvlbm_fv* v) { return v->af; }
template <>
FvArgs<double>& args_of<double>(tvlbm_fv* v) { return v->ad; }

template <typename R>
int launch(tvlbm_fv* v, int what, const void* src, void* dst, void* fields, double* partials) {
  FvArgs<R> A = args_of<R>(v);
  A.src = (const R*)src;
  A.dst = (R*)dst;
  A.om = (R*)v->d.omega;
  return launch_fv(v->hl.n, v->hl.order, v->comp, what, A, (R*)fields, partials, v->st) == hipSuccess
             ? TVLBM_OK
             : TVLBM_EHIP;
}

int run(tvlbm_fv* v, int what, const void* src, void* dst, void* fields = nullptr,
        double* partials = nullptr);

// the wall model on the state in dst; Newton from last step's roots when
// they are valid
int impose_walls(tvlbm_fv* v, void* dst) {
  v->af.nr_warm = v->ad.nr_warm = v->nr_cold ? 0 : 1;
  const int rc = run(v, FV_IMPOSE, nullptr, dst);
  v->af.nr_warm = v->ad.nr_warm = 0;
  if (rc == TVLBM_OK && v->slip_free) v->nr_cold = false;
  return rc;
}

int run(tvlbm_fv* v, int what, const void* src, void* dst, void* fields,
        double* partials) {
  return v->f64 ? launch<double>(v, what, src, dst, fields, partials)
                : launch<float>(v, what, src, dst, fields, partials);
}

}  // namespace

extern "C" {

int tvlbm_fv_init(const tvlbm_fv_desc* d, tvlbm_fv** out) {
  if (!d || !out) return TVLBM_EINVAL;
  *out = nullptr;
  if (d->dtype != TVLBM_F32 && d->dtype != TVLBM_F64) return TVLBM_EINVAL;
  const int walls = d->y_bc == TVLBM_BC_DIFFUSE_WALLS;
  if (d->y_bc != TVLBM_BC_PERIODIC && !walls) return TVLBM_EINVAL;
  if (d->nx < 2 || d->ny < (walls ? 3 : 2)) return TVLBM_EINVAL;
  if (!(d->dx > 0.0) || !std::isfinite(d->dx) || !(d->dt > 0.0) || !std::isfinite(d->dt))
    return TVLBM_EINVAL;
  if (d->collide && !(d->tau > 0.0)) return TVLBM_EINVAL;
  if (!d->f_a || !d->f_b || !d->omega || d->f_a == d->f_b || d->omega == d->f_a ||
      d->omega == d->f_b)
    return TVLBM_EINVAL;
  const int ns = walls ? d->ny - 1 : d->ny;
  std::vector<double> dy(ns, d->dx);
  if (d->dy)
    for (int j = 0; j < ns; ++j) {
      dy[j] = d->dy[j];
      if (!(dy[j] > 0.0) || !std::isfinite(dy[j])) return TVLBM_EINVAL;
    }
  tvlbm_fv* v = new (std::nothrow) tvlbm_fv();
  if (!v) return TVLBM_ENOMEM;
  if (!build_lattice(d->n_gh, d->eq_order, 0.9, 0, &v->hl)) { delete v; return TVLBM_EUNSUPPORTED; }
  v->d = *d;
  v->d.dy = nullptr;
  v->f64 = d->dtype == TVLBM_F64;
  v->comp = v->f64 ? false : d->compensated != 0;
  v->ld = d->ld ? d->ld : (d->nx + 63) / 64 * 64;
  if (v->ld < d->nx) { delete v; return TVLBM_EINVAL; }
  v->plane = (int64_t)d->ny * v->ld;
  if ((double)v->hl.q * (double)v->plane * (v->f64 ? 8.0 : 4.0) >= 4294967296.0) {
    delete v;
    return TVLBM_EUNSUPPORTED;
  }
  v->st = (hipStream_t)d->stream;
  v->buf[0] = d->f_a;
  v->buf[1] = d->f_b;
  // y-derivative factors 2 / (dy_{j-1} + dy_j), one-sided 2 / dy at walls,
  // and the dual-cell weights of the totals
  const int ny = d->ny;
  v->cyh.assign(ny, 0.0);
  v->volh.assign(ny, 0.0);
  for (int j = 0; j < ny; ++j) {
    double h;
    if (!walls) {
      const double dm = dy[(j - 1 + ny) % ny];
      v->cyh[j] = 2.0 / (dy[j] + dm);
      h = 0.5 * (dm + dy[j]);
    } else if (j == 0) {
      v->cyh[j] = 2.0 / dy[0];
      h = 0.5 * dy[0];
    } else if (j == ny - 1) {
      v->cyh[j] = 2.0 / dy[ny - 2];
      h = 0.5 * dy[ny - 2];
    } else {
      v->cyh[j] = 2.0 / (dy[j] + dy[j - 1]);
      h = 0.5 * (dy[j - 1] + dy[j]);
    }
    v->volh[j] = d->dx * h;
  }
  v->nblocks = (int)(((d->nx + 63) / 64) * ((ny + 3) / 4));
  const size_t esz = v->f64 ? 8 : 4;
  bool ok = hipMalloc(&v->d_cy, esz * ny) == hipSuccess &&
            hipMalloc(&v->d_vol, sizeof(double) * ny) == hipSuccess &&
            hipMalloc(&v->d_part, sizeof(double) * 4 * v->nblocks) == hipSuccess &&
            hipMalloc(&v->d_tot, sizeof(double) * 4) == hipSuccess &&
            hipMalloc(&v->d_wtab, sizeof(double) * 4 * QMAX) == hipSuccess &&
            hipMalloc(&v->d_wpar, sizeof(double) * 4 * d->nx) == hipSuccess;
  if (ok) {
    if (v->f64) {
      ok = hipMemcpy(v->d_cy, v->cyh.data(), 8 * ny, hipMemcpyHostToDevice) == hipSuccess;
    } else {
      std::vector<float> c(v->cyh.begin(), v->cyh.end());
      ok = hipMemcpy(v->d_cy, c.data(), 4 * ny, hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && hipMemcpy(v->d_vol, v->volh.data(), 8 * ny, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok) { tvlbm_fv_destroy(v); return TVLBM_ENOMEM; }
  fill_args(v, v->af);
  fill_args(v, v->ad);
  if (!upload_wall_table(v)) { tvlbm_fv_destroy(v); return TVLBM_EHIP; }
  *out = v;
  return TVLBM_OK;
}

int tvlbm_fv_destroy(tvlbm_fv* v) {
  if (!v) return TVLBM_EINVAL;
  if (v->st) hipStreamSynchronize(v->st);
  hipFree(v->d_cy);
  hipFree(v->d_vol);
  hipFree(v->d_part);
  hipFree(v->d_tot);
  hipFree(v->d_wtab);
  hipFree(v->d_wpar);
  delete v;
  return TVLBM_OK;
}

int tvlbm_fv_set_fields(tvlbm_fv* v, const void* rho, const void* ux, const void* uy,
                        const void* T, const void* noise) {
  if (!v || !rho || !ux || !uy || !T) return TVLBM_EINVAL;
  // f = feq(fields) + noise as deviations
  hipError_t e;
  if (v->f64) {
    FvArgs<double> A = v->ad;
    A.dst = (double*)v->buf[0];
    const FvInit<double> I{(const double*)rho, (const double*)ux, (const double*)uy,
                           (const double*)T, (const double*)noise};
    e = launch_fv_init(v->hl.n, v->hl.order, A, I, v->st);
  } else {
    FvArgs<float> A = v->af;
    A.dst = (float*)v->buf[0];
    const FvInit<float> I{(const float*)rho, (const float*)ux, (const float*)uy, (const float*)T,
                          (const float*)noise};
    e = launch_fv_init(v->hl.n, v->hl.order, A, I, v->st);
  }
  if (e != hipSuccess) return TVLBM_EHIP;
  v->cur = 0;
  v->step = 0;
  v->nr_cold = true;
  return impose_walls(v, v->buf[0]);
}

int tvlbm_fv_step(tvlbm_fv* v, int32_t nsteps) {
  if (!v || nsteps < 0) return TVLBM_EINVAL;
  for (int32_t s = 0; s < nsteps; ++s) {
    if (v->sched.fused) {
      const int rc = run(v, v->sched.fused == 2 ? FV_BAND : FV_MARCH, v->buf[v->cur],
                         v->buf[v->cur ^ 1]);
      if (rc) return rc;
    } else {
      int rc = run(v, FV_OMEGA, v->buf[v->cur], nullptr);
      if (rc) return rc;
      rc = run(v, FV_UPDATE, v->buf[v->cur], v->buf[v->cur ^ 1]);
      if (rc) return rc;
    }
    if (v->slip_free && v->d.y_bc == TVLBM_BC_DIFFUSE_WALLS) {
      const int rc = impose_walls(v, v->buf[v->cur ^ 1]);
      if (rc) return rc;
    }
    v->cur ^= 1;
    ++v->step;
  }
  return TVLBM_OK;
}

int tvlbm_fv_populations(tvlbm_fv* v, void* out) {
  if (!v || !out) return TVLBM_EINVAL;
  return run(v, FV_POPS, v->buf[v->cur], nullptr, out);
}

int tvlbm_fv_moments(tvlbm_fv* v, void* rho, void* ux, void* uy, void* T, double* totals) {
  if (!v) return TVLBM_EINVAL;
  const size_t esz = v->f64 ? 8 : 4;
  const int64_t np = (int64_t)v->d.nx * v->d.ny;
  void* fld = nullptr;
  const bool want = rho || ux || uy || T;
  if (want && hipMallocAsync(&fld, esz * 4 * np, v->st) != hipSuccess) return TVLBM_ENOMEM;
  int rc = run(v, FV_FIELDS, v->buf[v->cur], nullptr, fld, v->d_part);
  if (rc == TVLBM_OK && launch_reduce(v->d_part, v->nblocks, 4, v->d_tot, v->st) != hipSuccess)
    rc = TVLBM_EHIP;
  void* outs[4] = {rho, ux, uy, T};
  for (int k = 0; k < 4 && rc == TVLBM_OK && want; ++k)
    if (outs[k] &&
        hipMemcpyAsync(outs[k], (char*)fld + k * np * esz, np * esz, hipMemcpyDeviceToDevice,
                       v->st) != hipSuccess)
      rc = TVLBM_EHIP;
  double tot[4] = {0, 0, 0, 0};
  if (rc == TVLBM_OK &&
      hipMemcpyAsync(tot, v->d_tot, sizeof tot, hipMemcpyDeviceToHost, v->st) != hipSuccess)
    rc = TVLBM_EHIP;
  if (fld) hipFreeAsync(fld, v->st);
  if (hipStreamSynchronize(v->st) != hipSuccess && rc == TVLBM_OK) rc = TVLBM_EHIP;
  if (rc == TVLBM_OK && totals) std::memcpy(totals, tot, sizeof tot);
  return rc;
}

int tvlbm_fv_set_schedule(tvlbm_fv* v, const tvlbm_fv_schedule* s) {
  if (!v || !s) return TVLBM_EINVAL;
  if (s->fused == 2 && (v->f64 || v->hl.n > 4)) return TVLBM_EUNSUPPORTED;
  if (s->fused < 0 || s->fused > 2 || s->seg_rows < 0 || s->seg_rows > 65536 ||
      (s->prefetch != 0 && s->prefetch != 1))
    return TVLBM_EINVAL;
  v->sched.fused = s->fused;
  v->sched.prefetch = s->prefetch;
  if (s->seg_rows) v->sched.seg_rows = s->seg_rows;
  fill_args(v, v->af);
  fill_args(v, v->ad);
  return TVLBM_OK;
}

int tvlbm_fv_set_prandtl(tvlbm_fv* v, double tau_g, int32_t pressure_scaled) {
  if (!v || std::isnan(tau_g) || (pressure_scaled != 0 && pressure_scaled != 1)) return TVLBM_EINVAL;
  v->tau_g = (tau_g > 0.0 && std::isfinite(tau_g)) ? tau_g : 0.0;
  v->pscale = pressure_scaled;
  fill_args(v, v->af);
  fill_args(v, v->ad);
  return TVLBM_OK;
}

int tvlbm_fv_set_wall_model(tvlbm_fv* v, int32_t model) {
  if (!v || (model != TVLBM_FV_WALL_DIFFUSE && model != TVLBM_FV_WALL_SLIP_FREE))
    return TVLBM_EINVAL;
  v->slip_free = model == TVLBM_FV_WALL_SLIP_FREE;
  v->nr_cold = true;
  fill_args(v, v->af);
  fill_args(v, v->ad);
  return TVLBM_OK;
}

int tvlbm_fv_set_x_ends(tvlbm_fv* v, int32_t mode) {
  if (!v || (mode != TVLBM_FV_X_PERIODIC && mode != TVLBM_FV_X_ZERO_GRADIENT)) return TVLBM_EINVAL;
  v->x_open = mode == TVLBM_FV_X_ZERO_GRADIENT;
  fill_args(v, v->af);
  fill_args(v, v->ad);
  return TVLBM_OK;
}

int tvlbm_fv_get_schedule(const tvlbm_fv* v, tvlbm_fv_schedule* s) {
  if (!v || !s) return TVLBM_EINVAL;
  *s = v->sched;
  return TVLBM_OK;
}

int tvlbm_fv_step_count(const tvlbm_fv* v, int64_t* k) {
  if (!v || !k) return TVLBM_EINVAL;
  *k = v->step;
  return TVLBM_OK;
}

}  // extern "C"
