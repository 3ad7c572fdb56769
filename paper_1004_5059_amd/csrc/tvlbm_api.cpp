// tvlbm_api.cpp -- the C ABI of include/tvlbm.h: context set-up, tables,
// launch geometry, residual, checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/tvlbm.h"
#include "tvlbm_core.h"
#include "tvlbm_launch.h"
#include "tvlbm_tables.h"
#include "tvlbm_hostlat.h"

using namespace tvlbm;

namespace {

struct Variant {
  int width;     // columns per wavefront strip (lanes; pairs of columns if `pairs`)
  int rows;      // rows per lane segment
  int prefetch;  // software-pipelined rows
  int pairs;     // FP32 step on two adjacent columns per lane (8-byte accesses);
                 // grids it does not apply to run the same shape one column per lane
  int two;       // two steps per launch (k_march2, rows = output rows per segment)
                 // where it applies; single steps and other grids run variant 0
};
// Launch shapes of the fused step; all compute identical results.  Variant
// 0 is the default.
const Variant kVariants[] = {{64, 4, 0}, {64, 2, 1}, {64, 8, 1}, {64, 16, 1}, {64, 4, 1},
                             {64, 8, 0}, {32, 8, 1}, {32, 16, 1}, {16, 16, 1}, {64, 2, 0},
                             {32, 8, 0}, {64, 16, 0}, {64, 32, 0}, {32, 16, 0},
                             {64, 4, 0, 1}, {64, 8, 0, 1}, {64, 2, 0, 1}, {64, 16, 0, 1},
                             {32, 8, 0, 1},
                             {64, 3, 0, 0, 1}, {64, 4, 0, 0, 1}, {64, 5, 0, 0, 1},
                             {64, 6, 0, 0, 1}, {64, 8, 0, 0, 1},
                             // longer two-step segments: fewer wavefronts, so that a
                             // lattice at two waves per SIMD (D2Q36) fills one round
                             {64, 7, 0, 0, 1}, {64, 9, 0, 0, 1}, {64, 10, 0, 0, 1},
                             {64, 12, 0, 0, 1}};
const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Geometry {
  int tiles_x, n_tiles, nblocks;
};

// Non-uniform-row kernel: 64 columns x 4 rows per workgroup.
Geometry geometry_rows(int nx, int ny) {
  Geometry g;
  g.tiles_x = (int)ceil_div(nx, 64);
  g.n_tiles = (int)(g.tiles_x * ceil_div(ny, 4));
  g.nblocks = (int)(ceil_div(g.n_tiles, 8) * 8);
  return g;
}

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
  int cur = 0;          // buf[cur] holds g^k; buf[cur^1] holds g^{k-1} (or f^0),
                        // or g^{k-2} while `pending`
  bool pending = false; // the last launch was a two-step one: g^{k-1} not formed yet
  void* buf3 = nullptr; // library-owned population buffer for forming g^{k-1}
                        // (allocated when a two-step variant is selected)
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
  // non-uniform rows
  bool rows = false;
  void* d_taps = nullptr;
  void* d_inc = nullptr;
  double* d_dy = nullptr;
  int32_t* d_rowflag = nullptr;
  int inc_rows = 0;     // longest list of rows crossing a wall (entries used in d_inc)
  std::vector<double> dyh;
  int dev = 0;          // device current at tvlbm_init
  // fixed-point deviation masses (2^-32 units) of the reference state [0]
  // and of the last residual check [1], and the grid's area, for the mass
  // re-imposition of FP32 steady solves
  unsigned long long* d_mass = nullptr;
  double* d_area = nullptr;
  std::string err;
};

namespace {

double ovl(double a0, double a1, double b0, double b1) {
  const double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  return hi > lo ? hi - lo : 0.0;
}

struct TapD {
  int src[4];
  double w[4];
  double glo, ghi;
};
struct IncD {
  int j[4];
  double len[4];
};

// Overlap tables of the remap on rows of heights dy (x spacing 1): the
// shifted source interval [y_j + s, y_{j+1} + s] against target row k, with
// periodic images when there are no walls, the wall-emission intervals
// [0, s] (bottom, s > 0) and [H - |s|, H] (top, s < 0), and the lengths of
// shifted rows lying beyond a wall.  `p` are the displacements as the kernels
// use them (rounded to the dtype's unit-interval grid), so that on dyadic row
// heights every overlap is exact in the working precision and each source
// row's mass is redistributed exactly.  Returns false if a target row needs
// more than four source rows or more than four rows cross a wall.
bool build_row_tables(const HostLattice& H, const double* p, int ny, const double* dy, bool walls,
                      std::vector<TapD>& taps, std::vector<IncD>& inc, std::vector<int32_t>& flag) {
  const int n = H.n;
  std::vector<double> y(ny + 1, 0.0);
  for (int j = 0; j < ny; ++j) y[j + 1] = y[j] + dy[j];
  const double Hy = y[ny];
  taps.assign((size_t)n * ny, TapD{});
  inc.assign(n, IncD{});
  flag.assign(ny, 0);
  std::vector<int> used(ny, 1);  // longest tap list of each target row
  for (int b = 0; b < n; ++b) {
    const double s = (H.x[b] < 0 ? -1.0 : 1.0) * p[b];
    for (int k = 0; k < ny; ++k) {
      TapD& T = taps[(size_t)b * ny + k];
      int cnt = 0;
      for (int j = 0; j < ny; ++j) {
        const double a0 = (y[j] - y[k]) + s, a1 = (y[j + 1] - y[k]) + s;
        double len = ovl(a0, a1, 0.0, dy[k]);
        if (!walls) len += ovl(a0 - Hy, a1 - Hy, 0.0, dy[k]) + ovl(a0 + Hy, a1 + Hy, 0.0, dy[k]);
        if (len > 0.0) {
          if (cnt == 4) return false;
          T.src[cnt] = j;
          T.w[cnt] = len / dy[k];
          ++cnt;
        }
      }
      for (int t = cnt; t < 4; ++t) { T.src[t] = k; T.w[t] = 0.0; }
      used[k] = std::max(used[k], cnt);
      T.glo = T.ghi = 0.0;
      if (walls) {
        if (s > 0.0) T.glo = ovl(-y[k], s - y[k], 0.0, dy[k]) / dy[k];
        if (s < 0.0) T.ghi = ovl((Hy - y[k]) + s, Hy - y[k], 0.0, dy[k]) / dy[k];
        if (T.glo > 0.0) flag[k] |= 1;
        if (T.ghi > 0.0) flag[k] |= 2;
      }
    }
    if (walls) {
      IncD& I = inc[b];
      int cnt = 0;
      for (int j = 0; j < ny; ++j) {
        const double len = s < 0.0 ? ovl(y[j] + s, y[j + 1] + s, -1e300, 0.0)
                                   : ovl((y[j] - Hy) + s, (y[j + 1] - Hy) + s, 0.0, 1e300);
        if (len > 0.0) {
          if (cnt == 4) return false;
          I.j[cnt] = j;
          I.len[cnt] = len;
          ++cnt;
        }
      }
      for (int t = cnt; t < 4; ++t) { I.j[t] = 0; I.len[t] = 0.0; }
    }
  }
  // the kernels read this many entries of every tap list of the row (the
  // used ones come first; the rest have weight 0)
  for (int k = 0; k < ny; ++k) flag[k] |= (used[k] - 1) << 2;
  return true;
}

template <typename R>
int upload_rows(tvlbm_ctx* c, const std::vector<TapD>& taps, const std::vector<IncD>& inc,
                const std::vector<int32_t>& flag) {
  std::vector<RowTap<R>> t(taps.size());
  for (size_t k = 0; k < taps.size(); ++k) {
    std::memset(&t[k], 0, sizeof t[k]);
    for (int q = 0; q < 4; ++q) { t[k].src[q] = taps[k].src[q]; t[k].w[q] = (R)taps[k].w[q]; }
    t[k].glo = (R)taps[k].glo;
    t[k].ghi = (R)taps[k].ghi;
  }
  std::vector<IncRows<R>> in(inc.size());
  for (size_t b = 0; b < inc.size(); ++b)
    for (int q = 0; q < 4; ++q) { in[b].j[q] = inc[b].j[q]; in[b].len[q] = (R)inc[b].len[q]; }
  if (hipMalloc(&c->d_taps, sizeof(RowTap<R>) * t.size()) != hipSuccess ||
      hipMalloc(&c->d_inc, sizeof(IncRows<R>) * in.size()) != hipSuccess ||
      hipMalloc(&c->d_dy, sizeof(double) * c->dyh.size()) != hipSuccess ||
      hipMalloc(&c->d_rowflag, sizeof(int32_t) * flag.size()) != hipSuccess)
    return TVLBM_ENOMEM;
  if (hipMemcpy(c->d_taps, t.data(), sizeof(RowTap<R>) * t.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_inc, in.data(), sizeof(IncRows<R>) * in.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_dy, c->dyh.data(), sizeof(double) * c->dyh.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_rowflag, flag.data(), sizeof(int32_t) * flag.size(), hipMemcpyHostToDevice) != hipSuccess)
    return TVLBM_EHIP;
  return TVLBM_OK;
}

}  // namespace

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

// Per-instance constants: relaxation and the wall ghost coefficients.
// Bottom wall (y = 0): incident populations move down (x_b < 0); the
// re-emitted ones (x_b > 0) carry ghost values
//   g_l = (C + m) feqw_l / Z,  Z = sum_{x_b>0} p_b feqw_b-row,
//   C = sum_{x_b<0} p_b w_b  (rest-state part of the incident mass),
// i.e. the flux-weighted wall Maxwellian of eq.(IMPOSITION) with |c.n| dt
// equal to the displacement p_b.  In deviation form g_l - w_l =
// kap_l + phi_l m with phi_l = feqw_l / Z and kap_l = C phi_l - w_l.
template <typename R>
static double pull_frac(const HostLattice& H, int a) {
  const double ulp = std::is_same<R, float>::value ? 0x1p-24 : 0x1p-53;
  return std::nearbyint(H.p[a] / ulp) * ulp;
}

// Wall coefficients of the emitting populations (one wall) rounded to R so
// that the emitted deviation mass equals the incident one in exact
// arithmetic of the rounded values: sum_l p_l kap_l = 0 and
// sum_l p_l phi_l = 1, p_l the displacement of population l across the wall.
// The rounding residual is absorbed by the last emitting population.
template <typename R>
static void balance_wall(const std::vector<int>& ls, const std::vector<double>& pl,
                         const double* kap, const double* phi, R* kap_out, R* phi_out) {
  double sk = 0.0, sp = 0.0;
  for (size_t t = 0; t + 1 < ls.size(); ++t) {
    kap_out[ls[t]] = (R)kap[ls[t]];
    phi_out[ls[t]] = (R)phi[ls[t]];
    sk += pl[t] * (double)kap_out[ls[t]];
    sp += pl[t] * (double)phi_out[ls[t]];
  }
  const int last = ls.back();
  kap_out[last] = (R)(-sk / pl.back());
  phi_out[last] = (R)((1.0 - sp) / pl.back());
}

// Per-instance constants: relaxation and the wall ghost coefficients.
// Bottom wall (y = 0): incident populations move down (x_b < 0); the
// re-emitted ones (x_b > 0) carry ghost values
//   g_l = (C + m) feqw_l / Z,  Z = sum_{x_b>0} p_b feqw_l,
//   C = sum_{x_b<0} p_b w_l  (rest-state part of the incident mass),
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
      const double pb = pull_frac<R>(H, b);
      for (int a = 0; a < n; ++a) {
        const int l = a * n + b;
        if (H.x[b] > 0) { zlo += pb * fl[l]; chi += pb * H.w[l]; }
        if (H.x[b] < 0) { zhi += pb * fh[l]; clo += pb * H.w[l]; }
      }
    }
    double klo[36] = {0}, plo[36] = {0}, khi[36] = {0}, phi[36] = {0};
    std::vector<int> llo, lhi;
    std::vector<double> plo_w, phi_w;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const int l = a * n + b;
        if (H.x[b] > 0) {
          plo[l] = fl[l] / zlo;
          klo[l] = clo * plo[l] - H.w[l];
          llo.push_back(l);
          plo_w.push_back(pull_frac<R>(H, b));
        }
        if (H.x[b] < 0) {
          phi[l] = fh[l] / zhi;
          khi[l] = chi * phi[l] - H.w[l];
          lhi.push_back(l);
          phi_w.push_back(pull_frac<R>(H, b));
        }
      }
    balance_wall<R>(llo, plo_w, klo, plo, P.kap_lo, P.phi_lo);
    balance_wall<R>(lhi, phi_w, khi, phi, P.kap_hi, P.phi_hi);
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
// The column-pair step applies to FP32 grids periodic in y with uniform rows
// and an even width and pitch.
static bool pairs_ok(const tvlbm_ctx* c) {
  return !c->f64 && !c->rows && c->d.y_bc == TVLBM_BC_PERIODIC && c->d.nx % 2 == 0 && c->ld % 2 == 0;
}

// Two steps per launch: periodic in y, uniform rows; FP32 D2Q9/D2Q16/D2Q36,
// FP64 D2Q9/D2Q16 (FP64 D2Q36 would not fit the register file).
static bool two_ok(const tvlbm_ctx* c) {
  return kVariants[c->variant].two && !c->rows &&
         (c->hl.n == 3 || c->hl.n == 4 || (c->hl.n == 6 && !c->f64));
}

static f32x2 splat2(float v) { return f32x2{v, v}; }

// The single-grid step arguments restated in column-pair units.
static MarchArgs<f32x2> pair_args(const MarchArgs<float>& A) {
  MarchArgs<f32x2> B;
  std::memset(&B, 0, sizeof B);
  for (int k = 0; k < NMAX; ++k) {
    B.lat.p[k] = splat2(A.lat.p[k]);
    B.lat.qm[k] = splat2(A.lat.qm[k]);
    B.lat.x[k] = splat2(A.lat.x[k]);
    B.lat.x2[k] = splat2(A.lat.x2[k]);
    B.lat.xd[k] = A.lat.xd[k];
  }
  for (int l = 0; l < QMAX; ++l) {
    B.lat.w[l] = splat2(A.lat.w[l]);
    B.lat.wd[l] = A.lat.wd[l];
    B.inst.oww[l] = splat2(A.inst.oww[l]);
    B.inst.kap_lo[l] = splat2(A.inst.kap_lo[l]);
    B.inst.phi_lo[l] = splat2(A.inst.phi_lo[l]);
    B.inst.kap_hi[l] = splat2(A.inst.kap_hi[l]);
    B.inst.phi_hi[l] = splat2(A.inst.phi_hi[l]);
  }
  B.lat.sumw = A.lat.sumw;
  B.inst.off = A.inst.off / 2;
  B.inst.plane = A.inst.plane / 2;
  B.inst.ld = A.inst.ld / 2;
  B.inst.fld = A.inst.fld;
  B.inst.nx = A.inst.nx / 2;
  B.inst.ny = A.inst.ny;
  B.inst.walls = A.inst.walls;
  B.inst.id = A.inst.id;
  B.inst.omo = splat2(A.inst.omo);
  B.width = A.width;
  B.rows = A.rows;
  B.src = (const f32x2*)(const void*)A.src;
  B.dst = (f32x2*)(void*)A.dst;
  return B;
}

// Where a march's FP64 block partials, their reduction, the flag and the
// fixed-point mass tally go: the context's own buffers, or
// (tvlbm_moments_static) the library's static scratch and the caller's
// outputs.
struct Sink {
  double* part;
  int part_cap;   // blocks the partials hold
  double* tot;    // reduced totals (4 doubles), or null to skip the reduction
  int32_t* flag;
  bool v0;        // launch shape of variant 0 whatever the context's variant
  unsigned long long* mass = nullptr;  // fixed-point mass tally, or null
};
static Sink ctx_sink(tvlbm_ctx* c) { return Sink{c->d_part, c->part_cap, c->d_tot, c->d_flag, false}; }

template <typename R>
static int run_march(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst, void* fields,
                     bool want_totals, const Sink& k) {
  const Variant v = (k.v0 || kVariants[c->variant].two) ? kVariants[0] : kVariants[c->variant];
  if constexpr (std::is_same<R, float>::value) {
    if (v.pairs && mode == MODE_STEP && pairs_ok(c)) {
      const Geometry g = geometry(c->d.nx / 2, c->d.ny, v);
      MarchArgs<float> A;
      std::memset(&A, 0, sizeof A);
      A.lat = lat_of<float>(c);
      A.inst = inst_of<float>(c);
      A.width = v.width;
      A.rows = v.rows;
      A.src = (const float*)src;
      A.dst = (float*)dst;
      MarchArgs<f32x2> B = pair_args(A);
      B.tiles_x = g.tiles_x;
      B.n_tiles = g.n_tiles;
      HIPCHK(c, launch_march_pairs(c->hl.n, c->comp, B, g.nblocks, c->st));
      return TVLBM_OK;
    }
  }
  const Geometry g = c->rows ? geometry_rows(c->d.nx, c->d.ny) : geometry(c->d.nx, c->d.ny, v);
  MarchArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.lat = lat_of<R>(c);
  A.inst = inst_of<R>(c);
  A.width = v.width;
  A.rows = v.rows;
  A.prefetch = v.prefetch;
  A.aux = aux;
  A.tiles_x = g.tiles_x;
  A.n_tiles = g.n_tiles;
  A.src = (const R*)src;
  A.dst = (R*)dst;
  A.fields = (R*)fields;
  A.partials = k.part;
  A.flag = k.flag;
  A.mass = k.mass;
  if (c->rows) {
    A.taps = (const RowTap<R>*)c->d_taps;
    A.inc = (const IncRows<R>*)c->d_inc;
    A.dy = c->d_dy;
    A.rowflag = c->d_rowflag;
    A.inc_rows = c->inc_rows;
  }
  if (want_totals && g.nblocks > k.part_cap) return fail(c, TVLBM_EINVAL, "partials too small");
  HIPCHK(c, launch_march(c->hl.n, c->comp, mode, A, g.nblocks, c->st));
  if (want_totals && k.tot) HIPCHK(c, launch_reduce(k.part, g.nblocks, 4, k.tot, c->st));
  return TVLBM_OK;
}

static int march(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst, void* fields,
                 bool want_totals, const Sink& k) {
  return c->f64 ? run_march<double>(c, mode, aux, src, dst, fields, want_totals, k)
                : run_march<float>(c, mode, aux, src, dst, fields, want_totals, k);
}
static int march(tvlbm_ctx* c, int mode, int aux, const void* src, void* dst, void* fields,
                 bool want_totals) {
  return march(c, mode, aux, src, dst, fields, want_totals, ctx_sink(c));
}

// g^{k+2} from g^k in one launch (two_ok).
template <typename R>
static int run_march2(tvlbm_ctx* c, const void* src, void* dst) {
  const Variant v = kVariants[c->variant];
  MarchArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.lat = lat_of<R>(c);
  A.inst = inst_of<R>(c);
  const bool walls = c->d.y_bc == TVLBM_BC_DIFFUSE_WALLS;
  A.width = 64;
  A.rows = v.rows;
  // strips of 62 output columns (one halo lane each side), 60 with walls
  A.tiles_x = (int)ceil_div(c->d.nx, walls ? 60 : 62);
  A.n_tiles = (int)(A.tiles_x * ceil_div(ceil_div(c->d.ny, v.rows), 4));
  A.src = (const R*)src;
  A.dst = (R*)dst;
  const int nblocks = (int)(ceil_div(A.n_tiles, 8) * 8);
  if (walls)
    HIPCHK(c, launch_march2w(c->hl.n, c->comp, A, nblocks, c->st));
  else
    HIPCHK(c, launch_march2(c->hl.n, c->comp, A, nblocks, c->st));
  return TVLBM_OK;
}
static int march2(tvlbm_ctx* c, const void* src, void* dst) {
  return c->f64 ? run_march2<double>(c, src, dst) : run_march2<float>(c, src, dst);
}

static size_t esize(const tvlbm_ctx* c) { return c->f64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// Static scratch of tvlbm_moments_static: the per-block FP64 partials of the
// totals (SCRATCH_BLOCKS x 4 doubles, 2 MiB) and a flag word, in a
// file-scope device array, so that the call allocates nothing.  Each device
// the library runs on holds its own copy until the process ends.  In host
// code the array's name is only a stand-in for the device symbol: tvlbm_init
// resolves the array's address on the current device once, with
// hipGetSymbolAddress, and the entry point passes that address (never the
// name) to its kernels.
constexpr int SCRATCH_BLOCKS = 65536;
constexpr int SCRATCH_FLAG = SCRATCH_BLOCKS * 4;  // index of the flag word (as a double slot)
static __device__ __align__(256) double scratch[SCRATCH_BLOCKS * 4 + 32];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Address of `scratch` on the current device (resolved once per device).
static int resolve_scratch(int* dev_out, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return TVLBM_EHIP;
  }
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
    *err = "device ordinal beyond the static scratch table";
    return TVLBM_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return TVLBM_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *dev_out = dev;
  return TVLBM_OK;
}

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

int tvlbm_stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  if (!src || !dst || bytes < 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
    return TVLBM_EINVAL;
  if (bytes == 0) return TVLBM_OK;
  const int64_t n16 = bytes / 16;
  const int nblocks = (int)std::min<int64_t>(ceil_div(n16, 256), 65536);
  return launch_stream_copy(src, dst, n16, nblocks, (hipStream_t)stream) == hipSuccess ? TVLBM_OK
                                                                                     : TVLBM_EHIP;
}

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
  c->d = *d;
  c->d.dy = nullptr;
  if (d->dy) {
    for (int j = 0; j < d->ny; ++j)
      if (!(d->dy[j] > 0.0) || !std::isfinite(d->dy[j])) return bad(TVLBM_EINVAL, "dy");
    c->dyh.assign(d->dy, d->dy + d->ny);
    c->rows = true;
  }
  if (d->eq_order > 4 || !build_lattice(d->n_gh, d->eq_order, d->cfl, d->cfl_norm, &c->hl))
    return bad(TVLBM_EUNSUPPORTED, "lattice");
  c->f64 = d->dtype == TVLBM_F64;
  c->comp = c->f64 ? false : (d->compensated != 0);
  c->ld = d->ld ? d->ld : ceil_div(d->nx, 64) * 64;
  if (c->ld < d->nx) return bad(TVLBM_EINVAL, "ld");
  c->plane = (int64_t)d->ny * c->ld;
  if ((double)c->hl.q * (double)c->plane * (d->dtype == TVLBM_F64 ? 8.0 : 4.0) >= 4294967296.0)
    return bad(TVLBM_EUNSUPPORTED, "population block of 4 GiB or more");
  c->st = (hipStream_t)d->stream;
  c->buf[0] = d->f_a;
  c->buf[1] = d->f_b;
  {
    std::string e;
    const int rc = resolve_scratch(&c->dev, &e);
    if (rc != TVLBM_OK) return bad(rc, e.c_str());
  }
  const int walls = d->y_bc == TVLBM_BC_DIFFUSE_WALLS;
  fill_lat(c->hl, c->latf);
  fill_lat(c->hl, c->latd);
  fill_inst(c->hl, d->tau, d->collide, walls, d->wall_lo_ux, d->wall_lo_T, d->wall_hi_ux,
            d->wall_hi_T, d->nx, d->ny, c->ld, 0, 0, c->instf);
  fill_inst(c->hl, d->tau, d->collide, walls, d->wall_lo_ux, d->wall_lo_T, d->wall_hi_ux,
            d->wall_hi_T, d->nx, d->ny, c->ld, 0, 0, c->instd);
  int cap = 1024;  // also covers the residual reduction (<= 1024 blocks)
  for (int v = 0; v < kNumVariants; ++v) cap = std::max(cap, geometry(d->nx, d->ny, kVariants[v]).nblocks);
  cap = std::max(cap, geometry_rows(d->nx, d->ny).nblocks);
  c->part_cap = cap;
  const size_t fbytes = (size_t)4 * d->nx * d->ny * esize(c);
  if (hipMalloc(&c->d_part, sizeof(double) * 4 * (size_t)cap) != hipSuccess ||
      hipMalloc(&c->d_tot, sizeof(double) * 4) != hipSuccess ||
      hipMalloc(&c->d_flag, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_fld[0], fbytes) != hipSuccess || hipMalloc(&c->d_fld[1], fbytes) != hipSuccess ||
      hipMalloc(&c->d_mass, 2 * sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&c->d_area, sizeof(double)) != hipSuccess) {
    hipFree(c->d_part); hipFree(c->d_tot); hipFree(c->d_flag);
    hipFree(c->d_fld[0]); hipFree(c->d_fld[1]); hipFree(c->d_mass); hipFree(c->d_area);
    return bad(TVLBM_ENOMEM, "scratch");
  }
  {
    double area = 0.0;
    for (int j = 0; j < d->ny; ++j) area += c->dyh.empty() ? 1.0 : c->dyh[j];
    area *= d->nx;
    if (hipMemcpy(c->d_area, &area, sizeof area, hipMemcpyHostToDevice) != hipSuccess) {
      tvlbm_destroy(c);
      return TVLBM_EHIP;
    }
  }
  if (hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->st) != hipSuccess) {
    tvlbm_destroy(c);
    return TVLBM_EHIP;
  }
  if (c->rows) {
    std::vector<TapD> taps;
    std::vector<IncD> inc;
    std::vector<int32_t> flag;
    double pr[8];
    for (int q = 0; q < c->hl.n; ++q) pr[q] = c->f64 ? (double)c->latd.p[q] : (double)c->latf.p[q];
    if (!build_row_tables(c->hl, pr, d->ny, c->dyh.data(), walls != 0, taps, inc, flag)) {
      tvlbm_destroy(c);
      return TVLBM_EUNSUPPORTED;
    }
    // the kernels read this many entries of every list (the used ones come
    // first; the rest have length 0)
    for (const IncD& I : inc)
      for (int t = 0; t < 4; ++t)
        if (I.len[t] > 0.0) c->inc_rows = std::max(c->inc_rows, t + 1);
    const int rc = c->f64 ? upload_rows<double>(c, taps, inc, flag) : upload_rows<float>(c, taps, inc, flag);
    if (rc != TVLBM_OK) {
      tvlbm_destroy(c);
      return rc;
    }
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
  hipFree(c->d_taps);
  hipFree(c->d_inc);
  hipFree(c->d_dy);
  hipFree(c->d_rowflag);
  hipFree(c->d_mass);
  hipFree(c->d_area);
  hipFree(c->buf3);
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
  c->pending = false;
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
  if (two_ok(c) && c->buf3) {
    // two steps per launch; an odd count ends with a single step.  After a
    // two-step launch the other buffer holds g^{k-2}: g^{k-1}, from which
    // the populations and moments of step k are formed, is formed when one
    // of those is asked for (settle)
    for (int32_t p = 0; p < nsteps / 2; ++p) {
      int rc = march2(c, c->buf[c->cur], c->buf[c->cur ^ 1]);
      if (rc) return rc;
      c->cur ^= 1;
      c->step += 2;
      c->pending = true;
    }
    nsteps -= 2 * (nsteps / 2);
  }
  for (int32_t s = 0; s < nsteps; ++s) {
    int rc = march(c, MODE_STEP, 0, c->buf[c->cur], c->buf[c->cur ^ 1], nullptr, false);
    if (rc) return rc;
    c->cur ^= 1;
    ++c->step;
    c->pending = false;
  }
  return TVLBM_OK;
}

// After two-step launches the other buffer holds g^{k-2}.  One step from it
// into the library's third buffer forms g^{k-1} (bitwise what the two-step
// launch formed on the way), which is copied into the other buffer; the
// state is then as after single steps.  Allocates nothing: the third buffer
// exists whenever a two-step launch could have run.
static int settle(tvlbm_ctx* c) {
  if (!c->pending) return TVLBM_OK;
  if (!c->buf3) return fail(c, TVLBM_EINVAL, "internal: no buffer to form g^(k-1) in");
  int rc = march(c, MODE_STEP, 0, c->buf[c->cur ^ 1], c->buf3, nullptr, false);
  if (rc) return rc;
  // a copy kernel, not a runtime copy: tvlbm_moments_static enqueues kernels
  // only (the buffers are multiples of 256 bytes: ld is a multiple of 64)
  const int64_t n16 = (int64_t)c->hl.q * c->plane * (int64_t)esize(c) / 16;
  const int nblocks = (int)std::min<int64_t>(ceil_div(n16, 256), 65536);
  HIPCHK(c, launch_stream_copy(c->buf3, c->buf[c->cur ^ 1], n16, nblocks, c->st));
  c->pending = false;
  return TVLBM_OK;
}

// f^k = S(g^{k-1}) from buf[cur^1]; at k = 0 buf[cur^1] holds f^0 itself.
static int aux_from_state(tvlbm_ctx* c, int aux, void* dst, void* fields, bool totals,
                          unsigned long long* mass = nullptr) {
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  int rc = settle(c);
  if (rc) return rc;
  if (c->step == 0) aux |= AUX_IDENTITY;
  Sink k = ctx_sink(c);
  k.mass = mass;
  return march(c, MODE_AUX, aux, c->buf[c->cur ^ 1], dst, fields, totals, k);
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

int tvlbm_moments_static(tvlbm_ctx* c, void* fields, double* totals, int32_t* flag) {
  if (!c) return TVLBM_EINVAL;
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->dev)
    return fail(c, TVLBM_EINVAL, "the context's device is not the current device");
  double* base = (double*)g_scratch_ptr[dev];
  if (!base) return fail(c, TVLBM_EHIP, "static scratch not resolved on this device");
  const Geometry g = c->rows ? geometry_rows(c->d.nx, c->d.ny) : geometry(c->d.nx, c->d.ny, kVariants[0]);
  if (g.nblocks > SCRATCH_BLOCKS)
    return fail(c, TVLBM_EINVAL,
                "grid too large for tvlbm_moments_static: " + std::to_string(g.nblocks) +
                    " partial blocks, the static scratch holds " + std::to_string(SCRATCH_BLOCKS));
  int rc = settle(c);
  if (rc) return rc;
  int32_t* fl = flag ? flag : (int32_t*)(base + SCRATCH_FLAG);
  HIPCHK(c, launch_fill_i32(fl, 1, 0, c->st));
  const Sink k{base, SCRATCH_BLOCKS, totals, fl, true};
  const int aux = AUX_FIELDS | (c->step == 0 ? AUX_IDENTITY : 0);
  return march(c, MODE_AUX, aux, c->buf[c->cur ^ 1], nullptr, fields, true, k);
}

int tvlbm_residual(tvlbm_ctx* c, double* r) {
  if (!c || !r) return fail(c, TVLBM_EINVAL, "null");
  const int slot = c->fld_cur ^ 1;
  HIPCHK(c, launch_fill_i32((int32_t*)(c->d_mass + 1), 2, 0, c->st));
  int rc = aux_from_state(c, AUX_FIELDS, nullptr, c->d_fld[slot], true, c->d_mass + 1);
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

// FP32 storage: the collision's rounding (lattice constants rounded to
// FP32) shifts the mass by ~1e-9 of it per step where T != 1, which adds up
// over a steady solve of 10^5 steps.  At every residual check the deficit
// against the solve's starting mass, both tallied exactly in fixed point, is
// added back to the post-collision state as delta w_l per cell.  FP64
// conserves to round-off and is left untouched.
static int reimpose_mass(tvlbm_ctx* c) {
  if (c->f64) return TVLBM_OK;
  Inst<float> P = c->instf;
  P.id = 0;
  HIPCHK(c, launch_mass_fix((float*)c->buf[c->cur], nullptr, P, nullptr, c->d_mass, c->d_mass + 1,
                            c->d_area, c->latf, c->hl.q, 1, c->st));
  return TVLBM_OK;
}

int tvlbm_solve(tvlbm_ctx* c, int64_t max_steps, double tol, int32_t k_interval,
                int64_t* steps_done, double* r_final) {
  if (!c || k_interval < 1 || max_steps < 0) return fail(c, TVLBM_EINVAL, "solve args");
  double r = std::numeric_limits<double>::infinity();
  int rc = tvlbm_residual(c, &r);  // snapshot of the starting state
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync(c->d_mass, c->d_mass + 1, sizeof(unsigned long long),
                           hipMemcpyDeviceToDevice, c->st));
  const int64_t start = c->step;
  while (c->step - start < max_steps) {
    const int32_t k = (int32_t)std::min<int64_t>(k_interval, max_steps - (c->step - start));
    rc = tvlbm_step(c, k);
    if (rc) return rc;
    rc = tvlbm_residual(c, &r);
    if (rc) return rc;
    if (r < tol) break;
    rc = reimpose_mass(c);
    if (rc) return rc;
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

int tvlbm_lattice_table(int32_t n_gh, int32_t eq_order, double cfl, int32_t cfl_norm, double* xi,
                        double* w, double* shift, double* lambda) {
  HostLattice hl;
  if (!build_lattice(n_gh, eq_order, cfl, cfl_norm, &hl)) return TVLBM_EUNSUPPORTED;
  const int q = hl.q;
  if (xi) std::memcpy(xi, hl.xi, sizeof(double) * 2 * q);
  if (w) std::memcpy(w, hl.w, sizeof(double) * q);
  if (shift) std::memcpy(shift, hl.shift, sizeof(double) * 2 * q);
  if (lambda) *lambda = hl.lambda;
  return TVLBM_OK;
}

int tvlbm_steps_per_launch(const tvlbm_ctx* c, int32_t* k) {
  if (!c || !k) return TVLBM_EINVAL;
  *k = two_ok(c) ? 2 : 1;
  return TVLBM_OK;
}

int tvlbm_set_variant(tvlbm_ctx* c, int32_t v) {
  if (!c || v < 0 || v >= kNumVariants) return fail(c, TVLBM_EINVAL, "variant");
  c->variant = v;
  if (two_ok(c) && !c->buf3) {
    const size_t bytes = (size_t)c->hl.q * c->plane * esize(c);
    if (hipMalloc(&c->buf3, bytes) != hipSuccess) {
      c->buf3 = nullptr;
      (void)hipGetLastError();
      return fail(c, TVLBM_ENOMEM, "third population buffer for two-step launches");
    }
  }
  return TVLBM_OK;
}

// Checkpoint header, format 2: every descriptor field that fixes the
// arithmetic of a step, so that a state resumes only under the same update.
// Wall data are recorded as zero for periodic grids (they take no part).
struct CkptHeader {
  char magic[8];  // "TVLBMCK2"
  int32_t version;
  int32_t n_gh, eq_order, dtype, nx, ny, y_bc, collide, cfl_norm, compensated;
  int32_t pad;
  int64_t ld, step;
  double tau, cfl;
  double wall_lo_ux, wall_lo_T, wall_hi_ux, wall_hi_T;
  uint64_t rows_hash;  // FNV-1a (64-bit) of the ny row heights' bytes; 0 = unit rows
};
static_assert(sizeof(CkptHeader) == TVLBM_CKPT_HEADER_BYTES, "checkpoint header layout");

static uint64_t rows_hash(const double* dy, int32_t ny) {
  if (!dy) return 0;
  uint64_t h = 1469598103934665603ull;
  const unsigned char* p = (const unsigned char*)dy;
  for (size_t i = 0; i < sizeof(double) * (size_t)ny; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// header of a context built from d (dy: its row heights, or null)
static CkptHeader make_header(const tvlbm_desc& d, const double* dy, int64_t step) {
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, "TVLBMCK2", 8);
  h.version = 2;
  h.n_gh = d.n_gh; h.eq_order = d.eq_order; h.dtype = d.dtype; h.nx = d.nx; h.ny = d.ny;
  h.y_bc = d.y_bc; h.collide = d.collide; h.cfl_norm = d.cfl_norm;
  h.compensated = d.dtype == TVLBM_F64 ? 0 : (d.compensated != 0);
  h.ld = d.ld ? d.ld : ceil_div(d.nx, 64) * 64;
  h.step = step;
  h.tau = d.tau; h.cfl = d.cfl;
  if (d.y_bc == TVLBM_BC_DIFFUSE_WALLS) {
    h.wall_lo_ux = d.wall_lo_ux; h.wall_lo_T = d.wall_lo_T;
    h.wall_hi_ux = d.wall_hi_ux; h.wall_hi_T = d.wall_hi_T;
  }
  h.rows_hash = rows_hash(dy, d.ny);
  return h;
}

// first field in which a stored header differs from `want`, or null
static const char* header_mismatch(const CkptHeader& h, const CkptHeader& want) {
  if (std::memcmp(h.magic, "TVLBMCK1", 8) == 0)
    return "format 1 checkpoint (no cfl_norm, wall or row-height record)";
  if (std::memcmp(h.magic, "TVLBMCK2", 8) != 0 || h.version != 2) return "not a checkpoint of format 2";
#define TVLBM_CKPT_FIELD(f) \
  if (std::memcmp(&h.f, &want.f, sizeof h.f) != 0) return #f;
  TVLBM_CKPT_FIELD(n_gh) TVLBM_CKPT_FIELD(eq_order) TVLBM_CKPT_FIELD(dtype) TVLBM_CKPT_FIELD(nx)
  TVLBM_CKPT_FIELD(ny) TVLBM_CKPT_FIELD(y_bc) TVLBM_CKPT_FIELD(collide) TVLBM_CKPT_FIELD(cfl_norm)
  TVLBM_CKPT_FIELD(compensated) TVLBM_CKPT_FIELD(ld) TVLBM_CKPT_FIELD(tau) TVLBM_CKPT_FIELD(cfl)
  TVLBM_CKPT_FIELD(wall_lo_ux) TVLBM_CKPT_FIELD(wall_lo_T) TVLBM_CKPT_FIELD(wall_hi_ux)
  TVLBM_CKPT_FIELD(wall_hi_T) TVLBM_CKPT_FIELD(rows_hash)
#undef TVLBM_CKPT_FIELD
  return nullptr;
}

int tvlbm_ckpt_header(const tvlbm_desc* desc, int64_t step, void* out, int64_t out_bytes) {
  if (!desc || !out || out_bytes < (int64_t)sizeof(CkptHeader)) return TVLBM_EINVAL;
  const CkptHeader h = make_header(*desc, desc->dy, step);
  std::memcpy(out, &h, sizeof h);
  return TVLBM_OK;
}

int tvlbm_ckpt_check(const void* header, int64_t bytes, const tvlbm_desc* desc, int64_t* step) {
  if (!header || !desc) return TVLBM_EINVAL;
  if (bytes < (int64_t)sizeof(CkptHeader)) return TVLBM_EIO;
  CkptHeader h;
  std::memcpy(&h, header, sizeof h);
  if (header_mismatch(h, make_header(*desc, desc->dy, 0))) return TVLBM_EIO;
  if (step) *step = h.step;
  return TVLBM_OK;
}

int tvlbm_save(tvlbm_ctx* c, const char* path) {
  if (!c || !path) return TVLBM_EINVAL;
  if (!c->initialised) return fail(c, TVLBM_EINVAL, "populations not set");
  if (int rc = settle(c)) return rc;  // the file holds g^k and g^{k-1}
  const CkptHeader h = make_header(c->d, c->rows ? c->dyh.data() : nullptr, c->step);
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
  if (std::fread(&h, sizeof h, 1, fp) != 1) {
    std::fclose(fp);
    return fail(c, TVLBM_EIO, "short header");
  }
  if (const char* what = header_mismatch(h, make_header(c->d, c->rows ? c->dyh.data() : nullptr, 0))) {
    std::fclose(fp);
    return fail(c, TVLBM_EIO, std::string("checkpoint does not match this context: ") + what);
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
  c->pending = false;
  c->step = h.step;
  c->initialised = true;
  c->fld_valid = false;
  return TVLBM_OK;
}

}  // extern "C"

// ==========================================================================
// Batched steady solves
// ==========================================================================
struct tvlbm_batch {
  tvlbm_batch_desc d{};
  std::vector<tvlbm_inst> inst;
  HostLattice hl;
  bool f64 = false, comp = true;
  hipStream_t st = nullptr;
  void* buf[2] = {nullptr, nullptr};
  std::vector<int64_t> off, fld;
  std::vector<int32_t> ld;
  int64_t pop_elems = 0, field_elems = 0;
  void* d_insts = nullptr;
  Work* d_all = nullptr;
  Work* d_work = nullptr;
  int32_t* d_item_start = nullptr;
  double* d_rpart = nullptr;  // residual partials, n_inst * RESID_SLICES * 2
  int32_t* d_nwork = nullptr;
  int32_t* d_ntotal = nullptr;
  int32_t* d_remaining = nullptr;
  int32_t* d_active = nullptr;
  int32_t* d_have_prev = nullptr;
  int64_t* d_steps = nullptr;
  double* d_resid = nullptr;
  int32_t* d_flag = nullptr;
  void* d_fields = nullptr;
  void* d_prev = nullptr;
  // fixed-point deviation masses per instance: at the run's start and at the
  // last check; instance areas (FP32 mass re-imposition, as tvlbm_solve)
  unsigned long long* d_mass0 = nullptr;
  unsigned long long* d_mass = nullptr;
  double* d_area = nullptr;
  int32_t* h_remaining = nullptr;  // pinned
  struct Shape { int max_nx, width, rows; };
  std::vector<Shape> shapes;
  int n_items = 0;
  int items_cap = 0;
  // Tail phase: once at most tail_active instances are unconverged, the
  // work list is rebuilt from items of the single shape (tail_width,
  // tail_rows), which cuts the few remaining grids into more, shorter
  // segments; the arithmetic is the same.
  Work* d_all_tail = nullptr;
  int32_t* d_item_start_tail = nullptr;
  int n_items_tail = 0;
  int tail_cap = 0;
  int prefetch = 1;
  int tail_active = 0, tail_width = 64, tail_rows = 1;
  // Two steps per launch (k_march2_batch): its own bulk and tail work lists
  // (rows per segment two_rows and tail_rows), used when two_step is set,
  // the lattice has the kernel and K is a multiple of 4.
  int two_step = 1, two_rows = 8;
  Work* d_all2 = nullptr;
  int32_t* d_item_start2 = nullptr;
  Work* d_all2_tail = nullptr;
  int32_t* d_item_start2_tail = nullptr;
  int n_items2 = 0, n_items2_tail = 0, items2_cap = 0, tail2_cap = 0;
  bool chunk_two = false;  // kind of the chunks the current graphs hold
  // two-step chunks end with single steps, which walk this second live list
  Work* d_work1 = nullptr;
  int32_t* d_nwork1 = nullptr;
  hipGraphExec_t gexec_tail = nullptr;
  bool initialised = false;
  bool stepped = false;
  hipGraphExec_t gexec = nullptr;
  int g_K = 0;
  double g_tol = 0.0;
  int64_t g_max = 0;
  Lat<float> latf{};
  Lat<double> latd{};
  std::string err;
};

namespace {

int bfail(tvlbm_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

#define BHIP(b, expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return bfail((b), TVLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

int64_t align64(int64_t v) { return (v + 63) / 64 * 64; }

bool batch_layout(const tvlbm_batch_desc* d, int q, std::vector<int64_t>& off,
                  std::vector<int64_t>& fld, std::vector<int32_t>& ld, int64_t& pop,
                  int64_t& field) {
  off.assign(d->n_inst, 0);
  fld.assign(d->n_inst, 0);
  ld.assign(d->n_inst, 0);
  pop = 0;
  field = 0;
  const double esz = d->dtype == TVLBM_F64 ? 8.0 : 4.0;
  for (int b = 0; b < d->n_inst; ++b) {
    const tvlbm_inst& I = d->inst[b];
    if (I.nx < 2 || I.ny < 2) return false;
    ld[b] = (int32_t)((I.nx + 15) / 16 * 16);
    off[b] = pop;
    const int64_t block = (int64_t)q * I.ny * ld[b];
    if ((double)block * esz >= 4294967296.0) return false;
    pop = align64(pop + block);
    fld[b] = field;
    field += (int64_t)4 * I.nx * I.ny;
  }
  return true;
}

const tvlbm_batch::Shape& shape_for(const tvlbm_batch* b, int nx) {
  for (const auto& s : b->shapes)
    if (nx <= s.max_nx) return s;
  return b->shapes.back();
}

// Work items of every instance, each cut into strips of S.width columns and
// segments of S.rows rows; `start` gets each instance's first item.
template <typename ShapeOf>
void make_items(const tvlbm_batch* b, ShapeOf shape_of, std::vector<Work>& all,
                std::vector<int32_t>& start) {
  all.clear();
  start.assign(b->inst.size() + 1, 0);
  for (size_t k = 0; k < b->inst.size(); ++k) {
    start[k] = (int32_t)all.size();
    const tvlbm_inst& I = b->inst[k];
    const tvlbm_batch::Shape S = shape_of(I.nx);
    const int spw = 64 / S.width;
    const int nseg = (I.ny + S.rows - 1) / S.rows;
    for (int x0 = 0; x0 < I.nx; x0 += S.width)
      for (int sg = 0; sg < nseg; sg += spw)
        all.push_back(Work{(int32_t)k, x0, sg, S.width | (S.rows << 8)});
  }
  start[b->inst.size()] = (int32_t)all.size();
}

// Strip width of the two-step kernel for an instance nx columns wide: w
// output columns in a lane group of w + 4 lanes (two halo lanes each side),
// 64 / (w + 4) groups per wavefront.  Picks the w that needs the fewest
// lanes per row, ceil(nx / w) * 64 / G, the widest on ties (less halo).
int strip2_width(int nx) {
  int best_w = 60;
  double best = 1e30;
  for (int w = 60; w >= 4; --w) {
    const int G = 64 / (w + 4);
    const double lanes = (double)((nx + w - 1) / w) * 64.0 / G;
    if (lanes < best - 1e-9) best = lanes, best_w = w;
  }
  return best_w;
}

// Work items of the two-step kernel: strips of w output columns (lane
// groups of Wg = w + 4 lanes) and G = 64 / Wg consecutive segments of
// `rows` rows per item, one per lane group.
void make_items2(const tvlbm_batch* b, int rows, std::vector<Work>& all, std::vector<int32_t>& start) {
  all.clear();
  start.assign(b->inst.size() + 1, 0);
  for (size_t k = 0; k < b->inst.size(); ++k) {
    start[k] = (int32_t)all.size();
    const tvlbm_inst& I = b->inst[k];
    const int w = strip2_width(I.nx), wg = w + 4, G = 64 / wg;
    const int nseg = (I.ny + rows - 1) / rows;
    for (int x0 = 0; x0 < I.nx; x0 += w)
      for (int sg = 0; sg < nseg; sg += G) all.push_back(Work{(int32_t)k, x0, sg, wg | (rows << 8)});
  }
  start[b->inst.size()] = (int32_t)all.size();
}

bool two_kernel(const tvlbm_batch* b) {
  return b->hl.n == 3 || b->hl.n == 4 || (b->hl.n == 6 && !b->f64);
}

void drop_graphs(tvlbm_batch* b) {
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->gexec_tail) hipGraphExecDestroy(b->gexec_tail);
  b->gexec = b->gexec_tail = nullptr;
}

int build_items(tvlbm_batch* b) {
  std::vector<Work> all, tail;
  std::vector<int32_t> start, tail_start;
  make_items(b, [b](int nx) { return shape_for(b, nx); }, all, start);
  b->n_items = (int)all.size();
  b->n_items_tail = 0;
  if (b->tail_active > 0) {
    const tvlbm_batch::Shape T{0, b->tail_width, b->tail_rows};
    make_items(b, [T](int) { return T; }, tail, tail_start);
    b->n_items_tail = (int)tail.size();
  }
  if (b->n_items > b->items_cap) {
    hipFree(b->d_all);
    b->d_all = nullptr;
    BHIP(b, hipMalloc(&b->d_all, sizeof(Work) * b->n_items));
    b->items_cap = b->n_items;
  }
  if (b->n_items_tail > b->tail_cap) {
    hipFree(b->d_all_tail);
    b->d_all_tail = nullptr;
    BHIP(b, hipMalloc(&b->d_all_tail, sizeof(Work) * b->n_items_tail));
    b->tail_cap = b->n_items_tail;
  }
  std::vector<Work> all2, tail2;
  std::vector<int32_t> start2, tail2_start;
  make_items2(b, b->two_rows, all2, start2);
  make_items2(b, b->tail_rows, tail2, tail2_start);
  b->n_items2 = (int)all2.size();
  b->n_items2_tail = (int)tail2.size();
  if (b->n_items2 > b->items2_cap) {
    hipFree(b->d_all2);
    b->d_all2 = nullptr;
    BHIP(b, hipMalloc(&b->d_all2, sizeof(Work) * b->n_items2));
    b->items2_cap = b->n_items2;
  }
  if (b->n_items2_tail > b->tail2_cap) {
    hipFree(b->d_all2_tail);
    b->d_all2_tail = nullptr;
    BHIP(b, hipMalloc(&b->d_all2_tail, sizeof(Work) * b->n_items2_tail));
    b->tail2_cap = b->n_items2_tail;
  }
  BHIP(b, hipMemcpy(b->d_all2, all2.data(), sizeof(Work) * all2.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->d_item_start2, start2.data(), sizeof(int32_t) * start2.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->d_all2_tail, tail2.data(), sizeof(Work) * tail2.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->d_item_start2_tail, tail2_start.data(), sizeof(int32_t) * tail2_start.size(),
                    hipMemcpyHostToDevice));
  // the live work lists: items of any one list / of a one-step list
  hipFree(b->d_work);
  hipFree(b->d_work1);
  b->d_work = b->d_work1 = nullptr;
  const int cap = std::max(std::max(b->n_items, b->n_items_tail), std::max(b->n_items2, b->n_items2_tail));
  BHIP(b, hipMalloc(&b->d_work, sizeof(Work) * cap));
  BHIP(b, hipMalloc(&b->d_work1, sizeof(Work) * std::max(b->n_items, b->n_items_tail)));
  BHIP(b, hipMemcpy(b->d_all, all.data(), sizeof(Work) * all.size(), hipMemcpyHostToDevice));
  BHIP(b, hipMemcpy(b->d_item_start, start.data(), sizeof(int32_t) * start.size(), hipMemcpyHostToDevice));
  if (b->n_items_tail > 0) {
    BHIP(b, hipMemcpy(b->d_all_tail, tail.data(), sizeof(Work) * tail.size(), hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_item_start_tail, tail_start.data(), sizeof(int32_t) * tail_start.size(),
                      hipMemcpyHostToDevice));
  }
  BHIP(b, hipMemcpy(b->d_ntotal, &b->n_items, sizeof(int32_t), hipMemcpyHostToDevice));
  drop_graphs(b);
  return TVLBM_OK;
}

// Persistent grid of the batched step: one wavefront per item up to 2048
// workgroups, rounded to a multiple of 8 for the XCD-contiguous item order.
int batch_blocks(int n_items) {
  return (int)std::min<int64_t>(ceil_div(std::max<int64_t>(ceil_div(n_items, 4), 1), 8) * 8, 2048);
}

template <typename R>
int batch_march(tvlbm_batch* b, int mode, int aux, const void* src, void* dst, const int32_t* nwork,
                const Work* work, int nblocks, unsigned long long* mass) {
  MarchArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.lat = std::is_same<R, float>::value ? *(Lat<R>*)(void*)&b->latf : *(Lat<R>*)(void*)&b->latd;
  A.insts = (const Inst<R>*)b->d_insts;
  A.work = work;
  A.n_work = nwork;
  A.aux = aux;
  A.src = (const R*)src;
  A.dst = (R*)dst;
  A.fields = (R*)b->d_fields;
  A.flag = b->d_flag;
  A.mass = mass;
  BHIP(b, launch_march_batch(b->hl.n, b->comp, mode, b->prefetch != 0, A, nblocks, b->st));
  return TVLBM_OK;
}

int bmarch(tvlbm_batch* b, int mode, int aux, const void* src, void* dst, const int32_t* nwork,
           const Work* work, int nblocks, unsigned long long* mass = nullptr) {
  return b->f64 ? batch_march<double>(b, mode, aux, src, dst, nwork, work, nblocks, mass)
                : batch_march<float>(b, mode, aux, src, dst, nwork, work, nblocks, mass);
}

// Rebuild the live work list from the active instances' items of the bulk
// or the tail list.
int compact(tvlbm_batch* b, bool tail) {
  const int32_t* start1 = tail ? b->d_item_start_tail : b->d_item_start;
  const Work* all1 = tail ? b->d_all_tail : b->d_all;
  if (b->chunk_two) {
    BHIP(b, launch_batch_compact(b->d_active, tail ? b->d_item_start2_tail : b->d_item_start2,
                                 tail ? b->d_all2_tail : b->d_all2, b->d_work, b->d_nwork,
                                 b->d_remaining, (int)b->inst.size(), b->st));
    BHIP(b, launch_batch_compact(b->d_active, start1, all1, b->d_work1, b->d_nwork1, b->d_remaining,
                                 (int)b->inst.size(), b->st));
  } else {
    BHIP(b, launch_batch_compact(b->d_active, start1, all1, b->d_work, b->d_nwork, b->d_remaining,
                                 (int)b->inst.size(), b->st));
  }
  return TVLBM_OK;
}

// Two-step launch over the live work list.
template <typename R>
int batch_march2(tvlbm_batch* b, const void* src, void* dst, int nblocks) {
  MarchArgs<R> A;
  std::memset(&A, 0, sizeof A);
  A.lat = std::is_same<R, float>::value ? *(Lat<R>*)(void*)&b->latf : *(Lat<R>*)(void*)&b->latd;
  A.insts = (const Inst<R>*)b->d_insts;
  A.work = b->d_work;
  A.n_work = b->d_nwork;
  A.src = (const R*)src;
  A.dst = (R*)dst;
  BHIP(b, launch_march2_batch(b->hl.n, b->comp, A, nblocks, b->st));
  return TVLBM_OK;
}

template <typename R>
int batch_resid(tvlbm_batch* b, int K, double tol, int64_t max_steps) {
  BatchCtl<R> C;
  std::memset(&C, 0, sizeof C);
  C.insts = (const Inst<R>*)b->d_insts;
  C.fields = (const R*)b->d_fields;
  C.prev = (R*)b->d_prev;
  C.active = b->d_active;
  C.have_prev = b->d_have_prev;
  C.steps = b->d_steps;
  C.resid = b->d_resid;
  C.flag = b->d_flag;
  C.part = b->d_rpart;
  C.K = K;
  C.tol = tol;
  C.max_steps = max_steps;
  BHIP(b, launch_batch_resid(C, (int)b->inst.size(), b->st));
  return TVLBM_OK;
}

// One chunk: K steps (the last one also writes the fields), the residual
// and the compaction of the work list.  At chunk boundaries every instance's
// post-collision state is in buf[0] (K is even).
int enqueue_chunk(tvlbm_batch* b, int K, double tol, int64_t max_steps, bool tail) {
  const int n = (int)b->inst.size();
  BHIP(b, launch_fill_i32((int32_t*)b->d_mass, 2 * n, 0, b->st));
  if (b->chunk_two) {
    // n2 two-step launches, then n1 single steps (the last one the check):
    // the other buffer ends with g^{K-1}, and n2 + n1 is even, so the state
    // returns to buf[0]
    const int n1 = (K % 4 == 0) ? 4 : 2, n2 = (K - n1) / 2;
    const int nb2 = batch_blocks(tail ? b->n_items2_tail : b->n_items2);
    const int nb1 = batch_blocks(tail ? b->n_items_tail : b->n_items);
    for (int s = 0; s < n2 + n1; ++s) {
      const void* src = b->buf[s & 1];
      void* dst = b->buf[(s & 1) ^ 1];
      int rc;
      if (s < n2) {
        rc = b->f64 ? batch_march2<double>(b, src, dst, nb2) : batch_march2<float>(b, src, dst, nb2);
      } else {
        const int mode = (s == n2 + n1 - 1) ? MODE_CHECK : MODE_STEP;
        rc = bmarch(b, mode, 0, src, dst, b->d_nwork1, b->d_work1, nb1,
                    mode == MODE_CHECK ? b->d_mass : nullptr);
      }
      if (rc) return rc;
    }
  } else {
    const int nblocks = batch_blocks(tail ? b->n_items_tail : b->n_items);
    for (int s = 0; s < K; ++s) {
      const int mode = (s == K - 1) ? MODE_CHECK : MODE_STEP;
      int rc = bmarch(b, mode, 0, b->buf[s & 1], b->buf[(s & 1) ^ 1], b->d_nwork, b->d_work, nblocks,
                      mode == MODE_CHECK ? b->d_mass : nullptr);
      if (rc) return rc;
    }
  }
  int rc = b->f64 ? batch_resid<double>(b, K, tol, max_steps) : batch_resid<float>(b, K, tol, max_steps);
  if (rc) return rc;
  if (!b->f64) {
    // FP32: the instances that go on get their starting mass back (see
    // reimpose_mass); their post-collision state is in buf[0] (K even)
    Inst<float> none;
    std::memset(&none, 0, sizeof none);
    BHIP(b, launch_mass_fix((float*)b->buf[0], (const Inst<float>*)b->d_insts, none, b->d_active,
                            b->d_mass0, b->d_mass, b->d_area, b->latf, b->hl.q, n, b->st));
  }
  return compact(b, tail);
}

// The chunk captured as a graph on the batch's stream.
int capture_chunk(tvlbm_batch* b, int K, double tol, int64_t max_steps, bool tail,
                  hipGraphExec_t* out) {
  BHIP(b, hipStreamSynchronize(b->st));
  BHIP(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_chunk(b, K, tol, max_steps, tail);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->st, &g);
  if (rc) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return bfail(b, TVLBM_EHIP, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) { *out = nullptr; return bfail(b, TVLBM_EHIP, "graph instantiate"); }
  return TVLBM_OK;
}

}  // namespace

extern "C" {

int tvlbm_batch_sizes(const tvlbm_batch_desc* d, int64_t* pop_elems, int64_t* field_elems) {
  if (!d || d->n_inst < 1 || !d->inst) return TVLBM_EINVAL;
  if (!(d->n_gh == 3 || d->n_gh == 4 || d->n_gh == 6)) return TVLBM_EUNSUPPORTED;
  std::vector<int64_t> off, fld;
  std::vector<int32_t> ld;
  int64_t pop, field;
  if (!batch_layout(d, d->n_gh * d->n_gh, off, fld, ld, pop, field)) return TVLBM_EINVAL;
  if (pop_elems) *pop_elems = pop;
  if (field_elems) *field_elems = field;
  return TVLBM_OK;
}

int tvlbm_batch_destroy(tvlbm_batch* b) {
  if (!b) return TVLBM_EINVAL;
  if (b->st) hipStreamSynchronize(b->st);
  drop_graphs(b);
  hipFree(b->d_insts); hipFree(b->d_all); hipFree(b->d_work); hipFree(b->d_item_start);
  hipFree(b->d_all_tail); hipFree(b->d_item_start_tail);
  hipFree(b->d_all2); hipFree(b->d_item_start2); hipFree(b->d_all2_tail); hipFree(b->d_item_start2_tail);
  hipFree(b->d_rpart); hipFree(b->d_nwork); hipFree(b->d_nwork1); hipFree(b->d_work1); hipFree(b->d_ntotal); hipFree(b->d_remaining);
  hipFree(b->d_active); hipFree(b->d_have_prev); hipFree(b->d_steps); hipFree(b->d_resid);
  hipFree(b->d_flag); hipFree(b->d_fields); hipFree(b->d_prev);
  hipFree(b->d_mass0); hipFree(b->d_mass); hipFree(b->d_area);
  if (b->h_remaining) hipHostFree(b->h_remaining);
  delete b;
  return TVLBM_OK;
}

int tvlbm_batch_init(const tvlbm_batch_desc* d, tvlbm_batch** out) {
  if (!d || !out || d->n_inst < 1 || !d->inst || !d->arena_a || !d->arena_b || d->arena_a == d->arena_b)
    return TVLBM_EINVAL;
  if (!d->stream) return TVLBM_EINVAL;  // graph capture needs a non-null stream
  if (d->dtype != TVLBM_F32 && d->dtype != TVLBM_F64) return TVLBM_EINVAL;
  *out = nullptr;
  tvlbm_batch* b = new (std::nothrow) tvlbm_batch();
  if (!b) return TVLBM_ENOMEM;
  b->d = *d;
  b->inst.assign(d->inst, d->inst + d->n_inst);
  b->d.inst = nullptr;
  for (const auto& I : b->inst)
    if (!(I.tau > 0.5)) { delete b; return TVLBM_EINVAL; }
  if (d->eq_order > 4 || !build_lattice(d->n_gh, d->eq_order, d->cfl, d->cfl_norm, &b->hl)) {
    delete b;
    return TVLBM_EUNSUPPORTED;
  }
  b->f64 = d->dtype == TVLBM_F64;
  b->comp = b->f64 ? false : (d->compensated != 0);
  b->st = (hipStream_t)d->stream;
  b->buf[0] = d->arena_a;
  b->buf[1] = d->arena_b;
  if (!batch_layout(d, b->hl.q, b->off, b->fld, b->ld, b->pop_elems, b->field_elems)) {
    delete b;
    return TVLBM_EINVAL;
  }
  fill_lat(b->hl, b->latf);
  fill_lat(b->hl, b->latd);
  const int n = d->n_inst;
  const size_t isz = b->f64 ? sizeof(Inst<double>) : sizeof(Inst<float>);
  std::vector<char> hinst(isz * n);
  for (int k = 0; k < n; ++k) {
    const tvlbm_inst& I = b->inst[k];
    if (b->f64)
      fill_inst(b->hl, I.tau, 1, 1, I.wall_lo_ux, I.wall_lo_T, I.wall_hi_ux, I.wall_hi_T, I.nx, I.ny,
                b->ld[k], b->off[k], b->fld[k], *(Inst<double>*)(hinst.data() + isz * k));
    else
      fill_inst(b->hl, I.tau, 1, 1, I.wall_lo_ux, I.wall_lo_T, I.wall_hi_ux, I.wall_hi_T, I.nx, I.ny,
                b->ld[k], b->off[k], b->fld[k], *(Inst<float>*)(hinst.data() + isz * k));
    ((Inst<float>*)(hinst.data() + isz * k))->id = k;
  }
  const size_t esz = b->f64 ? 8 : 4;
  bool ok = hipMalloc(&b->d_insts, isz * n) == hipSuccess &&
            hipMalloc(&b->d_item_start, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            hipMalloc(&b->d_item_start_tail, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            hipMalloc(&b->d_item_start2, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            hipMalloc(&b->d_item_start2_tail, sizeof(int32_t) * (n + 1)) == hipSuccess &&
            hipMalloc(&b->d_rpart, sizeof(double) * 2 * RESID_SLICES * n) == hipSuccess &&
            hipMalloc(&b->d_nwork, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_nwork1, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_ntotal, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_remaining, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_active, sizeof(int32_t) * n) == hipSuccess &&
            hipMalloc(&b->d_have_prev, sizeof(int32_t) * n) == hipSuccess &&
            hipMalloc(&b->d_steps, sizeof(int64_t) * n) == hipSuccess &&
            hipMalloc(&b->d_resid, sizeof(double) * n) == hipSuccess &&
            hipMalloc(&b->d_flag, sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&b->d_fields, esz * b->field_elems) == hipSuccess &&
            hipMalloc(&b->d_prev, esz * b->field_elems) == hipSuccess &&
            hipMalloc(&b->d_mass0, sizeof(unsigned long long) * n) == hipSuccess &&
            hipMalloc(&b->d_mass, sizeof(unsigned long long) * n) == hipSuccess &&
            hipMalloc(&b->d_area, sizeof(double) * n) == hipSuccess &&
            hipHostMalloc((void**)&b->h_remaining, sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
  if (!ok) { tvlbm_batch_destroy(b); return TVLBM_ENOMEM; }
  std::vector<double> area(n);
  for (int k = 0; k < n; ++k) area[k] = (double)b->inst[k].nx * b->inst[k].ny;
  if (hipMemcpy(b->d_insts, hinst.data(), isz * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_area, area.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    tvlbm_batch_destroy(b);
    return TVLBM_EHIP;
  }
  const int32_t zero = 0;
  if (hipMemcpy(b->d_flag, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) {
    tvlbm_batch_destroy(b);
    return TVLBM_EHIP;
  }
  b->shapes = {{16, 16, 8}, {32, 32, 8}, {1 << 30, 64, 8}};
  if (build_items(b) != TVLBM_OK) { tvlbm_batch_destroy(b); return TVLBM_EHIP; }
  *out = b;
  return TVLBM_OK;
}

int tvlbm_batch_set_shape(tvlbm_batch* b, int32_t max_nx, int32_t width, int32_t rows) {
  if (!b || !(width == 16 || width == 32 || width == 64) || rows < 1 || rows > 255 || max_nx < 1)
    return bfail(b, TVLBM_EINVAL, "shape");
  bool found = false;
  for (auto& s : b->shapes)
    if (s.max_nx == max_nx) { s.width = width; s.rows = rows; found = true; }
  if (!found) b->shapes.push_back({max_nx, width, rows});
  std::sort(b->shapes.begin(), b->shapes.end(),
            [](const tvlbm_batch::Shape& x, const tvlbm_batch::Shape& y) { return x.max_nx < y.max_nx; });
  BHIP(b, hipStreamSynchronize(b->st));
  return build_items(b);
}

int tvlbm_batch_set_tuning(tvlbm_batch* b, const tvlbm_batch_tuning* t) {
  if (!b || !t || (t->prefetch != 0 && t->prefetch != 1) || t->tail_active < 0 ||
      !(t->tail_width == 16 || t->tail_width == 32 || t->tail_width == 64) || t->tail_rows < 1 ||
      t->tail_rows > 255 || (t->two_step != 0 && t->two_step != 1) || t->two_rows < 1 ||
      t->two_rows > 255)
    return bfail(b, TVLBM_EINVAL, "tuning");
  BHIP(b, hipStreamSynchronize(b->st));
  b->prefetch = t->prefetch;
  b->tail_active = t->tail_active;
  b->tail_width = t->tail_width;
  b->tail_rows = t->tail_rows;
  b->two_step = t->two_step;
  b->two_rows = t->two_rows;
  return build_items(b);
}

int tvlbm_batch_get_tuning(const tvlbm_batch* b, tvlbm_batch_tuning* t) {
  if (!b || !t) return TVLBM_EINVAL;
  t->prefetch = b->prefetch;
  t->tail_active = b->tail_active;
  t->tail_width = b->tail_width;
  t->tail_rows = b->tail_rows;
  t->two_step = b->two_step;
  t->two_rows = b->two_rows;
  return TVLBM_OK;
}

int tvlbm_batch_set_fields(tvlbm_batch* b, const void* fields) {
  if (!b || !fields) return bfail(b, TVLBM_EINVAL, "null");
  for (size_t k = 0; k < b->inst.size(); ++k) {
    const tvlbm_inst& I = b->inst[k];
    const int64_t np = (int64_t)I.nx * I.ny;
    if (b->f64) {
      InitArgs<double> A;
      std::memset(&A, 0, sizeof A);
      A.lat = b->latd;
      fill_inst(b->hl, I.tau, 1, 1, I.wall_lo_ux, I.wall_lo_T, I.wall_hi_ux, I.wall_hi_T, I.nx, I.ny,
                b->ld[k], b->off[k], b->fld[k], A.inst);
      const double* f = (const double*)fields + b->fld[k];
      A.rho = f; A.ux = f + np; A.uy = f + 2 * np; A.T = f + 3 * np;
      A.f0 = (double*)b->buf[1];
      A.g0 = (double*)b->buf[0];
      BHIP(b, launch_init(b->hl.n, false, A, b->st));
    } else {
      InitArgs<float> A;
      std::memset(&A, 0, sizeof A);
      A.lat = b->latf;
      fill_inst(b->hl, I.tau, 1, 1, I.wall_lo_ux, I.wall_lo_T, I.wall_hi_ux, I.wall_hi_T, I.nx, I.ny,
                b->ld[k], b->off[k], b->fld[k], A.inst);
      const float* f = (const float*)fields + b->fld[k];
      A.rho = f; A.ux = f + np; A.uy = f + 2 * np; A.T = f + 3 * np;
      A.f0 = (float*)b->buf[1];
      A.g0 = (float*)b->buf[0];
      BHIP(b, launch_init(b->hl.n, b->comp, A, b->st));
    }
  }
  b->initialised = true;
  b->stepped = false;
  return TVLBM_OK;
}

int tvlbm_batch_run(tvlbm_batch* b, int64_t max_steps, double tol, int32_t K, int64_t* steps_out,
                    double* r_out) {
  if (!b || K < 2 || (K & 1) || max_steps < 1 || !steps_out) return bfail(b, TVLBM_EINVAL, "run args");
  if (!b->initialised) return bfail(b, TVLBM_EINVAL, "fields not set");
  const int n = (int)b->inst.size();
  std::vector<int32_t> ones(n, 1), zeros(n, 0);
  std::vector<int64_t> zeros64(n, 0);
  BHIP(b, hipMemcpyAsync(b->d_flag, zeros.data(), sizeof(int32_t), hipMemcpyHostToDevice, b->st));
  BHIP(b, hipMemcpyAsync(b->d_active, ones.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, b->st));
  // snapshot of the starting fields, so the first chunk already yields a
  // residual (as the single-instance solve does)
  {
    const int aux = AUX_FIELDS | (b->stepped ? 0 : AUX_IDENTITY);
    BHIP(b, launch_fill_i32((int32_t*)b->d_mass0, 2 * n, 0, b->st));
    int rc = bmarch(b, MODE_AUX, aux, b->buf[1], nullptr, b->d_ntotal, b->d_all, batch_blocks(b->n_items),
                    b->d_mass0);
    if (rc) return rc;
    const size_t esz = b->f64 ? 8 : 4;
    BHIP(b, hipMemcpyAsync(b->d_prev, b->d_fields, esz * b->field_elems, hipMemcpyDeviceToDevice, b->st));
  }
  BHIP(b, hipMemcpyAsync(b->d_have_prev, ones.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, b->st));
  BHIP(b, hipMemcpyAsync(b->d_steps, zeros64.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, b->st));
  const bool two = b->two_step && two_kernel(b) && K >= 4;
  if (b->g_K != K || b->g_tol != tol || b->g_max != max_steps || b->chunk_two != two) drop_graphs(b);
  b->g_K = K; b->g_tol = tol; b->g_max = max_steps;
  b->chunk_two = two;
  auto want_tail = [b](int remaining) { return b->tail_active > 0 && remaining <= b->tail_active; };
  bool tail = want_tail(n);
  int rc = compact(b, tail);
  if (rc) return rc;
  const int64_t max_chunks = (max_steps + K - 1) / K + 1;
  for (int64_t c = 0; c < max_chunks; ++c) {
    hipGraphExec_t& ge = tail ? b->gexec_tail : b->gexec;
    if (!ge) {
      rc = capture_chunk(b, K, tol, max_steps, tail, &ge);
      if (rc) return rc;
    }
    BHIP(b, hipGraphLaunch(ge, b->st));
    BHIP(b, hipMemcpyAsync(b->h_remaining, b->d_remaining, sizeof(int32_t), hipMemcpyDeviceToHost, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    b->stepped = true;
    const int remaining = *b->h_remaining;
    if (remaining == 0) break;
    if (!tail && want_tail(remaining)) {
      tail = true;
      rc = compact(b, true);
      if (rc) return rc;
    }
  }
  std::vector<double> r(n);
  int32_t flag = 0;
  BHIP(b, hipMemcpyAsync(steps_out, b->d_steps, sizeof(int64_t) * n, hipMemcpyDeviceToHost, b->st));
  BHIP(b, hipMemcpyAsync(r.data(), b->d_resid, sizeof(double) * n, hipMemcpyDeviceToHost, b->st));
  BHIP(b, hipMemcpyAsync(&flag, b->d_flag, sizeof flag, hipMemcpyDeviceToHost, b->st));
  BHIP(b, hipStreamSynchronize(b->st));
  if (r_out) std::memcpy(r_out, r.data(), sizeof(double) * n);
  if (flag) return bfail(b, TVLBM_ENONFINITE, "non-finite residual");
  for (int k = 0; k < n; ++k)
    if (!(r[k] < tol)) return bfail(b, TVLBM_ENOTCONVERGED, "step limit reached");
  return TVLBM_OK;
}

int tvlbm_batch_fields(tvlbm_batch* b, void* out) {
  if (!b || !out) return bfail(b, TVLBM_EINVAL, "null");
  if (!b->initialised) return bfail(b, TVLBM_EINVAL, "fields not set");
  const int aux = AUX_FIELDS | (b->stepped ? 0 : AUX_IDENTITY);
  int rc = bmarch(b, MODE_AUX, aux, b->buf[1], nullptr, b->d_ntotal, b->d_all, batch_blocks(b->n_items));
  if (rc) return rc;
  const size_t esz = b->f64 ? 8 : 4;
  BHIP(b, hipMemcpyAsync(out, b->d_fields, esz * b->field_elems, hipMemcpyDeviceToDevice, b->st));
  int32_t flag = 0;
  BHIP(b, hipMemcpyAsync(&flag, b->d_flag, sizeof flag, hipMemcpyDeviceToHost, b->st));
  BHIP(b, hipStreamSynchronize(b->st));
  if (flag) return bfail(b, TVLBM_ENONFINITE, "non-finite moment");
  return TVLBM_OK;
}

}  // extern "C"
