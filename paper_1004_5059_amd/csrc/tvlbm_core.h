// tvlbm_core.h -- device-side building blocks of the fused TVLBM step for
// gfx950 (MI355X): kernel parameter blocks, compensated moment sums, the
// Hermite equilibrium in deviation form and the BGK update.
//
// Storage convention: population arrays hold d_l = f_l - w_l (the deviation
// from the rest equilibrium at rho = 1, u = 0, T = 1).  Volumetric streaming
// is a partition of unity, so it maps deviations to deviations, and all
// moment sums and equilibrium terms below are formed from small quantities,
// which keeps FP32 storage accurate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvlbm {

constexpr int NMAX = 6;   // Gauss-Hermite points per axis
constexpr int QMAX = 36;  // populations
constexpr double DIM = 2.0;

// ---------------------------------------------------------------- params --
// Lattice constants shared by every instance of a run (kernel argument
// space is constant memory; every lane reads the same entry, so these are
// scalar loads).
template <typename R>
struct Lat {
  R p[NMAX];    // |displacement| of node a along one axis (pull fraction)
  R qm[NMAX];   // 1 - p, exact
  R x[NMAX];    // node a (Hermite units)
  R x2[NMAX];   // x_a^2
  R w[QMAX];    // w_l
  R cD[QMAX];   // |xi_l|^2 - D
  R c4[QMAX];   // (|xi_l|^4 - 2(D+2)|xi_l|^2 + D(D+2)) / 8
  double xd[NMAX];
  double wd[QMAX];
  double sumw;  // sum of wd
};

// Per-instance parameters.  A single run passes one by value; a batched run
// keeps an array in device memory.
template <typename R>
struct Inst {
  int64_t off;    // element offset of the population block in the buffer
  int64_t plane;  // ny * ld
  int64_t ld;     // row pitch
  int64_t fld;    // element offset of this instance's [4][ny][nx] fields
  int32_t nx, ny;
  int32_t walls;  // 0 periodic in y, 1 diffuse walls
  int32_t id;
  R omo;          // 1 - 1/tau
  R oww[QMAX];    // w_l / tau
  R kap_lo[QMAX]; // ghost deviation at the bottom wall: kap + phi * X(m)
  R phi_lo[QMAX];
  R kap_hi[QMAX];
  R phi_hi[QMAX];
};

enum Mode { MODE_STEP = 0, MODE_CHECK = 1, MODE_AUX = 2 };
enum AuxBits { AUX_FIELDS = 1, AUX_POPS = 2, AUX_POST = 4, AUX_IDENTITY = 8 };

struct Work {      // one wavefront's share of a batched step
  int32_t inst;    // instance index
  int32_t x0;      // first column of the strip
  int32_t seg0;    // first row segment
  int32_t shape;   // strip width (16, 32, 64) | rows per lane segment << 8
};

// Non-uniform rows (the rectangular meshes of Sec. III, uniform in x):
// for y-node b and target row k, the pulled value is
//   sum_{t<4} w[t] X_a(row src[t]) + glo * ghost_lo + ghi * ghost_hi,
// where w = (overlap of the shifted source row with row k) / dy_k and the
// ghost weights are the overlaps of the wall-emission intervals.
template <typename R>
struct RowTap {
  int32_t src[4];
  R w[4];
  R glo, ghi;
};
// Rows whose shifted interval crosses a wall, per y-node b, with the length
// that crosses (bottom wall for x_b < 0, top wall for x_b > 0).
template <typename R>
struct IncRows {
  int32_t j[4];
  R len[4];
};

template <typename R>
struct MarchArgs {
  Lat<R> lat;
  Inst<R> inst;           // single-instance launches
  const Inst<R>* insts;   // batched launches (device)
  const Work* work;       // batched launches (device)
  const int32_t* n_work;  // batched launches: live length of the work list
  int32_t width;          // columns per wavefront strip: 16, 32 or 64
  int32_t rows;           // rows per lane segment
  int32_t aux;            // AuxBits for MODE_AUX
  int32_t prefetch;       // step kernel: software-pipelined rows
  int32_t tiles_x;        // strips across the grid (single-instance)
  int32_t n_tiles;        // workgroup tiles (single-instance)
  const R* src;           // deviations g^k (or f^0 with AUX_IDENTITY)
  R* dst;                 // STEP/CHECK: g^{k+1}; AUX_POPS/POST: [q][ny][nx] out
  R* fields;              // CHECK / AUX_FIELDS: [4][ny][nx] (may be null)
  double* partials;       // CHECK / AUX_FIELDS: [n_blocks][4] FP64 totals
  int32_t* flag;          // set to 1 on rho <= 0, T <= 0 or non-finite
  const RowTap<R>* taps;  // non-uniform rows: [n][ny]
  const IncRows<R>* inc;  // non-uniform rows with walls: [n]
  const double* dy;       // non-uniform rows: [ny] heights
  const int32_t* rowflag; // bit 0: row pulls the bottom ghost, bit 1: the top
};

// Fused multiply-add in the working precision (the double builtin would
// promote float operands).
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------ compensation -----
// Kahan's compensated summation: (s, c) accumulates x with the rounding
// error of every addition carried in c (the value is s - c).
template <typename R>
__device__ __forceinline__ void kahan_add(R& s, R& c, R x) {
  const R y = x - c;
  const R t = s + y;
  c = (t - s) - y;
  s = t;
}
// Compensated dot-product term: the product a*b is split exactly into
// p + e (TwoProduct with a fused multiply-add); p is added with Kahan's
// scheme and e into a separate low-order accumulator.
template <typename R>
__device__ __forceinline__ void kahan_dot(R& s, R& c, R& lo, R a, R b) {
  const R p = a * b;
  lo += fmaR(a, b, -p);
  kahan_add(s, c, p);
}

// ---------------------------------------------------------------- moments --
// Moments of one cell's deviations d_l (Sec. II):
//   drho = sum d,  j = sum xi d,  ed = sum |xi|^2 d.
// The tensor-product structure xi_l = (x_a, x_b) lets every moment be formed
// from row sums R_a = sum_b d_ab and column sums C_b = sum_a d_ab:
//   drho = sum_a R_a, jx = sum_a x_a R_a, jy = sum_b x_b C_b,
//   ed = sum_a x_a^2 R_a + sum_b x_b^2 C_b.
// COMP: every sum is compensated -- Kahan summation for the row and column
// sums and for drho, and compensated dot products (exact product split plus
// Kahan summation) for j and ed, with the low-order parts of the row and
// column sums carried into the dot products.
template <typename R, int N, bool COMP>
__device__ __forceinline__ void cell_moments(const Lat<R>& L, const R (&d)[N * N], R& drho,
                                             R& jx, R& jy, R& ed) {
  if constexpr (!COMP) {
    R ra[N], cb[N];
#pragma unroll
    for (int b = 0; b < N; ++b) cb[b] = d[b];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R s = d[a * N];
#pragma unroll
      for (int b = 1; b < N; ++b) s += d[a * N + b];
      ra[a] = s;
      if (a > 0) {
#pragma unroll
        for (int b = 0; b < N; ++b) cb[b] += d[a * N + b];
      }
    }
    R r = ra[0], x = L.x[0] * ra[0], y = L.x[0] * cb[0];
    R e = L.x2[0] * ra[0] + L.x2[0] * cb[0];
#pragma unroll
    for (int a = 1; a < N; ++a) {
      r += ra[a];
      x = fmaR(L.x[a], ra[a], x);
      y = fmaR(L.x[a], cb[a], y);
      e = fmaR(L.x2[a], ra[a], e);
      e = fmaR(L.x2[a], cb[a], e);
    }
    drho = r; jx = x; jy = y; ed = e;
  } else {
    // row sums (hi, -lo) and column sums
    R rh[N], rc[N], ch[N], cc[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R s = d[a * N], c = R(0);
#pragma unroll
      for (int b = 1; b < N; ++b) kahan_add(s, c, d[a * N + b]);
      rh[a] = s; rc[a] = c;
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R s = d[b], c = R(0);
#pragma unroll
      for (int a = 1; a < N; ++a) kahan_add(s, c, d[a * N + b]);
      ch[b] = s; cc[b] = c;
    }
    {  // drho = sum_a (rh_a - rc_a)
      R s = rh[0], c = R(0), lo = -rc[0];
#pragma unroll
      for (int a = 1; a < N; ++a) {
        kahan_add(s, c, rh[a]);
        lo -= rc[a];
      }
      drho = s + (lo - c);
    }
    {  // jx = sum_a x_a (rh_a - rc_a)
      R s = R(0), c = R(0), lo = R(0);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        kahan_dot(s, c, lo, L.x[a], rh[a]);
        lo = fmaR(-L.x[a], rc[a], lo);
      }
      jx = s + (lo - c);
    }
    {  // jy = sum_b x_b (ch_b - cc_b)
      R s = R(0), c = R(0), lo = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        kahan_dot(s, c, lo, L.x[b], ch[b]);
        lo = fmaR(-L.x[b], cc[b], lo);
      }
      jy = s + (lo - c);
    }
    {  // ed = sum_a x_a^2 (rh_a - rc_a) + sum_b x_b^2 (ch_b - cc_b)
      R s = R(0), c = R(0), lo = R(0);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        kahan_dot(s, c, lo, L.x2[a], rh[a]);
        lo = fmaR(-L.x2[a], rc[a], lo);
        kahan_dot(s, c, lo, L.x2[a], ch[a]);
        lo = fmaR(-L.x2[a], cc[a], lo);
      }
      ed = s + (lo - c);
    }
  }
}

// Macroscopic fields from the deviation moments:
//   rho = 1 + drho, u = j / rho,
//   D rho (T - 1) = ed - D drho - |j|^2 / rho   (equivalent to the central
//   form rho T = (1/D) sum |xi - u|^2 f of Sec. II, since sum w = 1,
//   sum xi w = 0 and sum |xi|^2 w = D).
template <typename R>
struct Fields {
  R rho, drho, ux, uy, th;
};

template <typename R>
__device__ __forceinline__ Fields<R> fields_from(R drho, R jx, R jy, R ed) {
  Fields<R> F;
  F.drho = drho;
  F.rho = R(1) + drho;
  R inv = R(1) / F.rho;
  F.ux = jx * inv;
  F.uy = jy * inv;
  F.th = (ed - R(DIM) * drho - (jx * F.ux + jy * F.uy)) * inv * R(1.0 / DIM);
  return F;
}

// ------------------------------------------------------------ equilibrium --
// Hermite equilibrium (Sec. II; scalar form of Appendix A) in deviation form:
//   feq_l - w_l = w_l [ drho + rho P_l ],
//   P_l = u_l + 1/2 (u_l^2 - u^2 + th cD)
//       + (u_l / 6)(u_l^2 - 3 u^2 + 3 th (cD - 2))                       [ORD>=3]
//       + (u_l^4 - 6 u_l^2 u^2 + 3 u^4)/24
//       + (th/4)((cD - 2)(u_l^2 - u^2) - 2 u_l^2) + th^2 c4              [ORD>=4]
// with u_l = u.xi_l, th = T - 1, cD = |xi_l|^2 - D and
// c4 = (|xi_l|^4 - 2(D+2)|xi_l|^2 + D(D+2))/8.  Collecting powers of s = u_l,
//   P_l = k0 + s (k1 + s (k2 + s (1/6 + s/24)))
//   k0 = -u^2/2 + (th/2) cD                  [+ u^4/8 + th u^2/2 + th^2 c4 - th u^2 cD/4]
//   k1 = 1 - u^2/2 - th + (th/2) cD
//   k2 = 1/2                                 [- u^2/4 - th + th cD/4]
// (bracketed terms for order 4; order 3 drops the s^4 term; order 2 keeps
// k0 = -u^2/2 + (th/2) cD, k1 = 1, k2 = 1/2 and no s^3 term).
template <typename R>
struct EqCell {
  R ua[NMAX], vb[NMAX];  // x_a ux, x_b uy
  R g0, be, al, mu, a2, thq, thsq;
};

template <typename R, int N, int ORD>
__device__ __forceinline__ EqCell<R> eq_cell(const Lat<R>& L, const Fields<R>& F) {
  EqCell<R> E;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    E.ua[a] = L.x[a] * F.ux;
    E.vb[a] = L.x[a] * F.uy;
  }
  const R u2 = F.ux * F.ux + F.uy * F.uy;
  const R th = F.th;
  E.be = R(0.5) * th;
  E.thq = R(0.25) * th;
  E.thsq = th * th;
  if constexpr (ORD >= 3) {
    E.al = R(1) - R(0.5) * u2 - th;
  } else {
    E.al = R(1);
  }
  if constexpr (ORD >= 4) {
    E.g0 = -R(0.5) * u2 + u2 * (R(0.125) * u2 + E.be);
    E.mu = E.be - E.thq * u2;
    E.a2 = R(0.5) - R(0.25) * u2 - th;
  } else {
    E.g0 = -R(0.5) * u2;
    E.mu = E.be;
    E.a2 = R(0.5);
  }
  return E;
}

// returns P_l (the equilibrium polynomial minus its leading 1)
template <typename R, int N, int ORD>
__device__ __forceinline__ R eq_poly(const Lat<R>& L, const EqCell<R>& E, int a, int b) {
  const int l = a * N + b;
  const R s = E.ua[a] + E.vb[b];
  const R cD = L.cD[l];
  R k0 = fmaR(cD, E.mu, E.g0);
  if constexpr (ORD >= 4) k0 = fmaR(E.thsq, L.c4[l], k0);
  const R k1 = (ORD >= 3) ? fmaR(cD, E.be, E.al) : E.al;
  R h;
  if constexpr (ORD >= 4) {
    const R k2 = fmaR(cD, E.thq, E.a2);
    h = fmaR(s, R(1.0 / 24.0), R(1.0 / 6.0));
    h = fmaR(s, h, k2);
  } else if constexpr (ORD == 3) {
    h = fmaR(s, R(1.0 / 6.0), E.a2);
  } else {
    h = E.a2;
  }
  h = fmaR(s, h, k1);
  return fmaR(s, h, k0);
}

// BGK update in deviation form (eq.(lb) integrated over one step, tau in
// steps):  d* = d + (feq_dev - d)/tau = (1 - 1/tau) d + (w/tau)(drho + rho P).
template <typename R>
__device__ __forceinline__ R bgk(R d, R oww_l, R omo, R rho, R drho, R P) {
  return fmaR(oww_l, fmaR(rho, P, drho), omo * d);
}

}  // namespace tvlbm
