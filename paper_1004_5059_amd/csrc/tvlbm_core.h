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
  int32_t pad;
};

template <typename R>
struct MarchArgs {
  Lat<R> lat;
  Inst<R> inst;           // single-instance launches
  const Inst<R>* insts;   // batched launches (device)
  const Work* work;       // batched launches (device)
  int32_t n_work;
  int32_t width;          // columns per wavefront strip: 16, 32 or 64
  int32_t rows;           // rows per lane segment
  int32_t aux;            // AuxBits for MODE_AUX
  int32_t tiles_x;        // strips across the grid (single-instance)
  int32_t n_tiles;        // workgroup tiles (single-instance)
  const R* src;           // deviations g^k (or f^0 with AUX_IDENTITY)
  R* dst;                 // STEP/CHECK: g^{k+1}; AUX_POPS/POST: [q][ny][nx] out
  R* fields;              // CHECK / AUX_FIELDS: [4][ny][nx] (may be null)
  double* partials;       // CHECK / AUX_FIELDS: [n_blocks][4] FP64 totals
  int32_t* flag;          // set to 1 on rho <= 0, T <= 0 or non-finite
};

// Fused multiply-add in the working precision (the double builtin would
// promote float operands).
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------ exact transforms --
// Knuth's TwoSum: s + e == a + b exactly (round-to-nearest).
template <typename R>
__device__ __forceinline__ void two_sum(R a, R b, R& s, R& e) {
  s = a + b;
  R z = s - a;
  e = (a - (s - z)) + (b - z);
}
// TwoProduct with a fused multiply-add: p + e == a * b exactly.
template <typename R>
__device__ __forceinline__ void two_prod(R a, R b, R& p, R& e) {
  p = a * b;
  e = fmaR(a, b, -p);
}

// ---------------------------------------------------------------- moments --
// Moments of one cell's deviations d_l (Sec. II):
//   drho = sum d,  j = sum xi d,  ed = sum |xi|^2 d.
// The tensor-product structure xi_l = (x_a, x_b) lets every moment be formed
// from row sums R_a = sum_b d_ab and column sums C_b = sum_a d_ab:
//   drho = sum_a R_a, jx = sum_a x_a R_a, jy = sum_b x_b C_b,
//   ed = sum_a x_a^2 R_a + sum_b x_b^2 C_b.
// COMP: the row/column sums use TwoSum and the dot products use the
// compensated dot product of Ogita, Rump & Oishi (Dot2), carrying the
// rounding error of every addition and product in a second accumulator.
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
    R ra[N], ea[N], cb[N], eb[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R s = d[a * N], e = R(0);
#pragma unroll
      for (int b = 1; b < N; ++b) {
        R t;
        two_sum(s, d[a * N + b], s, t);
        e += t;
      }
      ra[a] = s; ea[a] = e;
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R s = d[b], e = R(0);
#pragma unroll
      for (int a = 1; a < N; ++a) {
        R t;
        two_sum(s, d[a * N + b], s, t);
        e += t;
      }
      cb[b] = s; eb[b] = e;
    }
    // drho
    R s = ra[0], e = ea[0];
#pragma unroll
    for (int a = 1; a < N; ++a) {
      R t;
      two_sum(s, ra[a], s, t);
      e += t + ea[a];
    }
    drho = s + e;
    // Dot2 helpers over (coefficient, hi, lo) triples
    auto dot2 = [&](const R* c, const R* hi, const R* lo, R& S, R& E) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        R p, ep, t;
        two_prod(c[a], hi[a], p, ep);
        two_sum(S, p, S, t);
        E += t + fmaR(c[a], lo[a], ep);
      }
    };
    R Sx = R(0), Ex = R(0);
    dot2(L.x, ra, ea, Sx, Ex);
    jx = Sx + Ex;
    R Sy = R(0), Ey = R(0);
    dot2(L.x, cb, eb, Sy, Ey);
    jy = Sy + Ey;
    R Se = R(0), Ee = R(0);
    dot2(L.x2, ra, ea, Se, Ee);
    dot2(L.x2, cb, eb, Se, Ee);
    ed = Se + Ee;
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
//   feq_l - w_l = w_l [ drho + rho (P_l - 1) ],
//   P_l - 1 = u_l + 1/2 (u_l^2 - u^2 + th (c2 - D))
//           + (u_l / 6)(u_l^2 - 3 u^2 + 3 th (c2 - D - 2))             [ORD>=3]
//           + (u_l^4 - 6 u_l^2 u^2 + 3 u^4)/24
//           + (th/4)((c2 - D - 2)(u_l^2 - u^2) - 2 u_l^2)
//           + (th^2/8)(c2^2 - 2(D+2) c2 + D(D+2))                      [ORD>=4]
// with u_l = u.xi_l, c2 = |xi_l|^2, th = T - 1.  The per-cell scalars are
// hoisted into EqCell; per population the cost is a handful of FMAs.
template <typename R>
struct EqCell {
  R ua[NMAX], vb[NMAX];  // x_a ux, x_b uy
  R u2, th, th3, k3, u2x6, u2sq8, th4, thsq;
};

template <typename R, int N>
__device__ __forceinline__ EqCell<R> eq_cell(const Lat<R>& L, const Fields<R>& F) {
  EqCell<R> E;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    E.ua[a] = L.x[a] * F.ux;
    E.vb[a] = L.x[a] * F.uy;
  }
  E.u2 = F.ux * F.ux + F.uy * F.uy;
  E.th = F.th;
  E.th3 = R(3) * F.th;
  E.k3 = R(-2) * E.u2 - R(6) * F.th;
  E.u2x6 = R(6) * E.u2;
  E.u2sq8 = E.u2 * E.u2 * R(0.125);
  E.th4 = F.th * R(0.25);
  E.thsq = F.th * F.th;
  return E;
}

// returns P_l - 1
template <typename R, int N, int ORD>
__device__ __forceinline__ R eq_poly(const Lat<R>& L, const EqCell<R>& E, int a, int b) {
  const int l = a * N + b;
  R ul = E.ua[a] + E.vb[b];
  R ul2 = ul * ul;
  R d2 = ul2 - E.u2;
  R A = fmaR(E.th, L.cD[l], d2);
  R P = fmaR(R(0.5), A, ul);
  if constexpr (ORD >= 3) {
    R B = fmaR(E.th3, L.cD[l], d2 + E.k3);
    P = fmaR(ul * R(1.0 / 6.0), B, P);
  }
  if constexpr (ORD >= 4) {
    R q4 = ul2 * (ul2 - E.u2x6) * R(1.0 / 24.0) + E.u2sq8;
    R m = (L.cD[l] - R(2)) * d2 - R(2) * ul2;
    q4 = fmaR(E.th4, m, q4);
    q4 = fmaR(E.thsq, L.c4[l], q4);
    P += q4;
  }
  return P;
}

// BGK update in deviation form (eq.(lb) integrated over one step, tau in
// steps):  d* = d + (feq_dev - d)/tau = (1 - 1/tau) d + (w/tau)(drho + rho P).
template <typename R>
__device__ __forceinline__ R bgk(R d, R oww_l, R omo, R rho, R drho, R P) {
  return fmaR(oww_l, fmaR(rho, P, drho), omo * d);
}

}  // namespace tvlbm
