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

#include <type_traits>
#include <stdint.h>

namespace tvlbm {

// Two FP32 cells per lane: the step kernel can run on a pair of adjacent
// columns held as a 2-wide vector, with every operation elementwise (so each
// cell's arithmetic is exactly that of the scalar kernel) and 8-byte loads
// and stores.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename R>
inline constexpr bool is_pair_v = false;
template <>
inline constexpr bool is_pair_v<f32x2> = true;

constexpr int NMAX = 6;   // Gauss-Hermite points per axis
constexpr int QMAX = 36;  // populations
constexpr double DIM = 2.0;

// Buffer addressing: one resource per instance block (base and size in
// SGPRs); the lane offset (row, column) is a VGPR and the population plane
// offset l * plane is a wave-uniform SGPR offset, so no per-load address
// arithmetic is spent on the vector ALUs.  Accesses beyond the block return
// zero instead of faulting.
// Tables that no kernel writes while it reads them (instance parameters,
// work items): read through the constant address space, so that reads at a
// wave-uniform index become scalar loads, kept in SGPRs where they repeat.
template <typename T>
__device__ __forceinline__ const T& ro(const T* p, int i) {
  using cT = const __attribute__((address_space(4))) T;
  return *(const T*)((cT*)p + i);
}

using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename R>
__device__ __forceinline__ R bld(rsrc_t r, uint32_t v, uint32_t s);
template <>
__device__ __forceinline__ float bld<float>(rsrc_t r, uint32_t v, uint32_t s) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v * 4u, s * 4u, 0));
}
template <>
__device__ __forceinline__ double bld<double>(rsrc_t r, uint32_t v, uint32_t s) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v * 8u, s * 8u, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t v, uint32_t s, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, x), r, v * 4u, s * 4u, 0);
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t v, uint32_t s, double x) {
  using v2i = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, x), r, v * 8u, s * 8u, 0);
}
// column pairs: offsets count pairs (8 bytes)
template <>
__device__ __forceinline__ f32x2 bld<f32x2>(rsrc_t r, uint32_t v, uint32_t s) {
  return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, v * 8u, s * 8u, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t v, uint32_t s, f32x2 x) {
  using v2i = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, x), r, v * 8u, s * 8u, 0);
}

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
  const int32_t* rowflag; // bit 0: row pulls the bottom ghost, bit 1: the top;
                          // bits 2-3: source rows read per tap list - 1
  int32_t inc_rows;       // non-uniform rows with walls: entries used in inc[b] (max over b)
  unsigned long long* mass;  // CHECK / AUX_FIELDS: fixed-point deviation mass
                             // per instance (index Inst::id / work item), or null
};

// Fixed-point unit of the exact, order-independent mass tallies:
// sum_l (f_l - w_l) dy per cell rounded to multiples of 2^-32.
constexpr double MASS_FP_SCALE = 4294967296.0;

// Fused multiply-add in the working precision (the double builtin would
// promote float operands).
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ f32x2 fmaR(f32x2 a, f32x2 b, f32x2 c) {
  return __builtin_elementwise_fma(a, b, c);
}

// ------------------------------------------------------ compensation -----
// Compensated FP32 sums are accumulated in FP64: a product of an FP32 node
// and an FP32 deviation is exact there, and a sum of at most 36 such terms
// keeps ~53 - 5 bits, so the moments are rounded to FP32 once, at the end.
// On this chip FP64 vector operations issue at the FP32 rate, which makes
// this cheaper than Kahan summation in FP32 (one conversion per value
// instead of four operations per addition).
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename R>
struct WideT { using T = double; };
template <>
struct WideT<f32x2> { using T = f64x2; };
__device__ __forceinline__ double widen(float x) { return (double)x; }
__device__ __forceinline__ double widen(double x) { return x; }
__device__ __forceinline__ f64x2 widen(f32x2 x) { return __builtin_convertvector(x, f64x2); }
template <typename R>
__device__ __forceinline__ R narrow(typename WideT<R>::T x);
template <>
__device__ __forceinline__ float narrow<float>(double x) { return (float)x; }
template <>
__device__ __forceinline__ double narrow<double>(double x) { return x; }
template <>
__device__ __forceinline__ f32x2 narrow<f32x2>(f64x2 x) { return __builtin_convertvector(x, f32x2); }
__device__ __forceinline__ f64x2 fmaR(f64x2 a, f64x2 b, f64x2 c) {
  return __builtin_elementwise_fma(a, b, c);
}

// ---------------------------------------------------------------- moments --
// Moments of one cell's deviations d_l (Sec. II):
//   drho = sum d,  j = sum xi d,  ed = sum |xi|^2 d.
// The tensor-product structure xi_l = (x_a, x_b) lets every moment be formed
// from row sums R_a = sum_b d_ab and column sums C_b = sum_a d_ab:
//   drho = sum_a R_a, jx = sum_a x_a R_a, jy = sum_b x_b C_b,
//   ed = sum_a x_a^2 R_a + sum_b x_b^2 C_b.
// COMP: the same sums accumulated in FP64 (see above) and rounded once.
template <typename W, typename R>
__device__ __forceinline__ W as_w(R x) {
  if constexpr (std::is_same_v<W, R>) return x;
  else return widen(x);
}

template <typename W, typename R, int N>
__device__ __forceinline__ void tensor_moments(const Lat<R>& L, const W (&v)[N * N], W& r,
                                               W& x, W& y, W& e) {
  W ra[N], cb[N];
#pragma unroll
  for (int b = 0; b < N; ++b) cb[b] = v[b];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    W s = v[a * N];
#pragma unroll
    for (int b = 1; b < N; ++b) s += v[a * N + b];
    ra[a] = s;
    if (a > 0) {
#pragma unroll
      for (int b = 0; b < N; ++b) cb[b] += v[a * N + b];
    }
  }
  r = ra[0];
  x = as_w<W>(L.x[0]) * ra[0];
  y = as_w<W>(L.x[0]) * cb[0];
  e = as_w<W>(L.x2[0]) * ra[0] + as_w<W>(L.x2[0]) * cb[0];
#pragma unroll
  for (int a = 1; a < N; ++a) {
    r += ra[a];
    x = fmaR(as_w<W>(L.x[a]), ra[a], x);
    y = fmaR(as_w<W>(L.x[a]), cb[a], y);
    e = fmaR(as_w<W>(L.x2[a]), ra[a], e);
    e = fmaR(as_w<W>(L.x2[a]), cb[a], e);
  }
}

template <typename R, int N, bool COMP>
__device__ __forceinline__ void cell_moments(const Lat<R>& L, const R (&d)[N * N], R& drho,
                                             R& jx, R& jy, R& ed) {
  if constexpr (!COMP) {
    tensor_moments<R, R, N>(L, d, drho, jx, jy, ed);
  } else {
    using W = typename WideT<R>::T;
    W v[N * N];
#pragma unroll
    for (int l = 0; l < N * N; ++l) v[l] = widen(d[l]);
    W r, x, y, e;
    tensor_moments<W, R, N>(L, v, r, x, y, e);
    drho = narrow<R>(r);
    jx = narrow<R>(x);
    jy = narrow<R>(y);
    ed = narrow<R>(e);
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
//   P_l = s + 1/2 (s^2 - u^2 + th (c^2 - D))
//       + (s / 6)(s^2 - 3 u^2 + 3 th (c^2 - D - 2))                        [ORD>=3]
//       + (s^4 - 6 s^2 u^2 + 3 u^4)/24
//       + (th/4)((c^2 - D - 2)(s^2 - u^2) - 2 s^2)
//       + (th^2/8)(c^4 - 2(D+2) c^2 + D(D+2))                              [ORD>=4]
// with s = u.xi_l, c = |xi_l|, th = T - 1, D = 2.
//
// On the tensor-product set xi_l = (x_a, x_b), P_l is a polynomial of total
// degree ORD in (x, y) = (x_a, x_b).  Collecting its monomials x^i y^j splits
// it exactly into terms of one node each (with U = u_x, V = u_y,
// A2 = (U^2 + th)/2, A3 = U (U^2 + 3 th)/6, B2, B3 likewise in V):
//   P(x, y) = F(x) + G(y) + y K(x) + x M(y) + N(x) O(y),
//   K(x) = x (k0 + x (k1 + x k2)),  M(y) = y^2 (m0 + y m1),
//   N(x) O(y) = A2 x^2 B2 y^2                                      [ORD>=4]
// with the coefficients of eq_nodes below.  Per cell, the y-node terms G, M,
// O are evaluated once per node and the x-node terms F, K (scaled by rho,
// drho folded into F) once per row of the tensor; per population the
// equilibrium deviation then costs three or four fused operations.
template <typename R, int N>
struct EqNodes {
  R f0, f1, f2, f3, f4, k0, k1, k2, na;  // rho-scaled x-node coefficients
  R G[N], M[N], Ob[N];                   // y-node terms
};

template <typename R, int N, int ORD>
__device__ __forceinline__ void eq_nodes(const Lat<R>& L, const Fields<R>& Fd, EqNodes<R, N>& E) {
  const R U = Fd.ux, V = Fd.uy, th = Fd.th, rho = Fd.rho;
  const R U2 = U * U, V2 = V * V, u2 = U2 + V2, hth = R(0.5) * th;
  const R A2 = fmaR(R(0.5), U2, hth), B2 = fmaR(R(0.5), V2, hth);
  // polynomial coefficients: F = sum f_i x^i, G = sum_{i>=1} g_i y^i
  R f0, f1, f2, f3 = R(0), f4 = R(0), g1, g2, g3 = R(0), g4 = R(0);
  R k0, k1 = R(0), k2 = R(0), m0 = R(0), m1 = R(0);
  if constexpr (ORD == 2) {
    f0 = -fmaR(R(0.5), u2, th);
    f1 = U; f2 = A2; g1 = V; g2 = B2;
    k0 = U * V;
  } else {
    const R A3 = U * fmaR(R(3), th, U2) * R(1.0 / 6.0);
    const R B3 = V * fmaR(R(3), th, V2) * R(1.0 / 6.0);
    const R mm = R(1) - fmaR(R(0.5), u2, R(2) * th);  // 1 - u^2/2 - 2 th
    f1 = U * mm; g1 = V * mm;
    f3 = A3; g3 = B3;
    k1 = V * A2; m0 = U * B2;
    if constexpr (ORD == 3) {
      f0 = -fmaR(R(0.5), u2, th);
      f2 = A2; g2 = B2;
      k0 = U * V;
    } else {
      const R th2 = th * th;
      // u^4/8 + th u^2 - u^2/2 + th^2 - th
      f0 = fmaR(u2, fmaR(R(0.125), u2, th - R(0.5)), th2 - th);
      // -(U^2 u^2 + 7 U^2 th - 2 U^2 + V^2 th + 4 th^2 - 2 th)/4, and in V
      const R cth = fmaR(R(4), th2, R(-2) * th);
      f2 = R(-0.25) * fmaR(U2, u2 + fmaR(R(7), th, R(-2)), fmaR(V2, th, cth));
      g2 = R(-0.25) * fmaR(V2, u2 + fmaR(R(7), th, R(-2)), fmaR(U2, th, cth));
      // (U^4 + 6 U^2 th + 3 th^2)/24, and in V
      f4 = fmaR(U2, U2 + R(6) * th, R(3) * th2) * R(1.0 / 24.0);
      g4 = fmaR(V2, V2 + R(6) * th, R(3) * th2) * R(1.0 / 24.0);
      k0 = U * V * (R(1) - fmaR(R(0.5), u2, R(3) * th));
      k2 = V * A3; m1 = U * B3;
    }
  }
  // scale by rho; drho joins the constant term
  E.f0 = fmaR(rho, f0, Fd.drho);
  E.f1 = f1 * rho; E.f2 = f2 * rho; E.f3 = f3 * rho; E.f4 = f4 * rho;
  E.k0 = k0 * rho; E.k1 = k1 * rho; E.k2 = k2 * rho;
  E.na = rho * A2;
  g1 *= rho; g2 *= rho; g3 *= rho; g4 *= rho; m0 *= rho; m1 *= rho;
#pragma unroll
  for (int b = 0; b < N; ++b) {
    const R y = L.x[b], y2 = L.x2[b];
    R g = g2;
    if constexpr (ORD >= 3) {
      R h = g3;
      if constexpr (ORD >= 4) h = fmaR(y, g4, h);
      g = fmaR(y, h, g);
      E.M[b] = y2 * ((ORD >= 4) ? fmaR(y, m1, m0) : m0);
    } else {
      E.M[b] = R(0);
    }
    E.G[b] = y * fmaR(y, g, g1);
    if constexpr (ORD >= 4) E.Ob[b] = B2 * y2;
  }
}

// x-node terms of node a: F(x_a) (rho-scaled, drho folded in), K(x_a) and
// the rho A2 x_a^2 factor of the order-4 cross term
template <typename R, int N, int ORD>
__device__ __forceinline__ void eq_anode(const Lat<R>& L, const EqNodes<R, N>& E, int a, R& Fa,
                                         R& Ka, R& Na) {
  const R x = L.x[a];
  R f = E.f2, k = E.k0;
  if constexpr (ORD >= 3) {
    R t = E.f3;
    if constexpr (ORD >= 4) t = fmaR(x, E.f4, t);
    f = fmaR(x, t, f);
    k = fmaR(x, (ORD >= 4) ? fmaR(x, E.k2, E.k1) : E.k1, k);
  }
  Fa = fmaR(x, fmaR(x, f, E.f1), E.f0);
  Ka = x * k;
  Na = (ORD >= 4) ? E.na * L.x2[a] : R(0);
}

// drho + rho P_l for population l = (a, b), given node a's terms
template <typename R, int N, int ORD>
__device__ __forceinline__ R eq_dev(const Lat<R>& L, const EqNodes<R, N>& E, int a, int b, R Fa,
                                    R Ka, R Na) {
  R e = Fa + E.G[b];
  e = fmaR(L.x[b], Ka, e);
  if constexpr (ORD >= 3) e = fmaR(L.x[a], E.M[b], e);
  if constexpr (ORD >= 4) e = fmaR(Na, E.Ob[b], e);
  return e;
}

// BGK update in deviation form (eq.(lb) integrated over one step, tau in
// steps):  d* = d + (feq_dev - d)/tau = (1 - 1/tau) d + (w/tau) e,
// e = drho + rho P.
template <typename R>
__device__ __forceinline__ R bgk(R d, R oww_l, R omo, R e) {
  return fmaR(oww_l, e, omo * d);
}

// Equilibrium and BGK of one cell, in place: d[l] <- C(d)[l], given the
// cell's fields F.
template <typename R, int N, int ORD>
__device__ __forceinline__ void bgk_cell(const Lat<R>& L, const Inst<R>& P, const Fields<R>& F,
                                         R (&d)[N * N]) {
  EqNodes<R, N> E;
  eq_nodes<R, N, ORD>(L, F, E);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    R Fa, Ka, Na;
    eq_anode<R, N, ORD>(L, E, a, Fa, Ka, Na);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      d[l] = bgk(d[l], P.oww[l], P.omo, eq_dev<R, N, ORD>(L, E, a, b, Fa, Ka, Na));
    }
  }
}

}  // namespace tvlbm
