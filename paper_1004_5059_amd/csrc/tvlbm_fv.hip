// tvlbm_fv.hip -- HIP kernels of the finite-volume TVLBM update for gfx950:
// eq.(FVLB) on a rectangular mesh (uniform in x, spacings dy_j in y) with
// the second-order 9-point stencils of Sec. III, and diffuse-scattering
// wall points (eq.(FVLB2) with the one-sided stencils of Sec. VII, then
// eq.(IMPOSITION)).  Populations are stored as deviations d = f - w, SoA
// [q][ny][ld], one thread per mesh point, 64 x 4 points per workgroup.
//
// Two schedules of one step:
//   k_fv_march (fused, one pass): every wavefront marches down one row
//     segment of a 62-column strip (lanes 0 and 63 are halo columns),
//     reading d once and writing d' once; see the kernel for the separable
//     form of the stencils that makes this possible;
//   k_fv_omega then k_fv_update (two passes): Omega_l = -(f_l - feq_l)/tau
//     at every point into a scratch array, then d' = d + dt (Omega-bar -
//     c . grad d) with the 3 x 3 stencils reading d and Omega through the
//     caches.
// At wall points the incoming populations use the one-sided stencils and
// the outgoing ones are re-emitted from the new incoming normal flux with
// the fixed wall equilibrium, eq.(IMPOSITION); with slip-free walls
// k_fv_impose then re-emits them again with the Newton-iterated wall
// equilibrium (kept out of the step kernels, whose registers it would
// inflate).
#include "tvlbm_core.h"
#include "tvlbm_fv_launch.h"

namespace tvlbm {

// Equilibrium deviations of one cell, e_l = feq_l / w_l - 1 (Sec. II,
// Appendix A), for every population.  Orders 2-4: the per-node split of the
// lattice step; order 5: Appendix A term by term (u_l = u . c_l,
// c^2 = |c_l|^2, D = 2), e_l = drho + rho P_l with P_l the polynomial
// without its constant 1.
template <typename R, int N, int ORD>
__device__ __forceinline__ void eq_devs(const Lat<R>& L, const Fields<R>& F, R (&e)[N * N]) {
  if constexpr (ORD <= 4) {
    EqNodes<R, N> E;
    eq_nodes<R, N, ORD>(L, F, E);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R Fa, Ka, Na;
      eq_anode<R, N, ORD>(L, E, a, Fa, Ka, Na);
#pragma unroll
      for (int b = 0; b < N; ++b) e[a * N + b] = eq_dev<R, N, ORD>(L, E, a, b, Fa, Ka, Na);
    }
  } else {
    const R U = F.ux, V = F.uy, th = F.th;
    const R u2 = U * U + V * V, th2 = th * th;
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const R ul = fmaR(U, L.x[a], V * L.x[b]);
        const R c2 = L.x2[a] + L.x2[b];
        const R ul2 = ul * ul, ul3 = ul2 * ul;
        R p = ul + R(0.5) * (ul2 - u2 + th * (c2 - R(2)));
        p += ul * (ul2 - R(3) * u2 + R(3) * th * (c2 - R(4))) * R(1.0 / 6.0);
        p += (ul2 * ul2 - R(6) * ul2 * u2 + R(3) * u2 * u2) * R(1.0 / 24.0);
        p += th * ((c2 - R(4)) * (ul2 - u2) - R(2) * ul2) * R(0.25);
        p += th2 * (c2 * c2 - R(8) * c2 + R(8)) * R(0.125);
        p += (ul3 * ul2 - R(10) * u2 * ul3 + R(15) * u2 * u2 * ul) * R(1.0 / 120.0);
        p += th * (c2 * ul3 - R(8) * ul3 - R(3) * c2 * ul * u2 + R(18) * u2 * ul) * R(1.0 / 12.0);
        p += th2 * ul * (c2 * c2 - R(12) * c2 + R(24)) * R(0.125);
        e[a * N + b] = fmaR(F.rho, p, F.drho);
      }
    }
  }
}

// W = tau Omega of one cell from its deviations d (zero without collisions):
// single relaxation W_l = feq_l - f_l, then, when set, the non-unit-Prandtl
// term of eq.(FINAL) and the pressure-rescaled relaxation times (Sec. IX):
//   W_l = ps [ (feq_l - f_l) - (tau / tau_g) feq_l Pi:(c_l - u)(c_l - u) / (rho T^2) ],
//   Pi_ij = sum_l (f_l - feq_l) c_l^i c_l^j  (the central form of eq.(FINAL):
//   f - feq carries no mass or momentum),  ps = rho T or 1.
// The term enters with the sign that relaxes Pi at 2 / tau_g, which gives
// the paper's viscosity c_v rho T tau tau_g / (2 tau + tau_g).
template <typename R, int N, int ORD, bool COMP>
__device__ __forceinline__ void cell_w(const FvArgs<R>& A, const R (&d)[N * N], R (&w)[N * N]) {
  const Lat<R>& L = A.lat;
  if (!A.collide) {
#pragma unroll
    for (int l = 0; l < N * N; ++l) w[l] = R(0);
    return;
  }
  R drho, jx, jy, ed;
  cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
  const Fields<R> F = fields_from(drho, jx, jy, ed);
  eq_devs<R, N, ORD>(L, F, w);
#pragma unroll
  for (int l = 0; l < N * N; ++l) w[l] = fmaR(L.w[l], w[l], -d[l]);
  if (A.tau_ratio == R(0) && !A.pscale) return;
  const R T = R(1) + F.th;
  const R ps = A.pscale ? F.rho * T : R(1);
  if (A.tau_ratio != R(0)) {
    // S_ij = sum_l (feq_l - f_l) c_i c_j = -Pi_ij
    R sxx = R(0), sxy = R(0), syy = R(0), cb[N];
#pragma unroll
    for (int b = 0; b < N; ++b) cb[b] = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R ra = R(0), rx = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const R v = w[a * N + b];
        ra += v;
        rx = fmaR(L.x[b], v, rx);
        cb[b] += v;
      }
      sxx = fmaR(L.x2[a], ra, sxx);
      sxy = fmaR(L.x[a], rx, sxy);
    }
#pragma unroll
    for (int b = 0; b < N; ++b) syy = fmaR(L.x2[b], cb[b], syy);
    const R g = A.tau_ratio / (F.rho * T * T);
    R cy[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const R Y = L.x[b] - F.uy;
      cy[b] = syy * Y * Y;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const R X = L.x[a] - F.ux;
      const R ax = sxx * X * X, bx = R(2) * sxy * X;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const R Y = L.x[b] - F.uy;
        const R q = fmaR(bx, Y, ax) + cy[b];  // -Pi:(c - u)(c - u)
        const R feq = (w[l] + d[l]) + L.w[l];
        w[l] = ps * fmaR(g * feq, q, w[l]);
      }
    }
  } else {
#pragma unroll
    for (int l = 0; l < N * N; ++l) w[l] *= ps;
  }
}

template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_fv_omega(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= A.nx || j >= A.ny) return;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src, bytes);
  const rsrc_t o = make_rsrc(A.om, bytes);
  const uint32_t c = (uint32_t)(j * A.ld + i);
  R d[Q], w[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) d[l] = bld<R>(s, c, (uint32_t)(l * A.plane));
  cell_w<R, N, ORD, COMP>(A, d, w);
#pragma unroll
  for (int l = 0; l < Q; ++l) bst(o, c, (uint32_t)(l * A.plane), w[l] * A.inv_tau);
}

// eq.(IMPOSITION) at a wall point of the new state (tab: kap then phi of
// that wall, FP64 in device memory so that they are loaded only here).  The
// incoming flux and the re-emitted deviations are formed in FP64 and rounded
// once (FP32 copies of the constant kap, phi would add the same rounding to
// the wall mass flux every step).
template <typename R, int N>
__device__ __forceinline__ void impose(const Lat<R>& L, const double* __restrict__ tab, bool top,
                                       R* o) {
  double m = 0.0;
#pragma unroll
  for (int l = 0; l < N * N; ++l) {
    const R cn = top ? -L.x[l % N] : L.x[l % N];
    if (cn <= R(0)) m = __builtin_fma(-(double)L.xd[l % N] * (top ? -1.0 : 1.0), (double)o[l], m);
  }
#pragma unroll
  for (int l = 0; l < N * N; ++l) {
    const R cn = top ? -L.x[l % N] : L.x[l % N];
    if (cn > R(0)) o[l] = (R)__builtin_fma(tab[QMAX + l], m, tab[l]);
  }
}

// Outgoing-moment sums of the unit-density wall equilibrium feq(ue, 0, Te)
// in FP64: Z = sum |c.n| feq, So = sum feq, Sx = sum c_x feq,
// S2 = sum |c|^2 feq over the outgoing populations.
template <int N, int ORD>
__device__ __forceinline__ void wall_sums(const Lat<double>& Ld, const double* wd, bool top,
                                          double ue, double Te, double (&S)[4]) {
  Fields<double> F;
  F.rho = 1.0; F.drho = 0.0; F.ux = ue; F.uy = 0.0; F.th = Te - 1.0;
  double e[N * N];
  eq_devs<double, N, ORD>(Ld, F, e);
  S[0] = S[1] = S[2] = S[3] = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const double cn = top ? -Ld.x[b] : Ld.x[b];
      if (cn <= 0.0) continue;
      const double fe = wd[a * N + b] * (1.0 + e[a * N + b]);
      S[0] = __builtin_fma(cn, fe, S[0]);
      S[1] += fe;
      S[2] = __builtin_fma(Ld.x[a], fe, S[2]);
      S[3] = __builtin_fma(Ld.x2[a] + Ld.x2[b], fe, S[3]);
    }
  }
}

// Slip-free re-emission at a wall point (App. B): the wall equilibrium
// (ue, Te) that makes the point's own x velocity and temperature, after the
// outgoing populations are set to (m / Z) feq(ue, Te), the prescribed
// (uw, Tw):  F1 = rho uw - sum f c_x = 0,  F2 = 2 rho Tw + rho uw^2 - sum f c^2
// = 0.  Newton's method with Appendix B's flux-normalised derivatives plus
// the terms of the point's density (which change with the emitted
// populations), derivatives of the sums by forward differences, all in
// FP64.  par holds the start (the prescribed values, or last step's root)
// and receives the root; iters: 6 from the prescribed values, 3 from last
// step's root (Newton squares a 1e-6 change to round-off in two).  o holds
// the new deviations; the incoming ones are used, the outgoing ones written.
template <typename R, int N, int ORD>
__device__ __forceinline__ void impose_slip_free(const Lat<R>& L, bool top, double uw, double Tw,
                                                 int iters, double (&par)[2], R* o) {
  Lat<double> Ld;
#pragma unroll
  for (int a = 0; a < N; ++a) { Ld.x[a] = L.xd[a]; Ld.x2[a] = L.xd[a] * L.xd[a]; }
  double m = 0.0, rin = 0.0, jin = 0.0, ein = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const double cn = top ? -Ld.x[b] : Ld.x[b];
      if (cn > 0.0) continue;
      const double f = L.wd[a * N + b] + (double)o[a * N + b];
      m = __builtin_fma(-cn, f, m);
      rin += f;
      jin = __builtin_fma(Ld.x[a], f, jin);
      ein = __builtin_fma(Ld.x2[a] + Ld.x2[b], f, ein);
    }
  const double h = 1e-7, w2 = 2.0 * Tw + uw * uw;
  double ue = par[0], Te = par[1];
  for (int it = 0; it < iters; ++it) {
    double S[4], Su[4], St[4];
    wall_sums<N, ORD>(Ld, L.wd, top, ue, Te, S);
    wall_sums<N, ORD>(Ld, L.wd, top, ue + h, Te, Su);
    wall_sums<N, ORD>(Ld, L.wd, top, ue, Te + h, St);
    double du[4], dt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      du[k] = (Su[k] - S[k]) / h;
      dt[k] = (St[k] - S[k]) / h;
    }
    const double Z = S[0], s = m / Z;
    const double rho = rin + s * S[1];
    const double F1 = rho * uw - (jin + s * S[2]);
    const double F2 = w2 * rho - (ein + s * S[3]);
    // d(moment)/dp * Z / m = dS_k/dp - (dZ/dp) S_k / Z, k = density, c_x, c^2
    const double Ru = du[1] - du[0] * S[1] / Z, Rt = dt[1] - dt[0] * S[1] / Z;
    const double A = du[2] - du[0] * S[2] / Z - uw * Ru;
    const double B = dt[2] - dt[0] * S[2] / Z - uw * Rt;
    const double C = du[3] - du[0] * S[3] / Z - w2 * Ru;
    const double D = dt[3] - dt[0] * S[3] / Z - w2 * Rt;
    const double k = Z / ((A * D - B * C) * m);
    ue += k * (D * F1 - B * F2);
    Te += k * (A * F2 - C * F1);
  }
  par[0] = ue;
  par[1] = Te;
  double S[4];
  wall_sums<N, ORD>(Ld, L.wd, top, ue, Te, S);
  const double s = m / S[0];
  Fields<double> F;
  F.rho = 1.0; F.drho = 0.0; F.ux = ue; F.uy = 0.0; F.th = Te - 1.0;
  double e[N * N];
  eq_devs<double, N, ORD>(Ld, F, e);
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const double cn = top ? -Ld.x[b] : Ld.x[b];
      if (cn <= 0.0) continue;
      const int l = a * N + b;
      o[l] = (R)__builtin_fma(s, L.wd[l] * (1.0 + e[l]), -L.wd[l]);
    }
  }
}

template <typename R, int N, int ORD>
__global__ __launch_bounds__(256) void k_fv_update(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= A.nx || j >= A.ny) return;
  const Lat<R>& L = A.lat;
  const int nx = A.nx, ny = A.ny;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src, bytes);
  const rsrc_t om = make_rsrc(A.om, bytes);
  const rsrc_t dst = make_rsrc(A.dst, bytes);
  const uint32_t ld = (uint32_t)A.ld;
  // x neighbours: periodic, or the end point itself beyond a zero-gradient end
  const int ip = i + 1 == nx ? (A.x_open ? nx - 1 : 0) : i + 1;
  const int im = i == 0 ? (A.x_open ? 0 : nx - 1) : i - 1;
  const bool wlo = A.walls && j == 0, whi = A.walls && j == ny - 1;
  const R dt = A.dt, cxk = A.inv_dx, cyk = A.cy[j];
  const uint32_t r0 = (uint32_t)j * ld;
  if (!wlo && !whi) {
    // interior point (Sec. III): neighbours 1 (+x), 2 (+y), 3 (-x), 4 (-y),
    // 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y)
    const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
    const uint32_t rp = (uint32_t)jp * ld, rm = (uint32_t)jm * ld;
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const uint32_t pl = (uint32_t)(l * A.plane);
        const R f0 = bld<R>(s, r0 + i, pl);
        const R f1 = bld<R>(s, r0 + ip, pl), f2 = bld<R>(s, rp + i, pl);
        const R f3 = bld<R>(s, r0 + im, pl), f4 = bld<R>(s, rm + i, pl);
        const R f5 = bld<R>(s, rp + ip, pl), f6 = bld<R>(s, rp + im, pl);
        const R f7 = bld<R>(s, rm + im, pl), f8 = bld<R>(s, rm + ip, pl);
        const R dfx = cxk * (R(3.0 / 8.0) * f1 - R(3.0 / 8.0) * f3 + R(1.0 / 16.0) * f5 -
                             R(1.0 / 16.0) * f6 - R(1.0 / 16.0) * f7 + R(1.0 / 16.0) * f8);
        const R dfy = cyk * (R(3.0 / 8.0) * f2 - R(3.0 / 8.0) * f4 + R(1.0 / 16.0) * f5 +
                             R(1.0 / 16.0) * f6 - R(1.0 / 16.0) * f7 - R(1.0 / 16.0) * f8);
        const R w0 = bld<R>(om, r0 + i, pl);
        const R w1 = bld<R>(om, r0 + ip, pl), w2 = bld<R>(om, rp + i, pl);
        const R w3 = bld<R>(om, r0 + im, pl), w4 = bld<R>(om, rm + i, pl);
        const R w5 = bld<R>(om, rp + ip, pl), w6 = bld<R>(om, rp + im, pl);
        const R w7 = bld<R>(om, rm + im, pl), w8 = bld<R>(om, rm + ip, pl);
        const R omb = R(9.0 / 16.0) * w0 + R(3.0 / 32.0) * (((w1 + w2) + w3) + w4) +
                      R(1.0 / 64.0) * (((w5 + w6) + w7) + w8);
        const R out = f0 + dt * (omb - (L.x[a] * dfx + L.x[b] * dfy));
        bst(dst, r0 + i, pl, out);
      }
    }
    return;
  }
  // wall point (Sec. VII): neighbour 2 is the next point into the fluid, 5
  // and 6 its +x / -x neighbours; the y derivative is one-sided along the
  // inward normal
  const uint32_t r2 = (uint32_t)(whi ? ny - 2 : 1) * ld;
  R out[Q];
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      const R cn = whi ? -L.x[b] : L.x[b];
      out[l] = R(0);
      if (cn > R(0)) continue;
      const uint32_t pl = (uint32_t)(l * A.plane);
      const R f0 = bld<R>(s, r0 + i, pl);
      const R f1 = bld<R>(s, r0 + ip, pl), f3 = bld<R>(s, r0 + im, pl);
      const R f2 = bld<R>(s, r2 + i, pl), f5 = bld<R>(s, r2 + ip, pl), f6 = bld<R>(s, r2 + im, pl);
      const R dfx = cxk * (R(3.0 / 8.0) * f1 - R(3.0 / 8.0) * f3 + R(1.0 / 8.0) * f5 -
                           R(1.0 / 8.0) * f6);
      const R dn = cyk * (R(3.0 / 8.0) * f2 - R(3.0 / 8.0) * f0 + R(1.0 / 16.0) * f5 +
                          R(1.0 / 16.0) * f6 - R(1.0 / 16.0) * f1 - R(1.0 / 16.0) * f3);
      const R dfy = whi ? -dn : dn;
      const R w0 = bld<R>(om, r0 + i, pl);
      const R w1 = bld<R>(om, r0 + ip, pl), w3 = bld<R>(om, r0 + im, pl);
      const R w2 = bld<R>(om, r2 + i, pl), w5 = bld<R>(om, r2 + ip, pl), w6 = bld<R>(om, r2 + im, pl);
      const R omb = R(9.0 / 16.0) * w0 + R(3.0 / 32.0) * w1 + R(3.0 / 16.0) * w2 +
                    R(3.0 / 32.0) * w3 + R(1.0 / 32.0) * w5 + R(1.0 / 32.0) * w6;
      out[l] = f0 + dt * (omb - (L.x[a] * dfx + L.x[b] * dfy));
    }
  }
  // the outgoing populations: eq.(IMPOSITION) (a slip-free wall replaces
  // them afterwards, k_fv_impose)
  impose<R, N>(L, A.wtab + (whi ? 2 * QMAX : 0), whi, out);
#pragma unroll
  for (int l = 0; l < Q; ++l) bst(dst, r0 + i, (uint32_t)(l * A.plane), out[l]);
}

// The wall model in place at both wall rows: after tvlbm_fv_set_fields,
// and after every step with slip-free walls (the step kernels re-emit with
// the fixed wall equilibrium; this replaces the outgoing populations).
template <typename R, int N, int ORD>
__global__ __launch_bounds__(256) void k_fv_impose(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int side = blockIdx.y;  // 0: first row, 1: last row
  if (i >= A.nx || !A.walls) return;
  const bool whi = side == 1;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.dst, bytes);
  const uint32_t c = (uint32_t)((whi ? A.ny - 1 : 0) * A.ld + i);
  R o[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) o[l] = bld<R>(s, c, (uint32_t)(l * A.plane));
  if (A.slip_free) {
    double* wp = A.wpar + 2 * ((int64_t)side * A.nx + i);
    double par[2] = {A.wall_u[side], A.wall_T[side]};
    if (A.nr_warm) { par[0] = wp[0]; par[1] = wp[1]; }
    impose_slip_free<R, N, ORD>(A.lat, whi, A.wall_u[side], A.wall_T[side], A.nr_warm ? 3 : 6,
                                par, o);
    wp[0] = par[0];
    wp[1] = par[1];
  } else {
    impose<R, N>(A.lat, A.wtab + (whi ? 2 * QMAX : 0), whi, o);
  }
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const R cn = whi ? -A.lat.x[l % N] : A.lat.x[l % N];
    if (cn > R(0)) bst(s, c, (uint32_t)(l * A.plane), o[l]);
  }
}

// f = d + w into a dense [q][ny][nx] array.
template <typename R, int N>
__global__ __launch_bounds__(256) void k_fv_pops(const FvArgs<R> A, R* out) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= A.nx || j >= A.ny) return;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src, bytes);
  const int64_t np = (int64_t)A.nx * A.ny, o = (int64_t)j * A.nx + i;
#pragma unroll
  for (int l = 0; l < Q; ++l)
    out[l * np + o] = bld<R>(s, (uint32_t)(j * A.ld + i), (uint32_t)(l * A.plane)) + A.lat.w[l];
}

// Fields and FP64 totals (weights dx * dual-cell height) of the state.
template <typename R, int N, bool COMP>
__global__ __launch_bounds__(256) void k_fv_fields(const FvArgs<R> A, R* fields, double* partials) {
  constexpr int Q = N * N;
  __shared__ double sh[4][4];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const Lat<R>& L = A.lat;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < A.nx && j < A.ny) {
    const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
    const rsrc_t s = make_rsrc(A.src, bytes);
    const uint32_t c = (uint32_t)(j * A.ld + i);
    R d[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) d[l] = bld<R>(s, c, (uint32_t)(l * A.plane));
    R drho, jx, jy, ed;
    cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
    const Fields<R> F = fields_from(drho, jx, jy, ed);
    if (fields) {
      const int64_t np = (int64_t)A.nx * A.ny, o = (int64_t)j * A.nx + i;
      fields[o] = F.rho;
      fields[np + o] = F.ux;
      fields[2 * np + o] = F.uy;
      fields[3 * np + o] = R(1) + F.th;
    }
    const double v = A.vol[j];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const double fa = L.wd[l] + (double)d[l];
        t[0] += v * fa;
        t[1] += v * L.xd[a] * fa;
        t[2] += v * L.xd[b] * fa;
        t[3] += v * 0.5 * (L.xd[a] * L.xd[a] + L.xd[b] * L.xd[b]) * fa;
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] += __shfl_xor(t[k], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[wave][k] = t[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[b * 4 + k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
  }
}


// ------------------------------------------------------- fused march ---
// The stencils of Sec. III are tensor products of 1-D three-point stencils:
// with S = [1/8, 3/4, 1/8] and the central difference D = [-1, 0, 1],
//   Omega-bar = S_x S_y Omega,
//   d/dx f    = S_y D_x f / (2 dx),
//   d/dy f    = D_y S_x f * cy_j / 2,   cy_j = 2 / (dy_{j-1} + dy_j),
// and the wall stencils of eq.(FVLB2) are the same with S_y replaced by
// [3/4, 1/4] (wall row, row into the fluid) and D_y by the one-sided
// difference.  So one row r needs, per population, the row quantities
//   a = S_x d,  e = dt S_x Omega - dt c_x D_x d / (2 dx)
// and the update of row j is
//   d'_j = d_j + 3/4 e_j + 1/8 (e_{j-1} + e_{j+1}) - h_j (a_{j+1} - a_{j-1}),
//   h_j = dt c_y cy_j / 2,
// which a wavefront marching down y accumulates with two partial sums per
// population: P (row j, waiting for row j+1) and pre (row j+1, from row j).
// The x neighbours come from the adjacent lanes (DPP wave shifts).

// Value held by lane k-1 (FROM_PREV, wave_shr:1) or k+1 (FROM_NEXT,
// wave_shl:1) of the wavefront; the end lanes receive 0 (halo lanes).
constexpr int DPP_FROM_PREV = 0x138;
constexpr int DPP_FROM_NEXT = 0x130;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename R, int N>
__device__ __forceinline__ void load_row(rsrc_t s, uint32_t c, int64_t plane, R* d) {
#pragma unroll
  for (int l = 0; l < N * N; ++l) d[l] = bld<R>(s, c, (uint32_t)(l * plane));
}

template <typename R, int N>
__device__ __forceinline__ void store_row(rsrc_t dst, uint32_t c, int64_t plane, const R* o) {
#pragma unroll
  for (int l = 0; l < N * N; ++l) bst(dst, c, (uint32_t)(l * plane), o[l]);
}

// Per-wavefront constants of the march.  A segment's wavefront marches
// down (dir = +1) or up (dir = -1) its rows; neighbouring segments march in
// opposite directions, so the two reads of every halo row fall together and
// the second one hits L2.
template <typename R>
struct MarchC {
  rsrc_t s, dst;
  uint32_t ld, col;
  int ny, y0, y1, first, last, dir;
  bool walls, out_lane;
  R c1, c2, hx8, hh8;
  __device__ int wrap(int r) const { return r < 0 ? r + ny : (r >= ny ? r - ny : r); }
  __device__ uint32_t cell(int r) const { return (uint32_t)wrap(r) * ld + col; }
  __device__ bool out(int r) const { return r >= y0 && r < y1; }
  __device__ bool wall(int r) const { return walls && (r == 0 || r == ny - 1); }
};

// Scaled row quantities of population l: a8 = 8 a, e = E (= e / 8).
template <typename R, int N>
__device__ __forceinline__ void row_quant(const MarchC<R>& C, R hxa, R d, R w, R& a8, R& e) {
  const R dm = lane_shift<DPP_FROM_PREV>(d), dp = lane_shift<DPP_FROM_NEXT>(d);
  const R wm = lane_shift<DPP_FROM_PREV>(w), wp = lane_shift<DPP_FROM_NEXT>(w);
  a8 = fmaR(R(6), d, dm + dp);
  e = fmaR(C.c1, wm + wp, fmaR(C.c2, w, -(hxa * (dp - dm))));
}

// The marching form of d'_j = d_j + 6 E_j + E_{j-1} + E_{j+1}
// - (h_j / 8)(a8_{j+1} - a8_{j-1}): with p = r - dir the row finished when
// row r arrives and n = r + dir the row started,
//   d'_p = P + E_r - dir (h_p / 8) a8_r,   P <- d_r + 6 E_r + pre,
//   pre  <- E_r + dir (h_n / 8) a8_r.
// An interior row between interior rows: finish p (store), carry r, start n.
template <typename R, int N>
__device__ __forceinline__ void row_steady(const FvArgs<R>& A, const MarchC<R>& C, int r,
                                           const R (&d)[N * N], const R (&w)[N * N],
                                           R (&P)[N * N], R (&pre)[N * N]) {
  const Lat<R>& L = A.lat;
  const R sh = C.dir > 0 ? C.hh8 : -C.hh8;
  const R hp = sh * A.cy[C.wrap(r - C.dir)], hn = sh * A.cy[C.wrap(r + C.dir)];
  R hpb[N], hnb[N];
#pragma unroll
  for (int b = 0; b < N; ++b) { hpb[b] = hp * L.x[b]; hnb[b] = hn * L.x[b]; }
  const uint32_t cprev = C.cell(r - C.dir);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const R hxa = C.hx8 * L.x[a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      R a8, e;
      row_quant<R, N>(C, hxa, d[l], w[l], a8, e);
      const R v = fmaR(-hpb[b], a8, P[l] + e);
      if (C.out_lane) bst(C.dst, cprev, (uint32_t)(l * A.plane), v);
      P[l] = fmaR(R(6), e, d[l]) + pre[l];
      pre[l] = fmaR(hnb[b], a8, e);
    }
  }
}

// Any row (segment ends, wall rows): E-weights 1 in the interior and 2 (1/4
// unscaled) towards a wall row; a wall row's own a-term is +h a at the
// bottom and -h a at the top (one-sided difference, eq.(FVLB2)); wall rows
// are re-emitted, eq.(IMPOSITION), before they are stored.  A wall row that
// ends the march is finished on arrival.
template <typename R, int N, int ORD>
__device__ __forceinline__ void row_general(const FvArgs<R>& A, const MarchC<R>& C, int r,
                                            const R (&d)[N * N], const R (&w)[N * N],
                                            R (&P)[N * N], R (&pre)[N * N]) {
  const Lat<R>& L = A.lat;
  const int ny = C.ny, p = r - C.dir, n = r + C.dir;
  const bool prev_out = r != C.first && C.out(p);
  const bool cur_final = C.out(r) && r == C.last;
  const R sh = C.dir > 0 ? C.hh8 : -C.hh8;
  const R hp = sh * A.cy[C.wrap(p)], hn = sh * A.cy[C.wrap(n)];
  const R hc = C.hh8 * A.cy[C.wrap(r)];
  const R bprev = C.wall(p) ? R(2) : R(1), bnext = C.wall(n) ? R(2) : R(1);
  const R kc = (C.walls && r == 0) ? hc : ((C.walls && r == ny - 1) ? -hc : R(0));
  R o[N * N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const R hxa = C.hx8 * L.x[a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      R a8, e;
      row_quant<R, N>(C, hxa, d[l], w[l], a8, e);
      o[l] = fmaR(-(hp * L.x[b]), a8, fmaR(bprev, e, P[l]));          // row p
      P[l] = fmaR(kc * L.x[b], a8, fmaR(R(6), e, d[l]) + pre[l]);     // row r
      pre[l] = fmaR(hn * L.x[b], a8, bnext * e);                      // row n
    }
  }
  if (prev_out) {
    if (C.wall(p)) impose<R, N>(L, A.wtab + (p == 0 ? 0 : 2 * QMAX), p != 0, o);
    if (C.out_lane) store_row<R, N>(C.dst, C.cell(p), A.plane, o);
  }
  if (cur_final) {
    impose<R, N>(L, A.wtab + (r == 0 ? 0 : 2 * QMAX), r != 0, P);
    if (C.out_lane) store_row<R, N>(C.dst, C.cell(r), A.plane, P);
  }
}

template <typename R, int N, int ORD, bool COMP, bool PF>
__global__ __launch_bounds__(256) void k_fv_march(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // workgroups go round-robin to the 8 XCDs: give each XCD a contiguous
  // band of tiles (gridDim.x is a multiple of 8)
  const int nb = gridDim.x;
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int strip = t % A.strips;
  const int seg = (t / A.strips) * 4 + wave;
  if (seg >= A.segs) return;  // whole wavefront
  const Lat<R>& L = A.lat;
  const int nx = A.nx, ny = A.ny;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  MarchC<R> C;
  C.s = make_rsrc(A.src, bytes);
  C.dst = make_rsrc(A.dst, bytes);
  C.ld = (uint32_t)A.ld;
  C.ny = ny;
  C.walls = A.walls != 0;
  C.y0 = seg * A.seg_rows;
  C.y1 = min(C.y0 + A.seg_rows, ny);
  const int x0 = strip * 62;
  // lanes 0 and 63 hold the strip's halo columns: periodic images, or at a
  // zero-gradient end the end column itself (f(-dx) = f(0))
  C.col = A.x_open ? (uint32_t)min(max(x0 - 1 + lane, 0), nx - 1)
                   : (uint32_t)((x0 - 1 + lane + nx) % nx);
  C.out_lane = lane >= 1 && lane <= 62 && x0 - 1 + lane < nx;
  // Scaled row quantities: a8 = 8 a = (d_{i-1} + d_{i+1}) + 6 d and
  // E = e / 8 = c1 (W_{i-1} + W_{i+1}) + c2 W - hx8_a (d_{i+1} - d_{i-1}),
  // W = w_l feq-deviation - d = tau Omega, c1 = dt / (64 tau),
  // c2 = 3 dt / (32 tau), hx8_a = dt c_x / (16 dx), h_j / 8 = hh8 c_y cy_j.
  C.c1 = A.dt * A.inv_tau * R(1.0 / 64.0);
  C.c2 = A.dt * A.inv_tau * R(3.0 / 32.0);
  C.hx8 = A.dt * A.inv_dx * R(1.0 / 16.0);
  C.hh8 = A.dt * R(1.0 / 16.0);
  // rows rs..re: the segment and its halo (wall rows have none outside)
  const int rs = C.walls ? max(C.y0 - 1, 0) : C.y0 - 1;
  const int re = C.walls ? min(C.y1, ny - 1) : C.y1;
  C.dir = (seg & 1) ? -1 : 1;
  C.first = C.dir > 0 ? rs : re;
  C.last = C.dir > 0 ? re : rs;
  // steady rows: previous and next rows are interior rows of the march
  int s0, s1;
  if (C.dir > 0) { s0 = max(C.y0 + 1, rs + 1); s1 = min(C.y1 - 1, re - 1); }
  else { s0 = max(C.y0, rs + 1); s1 = min(C.y1 - 2, re - 1); }
  if (C.walls) { s0 = max(s0, 2); s1 = min(s1, ny - 3); }
  const int nst = s1 >= s0 ? s1 - s0 + 1 : 0;
  const int sa = C.dir > 0 ? s0 : s1;  // first steady row in march order

  R P[Q], pre[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) { P[l] = R(0); pre[l] = R(0); }
  // rows before the steady run (all rows if there is none)
  const int ng = nst ? (sa - C.first) * C.dir : (re - rs + 1);
  int r = C.first;
  for (int k = 0; k < ng; ++k, r += C.dir) {
    R d[Q], w[Q];
    load_row<R, N>(C.s, C.cell(r), A.plane, d);
    cell_w<R, N, ORD, COMP>(A, d, w);
    row_general<R, N, ORD>(A, C, r, d, w, P, pre);
  }
  if (!nst) return;
  if constexpr (PF) {
    // two row buffers in turn: the next row loads while this one is used
    R ba[Q], bb[Q];
    load_row<R, N>(C.s, C.cell(r), A.plane, ba);
    int k = 0;
    for (; k + 1 < nst; k += 2, r += 2 * C.dir) {
      load_row<R, N>(C.s, C.cell(r + C.dir), A.plane, bb);
      {
        R w[Q];
        cell_w<R, N, ORD, COMP>(A, ba, w);
        row_steady<R, N>(A, C, r, ba, w, P, pre);
      }
      if (k + 2 < nst) load_row<R, N>(C.s, C.cell(r + 2 * C.dir), A.plane, ba);
      {
        R w[Q];
        cell_w<R, N, ORD, COMP>(A, bb, w);
        row_steady<R, N>(A, C, r + C.dir, bb, w, P, pre);
      }
    }
    if (k < nst) {
      R w[Q];
      cell_w<R, N, ORD, COMP>(A, ba, w);
      row_steady<R, N>(A, C, r, ba, w, P, pre);
      r += C.dir;
    }
  } else {
    for (int k = 0; k < nst; ++k, r += C.dir) {
      R d[Q], w[Q];
      load_row<R, N>(C.s, C.cell(r), A.plane, d);
      cell_w<R, N, ORD, COMP>(A, d, w);
      row_steady<R, N>(A, C, r, d, w, P, pre);
    }
  }
  // rows after the steady run
  for (; r != C.last + C.dir; r += C.dir) {
    R d[Q], w[Q];
    load_row<R, N>(C.s, C.cell(r), A.plane, d);
    cell_w<R, N, ORD, COMP>(A, d, w);
    row_general<R, N, ORD>(A, C, r, d, w, P, pre);
  }
}

// ------------------------------------------------------------ band march ---
// The same update with the four wavefronts of a workgroup sharing one row
// segment of a strip: in band k, wavefront w processes row rs + 4k + w, so
// a long segment (few halo rows) still gives four wavefronts.  A row r
// contributes
//   A_r = d_r + 6 E_r [+- h_r/8 a8_r at a wall row]   (itself),
//   U_r = b E_r + (h_{r+1}/8) a8_r                     (the row above),
//   D_r = b E_r - (h_{r-1}/8) a8_r                     (the row below),
// b = 2 towards a wall row, 1 otherwise, and d'_r = A_r + U_{r-1} + D_{r+1}
// (the march's partial sums, regrouped).  U and D go through LDS; rows of
// wavefronts 0-2 finish in their band, wavefront 3's row in the next one
// (an extra band at the end finishes the last).  FP32 with q <= 16 (the
// exchange takes 8 q 64 4 bytes = 32 KiB of LDS for D2Q16).
template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_fv_band(const FvArgs<R> A) {
  constexpr int Q = N * N;
  __shared__ R xs[2][4][Q][64];  // [U, D][wavefront][population][lane]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int strip = t % A.strips, seg = t / A.strips;
  if (seg >= A.segs) return;  // whole workgroup
  const Lat<R>& L = A.lat;
  const int nx = A.nx, ny = A.ny;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  MarchC<R> C;
  C.s = make_rsrc(A.src, bytes);
  C.dst = make_rsrc(A.dst, bytes);
  C.ld = (uint32_t)A.ld;
  C.ny = ny;
  C.walls = A.walls != 0;
  C.y0 = seg * A.seg_rows;
  C.y1 = min(C.y0 + A.seg_rows, ny);
  const int x0 = strip * 62;
  C.col = A.x_open ? (uint32_t)min(max(x0 - 1 + lane, 0), nx - 1)
                   : (uint32_t)((x0 - 1 + lane + nx) % nx);
  C.out_lane = lane >= 1 && lane <= 62 && x0 - 1 + lane < nx;
  C.c1 = A.dt * A.inv_tau * R(1.0 / 64.0);
  C.c2 = A.dt * A.inv_tau * R(3.0 / 32.0);
  C.hx8 = A.dt * A.inv_dx * R(1.0 / 16.0);
  C.hh8 = A.dt * R(1.0 / 16.0);
  const int rs = C.walls ? max(C.y0 - 1, 0) : C.y0 - 1;
  const int re = C.walls ? min(C.y1, ny - 1) : C.y1;
  C.dir = 1;
  C.first = rs;
  C.last = re;
  const int bands = (re - rs + 1 + 3) / 4 + 1;

  R carry[Q], pend[Q];  // wavefront 0: U of the previous band's last row; 3: its own row
#pragma unroll
  for (int l = 0; l < Q; ++l) { carry[l] = R(0); pend[l] = R(0); }
  int prow = -1;
  for (int k = 0; k < bands; ++k) {
    const int r = rs + 4 * k + wave;
    const bool act = r <= re;
    R own[Q];
    if (act) {
      R d[Q], w[Q];
      load_row<R, N>(C.s, C.cell(r), A.plane, d);
      cell_w<R, N, ORD, COMP>(A, d, w);
      const R hp = C.hh8 * A.cy[C.wrap(r - 1)], hn = C.hh8 * A.cy[C.wrap(r + 1)];
      const R hc = C.hh8 * A.cy[C.wrap(r)];
      const R bp = C.wall(r - 1) ? R(2) : R(1), bn = C.wall(r + 1) ? R(2) : R(1);
      const R kc = (C.walls && r == 0) ? hc : ((C.walls && r == ny - 1) ? -hc : R(0));
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const R hxa = C.hx8 * L.x[a];
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          R a8, e;
          row_quant<R, N>(C, hxa, d[l], w[l], a8, e);
          own[l] = fmaR(kc * L.x[b], a8, fmaR(R(6), e, d[l]));
          xs[0][wave][l][lane] = fmaR(hn * L.x[b], a8, bn * e);
          xs[1][wave][l][lane] = fmaR(-(hp * L.x[b]), a8, bp * e);
        }
      }
    } else {
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        own[l] = R(0);
        xs[0][wave][l][lane] = R(0);
        xs[1][wave][l][lane] = R(0);
      }
    }
    __syncthreads();
    if (wave < 3) {
      if (act && C.out(r)) {
#pragma unroll
        for (int l = 0; l < Q; ++l)
          own[l] += (wave == 0 ? carry[l] : xs[0][wave - 1][l][lane]) + xs[1][wave + 1][l][lane];
        if (C.wall(r)) impose<R, N>(L, A.wtab + (r == 0 ? 0 : 2 * QMAX), r != 0, own);
        if (C.out_lane) store_row<R, N>(C.dst, C.cell(r), A.plane, own);
      }
      if (wave == 0) {
#pragma unroll
        for (int l = 0; l < Q; ++l) carry[l] = xs[0][3][l][lane];
      }
    } else {
      if (prow >= 0 && C.out(prow)) {
#pragma unroll
        for (int l = 0; l < Q; ++l) pend[l] += xs[1][0][l][lane];
        if (C.wall(prow)) impose<R, N>(L, A.wtab + (prow == 0 ? 0 : 2 * QMAX), prow != 0, pend);
        if (C.out_lane) store_row<R, N>(C.dst, C.cell(prow), A.plane, pend);
      }
      prow = act ? r : -1;
      if (act) {
#pragma unroll
        for (int l = 0; l < Q; ++l) pend[l] = own[l] + xs[0][2][l][lane];
      }
    }
    __syncthreads();
  }
}

// f = feq(rho, u, T) + noise as deviations d = f - w (Sec. II).
template <typename R, int N, int ORD>
__global__ __launch_bounds__(256) void k_fv_init(const FvArgs<R> A, const FvInit<R> I) {
  constexpr int Q = N * N;
  const int64_t n = (int64_t)A.nx * A.ny;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const int j = (int)(c / A.nx), i = (int)(c % A.nx);
  Fields<R> F;
  F.rho = I.rho[c];
  F.drho = F.rho - R(1);
  F.ux = I.ux[c];
  F.uy = I.uy[c];
  F.th = I.T[c] - R(1);
  R e[Q];
  eq_devs<R, N, ORD>(A.lat, F, e);
  const int64_t o = (int64_t)j * A.ld + i;
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    R v = A.lat.w[l] * e[l];
    if (I.noise) v += I.noise[l * n + c];
    A.dst[o + l * A.plane] = v;
  }
}

// ------------------------------------------------------------- dispatch ---
template <typename R, int N, int ORD, bool COMP>
static hipError_t fv_launch(int what, const FvArgs<R>& A, R* fields, double* partials,
                            hipStream_t st) {
  const dim3 g((unsigned)((A.nx + 63) / 64), (unsigned)((A.ny + 3) / 4)), b(256);
  switch (what) {
    case FV_OMEGA: hipLaunchKernelGGL((k_fv_omega<R, N, ORD, COMP>), g, b, 0, st, A); break;
    case FV_UPDATE: hipLaunchKernelGGL((k_fv_update<R, N, ORD>), g, b, 0, st, A); break;
    case FV_IMPOSE:
      hipLaunchKernelGGL((k_fv_impose<R, N, ORD>), dim3((unsigned)((A.nx + 255) / 256), 2), b, 0, st,
                         A);
      break;
    case FV_POPS: hipLaunchKernelGGL((k_fv_pops<R, N>), g, b, 0, st, A, fields); break;
    case FV_MARCH: {
      // one tile = 4 wavefronts = 4 consecutive segments of one strip
      const int tiles = A.strips * ((A.segs + 3) / 4);
      const dim3 gm((unsigned)((tiles + 7) / 8 * 8));
      if (A.prefetch)
        hipLaunchKernelGGL((k_fv_march<R, N, ORD, COMP, true>), gm, b, 0, st, A);
      else
        hipLaunchKernelGGL((k_fv_march<R, N, ORD, COMP, false>), gm, b, 0, st, A);
      break;
    }
    case FV_BAND: {
      if constexpr (sizeof(R) == 4 && N <= 4) {
        const int tiles = A.strips * A.segs;  // one workgroup per segment
        hipLaunchKernelGGL((k_fv_band<R, N, ORD, COMP>), dim3((unsigned)((tiles + 7) / 8 * 8)), b, 0, st,
                           A);
      } else {
        return hipErrorInvalidValue;
      }
      break;
    }
    default: hipLaunchKernelGGL((k_fv_fields<R, N, COMP>), g, b, 0, st, A, fields, partials); break;
  }
  return hipGetLastError();
}

template <typename R, bool COMP>
static hipError_t fv_lat(int n, int ord, int what, const FvArgs<R>& A, R* fields, double* partials,
                         hipStream_t st) {
  if (n == 3 && ord == 2) return fv_launch<R, 3, 2, COMP>(what, A, fields, partials, st);
  if (n == 4 && ord == 3) return fv_launch<R, 4, 3, COMP>(what, A, fields, partials, st);
  if (n == 6 && ord == 4) return fv_launch<R, 6, 4, COMP>(what, A, fields, partials, st);
  if (n == 6 && ord == 5) return fv_launch<R, 6, 5, COMP>(what, A, fields, partials, st);
  return hipErrorInvalidValue;
}

hipError_t launch_fv(int n, int ord, bool comp, int what, const FvArgs<float>& A, float* fields,
                     double* partials, hipStream_t st) {
  return comp ? fv_lat<float, true>(n, ord, what, A, fields, partials, st)
              : fv_lat<float, false>(n, ord, what, A, fields, partials, st);
}
hipError_t launch_fv(int n, int ord, bool comp, int what, const FvArgs<double>& A, double* fields,
                     double* partials, hipStream_t st) {
  (void)comp;
  return fv_lat<double, false>(n, ord, what, A, fields, partials, st);
}

template <typename R>
static hipError_t fv_init(int n, int ord, const FvArgs<R>& A, const FvInit<R>& I, hipStream_t st) {
  const dim3 g((unsigned)(((int64_t)A.nx * A.ny + 255) / 256)), b(256);
  if (n == 3 && ord == 2) hipLaunchKernelGGL((k_fv_init<R, 3, 2>), g, b, 0, st, A, I);
  else if (n == 4 && ord == 3) hipLaunchKernelGGL((k_fv_init<R, 4, 3>), g, b, 0, st, A, I);
  else if (n == 6 && ord == 4) hipLaunchKernelGGL((k_fv_init<R, 6, 4>), g, b, 0, st, A, I);
  else if (n == 6 && ord == 5) hipLaunchKernelGGL((k_fv_init<R, 6, 5>), g, b, 0, st, A, I);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_fv_init(int n, int ord, const FvArgs<float>& A, const FvInit<float>& I,
                          hipStream_t st) {
  return fv_init(n, ord, A, I, st);
}
hipError_t launch_fv_init(int n, int ord, const FvArgs<double>& A, const FvInit<double>& I,
                          hipStream_t st) {
  return fv_init(n, ord, A, I, st);
}

}  // namespace tvlbm
