// tvlbm_fv.hip -- HIP kernels of the finite-volume TVLBM update for gfx950:
// eq.(FVLB) on a rectangular mesh (uniform in x, spacings dy_j in y) with
// the second-order 9-point stencils of Sec. III, and diffuse-scattering
// wall points (eq.(FVLB2) with the one-sided stencils of Sec. VII, then
// eq.(IMPOSITION)).  Populations are stored as deviations d = f - w, SoA
// [q][ny][ld], one thread per mesh point, 64 x 4 points per workgroup.
//
// A step is two launches:
//   k_fv_omega: Omega_l = -(f_l - feq_l)/tau at every point (compensated
//     moments and the per-node equilibrium of the fused lattice step);
//   k_fv_update: d' = d + dt (Omega-bar - c . grad d), the stencils reading
//     d and Omega at the 3 x 3 neighbourhood through the caches; at wall
//     points the incoming populations use the one-sided stencils and the
//     outgoing ones are re-emitted from the new incoming normal flux.
#include "tvlbm_core.h"
#include "tvlbm_fv_launch.h"

namespace tvlbm {

template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_fv_omega(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= A.nx || j >= A.ny) return;
  const Lat<R>& L = A.lat;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src, bytes);
  const rsrc_t o = make_rsrc(A.om, bytes);
  const uint32_t c = (uint32_t)(j * A.ld + i);
  R d[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) d[l] = bld<R>(s, c, (uint32_t)(l * A.plane));
  if (!A.collide) {
#pragma unroll
    for (int l = 0; l < Q; ++l) bst(o, c, (uint32_t)(l * A.plane), R(0));
    return;
  }
  R drho, jx, jy, ed;
  cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
  const Fields<R> F = fields_from(drho, jx, jy, ed);
  EqNodes<R, N> E;
  eq_nodes<R, N, ORD>(L, F, E);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    R Fa, Ka, Na;
    eq_anode<R, N, ORD>(L, E, a, Fa, Ka, Na);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      // -(f - feq)/tau in deviations: (w_l e_l - d_l)/tau
      const R om = fmaR(L.w[l], eq_dev<R, N, ORD>(L, E, a, b, Fa, Ka, Na), -d[l]) * A.inv_tau;
      bst(o, c, (uint32_t)(l * A.plane), om);
    }
  }
}

template <typename R, int N>
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
  const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
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
  R m = R(0);  // incoming normal flux of the new deviations
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      const R cn = whi ? -L.x[b] : L.x[b];
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
      m = fmaR(-cn, out[l], m);
    }
  }
  // eq.(IMPOSITION) in deviations: d_l = kap_l + phi_l m for c.n > 0
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      const R cn = whi ? -L.x[b] : L.x[b];
      if (cn > R(0)) out[l] = whi ? fmaR(A.phi_hi[l], m, A.kap_hi[l]) : fmaR(A.phi_lo[l], m, A.kap_lo[l]);
      bst(dst, r0 + i, (uint32_t)(l * A.plane), out[l]);
    }
  }
}

// eq.(IMPOSITION) in place at both wall rows (state set from fields).
template <typename R, int N>
__global__ __launch_bounds__(256) void k_fv_impose(const FvArgs<R> A) {
  constexpr int Q = N * N;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int side = blockIdx.y;  // 0: first row, 1: last row
  if (i >= A.nx || !A.walls) return;
  const Lat<R>& L = A.lat;
  const bool whi = side == 1;
  const uint32_t bytes = (uint32_t)(Q * A.plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.dst, bytes);
  const uint32_t c = (uint32_t)((whi ? A.ny - 1 : 0) * A.ld + i);
  R m = R(0);
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const R cn = whi ? -L.x[l % N] : L.x[l % N];
    if (cn <= R(0)) m = fmaR(-cn, bld<R>(s, c, (uint32_t)(l * A.plane)), m);
  }
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    const R cn = whi ? -L.x[l % N] : L.x[l % N];
    if (cn > R(0))
      bst(s, c, (uint32_t)(l * A.plane),
          whi ? fmaR(A.phi_hi[l], m, A.kap_hi[l]) : fmaR(A.phi_lo[l], m, A.kap_lo[l]));
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

// ------------------------------------------------------------- dispatch ---
template <typename R, int N, int ORD, bool COMP>
static hipError_t fv_launch(int what, const FvArgs<R>& A, R* fields, double* partials,
                            hipStream_t st) {
  const dim3 g((unsigned)((A.nx + 63) / 64), (unsigned)((A.ny + 3) / 4)), b(256);
  switch (what) {
    case FV_OMEGA: hipLaunchKernelGGL((k_fv_omega<R, N, ORD, COMP>), g, b, 0, st, A); break;
    case FV_UPDATE: hipLaunchKernelGGL((k_fv_update<R, N>), g, b, 0, st, A); break;
    case FV_IMPOSE:
      hipLaunchKernelGGL((k_fv_impose<R, N>), dim3((unsigned)((A.nx + 255) / 256), 2), b, 0, st, A);
      break;
    case FV_POPS: hipLaunchKernelGGL((k_fv_pops<R, N>), g, b, 0, st, A, fields); break;
    default: hipLaunchKernelGGL((k_fv_fields<R, N, COMP>), g, b, 0, st, A, fields, partials); break;
  }
  return hipGetLastError();
}

template <typename R, bool COMP>
static hipError_t fv_lat(int n, int what, const FvArgs<R>& A, R* fields, double* partials,
                         hipStream_t st) {
  switch (n) {
    case 3: return fv_launch<R, 3, 2, COMP>(what, A, fields, partials, st);
    case 4: return fv_launch<R, 4, 3, COMP>(what, A, fields, partials, st);
    case 6: return fv_launch<R, 6, 4, COMP>(what, A, fields, partials, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fv(int n, bool comp, int what, const FvArgs<float>& A, float* fields,
                     double* partials, hipStream_t st) {
  return comp ? fv_lat<float, true>(n, what, A, fields, partials, st)
              : fv_lat<float, false>(n, what, A, fields, partials, st);
}
hipError_t launch_fv(int n, bool comp, int what, const FvArgs<double>& A, double* fields,
                     double* partials, hipStream_t st) {
  (void)comp;
  return fv_lat<double, false>(n, what, A, fields, partials, st);
}

}  // namespace tvlbm
