// tvlbm_fv_launch.h -- parameter block and launchers of the finite-volume
// TVLBM kernels (tvlbm_fv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "tvlbm_core.h"

namespace tvlbm {

template <typename R>
struct FvArgs {
  Lat<R> lat;           // nodes x_a, x_a^2, weights w_l (FP64 copies for totals)
  int32_t nx, ny;       // mesh points
  int32_t walls;        // 0 periodic in y, 1 wall points at j = 0 and ny-1
  int32_t x_open;       // 0 periodic in x, 1 zero-gradient x ends
  int32_t collide;      // 0: Omega = 0
  int64_t ld, plane;    // row pitch, ny * ld
  R dt, inv_tau;        // time step, 1/tau
  R inv_dx;             // 2 / (dx + dx)
  const R* cy;          // [ny] y-derivative factors: 2/(dy_{j-1} + dy_j), at walls 2/dy
  const double* vol;    // [ny] dx * dual-cell height (totals)
  R kap_lo[QMAX], phi_lo[QMAX];  // re-emission at the bottom wall: d = kap + phi m
  R kap_hi[QMAX], phi_hi[QMAX];  // and at the top wall
  const R* src;         // d at t
  R* dst;               // d at t + dt
  R* om;                // Omega at t (two-pass schedule)
  int32_t strips;       // fused march: 62-column strips, one wavefront wide
  int32_t segs;         // row segments of seg_rows rows
  int32_t seg_rows;
  int32_t prefetch;     // load row r+1 while row r is processed
  const double* wtab;   // FP64 kap_lo, phi_lo, kap_hi, phi_hi [4][QMAX] (device)
  R tau_ratio;          // tau / tau_g of the non-unit-Prandtl term, 0 = off
  int32_t pscale;       // 1: relaxation times divided by the local pressure
  int32_t slip_free;    // 1: wall equilibria by Newton iteration (App. B)
  int32_t nr_warm;      // 1: start from the stored roots of the last step
  double wall_u[2], wall_T[2];  // prescribed wall velocity / temperature (lo, hi)
  double* wpar;         // [2][nx][2] last (u_eq, T_eq) of every wall point
};

// FV_OMEGA + FV_UPDATE: the two-pass step; FV_MARCH: the fused one-pass step
// FV_BAND: the fused step with four wavefronts per row segment (FP32, q <= 16)
enum FvKernel { FV_OMEGA = 0, FV_UPDATE = 1, FV_FIELDS = 2, FV_IMPOSE = 3, FV_POPS = 4,
                FV_MARCH = 5, FV_BAND = 6 };

// FV_FIELDS: fields [4][ny][nx] or null, partials [blocks][4];
// FV_POPS: fields is the [q][ny][nx] output; FV_IMPOSE acts on A.dst.
// n: Gauss-Hermite points per axis, ord: equilibrium order.
hipError_t launch_fv(int n, int ord, bool comp, int what, const FvArgs<float>& A, float* fields,
                     double* partials, hipStream_t st);
hipError_t launch_fv(int n, int ord, bool comp, int what, const FvArgs<double>& A, double* fields,
                     double* partials, hipStream_t st);

// f = feq(rho, u, T) + noise into A.dst as deviations (device [ny][nx]
// fields, noise [q][ny][nx] or null).
template <typename R>
struct FvInit {
  const R *rho, *ux, *uy, *T, *noise;
};
hipError_t launch_fv_init(int n, int ord, const FvArgs<float>& A, const FvInit<float>& I,
                          hipStream_t st);
hipError_t launch_fv_init(int n, int ord, const FvArgs<double>& A, const FvInit<double>& I,
                          hipStream_t st);

}  // namespace tvlbm
