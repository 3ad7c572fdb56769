// tvlbm_launch.h -- host-callable launchers of the TVLBM kernels.
#pragma once

#include "tvlbm_core.h"

namespace tvlbm {

template <typename R>
struct InitArgs {
  Lat<R> lat;
  Inst<R> inst;
  const R* rho;    // [ny][nx] fields, or null when fabs is given
  const R* ux;
  const R* uy;
  const R* T;
  const R* noise;  // [q][ny][nx] or null
  const R* fabs;   // [q][ny][nx] absolute populations, or null
  R* f0;           // deviations f^0, pitch ld
  R* g0;           // deviations C(f^0), pitch ld
};

hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<float>& A, int nblocks,
                        hipStream_t st);
hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<double>& A, int nblocks,
                        hipStream_t st);
hipError_t launch_init(int n, bool comp, const InitArgs<float>& A, hipStream_t st);
hipError_t launch_init(int n, bool comp, const InitArgs<double>& A, hipStream_t st);
hipError_t launch_reduce(const double* part, int nblk, int width, double* out, hipStream_t st);
hipError_t launch_resid(const float* q, const float* qp, int64_t n, double* part, int nblk,
                        hipStream_t st);
hipError_t launch_resid(const double* q, const double* qp, int64_t n, double* part, int nblk,
                        hipStream_t st);

}  // namespace tvlbm
