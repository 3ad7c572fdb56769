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

// Control block of a batched run (device arrays, n_inst entries each).
template <typename R>
struct BatchCtl {
  const Inst<R>* insts;
  const R* fields;     // packed fields of the last check step
  R* prev;             // packed snapshot of the previous check
  int32_t* active;
  int32_t* have_prev;
  int64_t* steps;
  double* resid;
  int32_t* flag;
  double* part;        // [n_inst][RESID_SLICES][2] partial sums
  int32_t K;
  double tol;
  int64_t max_steps;
};
// Workgroups per instance in the batched residual's first pass.
constexpr int RESID_SLICES = 16;

// Step mode on column pairs (FP32, grid periodic in y, even width and pitch):
// A describes the grid in pair units (nx, ld, plane halved).
hipError_t launch_march_pairs(int n, bool comp, const MarchArgs<f32x2>& A, int nblocks,
                              hipStream_t st);
// prefetch selects the software-pipelined row loads for the step modes.
hipError_t launch_march_batch(int n, bool comp, int mode, bool prefetch, const MarchArgs<float>& A,
                              int nblocks, hipStream_t st);
hipError_t launch_march_batch(int n, bool comp, int mode, bool prefetch, const MarchArgs<double>& A,
                              int nblocks, hipStream_t st);
hipError_t launch_batch_resid(const BatchCtl<float>& C, int n_inst, hipStream_t st);
hipError_t launch_batch_resid(const BatchCtl<double>& C, int n_inst, hipStream_t st);
hipError_t launch_batch_compact(const int32_t* active, const int32_t* item_start, const Work* all,
                                Work* work, int32_t* n_work, int32_t* remaining, int n_inst,
                                hipStream_t st);
hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<float>& A, int nblocks,
                        hipStream_t st);
// Two steps per launch (g^{k+2} from g^k): grid periodic in x and y, uniform
// rows; FP32 D2Q9, D2Q16 or D2Q36, FP64 D2Q9 or D2Q16.  A.tiles_x = strips of
// 62 columns, A.rows = output rows per wavefront segment, A.n_tiles =
// tiles_x * ceil(segments/4).
hipError_t launch_march2(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st);
hipError_t launch_march2(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st);
hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<double>& A, int nblocks,
                        hipStream_t st);
// Two steps per launch on a grid with diffuse walls in y (uniform rows): as
// launch_march2 with strips of 60 output columns (A.tiles_x = ceil(nx/60)).
hipError_t launch_march2w(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st);
hipError_t launch_march2w(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st);
// Batched walled channels, two steps per launch; work items of the
// two-step shape (lane-group width | rows << 8).
hipError_t launch_march2_batch(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st);
hipError_t launch_march2_batch(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st);
hipError_t launch_init(int n, bool comp, const InitArgs<float>& A, hipStream_t st);
hipError_t launch_init(int n, bool comp, const InitArgs<double>& A, hipStream_t st);
hipError_t launch_reduce(const double* part, int nblk, int width, double* out, hipStream_t st);
// g += delta_b w_l for every cell of instance b (n_inst instances: insts[b],
// or `single` when insts is null), delta_b = (ref[b] - cur[b]) 2^-32 / area[b];
// instances with active[b] == 0 are skipped (active may be null).
hipError_t launch_mass_fix(float* g, const Inst<float>* insts, const Inst<float>& single,
                           const int32_t* active, const unsigned long long* ref,
                           const unsigned long long* cur, const double* area, const Lat<float>& L,
                           int q, int n_inst, hipStream_t st);
hipError_t launch_mass_fix(double* g, const Inst<double>* insts, const Inst<double>& single,
                           const int32_t* active, const unsigned long long* ref,
                           const unsigned long long* cur, const double* area, const Lat<double>& L,
                           int q, int n_inst, hipStream_t st);
// dst = src, n16 elements of 16 bytes, grid-stride over nblocks workgroups.
hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, int nblocks, hipStream_t st);
// p[0..n) = v on the stream (n <= 64 is one wavefront's pass).
hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st);
hipError_t launch_resid(const float* q, const float* qp, int64_t n, double* part, int nblk,
                        hipStream_t st);
hipError_t launch_resid(const double* q, const double* qp, int64_t n, double* part, int nblk,
                        hipStream_t st);

}  // namespace tvlbm
