// tvlbm_kernels.hip -- HIP kernels of the fused TVLBM step for gfx950.
//
// k_march: the fused step.  One lane owns one column of a strip and marches
// down a segment of rows.  Stored state is the post-collision deviation
// g^k; per row the lane
//   1. pulls f^{k+1} = S(g^k) with the exact-overlap weights: per axis the
//      shifted unit cell covers the same cell with weight 1-|s| and the
//      upstream neighbour with weight |s| (at most four cells in 2-D); the
//      x-pulled value of the previous row is kept in a register, so every
//      population costs two loads (centre and upstream column) per cell;
//   2. forms the moments (compensated sums in FP32), the Hermite equilibrium
//      and the BGK update in registers;
//   3. stores g^{k+1}, coalesced, structure-of-arrays.
// Diffuse walls (Sec. VII, eq.(IMPOSITION)) enter as ghost values at the
// first and last row: the mass carried through the wall by the incident
// populations of the wall row is re-emitted into the outgoing populations
// with the flux-weighted wall Maxwellian.
//
// Work distribution is XCD-aware: workgroups are dispatched round-robin over
// the 8 XCDs, so the tile index is remapped to give each XCD a contiguous
// band of tiles (neighbouring row segments share halo rows in that XCD's L2).
#include "tvlbm_core.h"
#include "tvlbm_launch.h"

namespace tvlbm {

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// sign of node a of an N-point symmetric rule: -1, 0 (odd N middle), +1
template <int N>
__host__ __device__ constexpr int node_sign(int a) {
  return (2 * a + 1 < N) ? -1 : ((2 * a + 1 > N) ? 1 : 0);
}

// Lane offsets of one row: centre, left and right neighbour (periodic in x).
struct RowOff {
  uint32_t c, m, p;
};
__device__ __forceinline__ RowOff row_off(uint32_t rowbase, int ic, int im, int ip) {
  return RowOff{rowbase + (uint32_t)ic, rowbase + (uint32_t)im, rowbase + (uint32_t)ip};
}

// x part of the overlap remap for node a: value landing in the centre
// column from the centre (weight 1-p) and the upstream column (weight p).
template <typename R, int N>
__device__ __forceinline__ R xpull(const Lat<R>& L, rsrc_t s, uint32_t lo, int a, const RowOff& o) {
  const int sg = node_sign<N>(a);
  R vc = bld<R>(s, o.c, lo);
  if constexpr (is_pair_v<R>) {
    // lane holds columns (2k, 2k+1); the upstream neighbours are (2k-1, 2k)
    // or (2k+1, 2k+2): one half from the adjacent pair, one from this one
    if (sg > 0) {
      const R m = bld<R>(s, o.m, lo);
      return fmaR(L.qm[a], vc, L.p[a] * R{m.y, vc.x});
    }
    if (sg < 0) {
      const R q = bld<R>(s, o.p, lo);
      return fmaR(L.qm[a], vc, L.p[a] * R{vc.y, q.x});
    }
    return vc;
  } else {
    if (sg > 0) return fmaR(L.qm[a], vc, L.p[a] * bld<R>(s, o.m, lo));
    if (sg < 0) return fmaR(L.qm[a], vc, L.p[a] * bld<R>(s, o.p, lo));
    return vc;
  }
}

// Deviation part of the mass (per unit column width) that the populations
// moving in direction dir (-1 down, +1 up) carry out of one row through the
// wall, landing in column c:  m(c) = sum_{b: sign(x_b)=dir} p_b sum_a X_a(d_ab)(c).
// The rest-state part sum p_b w_b is folded into the host constants kap_*.
template <typename R, int N>
__device__ __forceinline__ R wall_mass(const Lat<R>& L, rsrc_t s, int64_t plane,
                                       uint32_t rowbase, int c, int nx, int dir) {
  const RowOff o = row_off(rowbase, c, wrapc(c - 1, nx), wrapc(c + 1, nx));
  R m = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    if (node_sign<N>(b) != dir) continue;
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) acc += xpull<R, N>(L, s, (uint32_t)((a * N + b) * plane), a, o);
    m = fmaR(L.p[b], acc, m);
  }
  return m;
}

// x-pull of a ghost row whose value at column c is kap + phi * m(c)
template <typename R, int N>
__device__ __forceinline__ R ghost_pull(const Lat<R>& L, int a, R kap, R phi, R m_c, R m_m, R m_p) {
  const int sg = node_sign<N>(a);
  R mx = m_c;
  if (sg > 0) mx = fmaR(L.qm[a], m_c, L.p[a] * m_m);
  if (sg < 0) mx = fmaR(L.qm[a], m_c, L.p[a] * m_p);
  return fmaR(phi, mx, kap);
}

// Moments, equilibrium, collision and outputs of one cell whose pulled
// (post-stream, pre-collision) deviations are d[].  dyj: row height (for the
// area-weighted totals).
template <typename R, int N, int ORD, bool COMP, int MODE>
__device__ __forceinline__ void cell_tail(const MarchArgs<R>& A, const Inst<R>& P, rsrc_t dst,
                                          const R (&d)[N * N], int j, int i, bool active,
                                          double dyj, double (&tot)[5], int& bad) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const int nx = P.nx, ny = P.ny;
  R drho, jx, jy, ed;
  cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
  const Fields<R> F = fields_from(drho, jx, jy, ed);

  if constexpr (MODE != MODE_STEP) {
    const bool want_fields = (MODE == MODE_CHECK) || (A.aux & AUX_FIELDS);
    if (want_fields && active) {
      const R T = R(1) + F.th;
      if (!(F.rho > R(0)) || !(T > R(0)) || !__builtin_isfinite(F.ux + F.uy + F.rho + T)) bad = 1;
      if (A.fields) {
        R* fo = A.fields + P.fld + (int64_t)j * nx + i;
        const int64_t fp = (int64_t)nx * ny;
        fo[0] = F.rho;
        fo[fp] = F.ux;
        fo[2 * fp] = F.uy;
        fo[3 * fp] = T;
      }
      double m = 0.0, px = 0.0, py = 0.0, e = 0.0, dm = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          const double fa = L.wd[l] + (double)d[l];
          m += fa;
          dm += (double)d[l];
          px += L.xd[a] * fa;
          py += L.xd[b] * fa;
          e += 0.5 * (L.xd[a] * L.xd[a] + L.xd[b] * L.xd[b]) * fa;
        }
      }
      tot[0] += dyj * m; tot[1] += dyj * px; tot[2] += dyj * py; tot[3] += dyj * e;
      // the cell's deviation mass in fixed point (an integer, held exactly
      // in the double while |sum| < 2^53), for order-independent totals
      tot[4] += (double)__double2ll_rn(dyj * dm * MASS_FP_SCALE);
    }
  }

  if constexpr (MODE == MODE_AUX) {
    if (A.aux & AUX_POPS) {
      if (active) {
        const int64_t op = (int64_t)nx * ny;
#pragma unroll
        for (int l = 0; l < Q; ++l) A.dst[l * op + (int64_t)j * nx + i] = d[l] + L.w[l];
      }
      return;
    }
    if (!(A.aux & AUX_POST)) return;
  }

  R g[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) g[l] = d[l];
  bgk_cell<R, N, ORD>(L, P, F, g);
  if (active) {
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      if constexpr (MODE == MODE_AUX) {
        const int64_t op = (int64_t)nx * ny;
        A.dst[l * op + (int64_t)j * nx + i] = g[l] + L.w[l];
      } else {
        bst(dst, (uint32_t)j * (uint32_t)P.ld + (uint32_t)i, (uint32_t)(l * P.plane), g[l]);
      }
    }
  }
}

// Ghost value of an emitting population at the wall it leaves: sg > 0
// (moving up) is emitted by the bottom wall, sg < 0 by the top wall.
template <typename R, int N>
__device__ __forceinline__ R ghost_of(const Lat<R>& L, const Inst<R>& P, int a, int b, R m_c, R m_m,
                                      R m_p) {
  const int l = a * N + b;
  return node_sign<N>(b) > 0 ? ghost_pull<R, N>(L, a, P.kap_lo[l], P.phi_lo[l], m_c, m_m, m_p)
                             : ghost_pull<R, N>(L, a, P.kap_hi[l], P.phi_hi[l], m_c, m_m, m_p);
}

// Everything one lane does for one row j: pull, moments, equilibrium,
// collision, store (or the auxiliary outputs).  The lane marches in
// direction DIR (+1: increasing j, -1: decreasing j).  A population whose
// upstream row is the row visited before ("lead": sign(x_b) == DIR) pulls
// rows j (1-p) and j-DIR (p), the latter kept in hp from the previous row;
// the others ("trail") pull rows j and j+DIR, loading j+DIR now and keeping
// it for the next row.  GHOST: row j+DIR lies beyond a wall; the trail
// populations pull that wall's ghost (m_* is its incident mass).
template <typename R, int N, int ORD, bool COMP, int MODE, int DIR, bool GHOST>
__device__ __forceinline__ void march_row(const MarchArgs<R>& A, const Inst<R>& P,
                                          rsrc_t s, rsrc_t dst, R (&hp)[N * N], int j,
                                          int i, int ic, int im, int ip, bool active,
                                          bool ident, double (&tot)[5], int& bad) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const int nx = P.nx, ny = P.ny;
  const int64_t plane = P.plane;
  const uint32_t ld = (uint32_t)P.ld;
  const uint32_t rj = (uint32_t)j * ld;
  R d[Q];
  if (ident) {
#pragma unroll
    for (int l = 0; l < Q; ++l) d[l] = bld<R>(s, rj + (uint32_t)ic, (uint32_t)(l * plane));
  } else {
    const RowOff oj = row_off(rj, ic, im, ip);
    int jn = j + DIR;
    jn = jn < 0 ? ny - 1 : (jn >= ny ? 0 : jn);  // periodic; walls use GHOST
    const RowOff on = row_off((uint32_t)jn * ld, ic, im, ip);
    R m_c = R(0), m_m = R(0), m_p = R(0);
    if constexpr (GHOST) {
      // incident mass through the wall next to row j (top for DIR > 0)
      m_c = wall_mass<R, N>(L, s, plane, rj, ic, nx, DIR);
      m_m = wall_mass<R, N>(L, s, plane, rj, im, nx, DIR);
      m_p = wall_mass<R, N>(L, s, plane, rj, ip, nx, DIR);
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const int sg = node_sign<N>(b);
        const uint32_t pl = (uint32_t)(l * plane);
        if (sg == DIR) {  // lead
          R hn = xpull<R, N>(L, s, pl, a, oj);
          d[l] = fmaR(L.qm[b], hn, L.p[b] * hp[l]);
          hp[l] = hn;
        } else if (sg == -DIR) {  // trail
          R hn;
          if constexpr (GHOST)
            hn = ghost_of<R, N>(L, P, a, b, m_c, m_m, m_p);
          else
            hn = xpull<R, N>(L, s, pl, a, on);
          d[l] = fmaR(L.qm[b], hp[l], L.p[b] * hn);
          hp[l] = hn;
        } else {
          d[l] = xpull<R, N>(L, s, pl, a, oj);
        }
      }
    }
  }

  cell_tail<R, N, ORD, COMP, MODE>(A, P, dst, d, j, i, active, 1.0, tot, bad);
}

// Software-pipelined rows: the raw loads of the next row (centre and
// upstream column of every population) are issued before the current row
// is computed, so a wavefront always has a row of loads in flight.
template <typename R, int N, int DIR>
__device__ __forceinline__ void fetch_row(rsrc_t s, int64_t plane, uint32_t ld, int ny, int j, int ic,
                                          int im, int ip, R (&c)[N * N], R (&nb)[N * N]) {
  int jn = j + DIR;
  jn = jn < 0 ? ny - 1 : (jn >= ny ? 0 : jn);
  const uint32_t rj = (uint32_t)j * ld, rn = (uint32_t)jn * ld;
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      const uint32_t row = (node_sign<N>(b) == -DIR) ? rn : rj;
      const uint32_t pl = (uint32_t)(l * plane);
      c[l] = bld<R>(s, row + (uint32_t)ic, pl);
      const int sa = node_sign<N>(a);
      nb[l] = sa > 0 ? bld<R>(s, row + (uint32_t)im, pl) : (sa < 0 ? bld<R>(s, row + (uint32_t)ip, pl) : R(0));
    }
  }
}

template <typename R, int N, int DIR>
__device__ __forceinline__ void pull_row(const Lat<R>& L, const R (&c)[N * N], const R (&nb)[N * N],
                                         R (&hp)[N * N], R (&d)[N * N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const int l = a * N + b;
      const R h = node_sign<N>(a) != 0 ? fmaR(L.qm[a], c[l], L.p[a] * nb[l]) : c[l];
      const int sg = node_sign<N>(b);
      if (sg == DIR) {
        d[l] = fmaR(L.qm[b], h, L.p[b] * hp[l]);
        hp[l] = h;
      } else if (sg == -DIR) {
        d[l] = fmaR(L.qm[b], hp[l], L.p[b] * h);
        hp[l] = h;
      } else {
        d[l] = h;
      }
    }
  }
}

// One lane's segment of rows [j0, j1), marched in direction DIR.
template <typename R, int N, int ORD, bool COMP, int MODE, int DIR, bool PF>
__device__ __forceinline__ void march_dir(const MarchArgs<R>& A, const Inst<R>& P, int i,
                                          bool active, int j0, int j1, double (&tot)[5],
                                          int& bad) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const int nx = P.nx, ny = P.ny;
  const int64_t plane = P.plane;
  const uint32_t ld = (uint32_t)P.ld;
  const uint32_t bytes = (uint32_t)(Q * plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src + P.off, bytes);
  const rsrc_t dst = make_rsrc(A.dst + P.off, bytes);
  const int ic = active ? i : 0;  // inactive lanes read a valid column, store nothing
  const int im = ic == 0 ? nx - 1 : ic - 1;
  const int ip = ic == nx - 1 ? 0 : ic + 1;
  const bool ident = (MODE == MODE_AUX) && (A.aux & AUX_IDENTITY);
  const int jf = DIR > 0 ? j0 : j1 - 1;         // first row visited
  const int jl = DIR > 0 ? j1 - 1 : j0;         // last row visited
  // a wall lies before the first row / after the last row
  // (column pairs run only on grids periodic in y)
  const bool wall_first = !is_pair_v<R> && P.walls && (DIR > 0 ? j0 == 0 : j1 == ny);
  const bool wall_last = !is_pair_v<R> && P.walls && (DIR > 0 ? j1 == ny : j0 == 0);

  R hp[Q];
  if (!ident) {
    // lead populations need the row before jf (or that wall's ghost);
    // trail populations start from row jf itself.
    R m_c = R(0), m_m = R(0), m_p = R(0);
    const uint32_t rw = (uint32_t)(DIR > 0 ? 0 : ny - 1) * ld;  // wall row
    if (wall_first) {
      m_c = wall_mass<R, N>(L, s, plane, rw, ic, nx, -DIR);
      m_m = wall_mass<R, N>(L, s, plane, rw, im, nx, -DIR);
      m_p = wall_mass<R, N>(L, s, plane, rw, ip, nx, -DIR);
    }
    int jb = jf - DIR;
    jb = jb < 0 ? ny - 1 : (jb >= ny ? 0 : jb);
    const RowOff ob = row_off((uint32_t)jb * ld, ic, im, ip);
    const RowOff of = row_off((uint32_t)jf * ld, ic, im, ip);
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const int sg = node_sign<N>(b);
        if (sg == DIR) {
          hp[l] = wall_first ? ghost_of<R, N>(L, P, a, b, m_c, m_m, m_p)
                             : xpull<R, N>(L, s, (uint32_t)(l * plane), a, ob);
        } else if (sg == -DIR) {
          hp[l] = xpull<R, N>(L, s, (uint32_t)(l * plane), a, of);
        } else {
          hp[l] = R(0);
        }
      }
    }
  }

  const int nrow = j1 - j0;
  const int nmain = (wall_last && !ident) ? nrow - 1 : nrow;
  int j = jf;
  if constexpr (PF && MODE == MODE_STEP) {
    R cc[Q], cn[Q];
    if (nmain > 0) fetch_row<R, N, DIR>(s, plane, ld, ny, j, ic, im, ip, cc, cn);
    for (int r = 0; r < nmain; ++r, j += DIR) {
      R nc[Q], nn[Q];
      if (r + 1 < nmain) fetch_row<R, N, DIR>(s, plane, ld, ny, j + DIR, ic, im, ip, nc, nn);
      R d[Q];
      pull_row<R, N, DIR>(L, cc, cn, hp, d);
      cell_tail<R, N, ORD, COMP, MODE>(A, P, dst, d, j, i, active, 1.0, tot, bad);
#pragma unroll
      for (int l = 0; l < Q; ++l) { cc[l] = nc[l]; cn[l] = nn[l]; }
    }
  } else {
    for (int r = 0; r < nmain; ++r, j += DIR)
      march_row<R, N, ORD, COMP, MODE, DIR, false>(A, P, s, dst, hp, j, i, ic, im, ip, active, ident,
                                                   tot, bad);
  }
  if (nmain < nrow)
    march_row<R, N, ORD, COMP, MODE, DIR, true>(A, P, s, dst, hp, jl, i, ic, im, ip, active, ident,
                                                tot, bad);
}

// Segments alternate direction (group parity), so two neighbouring segments
// touch their shared halo rows at the same time -- both at their start or
// both at their end -- and the second read hits in L2.
template <typename R, int N, int ORD, bool COMP, int MODE, bool PF>
__device__ __forceinline__ void march_lane(const MarchArgs<R>& A, const Inst<R>& P, int i,
                                           bool active, int j0, int j1, int group, double (&tot)[5],
                                           int& bad) {
  if (group & 1)
    march_dir<R, N, ORD, COMP, MODE, -1, PF>(A, P, i, active, j0, j1, tot, bad);
  else
    march_dir<R, N, ORD, COMP, MODE, +1, PF>(A, P, i, active, j0, j1, tot, bad);
}

// Wave sum of the fixed-point mass tally tot[4], added to *slot by lane 0
// (integer addition: exact and independent of the order of the waves).
__device__ __forceinline__ void wave_mass(double t4, unsigned long long* slot) {
  long long v = (long long)t4;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(slot, (unsigned long long)v);
}

template <int MODE>
__device__ __forceinline__ void block_totals(const double (&tot)[5], int bad, double* partials,
                                             int32_t* flag) {
  __shared__ double sh[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[4] = {tot[0], tot[1], tot[2], tot[3]};
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] += __shfl_xor(v[c], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[wave][c] = v[c];
  }
  if (bad) flag[0] = 1;
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    partials[(int64_t)blockIdx.x * 4 + c] = ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
  }
}

template <typename R, int N, int ORD, bool COMP, int MODE, bool PF>
__global__ __launch_bounds__(256) void k_march(const MarchArgs<R> A) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = A.width;
  const int spw = 64 / W;       // lane segments per wavefront
  const int spb = 4 * spw;      // segments per workgroup
  const int nb = gridDim.x;     // multiple of 8
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  if (t < A.n_tiles) {
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int i = tx * W + (lane & (W - 1));
    const int group = ty * 4 + wave;  // wave-uniform segment group
    const int seg = group * spw + lane / W;
    const int j0 = seg * A.rows;
    const int j1 = min(j0 + A.rows, A.inst.ny);
    if (j0 < A.inst.ny)
      march_lane<R, N, ORD, COMP, MODE, PF>(A, A.inst, i, i < A.inst.nx, j0, j1, group, tot, bad);
  }
  if constexpr (MODE != MODE_STEP) {
    if (MODE == MODE_CHECK || (A.aux & AUX_FIELDS)) {
      block_totals<MODE>(tot, bad, A.partials, A.flag);
      if (A.mass) wave_mass(tot[4], A.mass);
    }
  }
}


// ----------------------------------------------- two steps per sweep --
// k_march2: g^{k+2} from g^k in one pass over the grid (periodic in x and y,
// uniform rows), without storing g^{k+1}: each population is read and
// written once per two steps.  A wavefront owns a strip of 62 output columns
// with one halo lane on each side, and a segment of output rows [j0, j1).
// Along the segment it forms g^{k+1} on rows j0-1 .. j1 as the one-step
// march does (centre and upstream column loaded, the x-pulled value of the
// previous row kept per population), and one row behind it g^{k+2}: the x
// part of the second remap takes the upstream column's g^{k+1} from the
// neighbouring lane (a DPP shift by one lane), the y part keeps the x-pulled
// values of the previous two rows in registers.  Every output cell sees the
// same operations, in the same order, as under two one-step launches.
constexpr int STRIP2 = 62;          // output columns per wavefront
constexpr int DPP_PREV = 0x138;     // wave_shr:1 -- lane l reads lane l-1
constexpr int DPP_NEXT = 0x130;     // wave_shl:1 -- lane l reads lane l+1

template <int CTRL>
__device__ __forceinline__ float lane_from(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_from(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// moments, Hermite equilibrium and BGK of one cell, result in registers
template <typename R, int N, int ORD, bool COMP>
__device__ __forceinline__ Fields<R> collide_regs(const Lat<R>& L, const Inst<R>& P,
                                                  const R (&d)[N * N], R (&g)[N * N]) {
  R drho, jx, jy, ed;
  cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
  const Fields<R> F = fields_from(drho, jx, jy, ed);
#pragma unroll
  for (int l = 0; l < N * N; ++l) g[l] = d[l];
  bgk_cell<R, N, ORD>(L, P, F, g);
  return F;
}

__device__ __forceinline__ int wrap_row(int j, int ny) {
  j %= ny;
  return j < 0 ? j + ny : j;
}

// Rows handed between the wavefronts of a workgroup (k_march2): the
// x-pulled g^{k+1} of a first-step row, for the N * (N / 2) populations of
// one y-sign, one value per lane.  Slot [0][w] holds what wave w hands over
// at the start of its sweep, [1][w] at the end.
template <typename R, int N>
struct XchRows {
  static constexpr int NL = N * (N / 2);
  R v[2][4][NL][64];
};

// index of population (a, b), sign(x_b) = sg != 0, among those of its sign
template <int N>
__host__ __device__ constexpr int sign_index(int a, int b) {
  return a * (N / 2) + (node_sign<N>(b) > 0 ? b - (N - N / 2) : b);
}

// One wave's segment [j0, j1) of the two-step march, direction DIR.
// Exchanges with the neighbouring segments of the workgroup (same strip):
//  * start (xs >= 0): the row behind the first output row is the first
//    output row of segment xs, which marches the other way from the same
//    boundary; each computes only its own and hands the other the x-pulled
//    values of the populations that other treats as lead (its y2);
//  * end (xe >= 0): the row past the last output row is the last output row
//    of segment xe, which arrives there at the same time from the other
//    side; each hands the other the values of the populations that other
//    treats as trail (its x in the last second step).
// Both hand-overs happen at fixed iterations (t = 1 and t = rows, barriers
// for the whole workgroup), so every wave runs the same trip count; a wave
// without a segment (live = false) takes part in the barriers only.  The
// values are those the partner would compute itself (the first step of a
// row does not depend on the direction of the march), so the results are
// unchanged; each exchange saves one first-step row.
template <typename R, int N, int ORD, bool COMP, int DIR>
__device__ __forceinline__ void march2_dir(const MarchArgs<R>& A, int ic, int im, int ip,
                                           bool active, bool live, int j0, int j1, int wave,
                                           int xs, int xe, XchRows<R, N>& X, int lane) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const Inst<R>& P = A.inst;
  const int ny = P.ny;
  const int64_t plane = P.plane;
  const uint32_t ld = (uint32_t)P.ld;
  const uint32_t bytes = (uint32_t)(Q * plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src + P.off, bytes);
  const rsrc_t dst = make_rsrc(A.dst + P.off, bytes);
  const int nout = j1 - j0;
  const int jf = DIR > 0 ? j0 : j1 - 1;  // first output row
  const int t0 = xs >= 0 ? 1 : 0;        // first first-step iteration
  const int nt = A.rows + 2;             // same for every wave of the workgroup

  // first-step rows r_t = jf + (t - 1) DIR; before r_{t0}, lead populations
  // need X^k of the row behind it, trail ones of r_{t0} itself
  R hp[Q], hq[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) hp[l] = hq[l] = R(0);
  if (live) {
    const int r0 = wrap_row(jf + (t0 - 1) * DIR, ny);
    const RowOff ob = row_off((uint32_t)wrap_row(r0 - DIR, ny) * ld, ic, im, ip);
    const RowOff of = row_off((uint32_t)r0 * ld, ic, im, ip);
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const int sg = node_sign<N>(b);
        if (sg == DIR)
          hp[l] = xpull<R, N>(L, s, (uint32_t)(l * plane), a, ob);
        else if (sg == -DIR)
          hp[l] = xpull<R, N>(L, s, (uint32_t)(l * plane), a, of);
        else
          hp[l] = R(0);
      }
    }
  }

  // One iteration t: first step on row r_t into x (xc, which on entry
  // still holds x of t - 2, the y2 of the second step), then the second
  // step on output row r_t - DIR from y1 = xp (x of t - 1), y2 and x.  The
  // sweep runs two iterations per trip with the buffers swapped, so rows
  // change roles without register moves; the lead part of the second step
  // (which needs y2) is formed before x overwrites it.  hi / ho: X^k of the
  // row behind, carried in, and carried out.
  auto iter = [&](const int t, R (&hi)[Q], R (&ho)[Q], R (&xp)[Q], R (&xc)[Q]) {
    const int r = wrap_row(jf + (t - 1) * DIR, ny);
    const bool second = live && t >= 2 && t <= nout + 1;
    R el[Q];  // lead part of the second step
    if (second) {
#pragma unroll
      for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          if (node_sign<N>(b) == DIR) el[l] = fmaR(L.qm[b], xp[l], L.p[b] * xc[l]);
        }
    }
    if (live && t >= t0 && t <= nout + 1 && !(xe >= 0 && t == nout + 1)) {
      const RowOff oj = row_off((uint32_t)r * ld, ic, im, ip);
      const RowOff on = row_off((uint32_t)wrap_row(r + DIR, ny) * ld, ic, im, ip);
      R d[Q];
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          const int sg = node_sign<N>(b);
          const uint32_t pl = (uint32_t)(l * plane);
          if (sg == DIR) {  // lead
            ho[l] = xpull<R, N>(L, s, pl, a, oj);
            d[l] = fmaR(L.qm[b], ho[l], L.p[b] * hi[l]);
          } else if (sg == -DIR) {  // trail
            ho[l] = xpull<R, N>(L, s, pl, a, on);
            d[l] = fmaR(L.qm[b], hi[l], L.p[b] * ho[l]);
          } else {
            d[l] = xpull<R, N>(L, s, pl, a, oj);
          }
        }
      }
      R g[Q];
      collide_regs<R, N, ORD, COMP>(L, P, d, g);
      // x part of the second remap, upstream column from the neighbouring lane
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const int sa = node_sign<N>(a);
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          if (sa > 0)
            xc[l] = fmaR(L.qm[a], g[l], L.p[a] * lane_from<DPP_PREV>(g[l]));
          else if (sa < 0)
            xc[l] = fmaR(L.qm[a], g[l], L.p[a] * lane_from<DPP_NEXT>(g[l]));
          else
            xc[l] = g[l];
        }
      }
    } else {
      // no first step (t = 0 before a start hand-over, the row taken from
      // the end partner, rows past the segment, no segment): the carried
      // row passes on; of x only the parts the hand-overs write are used
#pragma unroll
      for (int l = 0; l < Q; ++l) {
        ho[l] = hi[l];
        xc[l] = R(0);
      }
    }
    if (t == 1) {  // start hand-over: my first output row, the partner's lead
      if (xs >= 0) {
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b)
            if (node_sign<N>(b) == -DIR) X.v[0][wave][sign_index<N>(a, b)][lane] = xc[a * N + b];
      }
      __syncthreads();
      if (xs >= 0) {  // the row behind my first output row, as if from t = 0
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b)
            if (node_sign<N>(b) == DIR) xp[a * N + b] = X.v[0][xs][sign_index<N>(a, b)][lane];
      }
    }
    if (t == A.rows) {  // end hand-over: my last output row, the partner's trail
      if (xe >= 0) {
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b)
            if (node_sign<N>(b) == DIR) X.v[1][wave][sign_index<N>(a, b)][lane] = xc[a * N + b];
      }
      __syncthreads();
    }
    if (xe >= 0 && t == nout + 1) {  // the row past my last output row
#pragma unroll
      for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == -DIR) xc[a * N + b] = X.v[1][xe][sign_index<N>(a, b)][lane];
    }
    if (second) {  // second step on output row m = r - DIR
      const uint32_t om = (uint32_t)wrap_row(r - DIR, ny) * ld + (uint32_t)ic;
      R e[Q];
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          const int sg = node_sign<N>(b);
          if (sg == DIR)
            e[l] = el[l];
          else if (sg == -DIR)
            e[l] = fmaR(L.qm[b], xp[l], L.p[b] * xc[l]);
          else
            e[l] = xp[l];
        }
      }
      R g2[Q];
      collide_regs<R, N, ORD, COMP>(L, P, e, g2);
      if (active) {
#pragma unroll
        for (int l = 0; l < Q; ++l) bst(dst, om, (uint32_t)(l * plane), g2[l]);
      }
    }
  };

  // Pairs of iterations; a last iteration past nt does nothing (the
  // barriers sit at t = 1 and t = rows, below nt).
  R xa[Q], xb[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) xa[l] = xb[l] = R(0);
  for (int t = 0; t < nt; t += 2) {
    iter(t, hp, hq, xb, xa);
    iter(t + 1, hq, hp, xa, xb);
  }
}

// One workgroup = 4 wavefronts = 4 consecutive row segments of one strip,
// marching in alternating directions (even segments up), so that waves 1
// and 2 start from a common boundary and waves 0, 1 and 2, 3 end at one;
// those hand the boundary rows over (march2_dir) when both segments are
// whole.  At least two wavefronts per SIMD: the D2Q36 form would otherwise
// take a few registers past half the file and run one wavefront per SIMD,
// with no other to hide its load latency; the few values spilled under the
// bound cost less than that (the smaller lattices fit anyway).
template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_march2(const MarchArgs<R> A) {
  __shared__ XchRows<R, N> X;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;  // multiple of 8
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  if (t >= A.n_tiles) return;  // whole workgroup
  const int nx = A.inst.nx, ny = A.inst.ny, rows = A.rows;
  const int tx = t % A.tiles_x, ty = t / A.tiles_x;
  const int g0 = ty * 4;  // first segment of the workgroup
  const int group = g0 + wave;
  const int j0 = group * rows;
  const bool live = j0 < ny;  // wave-uniform; a wave without rows still meets the barriers
  const int j1 = min(j0 + rows, ny);
  // segment w of this workgroup is whole (rows rows, all inside the grid)
  auto whole = [&](int w) { return (g0 + w + 1) * rows <= ny; };
  int xs = -1, xe = -1;
  if (wave == 1 && whole(1) && (g0 + 2) * rows < ny) xs = 2;
  if (wave == 2 && whole(1) && (g0 + 2) * rows < ny) xs = 1;
  if ((wave == 0 || wave == 1) && whole(0) && whole(1)) xe = wave ^ 1;
  if ((wave == 2 || wave == 3) && whole(2) && whole(3)) xe = wave ^ 1;
  const int col = tx * STRIP2 - 1 + lane;  // lanes 0 and 63 are halo
  const bool active = live && lane >= 1 && lane <= STRIP2 && col < nx;
  int ic = col % nx;
  ic = ic < 0 ? ic + nx : ic;
  const int im = ic == 0 ? nx - 1 : ic - 1;
  const int ip = ic == nx - 1 ? 0 : ic + 1;
  if (group & 1)
    march2_dir<R, N, ORD, COMP, -1>(A, ic, im, ip, active, live, j0, j1, wave, xs, xe, X, lane);
  else
    march2_dir<R, N, ORD, COMP, +1>(A, ic, im, ip, active, live, j0, j1, wave, xs, xe, X, lane);
}

// ------------------------------------------- two steps per sweep, walls --
// Two-step march on grids with diffuse walls in y (uniform rows), for the
// walled single grid and the batched channels.  As k_march2, but:
//  * the first step on a wall row pulls the populations coming from beyond
//    the wall from that wall's ghost of g^k (the re-emitted incident mass,
//    eq.(IMPOSITION)), exactly as the one-step march does;
//  * when an output row is a wall row whose upstream row lies beyond the
//    wall, the second step takes the x-pulled ghost of g^{k+1} instead: the
//    incident mass of the wall row's g^{k+1} per column (x-pulled values of
//    this lane) and, for the ghost's own x-pull, of the neighbouring columns
//    (DPP lane shifts).  The ghost's x-reach is two columns (incident x-pull,
//    then emitted x-pull), so a strip carries two halo lanes on each side.
// Every output cell sees the operations of two one-step launches in the
// same order, so the result is bitwise that of the one-step march.
//
// A wavefront may hold several lane groups (row segments) whose wall rows
// differ, so no branch depends on the lane: every group runs the same
// first-step rows relative to its segment, rows beyond a wall or past the
// segment included (their loads are clamped into the grid and their values
// never reach a stored output), the ghosts are formed when any lane needs
// them and taken per lane by selects, and only the stores are masked.  The
// loads stay unconditional, so the compiler can issue them back to back.
//
// Per lane: segment [j0, j1) (live = the segment exists), its column
// ic (im, ip: periodic neighbours), active = stores.  nt = uniform trip count
// (rows per segment + 2).
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

template <typename R, int N, int ORD, bool COMP, int DIR>
__device__ __forceinline__ void march2_wall_seg(const MarchArgs<R>& A, const Inst<R>& P, int ic,
                                                int im, int ip, bool active, bool live, int j0,
                                                int j1, int nt) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const int ny = P.ny, nx = P.nx;
  const int64_t plane = P.plane;
  const uint32_t ld = (uint32_t)P.ld;
  const uint32_t bytes = (uint32_t)(Q * plane * (int64_t)sizeof(R));
  const rsrc_t s = make_rsrc(A.src + P.off, bytes);
  const rsrc_t dst = make_rsrc(A.dst + P.off, bytes);
  const int nout = j1 - j0;
  const int jf = DIR > 0 ? j0 : j1 - 1;  // first output row
  const int jl = DIR > 0 ? j1 - 1 : j0;  // last output row
  const int wb = DIR > 0 ? 0 : ny - 1;   // wall row behind the march / ahead of it
  const int wa = DIR > 0 ? ny - 1 : 0;
  const int rb = wb - DIR, ra = wa + DIR;  // first rows beyond those walls
  // output row at either end whose upstream row lies beyond a wall
  const bool gh_first = live && jf == wb;
  const bool gh_last = live && jl == wa;
  auto row_at = [&](int r) {  // load offsets of row r, clamped into the grid
    const int rc = r < 0 ? 0 : (r > ny - 1 ? ny - 1 : r);
    return row_off((uint32_t)rc * ld, ic, im, ip);
  };

  // before the first row r_0 = jf - DIR: lead populations need X^k of the
  // row behind r_0 (a wall's ghost when that row lies beyond the wall),
  // trail ones of r_0 itself
  R hp[Q];
  {
    const bool gb = live && jf - 2 * DIR == rb;
    const RowOff ob = row_at(jf - 2 * DIR);
    const RowOff of = row_at(jf - DIR);
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const int sg = node_sign<N>(b);
        hp[l] = sg == 0 ? R(0) : xpull<R, N>(L, s, (uint32_t)(l * plane), a, sg == DIR ? ob : of);
      }
    }
    if (wave_any(gb)) {
      // (loaded, not taken from the neighbouring lanes: with the ghost of
      // g^(k+1) that also takes its neighbours' masses, the reach would
      // exceed the two halo lanes)
      const uint32_t rw = (uint32_t)wb * ld;
      const R m_c = wall_mass<R, N>(L, s, plane, rw, ic, nx, -DIR);
      const R m_m = wall_mass<R, N>(L, s, plane, rw, im, nx, -DIR);
      const R m_p = wall_mass<R, N>(L, s, plane, rw, ip, nx, -DIR);
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == DIR)
            hp[a * N + b] = gb ? ghost_of<R, N>(L, P, a, b, m_c, m_m, m_p) : hp[a * N + b];
      }
    }
  }

  R y1[Q], y2[Q];
#pragma unroll
  for (int l = 0; l < Q; ++l) y1[l] = y2[l] = R(0);
  for (int t = 0; t < nt; ++t) {
    const int r = jf + (t - 1) * DIR;
    // first step on row r: lead populations pull rows r and r - DIR, trail
    // ones rows r and r + DIR; a row beyond a wall is that wall's ghost
    const bool glead = r == rb;         // row r lies beyond the wall behind
    const bool gtrail = r + DIR == ra;  // row r + DIR lies beyond the wall ahead
    const RowOff oj = row_at(r);
    const RowOff on = row_at(r + DIR);
    R hn[Q];
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        hn[l] = xpull<R, N>(L, s, (uint32_t)(l * plane), a, node_sign<N>(b) == -DIR ? on : oj);
      }
    }
    if (wave_any(live && glead)) {
      // (loaded, not taken from the neighbouring lanes: with the ghost of
      // g^(k+1) that also takes its neighbours' masses, the reach would
      // exceed the two halo lanes)
      const uint32_t rw = (uint32_t)wb * ld;
      const R m_c = wall_mass<R, N>(L, s, plane, rw, ic, nx, -DIR);
      const R m_m = wall_mass<R, N>(L, s, plane, rw, im, nx, -DIR);
      const R m_p = wall_mass<R, N>(L, s, plane, rw, ip, nx, -DIR);
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == DIR)
            hn[a * N + b] = glead ? ghost_of<R, N>(L, P, a, b, m_c, m_m, m_p) : hn[a * N + b];
      }
    }
    if (wave_any(live && gtrail)) {
      // (loaded, not taken from the neighbouring lanes: with the ghost of
      // g^(k+1) that also takes its neighbours' masses, the reach would
      // exceed the two halo lanes)
      const uint32_t rw = (uint32_t)wa * ld;
      const R m_c = wall_mass<R, N>(L, s, plane, rw, ic, nx, DIR);
      const R m_m = wall_mass<R, N>(L, s, plane, rw, im, nx, DIR);
      const R m_p = wall_mass<R, N>(L, s, plane, rw, ip, nx, DIR);
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == -DIR)
            hn[a * N + b] = gtrail ? ghost_of<R, N>(L, P, a, b, m_c, m_m, m_p) : hn[a * N + b];
      }
    }
    R d[Q];
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        const int sg = node_sign<N>(b);
        if (sg == DIR) {  // lead
          d[l] = fmaR(L.qm[b], hn[l], L.p[b] * hp[l]);
          hp[l] = hn[l];
        } else if (sg == -DIR) {  // trail
          d[l] = fmaR(L.qm[b], hp[l], L.p[b] * hn[l]);
          hp[l] = hn[l];
        } else {
          d[l] = hn[l];
        }
      }
    }
    R g[Q];
    collide_regs<R, N, ORD, COMP>(L, P, d, g);
    // x part of the second remap: upstream column from the neighbouring
    // lane (a neighbour in another lane group is a halo lane's, whose
    // results are not stored)
    R x[Q];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const int sa = node_sign<N>(a);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        if (sa > 0)
          x[l] = fmaR(L.qm[a], g[l], L.p[a] * lane_from<DPP_PREV>(g[l]));
        else if (sa < 0)
          x[l] = fmaR(L.qm[a], g[l], L.p[a] * lane_from<DPP_NEXT>(g[l]));
        else
          x[l] = g[l];
      }
    }
    if (t == 1 && wave_any(gh_first)) {
      // ghost of g^{k+1} behind the first output row (a wall row): mass its
      // populations carry through that wall, re-emitted into the lead ones
      R m = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        if (node_sign<N>(b) != -DIR) continue;
        R acc = R(0);
#pragma unroll
        for (int a = 0; a < N; ++a) acc += x[a * N + b];
        m = fmaR(L.p[b], acc, m);
      }
      const R m_m = lane_from<DPP_PREV>(m), m_p = lane_from<DPP_NEXT>(m);
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == DIR)
            y1[a * N + b] = gh_first ? ghost_of<R, N>(L, P, a, b, m, m_m, m_p) : y1[a * N + b];
      }
    }
    const bool gl_now = gh_last && t == nout + 1;
    if (wave_any(gl_now)) {
      // ghost of g^{k+1} beyond the last output row (a wall row), from that
      // row's x-pulled g^{k+1} (in y1), re-emitted into the trail populations
      R m = R(0);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        if (node_sign<N>(b) != DIR) continue;
        R acc = R(0);
#pragma unroll
        for (int a = 0; a < N; ++a) acc += y1[a * N + b];
        m = fmaR(L.p[b], acc, m);
      }
      const R m_m = lane_from<DPP_PREV>(m), m_p = lane_from<DPP_NEXT>(m);
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b)
          if (node_sign<N>(b) == -DIR)
            x[a * N + b] = gl_now ? ghost_of<R, N>(L, P, a, b, m, m_m, m_p) : x[a * N + b];
      }
    }
    if (t >= 2) {  // second step on output row r - DIR
      R e[Q];
#pragma unroll
      for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = 0; b < N; ++b) {
          const int l = a * N + b;
          const int sg = node_sign<N>(b);
          if (sg == DIR)
            e[l] = fmaR(L.qm[b], y1[l], L.p[b] * y2[l]);
          else if (sg == -DIR)
            e[l] = fmaR(L.qm[b], y1[l], L.p[b] * x[l]);
          else
            e[l] = y1[l];
        }
      }
      R g2[Q];
      collide_regs<R, N, ORD, COMP>(L, P, e, g2);
      if (active && t <= nout + 1) {
        const uint32_t om = (uint32_t)(r - DIR) * ld + (uint32_t)ic;
#pragma unroll
        for (int l = 0; l < Q; ++l) bst(dst, om, (uint32_t)(l * plane), g2[l]);
      }
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        if (node_sign<N>(b) == DIR) y2[l] = y1[l];
        y1[l] = x[l];
      }
    }
  }
}


// Walled grid, one instance: workgroup = 4 wavefronts = 4 consecutive row
// segments of a strip of 60 output columns (two halo lanes on each side).
constexpr int STRIP2W = 60;
template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_march2w(const MarchArgs<R> A) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;  // multiple of 8
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  if (t >= A.n_tiles) return;
  const Inst<R>& P = A.inst;
  const int nx = P.nx, ny = P.ny;
  const int tx = t % A.tiles_x, ty = t / A.tiles_x;
  const int group = ty * 4 + wave;
  const int j0 = group * A.rows;
  if (j0 >= ny) return;  // wave-uniform
  const int j1 = min(j0 + A.rows, ny);
  const int col = tx * STRIP2W - 2 + lane;
  const bool active = lane >= 2 && lane < 64 - 2 && col < nx;
  int ic = col % nx;
  ic = ic < 0 ? ic + nx : ic;
  const int im = ic == 0 ? nx - 1 : ic - 1;
  const int ip = ic == nx - 1 ? 0 : ic + 1;
  if (group & 1)
    march2_wall_seg<R, N, ORD, COMP, -1>(A, P, ic, im, ip, active, true, j0, j1, j1 - j0 + 2);
  else
    march2_wall_seg<R, N, ORD, COMP, +1>(A, P, ic, im, ip, active, true, j0, j1, j1 - j0 + 2);
}

// Batched walled channels, two steps per launch: persistent grid-stride
// over the live work list as k_march_batch.  An item is one strip of an
// instance (Wg - 4 output columns, two halo lanes each side, 5 <= Wg <= 64
// lanes) and G = 64 / Wg consecutive row segments, one per lane group
// (lanes past G Wg idle); the groups of a wavefront march in the same
// direction.  A chunk of steps ends with single-step launches (the
// library's state semantics: the other buffer holds g^{k-1}), which also do
// the check mode.
template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_march2_batch(const MarchArgs<R> A) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_work = *A.n_work;
  int lo = 0, hi = n_work, first = blockIdx.x * 4 + wave, stride = gridDim.x * 4;
  if ((gridDim.x & 7) == 0) {  // one contiguous range of the list per XCD
    const int x = blockIdx.x & 7;
    lo = (int)((int64_t)n_work * x / 8);
    hi = (int)((int64_t)n_work * (x + 1) / 8);
    first = lo + (int)(blockIdx.x >> 3) * 4 + wave;
    stride = (int)(gridDim.x >> 3) * 4;
  }
  for (int w = first; w < hi; w += stride) {
    const Work it = ro(A.work, w);
    const Inst<R>& P = ro(A.insts, it.inst);
    const int Wg = it.shape & 0xff, rows = (it.shape >> 8) & 0xff;
    const int G = 64 / Wg;
    const int g = lane / Wg, gl = lane - g * Wg;
    const int seg = it.seg0 + g;
    const int j0 = seg * rows;
    const bool live = g < G && j0 < P.ny;
    const int j1 = min(j0 + rows, P.ny);
    const int nx = P.nx;
    const int col = it.x0 - 2 + gl;
    const bool active = live && gl >= 2 && gl < Wg - 2 && col < nx;
    int ic = col % nx;
    ic = ic < 0 ? ic + nx : ic;
    const int im = ic == 0 ? nx - 1 : ic - 1;
    const int ip = ic == nx - 1 ? 0 : ic + 1;
    if ((it.seg0 / G) & 1)
      march2_wall_seg<R, N, ORD, COMP, -1>(A, P, ic, im, ip, active, live, j0, j1, rows + 2);
    else
      march2_wall_seg<R, N, ORD, COMP, +1>(A, P, ic, im, ip, active, live, j0, j1, rows + 2);
  }
}

// ------------------------------------------------------- non-uniform rows --
// Wall masses through a wall with non-uniform rows, at two columns ca and cb:
// the rows listed in I[b] carry the length len across the wall.  NT entries
// are read for every b (the longest list; shorter ones end in zero lengths
// on row 0, which add nothing), so that no load waits behind a branch.
template <typename R, int N, int NT>
__device__ __forceinline__ void wall_mass_rows(const Lat<R>& L, const IncRows<R> (&I)[N], rsrc_t s,
                                               int64_t plane, uint32_t ld, int ca, int cb, int nx,
                                               int dir, R& ma, R& mb) {
  const int cam = wrapc(ca - 1, nx), cap = wrapc(ca + 1, nx);
  const int cbm = wrapc(cb - 1, nx), cbp = wrapc(cb + 1, nx);
  ma = R(0);
  mb = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    if (node_sign<N>(b) != dir) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const uint32_t rb = (uint32_t)I[b].j[t] * ld;
      const RowOff oa = row_off(rb, ca, cam, cap), ob = row_off(rb, cb, cbm, cbp);
      R acca = R(0), accb = R(0);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const uint32_t pl = (uint32_t)((a * N + b) * plane);
        acca += xpull<R, N>(L, s, pl, a, oa);
        accb += xpull<R, N>(L, s, pl, a, ob);
      }
      ma = fmaR(I[b].len[t], acca, ma);
      mb = fmaR(I[b].len[t], accb, mb);
    }
  }
}

// Wall mass through one wall (dir) at the lane's column ic and at its
// neighbours im, ip.  Each lane forms the mass at its own column and the
// neighbouring ones come from the adjacent lanes (consecutive columns; an
// idle lane past the grid's last column holds column 0, its periodic
// neighbour), except at the wavefront's two edge lanes, which form their
// outer neighbour's mass themselves.  The arithmetic per column is the
// same wherever it is formed.
template <typename R, int N>
__device__ __forceinline__ void wall_masses(const MarchArgs<R>& A, rsrc_t s, int64_t plane,
                                            uint32_t ld, int ic, int im, int ip, int nx, int lane,
                                            int dir, R& mc, R& mm, R& mp) {
  IncRows<R> I[N];
#pragma unroll
  for (int b = 0; b < N; ++b)
    if (node_sign<N>(b) == dir) I[b] = A.inc[b];
  const int ce = lane == 0 ? im : (lane == 63 ? ip : ic);
  R me;
  switch (A.inc_rows) {
    case 1: wall_mass_rows<R, N, 1>(A.lat, I, s, plane, ld, ic, ce, nx, dir, mc, me); break;
    case 2: wall_mass_rows<R, N, 2>(A.lat, I, s, plane, ld, ic, ce, nx, dir, mc, me); break;
    case 3: wall_mass_rows<R, N, 3>(A.lat, I, s, plane, ld, ic, ce, nx, dir, mc, me); break;
    default: wall_mass_rows<R, N, 4>(A.lat, I, s, plane, ld, ic, ce, nx, dir, mc, me); break;
  }
  const R l = lane_from<DPP_PREV>(mc), r = lane_from<DPP_NEXT>(mc);
  mm = lane == 0 ? me : l;
  mp = lane == 63 ? me : r;
}

// One cell of a grid with tabulated (non-uniform) rows.
template <typename R, int N, int ORD, bool COMP, int MODE>
__device__ __forceinline__ void rows_cell(const MarchArgs<R>& A, const Inst<R>& P, rsrc_t s,
                                          rsrc_t dst, int k, int i, int lane, bool active,
                                          double (&tot)[5], int& bad) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const int nx = P.nx, ny = P.ny;
  const int64_t plane = P.plane;
  const uint32_t ld = (uint32_t)P.ld;
  const int ic = active ? i : 0;
  const int im = ic == 0 ? nx - 1 : ic - 1;
  const int ip = ic == nx - 1 ? 0 : ic + 1;
  R d[Q];
  if ((MODE == MODE_AUX) && (A.aux & AUX_IDENTITY)) {
#pragma unroll
    for (int l = 0; l < Q; ++l) d[l] = bld<R>(s, (uint32_t)k * ld + (uint32_t)ic, (uint32_t)(l * plane));
  } else {
    // the row's tables are read once, up front, and the taps are loaded
    // without a branch on their weights: the loads of a row are then issued
    // together instead of one table read and one round trip per tap
    const int flag = A.rowflag[k];
    RowTap<R> TT[N];
#pragma unroll
    for (int b = 0; b < N; ++b) TT[b] = A.taps[b * ny + k];
    // the first nt entries of every tap list of the row (nt: the longest
    // list, the rest of a shorter one has weight 0 and adds nothing); the
    // path is also specialised on the walls whose ghost the row pulls, so
    // that a wall row's wall-mass and tap loads go out together
    auto pull = [&](auto nt, auto wl) {
      constexpr int NT = decltype(nt)::value, WL = decltype(wl)::value;
      R lo_c = R(0), lo_m = R(0), lo_p = R(0), hi_c = R(0), hi_m = R(0), hi_p = R(0);
      if constexpr ((WL & 1) != 0)
        wall_masses<R, N>(A, s, plane, ld, ic, im, ip, nx, lane, -1, lo_c, lo_m, lo_p);
      if constexpr ((WL & 2) != 0)
        wall_masses<R, N>(A, s, plane, ld, ic, im, ip, nx, lane, +1, hi_c, hi_m, hi_p);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const RowTap<R>& T = TT[b];
        RowOff o[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) o[t] = row_off((uint32_t)T.src[t] * ld, ic, im, ip);
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const int l = a * N + b;
          const uint32_t pl = (uint32_t)(l * plane);
          R acc = R(0);
#pragma unroll
          for (int t = 0; t < NT; ++t) acc = fmaR(T.w[t], xpull<R, N>(L, s, pl, a, o[t]), acc);
          if ((WL & 1) && T.glo != R(0))
            acc = fmaR(T.glo, ghost_pull<R, N>(L, a, P.kap_lo[l], P.phi_lo[l], lo_c, lo_m, lo_p), acc);
          if ((WL & 2) && T.ghi != R(0))
            acc = fmaR(T.ghi, ghost_pull<R, N>(L, a, P.kap_hi[l], P.phi_hi[l], hi_c, hi_m, hi_p), acc);
          d[l] = acc;
        }
      }
    };
    auto taps = [&](auto wl) {
      switch ((flag >> 2) & 3) {
        case 0:
        case 1: pull(std::integral_constant<int, 2>{}, wl); break;
        case 2: pull(std::integral_constant<int, 3>{}, wl); break;
        default: pull(std::integral_constant<int, 4>{}, wl); break;
      }
    };
    if constexpr (N > 4) {
      // one wall path (both walls' masses; a row that does not pull a
      // wall's ghost has zero weights for it): less code for the
      // instruction cache
      if (flag & 3)
        taps(std::integral_constant<int, 3>{});
      else
        taps(std::integral_constant<int, 0>{});
    } else {
      switch (flag & 3) {
        case 0: taps(std::integral_constant<int, 0>{}); break;
        case 1: taps(std::integral_constant<int, 1>{}); break;
        case 2: taps(std::integral_constant<int, 2>{}); break;
        default: taps(std::integral_constant<int, 3>{}); break;
      }
    }
  }
  cell_tail<R, N, ORD, COMP, MODE>(A, P, dst, d, k, i, active, A.dy[k], tot, bad);
}

// Non-uniform-row step: a workgroup covers 64 columns x 4 rows, one row per
// wavefront, so every row-table read is wave-uniform.
template <typename R, int N, int ORD, bool COMP, int MODE>
__global__ __launch_bounds__(256) void k_rows(const MarchArgs<R> A) {
  constexpr int Q = N * N;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;
  const int t = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  const Inst<R>& P = A.inst;
  if (t < A.n_tiles) {
    const int tx = t % A.tiles_x, ty = t / A.tiles_x;
    const int i = tx * 64 + lane;
    const int k = ty * 4 + wave;
    if (k < P.ny) {
      const uint32_t bytes = (uint32_t)(Q * P.plane * (int64_t)sizeof(R));
      const rsrc_t s = make_rsrc(A.src + P.off, bytes);
      const rsrc_t dst = make_rsrc(A.dst + P.off, bytes);
      rows_cell<R, N, ORD, COMP, MODE>(A, P, s, dst, k, i, lane, i < P.nx, tot, bad);
    }
  }
  if constexpr (MODE != MODE_STEP) {
    if (MODE == MODE_CHECK || (A.aux & AUX_FIELDS)) {
      block_totals<MODE>(tot, bad, A.partials, A.flag);
      if (A.mass) wave_mass(tot[4], A.mass);
    }
  }
}


// ---------------------------------------------------------------- batched --
// Persistent grid-stride step over a device-resident work list: each
// wavefront takes work items (instance, strip, segment group) until the
// list, whose live length is read from device memory, is exhausted.  The
// per-instance parameters are read from device memory with scalar loads.
template <typename R, int N, int ORD, bool COMP, int MODE, bool PF>
__global__ __launch_bounds__(256) void k_march_batch(const MarchArgs<R> A) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_work = *A.n_work;
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  // Workgroups go round-robin to the 8 XCDs.  Split the live list into 8
  // equal contiguous ranges, one per XCD, so that adjacent segments of a
  // strip, which share halo rows, run on one XCD and hit its L2; within a
  // range the XCD's workgroups stride over the items.
  int lo = 0, hi = n_work, first = blockIdx.x * 4 + wave, stride = gridDim.x * 4;
  if ((gridDim.x & 7) == 0) {
    const int x = blockIdx.x & 7;
    lo = (int)((int64_t)n_work * x / 8);
    hi = (int)((int64_t)n_work * (x + 1) / 8);
    first = lo + (int)(blockIdx.x >> 3) * 4 + wave;
    stride = (int)(gridDim.x >> 3) * 4;
  }
  for (int w = first; w < hi; w += stride) {
    const Work it = ro(A.work, w);
    const Inst<R>& P = ro(A.insts, it.inst);
    const int W = it.shape & 0xff, rows = it.shape >> 8;
    const int i = it.x0 + (lane & (W - 1));
    const int seg = it.seg0 + lane / W;
    const int j0 = seg * rows;
    const int j1 = min(j0 + rows, P.ny);
    const int group = it.seg0 / (64 / W);
    if (j0 < P.ny) march_lane<R, N, ORD, COMP, MODE, PF>(A, P, i, i < P.nx, j0, j1, group, tot, bad);
    if constexpr (MODE != MODE_STEP) {
      if (A.mass && (MODE == MODE_CHECK || (A.aux & AUX_FIELDS))) {
        wave_mass(tot[4], A.mass + it.inst);  // the item's instance
        tot[4] = 0.0;
      }
    }
  }
  if constexpr (MODE != MODE_STEP) {
    if (bad) A.flag[0] = 1;
  }
}

// Per-instance residual after a chunk of K steps,
// r = ||q - q_prev|| / (K ||q||) over the instance's stacked fields, in two
// fixed-order passes.  Pass 1: RESID_SLICES workgroups per active instance
// each reduce one contiguous slice of its fields into a partial pair and
// refresh that slice of the snapshot.
template <typename R>
__global__ __launch_bounds__(256) void k_batch_resid_part(const BatchCtl<R> C) {
  __shared__ double sh[2][4];
  const int b = blockIdx.x / RESID_SLICES, sl = blockIdx.x % RESID_SLICES;
  if (!C.active[b]) return;
  const Inst<R>& P = C.insts[b];
  const int64_t n = (int64_t)4 * P.nx * P.ny;
  const int64_t k0 = n * sl / RESID_SLICES, k1 = n * (sl + 1) / RESID_SLICES;
  const R* q = C.fields + P.fld;
  R* qp = C.prev + P.fld;
  double a = 0.0, s = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
    const double v = (double)q[k], dv = v - (double)qp[k];
    a += dv * dv;
    s += v * v;
    qp[k] = q[k];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    s += __shfl_xor(s, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wave] = a; sh[1][wave] = s; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int c = threadIdx.x;
    C.part[(int64_t)blockIdx.x * 2 + c] = ((sh[c][0] + sh[c][1]) + sh[c][2]) + sh[c][3];
  }
}

// Pass 2 (one thread per instance): sum the slices in order, advance the
// step count, and retire the instance when r < tol or its step budget is
// spent.
template <typename R>
__global__ __launch_bounds__(256) void k_batch_resid_fin(const BatchCtl<R> C, int n_inst) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_inst || !C.active[b]) return;
  double A2 = 0.0, S2 = 0.0;
  for (int sl = 0; sl < RESID_SLICES; ++sl) {
    A2 += C.part[((int64_t)b * RESID_SLICES + sl) * 2];
    S2 += C.part[((int64_t)b * RESID_SLICES + sl) * 2 + 1];
  }
  const int64_t st = C.steps[b] + C.K;
  C.steps[b] = st;
  const double r = C.have_prev[b] ? __builtin_sqrt(A2) / ((double)C.K * __builtin_sqrt(S2))
                                  : __builtin_inf();
  C.have_prev[b] = 1;
  C.resid[b] = r;
  if (!(r == r)) C.flag[0] = 1;
  if (!(r >= C.tol) || st >= C.max_steps) C.active[b] = 0;
}

// Rebuild the work list from the active instances' items, in instance
// order; one workgroup per instance.  Each workgroup sums the item counts
// of the active instances before it (block b = 0 also writes the totals),
// then copies its own items.
__global__ __launch_bounds__(256) void k_batch_compact(const int32_t* __restrict__ active,
                                                       const int32_t* __restrict__ item_start,
                                                       const Work* __restrict__ all,
                                                       Work* __restrict__ work,
                                                       int32_t* __restrict__ n_work,
                                                       int32_t* __restrict__ remaining,
                                                       int n_inst) {
  __shared__ int sh[3][4];
  const int b = blockIdx.x;
  const int lim = b == 0 ? n_inst : b;
  int before = 0, total = 0, rem = 0;
  for (int k = threadIdx.x; k < lim; k += 256) {
    const int cnt = active[k] ? item_start[k + 1] - item_start[k] : 0;
    if (k < b) before += cnt;
    total += cnt;
    rem += active[k] ? 1 : 0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    before += __shfl_xor(before, off, 64);
    total += __shfl_xor(total, off, 64);
    rem += __shfl_xor(rem, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wave] = before; sh[1][wave] = total; sh[2][wave] = rem; }
  __syncthreads();
  const int o = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
  if (b == 0 && threadIdx.x == 0) {
    *n_work = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    *remaining = sh[2][0] + sh[2][1] + sh[2][2] + sh[2][3];
  }
  if (!active[b]) return;
  const int s0 = item_start[b], cnt = item_start[b + 1] - s0;
  for (int t = threadIdx.x; t < cnt; t += 256) work[o + t] = all[s0 + t];
}

// ----------------------------------------------------------------- init ---
// f^0 (deviations) into `f0`, and g^0 = C(f^0) into `g0`, pitch ld.
template <typename R, int N, int ORD, bool COMP>
__global__ __launch_bounds__(256) void k_init(const InitArgs<R> A) {
  constexpr int Q = N * N;
  const Lat<R>& L = A.lat;
  const Inst<R>& P = A.inst;
  const int64_t n = (int64_t)P.nx * P.ny;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int j = (int)(c / P.nx), i = (int)(c % P.nx);
  R d[Q];
  if (A.fabs) {
#pragma unroll
    for (int l = 0; l < Q; ++l) d[l] = A.fabs[l * n + c] - L.w[l];
  } else {
    Fields<R> F;
    F.rho = A.rho[c];
    F.drho = F.rho - R(1);
    F.ux = A.ux[c];
    F.uy = A.uy[c];
    F.th = A.T[c] - R(1);
    EqNodes<R, N> E;
    eq_nodes<R, N, ORD>(L, F, E);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      R Fa, Ka, Na;
      eq_anode<R, N, ORD>(L, E, a, Fa, Ka, Na);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int l = a * N + b;
        d[l] = L.w[l] * eq_dev<R, N, ORD>(L, E, a, b, Fa, Ka, Na);
        if (A.noise) d[l] += A.noise[l * n + c];
      }
    }
  }
  const int64_t o = P.off + (int64_t)j * P.ld + i;
#pragma unroll
  for (int l = 0; l < Q; ++l) A.f0[o + l * P.plane] = d[l];
  R drho, jx, jy, ed;
  cell_moments<R, N, COMP>(L, d, drho, jx, jy, ed);
  const Fields<R> F = fields_from(drho, jx, jy, ed);
  bgk_cell<R, N, ORD>(L, P, F, d);
#pragma unroll
  for (int l = 0; l < Q; ++l) A.g0[o + l * P.plane] = d[l];
}

// ------------------------------------------------------ mass re-imposition --
// Adds delta w_l to every population of an instance's post-collision state,
// delta = (M0 - M) / area from the fixed-point deviation masses of the
// reference state (ref) and of the last check (cur): the deficit re-enters
// as a uniform density increment at rest (zero momentum).  Batched runs
// (active != null) touch active instances only; RESID_SLICES workgroups per
// instance stride over its cells.
template <typename R>
__global__ __launch_bounds__(256) void k_mass_fix(R* __restrict__ g, const Inst<R>* __restrict__ insts,
                                                  Inst<R> single, const int32_t* __restrict__ active,
                                                  const unsigned long long* __restrict__ ref,
                                                  const unsigned long long* __restrict__ cur,
                                                  const double* __restrict__ area, Lat<R> L, int q) {
  const int b = blockIdx.x / RESID_SLICES, sl = blockIdx.x % RESID_SLICES;
  if (active && !active[b]) return;
  const Inst<R>& P = insts ? insts[b] : single;
  const long long dmi = (long long)(ref[b] - cur[b]);
  if (dmi == 0) return;
  const R delta = (R)((double)dmi / MASS_FP_SCALE / area[b]);
  const int64_t n = (int64_t)P.nx * P.ny;  // < 2^31 (a plane is 32-bit addressed)
  const int k0 = (int)(n * sl / RESID_SLICES), k1 = (int)(n * (sl + 1) / RESID_SLICES);
  const uint32_t nx = (uint32_t)P.nx;
  const int64_t pl = P.plane;
  for (int c = k0 + (int)threadIdx.x; c < k1; c += 256) {
    const uint32_t j = (uint32_t)c / nx, i = (uint32_t)c - j * nx;
    R* p = g + P.off + (int64_t)j * P.ld + i;
    // eight loads ahead of their stores: the compiler cannot tell the
    // populations' addresses apart, and would otherwise wait out one load
    // per population
    int l = 0;
    for (; l + 8 <= q; l += 8) {
      R v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(l + u) * pl];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[(l + u) * pl] = fmaR(L.w[l + u], delta, v[u]);
    }
    for (; l < q; ++l) p[l * pl] = fmaR(L.w[l], delta, p[l * pl]);
  }
}

// ------------------------------------------------------------ reductions --
// out[c] = sum_b part[b*width + c], fixed order (deterministic).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int nblk,
                                                int width, double* __restrict__ out) {
  __shared__ double sh[256];
  for (int c = 0; c < width; ++c) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(int64_t)b * width + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
    __syncthreads();
  }
}

// p[0..n) = v (a kernel rather than a memset, so that it may sit in a
// captured graph)
__global__ __launch_bounds__(64) void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  for (int k = threadIdx.x; k < n; k += 64) p[k] = v;
}

// Streaming copy of n 16-byte elements (grid-stride, four in flight per
// lane): the achievable HBM read + write rate on buffers larger than the
// Infinity Cache, the practical ceiling the step kernels are compared with.
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src,
                                                     float4* __restrict__ dst, int64_t n) {
  // plain grid-stride, one 16-byte element per lane per pass: with enough
  // workgroups in flight (up to 65536) this reached 5.4 TB/s on 1 GiB
  // buffers, more than the unrolled and non-temporal forms tried
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride) dst[k] = src[k];
}

// per-block partial sums of (q - qp)^2 and q^2 over n values
template <typename R>
__global__ __launch_bounds__(256) void k_resid(const R* __restrict__ q, const R* __restrict__ qp,
                                               int64_t n, double* __restrict__ part) {
  __shared__ double sh[2][4];
  double a = 0.0, b = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
    const double v = (double)q[k], dv = v - (double)qp[k];
    a += dv * dv;
    b += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sh[0][wave] = a; sh[1][wave] = b; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int c = threadIdx.x;
    part[(int64_t)blockIdx.x * 2 + c] = ((sh[c][0] + sh[c][1]) + sh[c][2]) + sh[c][3];
  }
}

// ------------------------------------------------------------- dispatch ---
template <typename R, int N, int ORD, bool COMP>
static hipError_t march_mode(int mode, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  if (A.taps) {
    switch (mode) {
      case MODE_STEP: hipLaunchKernelGGL((k_rows<R, N, ORD, COMP, MODE_STEP>), g, b, 0, st, A); break;
      case MODE_CHECK: hipLaunchKernelGGL((k_rows<R, N, ORD, COMP, MODE_CHECK>), g, b, 0, st, A); break;
      default: hipLaunchKernelGGL((k_rows<R, N, ORD, COMP, MODE_AUX>), g, b, 0, st, A); break;
    }
    return hipGetLastError();
  }
  switch (mode) {
    case MODE_STEP:
      if (A.prefetch)
        hipLaunchKernelGGL((k_march<R, N, ORD, COMP, MODE_STEP, true>), g, b, 0, st, A);
      else
        hipLaunchKernelGGL((k_march<R, N, ORD, COMP, MODE_STEP, false>), g, b, 0, st, A);
      break;
    case MODE_CHECK: hipLaunchKernelGGL((k_march<R, N, ORD, COMP, MODE_CHECK, false>), g, b, 0, st, A); break;
    default: hipLaunchKernelGGL((k_march<R, N, ORD, COMP, MODE_AUX, false>), g, b, 0, st, A); break;
  }
  return hipGetLastError();
}

template <typename R, bool COMP>
static hipError_t march_lat(int n, int mode, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  switch (n) {
    case 3: return march_mode<R, 3, 2, COMP>(mode, A, nblocks, st);
    case 4: return march_mode<R, 4, 3, COMP>(mode, A, nblocks, st);
    case 6: return march_mode<R, 6, 4, COMP>(mode, A, nblocks, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<float>& A, int nblocks,
                        hipStream_t st) {
  return comp ? march_lat<float, true>(n, mode, A, nblocks, st)
              : march_lat<float, false>(n, mode, A, nblocks, st);
}
hipError_t launch_march(int n, bool comp, int mode, const MarchArgs<double>& A, int nblocks,
                        hipStream_t st) {
  (void)comp;
  return march_lat<double, false>(n, mode, A, nblocks, st);
}

template <bool COMP>
static hipError_t march_pairs_lat(int n, const MarchArgs<f32x2>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  switch (n) {
    case 3: hipLaunchKernelGGL((k_march<f32x2, 3, 2, COMP, MODE_STEP, false>), g, b, 0, st, A); break;
    case 4: hipLaunchKernelGGL((k_march<f32x2, 4, 3, COMP, MODE_STEP, false>), g, b, 0, st, A); break;
    case 6: hipLaunchKernelGGL((k_march<f32x2, 6, 4, COMP, MODE_STEP, false>), g, b, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_march_pairs(int n, bool comp, const MarchArgs<f32x2>& A, int nblocks,
                              hipStream_t st) {
  return comp ? march_pairs_lat<true>(n, A, nblocks, st) : march_pairs_lat<false>(n, A, nblocks, st);
}

template <typename R, bool COMP>
static hipError_t march2_lat(int n, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  switch (n) {
    case 3: hipLaunchKernelGGL((k_march2<R, 3, 2, COMP>), g, b, 0, st, A); break;
    case 4: hipLaunchKernelGGL((k_march2<R, 4, 3, COMP>), g, b, 0, st, A); break;
    case 6:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((k_march2<R, 6, 4, COMP>), g, b, 0, st, A);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_march2(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st) {
  return comp ? march2_lat<float, true>(n, A, nblocks, st) : march2_lat<float, false>(n, A, nblocks, st);
}
hipError_t launch_march2(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st) {
  (void)comp;  // FP64 sums need no compensation
  return march2_lat<double, false>(n, A, nblocks, st);
}

template <typename R, bool COMP>
static hipError_t march2w_lat(int n, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  switch (n) {
    case 3: hipLaunchKernelGGL((k_march2w<R, 3, 2, COMP>), g, b, 0, st, A); break;
    case 4: hipLaunchKernelGGL((k_march2w<R, 4, 3, COMP>), g, b, 0, st, A); break;
    case 6:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((k_march2w<R, 6, 4, COMP>), g, b, 0, st, A);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_march2w(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st) {
  return comp ? march2w_lat<float, true>(n, A, nblocks, st) : march2w_lat<float, false>(n, A, nblocks, st);
}
hipError_t launch_march2w(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st) {
  (void)comp;
  return march2w_lat<double, false>(n, A, nblocks, st);
}

template <typename R, bool COMP>
static hipError_t march2_batch_lat(int n, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  switch (n) {
    case 3: hipLaunchKernelGGL((k_march2_batch<R, 3, 2, COMP>), g, b, 0, st, A); break;
    case 4: hipLaunchKernelGGL((k_march2_batch<R, 4, 3, COMP>), g, b, 0, st, A); break;
    case 6:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((k_march2_batch<R, 6, 4, COMP>), g, b, 0, st, A);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_march2_batch(int n, bool comp, const MarchArgs<float>& A, int nblocks, hipStream_t st) {
  return comp ? march2_batch_lat<float, true>(n, A, nblocks, st) : march2_batch_lat<float, false>(n, A, nblocks, st);
}
hipError_t launch_march2_batch(int n, bool comp, const MarchArgs<double>& A, int nblocks, hipStream_t st) {
  (void)comp;
  return march2_batch_lat<double, false>(n, A, nblocks, st);
}

template <typename R, bool COMP>
static hipError_t init_lat(int n, const InitArgs<R>& A, hipStream_t st) {
  const int64_t cells = (int64_t)A.inst.nx * A.inst.ny;
  dim3 g((unsigned)((cells + 255) / 256)), b(256);
  switch (n) {
    case 3: hipLaunchKernelGGL((k_init<R, 3, 2, COMP>), g, b, 0, st, A); break;
    case 4: hipLaunchKernelGGL((k_init<R, 4, 3, COMP>), g, b, 0, st, A); break;
    case 6: hipLaunchKernelGGL((k_init<R, 6, 4, COMP>), g, b, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(int n, bool comp, const InitArgs<float>& A, hipStream_t st) {
  return comp ? init_lat<float, true>(n, A, st) : init_lat<float, false>(n, A, st);
}
hipError_t launch_init(int n, bool comp, const InitArgs<double>& A, hipStream_t st) {
  (void)comp;
  return init_lat<double, false>(n, A, st);
}

template <typename R, int N, int ORD, bool COMP, bool PF>
static hipError_t batch_mode(int mode, const MarchArgs<R>& A, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(256);
  switch (mode) {
    case MODE_STEP: hipLaunchKernelGGL((k_march_batch<R, N, ORD, COMP, MODE_STEP, PF>), g, b, 0, st, A); break;
    case MODE_CHECK: hipLaunchKernelGGL((k_march_batch<R, N, ORD, COMP, MODE_CHECK, PF>), g, b, 0, st, A); break;
    default: hipLaunchKernelGGL((k_march_batch<R, N, ORD, COMP, MODE_AUX, false>), g, b, 0, st, A); break;
  }
  return hipGetLastError();
}

template <typename R, bool COMP>
static hipError_t batch_lat(int n, int mode, bool pf, const MarchArgs<R>& A, int nblocks,
                            hipStream_t st) {
  switch (n) {
    case 3: return pf ? batch_mode<R, 3, 2, COMP, true>(mode, A, nblocks, st)
                      : batch_mode<R, 3, 2, COMP, false>(mode, A, nblocks, st);
    case 4: return pf ? batch_mode<R, 4, 3, COMP, true>(mode, A, nblocks, st)
                      : batch_mode<R, 4, 3, COMP, false>(mode, A, nblocks, st);
    case 6: return pf ? batch_mode<R, 6, 4, COMP, true>(mode, A, nblocks, st)
                      : batch_mode<R, 6, 4, COMP, false>(mode, A, nblocks, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_march_batch(int n, bool comp, int mode, bool prefetch, const MarchArgs<float>& A,
                              int nblocks, hipStream_t st) {
  return comp ? batch_lat<float, true>(n, mode, prefetch, A, nblocks, st)
              : batch_lat<float, false>(n, mode, prefetch, A, nblocks, st);
}
hipError_t launch_march_batch(int n, bool comp, int mode, bool prefetch, const MarchArgs<double>& A,
                              int nblocks, hipStream_t st) {
  (void)comp;
  return batch_lat<double, false>(n, mode, prefetch, A, nblocks, st);
}

template <typename R>
static hipError_t batch_resid_impl(const BatchCtl<R>& C, int n_inst, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_resid_part<R>, dim3(n_inst * RESID_SLICES), dim3(256), 0, st, C);
  hipLaunchKernelGGL(k_batch_resid_fin<R>, dim3((n_inst + 255) / 256), dim3(256), 0, st, C, n_inst);
  return hipGetLastError();
}
hipError_t launch_batch_resid(const BatchCtl<float>& C, int n_inst, hipStream_t st) {
  return batch_resid_impl(C, n_inst, st);
}
hipError_t launch_batch_resid(const BatchCtl<double>& C, int n_inst, hipStream_t st) {
  return batch_resid_impl(C, n_inst, st);
}

hipError_t launch_batch_compact(const int32_t* active, const int32_t* item_start, const Work* all,
                                Work* work, int32_t* n_work, int32_t* remaining, int n_inst,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_batch_compact, dim3(n_inst), dim3(256), 0, st, active, item_start, all, work,
                     n_work, remaining, n_inst);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_copy, dim3(nblocks), dim3(256), 0, st, (const float4*)src, (float4*)dst,
                     n16);
  return hipGetLastError();
}

template <typename R>
static hipError_t mass_fix_impl(R* g, const Inst<R>* insts, const Inst<R>& single, const int32_t* active,
                                const unsigned long long* ref, const unsigned long long* cur,
                                const double* area, const Lat<R>& L, int q, int n_inst, hipStream_t st) {
  hipLaunchKernelGGL(k_mass_fix<R>, dim3(n_inst * RESID_SLICES), dim3(256), 0, st, g, insts, single, active,
                     ref, cur, area, L, q);
  return hipGetLastError();
}
hipError_t launch_mass_fix(float* g, const Inst<float>* insts, const Inst<float>& single,
                           const int32_t* active, const unsigned long long* ref,
                           const unsigned long long* cur, const double* area, const Lat<float>& L,
                           int q, int n_inst, hipStream_t st) {
  return mass_fix_impl(g, insts, single, active, ref, cur, area, L, q, n_inst, st);
}
hipError_t launch_mass_fix(double* g, const Inst<double>* insts, const Inst<double>& single,
                           const int32_t* active, const unsigned long long* ref,
                           const unsigned long long* cur, const double* area, const Lat<double>& L,
                           int q, int n_inst, hipStream_t st) {
  return mass_fix_impl(g, insts, single, active, ref, cur, area, L, q, n_inst, st);
}

hipError_t launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int nblk, int width, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, part, nblk, width, out);
  return hipGetLastError();
}

template <typename R>
static hipError_t resid_impl(const R* q, const R* qp, int64_t n, double* part, int nblk,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_resid<R>, dim3(nblk), dim3(256), 0, st, q, qp, n, part);
  return hipGetLastError();
}
hipError_t launch_resid(const float* q, const float* qp, int64_t n, double* part, int nblk,
                        hipStream_t st) {
  return resid_impl(q, qp, n, part, nblk, st);
}
hipError_t launch_resid(const double* q, const double* qp, int64_t n, double* part, int nblk,
                        hipStream_t st) {
  return resid_impl(q, qp, n, part, nblk, st);
}

}  // namespace tvlbm
