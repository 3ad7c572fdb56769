// tvnet_kernels.hip -- bf16 matrix-core (MFMA) kernels of the warm-start
// network for gfx950: 3x3 convolution forward as an implicit GEMM, the
// backward-data pass as the same kernel over the transposed filter, the
// backward-weights pass as a pixel-reduction GEMM, the masked MSE loss and
// Adam.  Activations are channels-last bf16; accumulation is fp32.
//
// MFMA used: v_mfma_f32_16x16x32_bf16 (D[16x16] += A[16x32] B[32x16]).
// Lane l holds A row (l mod 16) and B column (l mod 16), each with the 8
// consecutive k of group (l / 16); D rows 4 (l / 16) + r, column (l mod 16).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvnetk {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.7071067811865476f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.7071067811865476f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

enum Epi { EPI_GELU = 0, EPI_LINEAR = 1, EPI_BWD = 2 };

struct ConvArgs {
  const bf16* x;       // input [B][H][W][CIN_P]
  const bf16* wk;      // filter as a GEMM operand [NT*16][KP]
  const float* bias;   // [cout]
  const float* zprev;  // EPI_BWD: pre-activation of this pass's output channels [B][H][W][cout]
  float* z;            // EPI_GELU: pre-activation out; EPI_LINEAR: output [B][H][W][cout]
  bf16* a;             // EPI_GELU: activation out; EPI_BWD: gradient out [B][H][W][a_stride]
  int B, H, W, cout, a_stride;
};

// One workgroup: 64 pixels of one row of one image; wavefront w owns 16 of
// them and all output channels (NT tiles of 16).  The input rows y-1..y+1 of
// the segment (plus a one-pixel halo) are staged in LDS, channels last, so a
// lane's 8 consecutive k (8 channels of one filter tap) are one 16-byte read.
template <int CIN_P, int NT, int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvArgs A) {
  constexpr int KP = ((9 * CIN_P + 31) / 32) * 32;
  constexpr int CH = CIN_P / 8;
  __shared__ __attribute__((aligned(16))) bf16 tile[3][66][CIN_P];
  const int x0 = blockIdx.x * 64, y = blockIdx.y, b = blockIdx.z;
  for (int t = threadIdx.x; t < 3 * 66 * CH; t += 256) {
    const int r = t / (66 * CH), rem = t % (66 * CH), cc = rem / CH, q = rem % CH;
    const int yy = y + r - 1, xx = x0 + cc - 1;
    uint4 v = {0u, 0u, 0u, 0u};
    if (yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
      v = *(const uint4*)(A.x + (((int64_t)b * A.H + yy) * A.W + xx) * CIN_P + q * 8);
    *(uint4*)(&tile[r][cc][q * 8]) = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  f32x4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < KP / 32; ++kc) {
    const int k0 = kc * 32 + g * 8;
    const int tap = k0 / CIN_P, c0 = k0 % CIN_P;
    bf16x8 av;
    if (tap < 9) {
      av = *(const bf16x8*)(&tile[tap / 3][16 * w + i + tap % 3][c0]);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) av[e] = (bf16)0.0f;
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bf16x8 bv = *(const bf16x8*)(A.wk + (int64_t)(nt * 16 + i) * KP + k0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int px = x0 + 16 * w + 4 * g + r, ch = nt * 16 + i;
      if (px < A.W && ch < A.cout) {
        const int64_t pix = ((int64_t)b * A.H + y) * A.W + px;
        const float v = acc[nt][r];
        if constexpr (EPI == EPI_GELU) {
          const float z = v + A.bias[ch];
          A.z[pix * A.cout + ch] = z;
          A.a[pix * A.a_stride + ch] = (bf16)gelu(z);
        } else if constexpr (EPI == EPI_LINEAR) {
          A.z[pix * A.cout + ch] = v + A.bias[ch];
        } else {
          A.a[pix * A.a_stride + ch] = (bf16)(v * gelu_grad(A.zprev[pix * A.cout + ch]));
        }
      }
    }
  }
}

struct WgradArgs {
  const bf16* x;     // layer input [B][H][W][CIN_P]
  const bf16* dz;    // output gradient [B][H][W][DZS]
  float* part;       // [nblocks][OT*16][K9P + 1] partial dW (last column: db)
  int B, H, W, cout, rows;  // rows per workgroup
};

// dW[o][k] = sum over pixels of dz[pix][o] * xcol[pix][k], k = tap*CIN_P + c:
// an MFMA GEMM whose reduction dimension is the pixels (32 per instruction).
// A workgroup reduces `rows` image rows into one partial; a second kernel
// adds the partials in a fixed order.
template <int CIN_P, int DZS, int OT>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs A) {
  constexpr int K9 = 9 * CIN_P;
  constexpr int K9P = ((K9 + 15) / 16) * 16;
  constexpr int KT = K9P / 16;
  constexpr int NTILE = OT * KT;
  constexpr int TPW = (NTILE + 3) / 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int Wp = A.W + 2;
  bf16* xin = (bf16*)smem;                         // [3][W+2][CIN_P]
  bf16* dzr = xin + 3 * Wp * CIN_P;                // [W][DZS]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int rows_per_img = (A.H + A.rows - 1) / A.rows;
  const int b = blockIdx.x / rows_per_img;
  const int y0 = (blockIdx.x % rows_per_img) * A.rows;
  f32x4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbias = 0.0f;
  const int nchunk = (A.W + 31) / 32;
  for (int y = y0; y < min(y0 + A.rows, A.H); ++y) {
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * Wp * CIN_P; t += 256) {
      const int r = t / (Wp * CIN_P), rem = t % (Wp * CIN_P), cc = rem / CIN_P, c = rem % CIN_P;
      const int yy = y + r - 1, xx = cc - 1;
      bf16 v = (bf16)0.0f;
      if (yy >= 0 && yy < A.H && xx >= 0 && xx < A.W) v = A.x[(((int64_t)b * A.H + yy) * A.W + xx) * CIN_P + c];
      xin[t] = v;
    }
    for (int t = threadIdx.x; t < A.W * DZS; t += 256)
      dzr[t] = A.dz[((int64_t)b * A.H + y) * A.W * DZS + t];
    __syncthreads();
    if (threadIdx.x < A.cout) {
      float s = 0.0f;
      for (int p = 0; p < A.W; ++p) s += (float)dzr[p * DZS + threadIdx.x];
      dbias += s;
    }
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = w + 4 * tt;
      if (t >= NTILE) break;
      const int ot = t / KT, kt = t % KT;
      const int o = ot * 16 + i;
      const int k = kt * 16 + i;
      const int tap = k / CIN_P, c = k % CIN_P;
      const int dy = tap / 3, dx = tap % 3;
      for (int pc = 0; pc < nchunk; ++pc) {
        bf16x8 av, bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int p = pc * 32 + g * 8 + e;
          const bool pin = p < A.W;
          av[e] = (pin && o < A.cout && o < DZS) ? dzr[p * DZS + o] : (bf16)0.0f;
          bv[e] = (pin && k < K9) ? xin[(dy * Wp + p + dx) * CIN_P + c] : (bf16)0.0f;
        }
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[tt], 0, 0, 0);
      }
    }
  }
  float* out = A.part + (int64_t)blockIdx.x * (OT * 16) * (K9P + 1);
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    const int t = w + 4 * tt;
    if (t >= NTILE) break;
    const int ot = t / KT, kt = t % KT;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(ot * 16 + 4 * g + r) * (K9P + 1) + kt * 16 + i] = acc[tt][r];
  }
  if (threadIdx.x < OT * 16) out[threadIdx.x * (K9P + 1) + K9P] = threadIdx.x < A.cout ? dbias : 0.0f;
}

// Sum the partials (fixed order) into the flat gradient of one layer:
// W[o][c][dy][dx] then b[o].
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nblk,
                                                      int rows_t, int k9p, int cin, int cin_p,
                                                      int cout, float* __restrict__ grad) {
  const int nw = cout * cin * 9;
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= nw + cout) return;
  int row, col;
  if (id < nw) {
    const int o = id / (cin * 9), rem = id % (cin * 9), c = rem / 9, tap = rem % 9;
    row = o;
    col = tap * cin_p + c;
  } else {
    row = id - nw;
    col = k9p;
  }
  float s = 0.0f;
  for (int bk = 0; bk < nblk; ++bk) s += part[((int64_t)bk * rows_t + row) * (k9p + 1) + col];
  grad[id] = s;
}

// Filter of one layer as the B operand of k_conv: wk[n][k], k = tap*CIN_P + c.
// transposed: the backward-data filter, n = input channel c, k = tap'*CIN_P + o
// with tap' = 8 - tap.
__global__ __launch_bounds__(256) void k_prep_filter(const float* __restrict__ w, int cout, int cin,
                                                     int rows, int kp, int cin_p, int transposed,
                                                     bf16* __restrict__ wk) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= rows * kp) return;
  const int n = id / kp, k = id % kp;
  const int tap = k / cin_p, c = k % cin_p;
  float v = 0.0f;
  if (tap < 9) {
    if (!transposed) {
      if (n < cout && c < cin) v = w[(n * cin + c) * 9 + tap];
    } else {
      if (n < cin && c < cout) v = w[(c * cin + n) * 9 + (8 - tap)];
    }
  }
  wk[id] = (bf16)v;
}

// fp32 [pixels][c_in] -> bf16 [pixels][cin_p], zero channel padding
__global__ __launch_bounds__(256) void k_pack_input(const float* __restrict__ x, int64_t npix,
                                                    int cin, int cin_p, bf16* __restrict__ out) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= npix * cin_p) return;
  const int64_t p = id / cin_p;
  const int c = (int)(id % cin_p);
  out[id] = (bf16)(c < cin ? x[p * cin + c] : 0.0f);
}

// Masked MSE: loss partials per block and the output gradient as bf16
// [pixels][dzs] (channels >= cout zero).
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ mask, int64_t npix, int cout,
                                              int dzs, float scale, bf16* __restrict__ dz,
                                              double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (p < npix) {
    const float m = mask[p];
    for (int c = 0; c < dzs; ++c) {
      float gval = 0.0f;
      if (c < cout) {
        const float d = y[p * cout + c] - t[p * cout + c];
        l += (double)m * d * d;
        gval = 2.0f * m * d * scale;
      }
      dz[p * dzs + c] = (bf16)gval;
    }
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ part, int n, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += part[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// Adam with bias correction (Kingma & Ba, 2015) on fp32 master weights.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= n) return;
  const float gi = g[id];
  const float mi = b1 * m[id] + (1.0f - b1) * gi;
  const float vi = b2 * v[id] + (1.0f - b2) * gi * gi;
  m[id] = mi;
  v[id] = vi;
  p[id] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------- launch --
hipError_t conv_launch(int cin_p, int nt, int epi, const ConvArgs& A, hipStream_t st) {
  dim3 g((A.W + 63) / 64, A.H, A.B), b(256);
#define TVNET_CONV(CP, NT_, E)                                                    \
  if (cin_p == CP && nt == NT_ && epi == E) {                                     \
    hipLaunchKernelGGL((k_conv<CP, NT_, E>), g, b, 0, st, A);                     \
    return hipGetLastError();                                                     \
  }
  TVNET_CONV(8, 2, EPI_GELU)
  TVNET_CONV(32, 2, EPI_GELU)
  TVNET_CONV(32, 1, EPI_LINEAR)
  TVNET_CONV(8, 2, EPI_BWD)
  TVNET_CONV(32, 2, EPI_BWD)
#undef TVNET_CONV
  return hipErrorInvalidValue;
}

int wgrad_k9p(int cin_p) { return ((9 * cin_p + 15) / 16) * 16; }

hipError_t wgrad_launch(int cin_p, int dzs, int ot, const WgradArgs& A, int nblk, hipStream_t st) {
  const size_t lds = (size_t)(3 * (A.W + 2) * cin_p + A.W * dzs) * sizeof(bf16);
#define TVNET_WG(CP, DZ, OT_)                                                      \
  if (cin_p == CP && dzs == DZ && ot == OT_) {                                     \
    hipLaunchKernelGGL((k_wgrad<CP, DZ, OT_>), dim3(nblk), dim3(256), lds, st, A); \
    return hipGetLastError();                                                      \
  }
  TVNET_WG(32, 8, 1)
  TVNET_WG(32, 32, 2)
  TVNET_WG(8, 32, 2)
#undef TVNET_WG
  return hipErrorInvalidValue;
}

hipError_t wgrad_reduce_launch(const float* part, int nblk, int rows_t, int k9p, int cin, int cin_p,
                               int cout, float* grad, hipStream_t st) {
  const int n = cout * cin * 9 + cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((n + 255) / 256), dim3(256), 0, st, part, nblk, rows_t, k9p,
                     cin, cin_p, cout, grad);
  return hipGetLastError();
}

hipError_t prep_filter_launch(const float* w, int cout, int cin, int rows, int kp, int cin_p,
                              int transposed, bf16* wk, hipStream_t st) {
  const int n = rows * kp;
  hipLaunchKernelGGL(k_prep_filter, dim3((n + 255) / 256), dim3(256), 0, st, w, cout, cin, rows, kp,
                     cin_p, transposed, wk);
  return hipGetLastError();
}

hipError_t pack_input_launch(const float* x, int64_t npix, int cin, int cin_p, bf16* out, hipStream_t st) {
  const int64_t n = npix * cin_p;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, npix, cin, cin_p,
                     out);
  return hipGetLastError();
}

hipError_t loss_launch(const float* y, const float* t, const float* mask, int64_t npix, int cout, int dzs,
                       float scale, bf16* dz, double* part, double* out, hipStream_t st) {
  const int nblk = (int)((npix + 255) / 256);
  hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(256), 0, st, y, t, mask, npix, cout, dzs, scale, dz, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, part, nblk, out);
  return hipGetLastError();
}

hipError_t adam_launch(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace tvnetk
