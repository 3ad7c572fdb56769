// tvnet_api.cpp -- the C ABI of include/tvnet.h: parameter and activation
// storage, the forward / backward / Adam schedule over the MFMA kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tvlbm.h"
#include "../../include/tvnet.h"

namespace tvnetk {
typedef __bf16 bf16;
struct ConvArgs {
  const bf16* x;
  const bf16* wk;
  const float* bias;
  const float* zprev;
  float* z;
  bf16* a;
  int B, H, W, cout, a_stride;
};
struct WgradArgs {
  const bf16* x;
  const bf16* dz;
  float* part;
  int B, H, W, cout, rows;
};
hipError_t conv_launch(int cin_p, int nt, int epi, const ConvArgs& A, hipStream_t st);
int wgrad_k9p(int cin_p);
hipError_t wgrad_launch(int cin_p, int dzs, int ot, const WgradArgs& A, int nblk, hipStream_t st);
hipError_t wgrad_reduce_launch(const float* part, int nblk, int rows_t, int k9p, int cin, int cin_p,
                               int cout, float* grad, hipStream_t st);
hipError_t prep_filter_launch(const float* w, int cout, int cin, int rows, int kp, int cin_p,
                              int transposed, bf16* wk, hipStream_t st);
hipError_t pack_input_launch(const float* x, int64_t npix, int cin, int cin_p, bf16* out, hipStream_t st);
hipError_t loss_launch(const float* y, const float* t, const float* mask, int64_t npix, int cout, int dzs,
                       float scale, bf16* dz, double* part, double* out, hipStream_t st);
hipError_t adam_launch(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
enum { EPI_GELU = 0, EPI_LINEAR = 1, EPI_BWD = 2 };
}  // namespace tvnetk

using namespace tvnetk;

namespace {
constexpr int kRowsPerWgrad = 8;
int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Layer {
  int cin, cout, cin_p;     // forward
  int nt, kp;               // forward GEMM: NT output tiles, padded K
  int64_t off;              // offset of W in the flat parameters (b follows)
  int bwd_cin_p, bwd_kp;    // transposed filter (backward data)
  int wg_dzs, wg_ot;        // backward weights
  bf16* wk_f = nullptr;
  bf16* wk_b = nullptr;
};
}  // namespace

struct tvnet {
  tvnet_desc d{};
  hipStream_t st = nullptr;
  Layer L[4];
  int64_t nparam = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  bf16 *x0 = nullptr, *a[3] = {nullptr, nullptr, nullptr};
  float* z[3] = {nullptr, nullptr, nullptr};
  float* y = nullptr;
  bf16* dz[4] = {nullptr, nullptr, nullptr, nullptr};
  float* wpart = nullptr;
  double* lpart = nullptr;
  double* lsum = nullptr;
  int last_batch = 0;
  std::string err;
};

#define NHIP(expr)                                        \
  do {                                                    \
    if ((expr) != hipSuccess) return TVLBM_EHIP;          \
  } while (0)

static int prep_filters(tvnet* n) {
  for (int l = 0; l < 4; ++l) {
    Layer& L = n->L[l];
    NHIP(prep_filter_launch(n->p + L.off, L.cout, L.cin, L.nt * 16, L.kp, L.cin_p, 0, L.wk_f, n->st));
    if (l > 0)
      NHIP(prep_filter_launch(n->p + L.off, L.cout, L.cin, 32, L.bwd_kp, L.bwd_cin_p, 1, L.wk_b, n->st));
  }
  return TVLBM_OK;
}

extern "C" {

int tvnet_destroy(tvnet* n) {
  if (!n) return TVLBM_EINVAL;
  if (n->st) hipStreamSynchronize(n->st); else hipDeviceSynchronize();
  hipFree(n->p); hipFree(n->g); hipFree(n->m); hipFree(n->v);
  hipFree(n->x0); hipFree(n->y); hipFree(n->wpart); hipFree(n->lpart); hipFree(n->lsum);
  for (int k = 0; k < 3; ++k) { hipFree(n->a[k]); hipFree(n->z[k]); }
  for (int k = 0; k < 4; ++k) { hipFree(n->dz[k]); hipFree(n->L[k].wk_f); hipFree(n->L[k].wk_b); }
  delete n;
  return TVLBM_OK;
}

int tvnet_init(const tvnet_desc* d, tvnet** out) {
  if (!d || !out) return TVLBM_EINVAL;
  if (d->c_in < 1 || d->c_in > 8 || d->c_out < 1 || d->c_out > 8 || d->width != 32 || d->height < 1 ||
      d->cols < 1 || d->cols > 256 || d->max_batch < 1)
    return TVLBM_EUNSUPPORTED;
  tvnet* n = new (std::nothrow) tvnet();
  if (!n) return TVLBM_ENOMEM;
  n->d = *d;
  n->st = (hipStream_t)d->stream;
  const int chans[5] = {d->c_in, 32, 32, 32, d->c_out};
  int64_t off = 0;
  for (int l = 0; l < 4; ++l) {
    Layer& L = n->L[l];
    L.cin = chans[l];
    L.cout = chans[l + 1];
    L.cin_p = l == 0 ? 8 : 32;
    L.nt = (L.cout + 15) / 16;
    L.kp = round_up(9 * L.cin_p, 32);
    L.off = off;
    off += (int64_t)L.cout * L.cin * 9 + L.cout;
    L.bwd_cin_p = l == 3 ? 8 : 32;
    L.bwd_kp = round_up(9 * L.bwd_cin_p, 32);
    L.wg_dzs = l == 3 ? 8 : 32;
    L.wg_ot = (L.cout + 15) / 16;
  }
  n->nparam = off;
  const int64_t npix = (int64_t)d->max_batch * d->height * d->cols;
  const int nblk_w = d->max_batch * ((d->height + kRowsPerWgrad - 1) / kRowsPerWgrad);
  size_t wpart = 0;
  for (int l = 0; l < 4; ++l)
    wpart = std::max(wpart, (size_t)nblk_w * n->L[l].wg_ot * 16 * (wgrad_k9p(n->L[l].cin_p) + 1));
  bool ok = hipMalloc(&n->p, 4 * off) == hipSuccess && hipMalloc(&n->g, 4 * off) == hipSuccess &&
            hipMalloc(&n->m, 4 * off) == hipSuccess && hipMalloc(&n->v, 4 * off) == hipSuccess &&
            hipMalloc(&n->x0, 2 * npix * 8) == hipSuccess && hipMalloc(&n->y, 4 * npix * d->c_out) == hipSuccess &&
            hipMalloc(&n->wpart, 4 * wpart) == hipSuccess &&
            hipMalloc(&n->lpart, 8 * ((npix + 255) / 256)) == hipSuccess && hipMalloc(&n->lsum, 8) == hipSuccess;
  for (int k = 0; k < 3 && ok; ++k)
    ok = hipMalloc(&n->a[k], 2 * npix * 32) == hipSuccess && hipMalloc(&n->z[k], 4 * npix * 32) == hipSuccess;
  for (int k = 0; k < 4 && ok; ++k) ok = hipMalloc(&n->dz[k], 2 * npix * (k == 3 ? 8 : 32)) == hipSuccess;
  for (int l = 0; l < 4 && ok; ++l) {
    ok = hipMalloc(&n->L[l].wk_f, 2 * (size_t)n->L[l].nt * 16 * n->L[l].kp) == hipSuccess;
    if (ok && l > 0) ok = hipMalloc(&n->L[l].wk_b, 2 * (size_t)32 * n->L[l].bwd_kp) == hipSuccess;
  }
  if (!ok) {
    tvnet_destroy(n);
    return TVLBM_ENOMEM;
  }
  std::vector<float> zero(off, 0.0f);
  if (hipMemcpy(n->p, zero.data(), 4 * off, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->m, zero.data(), 4 * off, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->v, zero.data(), 4 * off, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(n->g, zero.data(), 4 * off, hipMemcpyHostToDevice) != hipSuccess || prep_filters(n) != TVLBM_OK) {
    tvnet_destroy(n);
    return TVLBM_EHIP;
  }
  *out = n;
  return TVLBM_OK;
}

int tvnet_num_params(const tvnet* n, int64_t* np) {
  if (!n || !np) return TVLBM_EINVAL;
  *np = n->nparam;
  return TVLBM_OK;
}

int tvnet_set_params(tvnet* n, const float* params) {
  if (!n || !params) return TVLBM_EINVAL;
  std::vector<float> zero(n->nparam, 0.0f);
  NHIP(hipMemcpyAsync(n->p, params, 4 * n->nparam, hipMemcpyHostToDevice, n->st));
  NHIP(hipMemcpyAsync(n->m, zero.data(), 4 * n->nparam, hipMemcpyHostToDevice, n->st));
  NHIP(hipMemcpyAsync(n->v, zero.data(), 4 * n->nparam, hipMemcpyHostToDevice, n->st));
  int rc = prep_filters(n);
  NHIP(hipStreamSynchronize(n->st));
  return rc;
}

int tvnet_get_params(tvnet* n, float* params) {
  if (!n || !params) return TVLBM_EINVAL;
  NHIP(hipMemcpyAsync(params, n->p, 4 * n->nparam, hipMemcpyDeviceToHost, n->st));
  NHIP(hipStreamSynchronize(n->st));
  return TVLBM_OK;
}

int tvnet_get_grads(tvnet* n, float* grads) {
  if (!n || !grads) return TVLBM_EINVAL;
  NHIP(hipMemcpyAsync(grads, n->g, 4 * n->nparam, hipMemcpyDeviceToHost, n->st));
  NHIP(hipStreamSynchronize(n->st));
  return TVLBM_OK;
}

int tvnet_forward(tvnet* n, const void* x, void* yout, int32_t batch) {
  if (!n || !x || !yout || batch < 1 || batch > n->d.max_batch) return TVLBM_EINVAL;
  const int H = n->d.height, W = n->d.cols;
  const int64_t npix = (int64_t)batch * H * W;
  NHIP(pack_input_launch((const float*)x, npix, n->d.c_in, 8, n->x0, n->st));
  const bf16* in = n->x0;
  for (int l = 0; l < 4; ++l) {
    const Layer& L = n->L[l];
    ConvArgs A;
    std::memset(&A, 0, sizeof A);
    A.x = in;
    A.wk = L.wk_f;
    A.bias = n->p + L.off + (int64_t)L.cout * L.cin * 9;
    A.B = batch; A.H = H; A.W = W; A.cout = L.cout;
    if (l < 3) {
      A.z = n->z[l];
      A.a = n->a[l];
      A.a_stride = 32;
      NHIP(conv_launch(L.cin_p, L.nt, EPI_GELU, A, n->st));
      in = n->a[l];
    } else {
      A.z = n->y;
      NHIP(conv_launch(L.cin_p, L.nt, EPI_LINEAR, A, n->st));
    }
  }
  NHIP(hipMemcpyAsync(yout, n->y, 4 * npix * n->d.c_out, hipMemcpyDeviceToDevice, n->st));
  n->last_batch = batch;
  return TVLBM_OK;
}

int tvnet_backward(tvnet* n, const void* target, const void* mask, int32_t batch, double mask_sum,
                   double* loss) {
  if (!n || !target || !mask || batch != n->last_batch || !(mask_sum > 0.0)) return TVLBM_EINVAL;
  const int H = n->d.height, W = n->d.cols;
  const int64_t npix = (int64_t)batch * H * W;
  const float scale = (float)(1.0 / ((double)n->d.c_out * mask_sum));
  NHIP(loss_launch(n->y, (const float*)target, (const float*)mask, npix, n->d.c_out, 8, scale, n->dz[3],
                   n->lpart, n->lsum, n->st));
  const int nblk = batch * ((H + kRowsPerWgrad - 1) / kRowsPerWgrad);
  for (int l = 3; l >= 0; --l) {
    const Layer& L = n->L[l];
    WgradArgs G;
    std::memset(&G, 0, sizeof G);
    G.x = l == 0 ? n->x0 : n->a[l - 1];
    G.dz = n->dz[l];
    G.part = n->wpart;
    G.B = batch; G.H = H; G.W = W; G.cout = L.cout; G.rows = kRowsPerWgrad;
    NHIP(wgrad_launch(L.cin_p, L.wg_dzs, L.wg_ot, G, nblk, n->st));
    NHIP(wgrad_reduce_launch(n->wpart, nblk, L.wg_ot * 16, wgrad_k9p(L.cin_p), L.cin, L.cin_p, L.cout,
                             n->g + L.off, n->st));
    if (l > 0) {
      ConvArgs A;
      std::memset(&A, 0, sizeof A);
      A.x = n->dz[l];
      A.wk = L.wk_b;
      A.zprev = n->z[l - 1];
      A.a = n->dz[l - 1];
      A.B = batch; A.H = H; A.W = W; A.cout = L.cin; A.a_stride = 32;
      NHIP(conv_launch(L.bwd_cin_p, 2, EPI_BWD, A, n->st));
    }
  }
  double lh = 0.0;
  NHIP(hipMemcpyAsync(&lh, n->lsum, sizeof lh, hipMemcpyDeviceToHost, n->st));
  NHIP(hipStreamSynchronize(n->st));
  if (loss) *loss = lh * (double)scale;
  return TVLBM_OK;
}

int tvnet_adam_step(tvnet* n, float lr, float b1, float b2, float eps, int32_t t) {
  if (!n || t < 1) return TVLBM_EINVAL;
  const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
  NHIP(adam_launch(n->p, n->g, n->m, n->v, (int)n->nparam, lr, b1, b2, eps, c1, c2, n->st));
  return prep_filters(n);
}

}  // extern "C"
