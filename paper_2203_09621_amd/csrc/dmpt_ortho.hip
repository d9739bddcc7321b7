// Non-orthogonal bases (Sec. II.A): the inverse factor Z of the overlap O
// (Z^T O Z = I) by the cubically convergent recursion the paper gives,
//   X_n = Z_n^T O Z_n,   Z_{n+1} = Z_n (1.875 I - 1.25 X_n + 0.375 X_n^2),
// started from Z_0 = c I with c^2 = 1 / (Gershgorin bound of O), and the
// congruences Z A Z that take H0, H1 to the orthogonalised representation and
// the density matrices back (D = Z D_perp Z^T).  With Z_0 a multiple of I every
// iterate is a polynomial in O, so Z is the symmetric (Lowdin) factor O^{-1/2}
// and Z^T = Z.  All products run on the direct MFMA kernels (FP64 or FP32):
// single products C = A B with symmetric operands, stored either on the upper
// tiles and mirrored (symmetric C) or on every tile (general C).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <string>
#include <vector>

#include "layer_common.h"

namespace dmpt {

namespace {

// Z = c I on the N x N block, zero elsewhere (padded rows x ld storage).
template <typename M>
__global__ void __launch_bounds__(kBlk) k_scaled_identity(M* z, double c, int64_t n, int64_t total,
                                                         int64_t ld) {
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t i = q / ld, j = q - i * ld;
    z[q] = (M)((i == j && i < n) ? c : 0.0);
  }
}

// Q = a0 I + a1 X + a2 T on the N x N block (T = X^2), zero elsewhere.
template <typename M>
__global__ void __launch_bounds__(kBlk) k_poly2(const M* x, const M* t, M* q, int64_t n,
                                               int64_t total, int64_t ld) {
  const double a0 = 1.875, a1 = -1.25, a2 = 0.375;
  for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * kBlk) {
    const int64_t i = p / ld, j = p - i * ld;
    double v = 0.0;
    if (i < n && j < n) v = (i == j ? a0 : 0.0) + a1 * (double)x[p] + a2 * (double)t[p];
    q[p] = (M)v;
  }
}

// ||X - I||_F^2 partials over the N x N block (FP64, fixed grid).
template <typename M>
__global__ void __launch_bounds__(kBlk) k_dev_identity(const M* x, int64_t n, int64_t ld,
                                                      double* part) {
  double v = 0.0;
  const int64_t total = n * n;
  for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * kBlk) {
    const int64_t i = p / n, j = p - i * n;
    const double d = (double)x[i * ld + j] - (i == j ? 1.0 : 0.0);
    v += d * d;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_sum_partials(const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int i = 0; i < nb; ++i) v += part[i];
  *out = v;
}

dmpt_status ofail(dmpt_status s, const std::string& m) {
  set_last_error(m.c_str());
  return s;
}

// Workspace of the single products: padded matrices and the two item lists.
struct ProductWork {
  dmpt_precision prec;
  int64_t n = 0, np = 0, ld = 0;
  size_t eb = 0;
  std::vector<void*> allocs;
  TileItem* items_sym = nullptr;
  TileItem* items_all = nullptr;
  int n_sym = 0, n_all = 0;
  double* part = nullptr;
  double* dscal = nullptr;

  hipError_t get(void** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
  hipError_t matrix(void** p) {
    hipError_t e = get(p, (size_t)np * ld * eb);
    if (e == hipSuccess) e = hipMemset(*p, 0, (size_t)np * ld * eb);
    return e;
  }
  hipError_t init(dmpt_precision pr, int64_t nn) {
    prec = pr;
    n = nn;
    const int tile = product_tile(prec);
    np = (n + tile - 1) / tile * tile;
    ld = np;
    eb = prec == DMPT_FP64 ? 8 : 4;
    const int T = (int)(np / tile);
    n_sym = T * (T + 1) / 2;
    n_all = T * T;
    std::vector<TileItem> sym(n_sym), all(n_all);
    product_items(T, 1, sym.data());
    product_items(T, 2, all.data());
    hipError_t e = get((void**)&items_sym, sym.size() * sizeof(TileItem));
    if (e == hipSuccess) e = get((void**)&items_all, all.size() * sizeof(TileItem));
    if (e == hipSuccess)
      e = hipMemcpy(items_sym, sym.data(), sym.size() * sizeof(TileItem), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(items_all, all.data(), all.size() * sizeof(TileItem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = get((void**)&part, 3 * 512 * sizeof(double));
    if (e == hipSuccess) e = get((void**)&dscal, 16 * sizeof(double));
    return e;
  }
  // C = A B (A, B symmetric); symmetric C on mirrored upper tiles, else every tile
  hipError_t product(const void* A, const void* B, void* C, bool symmetric, hipStream_t s) {
    ProductArgs a;
    memset(&a, 0, sizeof(a));
    a.s_hi = A;
    a.s1_hi[0] = B;
    a.x = C;
    a.items = symmetric ? items_sym : items_all;
    a.n_items = symmetric ? n_sym : n_all;
    a.ld = ld;
    a.kdim = np;
    a.mode = symmetric ? 1 : 2;
    return launch_products(prec, a, s);
  }
  ~ProductWork() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

bool direct_precision(int32_t p) { return p == DMPT_FP64 || p == DMPT_FP32; }

}  // namespace

}  // namespace dmpt

using namespace dmpt;

extern "C" {

dmpt_status dmpt_inverse_factor(int32_t precision, const double* O, int64_t N, double* Z,
                                int32_t max_iter, double tol, int32_t* iters, double* err,
                                void* stream) {
  if (!O || !Z || N < 1 || N > (1 << 17) || max_iter < 1 || !(tol > 0.0))
    return ofail(DMPT_EINVAL, "bad arguments");
  if (!direct_precision(precision))
    return ofail(DMPT_ENOTSUP, "the inverse factor runs in DMPT_FP64 or DMPT_FP32");
  hipStream_t s = (hipStream_t)stream;
  const dmpt_precision prec = (dmpt_precision)precision;
  ProductWork w;
  void *om = nullptr, *z = nullptr, *y = nullptr, *x = nullptr, *t = nullptr, *q = nullptr;
  hipError_t e = w.init(prec, N);
  for (void** p : {&om, &z, &y, &x, &t, &q})
    if (e == hipSuccess) e = w.matrix(p);
  if (e != hipSuccess)
    return ofail(e == hipErrorOutOfMemory ? DMPT_ENOMEM : DMPT_EHIP, "workspace allocation failed");
  const int64_t total = w.np * w.ld;
  double eps[2] = {0.0, 0.0};
  e = launch_gershgorin(O, N, w.part, nullptr, w.dscal, s);
  if (e == hipSuccess) e = hipMemcpyAsync(eps, w.dscal, sizeof(eps), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ofail(DMPT_EHIP, hipGetErrorString(e));
  if (!(eps[1] > 0.0) || !isfinite(eps[1]))
    return ofail(DMPT_ENONFINITE, "overlap matrix without a positive spectral bound");
  e = launch_from_f64(prec, O, N, w.np, w.ld, 0, 0, om, nullptr, nullptr, s);
  if (e != hipSuccess) return ofail(DMPT_EHIP, hipGetErrorString(e));
  const double c = 1.0 / sqrt(eps[1]);
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_scaled_identity<double>, dim3(2048), dim3(kBlk), 0, s, (double*)z, c, N,
                       total, w.ld);
  else
    hipLaunchKernelGGL(k_scaled_identity<float>, dim3(2048), dim3(kBlk), 0, s, (float*)z, c, N,
                       total, w.ld);
  int it = 0;
  double r = INFINITY;
  for (;; ++it) {
    // X = Z O Z (Y = Z O, general; X = Y Z, symmetric)
    e = w.product(z, om, y, false, s);
    if (e == hipSuccess) e = w.product(y, z, x, true, s);
    if (e != hipSuccess) break;
    if (prec == DMPT_FP64)
      hipLaunchKernelGGL(k_dev_identity<double>, dim3(512), dim3(kBlk), 0, s, (const double*)x, N,
                         w.ld, w.part);
    else
      hipLaunchKernelGGL(k_dev_identity<float>, dim3(512), dim3(kBlk), 0, s, (const float*)x, N,
                         w.ld, w.part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kWave), 0, s, w.part, 512, w.dscal);
    double r2 = 0.0;
    e = hipMemcpyAsync(&r2, w.dscal, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    r = sqrt(r2);
    if (!isfinite(r)) {
      e = hipSuccess;
      break;
    }
    if (r < tol || it >= max_iter) break;
    // Z <- Z (a0 I + a1 X + a2 X^2)
    e = w.product(x, x, t, true, s);
    if (e != hipSuccess) break;
    if (prec == DMPT_FP64)
      hipLaunchKernelGGL(k_poly2<double>, dim3(2048), dim3(kBlk), 0, s, (const double*)x,
                         (const double*)t, (double*)q, N, total, w.ld);
    else
      hipLaunchKernelGGL(k_poly2<float>, dim3(2048), dim3(kBlk), 0, s, (const float*)x,
                         (const float*)t, (float*)q, N, total, w.ld);
    e = w.product(z, q, y, true, s);
    if (e != hipSuccess) break;
    std::swap(z, y);
  }
  if (e != hipSuccess) return ofail(DMPT_EHIP, hipGetErrorString(e));
  e = launch_copy_plain(prec, z, w.ld, Z, N, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ofail(DMPT_EHIP, hipGetErrorString(e));
  if (iters) *iters = it;
  if (err) *err = r;
  if (!isfinite(r)) return ofail(DMPT_ENONFINITE, "inverse factor iteration diverged");
  if (!(r < tol)) return ofail(DMPT_ENOCONV, "inverse factor: tolerance not reached");
  return DMPT_OK;
}

dmpt_status dmpt_congruence(int32_t precision, int64_t N, const double* Z, const double* A,
                            double* out, void* stream) {
  if (!Z || !A || !out || N < 1 || N > (1 << 17)) return ofail(DMPT_EINVAL, "bad arguments");
  if (!direct_precision(precision))
    return ofail(DMPT_ENOTSUP, "congruences run in DMPT_FP64 or DMPT_FP32");
  hipStream_t s = (hipStream_t)stream;
  const dmpt_precision prec = (dmpt_precision)precision;
  ProductWork w;
  void *zm = nullptr, *am = nullptr, *y = nullptr, *r = nullptr;
  hipError_t e = w.init(prec, N);
  for (void** p : {&zm, &am, &y, &r})
    if (e == hipSuccess) e = w.matrix(p);
  if (e != hipSuccess)
    return ofail(e == hipErrorOutOfMemory ? DMPT_ENOMEM : DMPT_EHIP, "workspace allocation failed");
  e = launch_from_f64(prec, Z, N, w.np, w.ld, 0, 0, zm, nullptr, nullptr, s);
  if (e == hipSuccess) e = launch_from_f64(prec, A, N, w.np, w.ld, 0, 0, am, nullptr, nullptr, s);
  if (e == hipSuccess) e = w.product(zm, am, y, false, s);    // Y = Z A
  if (e == hipSuccess) e = w.product(y, zm, r, true, s);      // Z A Z
  if (e == hipSuccess) e = launch_copy_plain(prec, r, w.ld, out, N, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DMPT_OK : ofail(DMPT_EHIP, hipGetErrorString(e));
}

}  // extern "C"
