// Normalisation layer, per-layer decisions, fused update/split/norm and output
// kernels of the DNN-SP2-PT network.
//
// Every reduction is deterministic: a fixed grid, per-block partial sums in
// FP64 combined in a fixed order by a single-workgroup kernel.  No floating
// point atomics.
#include <math.h>

#include "dmpt_internal.h"

namespace dmpt {

constexpr int kBlk = 256;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// Block-wide reductions for kBlk threads; the result is valid in every thread.
__device__ double block_sum(double v) {
  __shared__ double sh[kBlk / kWave];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kBlk / kWave; ++i) r += sh[i];
  return r;
}
__device__ double block_max(double v) {
  __shared__ double sh[kBlk / kWave];
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < kBlk / kWave; ++i) r = fmax(r, sh[i]);
  return r;
}
__device__ double block_min(double v) {
  __shared__ double sh[kBlk / kWave];
  v = wave_min(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < kBlk / kWave; ++i) r = fmin(r, sh[i]);
  return r;
}

// Split scale: choose e with max|Y| 2^e in [1/16, 1/8), leaving room for the
// growth of one layer before the next choice.
__device__ __forceinline__ int split_exponent(double m) {
  if (!(m > 0.0) || !isfinite(m)) return 0;
  return -ilogb(m) - 4;
}

template <typename T16> struct Conv;
template <> struct Conv<_Float16> {
  static __device__ __forceinline__ uint16_t to(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  static __device__ __forceinline__ float from(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
};
template <> struct Conv<__bf16> {
  static __device__ __forceinline__ uint16_t to(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  static __device__ __forceinline__ float from(uint16_t b) { return (float)__builtin_bit_cast(__bf16, b); }
};

// hi = RN16(v 2^e), lo = RN16((v 2^e - hi) 2^t); the difference is exact.
template <typename T16>
__device__ __forceinline__ void split_one(float v, int e, int t, uint16_t* hi, uint16_t* lo) {
  const float xs = ldexpf(v, e);
  const uint16_t h = Conv<T16>::to(xs);
  *hi = h;
  *lo = Conv<T16>::to(ldexpf(xs - Conv<T16>::from(h), t));
}

// ------------------------------------------------------------------ Gershgorin
// One wave per row: r_i = sum_{j != i} |H_ij|, lo_i = H_ii - r_i, hi_i = H_ii + r_i.
__global__ void __launch_bounds__(kBlk) k_gersh_rows(const double* H, int64_t n, double* part) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t)blockIdx.x * (kBlk / kWave) + threadIdx.x / kWave;
  const int64_t nw = (int64_t)gridDim.x * (kBlk / kWave);
  double lo = INFINITY, hi = -INFINITY, tr = 0.0;
  for (int64_t i = w; i < n; i += nw) {
    const double* row = H + i * n;
    double r = 0.0;
    for (int64_t j = lane; j < n; j += kWave) r += (j == i) ? 0.0 : fabs(row[j]);
    r = wave_sum(r);
    const double d = row[i];
    lo = fmin(lo, d - r);
    hi = fmax(hi, d + r);
    tr += (lane == 0) ? d : 0.0;
  }
  lo = block_min(lo);
  hi = block_max(hi);
  tr = block_sum(tr);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = lo;
    part[gridDim.x + blockIdx.x] = hi;
    part[2 * gridDim.x + blockIdx.x] = tr;
  }
}

// eps_1, eps_N, and N_S = Tr S0 = (N eps_N - Tr H0)/(eps_N - eps_1) into the state.
__global__ void __launch_bounds__(kBlk) k_gersh_final(const double* part, int nb, int64_t n,
                                                     LayerState* st, double* eps_out) {
  double lo = INFINITY, hi = -INFINITY, tr = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlk) {
    lo = fmin(lo, part[i]);
    hi = fmax(hi, part[nb + i]);
  }
  // the trace partials are combined in block order by one thread (fixed order)
  lo = block_min(lo);
  hi = block_max(hi);
  if (threadIdx.x == 0) {
    for (int i = 0; i < nb; ++i) tr += part[2 * nb + i];
    if (eps_out) { eps_out[0] = lo; eps_out[1] = hi; }
    if (st) {
      st->eps1 = lo;
      st->epsN = hi;
      const double w = hi - lo;
      st->n_s0 = ((double)n * hi - tr) / w;
      if (!(w > 0.0) || !isfinite(w)) st->error = DMPT_ENONFINITE;
    }
  }
}

constexpr int kGershBlocks = 512;

hipError_t launch_gershgorin(const double* H, int64_t n, double* part, LayerState* st,
                             double* eps_out, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_rows, dim3(kGershBlocks), dim3(kBlk), 0, s, H, n, part);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(kBlk), 0, s, part, kGershBlocks, n, st, eps_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ input checks
__global__ void __launch_bounds__(kBlk) k_symcheck(const double* H, int64_t n, int32_t* flag) {
  const int64_t total = n * n;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t i = q / n, j = q - i * n;
    if (j > i && H[q] != H[j * n + i]) *flag = 1;
    if (!isfinite(H[q])) *flag = 2;
  }
}

hipError_t launch_symcheck(const double* H, int64_t n, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_symcheck, dim3(2048), dim3(kBlk), 0, s, H, n, flag);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlk) k_maxabs(const double* H, int64_t total, double* part) {
  double m = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const double v = fabs(H[q]);
    m = (v > m || v != v) ? v : m;   // keeps a NaN
  }
  m = block_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

hipError_t launch_maxabs(const double* H, int64_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_maxabs, dim3(kRedBlocks), dim3(kBlk), 0, s, H, n * n, part);
  return hipGetLastError();
}

// ------------------------------------------------------------------ normalisation layer
// S0 = (eps_N I - H0)/(eps_N - eps_1) in FP64, stored in the layer precision
// into a padded Np x Np matrix (padding is zero and stays zero: a zero
// eigenvalue is a fixed point of both x^2 and 2x - x^2).
template <typename M>
__global__ void __launch_bounds__(kBlk) k_init_s0(const double* H0, int64_t n, int64_t rows,
                                                 int64_t ld, const LayerState* st, M* s_init) {
  const double en = st->epsN, w = st->epsN - st->eps1;
  const int64_t total = rows * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t i = q / ld, j = q - i * ld;
    double v = 0.0;
    if (i < n && j < n) v = ((i == j ? en : 0.0) - H0[i * n + j]) / w;
    s_init[q] = (M)v;
  }
}

hipError_t launch_init_s0(dmpt_precision prec, const double* H0, int64_t n, int64_t rows,
                          int64_t ld, const LayerState* st, void* s_init, hipStream_t s) {
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_init_s0<double>, dim3(4096), dim3(kBlk), 0, s, H0, n, rows, ld, st,
                       (double*)s_init);
  else
    hipLaunchKernelGGL(k_init_s0<float>, dim3(4096), dim3(kBlk), 0, s, H0, n, rows, ld, st,
                       (float*)s_init);
  return hipGetLastError();
}

// master <- src (layer precision); split forms also write hi/lo with scale 2^e.
template <typename M, typename T16, bool SPLIT>
__global__ void __launch_bounds__(kBlk) k_load(const M* src, M* master, uint16_t* hi, uint16_t* lo,
                                              int64_t total, int64_t ld, int64_t kdim, int e,
                                              int t) {
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const M v = src[q];
    master[q] = v;
    if constexpr (SPLIT) {
      const int64_t r = q / ld, c = q - r * ld;
      if (c < kdim) {
        const int64_t pi = panel_index(r, c, kdim);
        split_one<T16>((float)v, e, t, hi + pi, lo + pi);
      }
    }
  }
}

hipError_t launch_load_s0(dmpt_precision prec, const void* s_init, void* master, void* hi, void* lo,
                          int64_t rows, int64_t ld, int t, hipStream_t s) {
  const int64_t total = rows * ld;
  switch (prec) {
    case DMPT_FP64:
      hipLaunchKernelGGL((k_load<double, _Float16, false>), dim3(4096), dim3(kBlk), 0, s,
                         (const double*)s_init, (double*)master, nullptr, nullptr, total, ld, rows,
                         0, 0);
      break;
    case DMPT_FP32:
      hipLaunchKernelGGL((k_load<float, _Float16, false>), dim3(4096), dim3(kBlk), 0, s,
                         (const float*)s_init, (float*)master, nullptr, nullptr, total, ld, rows,
                         0, 0);
      break;
    case DMPT_SPLIT_FP16:
      hipLaunchKernelGGL((k_load<float, _Float16, true>), dim3(4096), dim3(kBlk), 0, s,
                         (const float*)s_init, (float*)master, (uint16_t*)hi, (uint16_t*)lo, total,
                         ld, rows, 0, t);
      break;
    case DMPT_SPLIT_BF16:
      hipLaunchKernelGGL((k_load<float, __bf16, true>), dim3(4096), dim3(kBlk), 0, s,
                         (const float*)s_init, (float*)master, (uint16_t*)hi, (uint16_t*)lo, total,
                         ld, rows, 0, t);
      break;
  }
  return hipGetLastError();
}

// First-order input layer S1_0 = -H1/(eps_N - eps_1) (Sec. III.A expansion of
// the normalisation).  Step 1: split scale from max|H1|.
__global__ void __launch_bounds__(kBlk) k_s1_setup(const double* part, int nb, LayerState* st,
                                                  int j, int use_state_eps, double w_fixed) {
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlk) m = (part[i] > m || part[i] != part[i]) ? part[i] : m;
  m = block_max(m);
  if (threadIdx.x == 0) {
    const double w = use_state_eps ? st->epsN - st->eps1 : w_fixed;
    const double mx = m / w;
    if (!isfinite(mx)) st->error = DMPT_ENONFINITE;
    const int e = split_exponent(mx);
    st->s1_exp_split[j] = e;
    st->s1_exp_next[j] = e;
    st->s1_exp_hist[j][0] = e;
    st->s1_max[j] = mx;
  }
}

// Step 2: S1_0 (padded) in the layer precision, split with the state's scale.
template <typename M, typename T16, bool SPLIT>
__global__ void __launch_bounds__(kBlk) k_init_s1(const double* H1, int64_t n, int64_t rows,
                                                 int64_t ld, const LayerState* st, int j,
                                                 double w_fixed, int use_state_eps, M* s1,
                                                 uint16_t* hi, uint16_t* lo, int t) {
  const double w = use_state_eps ? st->epsN - st->eps1 : w_fixed;
  const int e = st->s1_exp_split[j];
  const int64_t total = rows * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t r = q / ld, c = q - r * ld;
    double v = 0.0;
    if (r < n && c < n) v = -H1[r * n + c] / w;
    const M mv = (M)v;
    s1[q] = mv;
    if constexpr (SPLIT) {
      if (c < rows) {
        const int64_t pi = panel_index(r, c, rows);
        split_one<T16>((float)mv, e, t, hi + pi, lo + pi);
      }
    }
  }
}

hipError_t launch_init_s1(dmpt_precision prec, const double* H1, int64_t n, int64_t rows,
                          int64_t ld, LayerState* st, int j, double* part, void* s1, void* hi,
                          void* lo, int t, double w_fixed, hipStream_t s) {
  const int use_state = w_fixed > 0.0 ? 0 : 1;
  hipLaunchKernelGGL(k_maxabs, dim3(kRedBlocks), dim3(kBlk), 0, s, H1, n * n, part);
  hipLaunchKernelGGL(k_s1_setup, dim3(1), dim3(kBlk), 0, s, part, kRedBlocks, st, j, use_state,
                     w_fixed);
  switch (prec) {
    case DMPT_FP64:
      hipLaunchKernelGGL((k_init_s1<double, _Float16, false>), dim3(4096), dim3(kBlk), 0, s, H1, n,
                         rows, ld, st, j, w_fixed, use_state, (double*)s1, nullptr, nullptr, t);
      break;
    case DMPT_FP32:
      hipLaunchKernelGGL((k_init_s1<float, _Float16, false>), dim3(4096), dim3(kBlk), 0, s, H1, n,
                         rows, ld, st, j, w_fixed, use_state, (float*)s1, nullptr, nullptr, t);
      break;
    case DMPT_SPLIT_FP16:
      hipLaunchKernelGGL((k_init_s1<float, _Float16, true>), dim3(4096), dim3(kBlk), 0, s, H1, n,
                         rows, ld, st, j, w_fixed, use_state, (float*)s1, (uint16_t*)hi, (uint16_t*)lo, t);
      break;
    case DMPT_SPLIT_BF16:
      hipLaunchKernelGGL((k_init_s1<float, __bf16, true>), dim3(4096), dim3(kBlk), 0, s, H1, n, rows, ld,
                         st, j, w_fixed, use_state, (float*)s1, (uint16_t*)hi, (uint16_t*)lo, t);
      break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ state reset
__global__ void k_reset_state(LayerState* st, int k, int max_layers, double nocc, int64_t n) {
  // one thread: a few hundred words
  if (threadIdx.x != 0) return;
  st->n_real = (int32_t)n;
  st->k = k;
  st->max_layers = max_layers;
  st->nocc = nocc;
  st->n = 0;
  st->done = 0;
  st->error = 0;
  st->converged = 0;
  st->d0 = 0;
  st->d0_layer = 0;
  st->x_computed = 0;
  st->upd_s0 = 0;
  st->d0_now = 0;
  st->sigma_cur = 0;
  st->n_s = st->n_s0;
  st->fro0 = 0.0;
  for (int i = 0; i <= kMaxLayers; ++i) {
    st->sigma[i] = 0;
    st->iderr[i] = 0.0;
  }
  for (int j = 0; j < kMaxK; ++j) {
    st->d1[j] = j < k ? 0 : 1;
    st->d1_layer[j] = 0;
    for (int i = 0; i <= kMaxLayers; ++i) st->fro1[j][i] = 0.0;
  }
}

hipError_t launch_reset_state(LayerState* st, int k, int max_layers, double nocc, int64_t n,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(kWave), 0, s, st, k, max_layers, nocc, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ decisions, part 1
// Algorithm 1 trace test and Algorithm 2: N_X = Tr X in FP64, IdErr, sigma,
// the D0 test and the N_S update.  After D0 converged: sigma flips.
template <typename M>
__global__ void __launch_bounds__(kBlk) k_decide0(LayerState* st, const M* x, int64_t ld) {
  const int done = st->done;
  if (done) return;
  const int d0 = st->d0;
  const int n_real = st->n_real;
  double nx = 0.0;
  if (!d0) {
    for (int i = threadIdx.x; i < n_real; i += kBlk) nx += (double)x[(int64_t)i * ld + i];
    nx = block_sum(nx);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int n = st->n + 1;
  st->n = n;
  int sig;
  if (!d0) {
    st->x_computed = 1;
    if (!isfinite(nx)) {
      st->error = DMPT_ENONFINITE;
      st->done = 1;
      return;
    }
    const double ns = st->n_s, nocc = st->nocc;
    const double iderr = ns - nx;
    const double a = fabs(2.0 * ns - nx - nocc), b = fabs(nx - nocc);
    sig = a > b ? 1 : -1;
    st->iderr[n] = iderr;
    const bool conv = iderr <= 0.0 ||
                      (n > 2 && st->sigma[n - 1] != st->sigma[n - 2] &&
                       iderr > 4.5 * st->iderr[n - 2] * st->iderr[n - 2]);
    if (conv) {
      st->d0 = 1;
      st->d0_layer = n;
      st->d0_now = 1;
      st->upd_s0 = 0;
      if (n > 1) sig = -st->sigma[n - 1];
    } else {
      st->d0_now = 0;
      st->upd_s0 = 1;
      st->n_s = sig * nx + (1 - sig) * ns;
    }
  } else {
    st->x_computed = 0;
    st->upd_s0 = 0;
    st->d0_now = 0;
    sig = -st->sigma[n - 1];
  }
  st->sigma[n] = sig;
  st->sigma_cur = sig;
}

hipError_t launch_decide0(dmpt_precision prec, LayerState* st, const void* x, int64_t ld,
                          hipStream_t s) {
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_decide0<double>, dim3(1), dim3(kBlk), 0, s, st, (const double*)x, ld);
  else
    hipLaunchKernelGGL(k_decide0<float>, dim3(1), dim3(kBlk), 0, s, st, (const float*)x, ld);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fused layer update
// dst = sigma X + (1 - sigma) S_old (Eqs. LinTransf / S_n detailed with the
// bias of Eq. dB), the 16-bit split of dst, and FP64 partial sums of
// ||S_old - X||_F^2 (the FroErr norms of Algorithms 2-3) and max|dst|.
// which < 0: zeroth order (in place, dst == S_old); which = j: response j
// (dst == X1_j, the previous S1_j stays intact in the other buffer).
template <typename M, typename T16, bool SPLIT>
__global__ void __launch_bounds__(kBlk) k_update(const LayerState* st, int which, const M* x,
                                                const M* s_old, M* dst, uint16_t* hi,
                                                uint16_t* lo, int64_t total, int64_t ld,
                                                int64_t kdim, int t, double* pfro, double* pmax) {
  if (st->done) return;
  const int sig = st->sigma_cur;
  bool active, want_fro;
  int e = 0;
  if (which < 0) {
    active = st->upd_s0;
    want_fro = st->x_computed;
  } else {
    active = !st->d1[which];
    want_fro = active && st->d0;
    e = st->s1_exp_next[which];
  }
  if (!active && !want_fro) return;
  double fro = 0.0, mx = 0.0;
  typedef M V4 __attribute__((ext_vector_type(4)));
  const int64_t n4 = total / 4;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < n4;
       q += (int64_t)gridDim.x * kBlk) {
    const V4 xv = ((const V4*)x)[q];
    const V4 sv = ((const V4*)s_old)[q];
    if (want_fro) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double d = (double)sv[r] - (double)xv[r];
        fro += d * d;
      }
    }
    if (active) {
      V4 nv;
#pragma unroll
      for (int r = 0; r < 4; ++r) nv[r] = sig > 0 ? xv[r] : (M)2 * sv[r] - xv[r];
      ((V4*)dst)[q] = nv;
#pragma unroll
      for (int r = 0; r < 4; ++r) mx = fmax(mx, fabs((double)nv[r]));
      if constexpr (SPLIT) {
        // four consecutive columns of one row (ld % 4 == 0) stay inside one panel block
        const int64_t row = (4 * q) / ld, col = 4 * q - row * ld;
        if (col < kdim) {
          uint16_t h[4], l[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) split_one<T16>((float)nv[r], e, t, h + r, l + r);
          typedef uint16_t U4 __attribute__((ext_vector_type(4)));
          const int64_t pi = panel_index(row, col, kdim) / 4;
          ((U4*)hi)[pi] = U4{h[0], h[1], h[2], h[3]};
          ((U4*)lo)[pi] = U4{l[0], l[1], l[2], l[3]};
        }
      }
    }
  }
  fro = block_sum(fro);
  mx = block_max(mx);
  if (threadIdx.x == 0) {
    pfro[blockIdx.x] = fro;
    if (pmax) pmax[blockIdx.x] = mx;
  }
}

hipError_t launch_update(dmpt_precision prec, const LayerState* st, int which, const void* x,
                         const void* s_old, void* dst, void* hi, void* lo, int64_t rows,
                         int64_t ld, int t, double* pfro, double* pmax, hipStream_t s) {
  const int64_t total = rows * ld;
  switch (prec) {
    case DMPT_FP64:
      hipLaunchKernelGGL((k_update<double, _Float16, false>), dim3(kRedBlocks), dim3(kBlk), 0, s, st,
                         which, (const double*)x, (const double*)s_old, (double*)dst, nullptr,
                         nullptr, total, ld, rows, t, pfro, pmax);
      break;
    case DMPT_FP32:
      hipLaunchKernelGGL((k_update<float, _Float16, false>), dim3(kRedBlocks), dim3(kBlk), 0, s, st,
                         which, (const float*)x, (const float*)s_old, (float*)dst, nullptr, nullptr,
                         total, ld, rows, t, pfro, pmax);
      break;
    case DMPT_SPLIT_FP16:
      hipLaunchKernelGGL((k_update<float, _Float16, true>), dim3(kRedBlocks), dim3(kBlk), 0, s, st,
                         which, (const float*)x, (const float*)s_old, (float*)dst, (uint16_t*)hi,
                         (uint16_t*)lo, total, ld, rows, t, pfro, pmax);
      break;
    case DMPT_SPLIT_BF16:
      hipLaunchKernelGGL((k_update<float, __bf16, true>), dim3(kRedBlocks), dim3(kBlk), 0, s, st,
                         which, (const float*)x, (const float*)s_old, (float*)dst, (uint16_t*)hi,
                         (uint16_t*)lo, total, ld, rows, t, pfro, pmax);
      break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ decisions, part 2
// FroErr^(0) at the D0 layer, FroErr^(1)_n per response, the parameter-free
// D1 test (Eq. ConvCrit, Algorithm 3, C_pt = 9), the next split scales, and
// the stop flag.
__global__ void __launch_bounds__(kBlk) k_decide1(LayerState* st, const double* pfro0,
                                                 const double* pfro1, const double* pmax1,
                                                 int split, int lo_shift) {
  if (st->done) return;
  const int k = st->k;
  const int d0_now = st->d0_now, d0 = st->d0;
  __shared__ double res[2 * kMaxK + 1];
  // sums in a fixed order: each thread a fixed strided subset, then the block tree
  if (d0_now) {
    double v = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kBlk) v += pfro0[i];
    v = block_sum(v);
    if (threadIdx.x == 0) res[2 * kMaxK] = v;
  }
  for (int j = 0; j < k; ++j) {
    if (st->d1[j]) continue;
    double v = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kBlk) {
      if (d0) v += pfro1[j * kRedBlocks + i];
      m = fmax(m, pmax1[j * kRedBlocks + i]);
    }
    v = block_sum(v);
    m = block_max(m);
    if (threadIdx.x == 0) {
      res[2 * j] = v;
      res[2 * j + 1] = m;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int n = st->n;
  if (d0_now) {
    st->fro0 = sqrt(res[2 * kMaxK]);
    if (!isfinite(st->fro0)) st->error = DMPT_ENONFINITE;
  }
  int all = 1;
  for (int j = 0; j < k; ++j) {
    if (st->d1[j]) continue;
    const double mx = res[2 * j + 1];
    // the split written this layer used s1_exp_next; check it stayed in range
    if (split && ldexp(mx, st->s1_exp_next[j] + lo_shift) > 32768.0) st->error = DMPT_ENONFINITE;
    if (!isfinite(mx)) st->error = DMPT_ENONFINITE;
    if (d0) {
      const double f = sqrt(res[2 * j]);
      st->fro1[j][n] = f;
      if (!isfinite(f)) st->error = DMPT_ENONFINITE;
      if (n - 2 >= st->d0_layer) {
        const double prev = st->fro1[j][n - 2];
        if (f > 9.0 * st->fro0 * prev || f == 0.0) {
          st->d1[j] = 1;
          st->d1_layer[j] = n;
        }
      }
    }
    st->s1_exp_hist[j][n] = st->s1_exp_next[j];   // the scale S1_n was just split with
    st->s1_exp_split[j] = st->s1_exp_next[j];
    st->s1_exp_next[j] = split_exponent(mx);
    st->s1_max[j] = mx;
    if (!st->d1[j]) all = 0;
  }
  if (all) {
    st->converged = 1;
    st->done = 1;
  } else if (n >= st->max_layers) {
    st->done = 1;
  }
  if (st->error) st->done = 1;
}

hipError_t launch_decide1(LayerState* st, const double* pfro0, const double* pfro1,
                          const double* pmax1, int split, int lo_shift, hipStream_t s) {
  hipLaunchKernelGGL(k_decide1, dim3(1), dim3(kBlk), 0, s, st, pfro0, pfro1, pmax1, split, lo_shift);
  return hipGetLastError();
}

// ------------------------------------------------------------------ outputs
// P (FP64, N x N) <- src (layer precision, padded).  For a response the
// source buffer follows the D1 layer: S1 of layer d1_layer - 1 sits in
// buffer (d1_layer - 1) & 1; without convergence the last layer's buffer.
template <typename M>
__global__ void __launch_bounds__(kBlk) k_copy_out(const LayerState* st, int which, const M* b0,
                                                  const M* b1, int64_t ld, double* dst, int64_t n) {
  const M* src = b0;
  if (which >= 0) {
    const int L = st->d1[which] && st->d1_layer[which] > 0 ? st->d1_layer[which] - 1 : st->n;
    src = (L & 1) ? b1 : b0;
  }
  const int64_t total = n * n;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t i = q / n, j = q - i * n;
    dst[q] = (double)src[i * ld + j];
  }
}

hipError_t launch_copy_out(dmpt_precision prec, const LayerState* st, int which, const void* b0,
                           const void* b1, int64_t ld, double* dst, int64_t n, hipStream_t s) {
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_copy_out<double>, dim3(4096), dim3(kBlk), 0, s, st, which,
                       (const double*)b0, (const double*)b1, ld, dst, n);
  else
    hipLaunchKernelGGL(k_copy_out<float>, dim3(4096), dim3(kBlk), 0, s, st, which, (const float*)b0,
                       (const float*)b1, ld, dst, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlk) k_trace(const double* P, int64_t n, double* out) {
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlk) v += P[i * n + i];
  v = block_sum(v);
  if (threadIdx.x == 0) *out = v;
}

hipError_t launch_trace(const double* P, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(kBlk), 0, s, P, n, out);
  return hipGetLastError();
}

// A (FP64 N x N) -> padded layer-precision master (+ split with scale 2^e).
template <typename M, typename T16, bool SPLIT>
__global__ void __launch_bounds__(kBlk) k_from_f64(const double* A, int64_t n, int64_t rows,
                                                  int64_t ld, int e, int t, M* master,
                                                  uint16_t* hi, uint16_t* lo) {
  const int64_t total = rows * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const int64_t i = q / ld, j = q - i * ld;
    const M v = (i < n && j < n) ? (M)A[i * n + j] : (M)0;
    master[q] = v;
    if constexpr (SPLIT) {
      if (j < rows) {
        const int64_t pi = panel_index(i, j, rows);
        split_one<T16>((float)v, e, t, hi + pi, lo + pi);
      }
    }
  }
}

hipError_t launch_from_f64(dmpt_precision prec, const double* A, int64_t n, int64_t rows,
                           int64_t ld, int e, int t, void* master, void* hi, void* lo,
                           hipStream_t s) {
  switch (prec) {
    case DMPT_FP64:
      hipLaunchKernelGGL((k_from_f64<double, _Float16, false>), dim3(4096), dim3(kBlk), 0, s, A, n,
                         rows, ld, e, t, (double*)master, nullptr, nullptr);
      break;
    case DMPT_FP32:
      hipLaunchKernelGGL((k_from_f64<float, _Float16, false>), dim3(4096), dim3(kBlk), 0, s, A, n,
                         rows, ld, e, t, (float*)master, nullptr, nullptr);
      break;
    case DMPT_SPLIT_FP16:
      hipLaunchKernelGGL((k_from_f64<float, _Float16, true>), dim3(4096), dim3(kBlk), 0, s, A, n,
                         rows, ld, e, t, (float*)master, (uint16_t*)hi, (uint16_t*)lo);
      break;
    case DMPT_SPLIT_BF16:
      hipLaunchKernelGGL((k_from_f64<float, __bf16, true>), dim3(4096), dim3(kBlk), 0, s, A, n, rows, ld,
                         e, t, (float*)master, (uint16_t*)hi, (uint16_t*)lo);
      break;
  }
  return hipGetLastError();
}

// Plain copy of a padded layer-precision matrix into FP64 N x N (products check).
hipError_t launch_copy_plain(dmpt_precision prec, const void* src, int64_t ld, double* dst,
                             int64_t n, hipStream_t s) {
  return launch_copy_out(prec, nullptr, -1, src, src, ld, dst, n, s);
}

}  // namespace dmpt
