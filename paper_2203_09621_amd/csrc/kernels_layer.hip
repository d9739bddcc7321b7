// Normalisation layer, per-layer decisions, fused update/split/norm and output
// kernels of the DNN-SP2-PT network.
//
// Every reduction is deterministic: a fixed grid, per-block partial sums in
// FP64 combined in a fixed order by a single-workgroup kernel.  No floating
// point atomics.
#include <math.h>

#include "layer_common.h"

namespace dmpt {

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
    if (H1 && r < n && c < n) v = -H1[r * n + c] / w;
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
  // H1 == NULL: a zero perturbation (the second-order chain without H2)
  hipLaunchKernelGGL(k_maxabs, dim3(kRedBlocks), dim3(kBlk), 0, s, H1, H1 ? n * n : 0, part);
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
__global__ void k_reset_state(LayerState* st, int k, int order2_slot, int max_layers, double nocc,
                              int64_t n) {
  // one thread: a few hundred words
  if (threadIdx.x != 0) return;
  st->n_real = (int32_t)n;
  st->k = k;
  st->order2_slot = order2_slot;
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
  st->s_par = 0;
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

hipError_t launch_reset_state(LayerState* st, int k, int order2_slot, int max_layers, double nocc,
                              int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(kWave), 0, s, st, k, order2_slot, max_layers,
                     nocc, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ decisions, part 1
// Algorithm 1 trace test and Algorithm 2: N_X = Tr X in FP64, IdErr, sigma,
// the D0 test and the N_S update.  After D0 converged: sigma flips.
template <typename M>
__global__ void __launch_bounds__(kBlk) k_decide0(LayerState* st, const M* x, int64_t ld) {
  decide0_body<M>(st, x, ld);
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
  update_body<M, T16, SPLIT>(st, which, x, s_old, dst, hi, lo,
                             (int64_t)blockIdx.x * kBlk + threadIdx.x, total / 4,
                             (int64_t)gridDim.x * kBlk, ld, kdim, t, pfro + blockIdx.x,
                             pmax ? pmax + blockIdx.x : nullptr);
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
  Partials pr;
  pr.fro0 = pfro0;
  pr.n0 = kRedBlocks;
  for (int j = 0; j < kMaxK; ++j) {
    pr.fro1[j] = pfro1 + (size_t)j * kRedBlocks;
    pr.max1[j] = pmax1 + (size_t)j * kRedBlocks;
    pr.n1[j] = kRedBlocks;
  }
  decide1_body(st, pr, split, lo_shift);
}

hipError_t launch_decide1(LayerState* st, const double* pfro0, const double* pfro1,
                          const double* pmax1, int split, int lo_shift, hipStream_t s) {
  hipLaunchKernelGGL(k_decide1, dim3(1), dim3(kBlk), 0, s, st, pfro0, pfro1, pmax1, split, lo_shift);
  return hipGetLastError();
}

// ------------------------------------------------------------------ observables
// Tr(A B) for symmetric B as sum_ij A_ij B_ij: FP64 partial per block in a
// fixed grid; the final sum runs in block order.
__global__ void __launch_bounds__(kBlk) k_contract(const double* A, const double* B, int64_t total,
                                                  double* part) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  double v = 0.0;
  const int64_t pairs = total / 2;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < pairs;
       q += (int64_t)gridDim.x * kBlk) {
    const D2 a = ((const D2*)A)[q], b = ((const D2*)B)[q];
    v += a[0] * b[0] + a[1] * b[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (total & 1)) v += A[total - 1] * B[total - 1];
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void k_contract_final(const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int i = 0; i < nb; ++i) v += part[i];
  *out = v;
}

hipError_t launch_contract(const double* A, const double* B, int64_t n, double* part, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_contract, dim3(kRedBlocks), dim3(kBlk), 0, s, A, B, n * n, part);
  hipLaunchKernelGGL(k_contract_final, dim3(1), dim3(kWave), 0, s, part, kRedBlocks, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ self-consistent response
// heff = (1 - mix) heff + mix (h1 + g)
__global__ void __launch_bounds__(kBlk) k_mix(const double* h1, const double* g, double* heff,
                                             double mix, int64_t total) {
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk)
    heff[q] = (1.0 - mix) * heff[q] + mix * (h1[q] + g[q]);
}

hipError_t launch_mix(const double* h1, const double* g, double* heff, double mix, int64_t n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mix, dim3(2048), dim3(kBlk), 0, s, h1, g, heff, mix, n * n);
  return hipGetLastError();
}

// partials of ||a - b||^2 (part[0..nb)) and ||a||^2 (part[nb..2 nb)); out[0..1] their sums
__global__ void __launch_bounds__(kBlk) k_diff_norms(const double* a, const double* b,
                                                    int64_t total, double* part) {
  double d2 = 0.0, a2 = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kBlk + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlk) {
    const double d = a[q] - b[q];
    d2 += d * d;
    a2 += a[q] * a[q];
  }
  d2 = block_sum(d2);
  a2 = block_sum(a2);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = d2;
    part[gridDim.x + blockIdx.x] = a2;
  }
}

__global__ void k_diff_norms_final(const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double d2 = 0.0, a2 = 0.0;
  for (int i = 0; i < nb; ++i) {
    d2 += part[i];
    a2 += part[nb + i];
  }
  out[0] = d2;
  out[1] = a2;
}

hipError_t launch_diff_norms(const double* a, const double* b, int64_t n, double* part,
                             double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norms, dim3(kRedBlocks), dim3(kBlk), 0, s, a, b, n * n, part);
  hipLaunchKernelGGL(k_diff_norms_final, dim3(1), dim3(kWave), 0, s, part, kRedBlocks, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fused split layer
__global__ void __launch_bounds__(kBlk) k_predecide(LayerState* st, const double* part, int np) {
  predecide_body(st, part, np);
}

hipError_t launch_predecide(LayerState* st, const double* part, int np, hipStream_t s) {
  hipLaunchKernelGGL(k_predecide, dim3(1), dim3(kBlk), 0, s, st, part, np);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlk) k_postdecide(LayerState* st, const TileItem* items,
                                                    int n_items, const double* part_f,
                                                    const double* part_m, int lo_shift) {
  postdecide_body(st, items, n_items, part_f, part_m, lo_shift);
}

hipError_t launch_postdecide(LayerState* st, const TileItem* items, int n_items,
                             const double* part_f, const double* part_m, int lo_shift,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_postdecide, dim3(1), dim3(kBlk), 0, s, st, items, n_items, part_f, part_m,
                     lo_shift);
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
