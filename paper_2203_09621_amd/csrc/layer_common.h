// Device helpers and per-problem bodies of the layer decisions and the fused
// update, shared by the single-problem kernels and the batched kernels.
#pragma once

#include <math.h>

#include "dmpt_internal.h"

namespace dmpt {

constexpr int kBlk = 256;

// ------------------------------------------------------------------ helpers
static __device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
static __device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
static __device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// Block-wide reductions for kBlk threads; the result is valid in every thread.
static __device__ double block_sum(double v) {
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
static __device__ double block_max(double v) {
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
static __device__ double block_min(double v) {
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
static __device__ __forceinline__ int split_exponent(double m) {
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
static __device__ __forceinline__ void split_one(float v, int e, int t, uint16_t* hi, uint16_t* lo) {
  const float xs = ldexpf(v, e);
  const uint16_t h = Conv<T16>::to(xs);
  *hi = h;
  *lo = Conv<T16>::to(ldexpf(xs - Conv<T16>::from(h), t));
}


// ------------------------------------------------------------------ decisions, part 1
// Algorithm 1 trace test and Algorithm 2 for layer n = st->n + 1, given
// N_X = Tr X_n (thread 0 only): IdErr, sigma, the D0 test and the N_S update.
// After D0 converged: sigma flips.
static __device__ void decide0_apply(LayerState* st, double nx) {
  const int d0 = st->d0;
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

// After the products of layer n: N_X = Tr X in FP64 from the diagonal of X.
template <typename M>
static __device__ void decide0_body(LayerState* st, const M* x, int64_t ld) {
  if (st->done) return;
  const int d0 = st->d0;
  const int n_real = st->n_real;
  double nx = 0.0;
  if (!d0) {
    for (int i = threadIdx.x; i < n_real; i += kBlk) nx += (double)x[(int64_t)i * ld + i];
    nx = block_sum(nx);
  }
  __syncthreads();
  if (threadIdx.x == 0) decide0_apply(st, nx);
}

// Fused split layer, before the products of layer n: N_X = Tr X_n from the
// diagonal-block partial sums part[0..np), then Algorithms 1-2.
static __device__ void predecide_body(LayerState* st, const double* part, int np) {
  if (st->done) return;
  double nx = 0.0;
  if (!st->d0) {
    for (int i = threadIdx.x; i < np; i += kBlk) nx += part[i];
    nx = block_sum(nx);
  }
  __syncthreads();
  if (threadIdx.x == 0) decide0_apply(st, nx);
}

// ------------------------------------------------------------------ fused layer update
// Thread range [q0 + tid*1, q1) with stride qs over float4/double4 vectors;
// the block's partial sums go to *pfro / *pmax (block-uniform slots).
template <typename M, typename T16, bool SPLIT>
static __device__ void update_body(const LayerState* st, int which, const M* x, const M* s_old,
                                   M* dst, uint16_t* hi, uint16_t* lo, int64_t q0, int64_t q1,
                                   int64_t qs, int64_t ld, int64_t kdim, int t, double* pfro,
                                   double* pmax) {
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
  for (int64_t q = q0; q < q1; q += qs) {
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
    *pfro = fro;
    if (pmax) *pmax = mx;
  }
}


// ------------------------------------------------------------------ decisions, part 2
// Partial-sum ranges of one problem: S0 update (fro0) and, per response j,
// its update (fro1[j], max1[j]), each with count entries.
struct Partials {
  const double* fro0;
  int n0;
  const double* fro1[kMaxK];
  const double* max1[kMaxK];
  int n1[kMaxK];
};

// Algorithm 2 FroErr^(0) at the D0 layer and, per active response, Algorithm
// 3 (thread 0 only): FroErr^(1)_n, the parameter-free D1 test (Eq. ConvCrit,
// C_pt = 9), the next split scale, and the stop flag.  The second-order chain
// (slot order2_slot) takes the same test on FroErr^(2)_n = ||S2 - X2||_F from
// two layers after the D1 layer of the first perturbation: with S0 and S1
// frozen its map has the same linear part as the first-order map.  f0sq = ||S - X||_F^2
// (used at the D0 layer), f1sq[j] = ||S1_j - X1_j||_F^2, m1[j] = max|S1_j,n|.
static __device__ void decide1_apply(LayerState* st, double f0sq, const double* f1sq,
                                     const double* m1, int split, int lo_shift) {
  const int k = st->k;
  const int d0 = st->d0;
  const int n = st->n;
  if (st->d0_now) {
    st->fro0 = sqrt(f0sq);
    if (!isfinite(st->fro0)) st->error = DMPT_ENONFINITE;
  }
  int all = 1;
  for (int j = 0; j < k; ++j) {
    if (st->d1[j]) continue;
    const double mx = m1[j];
    // the split written this layer used s1_exp_next; check it stayed in range
    if (split && ldexp(mx, st->s1_exp_next[j] + lo_shift) > 32768.0) st->error = DMPT_ENONFINITE;
    if (!isfinite(mx)) st->error = DMPT_ENONFINITE;
    if (d0) {
      const double f = sqrt(f1sq[j]);
      st->fro1[j][n] = f;
      if (!isfinite(f)) st->error = DMPT_ENONFINITE;
      // first order: two layers after D0; the second-order chain: two layers
      // after the D1 layer of the first perturbation (S0 and S1 frozen)
      const bool armed = j == st->order2_slot ? (st->d1[0] && n - 2 >= st->d1_layer[0])
                                              : n - 2 >= st->d0_layer;
      if (armed) {
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

static __device__ void decide1_body(LayerState* st, const Partials& pr, int split, int lo_shift) {
  if (st->done) return;
  const int k = st->k;
  const int d0_now = st->d0_now, d0 = st->d0;
  __shared__ double res[2 * kMaxK + 1];
  // sums in a fixed order: each thread a fixed strided subset, then the block tree
  if (d0_now) {
    double v = 0.0;
    for (int i = threadIdx.x; i < pr.n0; i += kBlk) v += pr.fro0[i];
    v = block_sum(v);
    if (threadIdx.x == 0) res[2 * kMaxK] = v;
  }
  for (int j = 0; j < k; ++j) {
    if (st->d1[j]) continue;
    double v = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < pr.n1[j]; i += kBlk) {
      if (d0) v += pr.fro1[j][i];
      m = fmax(m, pr.max1[j][i]);
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
  double f1[kMaxK], m1[kMaxK];
  for (int j = 0; j < kMaxK; ++j) {
    f1[j] = j < k ? res[2 * j] : 0.0;
    m1[j] = j < k ? res[2 * j + 1] : 0.0;
  }
  decide1_apply(st, d0_now ? res[2 * kMaxK] : 0.0, f1, m1, split, lo_shift);
}

// Fused split layer, after the products of layer n: the per-item partials of
// this problem's items (slots part + index) are combined in a fixed order.
// Output 0 carries ||S - X||_F^2 at the D0 layer; output 1 + j carries
// ||S1_j - X1_j||_F^2 (after D0) and max|S1_j,n|.  Outputs skipped this layer
// are ignored.
static __device__ void postdecide_body(LayerState* st, const TileItem* items, int n_items,
                                       const double* part_f, const double* part_m, int lo_shift,
                                       int prob = 0) {
  if (st->done) return;
  const int k = st->k;
  const int xc = st->x_computed;
  int act[kMaxK];
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) act[j] = j < k && !st->d1[j];
  double f[kMaxK + 1], m[kMaxK];
#pragma unroll
  for (int q = 0; q <= kMaxK; ++q) f[q] = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) m[j] = 0.0;
  for (int i = threadIdx.x; i < n_items; i += kBlk) {
    if (items[i].prob != prob) continue;       // another problem's item inside this range
    const int o = items[i].out;
    const double pf = part_f[i];
    if (o == 0) {
      if (xc) f[0] += pf;
      continue;
    }
    const double pm = part_m[i];
#pragma unroll
    for (int j = 0; j < kMaxK; ++j)
      if (o == 1 + j && act[j]) {
        f[1 + j] += pf;
        m[j] = fmax(m[j], pm);
      }
  }
  __shared__ double res[2 * kMaxK + 1];
  {
    const double v = block_sum(f[0]);
    if (threadIdx.x == 0) res[2 * kMaxK] = v;
  }
  for (int j = 0; j < k; ++j) {
    double v = 0.0, w = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxK; ++q)
      if (q == j) {
        v = f[1 + q];
        w = m[q];
      }
    v = block_sum(v);
    w = block_max(w);
    if (threadIdx.x == 0) {
      res[2 * j] = v;
      res[2 * j + 1] = w;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double f0sq = 0.0;
  if (xc) {
    if (st->upd_s0)
      st->s_par ^= 1;          // the epilogue wrote the split of S_n to the other buffer
    else
      f0sq = res[2 * kMaxK];
  }
  double f1[kMaxK], m1[kMaxK];
  for (int j = 0; j < kMaxK; ++j) {
    f1[j] = j < k ? res[2 * j] : 0.0;
    m1[j] = j < k ? res[2 * j + 1] : 0.0;
  }
  decide1_apply(st, f0sq, f1, m1, 1, lo_shift);
}


}  // namespace dmpt
