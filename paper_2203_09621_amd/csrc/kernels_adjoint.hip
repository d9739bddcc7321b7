// Adjoint (reverse mode) of the DNN-SP2-PT layer recursion for
// L = sum_k Tr(P1_k W_k).
//
// Forward layer n (sigma_n and the update flags fixed by the forward pass):
//   S1_n = sigma (S S1 + S1 S) + (1 - sigma) S1        (if response k is updated)
//   S_n  = sigma S^2 + (1 - sigma) S                   (if S is updated)
// with S = S_{n-1}, S1 = S1_{n-1}.  For symmetric matrices the adjoints are
//   Sh1_{n-1} = sigma (S Sh1 + Sh1 S) + (1 - sigma) Sh1                 (S1 updated)
//   Sh_{n-1}  = [sigma (S Sh + Sh S) + (1 - sigma) Sh]_(S updated)
//             + sum_k [sigma (Sh1_k S1_k + S1_k Sh1_k)]_(S1_k updated)
// seeded with Sh1_k = W_k (symmetrised) at the layer that produced P1_k and
// Sh = 0.  The normalisation layer gives dL/dH1_k = -Sh1_k,0/(eps_N - eps_1)
// and dL/dH0 = -Sh_0/(eps_N - eps_1); the Gershgorin bounds are treated as
// constants (the limits P0 and P1 do not depend on them).
#include "dmpt_internal.h"

namespace dmpt {

constexpr int kBlkA = 256;

template <typename T16> struct Conv16;
template <> struct Conv16<_Float16> {
  static __device__ __forceinline__ uint16_t to(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  static __device__ __forceinline__ float from(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
};
template <> struct Conv16<__bf16> {
  static __device__ __forceinline__ uint16_t to(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
  static __device__ __forceinline__ float from(uint16_t b) { return (float)__builtin_bit_cast(__bf16, b); }
};

// State for replaying forward layer n during recomputation: the sigma and
// the update flags the forward pass took, and the S1 split scales it used.
// No decision is taken again.
__global__ void k_replay_state(const LayerState* f, LayerState* r, int n) {
  if (threadIdx.x != 0) return;
  r->n = n;
  r->k = f->k;
  r->order2_slot = -1;
  r->n_real = f->n_real;
  r->done = 0;
  r->error = 0;
  const int d0l = f->d0_layer > 0 ? f->d0_layer : (1 << 30);
  r->d0 = n >= d0l ? 1 : 0;          // X is needed only while S is updated
  r->upd_s0 = n < d0l ? 1 : 0;
  r->x_computed = 0;
  r->d0_now = 0;
  r->sigma_cur = f->sigma[n];
  for (int j = 0; j < kMaxK; ++j) {
    const int d1l = (j < f->k && f->d1_layer[j] > 0) ? f->d1_layer[j] : (j < f->k ? (1 << 30) : 0);
    r->d1[j] = n >= d1l ? 1 : 0;
    r->s1_exp_split[j] = f->s1_exp_hist[j][n - 1];
    r->s1_exp_next[j] = f->s1_exp_hist[j][n];
  }
}

hipError_t launch_replay_state(const LayerState* fwd, LayerState* rep, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_replay_state, dim3(1), dim3(kWave), 0, s, fwd, rep, n);
  return hipGetLastError();
}

// hi/lo of a restored S1 (j >= 0, scale of layer `layer`) or S (j < 0, scale 1).
template <typename T16>
__global__ void __launch_bounds__(kBlkA) k_resplit(const LayerState* f, int j, int layer,
                                                  const float* m, uint16_t* hi, uint16_t* lo,
                                                  int64_t rows, int64_t ld, int t) {
  const int e = j >= 0 ? f->s1_exp_hist[j][layer] : 0;
  const int64_t elems = rows * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlkA + threadIdx.x; q < elems;
       q += (int64_t)gridDim.x * kBlkA) {
    const int64_t r = q / ld, c = q - r * ld;
    if (c >= rows) continue;
    const int64_t pi = panel_index(r, c, rows);
    const float xs = ldexpf(m[q], e);
    const uint16_t h = Conv16<T16>::to(xs);
    hi[pi] = h;
    lo[pi] = Conv16<T16>::to(ldexpf(xs - Conv16<T16>::from(h), t));
  }
}

hipError_t launch_resplit(dmpt_precision prec, const LayerState* fwd, int j, int layer,
                          const void* master, void* hi, void* lo, int64_t rows, int64_t ld, int t,
                          hipStream_t s) {
  if (prec == DMPT_SPLIT_FP16)
    hipLaunchKernelGGL(k_resplit<_Float16>, dim3(4096), dim3(kBlkA), 0, s, fwd, j, layer,
                       (const float*)master, (uint16_t*)hi, (uint16_t*)lo, rows, ld, t);
  else if (prec == DMPT_SPLIT_BF16)
    hipLaunchKernelGGL(k_resplit<__bf16>, dim3(4096), dim3(kBlkA), 0, s, fwd, j, layer,
                       (const float*)master, (uint16_t*)hi, (uint16_t*)lo, rows, ld, t);
  return hipGetLastError();
}

// Sh1 seed: (W + W^T)/2 into the padded workspace layout (zero elsewhere).
template <typename M>
__global__ void __launch_bounds__(kBlkA) k_adj_seed(const double* W, int64_t n, int64_t rows,
                                                   int64_t ld, M* dst) {
  const int64_t total = rows * ld;
  for (int64_t q = (int64_t)blockIdx.x * kBlkA + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlkA) {
    const int64_t i = q / ld, j = q - i * ld;
    double v = 0.0;
    if (i < n && j < n) v = 0.5 * (W[i * n + j] + W[j * n + i]);
    dst[q] = (M)v;
  }
}

hipError_t launch_adj_seed(dmpt_precision prec, const double* W, int64_t n, int64_t rows,
                           int64_t ld, void* dst, hipStream_t s) {
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_adj_seed<double>, dim3(4096), dim3(kBlkA), 0, s, W, n, rows, ld,
                       (double*)dst);
  else
    hipLaunchKernelGGL(k_adj_seed<float>, dim3(4096), dim3(kBlkA), 0, s, W, n, rows, ld,
                       (float*)dst);
  return hipGetLastError();
}

// One reverse layer: T2 = S Sh + Sh S, T1_k = S Sh1_k + Sh1_k S and
// T3_k = Sh1_k S1_k + S1_k Sh1_k were formed by the product kernel from the
// adjoints of layer n; this writes the adjoints of layer n - 1 in place.
struct AdjPtrs {
  const void* t1[kMaxK];
  void* sh1[kMaxK];
  const void* t3[kMaxK];
};

// One reverse layer (the adjoint of Eqs. LinTransf, S_n detailed, dB) from
// one-sided products: for symmetric A and B, A B + B A = M + M^T with M = A B,
// so T2 = M2 + M2^T (M2 = S Sh), T1_j = M1_j + M1_j^T (M1_j = S Sh1_j) and
// T3_j = M3_j + M3_j^T (M3_j = Sh1_j S1_j).  With sigma = sigma_n:
//   Sh1_j <- sigma T1_j + (1 - sigma) Sh1_j       (while S1_j was updated)
//   Sh    <- [sigma T2 + (1 - sigma) Sh] + sum_j sigma T3_j
// where the bracket applies while S was updated.  One 32 x 32 tile (ti, tj)
// per block; the mirror tile of each M comes through LDS, so every global
// access is a row of 32 consecutive elements.
template <typename M>
__global__ void __launch_bounds__(kBlkA) k_adj_update(const LayerState* f, int n, int k,
                                                     const M* m2, M* sh, AdjPtrs p, int64_t ld) {
  __shared__ M tr[32][33];
  const M sig = (M)f->sigma[n];
  const int d0l = f->d0_layer > 0 ? f->d0_layer : (1 << 30);
  const bool s_upd = n < d0l;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads, 4 rows each
  // (M + M^T) at the thread's four elements (r0 + ty + 8 q, c0 + tx)
  auto sym = [&](const M* m, M* out) {
    __syncthreads();                           // the previous mirror tile has been read
#pragma unroll
    for (int q = 0; q < 4; ++q) tr[ty + 8 * q][tx] = m[(c0 + ty + 8 * q) * ld + r0 + tx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = m[(r0 + ty + 8 * q) * ld + c0 + tx] + tr[tx][ty + 8 * q];
  };
  M v[4], t[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = sh[(r0 + ty + 8 * q) * ld + c0 + tx];
  if (s_upd) {
    sym(m2, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = sig * t[q] + ((M)1 - sig) * v[q];
  }
  for (int j = 0; j < k; ++j) {
    const int d1l = f->d1_layer[j] > 0 ? f->d1_layer[j] : (1 << 30);
    if (!(n < d1l)) continue;                  // uniform over the block
    sym((const M*)p.t3[j], t);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += sig * t[q];
    sym((const M*)p.t1[j], t);
    M* s1 = (M*)p.sh1[j];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t at = (r0 + ty + 8 * q) * ld + c0 + tx;
      s1[at] = sig * t[q] + ((M)1 - sig) * s1[at];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sh[(r0 + ty + 8 * q) * ld + c0 + tx] = v[q];
}

hipError_t launch_adj_update(dmpt_precision prec, const LayerState* fwd, int layer, int k,
                             const void* m2, void* sh, const void* const* m1, void* const* sh1,
                             const void* const* m3, int64_t np, int64_t ld, hipStream_t s) {
  if (np % 32 != 0) return hipErrorInvalidValue;
  AdjPtrs p;
  for (int j = 0; j < kMaxK; ++j) {
    p.t1[j] = j < k ? m1[j] : nullptr;
    p.sh1[j] = j < k ? sh1[j] : nullptr;
    p.t3[j] = j < k ? m3[j] : nullptr;
  }
  const dim3 grid((unsigned)(np / 32), (unsigned)(np / 32));
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_adj_update<double>, grid, dim3(kBlkA), 0, s, fwd, layer, k,
                       (const double*)m2, (double*)sh, p, ld);
  else
    hipLaunchKernelGGL(k_adj_update<float>, grid, dim3(kBlkA), 0, s, fwd, layer, k,
                       (const float*)m2, (float*)sh, p, ld);
  return hipGetLastError();
}

// dL/dH = -Sh_0 / (eps_N - eps_1)  (FP64, N x N).
template <typename M>
__global__ void __launch_bounds__(kBlkA) k_adj_out(const LayerState* f, const M* src, int64_t ld,
                                                  double* dst, int64_t n) {
  const double scale = -1.0 / (f->epsN - f->eps1);
  const int64_t total = n * n;
  for (int64_t q = (int64_t)blockIdx.x * kBlkA + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * kBlkA) {
    const int64_t i = q / n, j = q - i * n;
    dst[q] = scale * (double)src[i * ld + j];
  }
}

hipError_t launch_adj_out(dmpt_precision prec, const LayerState* fwd, const void* src, int64_t ld,
                          double* dst, int64_t n, hipStream_t s) {
  if (prec == DMPT_FP64)
    hipLaunchKernelGGL(k_adj_out<double>, dim3(4096), dim3(kBlkA), 0, s, fwd, (const double*)src,
                       ld, dst, n);
  else
    hipLaunchKernelGGL(k_adj_out<float>, dim3(4096), dim3(kBlkA), 0, s, fwd, (const float*)src, ld,
                       dst, n);
  return hipGetLastError();
}

}  // namespace dmpt
