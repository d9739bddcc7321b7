// Internal declarations shared by the HIP translation units of libdmpt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "dmpt.h"

namespace dmpt {

// ----------------------------------------------------------------- vectors
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kMaxK = DMPT_MAX_K;
constexpr int kMaxLayers = DMPT_MAX_LAYERS;
constexpr int kRedBlocks = 1024;  // fixed grid of the reducing elementwise kernels

// Scale of the low part of a split operand: lo = RN((x - hi) * 2^t).
// FP16 needs it to keep lo out of the subnormal range; BF16 has FP32's
// exponent range and uses t = 0.
constexpr int kLoShiftF16 = 11;
constexpr int kLoShiftBF16 = 0;

// Panel-major layout of the 16-bit split operands: the Np x Np matrix is cut
// into blocks of kPanelRows rows x kPanelK columns, each block stored
// contiguously (row-major inside), the blocks of one row panel consecutive
// along k.  A k-tile of a 256-row panel is then one contiguous 16 KB chunk.
constexpr int kPanelRows = 256;
constexpr int kPanelK = 32;
__host__ __device__ __forceinline__ int64_t panel_index(int64_t r, int64_t c, int64_t kdim) {
  return ((r / kPanelRows) * (kdim / kPanelK) + c / kPanelK) * (kPanelRows * kPanelK) +
         (r % kPanelRows) * kPanelK + (c % kPanelK);
}

// ----------------------------------------------------------------- layer state
// Scalar state of Algorithms 1-3 kept in device memory so that the layer loop
// needs no host round trip.  Written only by the single-workgroup decision
// kernels; read by every kernel of the next steps.
struct LayerState {
  // configuration
  int32_t n_real;            // N
  int32_t k;                 // number of responses
  int32_t max_layers;
  int32_t pad0;
  double nocc;
  // progress
  int32_t n;                 // index of the layer in progress / last run
  int32_t done;              // 1: every response stopped, cap reached, or error
  int32_t error;             // dmpt_status of a device-detected error (0 = none)
  int32_t converged;         // 1: every D1 test fired
  // zeroth order
  int32_t d0;                // D0 converged (before or at layer n)
  int32_t d0_layer;
  int32_t x_computed;        // X = S^2 was formed at layer n
  int32_t upd_s0;            // S0 is updated at layer n
  int32_t d0_now;            // the D0 test fired at layer n
  int32_t sigma_cur;         // sigma_n
  int32_t s_par;             // fused split forms: buffer of the current 16-bit split of S
  int32_t order2_slot;       // response slot of the second-order chain S2 (-1: none)
  double n_s;                // tracked occupation N_S
  double n_s0;               // Tr S0 of the normalisation layer
  double fro0;               // ||S - S^2||_F at the D0 layer
  double eps1, epsN;
  int32_t sigma[kMaxLayers + 1];   // sigma[n], n = 1..
  double iderr[kMaxLayers + 1];    // IdErr_n
  // first order
  int32_t d1[kMaxK];
  int32_t d1_layer[kMaxK];
  int32_t s1_exp_split[kMaxK];     // 2^e scale of the stored S1 hi/lo split (read by the products)
  int32_t s1_exp_next[kMaxK];      // scale the next update writes the split with
  double fro1[kMaxK][kMaxLayers + 1];
  double s1_max[kMaxK];
  int32_t s1_exp_hist[kMaxK][kMaxLayers + 1];   // split scale S1_n was written with
};

// One output tile of a layer product.  out = 0: X = S^2; out = 1 + j: X1_j,
// or X2 = S1_0 S1_0 + S S2 + S2 S when j is the state's second-order slot.
struct TileItem {
  int16_t out;               // 0: X, 1 + j: response j; < 0: placeholder, skipped
  int16_t prob;              // problem index (batched launches; 0 otherwise)
  int32_t ti, tj;            // tile row/col (ti <= tj)
  int32_t ti2 = -1, tj2 = -1;   // pair launches: second tile (ti2, tj2), sharing a row band
                                // (ti2 == ti) or a column band (tj2 == tj); ti2 < 0: none
};

constexpr int kMaxKB = 3;    // most responses per problem of a batch

// One 32-row diagonal block of X = S^2 whose diagonal enters Tr X.
struct TraceBlock {
  int32_t prob;
  int32_t blk;               // rows 32 blk .. 32 blk + 31
};

// Buffers of one problem for the fused layer (split forms): the products
// read the current 16-bit splits and their epilogue writes the updated FP32
// masters and the next splits.  The split of S alternates between its two
// buffers with every update of S (LayerState::s_par); the split and master of
// S1_j alternate with the layer parity (S1_n lives in buffers n & 1).
struct ProblemDesc {
  const void* s_hi[2];
  const void* s_lo[2];
  const void* s1_hi[kMaxK][2];
  const void* s1_lo[kMaxK][2];
  float* s_master;           // S, updated in place (each tile owns its block and its mirror)
  float* s1m[kMaxK][2];      // S1_j masters
  LayerState* state;
  int64_t ld;                // row stride of the masters
  int64_t kdim;              // k extent of the products: N rounded up to kPanelK (the
                             // operands are zero beyond N, so every k past N adds exact zeros)
  int64_t pdim;              // panel-layout size of the 16-bit operands (multiple of 256)
};

// Pointers of the layer products.  The product kernels read `state` to skip
// outputs whose order has converged and to find the S1 split scales.
struct ProductArgs {
  const void* s_hi;          // split: 16-bit hi of S; direct forms: S itself
  const void* s_lo;          // split: 16-bit scaled lo of S
  const void* s1_hi[kMaxK];
  const void* s1_lo[kMaxK];
  void* x;                   // X (FP32 or FP64)
  void* x1[kMaxK];           // X1_j
  const void* a_op[kMaxK];    // direct forms: A operand of output 1 + j (NULL: S)
  const void* s1b[2];        // direct forms: both buffers of S1_0 (second-order products)
  const ProblemDesc* probs;  // fused split layer: per-problem buffers (NULL: the fields here)
  double* part_f;            // fused: per-item FP64 sums (squares), slot slot_base + item
  double* part_m;            // fused: per-item max |S1_new|
  int32_t slot_base;
  int32_t mode;              // direct forms: 0 layer products; 1 one product C = A B (A = s_hi,
                             // B = s1_hi[0], C = x) on upper tiles, mirrored (symmetric C);
                             // 2 the same on all tiles, no mirror (general C); 3 for every
                             // output 1 + j one product x1[j] = A_j B_j (A_j = a_op[j] or
                             // s_hi, B_j = s1_hi[j]) on all tiles, no mirror
  const TileItem* items;
  const LayerState* state;   // NULL: compute every item, scales taken from s1_exp
  int32_t s1_exp[kMaxK];     // used when state == NULL
  int64_t ld;                // row stride of every matrix (elements, >= kdim)
  int64_t kdim;              // padded size Np: rows, columns and the k extent
  int32_t n_items;
  int32_t lo_shift;          // t
  int32_t plain_accum;       // FP32 direct form: nonzero runs one accumulator over the whole
                             // k range instead of blocked sums (faster, less accurate; the
                             // adjoint's reverse products, whose error the forward dominates)
  int32_t pad1;
};

// ----------------------------------------------------------------- launchers
// layer products (kernels_gemm.hip)
int product_tile(dmpt_precision prec);   // output tile edge used by the product kernels
// Order of n items (cost[i]: products times k-tiles) for a persistent launch
// on `grid` workgroups, where position r * grid + s runs on slot s.  Items
// keep their list order and are dealt round by round against a target cost
// max(ceil(total / grid), largest item); a slot that would pass it takes a
// placeholder (-1, skipped at once) and the item waits for the next slot, so
// that every slot ends within one item of the mean.  Returns, per position,
// the item index or -1; the plain order when n <= grid or when the result
// would exceed `limit` positions.
std::vector<int32_t> balanced_rounds(const std::vector<int64_t>& cost, int grid, size_t limit);
hipError_t launch_products(dmpt_precision prec, const ProductArgs& a, hipStream_t s);
// Tile items of an Np x Np output for the single-product modes: upper tiles
// (mode 1) or all tiles (mode 2), tile edge product_tile(prec).
void product_items(int T, int mode, TileItem* out);   // T (T + 1) / 2 or T * T entries
// Fused split layer with 256- or 128-row tiles (a.probs set): the products of
// layer n and, in their epilogue, the layer update, the next split and the
// per-item partial sums; sigma and the update flags come from each problem's
// state, decided before the launch.
hipError_t launch_products_fused(dmpt_precision prec, int tile, const ProductArgs& a,
                                 hipStream_t s);
// The same on items of two 128 x 128 tiles that share a row or a column band
// (TileItem::ti2, tj2), one workgroup per CU: the batch's small-tile class.
// First-order items only (X, X1_j): no problem may have a second-order slot.
hipError_t launch_products_pair(dmpt_precision prec, const ProductArgs& a, hipStream_t s);
// N_X = Tr X_n of the coming fused products, before them: the diagonal 32 x 32
// fragments of X_n = S_{n-1}^2, one wave each, with the product kernel's MFMA
// sequence, so every X_ii equals the product's bitwise; part[b] = FP64 sum of
// the diagonal of block b (problems with D0 open).
hipError_t launch_trace_diag(dmpt_precision prec, const ProblemDesc* probs,
                             const TraceBlock* blocks, int n_blocks, double* part, hipStream_t s);

// layer kernels (kernels_layer.hip)
hipError_t launch_gershgorin(const double* H, int64_t n, double* partial /* 3*512 */,
                             LayerState* st, double* eps_out, hipStream_t s);
hipError_t launch_symcheck(const double* H, int64_t n, int32_t* flag, hipStream_t s);
hipError_t launch_maxabs(const double* H, int64_t n, double* partial, hipStream_t s);
// Matrices in the workspace have `rows` = Np rows and row stride `ld` >= Np;
// the columns [Np, ld) and every entry outside the N x N block hold zero.
hipError_t launch_init_s0(dmpt_precision prec, const double* H0, int64_t n, int64_t rows,
                          int64_t ld, const LayerState* st, void* s_init, hipStream_t s);
hipError_t launch_load_s0(dmpt_precision prec, const void* s_init, void* master, void* hi, void* lo,
                          int64_t rows, int64_t ld, int t, hipStream_t s);
hipError_t launch_init_s1(dmpt_precision prec, const double* H1, int64_t n, int64_t rows,
                          int64_t ld, LayerState* st, int j, double* partial, void* s1, void* hi,
                          void* lo, int t, double w_fixed, hipStream_t s);
// k response slots; order2_slot (-1: none) carries the second-order chain.
hipError_t launch_reset_state(LayerState* st, int k, int order2_slot, int max_layers, double nocc,
                              int64_t n, hipStream_t s);
hipError_t launch_decide0(dmpt_precision prec, LayerState* st, const void* x, int64_t ld,
                          hipStream_t s);
hipError_t launch_update(dmpt_precision prec, const LayerState* st, int which, const void* x,
                         const void* s_old, void* dst, void* hi, void* lo, int64_t rows,
                         int64_t ld, int t, double* pfro, double* pmax, hipStream_t s);
hipError_t launch_decide1(LayerState* st, const double* pfro0, const double* pfro1,
                          const double* pmax1, int split, int lo_shift, hipStream_t s);
// Fused split layer: the decisions before the products (N_X from np trace
// partials) and after them (item partials of `items`, slot = index).
hipError_t launch_predecide(LayerState* st, const double* part, int np, hipStream_t s);
hipError_t launch_postdecide(LayerState* st, const TileItem* items, int n_items,
                             const double* part_f, const double* part_m, int lo_shift,
                             hipStream_t s);
hipError_t launch_copy_out(dmpt_precision prec, const LayerState* st, int which, const void* b0,
                           const void* b1, int64_t ld, double* dst, int64_t n, hipStream_t s);
hipError_t launch_trace(const double* P, int64_t n, double* out, hipStream_t s);
// self-consistent response: heff = (1 - mix) heff + mix (h1 + g); out[0] = ||a - b||^2,
// out[1] = ||a||^2 (part: 2 kRedBlocks FP64 partials)
hipError_t launch_mix(const double* h1, const double* g, double* heff, double mix, int64_t n,
                      hipStream_t s);
hipError_t launch_diff_norms(const double* a, const double* b, int64_t n, double* part,
                             double* out, hipStream_t s);
// out = Tr(A B) for symmetric B (part: kRedBlocks FP64 partials)
hipError_t launch_contract(const double* A, const double* B, int64_t n, double* part, double* out,
                           hipStream_t s);
hipError_t launch_from_f64(dmpt_precision prec, const double* A, int64_t n, int64_t rows,
                           int64_t ld, int e, int t, void* master, void* hi, void* lo,
                           hipStream_t s);
hipError_t launch_copy_plain(dmpt_precision prec, const void* src, int64_t ld, double* dst,
                             int64_t n, hipStream_t s);

// adjoint of the layer recursion (kernels_adjoint.hip)
hipError_t launch_replay_state(const LayerState* fwd, LayerState* rep, int n, hipStream_t s);
hipError_t launch_resplit(dmpt_precision prec, const LayerState* fwd, int j, int layer,
                          const void* master, void* hi, void* lo, int64_t rows, int64_t ld, int t,
                          hipStream_t s);
hipError_t launch_adj_seed(dmpt_precision prec, const double* W, int64_t n, int64_t rows,
                           int64_t ld, void* dst, hipStream_t s);
// One reverse layer from the one-sided products M2 = S Sh, M1_j = S Sh1_j,
// M3_j = Sh1_j S1_j (general np x np, row stride ld; np a multiple of 32).
hipError_t launch_adj_update(dmpt_precision prec, const LayerState* fwd, int layer, int k,
                             const void* m2, void* sh, const void* const* m1, void* const* sh1,
                             const void* const* m3, int64_t np, int64_t ld, hipStream_t s);
hipError_t launch_adj_out(dmpt_precision prec, const LayerState* fwd, const void* src, int64_t ld,
                          double* dst, int64_t n, hipStream_t s);
hipError_t launch_selftest_mfma(int32_t* result, hipStream_t s);
// MFMA rate probe: `blocks` workgroups of four waves, `iters` x 48 MFMAs each
// (32x32x16 f16 or bf16 for the split precisions, 16x16x4 f32 or f64 for the
// direct ones); out[blocks * 256] receives per-lane sums, ticks[2] the
// shader-clock and wall-clock ticks of workgroup 0.
hipError_t launch_mfma_rate(dmpt_precision prec, int blocks, int iters, float* out,
                            int64_t* ticks, hipStream_t s);
double mfma_probe_flops(dmpt_precision prec);   // flops of one MFMA of the probe
int device_cu_count();   // compute units of the current device (256 if unknown)

// Record the reason of a non-OK status for dmpt_last_error (dmpt_api.hip).
void set_last_error(const char* msg);

}  // namespace dmpt
