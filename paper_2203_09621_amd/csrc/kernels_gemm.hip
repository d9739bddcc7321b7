// Layer products of the DNN-SP2-PT network on gfx950 MFMA.
//
// One launch forms, for every output tile (ti <= tj) of the upper triangle,
//   X    = S S                      (zeroth-order activation, Eq. S0 tensor core)
//   X1_j = S S1_j + S1_j S          (first-order activation, Eqs. FP32S0S1 and
//                                    S0S1 tensor core, with the symmetry remark
//                                    that closes Sec. III.C)
// and mirrors the tile into (tj, ti): every operand and result is symmetric, so
// each product is read as two row panels that are contiguous along k (an
// A * B^T form) and only half of the tiles are computed.
//
// Split form (prior art: the dual half-precision representation, Eqs. DualMat,
// DualMat2): a symmetric operand Y is stored as hi = RN16(Y 2^e) and
// lo = RN16((Y 2^e - hi) 2^t).  With a single FP32 accumulator
//   acc = (2^t hi_A) hi_B + hi_A lo_B + lo_A hi_B  ( = 2^(t + eA + eB) A B )
// and the epilogue multiplies by 2^-(t + eA + eB).  The lo*lo term is dropped
// as in the paper.  The 2^t factor is applied to hi_A in registers (exact).
// The MFMA's rounding depends on the operand order, so the trace kernel below
// uses the same order.
#include <stdlib.h>

#include "layer_common.h"

namespace dmpt {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap(int b, int g) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous run of tile items so that the tiles resident on one XCD share
  // row panels in its L2.
  const int q = g / kXcds, r = g % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Workgroup-uniform values read from memory the kernel also writes come back
// in vector registers; these put them in scalar registers for address
// arithmetic.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) { return (T*)uni((int64_t)p); }

// ------------------------------------------------------------------ split form
template <typename T16> struct Split16;

template <> struct Split16<_Float16> {
  typedef f16x8 V;
  static constexpr int kShift = kLoShiftF16;
  static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ V up(V a) {
    return a * (_Float16)(float)(1 << kShift);
  }
};

template <> struct Split16<__bf16> {
  typedef bf16x8 V;
  static constexpr int kShift = kLoShiftBF16;
  static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ V up(V a) { return a; }  // t = 0
};

// Resolve the skip flags and the operand scale of one tile item.
// Returns false when the item has nothing to do.  Plain launches run after
// nothing was decided for the layer: X is skipped once D0 converged.  Fused
// launches run after the decision of layer n: X is still formed at the D0
// layer itself, for ||S - X||_F.
template <bool FUSED>
__device__ __forceinline__ bool item_active(const ProductArgs& a, const TileItem& it, int* sexp) {
  if (it.out < 0) return false;                 // placeholder of a balanced round
  const LayerState* st = FUSED ? a.probs[it.prob].state : a.state;
  if (st) {
    if (st->done) return false;
    if (it.out == 0) {
      if (FUSED ? (st->d0 && !st->d0_now) : st->d0) return false;
    } else if (st->d1[it.out - 1]) {
      return false;
    }
    *sexp = it.out == 0 ? 0 : st->s1_exp_split[it.out - 1];
  } else {
    *sexp = it.out == 0 ? 0 : a.s1_exp[it.out - 1];
  }
  return true;
}

// s_waitcnt immediate that waits until at most N vector-memory operations are
// outstanding and leaves the other counters unconstrained (gfx9 encoding).
template <int N>
struct VmWait {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  static constexpr int imm = (N & 15) | (((N >> 4) & 3) << 14) | (7 << 4) | (15 << 8);
};
// ... and until at most N LDS operations are outstanding, the others free.
template <int N>
struct LgkWait {
  static_assert(N >= 0 && N < 16, "lgkmcnt range");
  static constexpr int imm = 15 | (3 << 14) | (7 << 4) | (N << 8);
};

// Plain launches store X and X1_j.  Fused launches (FUSED) apply the layer
// update in the epilogue instead: with sigma of the problem's state,
//   S_n  = X    (sigma = +1)   or  2 S_{n-1}  - X     (sigma = -1)
//   S1_n = X1_j (sigma = +1)   or  2 S1_{n-1} - X1_j  (sigma = -1)
// (Eqs. LinTransf, S_n detailed, dB), written to the FP32 masters and split
// into the next 16-bit buffers with the state's scale, together with FP64
// partial sums for the decisions; X and X1 never reach memory.
template <typename T16, int BM, int BK, int WGM, int WGN, int SWZ, int STAGES, bool FUSED>
__global__ void __launch_bounds__(WGM * WGN * kWave)
k_products_split(const ProductArgs a) {
  using S = Split16<T16>;
  using V = typename S::V;
  constexpr int NT = WGM * WGN * kWave;
  constexpr int BN = BM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  constexpr int CH = BK / 8;                 // 16-byte chunks per row of a k-tile
  constexpr int ROWS = 2 * BM + 2 * BN;      // A_hi | A_lo | B_hi | B_lo
  constexpr int STAGE = ROWS * CH;           // chunks per pipeline stage
  constexpr int RPW = kWave / CH;            // rows one wave fills per load instruction
  constexpr int RPL = NT / CH;               // rows all waves fill per load round
  constexpr int LOADS = ROWS / RPL;          // load rounds per k-tile
  static_assert(ROWS % RPL == 0 && BM % RPL == 0, "load rounds must not straddle arrays");
  static_assert(BK % 16 == 0 && WTM % 32 == 0 && WTN % 32 == 0, "tile shape");
  extern __shared__ u32x4 lds[];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = uni(tid / kWave);
  const int wm = wave / WGN, wn = wave % WGN;
  // Loads go straight from global memory into LDS (global_load_lds_dwordx4):
  // lane l of a wave writes the 16-byte slot l of the wave's 1 KB destination,
  // i.e. row lrow, slot lsl.  The slot is the XOR-swizzled position of chunk
  // lsl ^ swz(row), so that lane fetches that chunk from global memory.
  const int lrow = tid / CH, lsl = tid % CH;

  // Persistent grid: round r hands item r * G + slot to this workgroup; the
  // slots of one XCD are contiguous, so in every round the CUs of an XCD work
  // on a compact block of tiles and step through k together.
  const int slot = xcd_remap(blockIdx.x, gridDim.x);
  for (int item_id = slot; item_id < a.n_items; item_id += gridDim.x) {
  const TileItem it = a.items[item_id];
  int sexp = 0;
  if (!item_active<FUSED>(a, it, &sexp)) continue;

  const int j = it.out - 1;
  // operands of this item: the problem's descriptor (fused) or the launch fields
  const ProblemDesc* pd = FUSED ? a.probs + it.prob : nullptr;
  const LayerState* fst = FUSED ? pd->state : nullptr;
  const int64_t ld = FUSED ? pd->ld : a.ld;
  const int64_t kdim = FUSED ? pd->kdim : a.kdim;
  const int64_t pdim = FUSED ? pd->pdim : a.kdim;
  // second-order chain (fused only): X2 = S1_0 S1_0 + S S2 + S2 S
  const bool second = FUSED && it.out > 0 && j == fst->order2_slot;
  const int nprod = it.out == 0 ? 1 : (second ? 3 : 2);
  // operand panels per product p: Q<p> = [hi_A, lo_A, hi_B, lo_B]
  const uint16_t *Q0[4], *Q1[4], *Q2[4];
  float rescale = 1.0f;      // second order: 2^(e2 - 2 e1) after the S1_0 S1_0 product
  {
    const int sp = FUSED ? fst->s_par : 0;
    const int lp = FUSED ? ((fst->n - 1) & 1) : 0;   // S1_{n-1} split
    const uint16_t* sh = (const uint16_t*)(FUSED ? pd->s_hi[sp] : a.s_hi);
    const uint16_t* sl = (const uint16_t*)(FUSED ? pd->s_lo[sp] : a.s_lo);
    const uint16_t* th = sh;
    const uint16_t* tl = sl;
    if (it.out != 0) {
      th = (const uint16_t*)(FUSED ? pd->s1_hi[j][lp] : a.s1_hi[j]);
      tl = (const uint16_t*)(FUSED ? pd->s1_lo[j][lp] : a.s1_lo[j]);
    }
    // X: S S;  X1_j: S S1_j, S1_j S;  X2: S1_0 S1_0, S S2, S2 S
    const uint16_t* uh = sh;
    const uint16_t* ul = sl;
    if (second) {
      // S1_0 frozen at its D1 result S1_{d1-1} once its test fired
      const bool fz = fst->d1[0] != 0;
      const int fp = fz ? ((fst->d1_layer[0] - 1) & 1) : lp;
      const int e1 = fz ? fst->s1_exp_hist[0][fst->d1_layer[0] - 1] : fst->s1_exp_split[0];
      uh = (const uint16_t*)pd->s1_hi[0][fp];
      ul = (const uint16_t*)pd->s1_lo[0][fp];
      rescale = ldexpf(1.0f, sexp - 2 * e1);
    }
    if (second) {
      Q0[0] = uh; Q0[1] = ul; Q0[2] = uh; Q0[3] = ul;
      Q1[0] = sh; Q1[1] = sl; Q1[2] = th; Q1[3] = tl;
      Q2[0] = th; Q2[1] = tl; Q2[2] = sh; Q2[3] = sl;
    } else {
      Q0[0] = sh; Q0[1] = sl; Q0[2] = th; Q0[3] = tl;
      Q1[0] = th; Q1[1] = tl; Q1[2] = sh; Q1[3] = sl;
      Q2[0] = th; Q2[1] = tl; Q2[2] = sh; Q2[3] = sl;
    }
  }
  const int64_t row_a0 = (int64_t)it.ti * BM, row_b0 = (int64_t)it.tj * BN;
  const int kt_per = uni((int)(kdim / BK));
  const int ktiles = uni(nprod * kt_per);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Q0[r] = uni(Q0[r]);
    Q1[r] = uni(Q1[r]);
    Q2[r] = uni(Q2[r]);
  }

  // Operands are panel-major: the k-tile kt of row tile I is the contiguous
  // block (I * kblocks + kt) of kPanelRows x kPanelK elements.  Per-thread
  // offset inside a block; the swizzle of row i*RPL + lrow does not depend on
  // i, so every load round adds only a wave-uniform offset.
  static_assert(kPanelRows % BM == 0 && BK == kPanelK, "tile inside a panel block");
  static_assert((RPL >> SWZ) % CH == 0, "swizzle must repeat every load round");
  static_assert(STAGES == 2 && BK == 32, "two stages of two 16-wide k steps");
  const int64_t kblocks = uni(pdim / kPanelK);
  const int csrc = lsl ^ ((lrow >> SWZ) & (CH - 1));
  const int voff = lrow * kPanelK + csrc * 8;
  const int64_t offa = uni((row_a0 / kPanelRows) * kblocks * (kPanelRows * kPanelK) +
                           (row_a0 % kPanelRows) * kPanelK);
  const int64_t offb = uni((row_b0 / kPanelRows) * kblocks * (kPanelRows * kPanelK) +
                           (row_b0 % kPanelRows) * kPanelK);
  // Tile t of the concatenated k range goes to stage t % 2.  Past the end the
  // last tile is fetched again (into a stage nobody reads any more), so the
  // loop body has no branches.  One load round moves RPL rows of one array.
  struct Fetch { const uint16_t* q[4]; u32x4* dst; };
  auto prep = [&](int t0) {
    Fetch f;
    const int t = t0 < ktiles ? t0 : ktiles - 1;
    const int p = (t >= kt_per) + (t >= 2 * kt_per);
    const int64_t kofs = (int64_t)(t - p * kt_per) * (kPanelRows * kPanelK);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      f.q[r] = (p == 0 ? Q0[r] : (p == 1 ? Q1[r] : Q2[r])) + (r < 2 ? offa : offb) + kofs;
    f.dst = lds + (t0 & 1) * STAGE;
    return f;
  };
  auto issue_round = [&](const Fetch& f, int i) {
    const int arr = (i * RPL) / BM;               // compile-time after unrolling
    const uint16_t* basep = f.q[arr] + (i * RPL - arr * BM) * kPanelK;
    u32x4* dst = f.dst + (i * RPL + wave * RPW) * CH;                  // wave-uniform
    __builtin_amdgcn_global_load_lds((const void*)(basep + voff), (void*)dst, 16, 0, 0);
  };
  auto issue = [&](int t0) {
    const Fetch f = prep(t0);
#pragma unroll
    for (int i = 0; i < LOADS; ++i) issue_round(f, i);
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int m = 0; m < FM; ++m)
#pragma unroll
    for (int n = 0; n < FN; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.0f;

  // Fragments of one 16-wide k step: rows of A (hi, lo) and of B (hi, lo).
  // Fragment g: hi_A m = g, lo_A m = g - FM, hi_B n = g - 2 FM, lo_B n = g - 2 FM - FN.
  constexpr int NF = 2 * (FM + FN);              // LDS reads per k step
  constexpr int NM = 3 * FM * FN;                // MFMAs per k step
  struct Frag { V ah[FM], al[FM], bh[FN], bl[FN]; };
  auto read_one = [&](int stage, int kk, Frag& f, int g) {
    const u32x4* base = lds + stage * STAGE;
    const int c = kk * 2 + (lane >> 5);
    const bool a_side = g < 2 * FM;
    const int idx = a_side ? g % FM : (g - 2 * FM) % FN;
    const bool lo = a_side ? g >= FM : g >= 2 * FM + FN;
    const int R = (a_side ? wm * WTM + idx * 32 : 2 * BM + wn * WTN + idx * 32) + (lane & 31);
    const int cc = c ^ ((R >> SWZ) & (CH - 1));
    const V v = __builtin_bit_cast(V, base[(R + (lo ? BM : 0)) * CH + cc]);
    if (a_side) {
      if (lo) f.al[idx] = v; else f.ah[idx] = v;
    } else {
      if (lo) f.bl[idx] = v; else f.bh[idx] = v;
    }
  };
  auto read = [&](int stage, int kk, Frag& f) {
#pragma unroll
    for (int g = 0; g < NF; ++g) read_one(stage, kk, f, g);
  };
  // MFMA number q of a k step, per accumulator in the order hi*hi (A scaled
  // by 2^t), hi*lo, lo*hi: q = prod * FM * FN + m * FN + n.
  auto mma_one = [&](const Frag& f, V* as, int q) {
    const int prod = q / (FM * FN), m = (q / FN) % FM, n = q % FN;
    if (prod == 0) {
      if (n == 0) as[m] = S::up(f.ah[m]);
      acc[m][n] = S::mma(as[m], f.bh[n], acc[m][n]);
    } else if (prod == 1) {
      acc[m][n] = S::mma(f.ah[m], f.bl[n], acc[m][n]);
    } else {
      acc[m][n] = S::mma(f.al[m], f.bh[n], acc[m][n]);
    }
  };
  // One k step of MFMAs on cur, cut into NF groups; group g also reads
  // fragment g of nxt and, with a Fetch, issues its share of the load rounds.
  // The fences keep that interleave: a single wave per SIMD has no other wave
  // to cover a stall, so reads and loads go out in small doses between MFMAs.
  auto step = [&](const Frag& cur, Frag& nxt, int rstage, int rkk, const Fetch* fetch) {
    V as[FM];
#pragma unroll
    for (int g = 0; g < NF; ++g) {
      read_one(rstage, rkk, nxt, g);
      if (fetch) {
#pragma unroll
        for (int i = (g * LOADS) / NF; i < ((g + 1) * LOADS) / NF; ++i) issue_round(*fetch, i);
      }
#pragma unroll
      for (int q = (g * NM) / NF; q < ((g + 1) * NM) / NF; ++q) mma_one(cur, as, q);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // Software pipeline.  Global loads run one stage ahead; the fragments of the
  // next k step are read from LDS while the MFMAs of the current one run.  The
  // one barrier per k-tile sits between its two k steps: by then every wave
  // holds the second step's fragments (its stage may be refilled) and every
  // wave's loads of the next tile have landed (it may be read).
  static_assert(NM >= NF, "at least one MFMA per LDS read");
  Frag f0, f1;
  issue(0);
  issue(1);
  __builtin_amdgcn_s_waitcnt(VmWait<LOADS>::imm);
  __syncthreads();
  read(0, 0, f0);
  auto body = [&](int t) {
    // f0 was read during the previous k step and has landed: wait for it
    // before more reads are queued (the counter cannot express "all but NF")
    __builtin_amdgcn_s_waitcnt(LgkWait<0>::imm);
    step(f0, f1, t & 1, 1, nullptr);
    const Fetch fe = prep(t + 2);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    step(f1, f0, (t + 1) & 1, 0, &fe);
  };
  // second-order items: the S1_0 S1_0 product (scale 2^(t + 2 e1)) is brought
  // to the scale of S S2 before the other two are accumulated
  int t = 0;
  const int tsplit = second ? kt_per : 0;
  for (; t < tsplit; ++t) body(t);
  if (second) {
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
      for (int n = 0; n < FN; ++n)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[m][n][r] *= rescale;
  }
  for (; t < ktiles; ++t) body(t);
  // the refetches past the end land before the LDS is reused
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  const float scale = ldexpf(1.0f, -(S::kShift + sexp));
  const bool diag = it.ti == it.tj;
  if constexpr (!FUSED) {
  // epilogue: unscale, store the tile and its mirror image
  float* C = (float*)(it.out == 0 ? a.x : a.x1[j]);
#pragma unroll
  for (int m = 0; m < FM; ++m)
#pragma unroll
    for (int n = 0; n < FN; ++n) {
      const int64_t gc = row_b0 + wn * WTN + n * 32 + (lane & 31);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t gr0 = row_a0 + wm * WTM + m * 32 + 8 * g + 4 * (lane >> 5);
        f32x4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = acc[m][n][4 * g + r] * scale;
        if (!diag) {
#pragma unroll
          for (int r = 0; r < 4; ++r) C[(gr0 + r) * ld + gc] = v[r];
          *(f32x4*)(C + gc * ld + gr0) = v;
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t gr = gr0 + r;
            if (gr <= gc) C[gr * ld + gc] = v[r];
            if (gr < gc) C[gc * ld + gr] = v[r];
          }
        }
      }
    }
  } else {
  // Fused epilogue: the layer update of this tile and of its mirror image.
  // The tile goes through LDS (free after the main loop) in FM rounds: in
  // round m every wave parks its 32-row fragment strip m, row-major, and the
  // workgroup then updates those SR rows (direct block, row-major) and their
  // mirror columns (transposed reads), with coalesced global accesses.
  // Element (lr, lc) of the upper triangle stands for itself and its mirror,
  // so the norms weigh it 2 (off the diagonal) or 1 (on it).
  constexpr int SR = 32 * WGM;               // tile rows staged per round
  constexpr int PT = BN + 4;                 // LDS row pitch (floats)
  constexpr int ITER = SR * BN / (4 * NT);   // float4 groups per thread and round
  constexpr int G = ITER < 4 ? ITER : 4;
  static_assert(SR * BN % (4 * NT) == 0 && ITER % G == 0, "whole float4 groups per thread");
  static_assert(SR * PT * 4 <= STAGES * STAGE * 16, "staging fits in the operand LDS");
  float* T = (float*)lds;
  const int sig = fst->sigma_cur;
  const bool isx = it.out == 0;
  const bool upd = isx ? fst->upd_s0 != 0 : true;
  // ||S - X||_F^2 at the D0 layer, ||S1_j - X1_j||_F^2 once D0 converged
  const bool diff = isx ? !upd : fst->d0 != 0;
  const bool need_old = diff || sig < 0;
  const int cur = fst->n & 1;
  const float* Mr = isx ? pd->s_master : pd->s1m[j][cur ^ 1];
  float* Mw = isx ? pd->s_master : pd->s1m[j][cur];
  uint16_t* Hw = (uint16_t*)(isx ? pd->s_hi[fst->s_par ^ 1] : pd->s1_hi[j][cur]);
  uint16_t* Lw = (uint16_t*)(isx ? pd->s_lo[fst->s_par ^ 1] : pd->s1_lo[j][cur]);
  const int esplit = isx ? 0 : fst->s1_exp_next[j];
  typedef uint16_t U4 __attribute__((ext_vector_type(4)));
  double pf = 0.0;
  float pm = 0.0f;
#pragma unroll
  for (int m = 0; m < FM; ++m) {
    // park: wave (wm, wn) writes rows wm*32 + [0, 32) of T, columns of its fragments
#pragma unroll
    for (int n = 0; n < FN; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        T[row * PT + wn * WTN + n * 32 + (lane & 31)] = acc[m][n][r] * scale;
      }
    __syncthreads();
    // direct block: T row tr is tile row (tr / 32) * WTM + m * 32 + tr % 32.
    // Groups of G float4 per thread: the G old-value loads go out together.
#pragma unroll 1
    for (int g0 = 0; g0 < ITER; g0 += G) {
      f32x4 sov[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int e = (tid + (g0 + i) * NT) * 4;
        const int tr = e / BN, lc = e % BN;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        sov[i] = need_old ? *(const f32x4*)(Mr + (row_a0 + lr) * ld + row_b0 + lc)
                          : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int e = (tid + (g0 + i) * NT) * 4;
        const int tr = e / BN, lc = e % BN;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        const f32x4 x = *(const f32x4*)(T + tr * PT + lc);
        const int64_t grow = row_a0 + lr, gcol = row_b0 + lc;
        const f32x4 so = sov[i];
        f32x4 sn;
        uint16_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sn[q] = sig > 0 ? x[q] : 2.0f * so[q] - x[q];
          const int c = lc + q;
          const double w = diag ? (lr < c ? 2.0 : (lr == c ? 1.0 : 0.0)) : 2.0;
          const double d = (double)so[q] - (double)x[q];
          if (diff) pf += w * d * d;
          if (w > 0.0) pm = fmaxf(pm, fabsf(sn[q]));
          split_one<T16>(sn[q], esplit, S::kShift, h + q, l + q);
        }
        if (!upd) continue;
        *(f32x4*)(T + tr * PT + lc) = sn;      // for the mirror pass
        const int64_t pi = panel_index(grow, gcol, pdim);   // four columns, one panel row
        if (!diag || lr < lc) {
          *(f32x4*)(Mw + grow * ld + gcol) = sn;
          *(U4*)(Hw + pi) = U4{h[0], h[1], h[2], h[3]};
          *(U4*)(Lw + pi) = U4{l[0], l[1], l[2], l[3]};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (lr <= lc + q) {
              Mw[grow * ld + gcol + q] = sn[q];
              Hw[pi + q] = h[q];
              Lw[pi + q] = l[q];
            }
        }
      }
    }
    __syncthreads();
    // mirror block: row lc of the mirror gets T rows 4 qd .. 4 qd + 3 of column lc
    if (upd) {
      for (int e = tid; e < BN * (SR / 4); e += NT) {
        const int qd = e % (SR / 4), lc = e / (SR / 4);
        const int tr = 4 * qd;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        if (diag && lr >= lc) continue;        // lr + q < lc for some q needs lr < lc
        f32x4 v;
        uint16_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          v[q] = T[(tr + q) * PT + lc];
          split_one<T16>(v[q], esplit, S::kShift, h + q, l + q);
        }
        const int64_t grow = row_b0 + lc, gcol = row_a0 + lr;
        const int64_t pi = panel_index(grow, gcol, pdim);
        if (!diag || lr + 3 < lc) {
          *(f32x4*)(Mw + grow * ld + gcol) = v;
          *(U4*)(Hw + pi) = U4{h[0], h[1], h[2], h[3]};
          *(U4*)(Lw + pi) = U4{l[0], l[1], l[2], l[3]};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (lr + q < lc) {
              Mw[grow * ld + gcol + q] = v[q];
              Hw[pi + q] = h[q];
              Lw[pi + q] = l[q];
            }
        }
      }
      __syncthreads();
    }
  }
  // workgroup partials in a fixed order: butterfly within each wave, then the
  // waves in index order
  __shared__ double red_f[WGM * WGN];
  __shared__ float red_m[WGM * WGN];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    pf += __shfl_xor(pf, o);
    pm = fmaxf(pm, __shfl_xor(pm, o));
  }
  if (lane == 0) {
    red_f[wave] = pf;
    red_m[wave] = pm;
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    float mx = 0.0f;
#pragma unroll
    for (int w = 0; w < WGM * WGN; ++w) {
      f += red_f[w];
      mx = fmaxf(mx, red_m[w]);
    }
    a.part_f[a.slot_base + item_id] = f;
    a.part_m[a.slot_base + item_id] = (double)mx;
  }
  }
  }  // items
}

// ------------------------------------------------------------------ batched pairs
// Barrier for hand-offs through the LDS: this wave's LDS accesses have
// completed and the compiler keeps memory accesses on their side of it.
// Outstanding global stores and direct-to-LDS loads are not waited for (a
// workgroup fence would wait for all of them); callers wait for their loads
// explicitly.  Global memory written in a launch is not read back in it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(LgkWait<0>::imm);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Memory that no kernel writes while the product launch runs (the items, the
// problem descriptors, the layer states, which the decision kernels write
// between launches), read through the constant address space: workgroup-
// uniform reads then become scalar loads, which do not queue behind the
// vector loads in flight and are not counted with them.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cst(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Fused layer products on items of two 128 x 128 tiles that share a band:
// (ti, tj) and (ti, tj2) read the same A panels (rows of S, or of S1_j for the
// second product of a response), (ti, tj) and (ti2, tj) the same B panels.
// One k-tile then loads the shared panels once for both tiles, 48 KB for 96
// MFMAs per wave pair instead of 64 KB.  Eight waves of 64 x 64 (waves with
// wn < 2 hold tile (ti, tj), the others the second tile), one
// workgroup per CU and three LDS stages, so the loads of k-tile t + 3 go out
// while tile t is multiplied and are waited for two tiles later: the batch's
// small problems miss the L2 often, and one tile of lead time does not cover
// that latency.  No barrier waits for global stores or for loads beyond the
// one the pipeline needs (lds_barrier).  A tile without a partner (ti2 < 0)
// loads its panels as a row pair whose second B panel repeats the first, and
// the waves of the right half only load and wait.  First-order items only
// (X and X1_j).
template <typename T16, int SWZ>
__global__ void __launch_bounds__(8 * kWave)
k_products_pair(const ProductArgs a) {
  using S = Split16<T16>;
  using V = typename S::V;
  constexpr int BM = 128, BK = kPanelK, WGM = 2, WGN = 4, STAGES = 3;
  constexpr int NT = WGM * WGN * kWave;
  constexpr int WTM = 64, WTN = 64, FM = WTM / 32, FN = WTN / 32;
  constexpr int CH = BK / 8;                 // 16-byte chunks per row of a k-tile
  constexpr int NARR = 6;                    // X_hi | X_lo | Y0_hi | Y0_lo | Y1_hi | Y1_lo
                                             // X: the shared panel, Y_h: tile h's other one
  constexpr int STAGE = NARR * BM * CH;      // chunks per pipeline stage
  constexpr int RPW = kWave / CH;            // rows one wave fills per load instruction
  constexpr int RPL = NT / CH;               // rows all waves fill per load round
  constexpr int LOADS = NARR;                // load rounds per k-tile, one per array
  constexpr int BN = 2 * BM;                 // columns of a pair
  constexpr int SR = 32 * WGM;               // epilogue: tile rows staged per round
  constexpr int PT = BN + 4;                 // epilogue: LDS row pitch (floats)
  static_assert(RPL == BM, "one load round fills one array");
  static_assert((RPL >> SWZ) % CH == 0, "swizzle must repeat every load round");
  static_assert(kPanelRows % BM == 0 && BK == 32, "tile inside a panel block, two k steps");
  static_assert(SR * PT * 4 <= STAGES * STAGE * 16, "epilogue staging fits in the operand LDS");
  extern __shared__ u32x4 lds[];

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = uni(tid / kWave);
  const int wm = wave / WGN, wn = wave % WGN;
  const int half = wn >> 1;
  // Loads go straight from global memory into LDS: lane l of a wave writes
  // 16-byte slot l of the wave's 1 KB destination (row lrow, slot lsl) and
  // fetches the chunk whose XOR-swizzled position that slot is.
  const int lrow = tid / CH, lsl = tid % CH;
  const int csrc = lsl ^ ((lrow >> SWZ) & (CH - 1));
  const int voff = lrow * kPanelK + csrc * 8;

  // Operands of one item: the split of S and of T = S1_j (X: T = S); product 0
  // is S T, product 1 (responses) T S.  Panel-major storage: the k-tile kt of
  // row tile I is the contiguous block I * kblocks + kt of kPanelRows x
  // kPanelK elements.
  struct Ops {
    TileItem it;
    int sexp, kt_per, ktiles, colp;            // colp: the tiles share their B panels
    const uint16_t* q[4];                      // hi_S, lo_S, hi_T, lo_T (T = S1_j or S)
    int64_t offx, offy0, offy1;
  };
  // The first item at or after position id (stepping by the grid) with work
  // to do; false if there is none.
  auto find = [&](int& id, Ops& o) -> bool {
    for (; id < a.n_items; id += gridDim.x) {
      // the item as five words (out | prob << 16, ti, tj, ti2, tj2)
      const auto* w = cst((const uint32_t*)(a.items + id));
      const uint32_t w0 = w[0];
      o.it.out = (int16_t)(w0 & 0xffffu);
      o.it.prob = (int16_t)(w0 >> 16);
      o.it.ti = (int32_t)w[1];
      o.it.tj = (int32_t)w[2];
      o.it.ti2 = (int32_t)w[3];
      o.it.tj2 = (int32_t)w[4];
      if (o.it.out < 0) continue;               // placeholder of a balanced round
      const auto* pd = cst(a.probs + o.it.prob);
      const auto* fst = cst(pd->state);
      const int j = o.it.out - 1;
      // skip flags as in item_active (fused launch)
      if (fst->done) continue;
      if (o.it.out == 0 ? (fst->d0 && !fst->d0_now) : fst->d1[j] != 0) continue;
      o.sexp = o.it.out == 0 ? 0 : fst->s1_exp_split[j];
      const int sp = fst->s_par;
      const int lp = (fst->n - 1) & 1;         // S1_{n-1} split
      const uint16_t* sh = (const uint16_t*)pd->s_hi[sp];
      const uint16_t* sl = (const uint16_t*)pd->s_lo[sp];
      const uint16_t* th = o.it.out != 0 ? (const uint16_t*)pd->s1_hi[j][lp] : sh;
      const uint16_t* tl = o.it.out != 0 ? (const uint16_t*)pd->s1_lo[j][lp] : sl;
      o.q[0] = sh; o.q[1] = sl; o.q[2] = th; o.q[3] = tl;
      const int64_t kblocks = uni(pd->pdim / kPanelK);
      auto block_of = [&](int64_t r0) {
        return uni((r0 / kPanelRows) * kblocks * (kPanelRows * kPanelK) + (r0 % kPanelRows) * kPanelK);
      };
      const int ti = uni(o.it.ti), tj = uni(o.it.tj);
      const int ti2 = uni(o.it.ti2), tj2 = uni(o.it.tj2);
      o.colp = ti2 >= 0 && ti2 != ti;
      o.offx = block_of((int64_t)(o.colp ? tj : ti) * BM);
      o.offy0 = block_of((int64_t)(o.colp ? ti : tj) * BM);
      o.offy1 = block_of((int64_t)(ti2 < 0 ? tj : (o.colp ? ti2 : tj2)) * BM);
      o.kt_per = uni((int)(pd->kdim / BK));
      o.ktiles = uni((o.it.out == 0 ? 1 : 2) * o.kt_per);
      return true;
    }
    return false;
  };
  // The fetch plan of the current item, read into scalar registers once per
  // item: values carried across the item loop can end up in vector registers,
  // and every load would then form its address per lane.
  struct Plan {
    const uint16_t* q[4];
    int64_t offx, offy0, offy1;
    int kt_per, ktiles, colp;
  };
  auto plan_of = [&](const Ops& o) {
    Plan pl;
#pragma unroll
    for (int r = 0; r < 4; ++r) pl.q[r] = uni(o.q[r]);
    pl.offx = uni(o.offx);
    pl.offy0 = uni(o.offy0);
    pl.offy1 = uni(o.offy1);
    pl.kt_per = uni(o.kt_per);
    pl.ktiles = uni(o.ktiles);
    pl.colp = uni(o.colp);
    return pl;
  };
  // k-tile t0 of an item; past the end the last tile is fetched again into a
  // stage nobody reads any more.  One load round moves one array.
  struct Fetch { const uint16_t* q[NARR]; u32x4* dst; };
  auto prep = [&](const Plan& o, int t0) {
    Fetch f;
    const int t = t0 < o.ktiles ? t0 : o.ktiles - 1;
    const int p = t >= o.kt_per;               // product 1: A = T, B = S
    const int64_t kofs = (int64_t)(t - p * o.kt_per) * (kPanelRows * kPanelK);
    const uint16_t* ah = p ? o.q[2] : o.q[0];
    const uint16_t* al = p ? o.q[3] : o.q[1];
    const uint16_t* bh = p ? o.q[0] : o.q[2];
    const uint16_t* bl = p ? o.q[1] : o.q[3];
    const uint16_t* xh = o.colp ? bh : ah;
    const uint16_t* xl = o.colp ? bl : al;
    const uint16_t* yh = o.colp ? ah : bh;
    const uint16_t* yl = o.colp ? al : bl;
    f.q[0] = xh + o.offx + kofs;
    f.q[1] = xl + o.offx + kofs;
    f.q[2] = yh + o.offy0 + kofs;
    f.q[3] = yl + o.offy0 + kofs;
    f.q[4] = yh + o.offy1 + kofs;
    f.q[5] = yl + o.offy1 + kofs;
    f.dst = lds + (t0 % STAGES) * STAGE;
    return f;
  };
  auto issue_round = [&](const Fetch& f, int i) {
    u32x4* dst = f.dst + (i * RPL + wave * RPW) * CH;                  // wave-uniform
    __builtin_amdgcn_global_load_lds((const void*)(f.q[i] + voff), (void*)dst, 16, 0, 0);
  };
  auto issue = [&](const Plan& o, int t0) {
    const Fetch f = prep(o, t0);
#pragma unroll
    for (int i = 0; i < LOADS; ++i) issue_round(f, i);
  };

  // Fragment g of a 16-wide k step: hi_A m = g, lo_A m = g - FM,
  // hi_B n = g - 2 FM, lo_B n = g - 2 FM - FN (B from this wave's half).
  constexpr int NF = 2 * (FM + FN);
  constexpr int NM = 3 * FM * FN;
  static_assert(NM >= NF, "at least one MFMA per LDS read");
  struct Frag { V ah[FM], al[FM], bh[FN], bl[FN]; };
  // first LDS row of the A and of the B panels of this wave's tile (hi; lo
  // follows BM rows later), set per item: the shared panel sits in arrays 0-1
  int rowA = 0, rowB = 0;
  auto read_one = [&](int stage, int kk, Frag& f, int g) {
    const u32x4* base = lds + stage * STAGE;
    const int c = kk * 2 + (lane >> 5);
    const bool a_side = g < 2 * FM;
    const int idx = a_side ? g % FM : (g - 2 * FM) % FN;
    const bool lo = a_side ? g >= FM : g >= 2 * FM + FN;
    const int rin = (a_side ? wm * WTM : (wn & 1) * WTN) + idx * 32 + (lane & 31);
    // the array offsets are multiples of BM rows, which the swizzle ignores
    const int cc = c ^ ((rin >> SWZ) & (CH - 1));
    const int R = (a_side ? rowA : rowB) + (lo ? BM : 0) + rin;
    const V v = __builtin_bit_cast(V, base[R * CH + cc]);
    if (a_side) {
      if (lo) f.al[idx] = v; else f.ah[idx] = v;
    } else {
      if (lo) f.bl[idx] = v; else f.bh[idx] = v;
    }
  };
  auto read = [&](int stage, int kk, Frag& f) {
#pragma unroll
    for (int g = 0; g < NF; ++g) read_one(stage, kk, f, g);
  };

  // Persistent grid: round r hands item r * G + slot to this workgroup; the
  // slots of one XCD are contiguous.
  const int slot = xcd_remap(blockIdx.x, gridDim.x);
  Ops cur;
  for (int id = slot; find(id, cur); id += gridDim.x) {
  const Plan pl = plan_of(cur);
  const TileItem it = cur.it;
  const int j = it.out - 1;
  const auto* pd = cst(a.probs + it.prob);
  const auto* fst = cst(pd->state);
  const int64_t ld = pd->ld, pdim = pd->pdim;
  // rows and columns from kdim on stay zero (cleared at set-up; X = S^2 and
  // the update keep them zero), so the epilogue neither reads nor stores them
  const int64_t kd = pd->kdim;
  const int ti2 = uni(it.ti2), tj2 = uni(it.tj2);
  const bool single = ti2 < 0;
  const bool live = !(single && half);       // wave-uniform
  rowA = pl.colp ? (2 + 2 * half) * BM : 0;
  rowB = pl.colp ? 0 : (2 + 2 * half) * BM;
  // origin of tile h: rows r0_h, columns c0_h
  const int64_t r0_0 = (int64_t)uni(it.ti) * BM, c0_0 = (int64_t)uni(it.tj) * BM;
  const int64_t r0_1 = single ? r0_0 : (int64_t)ti2 * BM;
  const int64_t c0_1 = single ? c0_0 : (int64_t)tj2 * BM;
  const int ktiles = pl.ktiles;

  f32x16 acc[FM][FN];
#pragma unroll
  for (int m = 0; m < FM; ++m)
#pragma unroll
    for (int n = 0; n < FN; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][n][r] = 0.0f;

  // MFMA q of a k step, per accumulator in the order hi*hi (A scaled by 2^t),
  // hi*lo, lo*hi: q = prod * FM * FN + m * FN + n.
  auto mma_one = [&](const Frag& f, V* as, int q) {
    const int prod = q / (FM * FN), m = (q / FN) % FM, n = q % FN;
    if (prod == 0) {
      if (n == 0) as[m] = S::up(f.ah[m]);
      acc[m][n] = S::mma(as[m], f.bh[n], acc[m][n]);
    } else if (prod == 1) {
      acc[m][n] = S::mma(f.ah[m], f.bl[n], acc[m][n]);
    } else {
      acc[m][n] = S::mma(f.al[m], f.bh[n], acc[m][n]);
    }
  };
  // One k step of MFMAs on cur in NF groups; group g also reads fragment g of
  // nxt and issues its share of the load rounds.
  auto step = [&](const Frag& fc, Frag& fn, int rstage, int rkk, const Fetch* fetch) {
    V as[FM];
#pragma unroll
    for (int g = 0; g < NF; ++g) {
      read_one(rstage, rkk, fn, g);
      if (fetch) {
#pragma unroll
        for (int i = (g * LOADS) / NF; i < ((g + 1) * LOADS) / NF; ++i) issue_round(*fetch, i);
      }
#pragma unroll
      for (int q = (g * NM) / NF; q < ((g + 1) * NM) / NF; ++q) mma_one(fc, as, q);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // Software pipeline over three stages.  At the barrier in the middle of k-tile t every wave has read all of tile t
  // (its stage may be refilled) and its loads of tile t + 1 have landed
  // (loads complete in order: only tile t + 2's may still be outstanding);
  // the loads of tile t + 3 then go out.  Waves without a tile run the same
  // loads and barriers and nothing else (a separate copy of the loop, so that
  // no branch sits between the MFMAs).
  issue(pl, 0);
  issue(pl, 1);
  issue(pl, 2);
  __builtin_amdgcn_s_waitcnt(VmWait<2 * LOADS>::imm);
  lds_barrier();
  if (live) {
    Frag f0, f1;
    read(0, 0, f0);
#pragma unroll 1
    for (int t = 0; t < ktiles; ++t) {
      __builtin_amdgcn_s_waitcnt(LgkWait<0>::imm);
      step(f0, f1, t % STAGES, 1, nullptr);
      const Fetch fe = prep(pl, t + 3);
      __builtin_amdgcn_s_waitcnt(VmWait<LOADS>::imm);
      lds_barrier();
      step(f1, f0, (t + 1) % STAGES, 0, &fe);
    }
  } else {
#pragma unroll 1
    for (int t = 0; t < ktiles; ++t) {
      const Fetch fe = prep(pl, t + 3);
      __builtin_amdgcn_s_waitcnt(VmWait<LOADS>::imm);
      lds_barrier();
#pragma unroll
      for (int i = 0; i < LOADS; ++i) issue_round(fe, i);
    }
  }
  // the refetches past the end land before the LDS is reused
  __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();

  // Fused epilogue, as in k_products_split, over the 256 staged columns of the
  // pair: column lc is column lc % 128 of tile lc / 128 (at r0_h, c0_h).
  const float scale = ldexpf(1.0f, -(S::kShift + cur.sexp));
  const bool diag0 = r0_0 == c0_0, diag1 = r0_1 == c0_1;
  constexpr int ITER = SR * BN / (4 * NT);   // float4 groups per thread and round
  constexpr int G = ITER < 4 ? ITER : 4;
  static_assert(SR * BN % (4 * NT) == 0 && ITER % G == 0, "whole float4 groups per thread");
  float* T = (float*)lds;
  const int sig = fst->sigma_cur;
  const bool isx = it.out == 0;
  const bool upd = isx ? fst->upd_s0 != 0 : true;
  const bool diff = isx ? !upd : fst->d0 != 0;
  const bool need_old = diff || sig < 0;
  const int cpar = fst->n & 1;
  const float* Mr = isx ? pd->s_master : pd->s1m[j][cpar ^ 1];
  float* Mw = isx ? pd->s_master : pd->s1m[j][cpar];
  uint16_t* Hw = (uint16_t*)(isx ? pd->s_hi[fst->s_par ^ 1] : pd->s1_hi[j][cpar]);
  uint16_t* Lw = (uint16_t*)(isx ? pd->s_lo[fst->s_par ^ 1] : pd->s1_lo[j][cpar]);
  const int esplit = isx ? 0 : fst->s1_exp_next[j];
  typedef uint16_t U4 __attribute__((ext_vector_type(4)));
  double pf = 0.0;
  float pm = 0.0f;
#pragma unroll
  for (int m = 0; m < FM; ++m) {
    if (live) {
#pragma unroll
      for (int n = 0; n < FN; ++n)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          T[row * PT + wn * WTN + n * 32 + (lane & 31)] = acc[m][n][r] * scale;
        }
    }
    lds_barrier();
    // direct block: T row tr is tile row (tr / 32) * WTM + m * 32 + tr % 32;
    // a thread's column lc is the same in every group (NT * 4 is a multiple of BN)
#pragma unroll 1
    for (int g0 = 0; g0 < ITER; g0 += G) {
      f32x4 sov[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int e = (tid + (g0 + i) * NT) * 4;
        const int tr = e / BN, lc = e % BN;
        const int h = lc / BM, lcl = lc % BM;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        const int64_t grow = (h ? r0_1 : r0_0) + lr, gcol = (h ? c0_1 : c0_0) + lcl;
        sov[i] = (need_old && !(single && h) && grow < kd && gcol < kd)
                     ? *(const f32x4*)(Mr + grow * ld + gcol)
                     : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      }
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int e = (tid + (g0 + i) * NT) * 4;
        const int tr = e / BN, lc = e % BN;
        const int h = lc / BM, lcl = lc % BM;
        if (single && h) continue;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        const int64_t grow = (h ? r0_1 : r0_0) + lr, gcol = (h ? c0_1 : c0_0) + lcl;
        // four columns from a multiple of 4: wholly inside kd or wholly past it
        // (X is zero there, so the partials would gain exact zeros)
        if (grow >= kd || gcol >= kd) continue;
        const bool diag = h ? diag1 : diag0;
        const f32x4 x = *(const f32x4*)(T + tr * PT + lc);
        const f32x4 so = sov[i];
        f32x4 sn;
        uint16_t hh[4], ll[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          sn[q] = sig > 0 ? x[q] : 2.0f * so[q] - x[q];
          const int c = lcl + q;
          const double w = diag ? (lr < c ? 2.0 : (lr == c ? 1.0 : 0.0)) : 2.0;
          const double d = (double)so[q] - (double)x[q];
          if (diff) pf += w * d * d;
          if (w > 0.0) pm = fmaxf(pm, fabsf(sn[q]));
          split_one<T16>(sn[q], esplit, S::kShift, hh + q, ll + q);
        }
        if (!upd) continue;
        // for the mirror pass: the splits, packed hi << 16 | lo, in place of X
        typedef uint32_t P4 __attribute__((ext_vector_type(4)));
        *(P4*)(T + tr * PT + lc) = P4{((uint32_t)hh[0] << 16) | ll[0], ((uint32_t)hh[1] << 16) | ll[1],
                                      ((uint32_t)hh[2] << 16) | ll[2], ((uint32_t)hh[3] << 16) | ll[3]};
        const int64_t pi = panel_index(grow, gcol, pdim);   // four columns, one panel row
        if (!diag || lr < lcl) {
          *(f32x4*)(Mw + grow * ld + gcol) = sn;
          *(U4*)(Hw + pi) = U4{hh[0], hh[1], hh[2], hh[3]};
          *(U4*)(Lw + pi) = U4{ll[0], ll[1], ll[2], ll[3]};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (lr <= lcl + q) {
              Mw[grow * ld + gcol + q] = sn[q];
              Hw[pi + q] = hh[q];
              Lw[pi + q] = ll[q];
            }
        }
      }
    }
    lds_barrier();
    // mirror block: row lc of the mirror gets T rows 4 qd .. 4 qd + 3 of column
    // lc, in the 16-bit splits only (the next products read whole row panels,
    // and the direct block left the splits in T);
    // the FP32 masters are read only on upper tiles, and the outputs are
    // mirrored when they are copied out
    if (upd) {
      for (int e = tid; e < BN * (SR / 4); e += NT) {
        const int qd = e % (SR / 4), lc = e / (SR / 4);
        const int h = lc / BM, lcl = lc % BM;
        if (single && h) continue;
        const bool diag = h ? diag1 : diag0;
        const int tr = 4 * qd;
        const int lr = (tr >> 5) * WTM + m * 32 + (tr & 31);
        if (diag && lr >= lcl) continue;       // lr + q < lcl for some q needs lr < lcl
        const int64_t grow = (h ? c0_1 : c0_0) + lcl, gcol = (h ? r0_1 : r0_0) + lr;
        if (grow >= kd || gcol >= kd) continue;  // T holds splits only where the direct block ran
        uint16_t hh[4], ll[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t u = __builtin_bit_cast(uint32_t, T[(tr + q) * PT + lc]);
          hh[q] = (uint16_t)(u >> 16);
          ll[q] = (uint16_t)(u & 0xffffu);
        }
        const int64_t pi = panel_index(grow, gcol, pdim);
        if (!diag || lr + 3 < lcl) {
          *(U4*)(Hw + pi) = U4{hh[0], hh[1], hh[2], hh[3]};
          *(U4*)(Lw + pi) = U4{ll[0], ll[1], ll[2], ll[3]};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (lr + q < lcl) {
              Hw[pi + q] = hh[q];
              Lw[pi + q] = ll[q];
            }
        }
      }
      lds_barrier();
    }
  }
  // workgroup partials in a fixed order: butterfly within each wave, then the
  // waves in index order
  __shared__ double red_f[WGM * WGN];
  __shared__ float red_m[WGM * WGN];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    pf += __shfl_xor(pf, o);
    pm = fmaxf(pm, __shfl_xor(pm, o));
  }
  if (lane == 0) {
    red_f[wave] = pf;
    red_m[wave] = pm;
  }
  lds_barrier();
  if (tid == 0) {
    double f = 0.0;
    float mx = 0.0f;
#pragma unroll
    for (int w = 0; w < WGM * WGN; ++w) {
      f += red_f[w];
      mx = fmaxf(mx, red_m[w]);
    }
    a.part_f[a.slot_base + id] = f;
    a.part_m[a.slot_base + id] = (double)mx;
  }
  }  // items
}

// ------------------------------------------------------------------ direct forms
template <typename T> struct Direct;
// Output element r of lane l sits in column l % 16 and in row
//   4 (l / 16) + r   for the f32 form,
//   l / 16 + 4 r     for the f64 form (rows interleaved).
template <> struct Direct<float> {
  typedef f32x4 Acc;
  static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Direct<double> {
  typedef f64x4 Acc;
  static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Same tiling with one operand copy per matrix and the 16x16x4 MFMA: a lane
// reads one 16-byte chunk (E consecutive k) per fragment and issues E MFMAs,
// the e-th taking element e; A and B use the same (lane group, e) -> k map.
// WPE waves per SIMD (4 WPE / (WGM WGN) workgroups per CU).  Operands go
// straight from global memory into LDS, two stages of BK-wide k-tiles.
//
// FLUSH > 0: blocked accumulation.  The FP32 16x16x4 MFMA adds its four
// products one at a time, each rounded to FP32 and then added with one more
// rounding, so one accumulator running over the whole k range takes 2 kdim
// roundings at the size of the full sum.  With FLUSH, the MFMAs accumulate
// FLUSH k-tiles from zero, and that partial sum is added to a second
// accumulator (one FP32 addition) before the next chunk starts: the error of
// a long sum then grows with FLUSH BK + kdim / (FLUSH BK) instead of kdim.
template <typename T, int BM, int BK, int WGM, int WGN, int SWZ, int WPE, int FLUSH = 0>
__global__ void __launch_bounds__(WGM * WGN * kWave) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_products_direct(const ProductArgs a) {
  using D = Direct<T>;
  using Acc = typename D::Acc;
  constexpr int E = 16 / sizeof(T);
  constexpr int NT = WGM * WGN * kWave;
  constexpr int BN = BM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int CH = BK / E;
  constexpr int ROWS = BM + BN;              // A | B
  constexpr int STAGE = ROWS * CH;
  constexpr int RPL = NT / CH;
  constexpr int LOADS = ROWS / RPL;
  static_assert(ROWS % RPL == 0 && BM % RPL == 0, "load rounds must not straddle arrays");
  static_assert(CH % 4 == 0, "k-tile must hold a multiple of 4 chunks");
  extern __shared__ u32x4 lds[];

  const int slot = xcd_remap(blockIdx.x, gridDim.x);
  for (int item_id = slot; item_id < a.n_items; item_id += gridDim.x) {
  const TileItem it = a.items[item_id];
  int sexp = 0;
  if (!item_active<false>(a, it, &sexp)) continue;
  (void)sexp;  // direct forms store S1 unscaled

  const int64_t ld = a.ld;
  const int j = it.out - 1;
  // the second-order chain: X2 = S1_0 S1_0 + S S2 + S2 S (S2 = s1_hi[j])
  const bool second = a.mode == 0 && it.out > 0 && a.state && j == a.state->order2_slot;
  const int nprod = (a.mode != 0 || it.out == 0) ? 1 : (second ? 3 : 2);
  const bool each = a.mode == 3;               // one product per output, every tile
  // out 0: S S;  out 1 + j: A B + B A with A = a_op[j] (default S), B = s1_hi[j];
  // X2: S1_0 S1_0, S S2, S2 S.  Operands of product p: [A rows, B rows].
  const T *Q0[2], *Q1[2], *Q2[2];
  {
    const T* s = (const T*)a.s_hi;
    const T* aa = s;
    const T* bb = s;
    if (each) {
      aa = a.a_op[j] ? (const T*)a.a_op[j] : s;   // output 1 + j: A_j B_j
      bb = (const T*)a.s1_hi[j];
    } else if (a.mode != 0) {
      aa = s;                                  // one product A B, A = s_hi, B = s1_hi[0]
      bb = (const T*)a.s1_hi[0];
    } else if (it.out != 0) {
      aa = a.a_op[j] ? (const T*)a.a_op[j] : s;
      bb = (const T*)a.s1_hi[j];
    }
    if (second) {
      // these products run before the layer's decisions: S1_{n-1} sits in
      // buffer state->n & 1, or S1_0 is frozen at S1_{d1-1}
      const LayerState* st = a.state;
      const int fp = st->d1[0] ? ((st->d1_layer[0] - 1) & 1) : (st->n & 1);
      const T* u = (const T*)a.s1b[fp];
      Q0[0] = u; Q0[1] = u; Q1[0] = s; Q1[1] = bb; Q2[0] = bb; Q2[1] = s;
    } else {
      Q0[0] = aa; Q0[1] = bb; Q1[0] = bb; Q1[1] = aa; Q2[0] = bb; Q2[1] = aa;
    }
  }
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lrow = tid / CH, lch = tid % CH;
  const int64_t row_a0 = (int64_t)it.ti * BM, row_b0 = (int64_t)it.tj * BN;
  const int kt_per = (int)(a.kdim / BK);
  const int ktiles = nprod * kt_per;

  // In load round i, lane l of wave w writes 16-byte slot l of the wave's
  // 1 KB block (global_load_lds_dwordx4), i.e. row i * RPL + lrow, slot lch,
  // so it fetches the chunk whose swizzled position that slot is; the swizzle
  // of a row does not depend on i.
  static_assert(((RPL >> SWZ) % CH) == 0, "swizzle must repeat every load round");
  static_assert(kWave % CH == 0, "a wave fills whole rows");
  const int wave_u = uni(wave);
  const int csrc = lch ^ ((lrow >> SWZ) & (CH - 1));
  auto issue = [&](int t) {
    const int p = t / kt_per;
    const int64_t k0 = (int64_t)(t - p * kt_per) * BK;
    u32x4* stage = lds + (t & 1) * STAGE;
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int arr = (i * RPL) / BM;             // compile-time after unrolling
      const int r = i * RPL - arr * BM + lrow;
      const int64_t grow = (arr == 0 ? row_a0 : row_b0) + r;
      const T* basep = p == 0 ? Q0[arr] : (p == 1 ? Q1[arr] : Q2[arr]);
      const T* src = basep + grow * ld + k0 + csrc * E;
      u32x4* dst = stage + (i * RPL + wave_u * (kWave / CH)) * CH;     // wave-uniform
      __builtin_amdgcn_global_load_lds((const void*)src, (void*)dst, 16, 0, 0);
    }
  };

  Acc acc[FM][FN], tot[FLUSH > 0 ? FM : 1][FLUSH > 0 ? FN : 1];
#pragma unroll
  for (int m = 0; m < FM; ++m)
#pragma unroll
    for (int n = 0; n < FN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = (T)0;
  if constexpr (FLUSH > 0) {
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
      for (int n = 0; n < FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[m][n][r] = (T)0;
  }
  // chunk sum into the running total (FLUSH > 0 only)
  auto flush = [&]() {
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
      for (int n = 0; n < FN; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tot[m][n][r] += acc[m][n][r];
          acc[m][n][r] = (T)0;
        }
  };

  issue(0);
  __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
  __syncthreads();
  for (int t = 0; t < ktiles; ++t) {
    const int cur = t & 1;
    // tile t + 1 goes to the stage that tile t - 1 used (every wave has left it)
    if (t + 1 < ktiles) issue(t + 1);
    const u32x4* base = lds + cur * STAGE;
#pragma unroll
    for (int kk = 0; kk < CH / 4; ++kk) {
      const int c = kk * 4 + (lane >> 4);
      u32x4 af[FM], bf[FN];
#pragma unroll
      for (int m = 0; m < FM; ++m) {
        const int R = wm * WTM + m * 16 + (lane & 15);
        af[m] = base[R * CH + (c ^ ((R >> SWZ) & (CH - 1)))];
      }
#pragma unroll
      for (int n = 0; n < FN; ++n) {
        const int R = BM + wn * WTN + n * 16 + (lane & 15);
        bf[n] = base[R * CH + (c ^ ((R >> SWZ) & (CH - 1)))];
      }
      // Accumulators in groups of GRP, each group through all E elements
      // before the next: the FP64 16x16x4 MFMA keeps about 90% of its rate
      // with four accumulators in turn and 72% with sixteen (FP32 keeps full
      // rate either way).  Every accumulator still takes its k in order.
      constexpr int GRP = sizeof(T) == 8 ? 4 : FM * FN;
      static_assert((FM * FN) % GRP == 0, "whole groups");
      typedef T TV __attribute__((ext_vector_type(E)));
#pragma unroll
      for (int g0 = 0; g0 < FM * FN; g0 += GRP) {
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int q = g0; q < g0 + GRP; ++q) {
            const int m = q / FN, n = q % FN;
            acc[m][n] = D::mma(__builtin_bit_cast(TV, af[m])[e], __builtin_bit_cast(TV, bf[n])[e],
                               acc[m][n]);
          }
        // (the scheduler would interleave the groups again)
        if constexpr (GRP < FM * FN) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (FLUSH > 0) {
      if ((t + 1) % FLUSH == 0 || t + 1 == ktiles) flush();
    }
    __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);   // this wave's part of tile t + 1
    __syncthreads();
  }
  if constexpr (FLUSH > 0) {
#pragma unroll
    for (int m = 0; m < FM; ++m)
#pragma unroll
      for (int n = 0; n < FN; ++n) acc[m][n] = tot[m][n];
  }

  T* C = (T*)(each ? a.x1[j] : ((a.mode != 0 || it.out == 0) ? a.x : a.x1[j]));
  const bool diag = it.ti == it.tj;
  const bool mirror = a.mode < 2;
#pragma unroll
  for (int m = 0; m < FM; ++m)
#pragma unroll
    for (int n = 0; n < FN; ++n) {
      const int64_t gc = row_b0 + wn * WTN + n * 16 + (lane & 15);
      const int64_t gr0 = row_a0 + wm * WTM + m * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gr = gr0 + D::row(lane, r);
        const T v = acc[m][n][r];
        if (!mirror) {
          C[gr * ld + gc] = v;
        } else {
          if (!diag || gr <= gc) C[gr * ld + gc] = v;
          if (!diag || gr < gc) C[gc * ld + gr] = v;
        }
      }
    }
  }  // items
}

// ------------------------------------------------------------------ dispatch
// Tile configurations (edge, k-tile, wave grid, LDS swizzle shift).
constexpr int kSplitBM = 256, kSplitWGM = 2, kSplitWGN = 2;
// 128 x 128 tiles, 16-wide k-tiles.  FP32: 4 waves of 64 x 64 per workgroup
// (32 KB of LDS); with the blocked accumulation (a second set of 64
// accumulators, 194 registers) two waves per SIMD and two workgroups per CU,
// without it four and four.  FP64: 8 waves of 64 x 32 (64 KB), two
// workgroups per CU, four waves per SIMD; its 16x16x4 MFMA keeps its rate
// only with few accumulators in turn, so a wave holds eight.
constexpr int kDirBM = 128, kDirWGM = 2;
constexpr int kDirBK32 = 16, kDirSWZ32 = 2, kDirWGN32 = 2, kDirWG32 = 4;
constexpr int kDirBK64 = 16, kDirSWZ64 = 1, kDirWGN64 = 4, kDirWG64 = 2;
// FP32: the MFMAs accumulate 4 k-tiles (64 k) before the partial sum joins the
// running total; the second set of accumulators takes two waves per SIMD.
constexpr int kDirFlush32 = 4;

int product_tile(dmpt_precision prec) {
  return (prec == DMPT_SPLIT_FP16 || prec == DMPT_SPLIT_BF16) ? kSplitBM : kDirBM;
}

void product_items(int T, int mode, TileItem* out) {
  int k = 0;
  for (int ti = 0; ti < T; ++ti)
    for (int tj = mode == 2 ? 0 : ti; tj < T; ++tj) {
      TileItem it;
      it.out = 0;
      it.prob = 0;
      it.ti = ti;
      it.tj = tj;
      out[k++] = it;
    }
}

static int device_cus() {
  // set once, by the first launch of any thread (a function-local static is
  // initialised exactly once even when threads race to it)
  static const int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    return n;
  }();
  return cus;
}

template <typename K>
static hipError_t launch_one(K kernel, int threads, size_t lds_bytes, int wg_per_cu,
                             const ProductArgs& a, hipStream_t s) {
  static_assert(sizeof(ProductArgs) < 4096, "kernel argument block");
  hipError_t e = hipFuncSetAttribute((const void*)kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  if (a.n_items <= 0) return hipSuccess;
  // as many workgroups as can be resident at once (LDS and registers decide)
  const int cap = wg_per_cu * device_cus();
  const int grid = a.n_items < cap ? a.n_items : cap;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds_bytes, s, a);
  return hipGetLastError();
}

template <typename T16, int BK, int WGM, int WGN, int SWZ, int STAGES, bool FUSED>
static hipError_t launch_split_cfg(const ProductArgs& a, hipStream_t s) {
  constexpr size_t lds = (size_t)STAGES * (4 * kSplitBM) * (BK / 8) * 16;
  static_assert(lds <= 160 * 1024 - 256, "LDS of one CU");
  return launch_one(k_products_split<T16, kSplitBM, BK, WGM, WGN, SWZ, STAGES, FUSED>,
                    WGM * WGN * kWave, lds, 1, a, s);
}

template <typename T16, bool FUSED>
static hipError_t launch_split(const ProductArgs& a, hipStream_t s) {
  return launch_split_cfg<T16, kPanelK, kSplitWGM, kSplitWGN, 2, 2, FUSED>(a, s);
}

template <typename T16>
static hipError_t launch_split_small(const ProductArgs& a, hipStream_t s) {
  // 128 x 128 tiles, 4 waves of 64 x 64, two workgroups per CU
  constexpr size_t lds = (size_t)2 * (4 * 128) * (kPanelK / 8) * 16;
  return launch_one(k_products_split<T16, 128, kPanelK, 2, 2, 2, 2, true>, 4 * kWave, lds, 2, a,
                    s);
}

template <typename T16>
static hipError_t launch_split_pair(const ProductArgs& a, hipStream_t s) {
  // 128 x 256 items, 8 waves of 64 x 64, three stages, one workgroup per CU
  constexpr size_t lds = (size_t)3 * (6 * 128) * (kPanelK / 8) * 16;
  static_assert(lds <= 160 * 1024 - 256, "LDS of one CU");
  return launch_one(k_products_pair<T16, 2>, 8 * kWave, lds, 1, a, s);
}

hipError_t launch_products_pair(dmpt_precision prec, const ProductArgs& a, hipStream_t s) {
  if (!a.probs || !a.part_f || !a.part_m) return hipErrorInvalidValue;
  if (prec == DMPT_SPLIT_FP16) return launch_split_pair<_Float16>(a, s);
  if (prec == DMPT_SPLIT_BF16) return launch_split_pair<__bf16>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_products_fused(dmpt_precision prec, int tile, const ProductArgs& a,
                                 hipStream_t s) {
  if (!a.probs || !a.part_f || !a.part_m || (tile != 128 && tile != 256))
    return hipErrorInvalidValue;
  if (prec == DMPT_SPLIT_FP16)
    return tile == 128 ? launch_split_small<_Float16>(a, s) : launch_split<_Float16, true>(a, s);
  if (prec == DMPT_SPLIT_BF16)
    return tile == 128 ? launch_split_small<__bf16>(a, s) : launch_split<__bf16, true>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_products(dmpt_precision prec, const ProductArgs& a, hipStream_t s) {
  // tiles cover [0, kdim)^2 exactly; rows must keep 16-byte alignment
  if (a.kdim % product_tile(prec) != 0 || a.ld < a.kdim || a.ld % 8 != 0)
    return hipErrorInvalidValue;
  if (a.mode != 0 && (prec == DMPT_SPLIT_FP16 || prec == DMPT_SPLIT_BF16 || a.state))
    return hipErrorInvalidValue;               // single products: direct forms, no state
  switch (prec) {
    case DMPT_SPLIT_FP16:
      return launch_split<_Float16, false>(a, s);
    case DMPT_SPLIT_BF16:
      return launch_split<__bf16, false>(a, s);
    case DMPT_FP32: {
      constexpr size_t lds = 2 * (2 * kDirBM) * (kDirBK32 / 4) * 16;
      if (a.plain_accum)
        return launch_one(k_products_direct<float, kDirBM, kDirBK32, kDirWGM, kDirWGN32, kDirSWZ32, 4>,
                          kDirWGM * kDirWGN32 * kWave, lds, kDirWG32, a, s);
      return launch_one(k_products_direct<float, kDirBM, kDirBK32, kDirWGM, kDirWGN32, kDirSWZ32,
                                          2, kDirFlush32>,
                        kDirWGM * kDirWGN32 * kWave, lds, kDirWG32 / 2, a, s);
    }
    case DMPT_FP64: {
      constexpr size_t lds = 2 * (2 * kDirBM) * (kDirBK64 / 2) * 16;
      return launch_one(k_products_direct<double, kDirBM, kDirBK64, kDirWGM, kDirWGN64, kDirSWZ64, 4>,
                        kDirWGM * kDirWGN64 * kWave, lds, kDirWG64, a, s);
    }
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ trace of X before the products
// One wave per 32 x 32 diagonal fragment of X = S^2: the same operand chunks,
// k order and MFMA sequence per 16-wide k step as k_products_split (for a
// diagonal fragment the A and B rows coincide), so the diagonal equals the
// product's bitwise.  Output element (row, col) of lane l sits in column
// l % 32 and row 8 (r / 4) + 4 (l / 32) + r % 4.
template <typename T16>
__global__ void __launch_bounds__(kWave) k_trace_diag(const ProblemDesc* probs,
                                                     const TraceBlock* blocks, double* part) {
  using S = Split16<T16>;
  using V = typename S::V;
  const TraceBlock tb = blocks[blockIdx.x];
  const ProblemDesc& d = probs[tb.prob];
  const LayerState* st = d.state;
  if (st->done || st->d0) return;
  const int lane = threadIdx.x;
  const int par = st->s_par;
  const uint16_t* hi = (const uint16_t*)d.s_hi[par];
  const uint16_t* lo = (const uint16_t*)d.s_lo[par];
  const int64_t row = (int64_t)tb.blk * 32 + (lane & 31);
  const int64_t base = panel_index(row, 0, d.pdim) + 8 * (lane >> 5);
  const int64_t kb = d.kdim / kPanelK;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  // U panel blocks per batch, the next batch's loads in flight while this
  // one's MFMAs run (the wave is alone on its SIMD: latency, not issue, is
  // the limit); the MFMA sequence is the product's, block after block.
  constexpr int U = 8, KS = kPanelK / 16;
  // global-memory loads (generic ones also count as LDS traffic, so every
  // wait on them would be a full drain)
  typedef const __attribute__((address_space(1))) V GV;
  V h[2][U][KS], l[2][U][KS];
  // batch i holds blocks i U .. min(kb, (i + 1) U) - 1; its fetch clamps the
  // block index to kb - 1, so every load is issued and stays in the buffer
  // (the copies past the end are never multiplied)
  auto fetch = [&](V (&hh)[U][KS], V (&ll)[U][KS], int64_t i) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int64_t b = min(i * U + u, kb - 1);
        const int64_t off = base + b * (kPanelRows * kPanelK) + 16 * kk;
        hh[u][kk] = *(GV*)(hi + off);
        ll[u][kk] = *(GV*)(lo + off);
      }
  };
  auto mma3 = [&](const V& ah, const V& al) {
    acc = S::mma(S::up(ah), ah, acc);
    acc = S::mma(ah, al, acc);
    acc = S::mma(al, ah, acc);
  };
  const int64_t nb = (kb + U - 1) / U;       // batches, the last one possibly partial
  auto consume = [&](const V (&hh)[U][KS], const V (&ll)[U][KS], int64_t i) {
    const int cnt = (int)min((int64_t)U, kb - i * U);   // uniform
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < cnt) {
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) mma3(hh[u][kk], ll[u][kk]);
      }
  };
  // Pairs of batches, the next batch's loads in flight while this one's
  // MFMAs run; every fetch is unconditional (a branch around one would make
  // the wait before the next MFMAs cover it too): past the last batch the
  // last one is fetched again, and nothing reads it.
  fetch(h[0], l[0], 0);
  // (scheduling fences keep each batch's loads ahead of the other's MFMAs)
  for (int64_t q = 0; q < nb; q += 2) {
    fetch(h[1], l[1], q + 1 < nb ? q + 1 : q);
    __builtin_amdgcn_sched_barrier(0);
    consume(h[0], l[0], q);
    __builtin_amdgcn_sched_barrier(0);
    fetch(h[0], l[0], q + 2 < nb ? q + 2 : q);
    __builtin_amdgcn_sched_barrier(0);
    if (q + 1 < nb) consume(h[1], l[1], q + 1);
    __builtin_amdgcn_sched_barrier(0);
  }
  // lane (c, h) holds the diagonal element of column c when h = (c / 4) % 2
  const int c = lane & 31;
  const float scale = ldexpf(1.0f, -S::kShift);
  double v = 0.0;
  if ((lane >> 5) == ((c >> 2) & 1) && tb.blk * 32 + c < st->n_real) {
    const int ri = 4 * (c >> 3) + (c & 3);
    float x = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (r == ri) x = acc[r] * scale;
    v = (double)x;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) part[blockIdx.x] = v;
}

hipError_t launch_trace_diag(dmpt_precision prec, const ProblemDesc* probs,
                             const TraceBlock* blocks, int n_blocks, double* part, hipStream_t s) {
  static_assert(kPanelK % 16 == 0, "k-steps of the split MFMA inside a panel block");
  if (n_blocks <= 0) return hipSuccess;
  if (prec == DMPT_SPLIT_FP16)
    hipLaunchKernelGGL(k_trace_diag<_Float16>, dim3(n_blocks), dim3(kWave), 0, s, probs, blocks,
                       part);
  else if (prec == DMPT_SPLIT_BF16)
    hipLaunchKernelGGL(k_trace_diag<__bf16>, dim3(n_blocks), dim3(kWave), 0, s, probs, blocks,
                       part);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------------ MFMA layout self-test
// Small integer operands (exact in every format); each lane compares the
// elements it holds under the assumed output layout with a direct sum.
__device__ __forceinline__ int ta(int m, int k) { return ((m * 7 + k * 3) % 5) - 2; }
__device__ __forceinline__ int tb(int k, int n) { return ((k * 5 + n * 11) % 5) - 2; }

__global__ void k_selftest_mfma(int32_t* out) {
  const int l = threadIdx.x;
  int bad = 0;
  {  // f16 32x32x16: A row l%32, k = 8*(l/32)+e ; B col l%32, same k
    f16x8 av, bv;
    for (int e = 0; e < 8; ++e) {
      av[e] = (_Float16)(float)ta(l & 31, 8 * (l >> 5) + e);
      bv[e] = (_Float16)(float)tb(8 * (l >> 5) + e, l & 31);
    }
    f32x16 c = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), col = l & 31;
      int ref = 0;
      for (int k = 0; k < 16; ++k) ref += ta(row, k) * tb(k, col);
      if (c[r] != (float)ref) bad |= 1;
    }
  }
  {  // bf16 32x32x16
    bf16x8 av, bv;
    for (int e = 0; e < 8; ++e) {
      av[e] = (__bf16)(float)ta(l & 31, 8 * (l >> 5) + e);
      bv[e] = (__bf16)(float)tb(8 * (l >> 5) + e, l & 31);
    }
    f32x16 c = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3), col = l & 31;
      int ref = 0;
      for (int k = 0; k < 16; ++k) ref += ta(row, k) * tb(k, col);
      if (c[r] != (float)ref) bad |= 2;
    }
  }
  {  // f32 16x16x4: A row l%16, k = l/16 ; out row 4*(l/16)+r, col l%16
    f32x4 c = {};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32((float)ta(l & 15, l >> 4), (float)tb(l >> 4, l & 15), c,
                                             0, 0, 0);
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * (l >> 4) + r, col = l & 15;
      int ref = 0;
      for (int k = 0; k < 4; ++k) ref += ta(row, k) * tb(k, col);
      if (c[r] != (float)ref) bad |= 4;
    }
  }
  {  // f64 16x16x4: out row l/16 + 4r, col l%16
    f64x4 c = {};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ta(l & 15, l >> 4), (double)tb(l >> 4, l & 15),
                                             c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) {
      const int row = (l >> 4) + 4 * r, col = l & 15;
      int ref = 0;
      for (int k = 0; k < 4; ++k) ref += ta(row, k) * tb(k, col);
      if (c[r] != (double)ref) bad |= 8;
    }
  }
  out[l] = bad;
}

hipError_t launch_selftest_mfma(int32_t* result, hipStream_t s) {
  hipLaunchKernelGGL(k_selftest_mfma, dim3(1), dim3(kWave), 0, s, result);
  return hipGetLastError();
}

// ------------------------------------------------------------------ MFMA rate probe
// Four waves per CU issue independent 32x32x16 MFMAs (eight accumulators, 48
// per iteration) on pseudo-random operands in [-1, 1), with no memory traffic.
// The chip's power management sets the clock from the switching activity, so
// random operands give the clock the product kernels run at.  Workgroup 0
// records the shader-clock (s_memtime) and wall-clock (s_memrealtime) ticks
// it spent; every lane stores its accumulator sum so that nothing is elided.
template <typename T16>
__global__ void __launch_bounds__(4 * kWave) k_mfma_rate(float* out, int64_t* ticks, int iters) {
  using S = Split16<T16>;
  typename S::V a, b;
  for (int e = 0; e < 8; ++e) {
    uint32_t h = (uint32_t)(threadIdx.x * 8 + e + 1) * 2654435761u + blockIdx.x * 40503u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    a[e] = (T16)((float)(h & 0xffff) * (2.0f / 65536.0f) - 1.0f);
    b[e] = (T16)((float)(h >> 16) * (2.0f / 65536.0f) - 1.0f);
  }
  f32x16 acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  const int64_t c0 = __builtin_amdgcn_s_memtime(), w0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int rep = 0; rep < 6; ++rep)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = S::mma(a, b, acc[j]);
  }
  const int64_t c1 = __builtin_amdgcn_s_memtime(), w1 = __builtin_amdgcn_s_memrealtime();
  float sum = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) sum += acc[j][r];
  out[blockIdx.x * blockDim.x + threadIdx.x] = sum;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ticks[0] = c1 - c0;
    ticks[1] = w1 - w0;
  }
}

// The same for the direct forms' 16x16x4 FP32 / FP64 MFMA, 48 MFMAs per
// iteration.  FP64 runs four accumulators: measured on gfx950, its 16x16x4
// MFMA sustains about 90% of the data-sheet rate with four accumulators in
// turn, 83% with eight and 72% with sixteen; FP32 keeps full rate with
// sixteen.
template <typename T>
__global__ void __launch_bounds__(4 * kWave) k_mfma_rate_direct(float* out, int64_t* ticks,
                                                                int iters) {
  using D = Direct<T>;
  constexpr int NACC = sizeof(T) == 8 ? 4 : 16;
  uint32_t h = (uint32_t)(threadIdx.x + 1) * 2654435761u + blockIdx.x * 40503u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const T a = (T)((float)(h & 0xffff) * (2.0f / 65536.0f) - 1.0f);
  const T b = (T)((float)(h >> 16) * (2.0f / 65536.0f) - 1.0f);
  typename D::Acc acc[NACC];
#pragma unroll
  for (int j = 0; j < NACC; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = (T)0;
  const int64_t c0 = __builtin_amdgcn_s_memtime(), w0 = __builtin_amdgcn_s_memrealtime();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int rep = 0; rep < 48 / NACC; ++rep)
#pragma unroll
      for (int j = 0; j < NACC; ++j) acc[j] = D::mma(a, b, acc[j]);
  }
  const int64_t c1 = __builtin_amdgcn_s_memtime(), w1 = __builtin_amdgcn_s_memrealtime();
  T sum = (T)0;
#pragma unroll
  for (int j = 0; j < NACC; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) sum += acc[j][r];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)sum;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ticks[0] = c1 - c0;
    ticks[1] = w1 - w0;
  }
}

double mfma_probe_flops(dmpt_precision prec) {
  // flops of one MFMA of the probe: 32x32x16 for the split forms, 16x16x4 else
  return (prec == DMPT_SPLIT_FP16 || prec == DMPT_SPLIT_BF16) ? 2.0 * 32 * 32 * 16
                                                              : 2.0 * 16 * 16 * 4;
}

hipError_t launch_mfma_rate(dmpt_precision prec, int blocks, int iters, float* out,
                            int64_t* ticks, hipStream_t s) {
  // one workgroup per CU: the LDS request leaves room for no second one
  constexpr size_t lds = 96 * 1024;
  const void* k = nullptr;
  switch (prec) {
    case DMPT_SPLIT_BF16: k = (const void*)k_mfma_rate<__bf16>; break;
    case DMPT_SPLIT_FP16: k = (const void*)k_mfma_rate<_Float16>; break;
    case DMPT_FP32: k = (const void*)k_mfma_rate_direct<float>; break;
    case DMPT_FP64: k = (const void*)k_mfma_rate_direct<double>; break;
  }
  if (!k) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  switch (prec) {
    case DMPT_SPLIT_BF16:
      hipLaunchKernelGGL(k_mfma_rate<__bf16>, dim3(blocks), dim3(4 * kWave), lds, s, out, ticks,
                         iters);
      break;
    case DMPT_SPLIT_FP16:
      hipLaunchKernelGGL(k_mfma_rate<_Float16>, dim3(blocks), dim3(4 * kWave), lds, s, out,
                         ticks, iters);
      break;
    case DMPT_FP32:
      hipLaunchKernelGGL(k_mfma_rate_direct<float>, dim3(blocks), dim3(4 * kWave), lds, s, out,
                         ticks, iters);
      break;
    case DMPT_FP64:
      hipLaunchKernelGGL(k_mfma_rate_direct<double>, dim3(blocks), dim3(4 * kWave), lds, s, out,
                         ticks, iters);
      break;
  }
  return hipGetLastError();
}

int device_cu_count() { return device_cus(); }

}  // namespace dmpt
