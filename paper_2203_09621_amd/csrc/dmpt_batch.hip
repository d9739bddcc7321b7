// Batched DNN-SP2-PT: many independent Hamiltonians of different sizes run
// Algorithms 1-3 together.  All problems advance layer by layer: the
// decisions run as one workgroup per problem, and one persistent fused
// product launch per tile class covers the tiles of every problem still
// running, with the layer update in its epilogue.  Each problem keeps its own
// LayerState, so problems stop independently; kernels skip problems that are
// done.  The whole response (normalisation, every
// layer up to the cap, outputs) is captured once into a HIP graph and
// replayed; inputs and outputs reach the graph through device pointer tables.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "layer_common.h"

namespace dmpt {

struct BatchProblem {
  LayerState* st;
  float* s_master;
  uint16_t* s_hi[2];
  uint16_t* s_lo[2];
  float* s1buf[kMaxKB][2];
  uint16_t* s1_hi[kMaxKB][2];
  uint16_t* s1_lo[kMaxKB][2];
  const TileItem* items;             // this problem's tile items in its class list
  int32_t n_items;
  int32_t slot_first;                // partial slot of items[0]
  int64_t n, np, ld;
  double nocc;
  int32_t k;
  int32_t h0_index, h1_first;        // positions in the input / output pointer tables
  int32_t u0_first, u0_count;        // S0 block-table range
  int32_t tr_first, tr_count;        // range of this problem's diagonal blocks of Tr X
  int32_t u1_first[kMaxKB], u1_count[kMaxKB];
};

struct Chunk {
  int32_t p, j;                      // problem, matrix (-1: S0, j: S1_j)
  int64_t q0, q1;                    // range of 4-element vectors of the padded storage
};

// One kOutB x kOutB block (bi, bj) of an output matrix (-1: P0, j: P1_j).
struct OutBlock {
  int32_t p, j, bi, bj;
};
constexpr int kOutB = 64;


struct ProblemSummary {
  int32_t layers, d0_layer, converged, error;
  int32_t d1_layer[kMaxKB];
  int32_t pad;
  double idem0;
  double idem1[kMaxKB];
};

constexpr int kChunkVec = 4 * kBlk;  // vectors per block-table chunk (16 K elements)

// ------------------------------------------------------------------ normalisation
// Gershgorin partials of H0 per block of 32 rows (the blocks of the Tr X
// table): min(H_ii - r_i), max(H_ii + r_i) and sum H_ii, one wave per row.
__global__ void __launch_bounds__(kBlk) k_b_gersh(const BatchProblem* P, const TraceBlock* T,
                                                 const double* const* h0tab, double* part) {
  const TraceBlock t = T[blockIdx.x];
  const BatchProblem& b = P[t.prob];
  const double* H = h0tab[b.h0_index];
  const int64_t n = b.n;
  const int64_t r0 = (int64_t)t.blk * 32, r1 = r0 + 32 < n ? r0 + 32 : n;
  const int lane = threadIdx.x & (kWave - 1);
  double lo = INFINITY, hi = -INFINITY, tr = 0.0;
  for (int64_t i = r0 + threadIdx.x / kWave; i < r1; i += kBlk / kWave) {
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
    part[3 * blockIdx.x] = lo;
    part[3 * blockIdx.x + 1] = hi;
    part[3 * blockIdx.x + 2] = tr;
  }
}

// Per problem: clear the state, combine the Gershgorin partials of its row
// blocks in a fixed order, N_S = Tr S0, and the Algorithm 1-3 scalars.
__global__ void __launch_bounds__(kBlk) k_b_setup(BatchProblem* P, const double* gpart,
                                                 int max_layers) {
  BatchProblem& b = P[blockIdx.x];
  LayerState* st = b.st;
  {
    int32_t* w = (int32_t*)st;
    for (size_t i = threadIdx.x; i < sizeof(LayerState) / 4; i += kBlk) w[i] = 0;
  }
  __syncthreads();
  const int64_t n = b.n;
  double lo = INFINITY, hi = -INFINITY, tr = 0.0;
  for (int c = threadIdx.x; c < b.tr_count; c += kBlk) {
    const double* g = gpart + 3 * (int64_t)(b.tr_first + c);
    lo = fmin(lo, g[0]);
    hi = fmax(hi, g[1]);
    tr += g[2];
  }
  lo = block_min(lo);
  hi = block_max(hi);
  tr = block_sum(tr);
  if (threadIdx.x != 0) return;
  const double w = hi - lo;
  st->n_real = (int32_t)n;
  st->k = b.k;
  st->order2_slot = -1;
  st->max_layers = max_layers;
  st->nocc = b.nocc;
  st->eps1 = lo;
  st->epsN = hi;
  st->n_s0 = ((double)n * hi - tr) / w;
  st->n_s = st->n_s0;
  for (int j = 0; j < kMaxK; ++j) st->d1[j] = j < b.k ? 0 : 1;
  if (!(w > 0.0) || !isfinite(w)) {
    st->error = DMPT_ENONFINITE;
    st->done = 1;
  }
}

// max |H1_j| per chunk of problem p, response j.
__global__ void __launch_bounds__(kBlk) k_b_maxabs1(const BatchProblem* P, const Chunk* C,
                                                   const double* const* h1tab, double* part) {
  const Chunk c = C[blockIdx.x];
  const BatchProblem& b = P[c.p];
  const double* H = h1tab[b.h1_first + c.j];
  double m = 0.0;
  for (int64_t q = c.q0 * 4 + threadIdx.x; q < c.q1 * 4; q += kBlk) {
    const int64_t r = q / b.ld, col = q - r * b.ld;
    if (r < b.n && col < b.n) {
      const double v = fabs(H[r * b.n + col]);
      m = (v > m || v != v) ? v : m;
    }
  }
  m = block_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Split scale of S1_0 = -H1/(eps_N - eps_1) per response.
__global__ void __launch_bounds__(kBlk) k_b_s1setup(const BatchProblem* P, const double* part) {
  const BatchProblem& b = P[blockIdx.x];
  LayerState* st = b.st;
  for (int j = 0; j < b.k; ++j) {
    double m = 0.0;
    for (int i = threadIdx.x; i < b.u1_count[j]; i += kBlk) {
      const double v = part[b.u1_first[j] + i];
      m = (v > m || v != v) ? v : m;
    }
    m = block_max(m);
    if (threadIdx.x == 0) {
      const double mx = m / (st->epsN - st->eps1);
      if (!isfinite(mx)) {
        st->error = DMPT_ENONFINITE;
        st->done = 1;
      }
      const int e = split_exponent(mx);
      st->s1_exp_split[j] = e;
      st->s1_exp_next[j] = e;
      st->s1_exp_hist[j][0] = e;
      st->s1_max[j] = mx;
    }
  }
}

// S0 = (eps_N I - H0)/(eps_N - eps_1) (j = -1) or S1_0 = -H1_j/(eps_N - eps_1),
// FP32 master plus panel-major hi/lo (buffers 0).
template <typename T16>
__global__ void __launch_bounds__(kBlk) k_b_init(const BatchProblem* P, const Chunk* C,
                                                const double* const* h0tab,
                                                const double* const* h1tab, int t) {
  const Chunk c = C[blockIdx.x];
  const BatchProblem& b = P[c.p];
  const LayerState* st = b.st;
  const double en = st->epsN, w = st->epsN - st->eps1;
  const double* H = c.j < 0 ? h0tab[b.h0_index] : h1tab[b.h1_first + c.j];
  float* m = c.j < 0 ? b.s_master : b.s1buf[c.j][0];
  uint16_t* hi = c.j < 0 ? b.s_hi[0] : b.s1_hi[c.j][0];
  uint16_t* lo = c.j < 0 ? b.s_lo[0] : b.s1_lo[c.j][0];
  const int e = c.j < 0 ? 0 : st->s1_exp_split[c.j];
  for (int64_t q = c.q0 * 4 + threadIdx.x; q < c.q1 * 4; q += kBlk) {
    const int64_t r = q / b.ld, col = q - r * b.ld;
    double v = 0.0;
    if (r < b.n && col < b.n) v = c.j < 0 ? ((r == col ? en : 0.0) - H[r * b.n + col]) / w
                                          : -H[r * b.n + col] / w;
    const float f = (float)v;
    m[q] = f;
    if (col < b.np) {
      const int64_t pi = panel_index(r, col, b.np);
      split_one<T16>(f, e, t, hi + pi, lo + pi);
    }
  }
}

// ------------------------------------------------------------------ layer decisions
// Before the products of a layer: N_X from this problem's diagonal-block
// partials of Tr X (launch_trace_diag).
__global__ void __launch_bounds__(kBlk) k_b_predecide(const BatchProblem* P, const double* part) {
  const BatchProblem& b = P[blockIdx.x];
  predecide_body(b.st, part + b.tr_first, b.tr_count);
}

// After the products: this problem's item partials.
__global__ void __launch_bounds__(kBlk) k_b_postdecide(const BatchProblem* P, const double* part_f,
                                                      const double* part_m, int t) {
  const BatchProblem& b = P[blockIdx.x];
  postdecide_body(b.st, b.items, b.n_items, part_f + b.slot_first, part_m + b.slot_first, t,
                  (int)blockIdx.x);
}

// ------------------------------------------------------------------ outputs
// The pair launch keeps only the upper triangle of the FP32 masters current
// (its mirror pass writes the 16-bit splits alone; the recursion reads the
// masters only on upper tiles), so output block (bi, bj) is read from the
// upper block (min, max) in coalesced rows and written through LDS,
// transposed below the diagonal.  The 256-row launch's full masters are
// symmetric, so the same read serves them.
__global__ void __launch_bounds__(kBlk) k_b_out(const BatchProblem* P, const OutBlock* B,
                                               double* const* p0tab, double* const* p1tab) {
  __shared__ float tile[kOutB][kOutB + 1];
  const OutBlock ob = B[blockIdx.x];
  const BatchProblem& b = P[ob.p];
  const LayerState* st = b.st;
  const float* src;
  double* dst;
  if (ob.j < 0) {
    src = b.s_master;
    dst = p0tab[b.h0_index];
  } else {
    const int L = st->d1[ob.j] && st->d1_layer[ob.j] > 0 ? st->d1_layer[ob.j] - 1 : st->n;
    src = b.s1buf[ob.j][L & 1];
    dst = p1tab[b.h1_first + ob.j];
  }
  if (!dst) return;
  const int64_t si = (int64_t)min(ob.bi, ob.bj) * kOutB, sj = (int64_t)max(ob.bi, ob.bj) * kOutB;
  for (int e = threadIdx.x; e < kOutB * kOutB; e += kBlk) {
    const int r = e / kOutB, c = e % kOutB;
    const int64_t gr = si + r, gc = sj + c;
    tile[r][c] = (gr < b.n && gc < b.n) ? src[gr * b.ld + gc] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kOutB * kOutB; e += kBlk) {
    const int r = e / kOutB, c = e % kOutB;
    const int64_t gr = (int64_t)ob.bi * kOutB + r, gc = (int64_t)ob.bj * kOutB + c;
    if (gr >= b.n || gc >= b.n) continue;
    const bool up = ob.bi < ob.bj || (ob.bi == ob.bj && r <= c);
    dst[gr * b.n + gc] = (double)(up ? tile[r][c] : tile[c][r]);
  }
}

__global__ void k_b_summary(const BatchProblem* P, ProblemSummary* out) {
  if (threadIdx.x != 0) return;
  const BatchProblem& b = P[blockIdx.x];
  const LayerState* st = b.st;
  ProblemSummary s;
  s.layers = st->n;
  s.d0_layer = st->d0_layer;
  s.converged = st->converged;
  s.error = st->error;
  s.pad = 0;
  s.idem0 = st->fro0;
  for (int j = 0; j < kMaxKB; ++j) {
    s.d1_layer[j] = j < b.k ? st->d1_layer[j] : 0;
    s.idem1[j] = (j < b.k && st->d1_layer[j] > 0) ? st->fro1[j][st->d1_layer[j]] : 0.0;
  }
  out[blockIdx.x] = s;
}

}  // namespace dmpt

// ====================================================================== host side
using namespace dmpt;

namespace {

dmpt_status bfail(dmpt_status s, const std::string& m) {
  set_last_error(m.c_str());
  return s;
}

#define BCHK(expr)                                                                      \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return bfail(DMPT_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

std::vector<TileItem> triangle_items(int T, int k, int prob) {
  std::vector<TileItem> v;
  const int GR = 8;
  auto add_out = [&](int out) {
    for (int g0 = 0; g0 < T; g0 += GR) {
      const int g1 = std::min(T, g0 + GR);
      for (int tj = g0; tj < T; ++tj)
        for (int ti = g0; ti < std::min(g1, tj + 1); ++ti) {
          TileItem it;
          it.out = (int16_t)out;
          it.prob = (int16_t)prob;
          it.ti = ti;
          it.tj = tj;
          v.push_back(it);
        }
    }
  };
  for (int j = 0; j < k; ++j) add_out(1 + j);
  add_out(0);
  return v;
}

// Items of the pair launch.  Per output, the tiles (ti, tj), tj >= ti, of
// each row band two by two from the diagonal (they share the A panels); a
// band with an odd count leaves its last tile (ti, T - 1), and these, all in
// the last column band, pair up two by two (sharing the B panels), the odd
// one out alone (ti2 = -1).
std::vector<TileItem> pair_items(int T, int k, int prob) {
  std::vector<TileItem> v;
  auto add = [&](int out, int ti, int tj, int ti2, int tj2) {
    TileItem it;
    it.out = (int16_t)out;
    it.prob = (int16_t)prob;
    it.ti = ti;
    it.tj = tj;
    it.ti2 = ti2;
    it.tj2 = tj2;
    v.push_back(it);
  };
  auto add_out = [&](int out) {
    std::vector<int> rest;
    for (int ti = 0; ti < T; ++ti) {
      int tj = ti;
      for (; tj + 1 < T; tj += 2) add(out, ti, tj, ti, tj + 1);
      if (tj < T) rest.push_back(ti);
    }
    for (size_t i = 0; i < rest.size(); i += 2) {
      if (i + 1 < rest.size()) add(out, rest[i], T - 1, rest[i + 1], T - 1);
      else add(out, rest[i], T - 1, -1, -1);
    }
  };
  for (int j = 0; j < k; ++j) add_out(1 + j);
  add_out(0);
  return v;
}

}  // namespace

struct dmpt_batch {
  int count;
  dmpt_precision prec;
  int t;
  int max_layers;
  int use_graph;
  hipStream_t stream;
  hipStream_t cap;
  std::vector<BatchProblem> hp;
  BatchProblem* dp = nullptr;
  std::vector<Chunk> c0, c1;
  Chunk* dc0 = nullptr;
  Chunk* dc1 = nullptr;
  std::vector<TraceBlock> tb;                  // diagonal blocks of Tr X
  TraceBlock* dtb = nullptr;
  std::vector<OutBlock> ob;                    // output blocks of every P0 and P1_j
  OutBlock* dob = nullptr;
  double* part_tr = nullptr;                   // per diagonal block: trace partial
  double* part_g = nullptr;                    // per diagonal block: Gershgorin partials (3)
  double* part1m = nullptr;                    // per S1 chunk: max |H1|
  double* part_f = nullptr;                    // per tile item: fused-layer partials
  double* part_m = nullptr;
  ProblemDesc* desc = nullptr;                 // per problem: buffers of the fused layer
  int threshold = 0;                           // problems with Np <= threshold use 128-row tiles
  TileItem* items[2] = {nullptr, nullptr};     // [0]: 256-row tiles, [1]: pairs of 128-row tiles
  int n_items[2] = {0, 0};
  int total_k = 0;
  int cus = 256;                               // compute units of the device
  const double** h0tab = nullptr;
  const double** h1tab = nullptr;
  double** p0tab = nullptr;
  double** p1tab = nullptr;
  void** host_tab = nullptr;                   // pinned staging of the four tables
  ProblemSummary* dsum = nullptr;
  ProblemSummary* hsum = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<void*> allocs;
  std::vector<double> tune_ms;                 // autotuner timings per candidate threshold
  std::vector<int> tune_cand;
};

namespace {

hipError_t balloc(dmpt_batch* b, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) b->allocs.push_back(*p);
  return e;
}

void batch_free(dmpt_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->host_tab) (void)hipHostFree(b->host_tab);
  if (b->hsum) (void)hipHostFree(b->hsum);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

// Item lists of the two tile classes for a given threshold, each problem's
// item range, and the per-problem buffer descriptors (the k extent follows
// the class).
hipError_t build_class_items(dmpt_batch* b, int threshold) {
  // Per class: problems in order of decreasing cost (products times k-tiles
  // over their tiles), their items dealt in balanced rounds over the launch's
  // workgroups (the 128-row class per XCD, below).  The 128-row class runs in
  // pairs of tiles of one row band (k_products_pair).  Each problem's items keep
  // their order; the range between its first and last position may hold
  // placeholders and other problems' items, which the kernels and the
  // decisions skip.
  std::vector<TileItem> cls[2];
  std::vector<int> first(b->count), count(b->count), which(b->count);
  std::vector<std::vector<TileItem>> own(b->count);
  std::vector<std::vector<int64_t>> own_cost(b->count);
  std::vector<int64_t> total(b->count, 0);
  for (int p = 0; p < b->count; ++p) {
    const BatchProblem& bp = b->hp[p];
    const int c = bp.np <= threshold ? 1 : 0;
    const int tile = c ? 128 : 256;
    const int T = (int)((bp.n + tile - 1) / tile);
    which[p] = c;
    own[p] = c ? pair_items(T, bp.k, p) : triangle_items(T, bp.k, p);
    for (const TileItem& it : own[p]) {
      own_cost[p].push_back((it.out == 0 ? 1 : 2) * ((int64_t)T * tile / kPanelK));
      total[p] += own_cost[p].back();
    }
  }
  for (int c = 0; c < 2; ++c) {
    std::vector<int> probs;
    for (int p = 0; p < b->count; ++p)
      if (which[p] == c) probs.push_back(p);
    std::stable_sort(probs.begin(), probs.end(), [&](int x, int y) { return total[x] > total[y]; });
    std::vector<TileItem> list;
    std::vector<int64_t> cost;
    for (int p : probs) {
      list.insert(list.end(), own[p].begin(), own[p].end());
      cost.insert(cost.end(), own_cost[p].begin(), own_cost[p].end());
    }
    const int cap = b->cus;                  // one workgroup per CU in both launches
    const int grid = (int)std::min<size_t>(list.size(), (size_t)cap);
    std::vector<int32_t> order;
    if (c == 1 && grid == cap && grid % kXcds == 0) {
      // Problems to XCDs by decreasing cost (each to the least-loaded XCD),
      // so that a problem's operand panels are fetched into one L2; each
      // XCD's items sorted by length (stable: problem and band order kept)
      // and dealt in balanced rounds over the XCD's slots (slot s runs on XCD
      // s / (grid / 8)), so that items running side by side have equal
      // length and step through k together.  The layer's partial slots
      // follow the positions, so the decisions see the same values.
      const int per = grid / kXcds;
      std::vector<std::vector<int32_t>> seq(kXcds);   // list indices per XCD
      std::vector<int64_t> load(kXcds, 0);
      int64_t all = 0;
      size_t li = 0;
      for (int p : probs) {
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
          if (load[y] < load[x]) x = y;
        load[x] += total[p];
        all += total[p];
        for (size_t i = 0; i < own[p].size(); ++i) seq[x].push_back((int32_t)(li + i));
        li += own[p].size();
      }
      // too few problems to load every XCD evenly: the plain deal over all
      // workgroups (a few large problems would otherwise leave XCDs idle)
      const int64_t most = *std::max_element(load.begin(), load.end());
      const bool even = 20 * most <= 21 * ((all + kXcds - 1) / kXcds);
      size_t rounds = 0;
      std::vector<std::vector<int32_t>> plan(kXcds);
      for (int x = 0; x < kXcds && even; ++x) {
        std::stable_sort(seq[x].begin(), seq[x].end(),
                         [&](int32_t u, int32_t v) { return cost[u] > cost[v]; });
        std::vector<int64_t> cx(seq[x].size());
        for (size_t i = 0; i < cx.size(); ++i) cx[i] = cost[seq[x][i]];
        plan[x] = balanced_rounds(cx, per, 2 * cx.size());
        rounds = std::max(rounds, (plan[x].size() + per - 1) / per);
      }
      order.assign(even ? rounds * grid : 0, -1);
      for (int x = 0; x < kXcds && even; ++x)
        for (size_t q = 0; q < plan[x].size(); ++q)
          if (plan[x][q] >= 0) order[(q / per) * grid + x * per + q % per] = seq[x][plan[x][q]];
      while (!order.empty() && order.back() < 0) order.pop_back();
      if (!even || order.size() > 2 * list.size())
        order = balanced_rounds(cost, grid, 2 * list.size());
    } else {
      order = balanced_rounds(cost, grid, 2 * list.size());
    }
    std::vector<int> lo(b->count, -1), hi(b->count, -1);
    for (size_t q = 0; q < order.size(); ++q) {
      TileItem it;
      if (order[q] >= 0) {
        it = list[order[q]];
        if (lo[it.prob] < 0) lo[it.prob] = (int)q;
        hi[it.prob] = (int)q;
      } else {
        it.out = -1;
        it.prob = 0;
        it.ti = it.tj = 0;
      }
      cls[c].push_back(it);
    }
    for (int p : probs) {
      first[p] = lo[p];
      count[p] = hi[p] - lo[p] + 1;
    }
  }
  b->threshold = threshold;
  b->n_items[0] = (int)cls[0].size();
  b->n_items[1] = (int)cls[1].size();
  hipError_t e = hipSuccess;
  for (int c = 0; c < 2 && e == hipSuccess; ++c)
    if (!cls[c].empty())
      e = hipMemcpy(b->items[c], cls[c].data(), cls[c].size() * sizeof(TileItem),
                    hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  std::vector<ProblemDesc> d(b->count);
  for (int p = 0; p < b->count; ++p) {
    BatchProblem& bp = b->hp[p];
    bp.items = b->items[which[p]] + first[p];
    bp.n_items = count[p];
    bp.slot_first = (which[p] ? b->n_items[0] : 0) + first[p];
    ProblemDesc& q = d[p];
    memset(&q, 0, sizeof(q));
    for (int par = 0; par < 2; ++par) {
      q.s_hi[par] = bp.s_hi[par];
      q.s_lo[par] = bp.s_lo[par];
      for (int j = 0; j < bp.k; ++j) {
        q.s1_hi[j][par] = bp.s1_hi[j][par];
        q.s1_lo[j][par] = bp.s1_lo[j][par];
        q.s1m[j][par] = bp.s1buf[j][par];
      }
    }
    q.s_master = bp.s_master;
    q.state = bp.st;
    q.ld = bp.ld;
    // the k loop runs over N rounded up to one k-tile: the padding rows and
    // columns are zero, so a longer k range would only add exact zeros
    q.kdim = (bp.n + kPanelK - 1) / kPanelK * kPanelK;
    q.pdim = bp.np;
  }
  e = hipMemcpy(b->desc, d.data(), b->count * sizeof(ProblemDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->dp, b->hp.data(), sizeof(BatchProblem) * b->count, hipMemcpyHostToDevice);
  return e;
}

hipError_t launch_products_all(dmpt_batch* b, hipStream_t s) {
  ProductArgs a;
  memset(&a, 0, sizeof(a));
  a.probs = b->desc;
  a.part_f = b->part_f;
  a.part_m = b->part_m;
  a.lo_shift = b->t;
  hipError_t e = hipSuccess;
  if (b->n_items[0] > 0) {
    a.items = b->items[0];
    a.n_items = b->n_items[0];
    a.slot_base = 0;
    e = launch_products_fused(b->prec, 256, a, s);
  }
  if (e == hipSuccess && b->n_items[1] > 0) {
    a.items = b->items[1];
    a.n_items = b->n_items[1];
    a.slot_base = b->n_items[0];
    e = launch_products_pair(b->prec, a, s);
  }
  return e;
}

template <typename T16>
hipError_t enqueue_response(dmpt_batch* b, hipStream_t s) {
  const int P = b->count;
  hipLaunchKernelGGL(k_b_gersh, dim3(b->tb.size()), dim3(kBlk), 0, s, b->dp, b->dtb, b->h0tab,
                     b->part_g);
  hipLaunchKernelGGL(k_b_setup, dim3(P), dim3(kBlk), 0, s, b->dp, b->part_g, b->max_layers);
  hipLaunchKernelGGL(k_b_maxabs1, dim3(b->c1.size()), dim3(kBlk), 0, s, b->dp, b->dc1, b->h1tab,
                     b->part1m);
  hipLaunchKernelGGL(k_b_s1setup, dim3(P), dim3(kBlk), 0, s, b->dp, b->part1m);
  hipLaunchKernelGGL(k_b_init<T16>, dim3(b->c0.size()), dim3(kBlk), 0, s, b->dp, b->dc0, b->h0tab,
                     b->h1tab, b->t);
  hipLaunchKernelGGL(k_b_init<T16>, dim3(b->c1.size()), dim3(kBlk), 0, s, b->dp, b->dc1, b->h0tab,
                     b->h1tab, b->t);
  hipError_t e = hipGetLastError();
  for (int n = 1; n <= b->max_layers && e == hipSuccess; ++n) {
    e = launch_trace_diag(b->prec, b->desc, b->dtb, (int)b->tb.size(), b->part_tr, s);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_b_predecide, dim3(P), dim3(kBlk), 0, s, b->dp, b->part_tr);
    e = launch_products_all(b, s);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_b_postdecide, dim3(P), dim3(kBlk), 0, s, b->dp, b->part_f, b->part_m,
                       b->t);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_out, dim3(b->ob.size()), dim3(kBlk), 0, s, b->dp, b->dob, b->p0tab,
                     b->p1tab);
  hipLaunchKernelGGL(k_b_summary, dim3(P), dim3(kWave), 0, s, b->dp, b->dsum);
  return hipGetLastError();
}

hipError_t enqueue(dmpt_batch* b, hipStream_t s) {
  return b->prec == DMPT_SPLIT_FP16 ? enqueue_response<_Float16>(b, s)
                                    : enqueue_response<__bf16>(b, s);
}

// Tile-class autotuner: time one fused product sweep over the whole batch for
// each candidate threshold (problems with padded size <= threshold use
// 128-row tiles) and keep the fastest.  It runs on the zero-initialised
// workspace with a cleared state (every tile active, all values zero), before
// any response; MFMA timing does not depend on the values.
hipError_t autotune(dmpt_batch* b) {
  int maxnp = 0;
  for (auto& p : b->hp) maxnp = std::max<int>(maxnp, (int)p.np);
  std::vector<int> cand = {0};
  for (int th = 256; th <= maxnp; th += 256) cand.push_back(th);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return e;
  double best = 1e30;
  int best_th = 0;
  b->tune_ms.clear();
  b->tune_cand = cand;
  for (int th : cand) {
    e = build_class_items(b, th);
    if (e != hipSuccess) break;
    e = launch_products_all(b, b->stream);      // warm-up
    if (e != hipSuccess) break;
    e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_products_all(b, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e != hipSuccess) break;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    b->tune_ms.push_back(ms / 3.0);
    if (ms < best) {
      best = ms;
      best_th = th;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  return build_class_items(b, best_th);
}

}  // namespace

extern "C" {

dmpt_status dmpt_batch_init(dmpt_batch** out, int32_t count, const int64_t* N, const int64_t* Nocc,
                            const int32_t* k, const dmpt_options* opt_in, void* stream) {
  if (!out) return bfail(DMPT_EINVAL, "batch pointer is NULL");
  *out = nullptr;
  if (count < 1 || count > 32767 || !N || !Nocc || !k) return bfail(DMPT_EINVAL, "bad batch");
  dmpt_options opt;
  dmpt_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.precision != DMPT_SPLIT_FP16 && opt.precision != DMPT_SPLIT_BF16)
    return bfail(DMPT_ENOTSUP, "batched solves run the split precisions only");
  if (opt.max_layers <= 0) opt.max_layers = 100;
  if (opt.max_layers > kMaxLayers) return bfail(DMPT_EINVAL, "max_layers above DMPT_MAX_LAYERS");
  for (int p = 0; p < count; ++p) {
    if (N[p] < 1 || N[p] > 65536) return bfail(DMPT_EINVAL, "N out of range");
    if (Nocc[p] <= 0 || Nocc[p] >= N[p]) return bfail(DMPT_EINVAL, "need 0 < Nocc < N");
    if (k[p] < 1 || k[p] > kMaxKB) return bfail(DMPT_EINVAL, "k out of [1, 3]");
  }
  dmpt_batch* b = new dmpt_batch();
  b->count = count;
  b->prec = (dmpt_precision)opt.precision;
  b->t = b->prec == DMPT_SPLIT_FP16 ? kLoShiftF16 : kLoShiftBF16;
  b->max_layers = opt.max_layers;
  b->use_graph = opt.graph;
  b->stream = (hipStream_t)stream;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      b->cus = cus;
  }
  auto bail = [&](dmpt_status s, const std::string& m) {
    batch_free(b);
    return bfail(s, m);
  };
  // sizes, block tables, sub-allocation offsets
  b->hp.resize(count);
  size_t f32 = 0, u16 = 0;
  int h1 = 0;
  for (int p = 0; p < count; ++p) {
    BatchProblem& q = b->hp[p];
    memset(&q, 0, sizeof(q));
    q.n = N[p];
    q.np = (N[p] + 255) / 256 * 256;
    q.ld = q.np;
    q.nocc = (double)Nocc[p];
    q.k = k[p];
    q.h0_index = p;
    q.h1_first = h1;
    h1 += k[p];
    const size_t m = (size_t)q.np * q.ld;
    f32 += m * (1 + 2 * q.k);                          // S, S1_j x 2
    u16 += (size_t)q.np * q.np * 4 * (1 + q.k);        // hi, lo x 2 buffers of S and S1_j
    const int64_t vec = m / 4;
    const int nch = (int)((vec + kChunkVec - 1) / kChunkVec);
    q.u0_first = (int)b->c0.size();
    q.u0_count = nch;
    q.tr_first = (int)b->tb.size();
    q.tr_count = (int)((q.n + 31) / 32);
    for (int r = 0; r < q.tr_count; ++r) b->tb.push_back(TraceBlock{p, r});
    const int nob = (int)((q.n + kOutB - 1) / kOutB);
    for (int j = -1; j < q.k; ++j)
      for (int bi = 0; bi < nob; ++bi)
        for (int bj = 0; bj < nob; ++bj) b->ob.push_back(OutBlock{p, j, bi, bj});
    for (int c = 0; c < nch; ++c)
      b->c0.push_back(Chunk{p, -1, (int64_t)c * kChunkVec, std::min<int64_t>(vec, (int64_t)(c + 1) * kChunkVec)});
    for (int j = 0; j < q.k; ++j) {
      q.u1_first[j] = (int)b->c1.size();
      q.u1_count[j] = nch;
      for (int c = 0; c < nch; ++c)
        b->c1.push_back(Chunk{p, j, (int64_t)c * kChunkVec, std::min<int64_t>(vec, (int64_t)(c + 1) * kChunkVec)});
    }
  }
  b->total_k = h1;
  hipError_t e = hipSuccess;
  float* fbase = nullptr;
  uint16_t* hbase = nullptr;
  LayerState* sbase = nullptr;
  auto get = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = balloc(b, ptr, bytes);
  };
  get((void**)&fbase, f32 * 4);
  get((void**)&hbase, u16 * 2);
  get((void**)&sbase, sizeof(LayerState) * count);
  get((void**)&b->dp, sizeof(BatchProblem) * count);
  get((void**)&b->dc0, sizeof(Chunk) * b->c0.size());
  get((void**)&b->dc1, sizeof(Chunk) * b->c1.size());
  get((void**)&b->dtb, sizeof(TraceBlock) * b->tb.size());
  if (b->ob.size() > (size_t)INT32_MAX || b->c0.size() > (size_t)INT32_MAX ||
      b->c1.size() > (size_t)INT32_MAX || b->tb.size() > (size_t)INT32_MAX)
    return bail(DMPT_EINVAL, "batch too large for one launch grid");
  get((void**)&b->dob, sizeof(OutBlock) * b->ob.size());
  get((void**)&b->part_tr, sizeof(double) * b->tb.size());
  get((void**)&b->part_g, sizeof(double) * 3 * b->tb.size());
  get((void**)&b->part1m, sizeof(double) * b->c1.size());
  get((void**)&b->desc, sizeof(ProblemDesc) * count);
  size_t n_big = 0, n_small = 0;
  for (auto& q : b->hp) {
    const int Tb = (int)((q.n + 255) / 256), Ts = (int)((q.n + 127) / 128);
    n_big += (size_t)(1 + q.k) * Tb * (Tb + 1) / 2;
    n_small += (size_t)(1 + q.k) * Ts * (Ts + 1) / 2;
  }
  // balanced rounds add placeholders: at most as many as there are items
  get((void**)&b->items[0], sizeof(TileItem) * 2 * n_big);
  get((void**)&b->items[1], sizeof(TileItem) * 2 * n_small);
  get((void**)&b->part_f, sizeof(double) * 2 * (n_big + n_small));
  get((void**)&b->part_m, sizeof(double) * 2 * (n_big + n_small));
  get((void**)&b->h0tab, sizeof(void*) * count);
  get((void**)&b->p0tab, sizeof(void*) * count);
  get((void**)&b->h1tab, sizeof(void*) * h1);
  get((void**)&b->p1tab, sizeof(void*) * h1);
  get((void**)&b->dsum, sizeof(ProblemSummary) * count);
  if (e != hipSuccess)
    return bail(e == hipErrorOutOfMemory ? DMPT_ENOMEM : DMPT_EHIP, "device allocation failed");
  if (hipHostMalloc((void**)&b->host_tab, sizeof(void*) * 2 * (count + h1), 0) != hipSuccess ||
      hipHostMalloc((void**)&b->hsum, sizeof(ProblemSummary) * count, 0) != hipSuccess)
    return bail(DMPT_ENOMEM, "pinned allocation failed");
  // carve the per-problem buffers (every block a multiple of 256 bytes)
  size_t fo = 0, ho = 0;
  for (int p = 0; p < count; ++p) {
    BatchProblem& q = b->hp[p];
    const size_t m = (size_t)q.np * q.ld, pm = (size_t)q.np * q.np;
    q.st = sbase + p;
    q.s_master = fbase + fo; fo += m;
    for (int j = 0; j < q.k; ++j) {
      q.s1buf[j][0] = fbase + fo; fo += m;
      q.s1buf[j][1] = fbase + fo; fo += m;
    }
    for (int par = 0; par < 2; ++par) {
      q.s_hi[par] = hbase + ho; ho += pm;
      q.s_lo[par] = hbase + ho; ho += pm;
      for (int j = 0; j < q.k; ++j) {
        q.s1_hi[j][par] = hbase + ho; ho += pm;
        q.s1_lo[j][par] = hbase + ho; ho += pm;
      }
    }
  }
  // the products never write outside each problem's k extent: start from zero
  if (hipMemset(fbase, 0, f32 * 4) != hipSuccess || hipMemset(hbase, 0, u16 * 2) != hipSuccess ||
      hipMemset(sbase, 0, sizeof(LayerState) * count) != hipSuccess ||
      hipMemcpy(b->dc0, b->c0.data(), sizeof(Chunk) * b->c0.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->dc1, b->c1.data(), sizeof(Chunk) * b->c1.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->dtb, b->tb.data(), sizeof(TraceBlock) * b->tb.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->dob, b->ob.data(), sizeof(OutBlock) * b->ob.size(), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bail(DMPT_EHIP, "workspace set-up failed");
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)
    return bail(DMPT_EHIP, "stream/event creation failed");
  if (opt.tile_threshold >= 0) {
    if (build_class_items(b, opt.tile_threshold) != hipSuccess)
      return bail(DMPT_EHIP, "tile item set-up failed");
  } else if (autotune(b) != hipSuccess) {
    return bail(DMPT_EHIP, "tile autotuning failed");
  }
  *out = b;
  return DMPT_OK;
}

dmpt_status dmpt_batch_response(dmpt_batch* b, const double* const* H0, const double* const* H1,
                                double* const* P0, double* const* P1, dmpt_problem_stats* st,
                                double* ms) {
  if (!b || !H0 || !H1 || !P1) return bfail(DMPT_EINVAL, "NULL argument");
  const int P = b->count, K = b->total_k;
  void** h = b->host_tab;
  for (int p = 0; p < P; ++p) {
    h[p] = (void*)H0[p];
    h[P + p] = P0 ? (void*)P0[p] : nullptr;
    if (!H0[p]) return bfail(DMPT_EINVAL, "NULL H0[p]");
  }
  for (int i = 0; i < K; ++i) {
    h[2 * P + i] = (void*)H1[i];
    h[2 * P + K + i] = (void*)P1[i];
    if (!H1[i] || !P1[i]) return bfail(DMPT_EINVAL, "NULL H1 or P1 entry");
  }
  hipStream_t s = b->stream;
  BCHK(hipMemcpyAsync(b->h0tab, h, sizeof(void*) * P, hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(b->p0tab, h + P, sizeof(void*) * P, hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(b->h1tab, h + 2 * P, sizeof(void*) * K, hipMemcpyHostToDevice, s));
  BCHK(hipMemcpyAsync(b->p1tab, h + 2 * P + K, sizeof(void*) * K, hipMemcpyHostToDevice, s));
  BCHK(hipEventRecord(b->ev0, s));
  if (b->use_graph) {
    if (!b->exec) {
      BCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      hipError_t ce = enqueue(b, b->cap);
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(b->cap, &g);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(DMPT_EHIP, std::string("graph capture: ") +
                                    hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      b->graph = g;
      BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    BCHK(hipGraphLaunch(b->exec, s));
  } else {
    BCHK(enqueue(b, s));
  }
  BCHK(hipEventRecord(b->ev1, s));
  BCHK(hipMemcpyAsync(b->hsum, b->dsum, sizeof(ProblemSummary) * P, hipMemcpyDeviceToHost, s));
  BCHK(hipStreamSynchronize(s));
  float t_ms = 0.f;
  if (hipEventElapsedTime(&t_ms, b->ev0, b->ev1) != hipSuccess) t_ms = 0.f;
  if (ms) *ms = t_ms;
  int err = 0, noconv = 0;
  for (int p = 0; p < P; ++p) {
    const ProblemSummary& q = b->hsum[p];
    if (q.error) err = q.error;
    if (!q.converged) noconv = 1;
    if (st) {
      st[p].layers = q.layers;
      st[p].d0_layer = q.d0_layer;
      st[p].converged = q.converged;
      st[p].k = b->hp[p].k;
      for (int j = 0; j < kMaxKB; ++j) st[p].d1_layer[j] = q.d1_layer[j];
      st[p].idem0 = q.idem0;
      for (int j = 0; j < kMaxKB; ++j) st[p].idem1[j] = q.idem1[j];
    }
  }
  if (err) return bfail((dmpt_status)err, "non-finite value or split overflow in a problem");
  if (noconv) return bfail(DMPT_ENOCONV, "layer cap reached before every D1 test fired");
  return DMPT_OK;
}

dmpt_status dmpt_batch_info(const dmpt_batch* b, int32_t* threshold, int32_t* n_items_256,
                            int32_t* n_items_128) {
  if (!b) return bfail(DMPT_EINVAL, "NULL batch");
  if (threshold) *threshold = b->threshold;
  if (n_items_256) *n_items_256 = b->n_items[0];
  if (n_items_128) *n_items_128 = b->n_items[1];
  return DMPT_OK;
}

void dmpt_batch_destroy(dmpt_batch* b) { batch_free(b); }

}  // extern "C"
