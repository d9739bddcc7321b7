// C ABI and host driver of the DNN-SP2-PT layer loop (Algorithm 1).
//
// The host only enqueues kernels: every decision of Algorithms 1-3 is taken
// by single-workgroup kernels on the device and stored in a LayerState, which
// the layer kernels read.  The host looks at the device stop flag every
// `poll_every` layers; kernels of layers enqueued after the stop return at once.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "dmpt_internal.h"

using namespace dmpt;

namespace {

thread_local std::string g_err;

dmpt_status fail(dmpt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

void dmpt::set_last_error(const char* msg) { g_err = msg; }

std::vector<int32_t> dmpt::balanced_rounds(const std::vector<int64_t>& cost, int grid,
                                           size_t limit) {
  const int n = (int)cost.size();
  std::vector<int32_t> plain(n);
  for (int i = 0; i < n; ++i) plain[i] = i;
  if (n <= grid || grid <= 0) return plain;
  int64_t total = 0, biggest = 1;
  for (int64_t c : cost) {
    total += c;
    biggest = std::max(biggest, c);
  }
  int64_t target = std::max<int64_t>((total + grid - 1) / grid, biggest);
  std::vector<int64_t> load(grid, 0);
  std::vector<int32_t> out;
  int pos = 0;
  while (pos < n) {
    bool placed = false;
    for (int s = 0; s < grid && pos < n; ++s) {
      if (load[s] + cost[pos] <= target) {
        load[s] += cost[pos];
        out.push_back(pos++);
        placed = true;
      } else {
        out.push_back(-1);
      }
    }
    if (out.size() > limit) return plain;
    if (!placed) ++target;
  }
  while (!out.empty() && out.back() < 0) out.pop_back();
  return out;
}

namespace {

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return fail(DMPT_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));       \
  } while (0)

bool is_split(dmpt_precision p) { return p == DMPT_SPLIT_FP16 || p == DMPT_SPLIT_BF16; }
size_t elem_bytes(dmpt_precision p) { return p == DMPT_FP64 ? 8 : 4; }
int lo_shift(dmpt_precision p) {
  return p == DMPT_SPLIT_FP16 ? kLoShiftF16 : (p == DMPT_SPLIT_BF16 ? kLoShiftBF16 : 0);
}

// Row stride of the workspace matrices: Np plus a pad of 128 elements, so
// that the rows of a panel (Np is a multiple of 256) do not all map onto the
// same L2 channels; at N = 16384 this raises the L2 hit rate of the products
// from 46% to 87%.  The pad columns hold zeros.  DMPT_LD_PAD (elements,
// multiple of 8) overrides it.
int64_t row_stride(int64_t np) {
  const char* env = getenv("DMPT_LD_PAD");
  int64_t pad = 128;
  if (env) pad = atoll(env);
  if (pad < 0 || pad % 8 != 0) pad = 128;
  return np + pad;
}

// Upper-triangle tiles of each output, grouped 8 tile-rows at a time and
// walked column by column, so that consecutive items share row panels.
// Responses first (two products per tile), then X = S^2.
std::vector<TileItem> build_items(int T, int k) {
  std::vector<TileItem> v;
  const int GR = 8;
  auto add_out = [&](int out) {
    for (int g0 = 0; g0 < T; g0 += GR) {
      const int g1 = std::min(T, g0 + GR);
      for (int tj = g0; tj < T; ++tj)
        for (int ti = g0; ti < std::min(g1, tj + 1); ++ti) {
          TileItem it;
          it.out = (int16_t)out;
          it.prob = 0;
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

// Single-problem lists: response tiles cost two products, tiles of X one.
std::vector<TileItem> balanced_items(const std::vector<TileItem>& items, int grid) {
  std::vector<int64_t> cost(items.size());
  for (size_t i = 0; i < items.size(); ++i) cost[i] = items[i].out == 0 ? 1 : 2;
  const std::vector<int32_t> order = balanced_rounds(cost, grid, 2 * items.size());
  std::vector<TileItem> out(order.size());
  for (size_t q = 0; q < order.size(); ++q) {
    if (order[q] >= 0) {
      out[q] = items[order[q]];
    } else {
      out[q].out = -1;
      out[q].prob = 0;
      out[q].ti = out[q].tj = 0;
    }
  }
  return out;
}

// Tile edge of a single problem's fused layer launch for k responses.  The
// 256-row launch (one workgroup per CU) needs several work units per CU to
// balance: with (1 + 2k) T (T + 1) / 2 units of 256-row tiles over the CUs
// below 3.4 per CU (N up to about 4096 for one response) the 128-row launch
// (two workgroups per CU, four times the units) finishes first.  Measured,
// split FP16, one box: N = 2048, k = 1: 9.0 against 14.5 ms per response;
// N = 4096, k = 1: 35.0 against 34.8; N = 4096 second order: 64.1 against
// 73.8; N = 6144: 99.3 against 93.6; N = 8192: 241 against 222.  Contexts
// that keep adjoint checkpoints stay on 256-row tiles: the adjoint's forward
// replay runs the same items through the 256-row non-fused kernel.
int fused_tile(int64_t N, int k, int cus, bool adjoint) {
  if (adjoint) return 256;
  const int64_t T = (N + 255) / 256;
  const double per_cu = (double)(1 + 2 * k) * T * (T + 1) / 2 / (cus > 0 ? cus : 256);
  return per_cu < 3.4 ? 128 : 256;
}

// Item positions of the fused launch for k responses on `grid` workgroups,
// and the per-item partial-slot capacity of a context sized for k_max.  The
// plan of balanced_items keeps at most twice the item count (its limit), and
// the item count grows with k, so 2 (1 + k_max) T (T + 1) / 2 covers every
// k <= k_max even though placeholders make the plan length non-monotonic in k.
int64_t fused_positions(int T, int k, int grid) {
  return (int64_t)balanced_items(build_items(T, k), grid).size();
}
int64_t fused_slot_capacity(int T, int k_max) {
  return 2 * (int64_t)(1 + k_max) * T * (T + 1) / 2;
}

// Items of the adjoint products: every tile of outputs 1 .. m (one general
// product each), bands of 8 tile rows walked column by column.
std::vector<TileItem> build_items_all_tiles(int T, int m) {
  std::vector<TileItem> v;
  const int GR = 8;
  for (int out = 1; out <= m; ++out)
    for (int g0 = 0; g0 < T; g0 += GR)
      for (int tj = 0; tj < T; ++tj)
        for (int ti = g0; ti < std::min(T, g0 + GR); ++ti) {
          TileItem it;
          it.out = (int16_t)out;
          it.prob = 0;
          it.ti = ti;
          it.tj = tj;
          v.push_back(it);
        }
  return v;
}

struct DevAlloc {
  std::vector<void*> ptrs;
  hipError_t get(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct dmpt_ctx {
  dmpt_precision prec;
  int64_t n, nocc, np, ld;
  int ftile[kMaxK + 1];   // split forms: tile edge of the fused launch for k responses
  int k_max, max_layers, poll, check_sym;
  hipStream_t stream;
  LayerState* st;
  void* s_init;
  void* s_master;
  void* s_hi[2];      // split forms: 16-bit split of S (two buffers, see ProblemDesc)
  void* s_lo[2];
  void* x;            // X = S^2 (direct forms and the adjoint's recomputation)
  void* s1buf[kMaxK][2];
  void* s1_hi[kMaxK][2];
  void* s1_lo[kMaxK][2];
  ProblemDesc* desc;  // split forms: buffers of the fused layer (device)
  double* part_f;     // split forms: per-item partials of the fused layer
  double* part_m;
  int64_t part_cap;   // entries of part_f / part_m (fused_slot_capacity)
  TraceBlock* tblocks;// split forms: diagonal blocks of Tr X
  int n_tblocks;
  double* part_tr;
  double* part;       // reduction partials
  double* dscal;      // device scalars (traces)
  int32_t* dflag;
  TileItem* items[kMaxK + 1];
  int n_items[kMaxK + 1];
  LayerState* hstate; // pinned host copy
  int32_t* hflag;     // pinned host flag
  double* hscal;      // pinned host scalars
  hipEvent_t ev0, ev1;
  int timing;
  hipEvent_t pev[2 * kMaxLayers];  // per-layer product launch bracket (timing on)
  // adjoint support (ckpt_every > 0)
  int ckpt;                        // checkpoint interval in layers
  int nslots;                      // checkpoint slots: layers 0, c, 2c, ...
  std::vector<void*> ck_s, ck_s1;  // [slot], [slot * k_max + j]
  std::vector<void*> seg_s, seg_s1;// [i], [i * k_max + j], i = 1..c (i = 0: the checkpoint)
  void* sh;                        // adjoint of S
  void* sh1[kMaxK];                // adjoints of S1_j
  void* t2;                        // S Sh + Sh S
  void* t1[kMaxK];                 // S Sh1_j + Sh1_j S
  void* t3[kMaxK];                 // Sh1_j S1_j + S1_j Sh1_j
  LayerState* st_rep;              // replay state
  TileItem* adj_items[4];          // outputs 1 .. 1 + 2k of the adjoint products, k = 1..3
  int adj_n_items[4];
  int last_k;                      // k of the last response (0: none)
  DevAlloc mem;
};

namespace {

constexpr size_t kPartFro0 = 0;
constexpr size_t kPartFro1 = kRedBlocks;
constexpr size_t kPartMax1 = kPartFro1 + (size_t)kMaxK * kRedBlocks;
constexpr size_t kPartGersh = kPartMax1 + (size_t)kMaxK * kRedBlocks;
constexpr size_t kPartMaxabs = kPartGersh + 3 * 512;
constexpr size_t kPartTotal = kPartMaxabs + kRedBlocks;

void ctx_free(dmpt_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->mem.release();
  if (c->hstate) (void)hipHostFree(c->hstate);
  if (c->hflag) (void)hipHostFree(c->hflag);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (int i = 0; i < 2 * kMaxLayers; ++i)
    if (c->pev[i]) (void)hipEventDestroy(c->pev[i]);
  delete c;
}

dmpt_status check_symmetric(const double* H, int64_t n, int32_t* dflag, int32_t* hflag,
                            hipStream_t s, const char* what) {
  HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int32_t), s));
  HIPCHK(launch_symcheck(H, n, dflag, s));
  HIPCHK(hipMemcpyAsync(hflag, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (*hflag == 1) return fail(DMPT_EASYM, std::string(what) + " is not exactly symmetric");
  if (*hflag == 2) return fail(DMPT_ENONFINITE, std::string(what) + " has a non-finite entry");
  return DMPT_OK;
}

// Gershgorin bounds and the normalised S0 of H0 into the context (Algorithm 1
// initial transform).  No allocation.
dmpt_status normalise(dmpt_ctx* c, const double* H0) {
  if (c->check_sym) {
    dmpt_status r = check_symmetric(H0, c->n, c->dflag, c->hflag, c->stream, "H0");
    if (r != DMPT_OK) return r;
  }
  hipStream_t s = c->stream;
  c->last_k = 0;   // checkpoints and decisions of an earlier response no longer apply
  HIPCHK(hipMemsetAsync(c->st, 0, sizeof(LayerState), s));
  HIPCHK(launch_gershgorin(H0, c->n, c->part + kPartGersh, c->st, c->dscal, s));
  HIPCHK(launch_init_s0(c->prec, H0, c->n, c->np, c->ld, c->st, c->s_init, s));
  HIPCHK(hipMemcpyAsync(c->hstate, c->st, sizeof(LayerState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (c->hstate->error) return fail((dmpt_status)c->hstate->error, "non-finite Gershgorin bounds");
  return DMPT_OK;
}

}  // namespace

extern "C" {

void dmpt_default_options(dmpt_options* opt) {
  if (!opt) return;
  opt->precision = DMPT_SPLIT_FP16;
  opt->max_layers = 100;
  opt->check_symmetry = 0;
  opt->poll_every = 0;
  opt->timing = 0;
  opt->ckpt_every = 0;
  opt->graph = 1;
  opt->tile_threshold = -1;
}

const char* dmpt_status_str(dmpt_status s) {
  switch (s) {
    case DMPT_OK: return "DMPT_OK";
    case DMPT_EINVAL: return "DMPT_EINVAL";
    case DMPT_ENOMEM: return "DMPT_ENOMEM";
    case DMPT_EHIP: return "DMPT_EHIP";
    case DMPT_ENOCONV: return "DMPT_ENOCONV";
    case DMPT_ENONFINITE: return "DMPT_ENONFINITE";
    case DMPT_EASYM: return "DMPT_EASYM";
    case DMPT_ENOTSUP: return "DMPT_ENOTSUP";
  }
  return "DMPT_UNKNOWN";
}

const char* dmpt_last_error(void) { return g_err.c_str(); }

dmpt_status dmpt_init(dmpt_ctx** out, const double* H0, int64_t N, int64_t Nocc, int32_t k_max,
                      const dmpt_options* opt_in, void* stream) {
  if (!out) return fail(DMPT_EINVAL, "ctx pointer is NULL");
  *out = nullptr;
  dmpt_options opt;
  dmpt_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (!H0) return fail(DMPT_EINVAL, "H0 is NULL");
  if (N < 1 || N > (1 << 17)) return fail(DMPT_EINVAL, "N out of range");
  if (Nocc <= 0 || Nocc >= N) return fail(DMPT_EINVAL, "need 0 < Nocc < N");
  if (k_max < 1 || k_max > kMaxK) return fail(DMPT_EINVAL, "k_max out of [1, DMPT_MAX_K]");
  if (opt.precision < DMPT_FP64 || opt.precision > DMPT_SPLIT_FP16)
    return fail(DMPT_ENOTSUP, "unknown precision");
  if (opt.max_layers <= 0) opt.max_layers = 100;
  if (opt.max_layers > kMaxLayers) return fail(DMPT_EINVAL, "max_layers above DMPT_MAX_LAYERS");

  dmpt_ctx* c = new dmpt_ctx();  // value-initialised: every pointer NULL
  c->prec = (dmpt_precision)opt.precision;
  c->n = N;
  c->nocc = Nocc;
  const int tile = product_tile(c->prec);
  c->np = (N + tile - 1) / tile * tile;
  c->ld = row_stride(c->np);
  c->k_max = k_max;
  c->max_layers = opt.max_layers;
  c->check_sym = opt.check_symmetry;
  c->poll = opt.poll_every > 0 ? opt.poll_every : (c->np >= 2048 ? 1 : 4);
  c->stream = (hipStream_t)stream;

  auto bail = [&](dmpt_status s, const std::string& m) {
    ctx_free(c);
    return fail(s, m);
  };
  const size_t eb = elem_bytes(c->prec);
  const size_t mat = (size_t)c->np * c->ld;
  hipError_t e = hipSuccess;
  auto get = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = c->mem.get(p, bytes);
  };
  get((void**)&c->st, sizeof(LayerState));
  get(&c->s_init, mat * eb);
  get(&c->s_master, mat * eb);
  const bool split = is_split(c->prec);
  c->ckpt = opt.ckpt_every > 0 ? opt.ckpt_every : 0;
  if (!split || c->ckpt) get(&c->x, mat * eb);
  const size_t pmat = (size_t)c->np * c->np;   // panel-major 16-bit operands
  if (split)
    for (int b = 0; b < 2; ++b) {
      get(&c->s_hi[b], pmat * 2);
      get(&c->s_lo[b], pmat * 2);
    }
  for (int j = 0; j < k_max; ++j) {
    get(&c->s1buf[j][0], mat * eb);
    get(&c->s1buf[j][1], mat * eb);
    if (split)
      for (int b = 0; b < 2; ++b) {
        get(&c->s1_hi[j][b], pmat * 2);
        get(&c->s1_lo[j][b], pmat * 2);
      }
  }
  get((void**)&c->part, kPartTotal * sizeof(double));
  get((void**)&c->dscal, 16 * sizeof(double));
  get((void**)&c->dflag, 16 * sizeof(int32_t));
  if (c->ckpt) {
    // checkpoints of (S, S1_j) at layers 0, c, 2c, ... and one segment of c + 1 layers
    c->nslots = c->max_layers / c->ckpt + 1;
    c->ck_s.assign(c->nslots, nullptr);
    c->ck_s1.assign((size_t)c->nslots * k_max, nullptr);
    c->seg_s.assign(c->ckpt + 1, nullptr);
    c->seg_s1.assign((size_t)(c->ckpt + 1) * k_max, nullptr);
    for (auto& p : c->ck_s) get(&p, mat * eb);
    for (auto& p : c->ck_s1) get(&p, mat * eb);
    // segment store: S_{b+i}, S1_{b+i} for i = 1 .. c (i = 0 is the checkpoint)
    for (size_t i = 1; i < c->seg_s.size(); ++i) get(&c->seg_s[i], mat * eb);
    for (size_t i = (size_t)k_max; i < c->seg_s1.size(); ++i) get(&c->seg_s1[i], mat * eb);
    get(&c->sh, mat * eb);
    get(&c->t2, mat * eb);
    for (int j = 0; j < k_max && j < 3; ++j) {
      get(&c->sh1[j], mat * eb);
      get(&c->t1[j], mat * eb);
      get(&c->t3[j], mat * eb);
    }
    get((void**)&c->st_rep, sizeof(LayerState));
    const int Ta = (int)(c->np / product_tile(c->prec == DMPT_FP64 ? DMPT_FP64 : DMPT_FP32));
    for (int k = 1; k <= 3 && k <= k_max; ++k) {
      std::vector<TileItem> items = build_items_all_tiles(Ta, 1 + 2 * k);
      c->adj_n_items[k] = (int)items.size();
      get((void**)&c->adj_items[k], items.size() * sizeof(TileItem));
      if (e == hipSuccess)
        e = hipMemcpy(c->adj_items[k], items.data(), items.size() * sizeof(TileItem),
                      hipMemcpyHostToDevice);
    }
    // outputs of the adjoint products leave the pad columns untouched
    if (e == hipSuccess) e = hipMemset(c->t2, 0, mat * eb);
    for (int j = 0; j < k_max && j < 3 && e == hipSuccess; ++j) {
      e = hipMemset(c->t1[j], 0, mat * eb);
      if (e == hipSuccess) e = hipMemset(c->t3[j], 0, mat * eb);
    }
  }
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  for (int k = 1; k <= k_max; ++k) {
    // split forms: the fused launch's tile and its rounds balanced over its
    // workgroups (the 256-row launch runs one per CU, the 128-row one two)
    c->ftile[k] = split ? fused_tile(N, k, cus, c->ckpt > 0) : tile;
    const int T = split ? (int)((N + c->ftile[k] - 1) / c->ftile[k]) : (int)(c->np / tile);
    const int fgrid = c->ftile[k] == 128 ? 2 * cus : cus;
    std::vector<TileItem> items = split ? balanced_items(build_items(T, k), fgrid)
                                        : build_items(T, k);
    c->n_items[k] = (int)items.size();
    get((void**)&c->items[k], items.size() * sizeof(TileItem));
    if (e == hipSuccess)
      e = hipMemcpy(c->items[k], items.data(), items.size() * sizeof(TileItem),
                    hipMemcpyHostToDevice);
  }
  if (split) {
    // one slot per item position of every k <= k_max (the plan's length is
    // not monotonic in k: placeholders of balanced rounds)
    // slots for the larger of the two tilings' plans
    c->part_cap = fused_slot_capacity((int)((N + 127) / 128), k_max);
    for (int k = 1; k <= k_max; ++k)
      if (c->n_items[k] > c->part_cap) return bail(DMPT_EINVAL, "item plan exceeds slot capacity");
    get((void**)&c->part_f, (size_t)c->part_cap * sizeof(double));
    get((void**)&c->part_m, (size_t)c->part_cap * sizeof(double));
    get((void**)&c->desc, sizeof(ProblemDesc));
    c->n_tblocks = (int)((N + 31) / 32);
    get((void**)&c->tblocks, (size_t)c->n_tblocks * sizeof(TraceBlock));
    get((void**)&c->part_tr, (size_t)c->n_tblocks * sizeof(double));
    if (e == hipSuccess) {
      std::vector<TraceBlock> tb(c->n_tblocks);
      for (int b = 0; b < c->n_tblocks; ++b) tb[b] = TraceBlock{0, b};
      e = hipMemcpy(c->tblocks, tb.data(), tb.size() * sizeof(TraceBlock), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
      ProblemDesc d;
      memset(&d, 0, sizeof(d));
      for (int b = 0; b < 2; ++b) {
        d.s_hi[b] = c->s_hi[b];
        d.s_lo[b] = c->s_lo[b];
        for (int j = 0; j < k_max; ++j) {
          d.s1_hi[j][b] = c->s1_hi[j][b];
          d.s1_lo[j][b] = c->s1_lo[j][b];
          d.s1m[j][b] = (float*)c->s1buf[j][b];
        }
      }
      d.s_master = (float*)c->s_master;
      d.state = c->st;
      d.ld = c->ld;
      d.kdim = (N + kPanelK - 1) / kPanelK * kPanelK;
      d.pdim = c->np;
      e = hipMemcpy(c->desc, &d, sizeof(d), hipMemcpyHostToDevice);
    }
  }
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return bail(DMPT_ENOMEM, "device allocation failed");
  // the products never write the pad columns of X and X1: they must start at zero
  if (e == hipSuccess && c->x) e = hipMemset(c->x, 0, mat * eb);
  for (int j = 0; j < k_max && e == hipSuccess; ++j) {
    e = hipMemset(c->s1buf[j][0], 0, mat * eb);
    if (e == hipSuccess) e = hipMemset(c->s1buf[j][1], 0, mat * eb);
  }
  if (e != hipSuccess) return bail(DMPT_EHIP, std::string("allocation: ") + hipGetErrorString(e));
  if (hipHostMalloc((void**)&c->hstate, sizeof(LayerState), 0) != hipSuccess ||
      hipHostMalloc((void**)&c->hflag, 16 * sizeof(int32_t), 0) != hipSuccess ||
      hipHostMalloc((void**)&c->hscal, 16 * sizeof(double), 0) != hipSuccess)
    return bail(DMPT_ENOMEM, "pinned host allocation failed");
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
    return bail(DMPT_EHIP, "event creation failed");
  c->timing = opt.timing;
  if (c->timing)
    for (int i = 0; i < 2 * c->max_layers; ++i)
      if (hipEventCreate(&c->pev[i]) != hipSuccess) return bail(DMPT_EHIP, "event creation failed");
  dmpt_status r = normalise(c, H0);
  if (r != DMPT_OK) {
    std::string m = g_err;
    return bail(r, m);
  }
  *out = c;
  return DMPT_OK;
}

dmpt_status dmpt_set_hamiltonian(dmpt_ctx* c, const double* H0) {
  if (!c || !H0) return fail(DMPT_EINVAL, "NULL argument");
  return normalise(c, H0);
}

void dmpt_destroy(dmpt_ctx* ctx) { ctx_free(ctx); }

}  // extern "C"

namespace {

// The layer loop of Algorithm 1 for k1 first-order responses and, with order2,
// the second-order chain of the first perturbation in response slot k1
// (initial matrix -H2/(eps_N - eps_1), zero when H2 is NULL; result into P2).
dmpt_status run_response(dmpt_ctx* c, const double* const* H1, int k1, bool order2,
                         const double* H2, double* P0, double* const* P1, double* P2,
                         dmpt_stats* stats) {
  const int k = k1 + (order2 ? 1 : 0);   // response slots
  auto slot_in = [&](int j) -> const double* { return j < k1 ? H1[j] : H2; };
  auto slot_out = [&](int j) -> double* { return j < k1 ? P1[j] : P2; };
  if (k > c->k_max) return fail(DMPT_EINVAL, "more response slots than the context holds");
  if (is_split(c->prec) && c->n_items[k] > c->part_cap)
    return fail(DMPT_EINVAL, "fused launch has more item positions than partial slots");
  hipStream_t s = c->stream;
  if (c->check_sym)
    for (int j = 0; j < k; ++j) {
      if (!slot_in(j)) continue;
      dmpt_status r = check_symmetric(slot_in(j), c->n, c->dflag, c->hflag, s, "H1");
      if (r != DMPT_OK) return r;
    }
  const dmpt_precision prec = c->prec;
  const int t = lo_shift(prec);
  const int split = is_split(prec) ? 1 : 0;
  const int64_t ld = c->ld, np = c->np, elems = np * ld;

  HIPCHK(hipEventRecord(c->ev0, s));
  HIPCHK(launch_reset_state(c->st, k, order2 ? k1 : -1, c->max_layers, (double)c->nocc, c->n, s));
  HIPCHK(launch_load_s0(prec, c->s_init, c->s_master, c->s_hi[0], c->s_lo[0], np, ld, t, s));
  for (int j = 0; j < k; ++j)
    HIPCHK(launch_init_s1(prec, slot_in(j), c->n, np, ld, c->st, j, c->part + kPartMaxabs,
                          c->s1buf[j][0], c->s1_hi[j][0], c->s1_lo[j][0], t, 0.0, s));

  const size_t mbytes = (size_t)elems * elem_bytes(prec);
  auto save_ckpt = [&](int layer) -> hipError_t {
    const int slot = layer / c->ckpt;
    if (slot >= c->nslots) return hipSuccess;
    hipError_t e2 = hipMemcpyAsync(c->ck_s[slot], c->s_master, mbytes, hipMemcpyDeviceToDevice, s);
    for (int j = 0; j < k && e2 == hipSuccess; ++j)
      e2 = hipMemcpyAsync(c->ck_s1[(size_t)slot * c->k_max + j], c->s1buf[j][layer & 1], mbytes,
                          hipMemcpyDeviceToDevice, s);
    return e2;
  };
  c->last_k = 0;
  if (c->ckpt) HIPCHK(save_ckpt(0));

  ProductArgs pa;
  memset(&pa, 0, sizeof(pa));
  pa.items = c->items[k];
  pa.n_items = c->n_items[k];
  pa.lo_shift = t;
  if (split) {
    // fused layer: decisions, then products with the update in their epilogue
    pa.probs = c->desc;
    pa.part_f = c->part_f;
    pa.part_m = c->part_m;
    pa.slot_base = 0;
  } else {
    pa.s_hi = c->s_master;
    pa.x = c->x;
    pa.state = c->st;
    pa.ld = ld;
    pa.kdim = np;
    pa.s1b[0] = c->s1buf[0][0];
    pa.s1b[1] = c->s1buf[0][1];
  }

  int n = 0;
  bool stopped = false;
  while (n < c->max_layers && !stopped) {
    ++n;
    const int cur = n & 1, prv = cur ^ 1;
    if (split) {
      HIPCHK(launch_trace_diag(prec, c->desc, c->tblocks, c->n_tblocks, c->part_tr, s));
      HIPCHK(launch_predecide(c->st, c->part_tr, c->n_tblocks, s));
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1)], s));
      HIPCHK(launch_products_fused(prec, c->ftile[k], pa, s));
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1) + 1], s));
      HIPCHK(launch_postdecide(c->st, c->items[k], c->n_items[k], c->part_f, c->part_m, t, s));
    } else {
      for (int j = 0; j < k; ++j) {
        pa.s1_hi[j] = c->s1buf[j][prv];
        pa.x1[j] = c->s1buf[j][cur];
      }
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1)], s));
      HIPCHK(launch_products(prec, pa, s));
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1) + 1], s));
      HIPCHK(launch_decide0(prec, c->st, c->x, ld, s));
      HIPCHK(launch_update(prec, c->st, -1, c->x, c->s_master, c->s_master, nullptr, nullptr, np,
                           ld, t, c->part + kPartFro0, nullptr, s));
      for (int j = 0; j < k; ++j)
        HIPCHK(launch_update(prec, c->st, j, c->s1buf[j][cur], c->s1buf[j][prv], c->s1buf[j][cur],
                             nullptr, nullptr, np, ld, t,
                             c->part + kPartFro1 + (size_t)j * kRedBlocks,
                             c->part + kPartMax1 + (size_t)j * kRedBlocks, s));
      HIPCHK(launch_decide1(c->st, c->part + kPartFro0, c->part + kPartFro1, c->part + kPartMax1,
                            split, t, s));
    }
    if (c->ckpt && n % c->ckpt == 0) HIPCHK(save_ckpt(n));
    if (n % c->poll == 0 || n == c->max_layers) {
      HIPCHK(hipMemcpyAsync(c->hflag, &c->st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      stopped = c->hflag[0] != 0;
    }
  }
  if (P0) HIPCHK(launch_copy_out(prec, c->st, -1, c->s_master, c->s_master, ld, P0, c->n, s));
  for (int j = 0; j < k; ++j)
    HIPCHK(launch_copy_out(prec, c->st, j, c->s1buf[j][0], c->s1buf[j][1], ld, slot_out(j), c->n,
                           s));
  HIPCHK(hipEventRecord(c->ev1, s));
  if (P0) HIPCHK(launch_trace(P0, c->n, c->dscal, s));
  for (int j = 0; j < k; ++j) HIPCHK(launch_trace(slot_out(j), c->n, c->dscal + 1 + j, s));
  HIPCHK(hipMemcpyAsync(c->hstate, c->st, sizeof(LayerState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->hscal, c->dscal, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const LayerState& h = *c->hstate;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->layers = h.n;
    stats->d0_layer = h.d0_layer;
    stats->k = k;
    stats->converged = h.converged;
    for (int i = 1; i <= h.n && i <= kMaxLayers; ++i) stats->sigma[i - 1] = (int8_t)h.sigma[i];
    stats->eps1 = h.eps1;
    stats->epsN = h.epsN;
    stats->n_s = h.n_s;
    stats->idem0 = h.fro0;
    stats->trace_p0 = P0 ? c->hscal[0] : 0.0;
    for (int j = 0; j < k; ++j) {
      stats->d1_layer[j] = h.d1_layer[j];
      stats->idem1[j] = h.d1_layer[j] > 0 ? h.fro1[j][h.d1_layer[j]] : 0.0;
      stats->trace_p1[j] = c->hscal[1 + j];
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) ms = 0.f;
    stats->ms = ms;
    stats->x_layers = h.d0_layer > 0 ? h.d0_layer : h.n;
    if (c->timing) {
      // launches of layers after the stop return at once; time only layers 1..h.n
      double tot = 0.0;
      for (int i = 0; i < h.n && i < n; ++i) {
        float t_ms = 0.f;
        if (hipEventElapsedTime(&t_ms, c->pev[2 * i], c->pev[2 * i + 1]) != hipSuccess) t_ms = 0.f;
        tot += t_ms;
      }
      stats->product_ms = tot;
      stats->product_launches = std::min(h.n, n);
    }
  }
  if (h.error) return fail((dmpt_status)h.error, "non-finite value or split overflow in a layer");
  if (!h.converged) return fail(DMPT_ENOCONV, "layer cap reached before every D1 test fired");
  c->last_k = order2 ? 0 : k;          // the adjoint covers first-order responses
  return DMPT_OK;
}

}  // namespace

extern "C" {

dmpt_status dmpt_response(dmpt_ctx* c, const double* const* H1, int32_t k, double* P0,
                          double* const* P1, dmpt_stats* stats) {
  if (!c) return fail(DMPT_EINVAL, "ctx is NULL");
  if (k < 1 || k > c->k_max) return fail(DMPT_EINVAL, "k out of [1, k_max]");
  if (!H1 || !P1) return fail(DMPT_EINVAL, "H1 / P1 array is NULL");
  for (int j = 0; j < k; ++j)
    if (!H1[j] || !P1[j]) return fail(DMPT_EINVAL, "NULL H1[j] or P1[j]");
  return run_response(c, H1, k, false, nullptr, P0, P1, nullptr, stats);
}

dmpt_status dmpt_cpscf(dmpt_ctx* c, const double* H1, dmpt_field_fn field, void* user,
                       double mix, double tol, int32_t max_iter, double* P0, double* P1,
                       double* G, int32_t* iters, double* change, dmpt_stats* stats) {
  if (!c) return fail(DMPT_EINVAL, "ctx is NULL");
  if (!H1 || !field || !P1 || !G) return fail(DMPT_EINVAL, "NULL H1, field, P1 or G");
  if (!(mix > 0.0 && mix <= 1.0) || !(tol > 0.0) || max_iter < 1)
    return fail(DMPT_EINVAL, "need 0 < mix <= 1, tol > 0, max_iter >= 1");
  hipStream_t s = c->stream;
  const int64_t n = c->n;
  const size_t bytes = (size_t)n * n * sizeof(double);
  double *heff = nullptr, *prev = nullptr, *part = nullptr, *dn = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(s);
    if (heff) (void)hipFree(heff);
    if (prev) (void)hipFree(prev);
    if (part) (void)hipFree(part);
    if (dn) (void)hipFree(dn);
  };
  if (hipMalloc((void**)&heff, bytes) != hipSuccess || hipMalloc((void**)&prev, bytes) != hipSuccess ||
      hipMalloc((void**)&part, 2 * kRedBlocks * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&dn, 2 * sizeof(double)) != hipSuccess) {
    release();
    return fail(DMPT_ENOMEM, "allocation failed");
  }
  dmpt_status r = DMPT_OK;
  double ch = INFINITY;
  int it = 0;
  hipError_t e = hipMemcpyAsync(heff, H1, bytes, hipMemcpyDeviceToDevice, s);
  const double* hp[1] = {heff};
  double* pp[1] = {P1};
  if (e == hipSuccess) r = run_response(c, hp, 1, false, nullptr, P0, pp, nullptr, stats);
  while (e == hipSuccess && r == DMPT_OK && it < max_iter) {
    // induced field of the current response, then the mixed effective perturbation
    e = hipMemcpyAsync(prev, P1, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) break;
    field(user, P1, G, (void*)s);
    ++it;
    e = launch_mix(H1, G, heff, mix, n, s);
    if (e != hipSuccess) break;
    r = run_response(c, hp, 1, false, nullptr, P0, pp, nullptr, stats);
    if (r != DMPT_OK) break;
    double h[2] = {0.0, 0.0};
    e = launch_diff_norms(P1, prev, n, part, dn, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h, dn, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    ch = h[1] > 0.0 ? sqrt(h[0] / h[1]) : sqrt(h[0]);
    if (!isfinite(ch)) {
      r = fail(DMPT_ENONFINITE, "self-consistent response diverged");
      break;
    }
    if (ch < tol) break;
  }
  release();
  if (iters) *iters = it;
  if (change) *change = ch;
  c->last_k = 0;                       // the adjoint does not cover the self-consistent loop
  if (e != hipSuccess) return fail(DMPT_EHIP, hipGetErrorString(e));
  if (r != DMPT_OK) return r;
  if (!(ch < tol)) return fail(DMPT_ENOCONV, "self-consistent response: tolerance not reached");
  return DMPT_OK;
}

dmpt_status dmpt_response2(dmpt_ctx* c, const double* H1, const double* H2, double* P0,
                           double* P1, double* P2, dmpt_stats* stats) {
  if (!c) return fail(DMPT_EINVAL, "ctx is NULL");
  if (c->k_max < 2) return fail(DMPT_EINVAL, "second order needs a context with k_max >= 2");
  if (!H1 || !P1 || !P2) return fail(DMPT_EINVAL, "NULL H1, P1 or P2");
  const double* h1[1] = {H1};
  double* p1[1] = {P1};
  return run_response(c, h1, 1, true, H2, P0, p1, P2, stats);
}

dmpt_status dmpt_adjoint(dmpt_ctx* c, const double* const* W, int32_t k, const double* W0,
                         double* dH0, double* const* dH1, dmpt_stats* stats) {
  if (!c) return fail(DMPT_EINVAL, "ctx is NULL");
  if (!c->ckpt) return fail(DMPT_EINVAL, "context created without checkpoints (ckpt_every = 0)");
  if (c->last_k == 0) return fail(DMPT_EINVAL, "no converged dmpt_response to differentiate");
  if (k != c->last_k || k > 3) return fail(DMPT_EINVAL, "k must match the last response (k <= 3)");
  if (!W || !dH1 || !dH0) return fail(DMPT_EINVAL, "NULL argument");
  for (int j = 0; j < k; ++j)
    if (!W[j] || !dH1[j]) return fail(DMPT_EINVAL, "NULL W[j] or dH1[j]");
  hipStream_t s = c->stream;
  const dmpt_precision prec = c->prec;
  const dmpt_precision aprec = prec == DMPT_FP64 ? DMPT_FP64 : DMPT_FP32;   // adjoint products
  const int t = lo_shift(prec);
  const bool split = is_split(prec);
  const int64_t ld = c->ld, np = c->np, elems = np * ld;
  const size_t mbytes = (size_t)elems * elem_bytes(prec);
  const LayerState& h = *c->hstate;   // the forward pass of the last response
  int top = 0;                        // last forward layer whose update reached a P1
  for (int j = 0; j < k; ++j) top = std::max(top, h.d1_layer[j] > 0 ? h.d1_layer[j] - 1 : h.n);
  const int cst = c->ckpt;

  HIPCHK(hipEventRecord(c->ev0, s));
  for (int j = 0; j < k; ++j) HIPCHK(launch_adj_seed(prec, W[j], c->n, np, ld, c->sh1[j], s));
  // The reverse pass starts at layer `top` >= d0 + 1, after S froze at P0 =
  // S_{d0-1}; a loss on P0 therefore seeds Sh there, and the frozen reverse
  // layers pass it on unchanged (plus their S1 terms) down to layer d0 - 1.
  if (W0)
    HIPCHK(launch_adj_seed(prec, W0, c->n, np, ld, c->sh, s));
  else
    HIPCHK(hipMemsetAsync(c->sh, 0, mbytes, s));

  ProductArgs fa;                     // forward replay (layer precision, replay state)
  memset(&fa, 0, sizeof(fa));
  fa.s_hi = split ? c->s_hi[0] : c->s_master;
  fa.s_lo = c->s_lo[0];
  fa.x = c->x;
  fa.items = c->items[k];
  fa.n_items = c->n_items[k];
  fa.state = c->st_rep;
  fa.ld = ld;
  fa.kdim = np;
  fa.lo_shift = t;

  ProductArgs ba;                     // adjoint products: T2, T1_j, T3_j
  memset(&ba, 0, sizeof(ba));
  ba.items = c->adj_items[k];
  ba.n_items = c->adj_n_items[k];
  ba.state = nullptr;
  ba.mode = 3;                        // one product per output on every tile
  ba.ld = ld;
  ba.kdim = np;
  // FP32 reverse products: one accumulator over k.  The gradients' error is
  // the forward's (split BF16 at 7e-4 against 1e-5 from these products), and
  // the blocked sums would cost 9% of the adjoint at N = 4096.
  ba.plain_accum = 1;

  for (int seg = top / cst; seg >= 0; --seg) {
    const int b = seg * cst, e = std::min(b + cst, top);
    if (e <= b) continue;
    // S_{b+i}, S1_{b+i} (i = 0 .. e-1-b): the checkpoint for i = 0, then the
    // segment store.  A layer that leaves S (after D0) or S1_j (after its D1
    // layer) as it was writes nothing, and its entry points at the previous one.
    std::vector<void*> sp(e - b), s1p((size_t)(e - b) * k);
    sp[0] = c->ck_s[seg];
    for (int j = 0; j < k; ++j) s1p[j] = c->ck_s1[(size_t)seg * c->k_max + j];
    auto seg_S = [&](int i) { return sp[i]; };
    auto seg_S1 = [&](int i, int j) { return s1p[(size_t)i * k + j]; };
    // recompute S_{b+1} .. S_{e-1} with the forward's decisions, each layer
    // writing its masters straight into the segment store
    if (e - 1 >= b + 1) {
      if (split) {
        HIPCHK(launch_resplit(prec, c->st, -1, 0, seg_S(0), c->s_hi[0], c->s_lo[0], np, ld, t, s));
        for (int j = 0; j < k; ++j)
          HIPCHK(launch_resplit(prec, c->st, j, b, seg_S1(0, j), c->s1_hi[j][0], c->s1_lo[j][0],
                                np, ld, t, s));
      }
      for (int n = b + 1; n <= e - 1; ++n) {
        const int i = n - b;
        const bool s_upd = h.d0_layer <= 0 || n < h.d0_layer;   // as the forward's flags
        HIPCHK(launch_replay_state(c->st, c->st_rep, n, s));
        fa.s_hi = split ? c->s_hi[0] : seg_S(i - 1);
        for (int j = 0; j < k; ++j) {
          fa.s1_hi[j] = split ? c->s1_hi[j][0] : seg_S1(i - 1, j);
          fa.s1_lo[j] = c->s1_lo[j][0];
          fa.x1[j] = c->seg_s1[(size_t)i * c->k_max + j];   // X1_j, updated in place to S1_j
        }
        HIPCHK(launch_products(prec, fa, s));
        HIPCHK(launch_update(prec, c->st_rep, -1, c->x, seg_S(i - 1), c->seg_s[i], c->s_hi[0],
                             c->s_lo[0], np, ld, t, c->part + kPartFro0, nullptr, s));
        sp[i] = s_upd ? c->seg_s[i] : sp[i - 1];
        for (int j = 0; j < k; ++j) {
          void* x1 = c->seg_s1[(size_t)i * c->k_max + j];
          HIPCHK(launch_update(prec, c->st_rep, j, x1, seg_S1(i - 1, j), x1, c->s1_hi[j][0],
                               c->s1_lo[j][0], np, ld, t,
                               c->part + kPartFro1 + (size_t)j * kRedBlocks,
                               c->part + kPartMax1 + (size_t)j * kRedBlocks, s));
          const bool s1_upd = h.d1_layer[j] <= 0 || n < h.d1_layer[j];
          s1p[(size_t)i * k + j] = s1_upd ? x1 : s1p[(size_t)(i - 1) * k + j];
        }
      }
    }
    // reverse layers e .. b+1
    for (int n = e; n >= b + 1; --n) {
      const int i = n - 1 - b;          // S_{n-1}, S1_{n-1} in the segment store
      ba.s_hi = seg_S(i);
      ba.a_op[0] = nullptr;
      ba.s1_hi[0] = c->sh;
      ba.x1[0] = c->t2;
      for (int j = 0; j < k; ++j) {
        ba.a_op[1 + j] = nullptr;
        ba.s1_hi[1 + j] = c->sh1[j];
        ba.x1[1 + j] = c->t1[j];
        ba.a_op[1 + k + j] = c->sh1[j];
        ba.s1_hi[1 + k + j] = seg_S1(i, j);
        ba.x1[1 + k + j] = c->t3[j];
      }
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1)], s));
      HIPCHK(launch_products(aprec, ba, s));
      if (c->timing) HIPCHK(hipEventRecord(c->pev[2 * (n - 1) + 1], s));
      HIPCHK(launch_adj_update(prec, c->st, n, k, c->t2, c->sh, c->t1, c->sh1, c->t3, np, ld, s));
    }
  }
  HIPCHK(launch_adj_out(prec, c->st, c->sh, ld, dH0, c->n, s));
  for (int j = 0; j < k; ++j) HIPCHK(launch_adj_out(prec, c->st, c->sh1[j], ld, dH1[j], c->n, s));
  HIPCHK(hipEventRecord(c->ev1, s));
  HIPCHK(hipStreamSynchronize(s));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->layers = h.n;
    stats->d0_layer = h.d0_layer;
    stats->k = k;
    stats->converged = h.converged;
    for (int j = 0; j < k; ++j) stats->d1_layer[j] = h.d1_layer[j];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) ms = 0.f;
    stats->ms = ms;
    if (c->timing) {
      // the reverse layers' product launches, one per layer 1 .. top
      double tot = 0.0;
      for (int i = 0; i < top; ++i) {
        float t_ms = 0.f;
        if (hipEventElapsedTime(&t_ms, c->pev[2 * i], c->pev[2 * i + 1]) != hipSuccess) t_ms = 0.f;
        tot += t_ms;
      }
      stats->product_ms = tot;
      stats->product_launches = top;
    }
  }
  return DMPT_OK;
}

dmpt_status dmpt_response_adjoint(dmpt_ctx* c, const double* const* H1, int32_t k,
                                  const double* const* W, const double* W0, double* P0,
                                  double* const* P1, double* dH0, double* const* dH1,
                                  dmpt_stats* stats) {
  if (!c) return fail(DMPT_EINVAL, "ctx is NULL");
  if (!c->ckpt) return fail(DMPT_EINVAL, "context created without checkpoints (ckpt_every = 0)");
  if (k < 1 || k > 3 || k > c->k_max) return fail(DMPT_EINVAL, "k out of [1, min(3, k_max)]");
  if (!W || !dH0 || !dH1) return fail(DMPT_EINVAL, "NULL argument");
  for (int j = 0; j < k; ++j)
    if (!W[j] || !dH1[j]) return fail(DMPT_EINVAL, "NULL W[j] or dH1[j]");
  dmpt_status r = dmpt_response(c, H1, k, P0, P1, stats);
  if (r != DMPT_OK) return r;
  dmpt_stats ast;
  r = dmpt_adjoint(c, W, k, W0, dH0, dH1, stats ? &ast : nullptr);
  if (r == DMPT_OK && stats) {
    stats->ms += ast.ms;
    stats->product_ms += ast.product_ms;
    stats->product_launches += ast.product_launches;
  }
  return r;
}

dmpt_status dmpt_layer_products(int32_t precision, int64_t N, const double* S, const double* S1,
                                double* X, double* X1, void* stream) {
  if (precision < DMPT_FP64 || precision > DMPT_SPLIT_FP16)
    return fail(DMPT_ENOTSUP, "unknown precision");
  if (N < 1 || !S || !X) return fail(DMPT_EINVAL, "bad arguments");
  if ((S1 == nullptr) != (X1 == nullptr)) return fail(DMPT_EINVAL, "S1 and X1 go together");
  const dmpt_precision prec = (dmpt_precision)precision;
  hipStream_t s = (hipStream_t)stream;
  const int tile = product_tile(prec);
  const int64_t np = (N + tile - 1) / tile * tile;
  const int64_t ld = row_stride(np);
  const size_t mat = (size_t)np * ld, eb = elem_bytes(prec);
  const bool split = is_split(prec);
  const int t = lo_shift(prec);
  DevAlloc mem;
  void *sm = nullptr, *sh = nullptr, *sl = nullptr, *tm = nullptr, *th = nullptr, *tl = nullptr;
  void *xo = nullptr, *x1o = nullptr, *items = nullptr;
  double *part = nullptr, *hmax = nullptr;
  hipError_t e = hipSuccess;
  auto get = [&](void** p, size_t b) {
    if (e == hipSuccess) e = mem.get(p, b);
  };
  const size_t pmat = (size_t)np * np;   // panel-major 16-bit operands
  get(&sm, mat * eb);
  get(&xo, mat * eb);
  if (split) {
    get(&sh, pmat * 2);
    get(&sl, pmat * 2);
  }
  if (S1) {
    get(&tm, mat * eb);
    get(&x1o, mat * eb);
    if (split) {
      get(&th, pmat * 2);
      get(&tl, pmat * 2);
    }
  }
  get((void**)&part, kRedBlocks * sizeof(double));
  const int T = (int)(np / tile);
  std::vector<TileItem> it = build_items(T, S1 ? 1 : 0);
  get(&items, it.size() * sizeof(TileItem));
  if (e != hipSuccess) {
    mem.release();
    return fail(e == hipErrorOutOfMemory ? DMPT_ENOMEM : DMPT_EHIP, "allocation failed");
  }
  auto done = [&](dmpt_status st, const std::string& m) {
    (void)hipStreamSynchronize(s);
    mem.release();
    if (hmax) (void)hipHostFree(hmax);
    return st == DMPT_OK ? DMPT_OK : fail(st, m);
  };
  if (hipHostMalloc((void**)&hmax, sizeof(double) * kRedBlocks, 0) != hipSuccess)
    return done(DMPT_ENOMEM, "pinned allocation failed");
  if (hipMemsetAsync(xo, 0, mat * eb, s) != hipSuccess ||
      (x1o && hipMemsetAsync(x1o, 0, mat * eb, s) != hipSuccess))
    return done(DMPT_EHIP, "clearing the outputs failed");
  if (hipMemcpyAsync(items, it.data(), it.size() * sizeof(TileItem), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return done(DMPT_EHIP, "item upload failed");
  int e1 = 0;
  if (S1) {
    if (launch_maxabs(S1, N, part, s) != hipSuccess ||
        hipMemcpyAsync(hmax, part, kRedBlocks * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return done(DMPT_EHIP, "max|S1| failed");
    double m = 0.0;
    for (int i = 0; i < kRedBlocks; ++i) m = std::max(m, hmax[i]);
    e1 = (m > 0.0) ? -ilogb(m) - 4 : 0;
  }
  ProductArgs pa;
  memset(&pa, 0, sizeof(pa));
  pa.s_hi = split ? sh : sm;
  pa.s_lo = sl;
  pa.x = xo;
  pa.items = (const TileItem*)items;
  pa.n_items = (int)it.size();
  pa.state = nullptr;
  pa.ld = ld;
  pa.kdim = np;
  pa.lo_shift = t;
  if (S1) {
    pa.s1_hi[0] = split ? th : tm;
    pa.s1_lo[0] = tl;
    pa.x1[0] = x1o;
    pa.s1_exp[0] = split ? e1 : 0;
  }
  if (launch_from_f64(prec, S, N, np, ld, 0, t, sm, sh, sl, s) != hipSuccess)
    return done(DMPT_EHIP, "split of S failed");
  if (S1 && launch_from_f64(prec, S1, N, np, ld, split ? e1 : 0, t, tm, th, tl, s) != hipSuccess)
    return done(DMPT_EHIP, "split of S1 failed");
  hipError_t le = launch_products(prec, pa, s);
  if (le != hipSuccess) return done(DMPT_EHIP, std::string("products: ") + hipGetErrorString(le));
  if (launch_copy_plain(prec, xo, ld, X, N, s) != hipSuccess)
    return done(DMPT_EHIP, "copy of X failed");
  if (S1 && launch_copy_plain(prec, x1o, ld, X1, N, s) != hipSuccess)
    return done(DMPT_EHIP, "copy of X1 failed");
  if (hipStreamSynchronize(s) != hipSuccess) return done(DMPT_EHIP, "synchronize failed");
  return done(DMPT_OK, "");
}

dmpt_status dmpt_layer_trace(int32_t precision, int64_t N, const double* S, double* part,
                             void* stream) {
  if (precision != DMPT_SPLIT_FP16 && precision != DMPT_SPLIT_BF16)
    return fail(DMPT_ENOTSUP, "the pre-product trace belongs to the split precisions");
  if (N < 1 || !S || !part) return fail(DMPT_EINVAL, "bad arguments");
  const dmpt_precision prec = (dmpt_precision)precision;
  hipStream_t s = (hipStream_t)stream;
  const int tile = product_tile(prec);
  const int64_t np = (N + tile - 1) / tile * tile;
  const int64_t ld = row_stride(np);
  const int t = lo_shift(prec);
  const int nb = (int)((N + 31) / 32);
  DevAlloc mem;
  void *sm = nullptr, *sh = nullptr, *sl = nullptr;
  LayerState* st = nullptr;
  ProblemDesc* desc = nullptr;
  TraceBlock* blocks = nullptr;
  double* dpart = nullptr;
  hipError_t e = hipSuccess;
  auto get = [&](void** p, size_t b) {
    if (e == hipSuccess) e = mem.get(p, b);
  };
  get(&sm, (size_t)np * ld * sizeof(float));
  get(&sh, (size_t)np * np * 2);
  get(&sl, (size_t)np * np * 2);
  get((void**)&st, sizeof(LayerState));
  get((void**)&desc, sizeof(ProblemDesc));
  get((void**)&blocks, (size_t)nb * sizeof(TraceBlock));
  get((void**)&dpart, (size_t)nb * sizeof(double));
  if (e != hipSuccess) {
    mem.release();
    return fail(e == hipErrorOutOfMemory ? DMPT_ENOMEM : DMPT_EHIP, "allocation failed");
  }
  std::vector<TraceBlock> tb(nb);
  for (int b = 0; b < nb; ++b) tb[b] = TraceBlock{0, b};
  ProblemDesc d;
  memset(&d, 0, sizeof(d));
  d.s_hi[0] = sh;
  d.s_lo[0] = sl;
  d.s_master = (float*)sm;
  d.state = st;
  d.ld = ld;
  d.kdim = np;
  d.pdim = np;
  const int32_t n_real = (int32_t)N;
  // a fresh state: D0 open, split buffer 0; only N is set
  if (e == hipSuccess) e = hipMemsetAsync(st, 0, sizeof(LayerState), s);
  if (e == hipSuccess) e = hipMemcpyAsync(&st->n_real, &n_real, sizeof(n_real), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(desc, &d, sizeof(d), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(blocks, tb.data(), tb.size() * sizeof(TraceBlock), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_from_f64(prec, S, N, np, ld, 0, t, sm, sh, sl, s);
  if (e == hipSuccess) e = launch_trace_diag(prec, desc, blocks, nb, dpart, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part, dpart, (size_t)nb * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipStreamSynchronize(s);
  mem.release();
  return e == hipSuccess ? DMPT_OK : fail(DMPT_EHIP, hipGetErrorString(e));
}

dmpt_status dmpt_contract(const double* const* A, int32_t na, const double* const* B, int32_t nb,
                          int64_t N, double* out, void* stream) {
  if (!A || !B || !out || na < 1 || nb < 1 || na > 64 || nb > 64 || N < 1)
    return fail(DMPT_EINVAL, "bad arguments");
  for (int i = 0; i < na; ++i)
    if (!A[i] || (uintptr_t)A[i] % 16) return fail(DMPT_EINVAL, "A[a] NULL or not 16-byte aligned");
  for (int i = 0; i < nb; ++i)
    if (!B[i] || (uintptr_t)B[i] % 16) return fail(DMPT_EINVAL, "B[b] NULL or not 16-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  double *part = nullptr, *dev = nullptr;
  const int np = na * nb;
  if (hipMalloc((void**)&part, (size_t)np * kRedBlocks * sizeof(double)) != hipSuccess)
    return fail(DMPT_ENOMEM, "allocation failed");
  if (hipMalloc((void**)&dev, (size_t)np * sizeof(double)) != hipSuccess) {
    (void)hipFree(part);
    return fail(DMPT_ENOMEM, "allocation failed");
  }
  hipError_t e = hipSuccess;
  for (int a = 0; a < na && e == hipSuccess; ++a)
    for (int b = 0; b < nb && e == hipSuccess; ++b)
      e = launch_contract(A[a], B[b], N, part + (size_t)(a * nb + b) * kRedBlocks,
                          dev + a * nb + b, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dev, (size_t)np * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  (void)hipFree(dev);
  return e == hipSuccess ? DMPT_OK : fail(DMPT_EHIP, hipGetErrorString(e));
}

// ------------------------------------------------ contraction without allocation
// Device scratch of dmpt_contract_noalloc: kNoAllocPairs blocks of kRedBlocks
// FP64 partials, then one FP64 result per pair (512.5 KiB).  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// the name is only a host-side stand-in: kernels and copies get the device
// address that hipGetSymbolAddress returns for the current device.
constexpr int kNoAllocPairs = 64;
static __device__ __align__(256) double scratch[(size_t)kNoAllocPairs * kRedBlocks + kNoAllocPairs];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of the scratch array on the current device, looked up once
// per device (with that device current) and kept.
dmpt_status scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DMPT_EHIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(DMPT_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(DMPT_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    if (!p) return fail(DMPT_EHIP, "scratch address: NULL");
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return DMPT_OK;
}

}  // namespace

dmpt_status dmpt_contract_noalloc(const double* const* A, int32_t na, const double* const* B,
                                  int32_t nb, int64_t N, double* out, void* stream) {
  if (!A || !B || !out || na < 1 || nb < 1 || N < 1)
    return fail(DMPT_EINVAL, "bad arguments");
  if ((int64_t)na * nb > kNoAllocPairs)
    return fail(DMPT_EINVAL, "contract_noalloc: na * nb = " + std::to_string((int64_t)na * nb) +
                                 " exceeds the scratch limit of " + std::to_string(kNoAllocPairs) +
                                 " pairs");
  for (int i = 0; i < na; ++i)
    if (!A[i] || (uintptr_t)A[i] % 16) return fail(DMPT_EINVAL, "A[a] NULL or not 16-byte aligned");
  for (int i = 0; i < nb; ++i)
    if (!B[i] || (uintptr_t)B[i] % 16) return fail(DMPT_EINVAL, "B[b] NULL or not 16-byte aligned");
  double* base = nullptr;
  const dmpt_status st = scratch_address(&base);
  if (st != DMPT_OK) return st;
  // every block writes its partial and the final kernel its result, so
  // nothing in the scratch needs clearing
  double* part = base;
  double* dev = base + (size_t)kNoAllocPairs * kRedBlocks;
  hipStream_t s = (hipStream_t)stream;
  const int np = na * nb;
  hipError_t e = hipSuccess;
  for (int a = 0; a < na && e == hipSuccess; ++a)
    for (int b = 0; b < nb && e == hipSuccess; ++b)
      e = launch_contract(A[a], B[b], N, part + (size_t)(a * nb + b) * kRedBlocks,
                          dev + a * nb + b, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dev, (size_t)np * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DMPT_OK : fail(DMPT_EHIP, hipGetErrorString(e));
}

dmpt_status dmpt_gershgorin(const double* H, int64_t N, double* eps, void* stream) {
  if (!H || !eps || N < 1) return fail(DMPT_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  double *part = nullptr, *dev = nullptr;
  if (hipMalloc((void**)&part, 3 * 512 * sizeof(double)) != hipSuccess)
    return fail(DMPT_ENOMEM, "allocation failed");
  if (hipMalloc((void**)&dev, 2 * sizeof(double)) != hipSuccess) {
    (void)hipFree(part);
    return fail(DMPT_ENOMEM, "allocation failed");
  }
  hipError_t e = launch_gershgorin(H, N, part, nullptr, dev, s);
  if (e == hipSuccess) e = hipMemcpyAsync(eps, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  (void)hipFree(dev);
  return e == hipSuccess ? DMPT_OK : fail(DMPT_EHIP, hipGetErrorString(e));
}

dmpt_status dmpt_plan_rounds(const int64_t* cost, int32_t n, int32_t grid, int64_t cap,
                             int32_t* order, int64_t* n_order) {
  if (!cost || !order || !n_order || n < 0 || grid < 1 || cap < n)
    return fail(DMPT_EINVAL, "plan_rounds: bad arguments");
  std::vector<int64_t> c(cost, cost + n);
  for (int64_t x : c)
    if (x < 1) return fail(DMPT_EINVAL, "plan_rounds: costs must be >= 1");
  const std::vector<int32_t> plan = balanced_rounds(c, grid, (size_t)cap);
  std::copy(plan.begin(), plan.end(), order);
  *n_order = (int64_t)plan.size();
  return DMPT_OK;
}

dmpt_status dmpt_plan_layer(int32_t T, int32_t k, int32_t k_max, int32_t grid, int64_t* n_positions,
                            int64_t* capacity) {
  if (T < 1 || k < 1 || k_max < k || k_max > kMaxK || grid < 1 || !n_positions || !capacity)
    return fail(DMPT_EINVAL, "plan_layer: bad arguments");
  *n_positions = fused_positions(T, k, grid);
  *capacity = fused_slot_capacity(T, k_max);
  return DMPT_OK;
}

dmpt_status dmpt_probe_mfma(int32_t precision, double* tflops, double* clock_ghz, void* stream) {
  if (precision < DMPT_FP64 || precision > DMPT_SPLIT_FP16)
    return fail(DMPT_EINVAL, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  const int blocks = device_cu_count(), iters = 20000;
  int dev = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      wall_khz <= 0)
    return fail(DMPT_EHIP, "wall-clock rate unavailable");
  float* out = nullptr;
  int64_t* ticks = nullptr;
  if (hipMalloc((void**)&out, (size_t)blocks * 4 * kWave * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&ticks, 2 * sizeof(int64_t)) != hipSuccess) {
    (void)hipFree(out);
    return fail(DMPT_ENOMEM, "allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one launch to settle the clock, then the timed one
  float ms = 0.0f;
  int64_t t[2] = {0, 0};
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_mfma_rate((dmpt_precision)precision, blocks, iters, out, ticks, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e == hipSuccess) e = hipMemcpy(t, ticks, sizeof(t), hipMemcpyDeviceToHost);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  (void)hipFree(ticks);
  if (e != hipSuccess) return fail(DMPT_EHIP, hipGetErrorString(e));
  const double flops = (double)blocks * 4 * iters * 48 * mfma_probe_flops((dmpt_precision)precision);
  if (tflops) *tflops = ms > 0.0f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  if (clock_ghz) *clock_ghz = t[1] > 0 ? (double)t[0] / ((double)t[1] / (wall_khz * 1e3)) / 1e9 : 0.0;
  return DMPT_OK;
}

dmpt_status dmpt_selftest_mfma(int32_t* detail, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int32_t* dev = nullptr;
  int32_t host[kWave];
  if (hipMalloc((void**)&dev, kWave * sizeof(int32_t)) != hipSuccess)
    return fail(DMPT_ENOMEM, "allocation failed");
  hipError_t e = launch_selftest_mfma(dev, s);
  if (e == hipSuccess) e = hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dev);
  if (e != hipSuccess) return fail(DMPT_EHIP, hipGetErrorString(e));
  int32_t bad = 0;
  for (int i = 0; i < kWave; ++i) bad |= host[i];
  if (detail) *detail = bad;
  return bad ? fail(DMPT_ENOTSUP, "MFMA lane layout differs from the kernels' assumption")
             : DMPT_OK;
}

}  // extern "C"
