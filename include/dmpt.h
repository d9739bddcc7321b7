/*
 * dmpt.h -- C ABI of the MI355X (gfx950) DNN-SP2-PT library: the zeroth-order
 * density matrix P0 and its first-order responses P1_k of a symmetric
 * Hamiltonian, computed as a deep layered network of SP2 steps.
 *
 * Method (arXiv:2203.09621):
 *   normalisation layer (Sec. III.A, Algorithm 1)
 *       S0 = (eps_N I - H0)/(eps_N - eps_1),  S1_k = -H1_k/(eps_N - eps_1),
 *       eps_1, eps_N Gershgorin bounds of H0 (Sec. II.B);
 *   deep layer n (Eqs. S_n detailed and dB, first order)
 *       X = S^2,  X1_k = S S1_k + S1_k S,
 *       S <- sigma X + (1 - sigma) S,  S1_k <- sigma X1_k + (1 - sigma) S1_k,
 *       sigma = +-1 from an FP64 trace test against Nocc (Algorithm 1);
 *   stopping: the D0 test of Algorithm 2 and the parameter-free D1 test of
 *       Eq. (ConvCrit) / Algorithm 3 with C_pt = 9.
 *   The limits are P0 = theta(mu I - H0) (Eq. theta) and P1_k, the Gateaux
 *   derivative of P along H1_k (Sec. IV).
 *
 * Conventions for every entry point:
 *   - Matrices are dense, symmetric, N x N, FP64, row-major with leading
 *     dimension N (symmetry makes row/column major identical).  All matrix
 *     pointers are DEVICE pointers owned by the caller.  Arrays of matrix
 *     pointers (H1, P1) are HOST arrays of device pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     is enqueued on it; the call returns after the results are written and
 *     the statistics are readable (one synchronisation at the end).
 *   - No exception crosses the ABI.  A non-OK status leaves the outputs
 *     undefined, except ENOCONV from a capped iteration: the outputs then
 *     hold its last layer (or iterate), as each call states.
 *     dmpt_last_error() gives a human-readable reason.
 *   - One context per stream; a context is not thread-safe, but distinct
 *     contexts may be used from different threads at the same time.
 *   - The library owns its workspace (allocated in dmpt_init, released by
 *     dmpt_destroy); H0 may be freed after dmpt_init returns.
 */
#ifndef DMPT_H
#define DMPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DMPT_OK = 0,
  DMPT_EINVAL = -1,      /* bad argument: sizes, Nocc not in (0, N), k out of range, NULL */
  DMPT_ENOMEM = -2,      /* device allocation failed */
  DMPT_EHIP = -3,        /* a HIP runtime call failed */
  DMPT_ENOCONV = -4,     /* layer cap reached before every response met its D1 test */
  DMPT_ENONFINITE = -5,  /* a trace or norm became NaN/Inf, or a split operand overflowed */
  DMPT_EASYM = -6,       /* symmetry check enabled and H0 or an H1 is not exactly symmetric */
  DMPT_ENOTSUP = -7      /* precision mode not built / not supported on this device */
} dmpt_status;

/* Arithmetic of the layer products.  Traces, sigma, stopping tests, the
 * Gershgorin bounds and the outputs are FP64 in every mode. */
typedef enum {
  DMPT_FP64 = 0,        /* FP64 MFMA products, FP64 layer state (the plain FP64 GPU form) */
  DMPT_FP32 = 1,        /* FP32 MFMA products, FP32 layer state */
  DMPT_SPLIT_BF16 = 2,  /* X ~ hi*hi + hi*lo + lo*hi with BF16 hi/lo parts, FP32 accumulate;
                           16 significant bits (split FP16: 22), so the noise-floor D0 test
                           fires earlier: P1 errors near 1e-3 on small problems with a narrow
                           relative gap (up to 2e-3 seen at N = 16) */
  DMPT_SPLIT_FP16 = 3   /* same with FP16 hi/lo parts; lo and S1 carry power-of-two scales */
} dmpt_precision;

#define DMPT_MAX_K 8          /* most perturbations per context */
#define DMPT_MAX_KB 3         /* most perturbations per problem of a batch */
#define DMPT_MAX_LAYERS 256   /* hard cap on the layer count */

typedef struct {
  int32_t precision;       /* dmpt_precision; default DMPT_SPLIT_FP16 */
  int32_t max_layers;      /* default 100, at most DMPT_MAX_LAYERS */
  int32_t check_symmetry;  /* nonzero: dmpt_init / dmpt_response verify exact symmetry (EASYM) */
  int32_t poll_every;      /* host checks the device stop flag every this many layers (0 = auto) */
  int32_t timing;          /* nonzero: time every layer-product launch with hipEvents on the
                              context's stream (dmpt_stats.product_ms / product_launches) */
  int32_t ckpt_every;      /* > 0: dmpt_response keeps (S, S1) every this many layers so that
                              dmpt_adjoint can run; 0 (default): no adjoint workspace */
  int32_t graph;           /* batched solves: nonzero (default) captures the whole response in
                              one HIP graph on first use and replays it */
  int32_t tile_threshold;  /* batched solves: < 0 (default) times the candidate thresholds at
                              init and keeps the fastest; >= 0 fixes it: problems whose size
                              padded to 256 is at most this use 128-row tiles, the others
                              256-row tiles */
} dmpt_options;

typedef struct {
  int32_t layers;                  /* layers run (index of the last layer) */
  int32_t d0_layer;                /* layer at which the D0 test fired (0 = never) */
  int32_t d1_layer[DMPT_MAX_K];    /* layer at which each D1 test fired (0 = never) */
  int32_t k;                       /* number of responses */
  int32_t converged;               /* 1 if every D1 test fired */
  int8_t sigma[DMPT_MAX_LAYERS];   /* sigma_n of layers 1..layers (+1: x^2, -1: 2x - x^2) */
  double eps1, epsN;               /* Gershgorin bounds of H0 */
  double n_s;                      /* tracked occupation N_S of the returned S0 */
  double idem0;                    /* ||P0 - P0^2||_F at the D0 layer (layer arithmetic) */
  double idem1[DMPT_MAX_K];        /* ||P1 - (P0 P1 + P1 P0)||_F at the D1 layer (layer arithmetic) */
  double trace_p0;                 /* Tr P0 (FP64 over the returned matrix) */
  double trace_p1[DMPT_MAX_K];     /* Tr P1_k (FP64 over the returned matrix) */
  double ms;                       /* device time of dmpt_response (hipEvents) */
  double product_ms;               /* summed duration of the layer-product launches (timing on) */
  int32_t product_launches;        /* layer-product launches timed */
  int32_t x_layers;                /* layers that formed X = S^2 (1..d0_layer) */
} dmpt_stats;

typedef struct dmpt_ctx dmpt_ctx;

/* Fill `opt` with the defaults. */
void dmpt_default_options(dmpt_options* opt);

/* Set up a context for H0 (device, N x N FP64, symmetric) with Nocc occupied
 * states.  Computes the Gershgorin bounds and the normalised S0 (Algorithm 1
 * initial transform) into library-owned workspace sized for up to k_max
 * responses.  Errors: EINVAL (N < 1, Nocc not in (0, N), k_max not in
 * [1, DMPT_MAX_K], NULL), ENOMEM, EHIP, ENOTSUP, EASYM, ENONFINITE. */
dmpt_status dmpt_init(dmpt_ctx** ctx, const double* H0, int64_t N, int64_t Nocc, int32_t k_max,
                      const dmpt_options* opt /* NULL = defaults */, void* stream);

/* Replace the Hamiltonian of a context (same N, Nocc, precision): recompute
 * the Gershgorin bounds and the normalised S0 into the existing workspace.
 * Allocates nothing.  Errors: EINVAL, EHIP, EASYM, ENONFINITE. */
dmpt_status dmpt_set_hamiltonian(dmpt_ctx* ctx, const double* H0);

/* Run Algorithms 1-3 for k perturbations H1[0..k-1] (host array of device
 * pointers).  Writes P0 (device N x N FP64, may be NULL) and P1[j] (host
 * array of k device pointers, N x N FP64).  The S0 chain is shared; each
 * response has its own D1 test and is frozen once it passes.  Returns
 * ENOCONV when the layer cap is reached first (outputs then hold the last
 * layer).  Every H1 is read before any output is written, and the context
 * holds its own copy of H0, so P0 and P1[j] may overwrite the H0 given to
 * dmpt_init and the H1 matrices.  `st` may be NULL. */
dmpt_status dmpt_response(dmpt_ctx* ctx, const double* const* H1, int32_t k, double* P0,
                          double* const* P1, dmpt_stats* st);

/* Second-order response (Sec. III, Eq. S_n detailed with k = 2): for
 * H(lambda) = H0 + lambda H1 + lambda^2 H2, returns P0, P1 = D^(1) and
 * P2 = D^(2), the lambda^2 coefficient of the density matrix.  The chain
 * S2_n = sigma_n (S S2 + S1 S1 + S2 S) + (1 - sigma_n) S2, S2_0 = -H2/(eps_N -
 * eps_1), runs in the second response slot of the context, so the context needs
 * k_max >= 2.  H2 may be NULL (no second-order term in H).  The paper gives
 * stopping tests for first order only; S2 takes Algorithm 3's test on
 * ||S2 - X2||_F from two layers after the D1 layer on, and P2 is S2 of the
 * layer before that test fired.  In `st`, index 1 of d1_layer, idem1 and
 * trace_p1 refers to P2.  P0 may be NULL.  Errors as dmpt_response (with
 * ENOCONV, P0, P1 and P2 hold the last layer); the adjoint does not cover
 * this form. */
dmpt_status dmpt_response2(dmpt_ctx* ctx, const double* H1, const double* H2, double* P0,
                           double* P1, double* P2, dmpt_stats* st);

/* Induced field of a self-consistent (coupled-perturbed) response: given the
 * current first-order density matrix P1 (device FP64 N x N), write G = H1_ind[P1]
 * (device FP64 N x N, symmetric) with work enqueued on `stream`, or finish it
 * before returning.  The physics builder stays with the caller. */
typedef void (*dmpt_field_fn)(void* user, const double* P1, double* G, void* stream);

/* Self-consistent first-order response (the coupled-perturbed loop of
 * Sec. V.B): P1 = DP[H1 + G[P1]] by the fixed-point iteration
 *   H_eff <- (1 - mix) H_eff + mix (H1 + field(P1)),   P1 <- response(H_eff),
 * from H_eff = H1, each response by Algorithms 1-3 in the context's precision.
 * Stops when ||P1_new - P1_old||_F / ||P1_new||_F < tol.  G is caller-provided
 * workspace (device FP64 N x N) that `field` fills; P0 may be NULL; iters and
 * change (may be NULL) receive the field evaluations and the last relative
 * change.  Allocates two N x N FP64 buffers for the duration of the call.
 * Errors: as dmpt_response, ENOCONV when max_iter field evaluations do not
 * reach tol, ENONFINITE on divergence.  The adjoint does not cover it. */
dmpt_status dmpt_cpscf(dmpt_ctx* ctx, const double* H1, dmpt_field_fn field, void* user,
                       double mix, double tol, int32_t max_iter, double* P0, double* P1,
                       double* G, int32_t* iters, double* change, dmpt_stats* st);

/* Reverse mode of the layer recursion for L = Tr(P0 W0) + sum_j Tr(P1_j W_j)
 * (the adjoint of Algorithms 1-3; P0 and P1_j are functions of H0 and H1_j,
 * Sec. IV), applied to the most recent successful dmpt_response of this
 * context (same k, k <= 3; the context needs ckpt_every > 0).  W[j] (host
 * array of device FP64 N x N) is the upstream gradient dL/dP1_j and W0 (device
 * FP64 N x N, may be NULL) dL/dP0; both are symmetrised.  Writes the
 * symmetric gradients dH0 = dL/dH0 and dH1[j] = dL/dH1_j (device FP64 N x N,
 * with dL = <G, dH> for symmetric dH; W0 reaches dH0 only).  The forward is
 * recomputed from the checkpoints segment by segment with the recorded sigma
 * sequence, scales and stop layers (no decision is taken again); the
 * products of the reverse layers run in FP32 MFMA (FP64 for an FP64
 * context).  The Gershgorin bounds are treated as constants.  `st` (may be
 * NULL) receives the forward's layer counts, the time of the whole adjoint
 * and, with timing on, product_ms / product_launches of the reverse layers'
 * product launches.  Errors: EINVAL (no converged response since the last
 * dmpt_init / dmpt_set_hamiltonian, k mismatch, NULL), EHIP. */
dmpt_status dmpt_adjoint(dmpt_ctx* ctx, const double* const* W, int32_t k, const double* W0,
                         double* dH0, double* const* dH1, dmpt_stats* st);

/* Forward and reverse in one call: dmpt_response for H1[0..k-1] (P0 may be
 * NULL, P1 as in dmpt_response), then dmpt_adjoint with W, W0 (may be NULL)
 * into dH0, dH1.  The context needs ckpt_every > 0 and k <= 3.  `st` receives
 * the forward's statistics with ms, product_ms and product_launches summed
 * over both passes.  Errors: as dmpt_response and dmpt_adjoint. */
dmpt_status dmpt_response_adjoint(dmpt_ctx* ctx, const double* const* H1, int32_t k,
                                  const double* const* W, const double* W0, double* P0,
                                  double* const* P1, double* dH0, double* const* dH1,
                                  dmpt_stats* st);

/* Release the context and its workspace.  NULL is allowed. */
void dmpt_destroy(dmpt_ctx* ctx);

/* ---- batched solves: many independent problems of different sizes ----
 * Algorithms 1-3 for `count` problems at once.  Problem p has N[p] orbitals,
 * Nocc[p] occupied states and k[p] in [1, DMPT_MAX_KB] perturbations.  All
 * problems advance layer by layer together; each keeps its own sigma
 * sequence and stopping tests and stops on its own.  Split precisions only
 * (DMPT_SPLIT_BF16 / DMPT_SPLIT_FP16).  The tile size of each problem's
 * products (256 or 128 rows) is chosen at init by timing candidate size
 * thresholds on this batch, unless options.tile_threshold fixes it.  With
 * options.graph (default) the whole response
 * (normalisation, every layer up to max_layers, outputs) is one HIP graph,
 * captured on the first dmpt_batch_response and replayed afterwards. */
typedef struct dmpt_batch dmpt_batch;

typedef struct {
  int32_t layers;                  /* layers run by this problem */
  int32_t d0_layer;
  int32_t converged;
  int32_t k;
  int32_t d1_layer[DMPT_MAX_KB];
  int32_t pad;
  double idem0;                    /* ||P0 - P0^2||_F at the D0 layer */
  double idem1[DMPT_MAX_KB];       /* first-order idempotency residual at the D1 layer */
} dmpt_problem_stats;

/* Allocate the workspace of a batch and tune its tiles.  N, Nocc, k: host
 * arrays of `count` entries.  Errors: EINVAL, ENOMEM, EHIP, ENOTSUP. */
dmpt_status dmpt_batch_init(dmpt_batch** batch, int32_t count, const int64_t* N,
                            const int64_t* Nocc, const int32_t* k,
                            const dmpt_options* opt /* NULL = defaults */, void* stream);

/* Solve every problem.  H0[p] (count entries) and H1[i] (sum of k entries,
 * problem-major) are host arrays of device FP64 pointers; P0[p] (may be NULL
 * as a whole or per entry) and P1[i] receive the results (device FP64, N x N
 * of their problem).  st (count entries, may be NULL) receives per-problem
 * statistics, ms (may be NULL) the device time.  Returns ENOCONV if some
 * problem hit the layer cap (every output then holds its problem's last
 * layer, and st tells which problems converged), ENONFINITE on a
 * non-finite value. */
dmpt_status dmpt_batch_response(dmpt_batch* batch, const double* const* H0,
                                const double* const* H1, double* const* P0, double* const* P1,
                                dmpt_problem_stats* st, double* ms);

/* Tile classes the autotuner chose (or options.tile_threshold fixed):
 * problems with padded size <= *threshold use 128-row tiles; number of item
 * positions of each launch (a 128-row item holds two tiles that share a row
 * or a column band, or one). */
dmpt_status dmpt_batch_info(const dmpt_batch* batch, int32_t* threshold, int32_t* n_items_256,
                            int32_t* n_items_128);

/* Release a batch.  NULL is allowed. */
void dmpt_batch_destroy(dmpt_batch* batch);

/* Observables of the response (the polarisability-type contractions of
 * Sec. V.B): out[a * nb + b] = Tr(A[a] B[b]) for symmetric B[b] (every H1 and
 * P1 of this library is), evaluated as sum_ij A_ij B_ij in FP64 with a
 * fixed-order reduction.  A, B: host arrays of na (nb) device pointers
 * (16-byte aligned) to N x N FP64 matrices; out: host array of na * nb
 * doubles.  With A = H1_a
 * and B = P1_b this is Pi_ab = Tr(H1_a P1_b), whose diagonal mean is the
 * isotropic value.  Errors: EINVAL (NULL or misaligned pointer, na or nb
 * outside [1, 64]), ENOMEM, EHIP. */
dmpt_status dmpt_contract(const double* const* A, int32_t na, const double* const* B, int32_t nb,
                          int64_t N, double* out, void* stream);

/* dmpt_contract without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and reduction order as
 * dmpt_contract (the results are bitwise the same), with its partial sums in a
 * fixed device array of the library (512.5 KiB per GPU, held until the process
 * ends) instead of per-call buffers.  At most 64 pairs: na * nb > 64 returns
 * EINVAL.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (several streams or threads at once) race and give undefined
 * results.  Errors: EINVAL (NULL or misaligned pointer, na or nb < 1, na * nb
 * > 64), EHIP. */
dmpt_status dmpt_contract_noalloc(const double* const* A, int32_t na, const double* const* B,
                                  int32_t nb, int64_t N, double* out, void* stream);

/* ---- non-orthogonal bases (Sec. II.A) ----
 * Inverse factor of a symmetric positive-definite overlap matrix O (device
 * FP64 N x N): Z with Z^T O Z = I by the recursion X_n = Z_n^T O Z_n,
 * Z_{n+1} = Z_n (1.875 I - 1.25 X_n + 0.375 X_n^2) from Z_0 = c I, c^2 = 1 over
 * the Gershgorin bound of O.  Every iterate is a polynomial in O, so Z is the
 * symmetric factor O^{-1/2}.  Products run on MFMA in `precision` (DMPT_FP64
 * or DMPT_FP32).  Stops when ||Z O Z - I||_F < tol (or after max_iter updates);
 * iters and err (may be NULL) receive the updates done and the last residual.
 * Writes Z (device FP64 N x N).  Errors: EINVAL, ENOTSUP (other precisions),
 * ENOMEM, EHIP, ENONFINITE (O not positive definite: divergence), ENOCONV
 * (tol not reached in max_iter updates; Z then holds the last iterate and
 * err its residual). */
dmpt_status dmpt_inverse_factor(int32_t precision, const double* O, int64_t N, double* Z,
                                int32_t max_iter, double tol, int32_t* iters, double* err,
                                void* stream);

/* out = Z A Z for symmetric Z and A (device FP64 N x N; out may not alias):
 * the orthogonalised H_perp = Z^T H Z of a symmetric Z and, back, D = Z D_perp
 * Z^T.  Products on MFMA in `precision` (DMPT_FP64 or DMPT_FP32).  Errors:
 * EINVAL, ENOTSUP, ENOMEM, EHIP. */
dmpt_status dmpt_congruence(int32_t precision, int64_t N, const double* Z, const double* A,
                            double* out, void* stream);

/* Short name of a status code (static storage). */
const char* dmpt_status_str(dmpt_status s);

/* Reason for the most recent non-OK status on the calling thread. */
const char* dmpt_last_error(void);

/* ---- kernel-level entry points (for parity tests of the layer products) ----
 * One activation of a deep layer without any decision: for symmetric S and S1
 * (device, N x N FP64) computes X = S^2 and X1 = S S1 + S1 S (device, N x N
 * FP64 out; X1 may be NULL when S1 is NULL) with the same split, tiling and
 * MFMA code the layers use (Eqs. S0 tensor core and S0S1 tensor core, in the
 * chosen precision).  The S1 split scale is chosen from max|S1| as in a
 * layer.  Errors: EINVAL, ENOMEM, EHIP, ENOTSUP. */
dmpt_status dmpt_layer_products(int32_t precision, int64_t N, const double* S, const double* S1,
                                double* X, double* X1, void* stream);

/* The trace the split precisions take before the layer products (Algorithm
 * 1's N_X = Tr X with X = S^2): part[b] (device, ceil(N/32) FP64 entries)
 * receives the FP64 sum of X_ii over rows 32 b .. 32 b + 31, each X_ii formed
 * from the 32 x 32 diagonal fragment alone with the operand chunks, k order
 * and MFMA sequence of dmpt_layer_products in the same precision, so that
 * every X_ii equals that product's diagonal bitwise.  S: device N x N FP64,
 * split as a layer splits it.  Errors: ENOTSUP (not a split precision),
 * EINVAL, ENOMEM, EHIP. */
dmpt_status dmpt_layer_trace(int32_t precision, int64_t N, const double* S, double* part,
                             void* stream);

/* Gershgorin bounds (Sec. II.B) of a device N x N FP64 matrix into host eps[2]. */
dmpt_status dmpt_gershgorin(const double* H, int64_t N, double* eps /* host, 2 */, void* stream);

/* Device check of the MFMA lane layouts the kernels assume (f16 32x32x16,
 * bf16 32x32x16, f32 16x16x4, f64 16x16x4).  Returns DMPT_OK when every
 * layout matches; `detail` (host, may be NULL) receives a bitmask of
 * mismatching instructions. */
dmpt_status dmpt_selftest_mfma(int32_t* detail, void* stream);

/* Sustained rate of the MFMA instruction a precision's product kernels use
 * (32x32x16 FP16 for DMPT_SPLIT_FP16, BF16 for DMPT_SPLIT_BF16, 16x16x4 FP32
 * for DMPT_FP32, FP64 for DMPT_FP64): four waves on every CU issue
 * independent MFMAs on pseudo-random operands, without memory traffic, for
 * tens of milliseconds (after one settling launch).  tflops (host, may be
 * NULL) receives the rate at 2 flops per multiply-add, clock_ghz (host, may
 * be NULL) the shader clock workgroup 0 saw.  Under such a load the chip
 * lowers its clock to stay within its power limit, so this is the ceiling the
 * product kernels can approach on the device, below the data-sheet peak.
 * Errors: EINVAL (unknown precision), ENOMEM, EHIP. */
dmpt_status dmpt_probe_mfma(int32_t precision, double* tflops, double* clock_ghz, void* stream);

/* The dealing plan of the library's persistent product launches, on the host
 * (no device involved).  Items of costs cost[0..n-1] keep their list order
 * and are dealt round by round to `grid` workgroup slots (position q runs on
 * slot q % grid) against the target max(ceil(total / grid), largest cost): a
 * slot the next item would take past the target gets a placeholder (-1,
 * skipped at once) and the item waits for the next slot; after a round that
 * placed nothing the target grows by one.  order (host, capacity `cap`
 * entries) receives, per position, the item index or -1, and *n_order the
 * number of positions (no trailing placeholders).  When n <= grid, or the plan
 * would need more than cap positions, the plan is the plain order 0 .. n-1.
 * Errors: EINVAL (NULL pointers, n < 0, grid < 1, cap < n, a cost < 1). */
dmpt_status dmpt_plan_rounds(const int64_t* cost, int32_t n, int32_t grid, int64_t cap,
                             int32_t* order, int64_t* n_order);

/* Size of the fused layer launch of a single-problem context, on the host (no
 * device involved): *n_positions receives the item positions (tiles plus the
 * placeholders of the balanced rounds of dmpt_plan_rounds) of the fused
 * split-precision launch for k responses over a T x T tile grid dealt to
 * `grid` workgroups, and *capacity the per-item partial-sum slots a context
 * with k_max responses allocates.  dmpt_init and dmpt_response refuse a plan
 * longer than the capacity.  Errors: EINVAL (T < 1, k < 1, k_max < k, k_max >
 * DMPT_MAX_K, grid < 1, NULL). */
dmpt_status dmpt_plan_layer(int32_t T, int32_t k, int32_t k_max, int32_t grid,
                            int64_t* n_positions, int64_t* capacity);

#ifdef __cplusplus
}
#endif
#endif /* DMPT_H */
