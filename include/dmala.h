/*
 * dmala.h -- C ABI of the MI355X (gfx950) DMALA MIMO detector.
 *
 * The library runs the many-chain sampler of Zhou et al., "Near-Optimal MIMO
 * Detection Using Gradient-Based MCMC in Discrete Spaces":
 *   - target: posterior of eq. post with metric f(x) = -||y - Hx||^2 / sigma^2
 *     (eq. f), tempered to f/tau as in Algorithm 2 (eq. aux);
 *   - proposal: the discrete Langevin proposal of eqs. dis_prop..softmax, or its
 *     preconditioned form (the Remark after Algorithm 1, M = (H^T H + gamma I)^-1);
 *   - correction: the MH acceptance of eq. acc_prob, Algorithm 1;
 *   - outputs: the minimum-residual hard decision (text after Algorithm 1), the
 *     IS-based bit LLRs of eq. llr_is (log-sum-exp form, eq. llr_simple), and
 *     symbol marginals from the symbol-level analogue of the IS estimator
 *     (Appendix C), computed from the final sample of every chain (Section IV-A).
 *
 * Conventions (all buffers are caller-owned; nothing here allocates device
 * memory, synchronises the stream or keeps pointers after a call returns):
 *   complex numbers are interleaved (re, im) pairs;
 *   H of instance b is Nr x Nt, column-major: element (i, m) at
 *     H[b*Nt*Nr + m*Nr + i];  y of instance b at y[b*Nr + i];
 *   precision DMALA_FP64 takes double-precision H, y, sigma2; every other
 *     precision takes single precision;
 *   points of M-QAM are indexed a = kI*Q + kQ (Q = sqrt(M)), kI/kQ the
 *     ascending level indices of the real/imaginary part, levels
 *     s*(2k - Q + 1) with s = sqrt(3 / (2 (M - 1))) (unit average energy);
 *   bit labels: per-axis binary-reflected Gray code of the level index, MSB
 *     first, antenna bits ordered [I bits, Q bits]; LLR = log P(b=0)/P(b=1);
 *   random numbers: Philox4x32-10, key (seed mod 2^32, seed >> 32), counter
 *     (block, t, chain, instance); outputs are a pure function of the inputs,
 *     the parameters and the seed.
 * Errors: every entry point returns a dmala_status; dmala_last_error() gives a
 * thread-local message for the last failure on the calling thread.  Argument
 * errors are detected on the host before anything is enqueued.
 */
#ifndef DMALA_H
#define DMALA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dmala_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
  DMALA_OK = 0,
  DMALA_ERR_ARG = -1,         /* invalid argument (shape, NULL input, ...) */
  DMALA_ERR_UNSUPPORTED = -2, /* valid but not supported (non-square or unknown QAM, size limits) */
  DMALA_ERR_NONFINITE = -3,   /* an instance has a non-finite entry in H or y, or sigma^2 is not
                                 positive and finite (Lemma 1 needs sigma^2 > 0): see dmala_outputs.status */
  DMALA_ERR_WORKSPACE = -4,   /* workspace NULL or smaller than dmala_workspace_size() */
  DMALA_ERR_HIP = -5          /* a HIP runtime call failed (message has the HIP error) */
} dmala_status;

/* Arithmetic of the chain update.
 *   FP64: every step in double precision (parity mode).
 *   FP32: the gradient contraction on MFMA with an exact two-term fp16 split of
 *         the proposal matrix and a three-term split of the energy matrix
 *         (chain states are small odd integers, exact in fp16), fp32
 *         accumulation; proposal normalisers and the MH test in fp32.
 *   BF16 / FP16: the proposal gradient from a single bf16 / fp16 MFMA pass;
 *         the energy difference and all normalisers stay fp32-class. */
typedef enum { DMALA_FP64 = 0, DMALA_FP32 = 1, DMALA_BF16 = 2, DMALA_FP16 = 3 } dmala_precision;

/* Proposal: PRECOND = the preconditioned discrete Langevin proposal (the
 * paper's evaluated variant); NAIVE = eq. exp_fac with the plain gradient;
 * LEARNED = per transition and chain, the PRECOND kernel with probability
 * mix_eps and otherwise the learned kernel: the same per-dimension discretised
 * Gaussian over the levels, with its centre and precision set by a small
 * per-antenna network (dmala_mlp_forward) from features of the current state.
 * Each kernel is a full MH step with its own forward and reverse proposal, so
 * pi_a stays invariant (the paper names such data-driven additions as future
 * work, Section V; admissibility follows from eq. acc_prob).  The kernel
 * choice uses the 24-bit uniform from the low bytes of words 4, 5, 6 of the
 * transition's random stream (plain iff u < mix_eps).  Not with DMALA_FP64. */
typedef enum { DMALA_PRECOND = 0, DMALA_NAIVE = 1, DMALA_LEARNED = 2, DMALA_MHGD = 3 } dmala_proposal;
/* DMALA_MHGD is the baseline the paper compares against (Section III-A, the Remark
 * on the visual comparison): the candidate is the continuous preconditioned
 * Langevin step x + (alpha/2) M grad(f/tau)(x) + sqrt(alpha beta) w, w ~ N(0, I),
 * mapped to the nearest lattice point per real dimension, and accepted with
 * min(1, pi_a(x')/pi_a(x)) -- without the mapping's proposal probability, so the
 * chain is biased (Section III-B).  w_n = Phi^-1(u_n) with u_n = (high 24 bits of
 * word n + 1/2) 2^-24; MH uniform and initial state as for the other proposals.
 * For comparisons only; not with the learned-network options. */

/* Bit LLR estimator from the final samples (one per chain):
 *   IS   -- eq. llr_is in the log-sum-exp form of eq. llr_simple (the default);
 *   LIST -- eq. llr_approx_app: APP sums over the distinct samples only, each sample
 *           on the side of its own bit; a side without samples gives +-20;
 *   MC   -- eq. mc on the bit indicators: log(#samples with b = +1 / # with b = -1),
 *           duplicates counted, +-20 when one side is empty (meaningful with tau = 1,
 *           i.e. samples of pi).  LIST and MC are clipped to [-20, 20]. */
typedef enum { DMALA_LLR_IS = 0, DMALA_LLR_LIST = 1, DMALA_LLR_MC = 2 } dmala_llr_mode;

/* The learned proposal's network: 7 features per antenna -> 64 -> 64 -> 4
 * (ReLU), parameters as one float32 array, row-major blocks in this order:
 *   W1[64][7], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]   (4932 floats).
 * Features of antenna m at state x (c = (Q-1)/2, h = Q/2, index units):
 *   (mu_re - c)/h, (mu_im - c)/h, (k_re - c)/h, (k_im - c)/h,
 *   log2(sigma^2 M_mm / (8 s^2)) / 8, log2(sigma^2 / (8 s^2 G_mm)) / 8, log2(Q) / 4
 * with k the level indices of x_m, mu the centre of the PRECOND proposal at x
 * in index units, G = H^H H, M = (G + gamma I)^-1.  Outputs (D_re, D_im,
 * b_re, b_im): the learned proposal of axis p has centre mu_p + D_p and
 * precision kappa * 2^clamp(b_p, -4, 4), kappa the PRECOND precision.
 * In the sampler the network runs in bfloat16 (parameters, inputs, hidden
 * activations rounded to nearest even) with fp32 sums. */
#define DMALA_MLP_PARAMS 4932
/* Floats per exported training row: 7 features, mu_re, mu_im, kappa (natural
 * log units), Q, 0. */
#define DMALA_TRAIN_ROW 12

typedef struct {
  int32_t n_chains;          /* parallel samplers per instance, 1..1024 */
  int32_t n_iters;           /* MH transitions per chain (the paper's T - 1), 0..65535 */
  uint64_t seed;             /* Philox key */
  dmala_precision precision;
  dmala_proposal proposal;
  double tau;                /* temperature of pi_a (eq. aux); <= 0 selects 2 (Section IV-A) */
  double alpha_mult;         /* alpha = alpha_mult * sigma^2;          <= 0 selects 1 */
  double beta_mult;          /* beta  = beta_mult * dmin^2 / sigma^2;  <= 0 selects 1 */
  double gamma_mult;         /* gamma = gamma_mult * sigma^2 / (2 dmin^2); <= 0 selects 1 */
  int32_t tile_config;       /* sampler work layout: 0 = automatic (32 dims: layout 0, 64: 9, 128: 7,
                                256: 8 (NAIVE: 1, 3, 4); LEARNED 64: 5, 128: 6); k >= 1 selects layout k - 1:
                                0: 32 dims, 1 wave / 16 chains, matrices in LDS
                                1: 64 dims, 1 wave / 16 chains, LDS
                                2: 128 dims, 1 wave / 16 chains, LDS
                                3: 128 dims, 2 waves / 16 chains, matrices read from L2
                                4: 256 dims, 4 waves / 16 chains, L2
                                5: 64 dims, 2 waves / 16 chains, LDS   (LEARNED only)
                                6: 128 dims, 4 waves / 16 chains, L2   (LEARNED only)
                                7: layout 3 with the matrices stored as complex planes (half the bytes;
                                   not LEARNED, not FP64)
                                8: layout 4 with complex-plane matrices (not LEARNED, not FP64)
                                9: layout 1 with complex-plane matrices in LDS (not LEARNED, not FP64)
                                (dims = 2 Nt rounded up to a power of two >= 32; a layout that does
                                not match the shape returns DMALA_ERR_UNSUPPORTED) */
  int32_t wg_chain_blocks;   /* 16-chain blocks of one instance per workgroup: 0 = automatic (up to 4),
                                or 1, 2, 4; layouts 0-2 share one LDS copy of the matrices, the two-wave
                                layouts 3 and 5 hold at most 2 blocks (their waves owning the same row
                                tiles read the same matrix fragments together), the four-wave layouts 1 */
  const float* mlp_weights;  /* LEARNED: device float32 [DMALA_MLP_PARAMS]; otherwise ignored.
                                LEARNED excludes layout 2; its defaults are layouts 0, 5, 6, 4 */
  double mix_eps;            /* LEARNED: probability of the PRECOND kernel per transition, in [0, 1] */
  dmala_llr_mode llr_mode;   /* bit LLR estimator (default IS) */
  uint32_t counter_base;     /* instance b of the call draws from the random stream of instance
                                counter_base + b (the counter's instance word); 0 by default.  A batch
                                split over several calls keeps its chains with the offsets of the parts */
} dmala_params;

/* Device output buffers; any pointer may be NULL to skip that output. */
typedef struct {
  int32_t* symbols;          /* [n_inst][Nt] hard decision (point index) */
  float* marginals;          /* [n_inst][Nt][M] symbol posterior estimates */
  float* llrs;               /* [n_inst][Nt][log2 M] bit LLRs */
  float* best_energy;        /* [n_inst] ||y - H x_hat||^2 of the hard decision */
  int8_t* final_state;       /* [n_inst][n_chains][2 Nt] final level indices, dims (Re x_m, Im x_m) interleaved */
  int32_t* accept_count;     /* [n_inst][n_chains] accepted transitions */
  float* marginals_mc;       /* [n_inst][Nt][M] plain Monte Carlo histogram of the final samples */
  uint32_t* trace_accept;    /* [n_inst][n_chains][ceil(n_iters/32)] accept bit of transition t at bit t%32 */
  uint32_t* trace_hash;      /* [n_inst][n_chains][n_iters] state fingerprint after transition t:
                                sum_n (k_n + 1) * ((2n + 1) * 0x9E3779B1) mod 2^32 */
  float* train_rows;         /* [n_inst][n_chains][Nt][DMALA_TRAIN_ROW] network training rows at the final
                                state (PRECOND or LEARNED only); plans index rows as
                                (sum_{j<b} Nt_j) * n_chains + chain * Nt_b + m */
  int32_t* status;           /* [n_inst] input check of each instance, written by the first kernel:
                                DMALA_OK, or DMALA_ERR_NONFINITE when H or y has a non-finite entry or
                                sigma^2 is not positive and finite.  A flagged instance runs no chain:
                                its symbols are -1, marginals, LLRs and best energy NaN, final states,
                                accept counts, traces and training rows 0.  Read it after the stream
                                has run, or let dmala_sync_status() do so. */
  void* stage_events[4];     /* optional hipEvent_t handles recorded on `stream` before the setup,
                                sampler and estimator kernels and after the last one (profiling);
                                NULL entries are skipped */
} dmala_outputs;

/* Bytes of device workspace dmala_detect needs for this shape (0 on invalid
 * arguments; see dmala_last_error()). */
size_t dmala_workspace_size(int32_t n_inst, int32_t nt, int32_t nr, int32_t qam_order,
                            const dmala_params* params);

/* Detect n_inst independent problems of one shape (Algorithm 2 per instance).
 *   H, y, sigma2: device inputs as described above; sigma2[b] > 0 (Lemma 1).
 *     The inputs live on the device, so they are checked there: an instance with a
 *     non-finite entry in H or y, or with sigma2[b] not positive and finite, is
 *     flagged in out->status (see dmala_outputs) and skipped; the call itself still
 *     returns DMALA_OK (it does not wait for the stream).
 *   constellation: NULL, or host array of M complex float points that must
 *     equal the canonical unit-energy QAM (validated; others are unsupported).
 *   Limits: 1 <= nt <= 128, 1 <= nr <= 4096, M in {4, 16, 64, 256}; FP64 needs nt <= 32.
 * Enqueues setup, sampler and estimator kernels on `stream` and returns. */
dmala_status dmala_detect(const void* H, const void* y, const void* sigma2,
                          int32_t n_inst, int32_t nt, int32_t nr, int32_t qam_order,
                          const float* constellation, const dmala_params* params,
                          const dmala_outputs* out, void* workspace, size_t workspace_bytes,
                          dmala_stream_t stream);

/* Wait for `stream`, then read status[0..n_inst) (device, as written through
 * dmala_outputs.status): DMALA_OK if no instance is flagged, otherwise
 * DMALA_ERR_NONFINITE with the number of flagged instances and the first one in
 * dmala_last_error().  Synchronises the stream; allocates nothing. */
dmala_status dmala_sync_status(const int32_t* status, int32_t n_inst, dmala_stream_t stream);

/* One problem with the defaults of Section IV-A (preconditioned proposal, tau = 2,
 * alpha = sigma^2, beta = dmin^2 / sigma^2, gamma = sigma^2 / (2 dmin^2)), fp32-class
 * arithmetic (DMALA_FP32), IS estimators; synchronous: returns when the outputs are
 * written.
 *   H: device complex float [Nt][Nr] (column-major), y: device complex float [Nr];
 *   sigma2: host value; not positive and finite -> DMALA_ERR_NONFINITE before anything
 *     is enqueued (Lemma 1 needs sigma^2 > 0);
 *   constellation: host array of M complex float points, validated against the
 *     canonical unit-energy square QAM (NULL: the canonical one);
 *   symbols: device int32 [Nt] (hard decision), marginals: device float [Nt][M]
 *     (may be NULL);
 *   workspace: device, 256-byte aligned, dmala_detect_one_workspace_size() bytes.
 * Returns DMALA_ERR_NONFINITE (outputs as for a flagged instance) when H or y has a
 * non-finite entry. */
size_t dmala_detect_one_workspace_size(int32_t nt, int32_t nr, int32_t qam_order, int32_t n_chains);
dmala_status dmala_detect_one(const void* H, const void* y, float sigma2, int32_t nt, int32_t nr,
                              const float* constellation, int32_t qam_order, int32_t n_chains,
                              int32_t n_iters, uint64_t seed, int32_t* symbols, float* marginals,
                              void* workspace, size_t workspace_bytes, dmala_stream_t stream);

/* ---- Detection without a caller workspace ----
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels
 * and outputs as dmala_detect, with the workspace taken from a fixed device array
 * of DMALA_STATIC_SCRATCH_BYTES bytes that the library keeps on every GPU it runs
 * on until the process ends (the array's device address is looked up once per
 * device, on the first call with that device current).  Calls no allocating
 * routine.  Returns DMALA_ERR_WORKSPACE, before anything is enqueued, when the
 * call's dmala_workspace_size() exceeds DMALA_STATIC_SCRATCH_BYTES.  The kernels
 * write every scratch byte before reading it, so no clearing is needed between
 * calls.  All calls on one GPU share its array: calls ordered on one stream are
 * safe, calls that overlap on one GPU (different streams or host threads without
 * ordering) race and give undefined results.  The stream must belong to the
 * current device. */
#define DMALA_STATIC_SCRATCH_BYTES (64u << 20)
dmala_status dmala_detect_static(const void* H, const void* y, const void* sigma2,
                                 int32_t n_inst, int32_t nt, int32_t nr, int32_t qam_order,
                                 const float* constellation, const dmala_params* params,
                                 const dmala_outputs* out, dmala_stream_t stream);

/* Evaluate the chain's transition quantities for given state pairs with the
 * same device code as the sampler (tests build exact transition matrices from
 * it).  x_from, x_to: device int8 [n_inst][n_pairs][2 Nt] level indices.
 * out: device double [n_inst][n_pairs][4] = (log q(x_to | x_from),
 * log q(x_from | x_to), f(x_to)/tau - f(x_from)/tau, log acceptance ratio),
 * natural logs, as the sampler computes them.
 * out_dim (optional, NULL to skip): device double [n_inst][n_pairs][2 Nt], the
 * per-dimension terms log q_n(x_to,n | x_from) of the forward proposal (eq.
 * dis_prop_fac1), whose sum is out[.][0].
 * A flagged instance (see dmala_outputs.status) gives NaN.  Workspace as for
 * dmala_detect with n_chains = n_pairs. */
dmala_status dmala_debug_eval(const void* H, const void* y, const void* sigma2,
                              int32_t n_inst, int32_t nt, int32_t nr, int32_t qam_order,
                              const dmala_params* params, const int8_t* x_from, const int8_t* x_to,
                              int32_t n_pairs, double* out, double* out_dim, void* workspace,
                              size_t workspace_bytes, dmala_stream_t stream);

/* ---- Uneven batches: instances of different Nt, Nr, M in one graph launch ----
 * (Section II-A: a base station detects many users' streams of different sizes at
 * once.)  A plan groups the instances of a batch by shape class (Nt, Nr, M) and runs
 * them all as one HIP graph.  Persistent form (the float chains of the plain
 * preconditioned and naive proposals): the work of all classes is split into items
 * (setup: an instance; sampler: an instance and a group of 16-chain blocks;
 * estimator: an instance), the items are grouped by the kernel instantiation that
 * runs them, and each group is one persistent launch whose resident workgroups take
 * items from a device list -- the classes with the largest items first (longest
 * processing time) -- through a global atomic counter; the groups run in stage order
 * on one stream.  A class's results are bit for bit those of dmala_detect over its
 * instances.  Other precisions and proposals (float64, learned, MHGD): per class a
 * setup, a sampler and an estimator kernel, the classes on parallel branches in
 * decreasing order of work.  Executions of one plan must not overlap (they share its
 * tables and counters).  Buffers are packed in instance order:
 *   H of instance b at complex offset sum_{j<b} Nt_j Nr_j (column-major per instance),
 *   y at sum_{j<b} Nr_j, sigma2[b]; symbols at sum Nt_j; marginals and marginals_mc at
 *   sum Nt_j M_j; llrs at sum Nt_j log2 M_j; best_energy[b]; final_state at
 *   sum n_chains 2 Nt_j; accept_count at b * n_chains; status at b; trace_accept and
 *   trace_hash as for dmala_detect with instance b (every instance has the same
 *   n_chains and n_iters).
 * The per-instance random counters use the instance index b, so a plan and a
 * dmala_detect call over the same instances give identical chains.
 * The plan owns small device tables (instance table at creation; work items,
 * per-class arguments and counters when its graph is built; freed by
 * dmala_plan_destroy) and its graph; the graph is rebuilt when execute is called
 * with different buffers (that call synchronises the device first).  Params: as for dmala_detect (tile_config 0 lets each
 * class use its tuned or default layout). */
typedef struct dmala_plan_s* dmala_plan;
typedef struct { int32_t nt, nr, qam_order; } dmala_shape;

/* shapes: host array [n_inst].  On success *plan is set and *workspace_bytes
 * receives the device workspace the plan needs. */
dmala_status dmala_plan_create(dmala_plan* plan, const dmala_shape* shapes, int32_t n_inst,
                               const dmala_params* params, size_t* workspace_bytes);

/* Run every instance of the plan (enqueued on `stream` as one graph launch). */
dmala_status dmala_plan_execute(dmala_plan plan, const void* H, const void* y, const void* sigma2,
                                const dmala_outputs* out, void* workspace, size_t workspace_bytes,
                                dmala_stream_t stream);

/* Time every admissible (layout, workgroup chain blocks) candidate of every
 * class on the given inputs and keep the fastest per class; when cache_path is
 * non-NULL, read earlier results from it first (classes already present are not
 * re-timed) and write the updated table back (JSON).  Synchronises `stream`. */
dmala_status dmala_plan_autotune(dmala_plan plan, const void* H, const void* y, const void* sigma2,
                                 void* workspace, size_t workspace_bytes, const char* cache_path,
                                 dmala_stream_t stream);

/* Number of shape classes; per class: its shape, instance count, chosen layout
 * (tile_config value, >= 1), chain blocks per workgroup and tuned time (ms, 0 if untuned). */
int32_t dmala_plan_num_classes(dmala_plan plan);
dmala_status dmala_plan_class_info(dmala_plan plan, int32_t k, dmala_shape* shape, int32_t* n_inst,
                                   int32_t* tile_config, int32_t* wg_chain_blocks, double* tuned_ms);

/* The plan's current graph: kernel nodes (*n_kernels) and whether it is the persistent
 * form (*persistent, 1 or 0); both -1 before the first execute. */
dmala_status dmala_plan_graph_info(dmala_plan plan, int32_t* n_kernels, int32_t* persistent);

void dmala_plan_destroy(dmala_plan plan);

/* ---- The learned proposal's network ----
 * Forward pass in the sampler's precision (bfloat16 operands, fp32 sums, the
 * same device code): rows = device float32 [n_rows][row_stride] whose first 7
 * entries are the features; out = device float32 [n_rows][4]. */
dmala_status dmala_mlp_forward(const float* weights, const float* rows, int32_t n_rows, int32_t row_stride,
                               float* out, dmala_stream_t stream);

/* Bytes of device workspace dmala_mlp_train_step needs for n_rows rows. */
size_t dmala_mlp_train_workspace_size(int32_t n_rows);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; `step`
 * counts from 1) on the mean over rows of the cross-entropy
 *   -log q_re(t_re) - log q_im(t_im)
 * of the learned proposal (float32, unrounded network) at target levels.
 *   weights, adam_m, adam_v: device float32 [DMALA_MLP_PARAMS], updated in place;
 *   rows: device float32 [n_rows][DMALA_TRAIN_ROW] as exported by the sampler;
 *   targets: device int32 [n_rows][2] level indices (Re, Im) in [0, Q);
 *   loss (optional): device float32 [1], the mean loss before the step;
 *   grad (optional): device float32 [DMALA_MLP_PARAMS], the gradient of that loss.
 * Deterministic (fixed summation order). */
dmala_status dmala_mlp_train_step(float* weights, float* adam_m, float* adam_v, int32_t step, float lr,
                                  const float* rows, const int32_t* targets, int32_t n_rows,
                                  float* loss, float* grad, void* workspace, size_t workspace_bytes,
                                  dmala_stream_t stream);

/* ---- Measurement: the gradient contraction alone ----
 * Runs the chain's G.X stage -- the product of the packed preconditioned matrix with the
 * chains' level vectors on MFMA, one bf16 (DMALA_BF16) or fp16 (DMALA_FP16) pass with fp32
 * accumulation, 8 Nt^2 flops per chain -- n_loops times per chain, with a synthetic update
 * between products (each level whose gradient entry is negative changes sign), to measure
 * the stage's fraction of the MFMA peak apart from the rest of the transition.  Same
 * fragments and lane layout as the sampler; the matrix stays in registers.
 *   params: DMALA_PRECOND with DMALA_BF16 or DMALA_FP16 (others: DMALA_ERR_UNSUPPORTED);
 *   run_setup: 1 runs the setup kernel first (packs the matrices into the workspace); 0
 *     reuses the matrices an earlier call with the same inputs, shape and params left there;
 *   sink: device float [dmala_gx_loop_sink_size(n_inst, nt, n_chains)] per-lane sums of the
 *     last products (keeps the work observable);
 *   workspace: as dmala_workspace_size() for the same shape and params. */
size_t dmala_gx_loop_sink_size(int32_t n_inst, int32_t nt, int32_t n_chains);
dmala_status dmala_gx_loop(const void* H, const void* y, const void* sigma2, int32_t n_inst, int32_t nt,
                           int32_t nr, int32_t qam_order, const dmala_params* params, int32_t n_loops,
                           int32_t run_setup, float* sink, void* workspace, size_t workspace_bytes,
                           dmala_stream_t stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* dmala_last_error(void);

/* Library version string. */
const char* dmala_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DMALA_H */
