/*
 * rwgt.h - C ABI of the MI355X matrix-element reweighting library (librwgt.so).
 *
 * The operation is the parameter-reweighting rule of the paper's teaRex
 * section: for events with weights w sampled under an original parameter card
 * theta, a new card theta' gives
 *
 *     w'_i = (w_i * (1 / |M|^2(p_i; theta))) * |M|^2(p_i; theta'),   1/0 -> 0
 *
 * (the normalise-then-multiply order of the teaRex section, the ratio of its
 * introduction), where |M|^2 is the tree-level squared matrix element summed
 * over helicities and colours and averaged over initial spins and colours
 * (MadtRex section: leading order, helicity-summed).  The per-event evaluation
 * of |M|^2 is the data-parallel hot path the MadtRex section hands to the
 * CUDACPP kernels; here it runs in hand-written HIP kernels on one gfx950 GPU.
 *
 * Conventions shared by every entry point:
 *  - momenta: [nevt][npart][4] doubles (E, px, py, pz) in GeV, particle order
 *    as in the process string, incoming first, DEVICE memory (rwgt_eval and
 *    rwgt_me2 also take host memory, see there);
 *  - weights_in [nevt], weights_out [nsets][nevt], me2_out [nsets][nevt]:
 *    doubles in DEVICE memory (host memory as for momenta);
 *  - param_sets [nsets][npar]: doubles in HOST memory, one row per new card,
 *    columns in the order reported by rwgt_param_layout;
 *  - the caller owns every array; the library never frees caller memory;
 *  - work is enqueued on the context's stream (rwgt_set_stream; default the
 *    null stream) and the call returns after enqueueing: synchronise the
 *    stream before reading outputs;
 *  - return value 0 on success, a negative RWGT_E* code on error, with a
 *    message in rwgt_last_error(ctx); no C++ exception crosses the ABI;
 *  - a context must not be used from two host threads at once; calls on one
 *    context are ordered by its stream.
 */
#ifndef RWGT_H
#define RWGT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rwgt_ctx rwgt_ctx;

enum {
  RWGT_OK = 0,
  RWGT_EINVAL = -1,   /* null pointer, negative size, nsets < 1 */
  RWGT_EPROCESS = -2, /* process string not supported */
  RWGT_ECARD = -3,    /* parameter card unparsable or missing an entry */
  RWGT_EDEVICE = -4,  /* HIP runtime error (launch, copy) */
  RWGT_ENOMEM = -5,   /* device or pinned allocation failed */
  RWGT_EPARAM = -6    /* a card changes a parameter fixed by the momenta (external mass) */
};

enum {
  RWGT_FP64 = 0,        /* every amplitude in double precision */
  RWGT_MIXED_FP16 = 1,  /* float amplitudes, FP16 hi/lo MFMA colour sum, double ratio */
  RWGT_MIXED_BF16 = 2   /* float amplitudes, BF16 hi/mid/lo MFMA colour sum, double ratio */
};

/* Create a context for one process on the current HIP device: the paper's
 * per-process reweighting object (Tensorial event adaption section, Generic
 * and SLHA parameter reweighting: a weight function per process, evaluated
 * under an original SLHA card that each iteration overrides; MadtRex section,
 * Usage: tree-level, helicity-summed amplitudes, precision chosen by fptype).
 *  process:    "e+ e- > mu+ mu-", "u u~ > e+ e- g" or "g g > t t~ g g"
 *              (whitespace-insensitive);
 *  param_card: SLHA text of the ORIGINAL card (blocks SMINPUTS 1 = 1/alpha,
 *              SMINPUTS 3 = alpha_s, RWGTEW 1 = sin^2 theta_W, MASS 6, MASS 23,
 *              DECAY 23); only the entries the process uses are required;
 *  precision:  RWGT_FP64 / RWGT_MIXED_FP16 / RWGT_MIXED_BF16.
 * On success *out owns device buffers until rwgt_destroy; on error *out = NULL.
 * Errors: RWGT_EINVAL, RWGT_EPROCESS, RWGT_ECARD, RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_create(const char *process, const char *param_card, int precision, rwgt_ctx **out);

/* Free the context and its device buffers (after its queued work).  NULL is a
 * no-op.  (The release counterpart of rwgt_create; the paper's objects are
 * scoped C++ values.) */
void rwgt_destroy(rwgt_ctx *ctx);

/* Number of columns of a param_sets row and their names ("SMINPUTS 3", ...):
 * the SLHA entries (block, index) a reweighting iteration may override
 * (Tensorial event adaption section, SLHA parameter reweighting).  names may
 * be NULL; otherwise it receives npar pointers owned by ctx. */
int rwgt_param_layout(const rwgt_ctx *ctx, int32_t *npar, const char **names);

/* The original card's values in layout order (host array of npar doubles). */
int rwgt_original_params(const rwgt_ctx *ctx, double *values);

/* Stream for subsequent calls: a hipStream_t passed as void* (NULL = null
 * stream).  (Device-side ordering of the data-parallel amplitude calls the
 * MadtRex section's Backend details hand to the GPU; the paper has no stream
 * interface of its own.) */
int rwgt_set_stream(rwgt_ctx *ctx, void *stream);

/* Reweight: weights_out[k][i] = (weights_in[i] * (1/|M|^2_orig[i])) * |M|^2_k[i]
 * for the nsets cards in param_sets.  nevt = 0 is a no-op.
 * momenta, weights_in and weights_out may each be memory of the context's
 * device or host memory (told apart with hipPointerGetAttributes): host
 * arrays, and other devices' memory, are copied through a device staging
 * buffer that the context keeps (grown as needed, freed by rwgt_destroy) on
 * the context's stream.  Pinned host memory (hipHostMalloc) keeps the call
 * asynchronous: synchronise the stream before reading a host weights_out or
 * reusing a host input.  With any pageable host array the call waits for the
 * stream before it returns, outputs copied back.  The device path is the same
 * either way, so results are equal bit for bit.
 * Errors: RWGT_EINVAL, RWGT_EPARAM, RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_eval(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *weights_in,
              const double *param_sets, int32_t nsets, double *weights_out);

/* Coupling-factored reweighting: the same result as rwgt_eval (up to
 * rounding), cheaper when there are many cards.  For e+ e- > mu+ mu- and
 * u u~ > e+ e- g every helicity amplitude factorises into a card-independent
 * kinematic part and F = A/s + B/(s - M_Z^2 + i M_Z Gamma_Z), with A and B
 * products of the two fermion lines' photon and Z couplings (B per chirality
 * class of the lines) and s the lepton pair's invariant mass; four probe
 * evaluations per event (Z couplings on one class) give the class weights,
 * then each card costs a few operations per event.  For g g > t t~ g g the
 * cards change alpha_s only and |M|^2 scales as alpha_s^4 (one evaluation).
 * Cost: 4 (or 1) matrix-element evaluations per event instead of 1 + nsets.
 * Errors as rwgt_eval. */
int rwgt_eval_factored(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *weights_in,
                       const double *param_sets, int32_t nsets, double *weights_out);

/* Reweighting with the strong coupling per event.  The original |M|^2 of
 * event i uses alphas_orig[i] (DEVICE, the alpha_s the event was generated
 * with, e.g. the LHE AQCDUP; NULL: the original card's alpha_s run to
 * scales[i]); card k uses its alpha_s (SMINPUTS 3, taken as alpha_s at
 * 91.1876 GeV) run to scales[i] (DEVICE, GeV) at one loop with five flavours:
 * a(mu) = a / (1 + a b0 ln(mu^2/91.1876^2)), b0 = 23/(12 pi).  Every diagram
 * of the supported processes carries the same power p of g_s (p = 0, 1, 4 for
 * e+ e- > mu+ mu-, u u~ > e+ e- g, g g > t t~ g g), so this is the full path
 * times (a_k(mu_i)/a_k)^p (a_0/a_0(i))^p per event; alphas_orig[i] = 0 gives
 * w' = 0.  Errors as rwgt_eval. */
int rwgt_eval_alphas(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *weights_in,
                     const double *alphas_orig, const double *scales, const double *param_sets, int32_t nsets,
                     double *weights_out);

/* |M|^2 itself for each card of param_sets: me2_out[k][i] -- the weight
 * function of parameter reweighting, which is also its normaliser under the
 * original card (MadtRex section, Backend details; Tensorial event adaption
 * section, Generic reweighting).  Same rules as rwgt_eval, host arrays
 * included. */
int rwgt_me2(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *param_sets, int32_t nsets,
             double *me2_out);

/* Cancellation guard of the mixed precisions (RWGT_MIXED_*).  Single-precision
 * rounding of the amplitude terms is amplified where the terms of a colour
 * flow cancel (the MadtRex section's usage notes warn that single precision
 * can lose accuracy through such cancellations).  For each event the mixed
 * kernel measures
 *     kappa = max over cards of  sum_hel sum_t m_t |A_t|^2 / sum_hel sum_c |J_c|^2,
 * A_t the amplitude terms (m_t: the colour flows term t enters), J_c the
 * colour-flow amplitudes; kappa = 1 without cancellation.  Events with kappa
 * above kappa_max are evaluated again, in double precision, within the same
 * rwgt_eval / rwgt_me2 call, and their outputs replaced.  kappa_max <= 0
 * turns the guard off; the default is the library's calibrated value.
 * Applies to rwgt_eval and rwgt_me2 on mixed contexts (the batched,
 * factored, per-event-alpha_s and card-per-event paths run unguarded). */
int rwgt_set_mixed_guard(rwgt_ctx *ctx, double kappa_max);
/* Events re-evaluated in double precision by the last rwgt_eval / rwgt_me2
 * call on ctx (0 if the guard did not run); waits for the stream. */
int rwgt_mixed_guard_count(rwgt_ctx *ctx, int64_t *n_reevaluated);
/* Mixed |M|^2 (me2_out [nsets][nevt], DEVICE, optional) and kappa per event
 * (kappa_out [nevt], DEVICE) without re-evaluation.  Errors: RWGT_EINVAL on a
 * double-precision context or a NULL kappa_out, else as rwgt_me2. */
int rwgt_cancellation(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *param_sets, int32_t nsets,
                      double *me2_out, double *kappa_out);

/* Number of non-finite entries (NaN or +-inf) in the output array of the
 * last rwgt_eval, rwgt_me2, rwgt_eval_factored, rwgt_eval_alphas,
 * rwgt_eval_cards or rwgt_sur_eval call on ctx (weights_out or me2_out,
 * nsets * nevt entries, or nevt); 0 when that call failed
 * or had nevt = 0.  Non-finite momenta or weights give non-finite outputs
 * (nothing is clamped), and a zero original |M|^2 gives w' = 0, which is
 * finite (teaRex section, the normaliser's guard).  The count is taken on the
 * device after the call's kernels, on the context's stream; this call waits
 * for it.  Errors: RWGT_EINVAL (NULL), RWGT_EDEVICE. */
int rwgt_nonfinite(rwgt_ctx *ctx, int64_t *count);

/* Message of the last failed call on ctx (empty string if none).  The
 * paper's library throws runtime errors or prints warnings (Tensorial event
 * adaption section, Generic reweighting); across this C ABI an error is a
 * return code plus this message. */
const char *rwgt_last_error(const rwgt_ctx *ctx);

/* Message of the last failed rwgt_create on this thread (no context exists then). */
const char *rwgt_create_error(void);

/* Process constants: particles, helicity combinations kept, colour flows, diagrams. */
int rwgt_process_info(const rwgt_ctx *ctx, int32_t *npart, int32_t *nhel_kept, int32_t *ncol, int32_t *ndiag);

/* Floating-point operations of one |M|^2 evaluation as the plain sum over
 * every kept helicity (colour sums and averaging included), counted by
 * running the generated amplitude code on the host with an
 * operation-counting scalar.  One rwgt_eval over nevt events and nsets cards
 * computes (1 + nsets) * nevt of them.  Used to express measured throughput
 * as FLOP/s against the peak (the algorithmic rate). */
int rwgt_flops(const rwgt_ctx *ctx, double *flops_per_me2);

/* Device bounds checks (test tooling, for callers that validate the
 * library's index arithmetic).  The check build of the library
 * (librwgt_check.so, compiled with -DRWGT_CHECK) compares every global-memory
 * index of the matrix-element, ingest, cross-section, factored, running-alpha_s,
 * non-finite-count, batched and card-per-event kernels with its array's extent;
 * an index outside it is counted and its access redirected to a scratch sink.
 * *enabled: 1 in the check build, 0 in the normal one (where *misses is 0).
 * *misses: indices out of range since the previous call (the counters are
 * cleared), summed over the kernels' translation units.  Reads device
 * counters of the current device; call after the work has finished.
 * Errors: RWGT_EINVAL (NULL argument), RWGT_EDEVICE (a counter copy failed). */
int rwgt_bounds_check(int32_t *enabled, uint64_t *misses);

/* The same count for the helicities the kernels actually evaluate.  For the
 * pure-QCD processes (g g > t t~ g g, g g > t t~ t t~) reversing every
 * helicity leaves |M_h|^2 unchanged (parity of QCD), so of the
 * helicity-summed |M|^2 (MadtRex section, Usage) one helicity of each
 * reversed pair is evaluated and counted twice: half of rwgt_flops.
 * Otherwise equal to rwgt_flops.  Gives the executed rate. */
int rwgt_flops_executed(const rwgt_ctx *ctx, double *flops_per_me2);

/* Reweighted cross sections and their errors for nsets cards (teaRex section):
 *   sigma'_k  = norm * sum_i w'_ki,
 *   dsigma'_k = dsigma * (1/N) sum_i w'_ki / w_i + sigma * std_i(w'_ki),
 * std the population standard deviation, terms with w_i = 0 counted as 0.
 * If dsigma'_k is infinite, NaN or not positive, a warning goes to stderr,
 * fallback[k] = 1 and dsigma'_k = dsigma * max(sigma'_k/sigma, sigma/sigma'_k).
 * weights_in [nevt], weights_out [nsets][nevt]: DEVICE; xsec, xerr [nsets] and
 * fallback [nsets] (optional): HOST.  The sums are reduced on the device in a
 * fixed order (reproducible); the call waits for the result. */
int rwgt_xsec(rwgt_ctx *ctx, const double *weights_in, const double *weights_out, int64_t nevt, int32_t nsets,
              double sigma, double dsigma, double norm, double *xsec, double *xerr, int32_t *fallback);

/* rwgt_xsec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result bit for bit, with the partial sums in a
 * static device array of the library (about 790 KB per GPU, held until the
 * process ends) instead of per-call allocations.  At most 64 cards
 * (nsets > 64: RWGT_EINVAL).  The array is shared by every call on a GPU:
 * calls that overlap on one GPU (two host threads, or two streams) race and
 * must be serialised by the caller.  Nothing in the array needs clearing (each
 * call writes every partial it reads).  Errors as rwgt_xsec. */
int rwgt_xsec_noalloc(rwgt_ctx *ctx, const double *weights_in, const double *weights_out, int64_t nevt,
                      int32_t nsets, double sigma, double dsigma, double norm, double *xsec, double *xerr,
                      int32_t *fallback);

/* Record HIP events around the ingest and matrix-element kernels of each
 * subsequent rwgt_eval / rwgt_me2 (on the context's stream). */
int rwgt_set_profiling(rwgt_ctx *ctx, int enable);

/* Durations in milliseconds of the two kernels of the last call made with
 * profiling on; waits for that call to finish. */
int rwgt_kernel_times(rwgt_ctx *ctx, float *ingest_ms, float *me_ms);

/* ------------------------------------------------------------------------
 * Batched form: many reweighting jobs of one process family in one launch.
 *
 * Each segment is one rwgt_eval-like job with a single new card: its events
 * (DEVICE momenta [nevt][npart][4], weights in/out [nevt]) are reweighted from
 * the original card of contexts[ctx] to the card in params (HOST, one
 * param_sets row of that context's layout).  All segments of one call go to
 * one persistent kernel (workgroups take event tiles from a shared counter),
 * captured once into a HIP graph and replayed while the number of segments,
 * tiles and the schedule stay the same.  The schedule (tile size, workgroup
 * size, workgroups per CU, helicity split) comes from rwgt_batch_set_schedule,
 * the tuning cache written by rwgt_batch_tune, or a default.  The paper runs
 * subprocesses on a CPU thread pool and notes that sequential subprocesses
 * leave the GPU latency-bound (MadtRex section, Runtime comparisons); this is
 * the single-launch alternative, and every rwgt_batch_* call below belongs to
 * it.
 * Family: e+ e- > mu+ mu- and u u~ > e+ e- g, all contexts of one precision.
 */
typedef struct rwgt_batch rwgt_batch;

typedef struct {
  int32_t ctx;                 /* index into the contexts of rwgt_batch_create */
  int32_t reserved;
  int64_t nevt;                /* events of the segment (0: skipped) */
  const double *momenta;       /* DEVICE [nevt][npart][4] */
  const double *weights_in;    /* DEVICE [nevt] */
  const double *params;        /* HOST [npar]: the new card */
  double *weights_out;         /* DEVICE [nevt] */
} rwgt_segment;

/* Bind contexts (not owned; they must outlive the batch).  Errors: RWGT_EINVAL,
 * RWGT_EPROCESS (a context outside the family), RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_batch_create(rwgt_ctx *const *contexts, int32_t ncontexts, rwgt_batch **out);
void rwgt_batch_destroy(rwgt_batch *batch);
/* Stream of subsequent launches (NULL: a stream owned by the batch, which
 * synchronises with the null stream). */
int rwgt_batch_set_stream(rwgt_batch *batch, void *stream);
/* Enqueue all segments as one graph launch.  Errors as rwgt_eval. */
int rwgt_batch_eval(rwgt_batch *batch, const rwgt_segment *segments, int32_t nsegments);
/* Milliseconds of the last graph launch (waits for it). */
int rwgt_batch_time(rwgt_batch *batch, float *ms);
/* Fix the schedule: events per tile, threads per workgroup (64..256, multiple
 * of 64), persistent workgroups per compute unit, and hel_split: 0 = one lane
 * per event (both cards, every kept helicity), 1 = one lane per (event, card,
 * kept helicity), the lanes of an event added in the one-lane order (the
 * same result to the bit).  Errors: RWGT_EINVAL. */
int rwgt_batch_set_schedule(rwgt_batch *batch, int32_t tile_events, int32_t block, int32_t blocks_per_cu,
                            int32_t hel_split);
/* hel_split may be NULL. */
int rwgt_batch_get_schedule(const rwgt_batch *batch, int32_t *tile_events, int32_t *block, int32_t *grid,
                            int32_t *hel_split);
/* Autotune the schedule on these segments (each candidate timed reps times
 * after one capture run); keeps the fastest and records it in the cache. */
int rwgt_batch_tune(rwgt_batch *batch, const rwgt_segment *segments, int32_t nsegments, int32_t reps);
const char *rwgt_batch_last_error(const rwgt_batch *batch);

/* ------------------------------------------------------------------------
 * Learned surrogate: a multilayer perceptron for log(w'/w) with a second
 * head for the log of its own error, trained and run by the library's own
 * kernels with FP32 master weights, Adam and FP32 accumulation.  Operand
 * types: in a BF16 network the first layer and the head are FP32 (VALU) and
 * the width x width hidden layers BF16 (matrix cores); in an FP32 network
 * (gradient checks) every layer is FP32.  Hidden layers use SiLU.
 *
 * Input row of one (event, card) pair, standardised with the mean and
 * standard deviation of rwgt_mlp_set_normalisation, from one of two maps
 * (rwgt_mlp_set_features; n_in must equal the map's width):
 *   RWGT_FEAT_RAW   [momenta (npart*4), M_Z, Gamma_Z, sin^2 theta_W]
 *   RWGT_FEAT_PHYS  with s_hat = 2 p0.p1, s_ij = 2 pi.pj (massless momenta):
 *                   [log s_hat, log(|s_ij| / s_hat) for i < j (row-major),
 *                    M_Z, Gamma_Z, sin^2 theta_W, asinh Re chi, asinh Im chi,
 *                    asinh Re chi0, asinh Im chi0],
 *                   chi = s / (s - M_Z^2 + i M_Z Gamma_Z) at s = s_ab of the
 *                   resonant pair (a, b) under the card, chi0 under the
 *                   original card: 1 + npart(npart-1)/2 + 7 inputs.
 * Targets y are standardised, y' = (y - y_mean) / y_std
 * (rwgt_mlp_set_target_scale); mu and s below are in y' units, and every
 * output (heads, gate) is converted back: mu_y = mu y_std + y_mean,
 * s_y = s + log y_std.  Loss per row:
 *   1/2 (y' - mu)^2 + lambda (1/2 r^2 exp(-2 s) + s),  r = y' - mu held fixed,
 * mu = head 0, s = head 1 (clamped at -15).  Device pointers unless noted;
 * calls enqueue on the network's stream (rwgt_mlp_set_stream).
 */
typedef struct rwgt_mlp rwgt_mlp;

enum { RWGT_MLP_BF16 = 0, RWGT_MLP_FP32 = 1 };
enum { RWGT_FEAT_RAW = 0, RWGT_FEAT_PHYS = 1 };

/* n_in (1..32) inputs, depth hidden layers of width (multiple of 32), n_out
 * heads (2..32); He-uniform initial weights from seed (last layer scaled by
 * 0.1), zero biases.  Errors: RWGT_EINVAL, RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t precision, uint64_t seed,
                    rwgt_mlp **out);
void rwgt_mlp_destroy(rwgt_mlp *mlp);
int rwgt_mlp_set_stream(rwgt_mlp *mlp, void *stream);
/* Number of parameters; get/set pack them (HOST float array) layer by layer as
 * W[out][in] row-major then b[out]; get_grads packs the last gradients. */
int rwgt_mlp_num_params(const rwgt_mlp *mlp, int64_t *n);
int rwgt_mlp_get_params(rwgt_mlp *mlp, float *host);
int rwgt_mlp_set_params(rwgt_mlp *mlp, const float *host);
int rwgt_mlp_get_grads(rwgt_mlp *mlp, float *host);
/* HOST arrays of n_in floats (standard deviations positive). */
int rwgt_mlp_set_normalisation(rwgt_mlp *mlp, const float *mean, const float *stdv);
/* Feature map (see above) for npart (4 or 5) external particles; res_a,
 * res_b: the resonant pair; mz0, wz0: the original card's Z mass and width.
 * Without this call a network uses the raw map of the npart passed to
 * rwgt_mlp_features.  Errors: RWGT_EINVAL (unknown map, width mismatch). */
int rwgt_mlp_set_features(rwgt_mlp *mlp, int32_t kind, int32_t npart, int32_t res_a, int32_t res_b, double mz0,
                          double wz0);
/* HOST outputs: mean and stdv (n_in floats each) of the input normalisation
 * and y_scale = (y_mean, y_std). */
int rwgt_mlp_get_normalisation(rwgt_mlp *mlp, float *mean, float *stdv, float *y_scale);
/* Target standardisation (y_std > 0). */
int rwgt_mlp_set_target_scale(rwgt_mlp *mlp, float y_mean, float y_std);
/* Sets the input normalisation to the mean and (population) standard
 * deviation of each feature over n rows given as in rwgt_mlp_features
 * (constant features: standard deviation 1); FP64 sums on the device, waits
 * for the stream. */
int rwgt_mlp_fit_normalisation(rwgt_mlp *mlp, const double *momenta, int32_t npart, const int32_t *event_index,
                               const int32_t *card_index, const float *card_params, int64_t n);
/* Sets the target scale to the mean and standard deviation of y [n] (device
 * FP32); waits for the stream. */
int rwgt_mlp_fit_target_scale(rwgt_mlp *mlp, const float *y, int64_t n);
/* Loss weight lambda of the error head and the Adam constants. */
int rwgt_mlp_set_training(rwgt_mlp *mlp, float lambda, float beta1, float beta2, float eps);
/* Quantile factor k: the error bound of a prediction is k exp(s_y). */
int rwgt_mlp_set_calibration(rwgt_mlp *mlp, float k);
/* Bytes of the FP32 input buffer for n rows (rows padded to a multiple of 64,
 * 32 columns). */
int rwgt_mlp_input_bytes(const rwgt_mlp *mlp, int64_t n, int64_t *bytes);
/* Input rows of the training path: row r = features of (momenta[event_index[r]]
 * (npart*4 doubles each; event_index NULL: r), card_params[card_index[r]]
 * (nparam = 3 floats: M_Z, Gamma_Z, sin^2 theta_W)), standardised. */
int rwgt_mlp_features(rwgt_mlp *mlp, const double *momenta, int32_t npart, const int32_t *event_index,
                      const int32_t *card_index, const float *card_params, int32_t nparam, int64_t n, void *x_out);
/* Layered forward pass: heads of n rows into heads_out [n][32] (FP32; column 0
 * = mu_y, 1 = s_y, the others the padding heads). */
int rwgt_mlp_forward(rwgt_mlp *mlp, const void *x, int64_t n, float *heads_out);
/* Fused forward pass from the momenta (rows as in rwgt_mlp_features):
 * heads_out [n][2] = (mu_y, s_y).  The first layer runs as three BF16
 * products of the high and low parts of its FP32 operands, the hidden layers
 * in BF16 as in training, the head in FP32.  BF16 networks of width 128 or
 * 256 and depth 2..9 only (else RWGT_EINVAL). */
int rwgt_mlp_predict(rwgt_mlp *mlp, const double *momenta, int32_t npart, const int32_t *event_index,
                     const int32_t *card_index, const float *card_params, int64_t n, float *heads_out);
/* Forward, loss, backward and (lr > 0) one Adam step on n rows with targets y
 * [n] (FP32, unstandardised); the summed loss goes to loss_out (device float)
 * if non-NULL. */
int rwgt_mlp_train_step(rwgt_mlp *mlp, const void *x, const float *y, int64_t n, float lr, float *loss_out);
/* Training targets y[i] = log(w_new[i] / w_old[i]) (w_old NULL: 1; w_old = 0: y = 0). */
int rwgt_mlp_targets(rwgt_mlp *mlp, const double *w_new, const double *w_old, int64_t n, float *y);
const char *rwgt_mlp_last_error(const rwgt_mlp *mlp);
/* Adam state (HOST outputs): first and second moments packed as
 * rwgt_mlp_get_params, and the number of Adam steps taken (the t of the bias
 * corrections 1 - beta^t).  Waits for the stream. */
int rwgt_mlp_get_adam(rwgt_mlp *mlp, float *first, float *second, int64_t *steps);

/* Training on a grid of (event, card) pairs.  Pair j of an nevt x ncards grid
 * is event j % nevt of momenta [nevt][npart][4] (DEVICE) with card j / nevt of
 * card_params [ncards][3] (DEVICE, M_Z, Gamma_Z, sin^2 theta_W), target
 * y[j] (DEVICE float [ncards][nevt], e.g. from rwgt_mlp_targets on
 * rwgt_eval's weights_out).
 *
 * Fits the input normalisation (mean and population standard deviation of
 * every feature over all pairs) and the target scale (of y); waits. */
int rwgt_mlp_fit_grid(rwgt_mlp *mlp, const double *momenta, int32_t npart, int64_t nevt, const float *card_params,
                      int32_t ncards, const float *y);

/* Schedule of rwgt_mlp_train: steps of batch pairs, floor(pairs / batch) per
 * epoch, each pair at most once per epoch; learning rate
 * lr (lr_final / lr)^(step / (steps - 1)) over the steps of all epochs. */
typedef struct rwgt_train_cfg {
  int64_t batch;      /* pairs per Adam step, 1..pairs */
  int32_t epochs;     /* epochs of the whole schedule */
  float lr, lr_final; /* learning rate at the first and at the last step */
  uint64_t seed;      /* order of the pairs in each epoch (rwgt_train_order) */
} rwgt_train_cfg;

/* Trains epochs [epochs done, epoch_end) of the schedule: per step, the next
 * batch of the epoch's pair order (rwgt_train_order of seed, epoch, pairs),
 * their standardised features, forward, loss, backward and one Adam step.  The
 * first call fixes the schedule; later calls (also after rwgt_mlp_load) must
 * pass the same one, so training in pieces gives the parameters of one
 * uninterrupted run.  epoch_loss (HOST, optional, epoch_end - epochs done
 * floats): mean loss per pair of each epoch, read on every 64th step (then
 * the call waits).  Errors: RWGT_EINVAL (bad sizes, schedule or epoch_end,
 * a changed schedule), RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_mlp_train(rwgt_mlp *mlp, const double *momenta, int32_t npart, int64_t nevt, const float *card_params,
                   int32_t ncards, const float *y, const rwgt_train_cfg *cfg, int32_t epoch_end, float *epoch_loss);
/* Epochs and steps of the schedule done, and Adam steps taken (HOST outputs). */
int rwgt_mlp_get_progress(const rwgt_mlp *mlp, int64_t *epoch, int64_t *steps, int64_t *adam_steps);
/* Pair order of training: out[i] (HOST) = the pair at position pos0 + i of
 * epoch `epoch` of a grid of n pairs, a bijection of [0, n) for each (seed,
 * epoch): a four-round Feistel network keyed by SplitMix64's mixer, cycle
 * walked into [0, n).  Host only. */
int rwgt_train_order(uint64_t seed, int64_t epoch, int64_t n, int64_t pos0, int64_t count, int64_t *out);

/* Calibration of the error head: over every pair of the grid, the residual
 * r = |y - mu_y| and its size in predicted errors z = r / exp(s_y) (FP64 on
 * the host, from the network's FP32 heads); k = the coverage quantile of z
 * (linear interpolation at position (pairs - 1) coverage between order
 * statistics) becomes the network's calibration factor.  stats (HOST, 4
 * doubles) = (k, median r, 0.9 quantile of r, 0.999 quantile of r).  Waits.
 * Errors: RWGT_EINVAL (coverage outside (0, 1), a non-finite residual). */
int rwgt_mlp_calibrate(rwgt_mlp *mlp, const double *momenta, int32_t npart, int64_t nevt, const float *card_params,
                       int32_t ncards, const float *y, double coverage, double *stats);

/* Checkpoints: one file with the network shape, feature map, normalisation,
 * target scale, calibration factor, loss weight and Adam constants, FP32
 * master parameters, both Adam moments and their step count, the training
 * schedule and the epochs and steps done, closed by a 64-bit FNV-1a hash.
 * rwgt_mlp_save writes (via a temporary file renamed over path; waits);
 * rwgt_mlp_load creates a network on the current device from a file;
 * rwgt_mlp_checkpoint_info reads and checks a file on the host only: shape
 * (5 ints: n_in, width, depth, n_out, precision), epochs done, Adam steps.
 * Errors: RWGT_EINVAL (unreadable or unwritable path), RWGT_ECARD (not a
 * checkpoint, wrong version, hash or size mismatch: message from
 * rwgt_mlp_checkpoint_error), RWGT_EDEVICE, RWGT_ENOMEM. */
int rwgt_mlp_save(rwgt_mlp *mlp, const char *path);
int rwgt_mlp_load(const char *path, rwgt_mlp **out);
int rwgt_mlp_checkpoint_info(const char *path, int32_t *shape, int64_t *epoch, int64_t *adam_steps);
const char *rwgt_mlp_checkpoint_error(void);

/* Exact reweighting with a card per event (the path rwgt_sur_eval falls back
 * to, on every event): event i gets card card_index[i] (DEVICE int32, in
 * [0, ncards)) of param_table (HOST [ncards][npar], the context's layout),
 * w'_i = (w_i / |M|^2(p_i; original)) |M|^2(p_i; card).  An index outside
 * [0, ncards) reads no card: that event's w' is NaN, counted by
 * rwgt_nonfinite.  Processes of the electroweak family.  Errors as rwgt_eval,
 * RWGT_EPROCESS for other processes. */
int rwgt_eval_cards(rwgt_ctx *ctx, const double *momenta, int64_t nevt, const double *weights_in,
                    const double *param_table, int32_t ncards, const int32_t *card_index, double *weights_out);

/* Reweighting through the surrogate with exact fallback (same result
 * definition as rwgt_eval): event i gets card card_index[i] (DEVICE int32) of
 * param_table (HOST [ncards][npar], the context's layout); where the predicted
 * error k exp(s) of log(w'/w) is at most err_threshold,
 * w'_i = w_i exp(mu_i); elsewhere w'_i is computed exactly by the
 * matrix-element path.  The network's inputs are its feature map of the
 * momenta and the card's (M_Z, Gamma_Z, sin^2 theta_W).  Networks eligible
 * for rwgt_mlp_predict run as one fused kernel (features, layers, heads and
 * gate), others layer by layer.  *n_fallback (HOST, optional; waits for the
 * call) receives the number of exact evaluations.  A card index outside
 * [0, ncards) gives that event NaN inputs, so it falls back, and the exact
 * path writes NaN for it (counted by rwgt_nonfinite).  Processes of the
 * electroweak family. */
int rwgt_sur_eval(rwgt_ctx *ctx, rwgt_mlp *mlp, const double *momenta, int64_t nevt, const double *weights_in,
                  const double *param_table, int32_t ncards, const int32_t *card_index, double err_threshold,
                  double *weights_out, int64_t *n_fallback);

/* ------------------------------------------------------------------------
 * Event files (host only, no device work).  An LHE v3 file is read into
 * memory; its events can be sorted by process (external partons: status -1
 * incoming, +1 outgoing, matched to the process string's particles by PDG
 * code, each slot taking the first unused matching parton in file order),
 * their momenta exported in the process's particle order as the AoS
 * [n][npart][4] (E, px, py, pz) that rwgt_eval takes, and weights appended:
 * each new weight id gets a <weight> entry in the header's <initrwgt> and a
 * <wgt> in every event's <rwgt> block (0 for events it was not set on, the
 * paper's zero weight for events without a matching process).  Everything
 * else in the file is written back byte for byte.  Numbers are read
 * correctly rounded (a leading '+' and Fortran 'D' exponents accepted) and
 * weights written with 17 significant digits, so they round-trip exactly.
 */
typedef struct rwgt_lhe rwgt_lhe;

/* Read a file (path) or a memory buffer (text, len bytes).  Errors:
 * RWGT_EINVAL (NULL, unreadable file), RWGT_ECARD (malformed: message from
 * rwgt_lhe_read_error), RWGT_ENOMEM. */
int rwgt_lhe_read(const char *path, rwgt_lhe **out);
int rwgt_lhe_parse(const char *text, int64_t len, rwgt_lhe **out);
const char *rwgt_lhe_read_error(void);
void rwgt_lhe_destroy(rwgt_lhe *lhe);
const char *rwgt_lhe_last_error(const rwgt_lhe *lhe);
int rwgt_lhe_num_events(const rwgt_lhe *lhe, int64_t *n);
/* Event i: particle count, process id, info = (XWGTUP, SCALUP, AQEDUP, AQCDUP). */
int rwgt_lhe_event_info(const rwgt_lhe *lhe, int64_t i, int32_t *nup, int32_t *idprup, double *info);
/* info [n][4] (HOST) = (XWGTUP, SCALUP, AQEDUP, AQCDUP) of events index[0..n). */
int rwgt_lhe_info(const rwgt_lhe *lhe, const int64_t *index, int64_t n, double *info);
/* Indices (file order) of the events of a process: *n_match gets the count,
 * index_out (HOST, capacity cap) the first min(cap, count).  Errors:
 * RWGT_EPROCESS (unknown particle name). */
int rwgt_lhe_select(rwgt_lhe *lhe, const char *process, int64_t *index_out, int64_t cap, int64_t *n_match);
/* HOST momenta [n][npart][4] and (optional) weights [n] = XWGTUP of the
 * events index[0..n); RWGT_EPROCESS if one does not belong to the process. */
int rwgt_lhe_momenta(rwgt_lhe *lhe, const char *process, const int64_t *index, int64_t n, double *momenta,
                     double *weights);
/* Set weight `id` (no quotes, spaces, '<', '>', '&') of events index[0..n)
 * to w (HOST); a new id starts at 0 on every event. */
int rwgt_lhe_add_weights(rwgt_lhe *lhe, const char *id, const char *description, const int64_t *index, int64_t n,
                         const double *w);
int rwgt_lhe_write(rwgt_lhe *lhe, const char *path);

/* Layout of a process's param_sets rows without a context (as
 * rwgt_param_layout); RWGT_EPROCESS for an unsupported process. */
int rwgt_process_layout(const char *process, int32_t *npar, const char **names);

/* Parameter sets from a reweighting card (the paper's SLHA reweighting:
 * "launch rwgt_name=NAME" opens a set equal to the original card, "set BLOCK
 * ID VALUE" overrides an entry; "change fptype X" is reported in fptype[0];
 * '#' comments).  Rows follow the process's layout (rwgt_param_layout);
 * entries outside it do not affect the process and are skipped.  Host only:
 * param_sets [cap][npar], names [cap][name_len] (optional), fptype [2]
 * (optional, untouched if the card has none).  *nsets gets the number of
 * sets, possibly above cap (then only cap rows are filled).  Errors:
 * RWGT_EINVAL, RWGT_EPROCESS, RWGT_ECARD (message from rwgt_create_error). */
int rwgt_reweight_card(const char *process, const char *param_card, const char *rwgt_card, int32_t cap,
                       double *param_sets, int32_t *nsets, char *names, int32_t name_len, char *fptype);

#ifdef __cplusplus
}
#endif

#endif /* RWGT_H */
