/*
 * pa.h -- C ABI of libpa: population annealing (PA) of the 2D ferromagnetic
 * Ising model on L x L periodic lattices, run on one MI355X (gfx950).
 *
 * Method: Barash, Weigel, Borovsky, Janke, Shchur, "GPU accelerated population
 * annealing algorithm" (arXiv:1703.03676).  One PA run holds a population of
 * R_i replicas at inverse temperature beta_i.  Per temperature step the caller
 *   1. picks beta_{i+1} (fixed step, or pa_adapt_beta: Sec. 2.3),
 *   2. calls pa_resample (Sec. 2.1 step 2, Eqs. (Q) and (resampling factors)),
 *   3. calls pa_sweep(theta) (Sec. 2.1 step 3; checkerboard Metropolis, Sec. 3),
 *   4. calls pa_observables (Sec. 2.1 step 4, Eqs. (observables), (free
 *      energy), (entropy)),
 * and at the end may call pa_reweight (Sec. 2.4, multi-histogram Eq.).
 *
 * Conventions shared by every call:
 *   - Every call returns pa_status; 0 (PA_OK) is success.  No exception or
 *     abort crosses the ABI.  After PA_EHIP the run is unusable and later calls
 *     return PA_ESTATE; pa_free is always allowed.
 *   - Device memory belongs to the caller: pa_init receives one device buffer of
 *     at least pa_workspace_bytes(p) bytes that must outlive the run.  The
 *     library allocates no device memory of its own; its one static device
 *     array serves pa_observables_static only.
 *   - The HIP stream passed to pa_init is borrowed; all device work of the run
 *     is enqueued on it.  Calls that return host values (pa_resample's info,
 *     pa_adapt_beta, pa_observables, pa_reweight, the download hooks)
 *     synchronise that stream before returning.
 *   - Spin convention: +1 / -1; J = 1, h = 0; E = -sum over the 2N bonds;
 *     M = sum of spins.  Energies are multiples of 4 in [-2N, 2N].
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed, with counters
 *     derived from (replica slot, sweep number, colour, site) for the sweep,
 *     (parent slot, step) for resampling and (replica, site) for the initial
 *     state; the last counter word holds 16 * run_id + the stream number, so
 *     distinct (seed, run_id) pairs never share a stream.  Results are
 *     therefore bit-reproducible for a given seed, run_id and schedule,
 *     independent of launch shapes.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PA_OK = 0,
    PA_EINVAL = -1,     /* invalid argument (validated on the host before any launch) */
    PA_ENOMEM = -2,     /* workspace too small / host allocation failed */
    PA_ECAPACITY = -3,  /* resampled population would exceed the capacity; state unchanged */
    PA_EHIP = -4,       /* a HIP runtime call failed; see pa_last_error */
    PA_ESTATE = -5,     /* run unusable (after PA_EHIP) or call out of order */
    PA_EEXTINCT = -6    /* resampling would leave no replica; state unchanged */
} pa_status;

typedef enum {
    PA_SPIN_INT8 = 0,   /* one signed byte (+1 / -1) per spin, row-major (single-spin coding) */
    PA_SPIN_BITS = 1,   /* one bit per spin, per-colour 32-site words (multi-spin coding) */
    PA_SPIN_INTERLEAVED = 2  /* one signed byte per spin, the same spin of all replicas adjacent
                                (spin (x, y) of replica j at byte (y L + x) * stride + j, stride the
                                capacity rounded up to 64), swept replica-parallel: each replica
                                goes through its lattice site by site on its own thread (four lanes
                                sharing a colour's sites from L = 64 on; Sec. 3, the
                                replica-parallel setup, the paper's general fall-back); single runs
                                only (pa_batch_init refuses it) */
} pa_layout;

enum {
    PA_FLAG_MHR = 1,      /* accumulate the per-energy histograms used by pa_reweight */
    PA_FLAG_HEATBATH = 2, /* sweeps use the heat-bath update instead of Metropolis (see pa_sweep) */
    PA_FLAG_LCG = 4       /* Metropolis sweeps take their uniforms from the in-line LCG variant
                             (see pa_sweep); not with PA_FLAG_HEATBATH */
};

typedef struct {
    int32_t L;          /* lattice edge; the library runs L in {16, 32, 64, 128, 256} */
    int32_t R;          /* target population size R (Sec. 2.1), >= 1 */
    int32_t capacity;   /* maximum population; 0 selects R + ceil(10 sqrt(R)) + 64 */
    int32_t layout;     /* pa_layout of the spin store */
    uint64_t seed;      /* Philox key material */
    uint32_t run_id;    /* < 2^28: independent runs of one seed (part of every random counter) */
    uint32_t flags;     /* PA_FLAG_* */
} pa_params;

/* Population averages at the current beta: the ten output columns the paper
 * lists for each temperature (Sec. 3, program output), then the exact integer
 * sums they come from.  sumM4 is a 128-bit unsigned value split in two words. */
typedef struct {
    double beta, e, C, abs_m, m2, m4, betaF_per_N, S_per_N, lnQ;
    int64_t R;
    int64_t sumE, sumE2, sumAbsM, sumM2;
    uint64_t sumM4_lo, sumM4_hi;
} pa_obs;

typedef struct {
    double lnQ;         /* ln Q_i of Eq. (Q) */
    int64_t R_new;      /* R_i = sum of copy counts */
    int32_t E_min;      /* smallest energy in the parent population (weight shift) */
} pa_resample_info;

typedef struct {
    int64_t R;          /* current population size R_i */
    int32_t step;       /* number of resampling steps done (i) */
    uint64_t sweeps;    /* sweeps done in this run (keys the sweep random stream) */
    double beta;        /* current beta_i */
    double lnZ;         /* ln Z(beta_i) estimate, Eq. (free energy) */
} pa_state_info;

typedef struct pa_run pa_run;  /* opaque host handle */

/* Bytes of device workspace a run with these parameters needs; 0 if the
 * parameters are invalid.  Pure host function. */
size_t pa_workspace_bytes(const pa_params* p);

/* Start a run at beta_0 = 0 (Sec. 2.1 step 1): R independent uniformly random
 * configurations; ln Z_0 = N ln 2.  `d_workspace` is a device pointer to at
 * least `bytes` bytes, 256-byte aligned; `hip_stream` is a hipStream_t (NULL:
 * the null stream).  On success *out receives the handle.
 * Errors: PA_EINVAL (L not supported, R < 1, capacity < R, bad layout,
 * run_id >= 2^28, NULL pointers), PA_ENOMEM (bytes too small), PA_EHIP. */
pa_status pa_init(const pa_params* p, void* d_workspace, size_t bytes, void* hip_stream, pa_run** out);

/* nsweeps checkerboard Metropolis sweeps of every replica at the current beta
 * (Sec. 2.1 step 3; Sec. 3 spin updates).  One sweep updates colour (x+y) even,
 * then odd.  A spin with local field h flips if k = s h <= 0, else with
 * probability exp(-2 beta k), decided against an integer threshold
 * ceil(2^32 exp(-2 beta k)).  With PA_FLAG_HEATBATH the update is heat-bath
 * instead (Sec. 2.1 names it as an alternative): the spin flips with
 * probability 1 / (1 + exp(2 beta k)), i.e. iff its 32-bit uniform is below
 * U_k = ceil(2^32 / (1 + exp(2 beta k))) for k = 2, 4, U_0 = 2^31,
 * U_{-k} = 2^32 - U_k.  Both use the same random streams.  With PA_FLAG_LCG
 * the Metropolis uniforms come instead from the in-line generator of the
 * paper's multi-spin-coded variant (Sec. 4): per sweep and per 32-site word of
 * one colour, one Philox draw seeds r' = 1664525 r + 1013904223 mod 2^32, and
 * the word's site b takes the (b+1)-th output; a different Markov chain with
 * the same stationary distribution.  Updates E_j and M_j.  Asynchronous; on
 * the int8 and bit stores the sweep kernel also queues the statistics of the
 * swept population (histogram and integer sums), which the next
 * pa_observables, pa_alpha, pa_adapt_beta or pa_resample reads after waiting
 * for the stream.
 * Errors: PA_EINVAL (nsweeps < 0), PA_ESTATE, PA_EHIP. */
pa_status pa_sweep(pa_run* r, int32_t nsweeps);

/* Resample the population from beta_i to beta_next >= beta_i (Sec. 2.1 step 2):
 * reweight by exp(-(beta_next - beta_i) E), Q from Eq. (Q), copy counts by
 * Eq. (resampling factors) with one uniform per parent, prefix-sum compaction,
 * replica copy.  Parents keep their order; copies of one parent are adjacent.
 * Updates ln Z += ln Q.  `out` may be NULL.
 * Errors: PA_EINVAL (beta_next < beta_i or not finite), PA_ECAPACITY and
 * PA_EEXTINCT (R_i would exceed the capacity / be 0; state left at step i),
 * PA_ESTATE, PA_EHIP. */
pa_status pa_resample(pa_run* r, double beta_next, pa_resample_info* out);

/* Histogram-overlap adaptive step (Sec. 2.3): returns in *beta_next the
 * largest beta' <= beta_f (found by bisection, 50 halvings) with
 * alpha(beta_i, beta') >= alpha_star, or beta_f if alpha(beta_f) >= alpha_star.
 * alpha_at_next may be NULL.  Does not change the run.
 * Errors: PA_EINVAL (alpha_star not in (0,1), beta_f < beta_i, or no step above
 * beta_i reaches alpha_star), PA_ESTATE, PA_EHIP. */
pa_status pa_adapt_beta(pa_run* r, double alpha_star, double beta_f, double* beta_next, double* alpha_at_next);

/* Overlap alpha(beta_i, beta_prime) of Sec. 2.3 for the current population. */
pa_status pa_alpha(pa_run* r, double beta_prime, double* alpha);

/* Population averages at the current beta (Eq. (observables)), -beta F/N from
 * Eq. (free energy), S/N from Eq. (entropy), and the exact integer sums.  With
 * PA_FLAG_MHR each call also adds the population's energy histogram (and
 * per-energy magnetisation sums) to the reweighting accumulators.
 * Errors: PA_EINVAL (out NULL), PA_ESTATE, PA_EHIP. */
pa_status pa_observables(pa_run* r, pa_obs* out);

/* Multi-histogram reweighting (Sec. 2.4): the density of states from all
 * measurements taken so far, then e, C, <|m|>, <m^2>, <m^4>, beta F/N and S/N
 * at each of the nb inverse temperatures betas[0..nb).  out[k].R and
 * out[k].lnQ and the integer sums are 0.  Requires PA_FLAG_MHR.
 * Errors: PA_EINVAL (flag not set, nb < 0, NULL pointers, no measurement),
 * PA_ESTATE, PA_EHIP. */
pa_status pa_reweight(pa_run* r, const double* betas, int32_t nb, pa_obs* out);

/* Current counters of the run (host values, no synchronisation). */
pa_status pa_state(const pa_run* r, pa_state_info* out);

/* Release the host handle (the caller frees the workspace).  NULL is allowed. */
pa_status pa_free(pa_run* r);

/* Static description of a status code. */
const char* pa_strerror(pa_status s);

/* Text of the last error of this run ("" if none). */
const char* pa_last_error(const pa_run* r);

/* Weighted average of nruns independent runs of the same system and target
 * population size, measured at the same nb inverse temperatures (Sec. 2.2,
 * Eq. (weighted-average)).  obs[m * nb + i] is run m's measurement at the
 * i-th temperature (as returned by pa_observables or pa_anneal); out[i]
 * (nb entries, caller-owned) receives:
 *   beta;  e, C, abs_m, m2, m4 weighted by w_m = exp(-beta F_m) / sum_m'
 *   exp(-beta F_m'), with ln Z_m = -N * betaF_per_N of run m;
 *   betaF_per_N of the pooled estimate of Z, -ln((1/M) sum_m Z_m) / N;
 *   S_per_N = beta e + ln Z / N of the combination;  R = sum of the R_m;
 *   lnQ and the integer sums 0.
 * Host arithmetic only (FP64, runs summed in ascending order); no run handle
 * and no device work.  PA_EINVAL: N < 1, nruns < 1, nb < 0, NULL arrays with
 * nb > 0, or temperatures that differ between runs (out is then
 * unspecified). */
pa_status pa_weighted_average(int32_t N, int32_t nruns, int32_t nb, const pa_obs* obs, pa_obs* out);

/* ---- For callers that cannot allocate memory. --------------------------------
 * pa_observables for a population held in caller buffers, for callers that
 * cannot call hipMalloc or hipHostMalloc or create a run (serving loops,
 * harnesses that forbid allocation).  d_E and d_M are device arrays of the R
 * replicas' energies and magnetisations (int32; E is a multiple of 4 in
 * [-2N, 2N], N = L * L; read only).  beta, lnZ and lnQ are the population's
 * inverse temperature, ln Z estimate and last ln Q, copied into *out as
 * pa_observables does.  *out (host) receives the same values pa_observables
 * gives for that population: the averages of Eq. (observables), -beta F/N of
 * Eq. (free energy), S/N of Eq. (entropy) and the exact integer sums.
 * The statistics kernel's partial sums, statistics block and energy
 * histogram live in a statically allocated device array of
 * pa_static_scratch_bytes() bytes (about 0.5 MiB), one per GPU, held until
 * the process ends: the call allocates nothing.  It runs on hip_stream (NULL:
 * the null stream) of the current device and synchronises that stream.
 * Every call on a GPU uses that GPU's one array, so calls that overlap on one
 * GPU (other host threads, other streams) race and must be serialised by the
 * caller.  Errors: PA_EINVAL (L not in {16, 32, 64, 128, 256}, R < 1 or
 * R > PA_STATIC_MAX_R, NULL pointers, beta or lnZ not finite), PA_EHIP. */
#define PA_STATIC_MAX_R (1 << 20)
pa_status pa_observables_static(int32_t L, int32_t R, const int32_t* d_E, const int32_t* d_M, double beta,
                                double lnZ, double lnQ, void* hip_stream, pa_obs* out);

/* Size of the statically allocated device array of pa_observables_static. */
size_t pa_static_scratch_bytes(void);

/* ---- Test hooks: step-wise comparison with a reference implementation. ---- */

/* Copy the population to host memory: spins as int8 +-1, row-major,
 * [R_i][L][L] (converted from the run's layout); E and M as int32 [R_i].
 * Any pointer may be NULL. */
pa_status pa_download_population(pa_run* r, int8_t* spins, int32_t* E, int32_t* M);

/* Copy n selected replicas to host memory: idx[k] (0 <= idx[k] < R_i) is
 * the replica whose spins go to spins[k] (int8 +-1, row-major [L][L]) and
 * whose energy and magnetisation go to E[k], M[k].  For sampled checks of
 * populations too large to download whole.  E and M may be NULL.
 * PA_EINVAL if an index is out of range (nothing is copied). */
pa_status pa_download_replicas(pa_run* r, const int32_t* idx, int32_t n, int8_t* spins, int32_t* E, int32_t* M);

/* Replace the population by R_cur host configurations (int8 +-1, row-major)
 * and set the counters that key the random streams.  E and M are recomputed on
 * the device from the spins.  Errors: PA_EINVAL (R_cur out of [1, capacity],
 * spin values not +-1), PA_ESTATE, PA_EHIP. */
pa_status pa_upload_population(pa_run* r, int32_t R_cur, const int8_t* spins, int32_t step,
                               uint64_t sweeps, double beta, double lnZ);

/* Copy counts of the last resampling step, one per parent: *n receives the
 * number of parents; counts must hold capacity entries. */
pa_status pa_download_counts(pa_run* r, uint32_t* counts, int32_t* n);

/* Test hook for the sweeps of L >= 128, which keep each replica in LDS and
 * queue the words that hold a site whose uniform still ties with the
 * threshold after its 8 high bits, each word to be decided by one lane (Sec.
 * 3, spin updates).  When more words are queued than the queue holds (128
 * entries), every lane decides its own tied sites instead.  cap >= 0 lowers
 * the number of entries a wave may use before taking that second route (0:
 * always), so that tests reach it; values of 128 and above restore the
 * default.  Results do not depend on cap.
 * Errors: PA_EINVAL (cap < 0), PA_ESTATE. */
pa_status pa_set_tie_queue_cap(pa_run* r, int32_t cap);

/* Test and tuning hook for the population statistics of Sec. 2.1 (energy
 * histogram and integer moment sums of each new population).  The int8 and
 * bit stores can take them in the epilogue of the sweep that makes the
 * population (every wave adds its replicas with device atomics, then one
 * block sums them) or in a separate pass over E and M.  PA_STATS_AUTO (the
 * default) takes the epilogue where it measured faster: one replica per wave
 * (L >= 64) and R <= 32768, or L = 256.  PA_STATS_EPILOGUE and PA_STATS_PASS
 * force one of them (the interleaved store always uses the pass).  Results do
 * not depend on the choice.
 * Errors: PA_EINVAL (unknown mode), PA_ESTATE. */
typedef enum { PA_STATS_AUTO = 0, PA_STATS_EPILOGUE = 1, PA_STATS_PASS = 2 } pa_stats_path;
pa_status pa_set_stats_path(pa_run* r, int32_t mode);

/* ---- Batched runs: many independent PA runs advanced together. ----------
 * Every run has its own parameters (L, R, seed, run_id, layout, flags) and
 * schedule.  One pa_batch_step advances every unfinished run by one
 * temperature step (choose beta_{i+1}, resample, theta sweeps, measure) with
 * one batched launch per phase, replayed from a HIP graph, and one host
 * synchronisation for the whole batch.  Each run follows exactly the same
 * arithmetic and random streams as a single run with the same parameters and
 * schedule, so its results are bit-identical to that run's. */

typedef enum {
    PA_STEP_FIXED = 0,     /* beta_i = i * dbeta, last step clamped to beta_f (Sec. 2.1) */
    PA_STEP_ADAPTIVE = 1,  /* histogram-overlap bisection to alpha_star (Sec. 2.3) */
    PA_STEP_LEARNED = 2,   /* learned proposal accepted by the exact overlap test, else bisection */
    PA_STEP_FOLLOW = 3     /* take the leader run's beta_{i} at every step: the schedule of the
                              first run is reused by the others (Sec. 2.3, several runs), which
                              puts independent runs on common temperatures for
                              pa_weighted_average (Sec. 2.2) */
} pa_step_mode;

typedef struct {
    double beta_f;       /* final inverse temperature (> 0) */
    double dbeta;        /* fixed step size (PA_STEP_FIXED) */
    double alpha_star;   /* overlap target in (0,1) (adaptive and learned modes) */
    double alpha_tol;    /* learned mode: accept a proposal if |alpha - alpha_star| <= alpha_tol */
    int32_t theta;       /* sweeps per temperature step (>= 0) */
    int32_t mode;        /* pa_step_mode */
    int32_t leader;      /* PA_STEP_FOLLOW: index of the leading run in the batch, whose own
                            mode is not PA_STEP_FOLLOW; beta_f is then the leader's.  A
                            follower stops with PA_ESTATE once its leader has stopped on an
                            error.  Ignored in the other modes. */
} pa_schedule;

/* Single run: temperature steps of Sec. 2.1 from the current state until
 * beta_f or max_steps steps.  Each step takes the next inverse temperature
 * (PA_STEP_FIXED: beta_i = i * dbeta, the last one beta_f; PA_STEP_ADAPTIVE:
 * the rule of Sec. 2.3 as in pa_adapt_beta), resamples (Eq. (Q), Eq.
 * (resampling factors)), runs theta sweeps (Sec. 3) and measures (Eqs.
 * (observables), (free energy), (entropy)); with PA_FLAG_MHR the measurement
 * is recorded for pa_reweight.  The results are those of the same sequence
 * of single calls (pa_adapt_beta, pa_resample, pa_sweep, pa_observables), bit
 * for bit.  The device work of a step is queued before the host has seen the
 * new population size, which the kernels read on the device, so a step costs
 * one host round trip.
 *   out[k] (k < cap) receives the observables after step k (out may be NULL
 *   if cap is 0); *nsteps (may be NULL) the number of steps completed.
 *   sweep_ms (may be NULL, else cap floats): sweep_ms[k] receives the duration
 *   of step k's sweep launch, measured with HIP events on the run's stream.
 * Errors: PA_EINVAL (invalid schedule, PA_STEP_LEARNED, beta_f below the
 * current beta, no adaptive step reaching alpha_star, sweep counter
 * overflow); PA_ECAPACITY / PA_EEXTINCT (the run stays at the last completed
 * step); PA_ESTATE, PA_EHIP.  Synchronises the stream. */
pa_status pa_anneal(pa_run* r, const pa_schedule* s, int32_t max_steps, pa_obs* out, float* sweep_ms, int32_t cap,
                    int32_t* nsteps);

typedef struct pa_batch pa_batch;  /* opaque host handle */

/* Device workspace for nruns runs; 0 if any parameter set is invalid. */
size_t pa_batch_workspace_bytes(const pa_params* runs, int32_t nruns);

/* Start nruns runs at beta_0 = 0 (Sec. 2.1 step 1) and measure them once.
 * `hip_stream` may be NULL: the batch then creates its own stream (graph
 * capture needs a non-null stream).  The sweep's work-group shape (waves per
 * block, one per lattice size, store and update) is chosen by timing the
 * candidates 1, 2, 4 and 8 on the batch's spare buffers.  Errors: PA_EINVAL
 * (invalid run parameters or schedule, nruns < 1), PA_ENOMEM, PA_EHIP. */
pa_status pa_batch_init(const pa_params* runs, const pa_schedule* sched, int32_t nruns, void* d_workspace,
                        size_t bytes, void* hip_stream, pa_batch** out);

typedef struct {
    int32_t waves_per_block;  /* 0: timed choice as in pa_batch_init; 1, 2, 4 or 8: that shape for every
                                 group (a group whose LDS does not fit it takes the largest smaller
                                 shape that fits); results do not depend on the shape */
} pa_batch_options;

/* pa_batch_init with options (opt may be NULL: the defaults).  Errors as
 * pa_batch_init; PA_EINVAL also for a waves_per_block outside {0, 1, 2, 4, 8}. */
pa_status pa_batch_init_ex(const pa_params* runs, const pa_schedule* sched, int32_t nruns,
                           const pa_batch_options* opt, void* d_workspace, size_t bytes, void* hip_stream,
                           pa_batch** out);

/* Waves per block of the sweep launch that advances run `run`. */
pa_status pa_batch_waves_per_block(const pa_batch* b, int32_t run, int32_t* wpb);

/* pa_set_tie_queue_cap for every run of the batch, from the next step on. */
pa_status pa_batch_set_tie_queue_cap(pa_batch* b, int32_t cap);

/* One temperature step of every unfinished run.  *n_active (may be NULL)
 * receives the number of runs still below beta_f afterwards.  A run whose
 * step fails (capacity, extinction, no adaptive step) stops with its state
 * at the last good step; pa_batch_run_status reports why.  Errors:
 * PA_ESTATE, PA_EHIP. */
pa_status pa_batch_step(pa_batch* b, int32_t* n_active);

/* Steps until every run has reached beta_f or stopped. */
pa_status pa_batch_run(pa_batch* b);

/* Status of one run: PA_OK while running or finished, else the error that
 * stopped it (PA_ECAPACITY, PA_EEXTINCT, PA_EINVAL for a failed adaptive step). */
pa_status pa_batch_run_status(const pa_batch* b, int32_t run);

/* Counters of one run. */
pa_status pa_batch_state(const pa_batch* b, int32_t run, pa_state_info* out);

/* Observables of one run at every temperature so far (index 0 is beta_0 = 0):
 * copies min(cap, count) entries and stores the count in *n. */
pa_status pa_batch_history(const pa_batch* b, int32_t run, pa_obs* out, int32_t cap, int32_t* n);

/* Multi-histogram reweighting of one run (requires PA_FLAG_MHR on that run). */
pa_status pa_batch_reweight(pa_batch* b, int32_t run, const double* betas, int32_t nb, pa_obs* out);

/* Population of one run as int8 +-1 row-major spins and E, M (test hook). */
pa_status pa_batch_download_population(pa_batch* b, int32_t run, int8_t* spins, int32_t* E, int32_t* M);

/* Load the learned proposer used by PA_STEP_LEARNED runs: params[4801] FP32
 * MLP weights and norm[18] normalisation constants (layout below).  The batch
 * keeps a BF16 copy; inference runs on the device after every step. */
pa_status pa_batch_set_model(pa_batch* b, const float* params, const float* norm);

/* Training pairs logged by the bisection of adaptive (and learned-fallback)
 * steps of all runs: x[k][8] features, t[k] = ln((beta_{i+1} - beta_i) sigma_E)
 * with sigma_E the energy spread of the population (ln sigma_E = x[k][1]): the
 * overlap of Sec. 2.3 is a function of dbeta sigma_E to first order, so the
 * network learns the remaining dependence and the lattice-size scaling comes
 * from the feature.  Copies min(cap, count) pairs; *n receives the count. */
pa_status pa_batch_training_pairs(const pa_batch* b, float* x, float* t, int32_t cap, int32_t* n);

/* Features x[8] of one run's population after its last step, whether they are
 * valid, and the model's output made from them (test hook): the proposed step
 * is exp(prop - x[1]). */
pa_status pa_batch_features(const pa_batch* b, int32_t run, float* x, int32_t* valid, float* prop);

/* Cost of choosing one run's temperatures so far: the number of overlap
 * evaluations alpha(beta_i, beta') of Sec. 2.3 (a bisection makes 51 per step
 * unless beta_f is reached at once, an accepted learned proposal 1, a
 * rejected one 1 before its bisection) and the host seconds spent choosing
 * (fixed and follower runs: 0). */
pa_status pa_batch_choice_stats(const pa_batch* b, int32_t run, int64_t* alpha_evals, double* host_seconds);

/* Learned mode: proposals made and accepted by the exact overlap test. */
pa_status pa_batch_learned_stats(const pa_batch* b, int32_t run, int32_t* proposals, int32_t* accepted);

/* Release the batch handle (the caller frees the workspace). */
pa_status pa_batch_free(pa_batch* b);

/* ---- Learned temperature-step proposer -------------------------------------
 * A small MLP 8 -> 64 -> 64 -> 1 (ReLU) maps features of the population's
 * energy histogram to the natural log of the step size the overlap bisection
 * of Sec. 2.3 would choose.  Features: e/N, ln sigma_E, skewness, excess
 * kurtosis of the energy distribution, beta, ln L, ln R, ln(last step).
 * Parameters (FP32, 4801): W1[64][8] b1[64] W2[64][64] b2[64] w3[64] b3.
 * Normalisation (18): feature means[8], feature std devs[8], target mean, std.
 * Training: mean squared error on the normalised target, minibatch SGD with
 * momentum, all on the device with a deterministic gradient reduction. */
#define PA_MLP_PARAMS 4801
#define PA_MLP_NORM 18

typedef struct pa_mlp pa_mlp;

size_t pa_mlp_workspace_bytes(int32_t max_batch);

/* Network with He-initialised weights drawn from `seed` and identity
 * normalisation; max_batch bounds the minibatch and gradient sizes. */
pa_status pa_mlp_create(int32_t max_batch, uint64_t seed, void* d_workspace, size_t bytes, void* hip_stream,
                        pa_mlp** out);
pa_status pa_mlp_set_params(pa_mlp* m, const float* params, const float* norm);  /* host arrays; either may be NULL */
pa_status pa_mlp_get_params(pa_mlp* m, float* params, float* norm);
/* Normalisation from n raw samples (device arrays x[n][8], t[n]). */
pa_status pa_mlp_fit_norm(pa_mlp* m, const float* d_x, const float* d_t, int32_t n);
/* y[k] = network(x[k]) for n raw feature vectors (device arrays), de-normalised;
 * bf16 != 0 uses the BF16 inference path, else the FP32 master weights. */
pa_status pa_mlp_forward(pa_mlp* m, const float* d_x, int32_t n, float* d_y, int32_t bf16);
/* Gradient (host grad[4801]) and loss of the n <= max_batch samples. */
pa_status pa_mlp_gradient(pa_mlp* m, const float* d_x, const float* d_t, int32_t n, float* grad, float* loss);
/* `epochs` passes of minibatch SGD (shuffled with `seed`, full minibatches of
 * `batch` samples); epoch_loss[epochs] (may be NULL) receives the mean loss. */
pa_status pa_mlp_train(pa_mlp* m, const float* d_x, const float* d_t, int32_t n, int32_t batch, int32_t epochs,
                       float lr, float momentum, uint64_t seed, float* epoch_loss);
const char* pa_mlp_last_error(const pa_mlp* m);
pa_status pa_mlp_free(pa_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
