/*
 * pa.h -- C ABI of the population-annealing (PA) hot path on MI355X (gfx950).
 *
 * The calls follow the enumerated algorithm of Sec. 2 of "Optimized population
 * Monte Carlo" (Ebert, Gessert, Janke, Weigel):
 *
 *   pa_init        step 1: R replicas drawn exactly at beta_0 = 0
 *   pa_reweight    step 2: Q(beta_{i-1}, beta_i) of Eq. (1) for the next beta
 *   pa_resample    step 2 + Sec. 3: copy numbers with <r_j> = tau_j (Eq. (3))
 *                  and the new population; beta_i becomes current
 *   pa_sweep       step 3: theta Metropolis sweeps at the current beta
 *   pa_observables step 4: plain population averages, family statistics
 *                  (Eq. (6)) and the sampling variance (Eq. (5))
 *   pa_free_energy ln Z_hat = ln Z_{beta_0} + sum_k ln Q_k, Eq. (7)
 *   pa_resample_conditional
 *                  Sec. 3 remark: resample only when the weights' variance is
 *                  large; otherwise keep the population with importance weights
 *
 * Conventions (every call):
 *  - The return value is a pa_status; nothing aborts or throws across the ABI.
 *    On any status other than PA_OK, pa_last_error(ctx) holds a message.
 *  - Arguments are checked before any launch.  A failed call leaves the run's
 *    state as it was (PA_E_CAPACITY and PA_E_EXTINCT included).
 *  - Device memory is owned by the caller: pa_init receives one device buffer
 *    of pa_required_bytes() bytes and a hipStream_t; every kernel of the run
 *    goes to that stream.  The context owns only host memory (pa_destroy).
 *  - A context is not thread-safe; distinct contexts may run concurrently on
 *    distinct streams.  Calls that return results to the host (pa_reweight,
 *    pa_resample, pa_resample_conditional, pa_observables, pa_free_energy,
 *    pa_export_state, pa_log_weights) synchronise the stream; pa_sweep only
 *    enqueues.
 *  - Deferred calls: pa_reweight, pa_resample, pa_resample_conditional and
 *    pa_observables given NULL result pointers only enqueue their kernels and
 *    return at once, so that a whole temperature step runs without waiting
 *    for the device (and can be captured into a HIP graph).  A failure
 *    that pa_resample would report (PA_E_CAPACITY, PA_E_EXTINCT,
 *    PA_E_NONFINITE) then freezes the run instead: its population stays as it
 *    was before that resampling, every later kernel of the run does nothing,
 *    and every later call that synchronises returns that error.
 *    pa_export_state still reads the frozen population; pa_import_state
 *    replaces it and lifts the freeze.
 *
 * Spin layout in device memory (and in pa_host_state): replica r = 64 w + b is
 * bit b of word [w][s] (uint64, site-minor: word index w * N + s).  Bit 1 means
 * sigma = -1.  Sites s = x + L y + L^2 z of the periodic hypercubic lattice.
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
    PA_E_INVAL = 1,     /* bad argument (shape, range, NULL, too small a buffer) */
    PA_E_NOMEM = 2,     /* host allocation failed */
    PA_E_STATE = 3,     /* call out of order, e.g. pa_resample before pa_reweight */
    PA_E_CAPACITY = 4,  /* resampled population would exceed the capacity */
    PA_E_EXTINCT = 5,   /* resampled population would be empty */
    PA_E_NONFINITE = 6, /* ln Q is not finite */
    PA_E_DEVICE = 7     /* a HIP call failed; the run should be destroyed */
} pa_status;

/* Sec. 3: the four schemes.  Multinomial and systematic keep R fixed (Fig. 2);
 * Poisson and nearest integer let it fluctuate around the target R. */
typedef enum {
    PA_RS_MULTINOMIAL = 0,
    PA_RS_POISSON = 1,
    PA_RS_NEAREST_INT = 2,
    PA_RS_SYSTEMATIC = 3
} pa_resampler;

typedef struct {
    int32_t dim;       /* 2 or 3 */
    int32_t L;         /* even, >= 2; N = L^dim <= 16384 */
    int64_t R;         /* target population size, >= 1 */
    int64_t capacity;  /* max replicas after a resampling (>= R, <= 2^24 - 64);
                          0 = R + 8 ceil(sqrt R) + 64 rounded up to 64 */
    uint32_t seed;     /* Philox key word 0 */
    uint32_t run_id;   /* Philox key word 1: independent runs differ here */
    /* Bond couplings J(s, mu) in {+1, -1} of H = -sum J sigma_s sigma_{s+e_mu}
       (Eq. (4); a +-J Edwards-Anderson sample when random), host memory,
       int8[N * dim] at index s * dim + mu.  NULL = ferromagnet (all +1).
       Copied during pa_init; the caller keeps ownership. */
    const int8_t *couplings;
} pa_config;

/* Population averages after the latest step (Sec. 2, step 4). */
typedef struct {
    int64_t R;            /* replicas in the population, R_i */
    double beta;          /* current inverse temperature */
    int64_t sum_E;        /* exact sums over replicas */
    int64_t sum_E2;
    int64_t sum_absM;     /* M = sum_s sigma_s */
    int64_t sum_M2;
    int64_t sum_c2;       /* sum over families of (family size)^2 */
    int64_t families;     /* families with at least one member */
    double e, e2;         /* <E>/N, <E^2>/N^2 */
    double abs_m, m2;     /* <|M|>/N, <M^2>/N^2 */
    double rho_t;         /* Eq. (6): R sum_k n_k^2 = sum_k c_k^2 / R_i */
    double S_f;           /* family entropy -sum_k n_k ln n_k */
    double sv;            /* Eq. (5) of the latest resampling, over R_{i-1} */
    int64_t sum_E3_hi;    /* sum of E^3 over replicas, exact: the signed 128-bit */
    uint64_t sum_E3_lo;   /*   integer sum_E3_hi * 2^64 + sum_E3_lo */
    double e3;            /* <E^3>/N^3 */
    double ess;           /* (sum w)^2 / sum w^2 of the importance weights (R if uniform) */
    int32_t weighted;     /* 1: the population carries importance weights (a step
                             kept it, pa_resample_conditional); e, e2, e3, abs_m
                             and m2 are then the weighted averages
                             sum_j w_j O_j / sum_j w_j, w_j = exp(lw_j), while
                             the sums, rho_t, S_f and families stay those of the
                             members */
    int32_t pad;
} pa_obs;

/* Host copy of a run's state (pa_export_state / pa_import_state).  Array
 * pointers may be NULL to skip them; non-NULL arrays must hold R entries
 * (spins: ceil(R/64) * N words).  Memory is the caller's.  The importance
 * weights of a kept population are not part of it (pa_log_weights reads
 * them); an imported population is uniform. */
typedef struct {
    int64_t R;
    uint32_t step;        /* temperature index i */
    uint32_t sweeps;      /* sweeps done at step i */
    double beta;
    double lnZ;
    uint64_t *spins;
    int32_t *energy;
    int32_t *magnetization;
    uint32_t *label;      /* family: index of the ancestor at beta_0 */
} pa_host_state;

/* Work counters of a run since pa_init (for throughput accounting). */
typedef struct {
    uint64_t philox_calls;  /* Philox4x32-10 evaluations the sweeps needed: per
                               64-replica word and site visit, plane pairs until
                               every replica's u < T is decided */
    uint64_t site_updates;  /* 64-replica word-site updates (64 attempts each,
                               dead replicas of the last word included) */
    uint64_t sweeps;        /* sweeps over all sites, summed over pa_sweep calls */
    uint64_t spin_attempts; /* Metropolis attempts: theta N R_i summed over pa_sweep
                               calls (R_i the population at the call) */
    uint64_t resamplings;   /* resamplings applied (a kept step is not one) */
} pa_counters;

typedef struct pa_ctx pa_ctx;

/* Device bytes a run of this configuration needs (pa_init's workspace).
 * PA_E_INVAL if the configuration is invalid. */
pa_status pa_required_bytes(const pa_config *cfg, uint64_t *bytes);

/* Step 1 of Sec. 2 at beta_0 = 0: exact sampling, R i.i.d. uniform spin states
 * (replica r = 64w+b takes bit b of Philox4x32-10 with counter (s, w, 0, 1<<28)
 * under key (seed, run_id) at site s); energies, magnetisations, family labels
 * f_j = j; ln Z_0 = N ln 2.  workspace: device pointer, >= pa_required_bytes,
 * 256-byte aligned.  stream: a hipStream_t (NULL = default stream). */
pa_status pa_init(const pa_config *cfg, void *workspace, uint64_t workspace_bytes,
                  void *stream, pa_ctx **out);

/* Step 3 of Sec. 2: theta >= 0 Metropolis sweeps at the current beta (each
 * sweep: sites with x+y+z even, then odd).  A flip raising the energy by dE is
 * taken iff the replica's 32-bit uniform u < min(2^32, floor(2^32 exp(-beta dE))),
 * u's bit 31-k being bit b of plane k of Philox counters
 * (s, w, i, 2<<28 | t<<8 | q), q = k/2, t = the sweep index within step i. */
pa_status pa_sweep(pa_ctx *ctx, int32_t theta);

/* Step 3 of Sec. 2 with cluster updates as the driver (Sec. 1 names them
 * among the update algorithms the scheme can use): nsteps >= 0 Wolff
 * single-cluster updates of every replica at the current beta.  Replica
 * r = 64w+b seeds its cluster at site floor(x0 N / 2^32), x0 of Philox
 * counter (b, w, i, 8<<28 | t<<8); a bond (s, mu) joins the cluster iff it
 * is satisfied (J sigma_s sigma_{s+e_mu} = +1) and the replica's uniform
 * u < min(2^32, floor(2^32 (1 - exp(-2 beta)))), u's bit 31-k being bit b of
 * plane k of counters (s, w, i, 9<<28 | t<<8 | mu<<4 | q), q = k/2; the whole
 * cluster flips.  t counts sweeps and cluster updates together within step i
 * (at most 2^20).  Energies and magnetisations are recounted afterwards.
 * PA_E_INVAL if nsteps < 0, if the step's updates would pass 2^20, or if a
 * lattice needs more LDS per workgroup than the device has (4 N 8 bytes and
 * 24 KiB of queues, plus N with couplings: N <= 4352, or 4220 with
 * couplings, on 160 KiB).  Enqueued on the run's stream. */
pa_status pa_cluster(pa_ctx *ctx, int32_t nsteps);

/* Step 2 of Sec. 2: for beta_next >= beta, ln Q of Eq. (1) over the current
 * population, written as -dbeta E_min + ln((1/R) sum_j exp(-dbeta (E_j - E_min))).
 * Also fixes the integer resampling weights floor(2^40 exp(-dbeta (E_j - E_min))).
 * A weighted population (log-weights lw_j <= 0, largest 0, left by
 * pa_resample_conditional) uses x_j = lw_j + (-(dbeta (E_j - E_min))) and
 * m = min_j |x_j|: W_j = floor(2^40 exp(x_j + m)) and
 * ln Q = -dbeta E_min - m + ln sum_j exp(x_j + m) - ln sum_j exp(lw_j)
 * (every operation IEEE-754 rounded on its own; exp is the library's own).
 * The population is unchanged; a second call replaces the first.
 * lnQ_out NULL: deferred (see the conventions above). */
pa_status pa_reweight(pa_ctx *ctx, double beta_next, double *lnQ_out);

/* Step 2 of Sec. 2 with a scheme of Sec. 3: copy numbers r_j with
 * <r_j> = tauhat_j = R W_j / S (Eq. (3), R the target size), the new
 * population (r_j copies of replica j, in ascending j; spins, energies,
 * magnetisations and labels copied), then beta := beta_next, i := i + 1,
 * ln Z_hat += ln Q.  Needs a pa_reweight first.  R_new_out NULL: deferred
 * (a failure freezes the run, see the conventions above). */
pa_status pa_resample(pa_ctx *ctx, pa_resampler scheme, int64_t *R_new_out);

/* Conditional resampling (Sec. 3: resampling need not happen at every step;
 * population control once the variance of the importance weights is too large
 * can be enough).  After pa_reweight, with the step's integer weights W_j:
 *   ESS = S^2 / sum_j W_j^2 < kappa R_i  ->  resample exactly as pa_resample;
 *   otherwise keep the population: every member stays, replica j's log-weight
 *   becomes lw_j := x_j + m (see pa_reweight), and beta := beta_next,
 *   i := i + 1, ln Z_hat += ln Q as after a resampling, SV := 0.
 * kappa in [0, 1] counts in units of 2^-16 (kq = floor(kappa 2^16 + 1/2)); the
 * test is exact: 2^16 S^2 < kq R_i sum_j W_j^2.  kappa = 0 never resamples,
 * kappa = 1 resamples unless all weights are equal.  A resampled population is
 * uniform again.  Outputs: R_new_out (population after the step), resampled_out
 * (1 resampled, 0 kept); both NULL: deferred (a failure freezes the run, see the
 * conventions above).  Failures as pa_resample (PA_E_NONFINITE also when kept). */
pa_status pa_resample_conditional(pa_ctx *ctx, pa_resampler scheme, double kappa, int64_t *R_new_out,
                                  int32_t *resampled_out);

/* Importance log-weights of the current population: out (host, double[R_i])
 * gets lw_j (all 0 for a uniform population); weighted_out (optional) 1 if a
 * kept step left weights.  Synchronises the stream. */
pa_status pa_log_weights(pa_ctx *ctx, double *out, int32_t *weighted_out);

/* Step 4 of Sec. 2 over the current population.  out NULL: deferred (the
 * averages are still computed on the device, e.g. for pa_features).  For a
 * weighted population see pa_obs.weighted. */
pa_status pa_observables(pa_ctx *ctx, pa_obs *out);

/* -beta_i F_hat_i = ln Z_{beta_0} + sum_{k<=i} ln Q_k (Eq. (7)). */
pa_status pa_free_energy(pa_ctx *ctx, double *lnZ_out);

/* Copies the state to the host (arrays optional, see pa_host_state). */
pa_status pa_export_state(pa_ctx *ctx, pa_host_state *st);

/* Replaces the population (1 <= st->R <= capacity; spins, energy,
 * magnetization and label all required) and the scalars step, sweeps, beta,
 * lnZ.  Energies and magnetisations are taken as given. */
pa_status pa_import_state(pa_ctx *ctx, const pa_host_state *st);

/* Overlap distribution between two runs of the same lattice: replica d of a
 * paired with replica d of b, d < min(R_a, R_b); q = (N - 2 popcount(a ^ b)) / N.
 * hist_out: host, int64[N + 1], entry k counts pairs with N - 2 popcount = 2k - N
 * (i.e. k = N - popcount). */
pa_status pa_overlap(pa_ctx *a, pa_ctx *b, int64_t *hist_out);

/* pa_overlap without workspace scratch, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same histogram, accumulated in the library's
 * file-scope device array of 16385 counters (128 KiB per device, held until
 * the process ends) instead of run a's workspace.  It allocates nothing and
 * calls no allocating routine; hist_out (host, int64[N + 1]) is written
 * directly.  PA_E_INVAL if N + 1 > 16385 or the lattices differ.  Every
 * call on a device shares that device's array (each call clears the N + 1
 * counters it uses), so calls that overlap on one device race: issue them one
 * at a time.  Synchronises both runs' streams. */
pa_status pa_overlap_noalloc(pa_ctx *a, pa_ctx *b, int64_t *hist_out);

/* Throughput probe of the generator the sweeps draw from (no step of the
 * method): each of nthreads threads (a multiple of 256, <= 2^24) evaluates
 * 3 * iters Philox4x32-10 calls as three independent chains (the sweep's
 * first plane pairs) and writes the xor of all outputs to out[thread]
 * (device memory, uint32[nthreads], caller-owned).  Enqueued on `stream`;
 * returns without waiting.  Timing it gives the device's Philox rate, the
 * ceiling of any sweep that decides u < T from these bits. */
pa_status pa_philox_probe(void *out, int64_t nthreads, int32_t iters, void *stream);

/* Adaptive temperature steps (Sec. 5 names them; the rule is a reading):
 * overlap of the current population with its reweighting by dbeta,
 *   alpha(dbeta) = (1/R) sum_j min(1, tauhat_j),  tauhat_j = R W_j / S,
 * with the integer resampling weights W_j = floor(2^40 exp(-dbeta (E_j - E_min)))
 * and S = sum_j W_j (tau of Eq. (1) as the resampling uses it), i.e. one minus
 * the total-variation distance between the population and its reweighted
 * version; alpha(0) = 1.  Evaluated exactly as sum_j min(S, R W_j) / (R S).
 * Synchronises the stream. */
pa_status pa_step_alpha(pa_ctx *ctx, double dbeta, double *alpha_out);

/* Largest dbeta in [0, dbeta_max] with alpha(dbeta) >= alpha_star: dbeta_max
 * itself if it qualifies, else `iterations` halvings of [0, dbeta_max]
 * keeping the lower end qualified (0 < alpha_star < 1, 1 <= iterations <= 200).
 * alpha_star counts to 2^-32 (A = nearest integer to 2^32 alpha_star, ties to
 * even; qualifies iff 2^32 sum_j min(S, R W_j) >= A R S, exact).
 * The population is unchanged; pass beta + dbeta to pa_reweight.
 * The rule (and pa_step_alpha, pa_features, pa_step_learned) needs a uniform
 * population: PA_E_STATE after a kept step until the next resampling. */
pa_status pa_step_rule(pa_ctx *ctx, double alpha_star, double dbeta_max, int32_t iterations,
                       double *dbeta_out);

/* Work counters since pa_init; synchronises the stream. */
pa_status pa_get_counters(pa_ctx *ctx, pa_counters *out);

/* Releases the context's host memory (not the caller's workspace). */
void pa_destroy(pa_ctx *ctx);

/* Message of the latest failed call on ctx (or of the latest failed pa_init
 * when ctx is NULL).  Valid until the next call on ctx. */
const char *pa_last_error(const pa_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Batches: many independent runs (own lattice shape, R, couplings, seeds)
 * annealed together on one stream.  Every kernel serves all runs of the batch
 * at once; run state stays on the device, so an anneal needs no host round
 * trip and can be captured whole in one HIP graph.  A batch gives the same
 * bits as running each of its runs alone through the calls above.
 * ------------------------------------------------------------------------- */
typedef struct pa_batch pa_batch;

/* One row per run and temperature point of a batched anneal (Sec. 2 step 4
 * and Eq. (7) at beta_i). */
typedef struct {
    double beta, lnQ, lnZ, sv, e, e2, abs_m, m2, rho_t, S_f;
    int64_t R, sum_E, sum_E2, sum_absM, sum_M2, sum_c2, families;
    uint32_t status;      /* bit 1 capacity, 2 extinct, 3 non-finite, 4 frozen */
    uint32_t pad;
} pa_step_record;

/* Free-energy-weighted combination of the runs of one group (Sec. 4,
 * Eqs. (9)-(12)). */
typedef struct {
    double lnZ;          /* ln of the pooled Z estimate: ln(sum_m R_m Z_m / sum_m R_m) */
    double e, e2, abs_m, m2; /* W[O] = sum_m omega_m O_m, omega of Eq. (10) */
    double c;            /* W_var of the specific heat, Eq. (11) */
    double chi;          /* W_var of the susceptibility, Eq. (12), with |m| */
    double n_eff;        /* 1 / sum_m omega_m^2 */
    double beta;
    /* for comparison (Fig. 5 left, Fig. 8): the naive weighted averages
       sum_m omega_m c_m, sum_m omega_m chi_m of each run's own c_m, chi_m, and
       the plain means over the runs of e, c_m and chi_m */
    double c_naive, chi_naive, e_plain, c_plain, chi_plain;
    int32_t runs, pad;
} pa_combined;

/* Device bytes for a batch of nruns configurations (each as for pa_init) whose
 * anneals have at most max_points temperature points. */
pa_status pa_batch_required_bytes(const pa_config *cfgs, int32_t nruns, int32_t max_points,
                                  uint64_t *bytes);

/* Lays out the batch in the caller's workspace (256-byte aligned) and draws
 * every run's initial population (step 1 of Sec. 2).  Runs are grouped by
 * (dim, L, couplings given or NULL); at most 16 groups. */
pa_status pa_batch_create(const pa_config *cfgs, int32_t nruns, int32_t max_points, void *workspace,
                          uint64_t workspace_bytes, void *stream, pa_batch **out);

/* Autotuner: times the sweep workgroup size (64..768 lanes in steps of 64,
 * where the lattice allows) per group with theta sweeps of the current
 * populations under the Metropolis thresholds of `beta` (a temperature of the
 * coming anneal: the cost of a sweep depends on the thresholds), keeps the
 * fastest and re-draws the initial populations.  Results do not depend on
 * the choice.  threads_out (optional): one entry per group.  ms_out
 * (optional): float[ngroups * 12], entry [g * 12 + t/64 - 1] the time of
 * workgroup size t for group g in ms, -1 where t is not usable.
 * PA_E_INVAL unless 1 <= theta <= 64 and beta >= 0 is finite. */
pa_status pa_batch_tune(pa_batch *b, int32_t theta, double beta, int32_t *threads_out, float *ms_out);

/* Sets group `group`'s sweep workgroup size (as pa_batch_tune would) to
 * `threads`: 64..768 in steps of 64, within the device's LDS and at most 255
 * bonds per lane (PA_E_INVAL otherwise). */
pa_status pa_batch_set_threads(pa_batch *b, int32_t group, int32_t threads);

/* Groups of the batch (see pa_batch_create) and their sweep workgroup sizes. */
pa_status pa_batch_groups(pa_batch *b, int32_t *ngroups, int32_t *threads);

/* A whole anneal of every run from a fresh initial population: betas[0] = 0,
 * then for i >= 1 reweight to betas[i], resample with `scheme`, theta sweeps,
 * observables into the records.  A run whose resampling fails (capacity,
 * extinction) is frozen at its last good step (status bits in its records).
 * use_graph != 0 captures the anneal in one HIP graph, instantiates it and
 * launches it; the batch keeps the instantiated graph, and a later call with
 * the same betas, theta and scheme (and unchanged workgroup sizes) replays it
 * without capturing again.  Any other use_graph call replaces the kept graph;
 * pa_batch_destroy releases it.  Synchronises the stream. */
pa_status pa_batch_anneal(pa_batch *b, const double *betas, int32_t npoints, int32_t theta,
                          pa_resampler scheme, int32_t use_graph);

/* Records of the last anneal: out[run * npoints + i]. */
pa_status pa_batch_records(pa_batch *b, pa_step_record *out);

/* Final state of one run (as pa_export_state). */
pa_status pa_batch_export_run(pa_batch *b, int32_t run, pa_host_state *st);

/* Overlap distribution (Figs. 6-7) between runs run_a and run_b of the batch,
 * in their current state (after pa_batch_anneal: at its last point), exactly
 * as pa_overlap: replica d of run_a paired with replica d of run_b,
 * d < min(R_a, R_b); hist_out (host, int64[N + 1]) entry k counts pairs with
 * N - popcount(a ^ b) = k.  The two runs must share dim and L (PA_E_INVAL
 * otherwise).  Uses run_a's overlap buffer; synchronises the stream. */
pa_status pa_batch_overlap(pa_batch *b, int32_t run_a, int32_t run_b, int64_t *hist_out);

/* Eqs. (9)-(10) at temperature point `point` of the last anneal: runs m with
 * group_of_run[m] = g (-1: none) are combined into out[g], g < ngroups;
 * frozen runs are left out. */
pa_status pa_batch_combine(pa_batch *b, const int32_t *group_of_run, int32_t ngroups, int32_t point,
                           pa_combined *out);

void pa_batch_destroy(pa_batch *b);
const char *pa_batch_last_error(const pa_batch *b);

/* ---------------------------------------------------------------------------
 * Learned temperature steps (not in the paper; the overlap rule above stays
 * the arbiter and the fallback).  A network 8 -> 64 -> 64 -> 1 with tanh hidden
 * layers maps population statistics to a proposed ln(dbeta):
 *   inputs  beta, <E>/N, sd(E)/sqrt(N), skewness of E, the last three ln Q
 *           (Eq. (1)) divided by N, family entropy / ln R;
 *   params  one float vector of PA_MLP_PARAMS: W1[64][8], b1[64], W2[64][64],
 *           b2[64], W3[64], b3, acting on standardised inputs and target.
 * Training runs on the GPU in float32 (loss (1/2n) sum (y_hat - y)^2, Adam
 * with beta1 = 0.9, beta2 = 0.999, eps = 1e-8); inference in bfloat16.
 * ------------------------------------------------------------------------- */
#define PA_MLP_PARAMS 4801

typedef struct {
    float x_mean[8], x_std[8]; /* input standardisation: (x - mean) / std */
    float y_mean, y_std;       /* target ln(dbeta) standardisation */
} pa_mlp_norm;

typedef struct pa_mlp pa_mlp;

pa_status pa_mlp_required_bytes(int32_t max_samples, uint64_t *bytes);
/* params: PA_MLP_PARAMS floats (host, copied). */
pa_status pa_mlp_create(int32_t max_samples, const float *params, const pa_mlp_norm *norm,
                        void *workspace, uint64_t workspace_bytes, void *stream, pa_mlp **out);
/* Training set: X [n][8] raw inputs, y [n] raw targets ln(dbeta) (host, copied). */
pa_status pa_mlp_set_data(pa_mlp *m, const float *X, const float *y, int32_t n);
/* Gradient of the loss at the current parameters (float32, PA_MLP_PARAMS). */
pa_status pa_mlp_gradient(pa_mlp *m, float *grad_out, double *loss_out);
/* `epochs` full-batch Adam steps with learning rate lr; loss after them. */
pa_status pa_mlp_train(pa_mlp *m, int32_t epochs, float lr, double *loss_out);
pa_status pa_mlp_params(pa_mlp *m, float *out);
/* bfloat16 inference: dbeta_out[i] = exp(ln dbeta predicted for X[i]).  Uses
 * the training-data slot; set the data again before training further. */
pa_status pa_mlp_predict(pa_mlp *m, const float *X, int32_t n, float *dbeta_out);
/* The model inputs of the current population (uses the family entropy of
 * the latest pa_observables). */
pa_status pa_features(pa_ctx *ctx, float *out8);
/* Learned step: the model's proposal c = min(prediction, dbeta_max) is kept
 * only where alpha(c) >= alpha_star (exact check as in pa_step_rule).
 * refine = 0: c itself if it qualifies.  refine > 0 (bracket > 1): the
 * proposal seeds a short exact search instead: if c qualifies, the top of
 * [c, min(bracket c, dbeta_max)] if that qualifies, else that bracket halved
 * `refine` times keeping the lower end qualified; if c does not qualify but
 * c / bracket does, [c / bracket, c] halved `refine` times.  Where none of
 * this applies (c <= 0, or neither end qualifies) pa_step_rule's bisection
 * over [0, dbeta_max] with `iterations` halvings decides and
 * *fallback_out = 1.  Every step returned has alpha >= alpha_star.
 * 1 <= iterations <= 200, 0 <= refine <= 64, bracket >= 1.
 * proposal_out (optional): c.  Synchronises the stream. */
pa_status pa_step_learned(pa_ctx *ctx, pa_mlp *m, double alpha_star, double dbeta_max, int32_t iterations,
                          double bracket, int32_t refine, double *dbeta_out, int32_t *fallback_out,
                          double *proposal_out);
void pa_mlp_destroy(pa_mlp *m);
const char *pa_mlp_last_error(const pa_mlp *m);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
