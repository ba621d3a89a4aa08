// Internal interface between the host side (pa_api.cpp) and the kernels
// (pa_kernels.hip).  Not part of the public C ABI.
//
// Every kernel works on a batch of independent runs: the run a workgroup
// serves comes from a per-launch block map in device memory, and each run's
// state (population size, ping-pong index, temperature, step) lives in its
// device record, so a whole anneal of many runs needs no host round trip and
// can be captured in one HIP graph.  A single run is a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Status bits of a run (PaRecord::status).
#define PA_ST_SCAN_TIMEOUT 1u
#define PA_ST_CAPACITY 2u
#define PA_ST_EXTINCT 4u
#define PA_ST_NONFINITE 8u
#define PA_ST_FROZEN 16u // batch mode: a failed step froze the run

// Per-run scalars that live in device memory, written by the kernels.
struct PaRecord {
    int32_t cur;      // ping-pong buffer holding the population
    uint32_t status;  // PA_ST_* bits of the latest resampling (sticky when frozen)
    uint32_t skip;    // latest resampling was not applied
    uint32_t step;    // temperature index i
    uint32_t sweeps;  // sweeps done at step i
    uint32_t gather;  // 1: the latest resampling's spins are still to be gathered from the other buffer
    uint64_t Rcur;    // replicas in the population
    double beta;      // current inverse temperature
    // histogram of the current population (reweight, adaptive step)
    int32_t emin, emax;
    int32_t wemin, pad2; // E_min of the latest reweighting (its weights are per level above it)
    // Q(beta_cur, beta_next): Eq. (1) with the shift by E_min
    double qsum, lnQ, dbeta, beta_next;
    uint64_t S;     // sum of integer weights
    uint64_t Tn[3]; // Metropolis thresholds at beta_next for dE = 4, 8, 12
    uint64_t T[3];  // thresholds at the current beta (used by the sweeps)
    // resampling
    uint64_t Rprev;
    unsigned long long Rnew, Ctot;
    double sv;
    double lnZ; // ln Z_0 + sum_k ln Q_k, Eq. (7)
    // observables (exact integer sums, then the finalised averages)
    unsigned long long sumE, sumE2, sumAbsM, sumM2, sumC2, families;
    // accumulators of the observables pass; k_obs_final publishes them into
    // the sums above and returns them to zero for the next pass
    unsigned long long accE, accE2, accAbsM, accM2, accC2, accFam;
    // sum of E^3 as a signed 128-bit integer (two's complement, low word first)
    unsigned long long sumE3[2], accE3[2];
    double e3;
    double sumClnC;
    double e, e2, abs_m, m2, rho_t, S_f;
    double rule_dbeta, rule_alpha; // adaptive step: chosen dbeta and its overlap
    double lnq_hist[3];            // ln Q of the last three applied steps, oldest first
    float feat[8];                 // inputs of the learned step model
    double cand_dbeta;             // the model's proposal
    uint32_t fallback, pad1;       // 1: the proposal failed the overlap check
    unsigned long long philox_calls; // Philox4x32-10 evaluations of all sweeps so far
    unsigned long long site_updates; // word-site updates (64 attempts each) so far
    unsigned long long attempts;     // spin-flip attempts so far: theta N R per sweep call
    uint32_t ticket[2];              // tile tickets of the two prefix sums of a resampling
    // Weighted populations (conditional resampling): after a step that kept
    // its population, replica j carries the log-weight lw[j] <= 0 (largest 0).
    uint32_t weighted;              // 1: lw holds the population's log-weights; 0: uniform
    uint32_t keep;                  // the latest conditional resampling kept the population
    unsigned long long xmag;        // min_j |x_j| as IEEE bits, x_j = lw_j - dbeta (E_j - E_min) <= 0
    unsigned long long Q2[2];       // sum_j W_j^2 of the step's integer weights, 128-bit, low word first
    unsigned long long resamplings; // resamplings applied so far
    double ess;                     // (sum w)^2 / sum w^2 of the population's weights (observables)
};

// One row per run and temperature point of a batched anneal.
struct PaStepRecord {
    double beta, lnQ, lnZ, sv, e, e2, abs_m, m2, rho_t, S_f;
    long long R, sumE, sumE2, sumAbsM, sumM2, sumC2, families;
    uint32_t status, pad;
};

// Published state of a scan tile in one 64-bit word, so that a single atomic
// store makes the status and its value visible together: bits 63..62 are the
// status (0 none, 1 aggregate, 2 inclusive prefix), bits 61..0 the value.
struct PaScanTile {
    unsigned long long word;
};
#define PA_TILE_AGG (1ull << 62)
#define PA_TILE_INCL (2ull << 62)
#define PA_TILE_VALUE ((1ull << 62) - 1ull)

#define PA_SCAN_THREADS 512
#define PA_SCAN_ITEMS 16
#define PA_SCAN_TILE (PA_SCAN_THREADS * PA_SCAN_ITEMS)
#define PA_CHUNK 1024  // replicas (or families) per workgroup of the per-replica kernels
#define PA_HCHUNK 4096 // replicas per workgroup of the energy histogram (LDS-private counts)

// Tile flags of a run's two prefix sums of a resampling (weights, copy
// numbers): ceil(cap / PA_CHUNK) each, enough for tiles of PA_CHUNK or more
// slots.
__host__ __device__ inline int64_t pa_tiles_per_sum(int64_t cap) { return (cap + PA_CHUNK - 1) / PA_CHUNK; }

// Replica slots per tile of the passes that sum the weights or draw and sum
// nearest-integer or Poisson copy numbers: 4 per thread of 256, or 16 per
// thread once the run is large enough that the look-back over the smaller
// tiles would take longer than the work.  A run's tiles depend on its
// capacity alone, so a run's results do not depend on the batch it is in.
#define PA_COUNTS_WIDE_CAP (1 << 18)
__host__ __device__ inline int64_t pa_counts_tile(int64_t cap) { return cap >= PA_COUNTS_WIDE_CAP ? 4096 : 1024; }

// Device buffers of one run, carved from the caller's workspace.
struct PaDev {
    uint64_t *spins[2]; // [W][N] words, bit b of word (w, s) = replica 64w+b at site s
    int32_t *E[2], *M[2];
    uint32_t *label[2];
    uint8_t *jmask; // per site: bit mu = J(s,mu) is -1, bit d+mu = J(s-e_mu,mu) is -1
    uint32_t *hist; // [H] replicas per energy level h = (E + dN) / 4
    uint64_t *wtab; // [H] integer weight per level above the lowest
    uint32_t *r, *anc;
    uint64_t *C;
    unsigned long long *qhist; // [N+1] overlap histogram
    PaScanTile *tiles;
    double *partial; // fixed-order partial sums, one per chunk
    uint32_t *fam;   // [R0] replicas per family
    double *lw;      // [slots] log-weights of a weighted population
    uint64_t *Wj;    // [slots] integer weights of a weighted population's reweighting
    double *wpart;   // [PA_WPARTS][chunks] fixed-order partial sums of the weighted passes
    PaRecord *rec;
};

#define PA_WPARTS 7 // weighted partial sums per chunk: w, wE, wE^2, wE^3, w|M|, wM^2, w^2

struct PaRunDesc {
    int d, L, N, H;
    uint32_t seed, run_id;
    int64_t R0, cap;
    PaDev dv;
};

// Block map entry: the run a workgroup serves and its index within the run.
struct PaBlk {
    uint32_t run, idx;
};

#define PA_MAX_GROUPS 16
#define PA_COMBINE_FIELDS 15 // doubles per group written by the combination kernel

// Learned temperature-step model: 8 -> 64 -> 64 -> 1.
#define PA_MLP_HIDDEN 64
#ifndef PA_MLP_PARAMS
#define PA_MLP_PARAMS 4801 // 64*8 + 64 + 64*64 + 64 + 64 + 1
#endif

struct PaMlpNorm {
    float x_mean[8], x_std[8];
    float y_mean, y_std;
};

struct PaMlpDev {
    float *P, *M, *V, *G;   // parameters, Adam moments, last gradient
    PaMlpNorm *norm;
    float *X, *Y;           // training data [n][8], [n]
    float *Xn, *H1, *H2, *D1, *D2, *dY, *r2; // per-sample work
    double *loss;
    float *pred;            // predictions [n]
    hipStream_t stream;
};

// What the launchers need to address a batch (device pointers + counts).
struct PaBatchView {
    const PaRunDesc *runs; // [nruns]
    uint32_t nruns;
    const PaBlk *rep;  // chunks of PA_CHUNK replica slots (capacity)
    uint32_t nrep;
    const PaBlk *hrep; // chunks of PA_HCHUNK replica slots (histogram)
    uint32_t nhrep;
    const PaBlk *crep; // tiles of the copy-number pass (pa_counts_tile slots)
    uint32_t ncrep;
    const PaBlk *fam;  // chunks of PA_HCHUNK families
    uint32_t nfam;
    const PaBlk *col;  // all 64-replica columns (capacity)
    uint32_t ncol;
    const PaBlk *tile; // scan tiles, run-major
    uint32_t ntile;
    int maxH;
    int ngroups;       // runs grouped by lattice shape for the sweeps
    const PaBlk *gcol[PA_MAX_GROUPS];
    uint32_t gncol[PA_MAX_GROUPS];
    int gd[PA_MAX_GROUPS], gN[PA_MAX_GROUPS], gJ[PA_MAX_GROUPS], gthreads[PA_MAX_GROUPS];
    bool weights;          // some run may hold a weighted population (conditional resampling)
    PaStepRecord *steprec; // batched anneal: [nruns][npoints]
    int npoints;
    hipStream_t stream;
    // with several groups: one side stream per group, so that the groups'
    // sweeps run side by side (fork on `stream`, join back into it)
    hipStream_t gstream[PA_MAX_GROUPS];
    hipEvent_t fork, join[PA_MAX_GROUPS];
};

// launchers (pa_kernels.hip); each returns the first launch error
hipError_t pa_b_init(const PaBatchView &v);
// t0: sweeps already done at this beta; gather: the populations' spins may
// still be in the other buffer (PaRecord::gather), taken in by the sweep
hipError_t pa_b_sweep(const PaBatchView &v, int theta, uint32_t t0, int gather);
hipError_t pa_b_gather(const PaBatchView &v); // gathers the spins a resampling left for the sweeps to gather
hipError_t pa_b_sweep_group(const PaBatchView &v, int g, int theta, int threads);
// hist_clean: the level histogram is zero (observables or init ran since it was last built)
// State of each run's level histogram, tracked by the host: all zero (with
// the energy extremes reset), valid for the current population, or stale.
#define PA_HIST_ZERO 0
#define PA_HIST_VALID 1
#define PA_HIST_STALE 2
hipError_t pa_b_reweight(const PaBatchView &v, double beta_next, int hist_state);
// kq >= 0: conditional, resample only when ESS < kq 2^-16 R_cur (else keep the population)
// prepped: a pa_b_reweight came right before (it clears the resampling's flags and status)
hipError_t pa_b_resample(const PaBatchView &v, int scheme, int freeze, int kq, bool prepped);
hipError_t pa_b_observables(const PaBatchView &v, int point, int hist_state); // builds the histogram if not valid
hipError_t pa_b_rule(const PaBatchView &v, double alpha_star, double dbeta_max, int iterations, int bisect,
                     int hist_state);
hipError_t pa_b_tune_beta(const PaBatchView &v, double beta); // every run's thresholds at beta
hipError_t pa_b_set_beta(const PaBatchView &v, double beta, double lnZ, uint32_t step, uint32_t sweeps,
                         uint64_t R);
hipError_t pa_launch_combine(const PaBatchView &v, int point, const int32_t *group_of, int ngroups,
                             const int32_t *Ns, double *out);
hipError_t pa_launch_philox_probe(uint32_t *out, int64_t nthreads, int iters, hipStream_t st);
// Counters of the allocation-free overlap's file-scope histogram (N + 1 <= 16385).
#define PA_NOALLOC_HIST_MAX 16385
// Device address of that histogram on `device` (looked up once per device).
hipError_t pa_noalloc_scratch(int device, unsigned long long **out);
hipError_t pa_launch_overlap(const PaRunDesc *a, const PaRunDesc *b, int N, uint32_t ncols_a,
                             unsigned long long *hist, hipStream_t st);
hipError_t pa_b_features(const PaBatchView &v, int hist_state);
hipError_t pa_b_check_candidate(const PaBatchView &v, double alpha_star, double dbeta_max, int iterations,
                                double bracket, int refine);
hipError_t pa_mlp_launch_grad(const PaMlpDev &m, int n, int adam, int t, float lr);
hipError_t pa_mlp_launch_predict(const PaMlpDev &m, const float *X, int n, float *out);
hipError_t pa_mlp_launch_propose(const PaBatchView &v, const PaMlpDev &m, double dbeta_max);
hipError_t pa_query_lds(int *max_lds);
size_t pa_sweep_lds_bytes(int N, int d, int threads, bool J); // dynamic LDS of a sweep workgroup (J: bond masks)
size_t pa_cluster_lds_bytes(int N, bool J);                   // dynamic LDS of a cluster-update workgroup
hipError_t pa_b_cluster(const PaBatchView &v, int nsteps, uint32_t t0); // Wolff updates of every run
