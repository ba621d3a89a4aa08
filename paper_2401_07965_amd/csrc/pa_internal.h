// Internal interface between the host state machine (pa_api.cpp) and the
// kernels (pa_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Per-run scalars that live in device memory, written by the kernels.
struct PaRecord {
    // histogram of the current population (pa_reweight)
    int32_t emin, emax;
    // Q(beta_cur, beta_next): Eq. (1) with the shift by E_min
    double qsum, lnQ, dbeta, beta_next;
    uint64_t S;     // sum of integer weights
    uint64_t Tn[3]; // Metropolis thresholds at beta_next for dE = 4, 8, 12
    uint64_t T[3];  // thresholds at the current beta (used by the sweeps)
    // resampling
    uint64_t Rprev, Rnew;
    double sv;
    double lnZ; // ln Z_0 + sum_k ln Q_k, Eq. (7)
    unsigned long long Ctot; // total of the weight scan (equals S)
    // observables (exact integer sums, then the finalised averages)
    unsigned long long sumE, sumE2, sumAbsM, sumM2, sumC2, families;
    double sumClnC;
    double e, e2, abs_m, m2, rho_t, S_f;
    double rule_dbeta, rule_alpha; // adaptive step: chosen dbeta and its overlap
    unsigned long long philox_calls; // Philox4x32-10 evaluations of all sweeps so far
    unsigned long long site_updates; // word-site updates (64 attempts each) so far
    uint32_t err; // bit 0: scan look-back gave up waiting
    uint32_t pad;
};

struct PaScanTile {
    unsigned long long agg, incl;
    uint32_t flag, pad;
};

#define PA_SCAN_THREADS 256
#define PA_SCAN_ITEMS 8
#define PA_SCAN_TILE (PA_SCAN_THREADS * PA_SCAN_ITEMS)
#define PA_RED_BLOCKS 256 // partial sums of the fixed-order reductions

// Device buffers of one run, carved from the caller's workspace.
struct PaDev {
    uint64_t *spins[2]; // [W][N] words, bit b of word (w, s) = replica 64w+b at site s
    int32_t *E[2], *M[2];
    uint32_t *label[2];
    uint8_t *jmask; // per site: bit mu = J(s,mu) is -1, bit d+mu = J(s-e_mu,mu) is -1
    uint32_t *hist; // [H] replicas per energy level h = (E + dN) / 4
    uint64_t *wtab; // [H] integer weight per level above the lowest
    uint32_t *r, *P, *anc;
    uint64_t *C;
    unsigned long long *qhist; // [N+1] overlap histogram
    PaScanTile *tiles;
    uint32_t *ticket;
    uint32_t *fam; // [R0] replicas per family
    double *partial; // [PA_RED_BLOCKS]
    PaRecord *rec;
};

struct PaLaunch {
    int d, L, N, H;
    uint32_t seed, run_id;
    int64_t R0, cap;
    hipStream_t stream;
};

// kernels' host launchers (pa_kernels.hip); each returns the launch error
hipError_t pa_launch_init(const PaLaunch &p, const PaDev &dv, int cur);
hipError_t pa_launch_sweep(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, uint32_t step,
                           uint32_t t0, int theta);
hipError_t pa_launch_reweight(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, double dbeta,
                              double beta_next);
hipError_t pa_launch_counts(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rprev, int64_t Rt,
                            int scheme, uint32_t step);
hipError_t pa_launch_apply(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rprev, int64_t Rnew);
hipError_t pa_launch_observables(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur);
hipError_t pa_launch_overlap(const PaLaunch &p, const uint64_t *a, const uint64_t *b, int64_t R,
                             unsigned long long *hist);
hipError_t pa_launch_rule(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, double alpha_star,
                          double dbeta_max, int iterations, int bisect);
hipError_t pa_launch_set_beta(const PaLaunch &p, const PaDev &dv, double beta, double lnZ);
hipError_t pa_configure_kernels(int *max_lds); // largest LDS a workgroup may use
size_t pa_sweep_lds_bytes(int N);
