/*
 * pa_oracle.c -- CPU oracle for the population-annealing (PA) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * restatement of the method in "Optimized population Monte Carlo" (Ebert,
 * Gessert, Janke, Weigel), used to check the GPU library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never calls it and shares no code with it.
 *
 * Spins are int8 (+1/-1), one byte per site per replica, row = replica.
 * All floating point is IEEE double with every operation rounded separately
 * (built with -ffp-contract=off), so that the decisions below are fixed.
 *
 * What the paper fixes and what is a reading:
 *  - Population, resampling factor tau = exp(-dbeta E)/Q and Q itself: Sec. 2,
 *    step 2 of the algorithm and Eq. (1).
 *  - Single-replica updates ("e.g. MCMC", Sec. 2 step 3): reading = Metropolis
 *    sweeps in checkerboard order (all even sites, then all odd sites).
 *  - The four resampling schemes and the rescaled factors of Eq. (3): Sec. 3.
 *    Reading: all decisions are taken in exact integer arithmetic on weights
 *    quantised to 2^-40 of the largest weight of the step.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), counter-based, one
 *    counter layout per purpose (listed at philox_* below).
 *  - exp() feeding a decision: pa_exp below, a fixed sequence of rounded
 *    double operations (Cody-Waite reduction + degree-13 Taylor polynomial).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of a multiply-xor bijection on a     */
/* 128-bit counter, keyed by a 64-bit key bumped by Weyl constants.         */
/* ------------------------------------------------------------------------ */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox4(uint32_t seed, uint32_t run_id, uint32_t c0, uint32_t c1,
                    uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    orc_philox(seed, run_id, ctr, out);
}

/* Purpose codes, held in bits 31..28 of the last counter word. */
#define PURPOSE_INIT 1u
#define PURPOSE_METRO 2u
#define PURPOSE_RS_NI 4u
#define PURPOSE_RS_POIS 5u
#define PURPOSE_RS_MULT 6u
#define PURPOSE_RS_SYS 7u
#define PURPOSE_WSEED 8u
#define PURPOSE_WBOND 9u

/* Threads the oracle's OpenMP loops use (reported with its timings). */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ------------------------------------------------------------------------ */
/* Deterministic exponential for every exp() whose value feeds a decision.  */
/* exp(x) = 2^k exp(r), k = nearest integer to x/ln2, r = x - k ln2 in two   */
/* pieces (Cody & Waite); exp(r) by its Taylor series to degree 13 in Horner */
/* form; every operation rounded on its own.  Returns 0 below -700 (and for */
/* NaN), where no caller needs a nonzero value.                              */
/* ------------------------------------------------------------------------ */
static const double INV_LN2 = 0x1.71547652b82fep+0; /* 1/ln 2 rounded to nearest  */
static const double LN2_HI = 0x1.62e42fee00000p-1;  /* ln 2 cut to 32 significant */
static const double LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - LN2_HI, rounded      */

double orc_exp(double x)
{
    if (!(x >= -700.0))
        return 0.0;
    double k = rint(x * INV_LN2); /* round half to even */
    double r = (x - k * LN2_HI) - k * LN2_LO;
    /* 1/n! for n = 0..13; n! is exact in double, so each quotient is RN(1/n!) */
    double c[14];
    double fact = 1.0;
    for (int n = 0; n <= 13; ++n) {
        if (n > 0)
            fact = fact * (double)n;
        c[n] = 1.0 / fact;
    }
    double p = c[13];
    for (int n = 12; n >= 0; --n)
        p = p * r + c[n];
    return ldexp(p, (int)k);
}

void orc_exp_array(int64_t n, const double *x, double *out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = orc_exp(x[k]);
}

/* ------------------------------------------------------------------------ */
/* Lattice: hypercubic, side L, dimension d in {2,3}, periodic.  Site       */
/* s = x + L*y + L*L*z.  Bond (s,mu) joins s and s+e_mu with coupling        */
/* J[s*d+mu] in {+1,-1}; H = -sum_{s,mu} J sigma_s sigma_{s+e_mu}, Eq. (4)   */
/* (the +-J Edwards-Anderson glass is the same form with random J).          */
/* ------------------------------------------------------------------------ */
static int64_t n_sites(int d, int L)
{
    int64_t n = 1;
    for (int k = 0; k < d; ++k)
        n *= L;
    return n;
}

static int64_t stride_of(int L, int mu)
{
    int64_t st = 1;
    for (int k = 0; k < mu; ++k)
        st *= L;
    return st;
}

static int coord_of(int64_t s, int L, int mu) { return (int)((s / stride_of(L, mu)) % L); }

static int64_t neighbor(int64_t s, int L, int mu, int dir)
{
    int64_t st = stride_of(L, mu);
    int c = coord_of(s, L, mu);
    int cn = (c + dir + L) % L;
    return s + (int64_t)(cn - c) * st;
}

static int color_of(int64_t s, int d, int L)
{
    int sum = 0;
    for (int mu = 0; mu < d; ++mu)
        sum += coord_of(s, L, mu);
    return sum & 1;
}

int64_t orc_energy(int d, int L, const int8_t *J, const int8_t *spin)
{
    int64_t N = n_sites(d, L);
    int64_t e = 0;
    for (int64_t s = 0; s < N; ++s)
        for (int mu = 0; mu < d; ++mu)
            e -= (int64_t)J[s * d + mu] * spin[s] * spin[neighbor(s, L, mu, +1)];
    return e;
}

/* ------------------------------------------------------------------------ */
/* Step 1 of the algorithm at beta_0 = 0: exact i.i.d. sampling (Sec. 2).   */
/* Replica r = 64w + b takes, at site s, bit b of x0 | x1<<32 of            */
/* Philox(ctr = (s, w, 0, INIT<<28)); bit 1 means sigma = -1.  Row n holds  */
/* replica rep[n], so a sample of a large population can be drawn alone.    */
/* ------------------------------------------------------------------------ */
void orc_init(int d, int L, int64_t nrows, const int64_t *rep, uint32_t seed, uint32_t run_id,
              const int8_t *J, int8_t *spins, int32_t *E, uint32_t *label)
{
    int64_t N = n_sites(d, L);
    for (int64_t n = 0; n < nrows; ++n) {
        int64_t r = rep[n];
        uint32_t w = (uint32_t)(r >> 6), b = (uint32_t)(r & 63);
        int8_t *sp = spins + n * N;
        for (int64_t s = 0; s < N; ++s) {
            uint32_t x[4];
            philox4(seed, run_id, (uint32_t)s, w, 0u, PURPOSE_INIT << 28, x);
            uint64_t bits = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
            sp[s] = ((bits >> b) & 1u) ? -1 : 1;
        }
        E[n] = (int32_t)orc_energy(d, L, J, sp);
        label[n] = (uint32_t)r;
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3 of the algorithm: theta Metropolis sweeps at beta (reading of      */
/* "e.g. MCMC").  A sweep visits the sites of colour 0, then colour 1, where */
/* colour = (x+y+z) mod 2.  Flipping site s changes the energy by            */
/* dE = 2 sigma_s sum_nb J sigma_nb; the move is taken if dE <= 0, else iff  */
/* u < T(dE) with T(dE) = min(2^32, floor(2^32 pa_exp(-beta dE))) and u the  */
/* replica's 32-bit uniform.  u of replica r = 64w+b at (site s, step i,     */
/* sweep t): 16 Philox calls, ctr = (s, w, i, METRO<<28 | t<<8 | q), q=0..15, */
/* give 32 bit-planes (plane 2q = x0|x1<<32, plane 2q+1 = x2|x3<<32) and    */
/* u = sum_k bit_b(plane_k) 2^(31-k).                                         */
/*                                                                          */
/* rows[n] holds replica index rep[n] (ascending); E is updated with each   */
/* accepted dE.  Replicas are independent chains, so they are visited one   */
/* word (64 replicas) at a time to reuse the planes of that word.           */
/*                                                                          */
/* Work count (accounting, not part of the method): u < T is decided at the */
/* first plane k where bit 31-k of u and of T differ (k = 32 if u = T).  A  */
/* word-site needs plane pairs 0..k/2 of its slowest drawing replica (dE > 0 */
/* and 0 < T < 2^32), at most 16; *calls (if not NULL) gets the sum of the  */
/* pairs over the word-sites visited, i.e. the Philox evaluations that      */
/* deciding replica by replica in plane order needs.                        */
/* ------------------------------------------------------------------------ */
uint64_t orc_threshold(double beta, int dE)
{
    double p = orc_exp(-(beta * (double)dE));
    double t = floor(ldexp(p, 32));
    uint64_t T = (uint64_t)t;
    if (T > ((uint64_t)1 << 32))
        T = (uint64_t)1 << 32;
    return T;
}

static void metro_planes(uint32_t seed, uint32_t run_id, uint32_t s, uint32_t w, uint32_t step,
                         uint32_t t, uint64_t planes[32])
{
    for (uint32_t q = 0; q < 16; ++q) {
        uint32_t x[4];
        philox4(seed, run_id, s, w, step, (PURPOSE_METRO << 28) | (t << 8) | q, x);
        planes[2 * q] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        planes[2 * q + 1] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
    }
}

static uint32_t uniform_of(const uint64_t planes[32], uint32_t b)
{
    uint32_t u = 0;
    for (int k = 0; k < 32; ++k)
        u |= (uint32_t)((planes[k] >> b) & 1u) << (31 - k);
    return u;
}

static int decision_plane(uint32_t u, uint64_t T)
{
    for (int k = 0; k < 32; ++k) {
        uint32_t ub = (u >> (31 - k)) & 1u, tb = (uint32_t)(T >> (31 - k)) & 1u;
        if (ub != tb)
            return k;
    }
    return 32;
}

void orc_sweep(int d, int L, const int8_t *J, int64_t nrows, const int64_t *rep, int8_t *spins,
               int32_t *E, uint32_t seed, uint32_t run_id, uint32_t step, uint32_t t0,
               int32_t theta, double beta, uint64_t *calls)
{
    uint64_t total_calls = 0;
    int64_t N = n_sites(d, L);
    uint64_t T[4 * 3 + 1];
    for (int dE = 0; dE <= 12; ++dE)
        T[dE] = (dE > 0) ? orc_threshold(beta, dE) : 0;

    /* groups of consecutive rows that share a 64-replica word */
    int64_t *gstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nrows + 1));
    int64_t ng = 0;
    for (int64_t n = 0; n < nrows; ++n)
        if (n == 0 || (rep[n] >> 6) != (rep[n - 1] >> 6))
            gstart[ng++] = n;
    gstart[ng] = nrows;

#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total_calls)
    for (int64_t g = 0; g < ng; ++g) {
        uint32_t w = (uint32_t)(rep[gstart[g]] >> 6);
        uint64_t planes[32];
        for (int32_t tt = 0; tt < theta; ++tt) {
            uint32_t t = t0 + (uint32_t)tt;
            for (int color = 0; color < 2; ++color) {
                for (int64_t s = 0; s < N; ++s) {
                    if (color_of(s, d, L) != color)
                        continue;
                    metro_planes(seed, run_id, (uint32_t)s, w, step, t, planes);
                    int pairs = 0;
                    for (int64_t n = gstart[g]; n < gstart[g + 1]; ++n) {
                        int8_t *sp = spins + n * N;
                        int field = 0;
                        for (int mu = 0; mu < d; ++mu) {
                            int64_t up = neighbor(s, L, mu, +1);
                            int64_t dn = neighbor(s, L, mu, -1);
                            field += J[s * d + mu] * sp[up] + J[dn * d + mu] * sp[dn];
                        }
                        int dE = 2 * sp[s] * field;
                        int accept;
                        if (dE <= 0) {
                            accept = 1;
                        } else {
                            uint32_t u = uniform_of(planes, (uint32_t)(rep[n] & 63));
                            accept = (uint64_t)u < T[dE];
                            if (T[dE] > 0 && T[dE] < ((uint64_t)1 << 32)) {
                                int k = decision_plane(u, T[dE]);
                                int need = (k < 32 ? k : 31) / 2 + 1;
                                if (need > pairs)
                                    pairs = need;
                            }
                        }
                        if (accept) {
                            sp[s] = (int8_t)-sp[s];
                            E[n] += dE;
                        }
                    }
                    total_calls += (uint64_t)pairs;
                }
            }
        }
    }
    free(gstart);
    if (calls)
        *calls = total_calls;
}

/* ------------------------------------------------------------------------ */
/* Cluster updates as the driver of step 3 (Sec. 1 names them among the     */
/* update algorithms the scheme can use; reading: Wolff's single-cluster    */
/* update).  One update of replica r = 64w + b at (step i, update t):        */
/*  - the seed site is s0 = floor(x0 N / 2^32), x0 from                      */
/*    Philox(ctr = (b, w, i, WSEED<<28 | t<<8));                             */
/*  - the bond (s, mu) joining s and s + e_mu is active iff it is satisfied */
/*    (J sigma_s sigma_{s+e_mu} = +1) and u < T_p, T_p = min(2^32,           */
/*    floor(2^32 (1 - pa_exp(-2 beta)))), u the replica's 32-bit uniform of  */
/*    the bit planes of Philox(ctr = (s, w, i, WBOND<<28 | t<<8 | mu<<4 | q)), */
/*    q = 0..15, laid out as for the Metropolis decisions;                   */
/*  - the cluster is the set of sites joined to s0 by active bonds, found   */
/*    by a breadth-first search here; all its spins flip.                   */
/* Whether a bond is active is fixed before the search, so the cluster does  */
/* not depend on the order in which it is grown.  csize (if not NULL) gets   */
/* the cluster sizes, row-major [nrows][nsteps].                            */
/* ------------------------------------------------------------------------ */
uint64_t orc_wolff_threshold(double beta)
{
    double p = 1.0 - orc_exp(-(2.0 * beta));
    double t = floor(ldexp(p, 32));
    uint64_t T = (uint64_t)t;
    if (T > ((uint64_t)1 << 32))
        T = (uint64_t)1 << 32;
    return T;
}

/* u < T for replica b of word w on bond (s, mu), compared from the most   */
/* significant bit down (bit 31 - k of u is bit b of plane k), stopping at   */
/* the first bit where u and T differ; equal in all 32 bits means u = T.    */
static int bond_active(uint32_t seed, uint32_t run_id, uint32_t s, uint32_t w, uint32_t step,
                       uint32_t t, int mu, uint32_t b, uint64_t T)
{
    if (T >= ((uint64_t)1 << 32))
        return 1;
    for (uint32_t q = 0; q < 16; ++q) {
        uint32_t x[4];
        philox4(seed, run_id, s, w, step, (PURPOSE_WBOND << 28) | (t << 8) | ((uint32_t)mu << 4) | q, x);
        const uint64_t planes[2] = {(uint64_t)x[0] | ((uint64_t)x[1] << 32), (uint64_t)x[2] | ((uint64_t)x[3] << 32)};
        for (int h = 0; h < 2; ++h) {
            int bit = 31 - (int)(2 * q) - h;
            uint32_t ub = (uint32_t)(planes[h] >> b) & 1u, tb = (uint32_t)(T >> bit) & 1u;
            if (ub != tb)
                return ub < tb;
        }
    }
    return 0;
}

void orc_wolff(int d, int L, const int8_t *J, int64_t nrows, const int64_t *rep, int8_t *spins,
               int32_t *E, uint32_t seed, uint32_t run_id, uint32_t step, uint32_t t0, int32_t nsteps,
               double beta, int64_t *csize)
{
    int64_t N = n_sites(d, L);
    uint64_t T = orc_wolff_threshold(beta);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t n = 0; n < nrows; ++n) {
        uint32_t w = (uint32_t)(rep[n] >> 6), b = (uint32_t)(rep[n] & 63);
        int8_t *sp = spins + n * N;
        uint8_t *in = (uint8_t *)malloc((size_t)N);
        int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
        for (int32_t k = 0; k < nsteps; ++k) {
            uint32_t t = t0 + (uint32_t)k;
            uint32_t x[4];
            philox4(seed, run_id, b, w, step, (PURPOSE_WSEED << 28) | (t << 8), x);
            int64_t s0 = (int64_t)(((uint64_t)x[0] * (uint64_t)N) >> 32);
            memset(in, 0, (size_t)N);
            int64_t head = 0, tail = 0;
            queue[tail++] = s0;
            in[s0] = 1;
            while (head < tail) {
                int64_t s = queue[head++];
                for (int mu = 0; mu < d; ++mu)
                    for (int dir = -1; dir <= 1; dir += 2) {
                        int64_t nb = neighbor(s, L, mu, dir);
                        if (in[nb])
                            continue;
                        int64_t owner = dir > 0 ? s : nb; /* bond (owner, mu) */
                        if (J[owner * d + mu] * sp[s] * sp[nb] != 1)
                            continue;
                        if (bond_active(seed, run_id, (uint32_t)owner, w, step, t, mu, b, T)) {
                            in[nb] = 1;
                            queue[tail++] = nb;
                        }
                    }
            }
            for (int64_t s = 0; s < N; ++s)
                if (in[s])
                    sp[s] = (int8_t)-sp[s];
            E[n] = (int32_t)orc_energy(d, L, J, sp);
            if (csize)
                csize[n * nsteps + k] = tail;
        }
        free(in);
        free(queue);
    }
}

/* ------------------------------------------------------------------------ */
/* Step 2 of the algorithm: Q of Eq. (1) and the integer weights.           */
/* Q = (1/R) sum_j exp(-dbeta E_j) is written with the shift by E_min so    */
/* that no term overflows: ln Q = -dbeta E_min + ln((1/R) sum_j             */
/* exp(-dbeta (E_j - E_min))).  The weights that decide the resampling are  */
/* W_j = floor(2^40 pa_exp(-dbeta (E_j - E_min))), so W_j <= 2^40 and       */
/* tau_j = R W_j / S with S = sum_j W_j (reading: 2^-40 resolution).        */
/* ------------------------------------------------------------------------ */
void orc_reweight(int64_t R, const int32_t *E, double dbeta, double *lnQ, uint64_t *W,
                  uint64_t *S)
{
    int32_t emin = E[0];
    for (int64_t j = 1; j < R; ++j)
        if (E[j] < emin)
            emin = E[j];
    /* compensated (Neumaier) sum, so that its rounding error does not grow */
    /* with R: ln Q is small where the two terms below nearly cancel        */
    double sum = 0.0, comp = 0.0;
    for (int64_t j = 0; j < R; ++j) {
        double x = exp(-dbeta * (double)(E[j] - emin));
        double t = sum + x;
        if (fabs(sum) >= fabs(x))
            comp += (sum - t) + x;
        else
            comp += (x - t) + sum;
        sum = t;
    }
    sum += comp;
    *lnQ = -dbeta * (double)emin + log(sum / (double)R);
    uint64_t tot = 0;
    for (int64_t j = 0; j < R; ++j) {
        double w = orc_exp(-(dbeta * (double)(E[j] - emin)));
        W[j] = (uint64_t)floor(ldexp(w, 40));
        tot += W[j];
    }
    *S = tot;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3: copy numbers r_j with <r_j> = tau_j.  tauhat_j = Rt W_j / S      */
/* (Eq. (3): Rt is the target size; for the fixed-size schemes the sizes    */
/* before and after are both Rt).                                           */
/* ------------------------------------------------------------------------ */

/* Nearest integer (Sec. 3, variable size): floor(tauhat) copies plus one   */
/* more with probability tauhat - floor(tauhat); u_j = x0 of                */
/* Philox(ctr = (j, 0, i, RS_NI<<28)), the extra copy iff u_j/2^32 <        */
/* frac(tauhat), compared exactly as u_j S < (Rt W_j mod S) 2^32.           */
static void counts_nearest(int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
                           uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r)
{
    for (int64_t j = 0; j < Rprev; ++j) {
        u128 a = (u128)(uint64_t)Rt * (u128)W[j];
        u128 q = a / S;
        u128 rho = a % S;
        uint32_t x[4];
        philox4(seed, run_id, (uint32_t)j, 0u, step, PURPOSE_RS_NI << 28, x);
        int extra = ((u128)x[0] * (u128)S) < (rho << 32);
        r[j] = (uint32_t)q + (uint32_t)extra;
    }
}

/* Poisson (Sec. 3, variable size): r_j ~ Poisson(tauhat_j) by inversion of */
/* the cumulative distribution.  tauhat is cut into m = ceil(tauhat/32)      */
/* equal pieces when above 32 (a sum of Poissons is Poisson); piece p draws  */
/* u = ((x0>>5) 2^26 + (x1>>6)) 2^-53 from Philox(ctr = (j, p, i,            */
/* RS_POIS<<28)).  The search stops once the cumulative sum stops growing.   */
static uint32_t poisson_inv(double mu, double u)
{
    uint32_t k = 0;
    double p = orc_exp(-mu);
    double F = p;
    while (u >= F) {
        k += 1;
        p = (p * mu) / (double)k;
        double Fn = F + p;
        if (Fn == F)
            break;
        F = Fn;
    }
    return k;
}

static void counts_poisson(int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
                           uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r)
{
    for (int64_t j = 0; j < Rprev; ++j) {
        double tau = ((double)W[j] / (double)S) * (double)Rt;
        uint32_t m = 1;
        if (tau > 32.0)
            m = (uint32_t)ceil(tau / 32.0);
        double mu = tau / (double)m;
        uint32_t tot = 0;
        for (uint32_t p = 0; p < m; ++p) {
            uint32_t x[4];
            philox4(seed, run_id, (uint32_t)j, p, step, PURPOSE_RS_POIS << 28, x);
            double u = ((double)(x[0] >> 5) * 67108864.0 + (double)(x[1] >> 6)) *
                       (1.0 / 9007199254740992.0);
            tot += poisson_inv(mu, u);
        }
        r[j] = tot;
    }
}

/* Multinomial (Sec. 3 and Fig. 2a, fixed size): Rt points U_k uniform on   */
/* [0, S), replica j owning the box [C_{j-1}, C_j) with C the inclusive      */
/* prefix sum of W.  U_k = floor(r S / 2^128) with r the 128 bits of         */
/* Philox(ctr = (k, 0, i, RS_MULT<<28)), x0 least significant.               */
static void counts_multinomial(int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
                               uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r)
{
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)Rprev);
    uint64_t acc = 0;
    for (int64_t j = 0; j < Rprev; ++j) {
        acc += W[j];
        C[j] = acc;
        r[j] = 0;
    }
    for (int64_t k = 0; k < Rt; ++k) {
        uint32_t x[4];
        philox4(seed, run_id, (uint32_t)k, 0u, step, PURPOSE_RS_MULT << 28, x);
        uint64_t lo = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        uint64_t hi = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
        /* floor((hi 2^64 + lo) S / 2^128), exactly */
        u128 a = (u128)lo * (u128)S;
        u128 b = (u128)hi * (u128)S;
        uint64_t U = (uint64_t)((b + (a >> 64)) >> 64);
        /* first j with C_j > U */
        int64_t lo_i = 0, hi_i = Rprev - 1;
        while (lo_i < hi_i) {
            int64_t mid = lo_i + (hi_i - lo_i) / 2;
            if (C[mid] > U)
                hi_i = mid;
            else
                lo_i = mid + 1;
        }
        r[lo_i] += 1;
    }
    free(C);
}

/* Systematic (Sec. 3 and Fig. 2b, fixed size): one uniform U/2^32 with     */
/* U = x0 of Philox(ctr = (0, 0, i, RS_SYS<<28)); the points are             */
/* (k + U/2^32) S / Rt, k = 0..Rt-1, and replica j takes those falling in    */
/* [C_{j-1}, C_j).  Point k lies below c iff (k 2^32 + U) S < c Rt 2^32.     */
static void counts_systematic(int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
                              uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r)
{
    uint32_t x[4];
    philox4(seed, run_id, 0u, 0u, step, PURPOSE_RS_SYS << 28, x);
    uint32_t U = x[0];
    int64_t j = 0;
    uint64_t C = W[0];
    for (int64_t jj = 0; jj < Rprev; ++jj)
        r[jj] = 0;
    for (int64_t k = 0; k < Rt; ++k) {
        u128 lhs = (((u128)(uint64_t)k << 32) + (u128)U) * (u128)S;
        while (!(lhs < (((u128)C * (u128)(uint64_t)Rt) << 32))) {
            j += 1;
            C += W[j];
        }
        r[j] += 1;
    }
}

/* scheme: 0 multinomial, 1 Poisson, 2 nearest integer, 3 systematic */
int orc_counts(int scheme, int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
               uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r)
{
    if (S == 0 || Rprev < 1 || Rt < 1)
        return -1;
    switch (scheme) {
    case 0: counts_multinomial(Rprev, Rt, W, S, seed, run_id, step, r); return 0;
    case 1: counts_poisson(Rprev, Rt, W, S, seed, run_id, step, r); return 0;
    case 2: counts_nearest(Rprev, Rt, W, S, seed, run_id, step, r); return 0;
    case 3: counts_systematic(Rprev, Rt, W, S, seed, run_id, step, r); return 0;
    default: return -1;
    }
}

/* Apply the copy numbers: the new population lists r_j copies of each old  */
/* replica j, in ascending j (reading: the paper leaves the order open).     */
void orc_apply(int64_t N, int64_t Rprev, const uint32_t *r, const int8_t *spins_in,
               const int32_t *E_in, const uint32_t *label_in, int8_t *spins_out,
               int32_t *E_out, uint32_t *label_out)
{
    int64_t d = 0;
    for (int64_t j = 0; j < Rprev; ++j)
        for (uint32_t c = 0; c < r[j]; ++c) {
            memcpy(spins_out + d * N, spins_in + j * N, (size_t)N);
            E_out[d] = E_in[j];
            label_out[d] = label_in[j];
            d += 1;
        }
}
