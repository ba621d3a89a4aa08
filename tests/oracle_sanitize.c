/* Drives the CPU oracle's C functions (oracle/pa_oracle.c) over small
 * populations, so that test_oracle_sanitizers.py can run them built with
 * AddressSanitizer and UndefinedBehaviorSanitizer: initial sampling, the
 * reweighting, all four copy-number schemes, the copy step, Metropolis
 * sweeps and cluster updates, in 2D and 3D with +-J couplings, checking the
 * tracked energies against recounts.  Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_energy(int d, int L, const int8_t *J, const int8_t *spin);
void orc_init(int d, int L, int64_t nrows, const int64_t *rep, uint32_t seed, uint32_t run_id,
              const int8_t *J, int8_t *spins, int32_t *E, uint32_t *label);
void orc_sweep(int d, int L, const int8_t *J, int64_t nrows, const int64_t *rep, int8_t *spins,
               int32_t *E, uint32_t seed, uint32_t run_id, uint32_t step, uint32_t t0,
               int32_t theta, double beta, uint64_t *calls);
void orc_wolff(int d, int L, const int8_t *J, int64_t nrows, const int64_t *rep, int8_t *spins,
               int32_t *E, uint32_t seed, uint32_t run_id, uint32_t step, uint32_t t0, int32_t nsteps,
               double beta, int64_t *csize);
void orc_reweight(int64_t R, const int32_t *E, double dbeta, double *lnQ, uint64_t *W, uint64_t *S);
int orc_counts(int scheme, int64_t Rprev, int64_t Rt, const uint64_t *W, uint64_t S,
               uint32_t seed, uint32_t run_id, uint32_t step, uint32_t *r);
void orc_apply(int64_t N, int64_t Rprev, const uint32_t *r, const int8_t *spins_in,
               const int32_t *E_in, const uint32_t *label_in, int8_t *spins_out,
               int32_t *E_out, uint32_t *label_out);

static int run(int d, int L, int64_t R0, uint32_t seed)
{
    int64_t N = 1;
    for (int k = 0; k < d; ++k)
        N *= L;
    const int64_t cap = 2 * R0 + 64;
    int8_t *J = malloc((size_t)(N * d));
    uint32_t x = seed * 2654435761u + 1u;
    for (int64_t b = 0; b < N * d; ++b) {
        x ^= x << 13, x ^= x >> 17, x ^= x << 5;
        J[b] = (x & 1u) ? -1 : 1;
    }
    int8_t *sp = malloc((size_t)(cap * N)), *sp2 = malloc((size_t)(cap * N));
    int32_t *E = malloc((size_t)cap * 4), *E2 = malloc((size_t)cap * 4);
    uint32_t *lab = malloc((size_t)cap * 4), *lab2 = malloc((size_t)cap * 4), *r = malloc((size_t)cap * 4);
    uint64_t *W = malloc((size_t)cap * 8);
    int64_t *rep = malloc((size_t)cap * 8), *cs = malloc((size_t)cap * 8);
    int64_t R = R0;
    for (int64_t n = 0; n < cap; ++n)
        rep[n] = n;
    orc_init(d, L, R, rep, seed, 7u, J, sp, E, lab);
    double beta = 0.0;
    for (uint32_t step = 1; step <= 8; ++step) {
        const double b = 0.3 * step;
        double lnQ;
        uint64_t S;
        orc_reweight(R, E, b - beta, &lnQ, W, &S);
        const int scheme = (int)(step % 4);
        if (orc_counts(scheme, R, R0, W, S, seed, 7u, step, r) != 0)
            return 1;
        int64_t Rn = 0;
        for (int64_t j = 0; j < R; ++j)
            Rn += r[j];
        if (Rn < 1 || Rn > cap)
            return 2;
        orc_apply(N, R, r, sp, E, lab, sp2, E2, lab2);
        int8_t *ts = sp; sp = sp2; sp2 = ts;
        int32_t *te = E; E = E2; E2 = te;
        uint32_t *tl = lab; lab = lab2; lab2 = tl;
        R = Rn;
        beta = b;
        uint64_t calls = 0;
        orc_sweep(d, L, J, R, rep, sp, E, seed, 7u, step, 0u, 2, beta, &calls);
        orc_wolff(d, L, J, R, rep, sp, E, seed, 7u, step, 2u, 1, beta, cs);
        for (int64_t n = 0; n < R; ++n)
            if (orc_energy(d, L, J, sp + n * N) != E[n])
                return 3;
    }
    free(J); free(sp); free(sp2); free(E); free(E2); free(lab); free(lab2); free(r); free(W); free(rep); free(cs);
    return 0;
}

int main(void)
{
    int rc = run(2, 8, 130, 1u);
    if (rc == 0)
        rc = run(3, 4, 200, 2u) * 10;
    if (rc == 0)
        rc = run(2, 2, 65, 3u) * 100; /* L = 2: double bonds */
    printf("oracle sanitizer run: %s (code %d)\n", rc ? "FAILED" : "ok", rc);
    return rc;
}
