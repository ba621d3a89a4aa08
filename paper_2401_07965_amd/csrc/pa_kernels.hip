// HIP kernels of the population-annealing hot path for gfx950 (MI355X).
//
// Spins are multi-spin coded: bit b of word [w][s] is replica 64w+b at site s,
// 1 meaning sigma = -1.  One workgroup owns one 64-replica word column: the
// whole lattice of its 64 replicas (N words) sits in LDS while it is swept.
#include "pa_device.h"
#include "pa_internal.h"

#include <climits>

namespace {

constexpr int kThreads = 256;

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int grid_for(int64_t n, int threads = kThreads, int cap = 4096)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1)
        g = 1;
    return (int)(g > cap ? cap : g);
}

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    k_fill_u32<<<grid_for(n), kThreads, 0, st>>>(p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ step 1: init
// Replica 64w+b, site s: bit b of x0 | x1<<32 of Philox(s, w, 0, INIT<<28).
__global__ void k_init_spins(uint64_t *spins, int N, int64_t W, uint32_t seed, uint32_t run_id)
{
    const int64_t n = W * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = (uint32_t)(i / N), s = (uint32_t)(i - (int64_t)w * N);
        const pa_philox_out o = pa_philox(seed, run_id, s, w, 0u, PA_PURPOSE_INIT << 28);
        spins[i] = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
    }
}

__global__ void k_init_labels(uint32_t *label, int64_t R)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R;
         i += (int64_t)gridDim.x * blockDim.x)
        label[i] = (uint32_t)i;
}

// ------------------------------------------------------------------ step 3: sweeps
// Bit-sliced counter: adds a 1-bit-per-replica mask to an 8-plane count.
__device__ __forceinline__ void vadd8(uint64_t c[8], uint64_t x)
{
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint64_t t = c[k] & x;
        c[k] ^= x;
        x = t;
    }
}

// Sum of the 16-plane bit-sliced counters of all 64 lanes (ripple adds over
// a butterfly); every lane ends with the wave total.
__device__ __forceinline__ void wave_vsum16(uint64_t c[16])
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        uint64_t carry = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint64_t o = pa_shfl_xor_u64(c[k], m);
            const uint64_t x = c[k] ^ o;
            const uint64_t s = x ^ carry;
            carry = (c[k] & o) | (carry & x);
            c[k] = s;
        }
    }
}

__device__ __forceinline__ uint64_t jbit(uint32_t jb, int k) { return 0ull - (uint64_t)((jb >> k) & 1u); }

// One workgroup = one word column w (64 replicas); the lattice stays in LDS
// for all theta sweeps, then each replica's unsatisfied-bond count U and
// number of down spins are counted bit-sliced: E = 2U - dN, M = N - 2 n_down.
template <int D>
__global__ __launch_bounds__(kThreads) void k_sweep(uint64_t *__restrict__ spins,
                                                    const uint8_t *__restrict__ jmask, int L, int N,
                                                    int32_t *__restrict__ E, int32_t *__restrict__ M,
                                                    int64_t Rlive, PaRecord *__restrict__ rec,
                                                    uint32_t seed, uint32_t run_id, uint32_t step,
                                                    uint32_t t0, int theta)
{
    extern __shared__ uint64_t lat[];
    uint8_t *jl = reinterpret_cast<uint8_t *>(lat + N);
    __shared__ uint64_t red[kThreads / 64][32];

    const int tid = threadIdx.x, bs = blockDim.x;
    const uint32_t w = blockIdx.x;
    uint64_t *g = spins + (size_t)w * N;
    for (int s = tid; s < N; s += bs) {
        lat[s] = g[s];
        jl[s] = jmask[s];
    }
    __syncthreads();

    const uint64_t two32 = 1ull << 32;
    const uint64_t T4 = rec->T[0], T8 = rec->T[1], T12 = rec->T[2];
    const uint32_t t4 = (uint32_t)T4, t8 = (uint32_t)T8, t12 = (uint32_t)T12;
    // classes whose threshold is 2^32 accept outright, those at 0 never accept
    const uint64_t sure4 = T4 >= two32 ? ~0ull : 0ull, sure8 = T8 >= two32 ? ~0ull : 0ull,
                   sure12 = T12 >= two32 ? ~0ull : 0ull;
    const uint64_t draw4 = (T4 > 0 && T4 < two32) ? ~0ull : 0ull,
                   draw8 = (T8 > 0 && T8 < two32) ? ~0ull : 0ull,
                   draw12 = (T12 > 0 && T12 < two32) ? ~0ull : 0ull;
    const int half = L >> 1, nh = N >> 1, LL = L * L;
    uint32_t calls = 0; // Philox evaluations this lane's words needed

    for (int tt = 0; tt < theta; ++tt) {
        const uint32_t t = t0 + (uint32_t)tt;
        for (int c = 0; c < 2; ++c) {
            for (int k = tid; k < nh; k += bs) {
                const int row = k / half, m = k - row * half; // row = y + L z
                const int y = (D == 2) ? row : row % L;
                const int z = (D == 2) ? 0 : row / L;
                const int x = 2 * m + ((y + z + c) & 1);
                const int s = x + L * row;
                const uint32_t jb = jl[s];
                const uint64_t S = lat[s];
                const uint64_t a0 = S ^ lat[x == L - 1 ? s - (L - 1) : s + 1] ^ jbit(jb, 0);
                const uint64_t a1 = S ^ lat[x == 0 ? s + (L - 1) : s - 1] ^ jbit(jb, D);
                const uint64_t a2 = S ^ lat[y == L - 1 ? s - L * (L - 1) : s + L] ^ jbit(jb, 1);
                const uint64_t a3 = S ^ lat[y == 0 ? s + L * (L - 1) : s - L] ^ jbit(jb, D + 1);
                // u = number of unsatisfied bonds among 2d; dE = 4(d - u)
                uint64_t always, m4, m8, m12;
                if (D == 2) {
                    const uint64_t s0 = a0 ^ a1, c0 = a0 & a1, s1 = a2 ^ a3, c1 = a2 & a3;
                    always = c0 | c1 | (s0 & s1);     // u >= 2
                    m4 = (s0 ^ s1) & ~(c0 | c1);      // u == 1
                    m8 = ~(s0 | s1 | c0 | c1);        // u == 0
                    m12 = 0;
                } else {
                    const uint64_t a4 = S ^ lat[z == L - 1 ? s - LL * (L - 1) : s + LL] ^ jbit(jb, 2);
                    const uint64_t a5 = S ^ lat[z == 0 ? s + LL * (L - 1) : s - LL] ^ jbit(jb, 5);
                    const uint64_t sA = a0 ^ a1 ^ a2, cA = (a0 & a1) | (a2 & (a0 ^ a1));
                    const uint64_t sB = a3 ^ a4 ^ a5, cB = (a3 & a4) | (a5 & (a3 ^ a4));
                    const uint64_t ls = sA ^ sB, lc = sA & sB;
                    // u = 2 (cA + cB + lc) + ls
                    const uint64_t maj = (cA & cB) | (lc & (cA ^ cB));
                    const uint64_t odd = cA ^ cB ^ lc;
                    const uint64_t none = ~(cA | cB | lc);
                    always = maj | (odd & ls);        // u >= 3
                    m4 = odd & ~maj & ~ls;            // u == 2
                    m8 = none & ls;                   // u == 1
                    m12 = none & ~ls;                 // u == 0
                }
                uint64_t acc = always | (m4 & sure4) | (m8 & sure8) | (m12 & sure12);
                uint64_t und = (m4 & draw4) | (m8 & draw8) | (m12 & draw12);
                // u < T decided plane by plane from the most significant bit
                for (uint32_t q = 0; und != 0 && q < 16; ++q) {
                    ++calls;
                    const pa_philox_out o = pa_philox(seed, run_id, (uint32_t)s, w, step,
                                                      (PA_PURPOSE_METRO << 28) | (t << 8) | q);
                    const uint64_t P0 = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
                    const uint64_t P1 = (uint64_t)o.x2 | ((uint64_t)o.x3 << 32);
                    const int b0 = 31 - 2 * (int)q, b1 = b0 - 1;
                    uint64_t Tp = (m4 & (0ull - ((t4 >> b0) & 1u))) | (m8 & (0ull - ((t8 >> b0) & 1u))) |
                                  (m12 & (0ull - ((t12 >> b0) & 1u)));
                    acc |= und & ~P0 & Tp;
                    und &= ~(P0 ^ Tp);
                    Tp = (m4 & (0ull - ((t4 >> b1) & 1u))) | (m8 & (0ull - ((t8 >> b1) & 1u))) |
                         (m12 & (0ull - ((t12 >> b1) & 1u)));
                    acc |= und & ~P1 & Tp;
                    und &= ~(P1 ^ Tp);
                }
                lat[s] = S ^ acc;
            }
            __syncthreads();
        }
    }

    // measure: forward bonds once each, plus the down-spin count
    uint64_t ve[8] = {0, 0, 0, 0, 0, 0, 0, 0}, vm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = tid; s < N; s += bs) {
        const int x = s % L;
        const int row = s / L;
        const int y = (D == 2) ? row : row % L;
        const int z = (D == 2) ? 0 : row / L;
        const uint32_t jb = jl[s];
        const uint64_t S = lat[s];
        vadd8(ve, S ^ lat[x == L - 1 ? s - (L - 1) : s + 1] ^ jbit(jb, 0));
        vadd8(ve, S ^ lat[y == L - 1 ? s - L * (L - 1) : s + L] ^ jbit(jb, 1));
        if (D == 3)
            vadd8(ve, S ^ lat[z == L - 1 ? s - LL * (L - 1) : s + LL] ^ jbit(jb, 2));
        vadd8(vm, S);
        g[s] = S;
    }
    if (theta > 0) {
        const uint64_t tot = pa_wave_sum_u64(calls);
        if ((tid & 63) == 0)
            atomicAdd(&rec->philox_calls, (unsigned long long)tot);
        if (tid == 0)
            atomicAdd(&rec->site_updates, (unsigned long long)theta * (unsigned long long)N);
    }
    uint64_t ce[16], cm[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        ce[k] = k < 8 ? ve[k] : 0;
        cm[k] = k < 8 ? vm[k] : 0;
    }
    wave_vsum16(ce);
    wave_vsum16(cm);
    const int wave = tid >> 6, lane = tid & 63, nw = bs >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            red[wave][k] = ce[k];
            red[wave][16 + k] = cm[k];
        }
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t U = 0, nd = 0;
        for (int v = 0; v < nw; ++v)
            for (int k = 0; k < 16; ++k) {
                U += (uint32_t)((red[v][k] >> lane) & 1u) << k;
                nd += (uint32_t)((red[v][16 + k] >> lane) & 1u) << k;
            }
        const int64_t r = 64 * (int64_t)w + lane;
        if (r < Rlive) {
            E[r] = 2 * (int32_t)U - D * N;
            M[r] = N - 2 * (int32_t)nd;
        }
    }
}

// ------------------------------------------------------------------ step 2: Q
// Energy levels h = (E + dN) / 4: all energies of a run share E mod 4, since a
// flip changes E by a multiple of 4.
__global__ void k_hist_prep(uint32_t *hist, int H, PaRecord *rec)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H; i += gridDim.x * blockDim.x)
        hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rec->emin = INT_MAX;
        rec->emax = INT_MIN;
    }
}

__global__ __launch_bounds__(kThreads) void k_hist(const int32_t *__restrict__ E, int64_t R, int DN,
                                                   int H, uint32_t *hist, PaRecord *rec)
{
    extern __shared__ uint32_t lh[];
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        lh[i] = 0;
    __syncthreads();
    int64_t lo = INT_MAX, hi = INT_MIN;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < R;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = E[j];
        atomicAdd(&lh[(e + DN) >> 2], 1u);
        lo = e < lo ? e : lo;
        hi = e > hi ? e : hi;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        if (lh[i])
            atomicAdd(&hist[i], lh[i]);
    lo = pa_wave_min_i64(lo);
    hi = pa_wave_max_i64(hi);
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&rec->emin, (int)lo);
        atomicMax(&rec->emax, (int)hi);
    }
}

// Single workgroup: weights per level above the lowest, the Q sum in a fixed
// order (contiguous chunk per thread, then the block's fixed tree), S exactly,
// ln Q and the Metropolis thresholds of the next beta.
__global__ __launch_bounds__(1024) void k_reweight(const uint32_t *__restrict__ hist,
                                                   uint64_t *__restrict__ wtab, PaRecord *rec, int DN,
                                                   int64_t Rprev, double dbeta, double beta_next)
{
    __shared__ double sd[16];
    __shared__ uint64_t su[16];
    const int32_t emin = rec->emin, emax = rec->emax;
    const int hmin = (emin + DN) >> 2, hmax = (emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    const int chunk = (nlev + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = (int)threadIdx.x * chunk;
    const int hi = lo + chunk < nlev ? lo + chunk : nlev;
    double q = 0.0;
    uint64_t s = 0;
    for (int k = lo; k < hi; ++k) {
        const uint32_t n = hist[hmin + k];
        const double wv = pa_exp(-(dbeta * (double)(4 * k)));
        const uint64_t W = (uint64_t)floor(ldexp(wv, 40));
        wtab[k] = W;
        q = q + (double)n * wv;
        s += (uint64_t)n * W;
    }
    const double Q = pa_block_sum_f64(q, sd);
    const uint64_t S = pa_block_sum_u64(s, su);
    if (threadIdx.x == 0) {
        rec->qsum = Q;
        rec->S = S;
        rec->dbeta = dbeta;
        rec->beta_next = beta_next;
        rec->lnQ = -dbeta * (double)emin + log(Q / (double)Rprev);
        rec->Tn[0] = pa_threshold(beta_next, 4);
        rec->Tn[1] = pa_threshold(beta_next, 8);
        rec->Tn[2] = pa_threshold(beta_next, 12);
    }
}

// ------------------------------------------------------------------ adaptive step
// Overlap of the population with its reweighting by dbeta,
// alpha = (1/R) sum_j min(1, R w_j / sum_k w_k), w_j = pa_exp(-dbeta (E_j - E_min)),
// evaluated per energy level (fixed chunk per thread, fixed tree), and the
// bisection for the largest dbeta in [0, dbeta_max] with alpha >= alpha_star.
constexpr int kRuleThreads = 1024;
constexpr int kRuleCache = 4096; // levels whose weights stay in LDS between the two sums

__device__ double rule_alpha(const uint32_t *__restrict__ hist, int hmin, int nlev, double R, double dbeta,
                             double *wcache, double *sd)
{
    const int chunk = (nlev + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = (int)threadIdx.x * chunk;
    const int hi = lo + chunk < nlev ? lo + chunk : nlev;
    double wsum = 0.0;
    for (int k = lo; k < hi; ++k) {
        const double wv = pa_exp(-(dbeta * (double)(4 * k)));
        if (k < kRuleCache)
            wcache[k] = wv;
        wsum = wsum + (double)hist[hmin + k] * wv;
    }
    const double W = pa_block_sum_f64(wsum, sd);
    double a = 0.0;
    for (int k = lo; k < hi; ++k) {
        const double wv = k < kRuleCache ? wcache[k] : pa_exp(-(dbeta * (double)(4 * k)));
        const double tau = (R * wv) / W;
        a = a + (double)hist[hmin + k] * (tau < 1.0 ? tau : 1.0);
    }
    return pa_block_sum_f64(a, sd) / R;
}

__global__ __launch_bounds__(kRuleThreads) void k_rule(const uint32_t *__restrict__ hist, PaRecord *rec, int DN,
                                                       int64_t Rcur, double alpha_star, double dbeta_max,
                                                       int iterations, int bisect)
{
    __shared__ double sd[16];
    __shared__ double wcache[kRuleCache];
    const int hmin = (rec->emin + DN) >> 2, hmax = (rec->emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    const double R = (double)Rcur;
    double a = rule_alpha(hist, hmin, nlev, R, dbeta_max, wcache, sd);
    double lo = 0.0, hi = dbeta_max, best = dbeta_max, abest = a;
    if (bisect && !(a >= alpha_star)) {
        best = 0.0;
        abest = 1.0;
        for (int it = 0; it < iterations; ++it) {
            const double mid = 0.5 * (lo + hi);
            const double am = rule_alpha(hist, hmin, nlev, R, mid, wcache, sd);
            if (am >= alpha_star) {
                lo = mid;
                abest = am;
            } else {
                hi = mid;
            }
        }
        best = lo;
    }
    if (threadIdx.x == 0) {
        rec->rule_dbeta = best;
        rec->rule_alpha = abest;
    }
}

// ------------------------------------------------------------------ resampling
__device__ __forceinline__ uint64_t weight_of(int32_t e, int DN, int hmin, const uint64_t *wtab)
{
    return wtab[((e + DN) >> 2) - hmin];
}

// Nearest integer: floor(tauhat) + [u S < (R W mod S) 2^32], u = x0 of
// Philox(j, 0, i, RS_NI<<28).
__global__ void k_counts_nearest(const int32_t *__restrict__ E, int64_t Rprev, uint64_t Rt,
                                 const uint64_t *__restrict__ wtab, const PaRecord *__restrict__ rec,
                                 int DN, uint32_t seed, uint32_t run_id, uint32_t step,
                                 uint32_t *__restrict__ r)
{
    const int hmin = (rec->emin + DN) >> 2;
    const uint64_t S = rec->S;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Rprev;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t W = weight_of(E[j], DN, hmin, wtab);
        const uint64_t a = Rt * W;
        const uint64_t qt = a / S;
        const uint64_t rho = a - qt * S;
        const pa_philox_out o = pa_philox(seed, run_id, (uint32_t)j, 0u, step, PA_PURPOSE_RS_NI << 28);
        const bool extra = ((pa_u128)o.x0 * S) < ((pa_u128)rho << 32);
        r[j] = (uint32_t)qt + (extra ? 1u : 0u);
    }
}

// Poisson by inversion; tauhat > 32 is cut into ceil(tauhat/32) equal pieces,
// piece p using u from Philox(j, p, i, RS_POIS<<28).
__global__ void k_counts_poisson(const int32_t *__restrict__ E, int64_t Rprev, uint64_t Rt,
                                 const uint64_t *__restrict__ wtab, const PaRecord *__restrict__ rec,
                                 int DN, uint32_t seed, uint32_t run_id, uint32_t step,
                                 uint32_t *__restrict__ r)
{
    const int hmin = (rec->emin + DN) >> 2;
    const uint64_t S = rec->S;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Rprev;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t W = weight_of(E[j], DN, hmin, wtab);
        const double tau = ((double)W / (double)S) * (double)Rt;
        uint32_t m = 1;
        if (tau > 32.0)
            m = (uint32_t)ceil(tau / 32.0);
        const double mu = tau / (double)m;
        uint32_t tot = 0;
        for (uint32_t p = 0; p < m; ++p) {
            const pa_philox_out o = pa_philox(seed, run_id, (uint32_t)j, p, step, PA_PURPOSE_RS_POIS << 28);
            const double u = ((double)(o.x0 >> 5) * 67108864.0 + (double)(o.x1 >> 6)) *
                             (1.0 / 9007199254740992.0);
            uint32_t k = 0;
            double pr = pa_exp(-mu);
            double F = pr;
            while (u >= F) {
                k += 1;
                pr = (pr * mu) / (double)k;
                const double Fn = F + pr;
                if (Fn == F)
                    break;
                F = Fn;
            }
            tot += k;
        }
        r[j] = tot;
    }
}

__global__ void k_weights(const int32_t *__restrict__ E, int64_t Rprev, const uint64_t *__restrict__ wtab,
                          const PaRecord *__restrict__ rec, int DN, uint64_t *__restrict__ C)
{
    const int hmin = (rec->emin + DN) >> 2;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Rprev;
         j += (int64_t)gridDim.x * blockDim.x)
        C[j] = weight_of(E[j], DN, hmin, wtab);
}

// Systematic: #points (k + U/2^32) S/R below c, k < R, is
// min(R, q + [rho 2^32 > U S]) with c R = q S + rho.
__device__ __forceinline__ uint64_t sys_below(uint64_t c, uint64_t Rt, uint64_t S, uint32_t U)
{
    const pa_u128 cR = (pa_u128)c * Rt;
    uint64_t q = (uint64_t)floor(((double)c * (double)Rt) / (double)S);
    if (q > Rt)
        q = Rt;
    while (q > 0 && (pa_u128)q * S > cR)
        --q;
    while ((pa_u128)(q + 1) * S <= cR)
        ++q;
    const uint64_t rho = (uint64_t)(cR - (pa_u128)q * S);
    const uint64_t n = q + ((((pa_u128)rho) << 32) > ((pa_u128)U * S) ? 1u : 0u);
    return n < Rt ? n : Rt;
}

__global__ void k_counts_systematic(const uint64_t *__restrict__ C, int64_t Rprev, uint64_t Rt,
                                    const PaRecord *__restrict__ rec, uint32_t seed, uint32_t run_id,
                                    uint32_t step, uint32_t *__restrict__ r)
{
    const uint64_t S = rec->S;
    const uint32_t U = pa_philox(seed, run_id, 0u, 0u, step, PA_PURPOSE_RS_SYS << 28).x0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Rprev;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t hi = sys_below(C[j], Rt, S, U);
        const uint64_t lo = j > 0 ? sys_below(C[j - 1], Rt, S, U) : 0;
        r[j] = (uint32_t)(hi - lo);
    }
}

// Multinomial: U_k = floor(r S / 2^128), r = 128 bits of Philox(k, 0, i,
// RS_MULT<<28); the box of replica j is [C_{j-1}, C_j).
__global__ void k_counts_multinomial(const uint64_t *__restrict__ C, int64_t Rprev, uint64_t Rt,
                                     const PaRecord *__restrict__ rec, uint32_t seed, uint32_t run_id,
                                     uint32_t step, uint32_t *__restrict__ r)
{
    const uint64_t S = rec->S;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (int64_t)Rt;
         k += (int64_t)gridDim.x * blockDim.x) {
        const pa_philox_out o = pa_philox(seed, run_id, (uint32_t)k, 0u, step, PA_PURPOSE_RS_MULT << 28);
        const uint64_t lo = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
        const uint64_t hi = (uint64_t)o.x2 | ((uint64_t)o.x3 << 32);
        const pa_u128 A = (pa_u128)lo * S, B = (pa_u128)hi * S;
        const uint64_t U = (uint64_t)((B + (A >> 64)) >> 64);
        int64_t a = 0, b = Rprev - 1;
        while (a < b) {
            const int64_t mid = a + ((b - a) >> 1);
            if (C[mid] > U)
                b = mid;
            else
                a = mid + 1;
        }
        atomicAdd(&r[a], 1u);
    }
}

// Sampling variance, Eq. (5): fixed blocks of contiguous replicas, fixed
// per-thread stride, fixed tree; partial[b] of block b.
__global__ __launch_bounds__(kThreads) void k_sv_partial(const int32_t *__restrict__ E, int64_t Rprev,
                                                          uint64_t Rt, const uint64_t *__restrict__ wtab,
                                                          const PaRecord *__restrict__ rec, int DN,
                                                          const uint32_t *__restrict__ r,
                                                          double *__restrict__ partial)
{
    __shared__ double sd[16];
    const int hmin = (rec->emin + DN) >> 2;
    const double S = (double)rec->S;
    const int64_t chunk = (Rprev + gridDim.x - 1) / gridDim.x;
    const int64_t beg = blockIdx.x * chunk;
    const int64_t end = beg + chunk < Rprev ? beg + chunk : Rprev;
    double acc = 0.0;
    for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
        const double tau = ((double)weight_of(E[j], DN, hmin, wtab) / S) * (double)Rt;
        const double dlt = (double)r[j] - tau;
        acc = acc + dlt * dlt;
    }
    const double t = pa_block_sum_f64(acc, sd);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = t;
}

// Decoupled look-back scan (Merrill & Garland 2016): tiles take their order
// from an atomic ticket, so every tile a tile waits on is already running.
template <typename T, bool INCLUSIVE>
__global__ __launch_bounds__(PA_SCAN_THREADS) void k_scan(const T *__restrict__ in, T *__restrict__ out,
                                                          int64_t n, PaScanTile *tiles, uint32_t *ticket,
                                                          unsigned long long *total, uint32_t *err)
{
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_wave[PA_SCAN_THREADS / 64];
    __shared__ unsigned long long s_excl;
    if (threadIdx.x == 0)
        s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * PA_SCAN_TILE + (int64_t)threadIdx.x * PA_SCAN_ITEMS;
    unsigned long long v[PA_SCAN_ITEMS];
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < PA_SCAN_ITEMS; ++k) {
        const int64_t i = base + k;
        v[k] = i < n ? (unsigned long long)in[i] : 0ull;
        run += v[k];
    }
    // exclusive prefix of the thread totals within the tile
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = (unsigned long long)__shfl_up((long long)incl, off, 64);
        if (lane >= off)
            incl += o;
    }
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    unsigned long long wave_off = 0, agg = 0;
    for (int k = 0; k < PA_SCAN_THREADS / 64; ++k) {
        if (k < wave)
            wave_off += s_wave[k];
        agg += s_wave[k];
    }
    const unsigned long long thread_excl = wave_off + incl - run;
    if (threadIdx.x == 0) {
        PaScanTile *me = tiles + tile;
        unsigned long long excl = 0;
        if (tile == 0) {
            me->incl = agg;
            pa_store_release(&me->flag, 2u);
        } else {
            me->agg = agg;
            pa_store_release(&me->flag, 1u);
            int64_t p = (int64_t)tile - 1;
            while (p >= 0) {
                uint32_t f;
                uint32_t spins = 0;
                while ((f = pa_load_acquire(&tiles[p].flag)) == 0u) {
                    if (++spins > (1u << 26)) {
                        atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (f == 2u) {
                    excl += tiles[p].incl;
                    break;
                }
                if (f == 0u)
                    break; // gave up; the error flag is set
                excl += tiles[p].agg;
                --p;
            }
            me->incl = excl + agg;
            pa_store_release(&me->flag, 2u);
        }
        s_excl = excl;
        if ((int64_t)(tile + 1) * PA_SCAN_TILE >= n)
            *total = excl + agg;
    }
    __syncthreads();
    unsigned long long acc = s_excl + thread_excl;
#pragma unroll
    for (int k = 0; k < PA_SCAN_ITEMS; ++k) {
        const int64_t i = base + k;
        if (INCLUSIVE)
            acc += v[k];
        if (i < n)
            out[i] = (T)acc;
        if (!INCLUSIVE)
            acc += v[k];
    }
}

template <typename T, bool INCLUSIVE>
hipError_t scan(const T *in, T *out, int64_t n, const PaDev &dv, unsigned long long *total,
                hipStream_t st)
{
    const int64_t ntiles = (n + PA_SCAN_TILE - 1) / PA_SCAN_TILE;
    hipError_t e = fill_u32(reinterpret_cast<uint32_t *>(dv.tiles), ntiles * (int64_t)(sizeof(PaScanTile) / 4),
                            0u, st);
    if (e != hipSuccess)
        return e;
    if ((e = fill_u32(dv.ticket, 1, 0u, st)) != hipSuccess)
        return e;
    k_scan<T, INCLUSIVE><<<(unsigned)ntiles, PA_SCAN_THREADS, 0, st>>>(in, out, n, dv.tiles, dv.ticket,
                                                                      total, &dv.rec->err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ apply
__global__ void k_ancestors(const uint32_t *__restrict__ r, const uint32_t *__restrict__ P, int64_t Rprev,
                            uint32_t *__restrict__ anc)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Rprev;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = r[j], p = P[j];
        for (uint32_t k = 0; k < c; ++k)
            anc[p + k] = (uint32_t)j;
    }
}

__global__ void k_gather_rep(const uint32_t *__restrict__ anc, int64_t Rnew, const int32_t *__restrict__ E0,
                             const int32_t *__restrict__ M0, const uint32_t *__restrict__ L0,
                             int32_t *__restrict__ E1, int32_t *__restrict__ M1, uint32_t *__restrict__ L1)
{
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < Rnew;
         d += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t a = anc[d];
        E1[d] = E0[a];
        M1[d] = M0[a];
        L1[d] = L0[a];
    }
}

// Destination word column w takes the bits of its 64 ancestors.  Ancestors are
// non-decreasing, so the column splits into runs of consecutive source bits
// within one source word; each run is one shift-and-mask per site.
__global__ __launch_bounds__(kThreads) void k_gather_spins(const uint64_t *__restrict__ src,
                                                           uint64_t *__restrict__ dst,
                                                           const uint32_t *__restrict__ anc, int64_t Rnew,
                                                           int N)
{
    __shared__ uint32_t r_word[64];
    __shared__ uint32_t r_shift[64], r_b0[64], r_len[64];
    __shared__ int s_nruns;
    const uint32_t w = blockIdx.x;
    if (threadIdx.x < 64) {
        const int b = threadIdx.x;
        const int64_t d = 64 * (int64_t)w + b;
        const bool valid = d < Rnew;
        const uint32_t a = valid ? anc[d] : 0u;
        const uint32_t ap = (uint32_t)__shfl_up((int)a, 1, 64);
        const bool start = valid && (b == 0 || a != ap + 1u || (a & 63u) == 0u);
        const uint64_t sm = __ballot(start);
        const uint64_t vm = __ballot(valid);
        if (start) {
            const int idx = __popcll(sm & ((1ull << b) - 1ull));
            const uint64_t above = b == 63 ? 0ull : ((sm | ~vm) & ~((2ull << b) - 1ull));
            const int end = above ? __ffsll((long long)above) - 1 : 64;
            r_word[idx] = a >> 6;
            r_shift[idx] = a & 63u;
            r_b0[idx] = (uint32_t)b;
            r_len[idx] = (uint32_t)(end - b);
        }
        if (b == 0)
            s_nruns = __popcll(sm);
    }
    __syncthreads();
    const int nr = s_nruns;
    for (int s = threadIdx.x; s < N; s += blockDim.x) {
        uint64_t out = 0, v = 0;
        uint32_t last = 0xFFFFFFFFu;
        for (int i = 0; i < nr; ++i) {
            const uint32_t sw = r_word[i];
            if (sw != last) {
                v = src[(size_t)sw * N + s];
                last = sw;
            }
            const uint32_t len = r_len[i];
            const uint64_t mask = len >= 64 ? ~0ull : ((1ull << len) - 1ull);
            out |= ((v >> r_shift[i]) & mask) << r_b0[i];
        }
        dst[(size_t)w * N + s] = out;
    }
}

__global__ __launch_bounds__(kThreads) void k_commit(PaRecord *rec, const double *__restrict__ partial,
                                                     int nparts, int64_t Rprev, int64_t Rnew)
{
    __shared__ double sd[16];
    double v = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x)
        v = v + partial[k];
    const double t = pa_block_sum_f64(v, sd);
    if (threadIdx.x == 0) {
        rec->sv = t / (double)Rprev;
        rec->lnZ = rec->lnZ + rec->lnQ;
        rec->T[0] = rec->Tn[0];
        rec->T[1] = rec->Tn[1];
        rec->T[2] = rec->Tn[2];
        rec->Rprev = (uint64_t)Rprev;
        rec->Rnew = (uint64_t)Rnew;
    }
}

// ------------------------------------------------------------------ step 4: observables
__global__ void k_obs_prep(uint32_t *fam, int64_t R0, PaRecord *rec)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < R0;
         i += (int64_t)gridDim.x * blockDim.x)
        fam[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rec->sumE = rec->sumE2 = rec->sumAbsM = rec->sumM2 = rec->sumC2 = rec->families = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_obs_rep(const int32_t *__restrict__ E, const int32_t *__restrict__ M,
                                                      const uint32_t *__restrict__ label, int64_t R,
                                                      uint32_t *fam, PaRecord *rec)
{
    __shared__ uint64_t su[16];
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0;
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < R;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = E[d], m = M[d];
        sE += (uint64_t)e;
        sE2 += (uint64_t)(e * e);
        sA += (uint64_t)(m < 0 ? -m : m);
        sM2 += (uint64_t)(m * m);
        atomicAdd(&fam[label[d]], 1u);
    }
    sE = pa_block_sum_u64(sE, su);
    sE2 = pa_block_sum_u64(sE2, su);
    sA = pa_block_sum_u64(sA, su);
    sM2 = pa_block_sum_u64(sM2, su);
    if (threadIdx.x == 0) {
        atomicAdd(&rec->sumE, (unsigned long long)sE);
        atomicAdd(&rec->sumE2, (unsigned long long)sE2);
        atomicAdd(&rec->sumAbsM, (unsigned long long)sA);
        atomicAdd(&rec->sumM2, (unsigned long long)sM2);
    }
}

__global__ __launch_bounds__(kThreads) void k_obs_fam(const uint32_t *__restrict__ fam, int64_t R0,
                                                      PaRecord *rec, double *__restrict__ partial)
{
    __shared__ uint64_t su[16];
    __shared__ double sd[16];
    const int64_t chunk = (R0 + gridDim.x - 1) / gridDim.x;
    const int64_t beg = blockIdx.x * chunk;
    const int64_t end = beg + chunk < R0 ? beg + chunk : R0;
    uint64_t c2 = 0, nf = 0;
    double cl = 0.0;
    for (int64_t f = beg + threadIdx.x; f < end; f += blockDim.x) {
        const uint64_t c = fam[f];
        c2 += c * c;
        if (c) {
            nf += 1;
            cl = cl + (double)c * log((double)c);
        }
    }
    c2 = pa_block_sum_u64(c2, su);
    nf = pa_block_sum_u64(nf, su);
    cl = pa_block_sum_f64(cl, sd);
    if (threadIdx.x == 0) {
        atomicAdd(&rec->sumC2, (unsigned long long)c2);
        atomicAdd(&rec->families, (unsigned long long)nf);
        partial[blockIdx.x] = cl;
    }
}

// Averages of step 4 and the family statistics: rho_t = sum_k c_k^2 / R
// (Eq. (6) with n_k = c_k / R), S_f = ln R - (1/R) sum_k c_k ln c_k.
__global__ __launch_bounds__(kThreads) void k_obs_final(PaRecord *rec, const double *__restrict__ partial,
                                                        int nparts, int N, int64_t R)
{
    __shared__ double sd[16];
    double v = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x)
        v = v + partial[k];
    const double t = pa_block_sum_f64(v, sd);
    if (threadIdx.x == 0) {
        const double n = (double)N, r = (double)R;
        rec->sumClnC = t;
        rec->e = (double)(long long)rec->sumE / (n * r);
        rec->e2 = (double)(long long)rec->sumE2 / (n * n * r);
        rec->abs_m = (double)(long long)rec->sumAbsM / (n * r);
        rec->m2 = (double)(long long)rec->sumM2 / (n * n * r);
        rec->rho_t = (double)rec->sumC2 / r;
        rec->S_f = log(r) - t / r;
    }
}

// ------------------------------------------------------------------ overlap
// Pairs replica d of population a with replica d of b: per word column, the
// bit-sliced count of differing sites per replica, then q-histogram entry
// N - count.
__global__ __launch_bounds__(kThreads) void k_overlap(const uint64_t *__restrict__ A,
                                                      const uint64_t *__restrict__ B, int N, int64_t R,
                                                      unsigned long long *hist)
{
    __shared__ uint64_t red[kThreads / 64][16];
    const uint32_t w = blockIdx.x;
    uint64_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t c16[16];
    // up to 255 sites per thread in 8 planes: N <= 16384 with 256 threads -> 64
    for (int s = threadIdx.x; s < N; s += blockDim.x)
        vadd8(v, A[(size_t)w * N + s] ^ B[(size_t)w * N + s]);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        c16[k] = k < 8 ? v[k] : 0;
    wave_vsum16(c16);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 16; ++k)
            red[wave][k] = c16[k];
    __syncthreads();
    if (wave == 0) {
        uint32_t cnt = 0;
        for (int q = 0; q < nw; ++q)
            for (int k = 0; k < 16; ++k)
                cnt += (uint32_t)((red[q][k] >> lane) & 1u) << k;
        const int64_t d = 64 * (int64_t)w + lane;
        if (d < R)
            atomicAdd(&hist[N - (int)cnt], 1ull);
    }
}

// Thresholds of an imported inverse temperature.
__global__ void k_set_beta(PaRecord *rec, double beta, double lnZ)
{
    if (threadIdx.x == 0) {
        rec->T[0] = pa_threshold(beta, 4);
        rec->T[1] = pa_threshold(beta, 8);
        rec->T[2] = pa_threshold(beta, 12);
        rec->lnZ = lnZ;
        rec->sv = 0.0;
    }
}

} // namespace

// ====================================================================== launchers
size_t pa_sweep_lds_bytes(int N) { return ((size_t)N * 9 + 7) & ~(size_t)7; }

static int sweep_threads(int N)
{
    int t = ((N / 2 + 63) / 64) * 64;
    return t > kThreads ? kThreads : (t < 64 ? 64 : t);
}

hipError_t pa_launch_init(const PaLaunch &p, const PaDev &dv, int cur)
{
    const int64_t W = (p.R0 + 63) / 64;
    k_init_spins<<<grid_for(W * p.N), kThreads, 0, p.stream>>>(dv.spins[cur], p.N, W, p.seed, p.run_id);
    k_init_labels<<<grid_for(p.R0), kThreads, 0, p.stream>>>(dv.label[cur], p.R0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return pa_launch_sweep(p, dv, cur, p.R0, 0u, 0u, 0);
}

hipError_t pa_launch_sweep(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, uint32_t step,
                           uint32_t t0, int theta)
{
    const unsigned W = (unsigned)((Rcur + 63) / 64);
    const size_t lds = pa_sweep_lds_bytes(p.N);
    const int th = sweep_threads(p.N);
    if (p.d == 2)
        k_sweep<2><<<W, th, lds, p.stream>>>(dv.spins[cur], dv.jmask, p.L, p.N, dv.E[cur], dv.M[cur], Rcur,
                                             dv.rec, p.seed, p.run_id, step, t0, theta);
    else
        k_sweep<3><<<W, th, lds, p.stream>>>(dv.spins[cur], dv.jmask, p.L, p.N, dv.E[cur], dv.M[cur], Rcur,
                                             dv.rec, p.seed, p.run_id, step, t0, theta);
    return hipGetLastError();
}

hipError_t pa_launch_reweight(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, double dbeta,
                              double beta_next)
{
    const int DN = p.d * p.N;
    k_hist_prep<<<grid_for(p.H), kThreads, 0, p.stream>>>(dv.hist, p.H, dv.rec);
    const int g = grid_for(Rcur, 4096, 1024);
    k_hist<<<g, kThreads, (size_t)p.H * 4, p.stream>>>(dv.E[cur], Rcur, DN, p.H, dv.hist, dv.rec);
    k_reweight<<<1, 1024, 0, p.stream>>>(dv.hist, dv.wtab, dv.rec, DN, Rcur, dbeta, beta_next);
    return hipGetLastError();
}

hipError_t pa_launch_counts(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rprev, int64_t Rt,
                            int scheme, uint32_t step)
{
    const int DN = p.d * p.N;
    const int g = grid_for(Rprev);
    hipError_t e;
    switch (scheme) {
    case 2:
        k_counts_nearest<<<g, kThreads, 0, p.stream>>>(dv.E[cur], Rprev, (uint64_t)Rt, dv.wtab, dv.rec, DN, p.seed,
                                                       p.run_id, step, dv.r);
        break;
    case 1:
        k_counts_poisson<<<g, kThreads, 0, p.stream>>>(dv.E[cur], Rprev, (uint64_t)Rt, dv.wtab, dv.rec, DN, p.seed,
                                                       p.run_id, step, dv.r);
        break;
    case 3:
    case 0:
        k_weights<<<g, kThreads, 0, p.stream>>>(dv.E[cur], Rprev, dv.wtab, dv.rec, DN, dv.C);
        if ((e = scan<uint64_t, true>(dv.C, dv.C, Rprev, dv, &dv.rec->Ctot, p.stream)) != hipSuccess)
            return e;
        if (scheme == 3) {
            k_counts_systematic<<<g, kThreads, 0, p.stream>>>(dv.C, Rprev, (uint64_t)Rt, dv.rec, p.seed, p.run_id,
                                                              step, dv.r);
        } else {
            if ((e = fill_u32(dv.r, Rprev, 0u, p.stream)) != hipSuccess)
                return e;
            k_counts_multinomial<<<grid_for(Rt), kThreads, 0, p.stream>>>(dv.C, Rprev, (uint64_t)Rt, dv.rec, p.seed,
                                                                          p.run_id, step, dv.r);
        }
        break;
    default:
        return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    k_sv_partial<<<PA_RED_BLOCKS, kThreads, 0, p.stream>>>(dv.E[cur], Rprev, (uint64_t)Rt, dv.wtab, dv.rec, DN,
                                                           dv.r, dv.partial);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    return scan<uint32_t, false>(dv.r, dv.P, Rprev, dv, reinterpret_cast<unsigned long long *>(&dv.rec->Rnew),
                                 p.stream);
}

hipError_t pa_launch_apply(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rprev, int64_t Rnew)
{
    const int nxt = cur ^ 1;
    k_ancestors<<<grid_for(Rprev), kThreads, 0, p.stream>>>(dv.r, dv.P, Rprev, dv.anc);
    k_gather_rep<<<grid_for(Rnew), kThreads, 0, p.stream>>>(dv.anc, Rnew, dv.E[cur], dv.M[cur], dv.label[cur],
                                                            dv.E[nxt], dv.M[nxt], dv.label[nxt]);
    const unsigned W = (unsigned)((Rnew + 63) / 64);
    k_gather_spins<<<W, kThreads, 0, p.stream>>>(dv.spins[cur], dv.spins[nxt], dv.anc, Rnew, p.N);
    k_commit<<<1, kThreads, 0, p.stream>>>(dv.rec, dv.partial, PA_RED_BLOCKS, Rprev, Rnew);
    return hipGetLastError();
}

hipError_t pa_launch_observables(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur)
{
    k_obs_prep<<<grid_for(p.R0), kThreads, 0, p.stream>>>(dv.fam, p.R0, dv.rec);
    k_obs_rep<<<grid_for(Rcur, kThreads, 1024), kThreads, 0, p.stream>>>(dv.E[cur], dv.M[cur], dv.label[cur],
                                                                         Rcur, dv.fam, dv.rec);
    k_obs_fam<<<PA_RED_BLOCKS, kThreads, 0, p.stream>>>(dv.fam, p.R0, dv.rec, dv.partial);
    k_obs_final<<<1, kThreads, 0, p.stream>>>(dv.rec, dv.partial, PA_RED_BLOCKS, p.N, Rcur);
    return hipGetLastError();
}

hipError_t pa_launch_overlap(const PaLaunch &p, const uint64_t *a, const uint64_t *b, int64_t R,
                             unsigned long long *hist)
{
    const unsigned W = (unsigned)((R + 63) / 64);
    k_overlap<<<W, kThreads, 0, p.stream>>>(a, b, p.N, R, hist);
    return hipGetLastError();
}

hipError_t pa_launch_rule(const PaLaunch &p, const PaDev &dv, int cur, int64_t Rcur, double alpha_star,
                          double dbeta_max, int iterations, int bisect)
{
    const int DN = p.d * p.N;
    k_hist_prep<<<grid_for(p.H), kThreads, 0, p.stream>>>(dv.hist, p.H, dv.rec);
    k_hist<<<grid_for(Rcur, 4096, 1024), kThreads, (size_t)p.H * 4, p.stream>>>(dv.E[cur], Rcur, DN, p.H, dv.hist,
                                                                                dv.rec);
    k_rule<<<1, kRuleThreads, 0, p.stream>>>(dv.hist, dv.rec, DN, Rcur, alpha_star, dbeta_max, iterations, bisect);
    return hipGetLastError();
}

hipError_t pa_launch_set_beta(const PaLaunch &p, const PaDev &dv, double beta, double lnZ)
{
    k_set_beta<<<1, 64, 0, p.stream>>>(dv.rec, beta, lnZ);
    return hipGetLastError();
}

// ROCm lets a launch use dynamic LDS up to the device's per-workgroup limit
// without a per-function attribute; only the limit is needed here.
hipError_t pa_configure_kernels(int *max_lds)
{
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess)
        return e;
    *max_lds = v;
    return hipSuccess;
}
