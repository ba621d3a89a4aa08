// HIP kernels of the population-annealing hot path for gfx950 (MI355X).
//
// Spins are multi-spin coded: bit b of word [w][s] is replica 64w+b at site s,
// 1 meaning sigma = -1.  One workgroup owns one 64-replica word column: the
// whole lattice of its 64 replicas (N words) sits in LDS while it is swept.
//
// Every kernel serves a batch of runs through a block map (PaBlk: run, index
// within the run); a run's population size, ping-pong index, temperature and
// step are read from its device record, so launches need no host knowledge
// of the state and a whole anneal can be captured in a graph.  Grids cover
// each run's capacity; workgroups past the live population return at once.
#include "pa_sweep.h"

#include <climits>
#include <mutex>
#include <type_traits>

namespace {

// ------------------------------------------------------------------ helpers
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

// ------------------------------------------------------------------ step 1: init
// Record of a fresh run at beta_0 = 0: ln Z_0 = N ln 2, every move accepted.
__global__ void k_init_rec(const PaRunDesc *__restrict__ runs)
{
    const PaRunDesc &rd = runs[blockIdx.x];
    if (threadIdx.x != 0)
        return;
    PaRecord *rec = rd.dv.rec;
    rec->cur = 0;
    rec->status = 0;
    rec->skip = 0;
    rec->step = 0;
    rec->sweeps = 0;
    rec->gather = 0;
    rec->Rcur = (uint64_t)rd.R0;
    rec->beta = 0.0;
    rec->lnQ = 0.0;
    rec->lnZ = (double)rd.N * 0x1.62e42fefa39efp-1; // N * RN(ln 2)
    rec->sv = 0.0;
    for (int k = 0; k < 3; ++k)
        rec->T[k] = rec->Tn[k] = 1ull << 32;
    rec->philox_calls = 0;
    rec->site_updates = 0;
    rec->attempts = 0;
    rec->accE = rec->accE2 = rec->accAbsM = rec->accM2 = rec->accC2 = rec->accFam = 0;
    rec->accE3[0] = rec->accE3[1] = 0;
    rec->lnq_hist[0] = rec->lnq_hist[1] = rec->lnq_hist[2] = 0.0;
    rec->S_f = log((double)rd.R0);
    rec->weighted = 0;
    rec->keep = 0;
    rec->resamplings = 0;
    rec->ess = (double)rd.R0;
}

// Replica 64w+b, site s: bit b of x0 | x1<<32 of Philox(s, w, 0, INIT<<28).
__global__ __launch_bounds__(kThreads) void k_init_spins(const PaRunDesc *__restrict__ runs,
                                                         const PaBlk *__restrict__ map)
{
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    const uint32_t w = b.idx;
    if ((int64_t)w * 64 >= rd.R0)
        return;
    uint64_t *g = rd.dv.spins[0] + (size_t)w * rd.N;
    for (int s = threadIdx.x; s < rd.N; s += blockDim.x) {
        const pa_philox_out o = pa_philox(rd.seed, rd.run_id, (uint32_t)s, w, 0u, PA_PURPOSE_INIT << 28);
        g[s] = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
    }
}

__global__ __launch_bounds__(kThreads) void k_init_labels(const PaRunDesc *__restrict__ runs,
                                                          const PaBlk *__restrict__ map)
{
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    const int64_t beg = (int64_t)b.idx * PA_CHUNK;
    for (int64_t j = beg + threadIdx.x; j < beg + PA_CHUNK && j < rd.R0; j += blockDim.x) {
        rd.dv.label[0][j] = (uint32_t)j;
        rd.dv.fam[j] = 0; // family counts start at zero; k_obs_fam returns them to zero
    }
}


// ------------------------------------------------------------------ cluster updates
// The cluster-update driver (Sec. 1 names cluster updates among the update
// algorithms the scheme can use): nsteps Wolff single-cluster updates of
// every replica at the run's current beta.  For replica b of column w at
// (step i, update t):
//  - seed site floor(x0 N / 2^32), x0 of Philox(b, w, i, WSEED<<28 | t<<8);
//  - bond (s, mu) to s + e_mu active iff satisfied and u < T_p, T_p =
//    min(2^32, floor(2^32 (1 - pa_exp(-2 beta)))), u's bits from the planes
//    of Philox(s, w, i, WBOND<<28 | t<<8 | mu<<4 | q), q = 0..15, decided
//    from the most significant bit as for the Metropolis thresholds;
//  - the cluster is every site joined to the seed by active bonds; it flips.
// Growth is bit-parallel over the 64 replicas: each pass, every site takes
// the replicas newly added at a neighbour last pass (frontier F) across
// satisfied bonds whose activity the pass decides for just those replicas;
// a site writes only its own words, and a (bond, replica) pair is decided at
// most once.  The component does not depend on the order of growth.

// Activity of bond (owner, mu) for the replicas in cnd.
__device__ __forceinline__ uint64_t wolff_bond(const PlaneCtx &pc, uint32_t owner, uint32_t mu, uint64_t cnd,
                                               uint64_t T)
{
    if (T >= (1ull << 32))
        return cnd;
    if (T == 0)
        return 0;
    uint64_t und = cnd, acc = 0;
    for (uint32_t q = 0; q < 16u && und != 0; ++q) {
        const pa_philox_out o = pa_philox(pc.seed, pc.run_id, owner, pc.w, pc.step,
                                          (PA_PURPOSE_WBOND << 28) | (pc.t << 8) | (mu << 4) | q);
        const int b0 = 31 - 2 * (int)q;
        pair_core<false>(o, tbit((uint32_t)T, b0), tbit((uint32_t)T, b0 - 1), und, und, acc);
    }
    return acc;
}

// Bond decisions are batched per wave: a site's candidate bonds (site,
// direction k = 2 mu + [towards -e_mu], candidate replicas) go to a queue
// and are decided 64 at a time, one per lane, so that a decision does not
// run a whole wave for the one lane that needs it.
constexpr int kClusterQueue = 128; // per wave; never more than 127 items are live
// Lanes of a cluster-update workgroup: one workgroup per CU fits in LDS, so
// its waves are all the latency hiding there is.
constexpr int kClusterThreads = 1024;

struct ClusterQueue {
    uint32_t *sk;  // site | k << 16
    uint64_t *cnd; // candidate replicas
};

__device__ __forceinline__ uint32_t cluster_push(const ClusterQueue &Q, uint32_t head, uint32_t cnt, bool has,
                                                 uint32_t sk, uint64_t cnd)
{
    const uint64_t bal = __ballot(has);
    if (has) {
        const uint32_t slot = (head + cnt + (uint32_t)__popcll(bal & lanemask_lt())) & (kClusterQueue - 1);
        Q.sk[slot] = sk;
        Q.cnd[slot] = cnd;
    }
    __builtin_amdgcn_wave_barrier();
    return cnt + (uint32_t)__popcll(bal);
}

// Decides up to 64 queued bonds and adds the replicas they join to Fn[site].
template <int D>
__device__ __forceinline__ void cluster_pass(const ClusterQueue &Q, const PlaneCtx &pc, uint64_t T, uint64_t *Fn,
                                             int L, int LL, uint32_t mL, uint32_t &head, uint32_t &cnt)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t n = cnt < 64u ? cnt : 64u;
    const bool act = lane < n;
    uint32_t sk = 0;
    uint64_t cnd = 0;
    if (act) {
        const uint32_t slot = (head + lane) & (kClusterQueue - 1);
        sk = Q.sk[slot];
        cnd = Q.cnd[slot];
    }
    __builtin_amdgcn_wave_barrier();
    head += n;
    cnt -= n;
    if (act) {
        const int s = (int)(sk & 0xFFFFu), k = (int)(sk >> 16), mu = k >> 1;
        const int row = (int)__umulhi((uint32_t)s, mL);
        const int x = s - row * L;
        const int z = (D == 2) ? 0 : (int)__umulhi((uint32_t)row, mL);
        const int y = row - z * L;
        const int c = mu == 0 ? x : (mu == 1 ? y : z);
        const int st = mu == 0 ? 1 : (mu == 1 ? L : LL);
        // bond (s, mu) to s + e_mu is owned by s, bond (s - e_mu, mu) by s - e_mu
        const int owner = (k & 1) ? (c == 0 ? s + st * (L - 1) : s - st) : s;
        const uint64_t a = wolff_bond(pc, (uint32_t)owner, (uint32_t)mu, cnd, T);
        if (a)
            atomicOr((unsigned long long *)&Fn[s], (unsigned long long)a);
    }
}

template <int D, bool J>
__global__ __launch_bounds__(kClusterThreads) void k_cluster(const PaRunDesc *__restrict__ runs,
                                                      const PaBlk *__restrict__ map, int nsteps, uint32_t t0)
{
    // dynamic LDS: lattice [N] | cluster C [N] | frontiers F0, F1 [N] (at
    // least 32 per wave in all, reused by the recount) | queue candidates
    // [waves][kClusterQueue] u64 | queue sites [waves][kClusterQueue] u32 |
    // jmask [N] bytes
    extern __shared__ uint64_t lat[];
    const PaBlk blk = map[blockIdx.x];
    const PaRunDesc &rd = runs[blk.run];
    PaRecord *rec = rd.dv.rec;
    const uint32_t w = blk.idx;
    const int64_t Rlive = (int64_t)rec->Rcur;
    if ((int64_t)w * 64 >= Rlive || frozen(rec))
        return;
    const int L = uni(rd.L), N = uni(rd.N), LL = L * L;
    const int cur = uni(rec->cur);
    const int tid = threadIdx.x, bs = blockDim.x;
    uint64_t *C = lat + N, *F0 = C + N, *F1 = F0 + N;
    const int nw = bs >> 6, nred = 3 * N > 32 * nw ? 3 * N : 32 * nw;
    uint64_t *qc = lat + N + nred;                                        // [waves][kClusterQueue]
    uint32_t *qs = reinterpret_cast<uint32_t *>(qc + nw * kClusterQueue); // [waves][kClusterQueue]
    uint8_t *jl = reinterpret_cast<uint8_t *>(qs + nw * kClusterQueue);
    const ClusterQueue Q = {qs + (tid >> 6) * kClusterQueue, qc + (tid >> 6) * kClusterQueue};
    uint64_t *g = rd.dv.spins[cur] + (size_t)w * N;
    load_column<J>(lat, jl, g, rd.dv.jmask, N);
    const uint32_t mL = uni((uint32_t)(((1ull << 32) + (uint64_t)L - 1) / (uint64_t)L));
    const double p = 1.0 - pa_exp(-(2.0 * rec->beta));
    const double tf = floor(ldexp(p, 32));
    uint64_t T = (uint64_t)tf;
    if (T > (1ull << 32))
        T = 1ull << 32;
    PlaneCtx pc;
    pc.seed = uni(rd.seed);
    pc.run_id = uni(rd.run_id);
    pc.w = w;
    pc.step = uni(rec->step);
    for (int k = 0; k < nsteps; ++k) {
        pc.t = t0 + (uint32_t)k;
        for (int s = tid; s < N; s += bs)
            C[s] = F0[s] = 0;
        __syncthreads();
        if (tid < 64) { // the seed of replica tid
            const pa_philox_out o = pa_philox(pc.seed, pc.run_id, (uint32_t)tid, w, pc.step,
                                              (PA_PURPOSE_WSEED << 28) | (pc.t << 8));
            const uint32_t s0 = (uint32_t)(((uint64_t)o.x0 * (uint64_t)N) >> 32);
            atomicOr((unsigned long long *)&C[s0], 1ull << tid);
            atomicOr((unsigned long long *)&F0[s0], 1ull << tid);
        }
        __syncthreads();
        uint64_t *Fc = F0, *Fn = F1;
        // every pass that continues adds a (site, replica) pair: at most 64 N
        for (int pass = 0; pass <= 64 * N; ++pass) {
            for (int s = tid; s < N; s += bs)
                Fn[s] = 0;
            __builtin_amdgcn_wave_barrier(); // a wave's queue only adds to its own sites
            uint32_t head = 0, cnt = 0;
            for (int kb = 0; kb < N; kb += bs) {
                const int s = kb + tid;
                const bool in = s < N;
                const int t = in ? s : 0;
                const int row = (int)__umulhi((uint32_t)t, mL);
                const int x = t - row * L;
                const int z = (D == 2) ? 0 : (int)__umulhi((uint32_t)row, mL);
                const int y = row - z * L;
                const uint32_t jb = J ? (uint32_t)jl[t] : 0u;
                const uint64_t S = lat[t], cs = C[t];
#pragma unroll
                for (int k = 0; k < 2 * D; ++k) {
                    const int mu = k >> 1;
                    const int c = mu == 0 ? x : (mu == 1 ? y : z);
                    const int st = mu == 0 ? 1 : (mu == 1 ? L : LL);
                    const int nb = (k & 1) ? (c == 0 ? t + st * (L - 1) : t - st)
                                           : (c == L - 1 ? t - st * (L - 1) : t + st);
                    // the replicas newly added at the neighbour, not yet here,
                    // across a satisfied bond (coupling bit mu or D + mu)
                    uint64_t cnd = in ? Fc[nb] & ~cs : 0;
                    if (cnd)
                        cnd &= ~bond<J>(S, lat[nb], jb, (k & 1) ? D + mu : mu);
                    cnt = cluster_push(Q, head, cnt, cnd != 0, (uint32_t)t | ((uint32_t)k << 16), cnd);
                    while (cnt >= 64u)
                        cluster_pass<D>(Q, pc, T, Fn, L, LL, mL, head, cnt);
                }
            }
            while (cnt > 0u)
                cluster_pass<D>(Q, pc, T, Fn, L, LL, mL, head, cnt);
            __builtin_amdgcn_wave_barrier();
            int any = 0;
            for (int s = tid; s < N; s += bs) {
                const uint64_t add = Fn[s] & ~C[s];
                if (add) {
                    C[s] |= add;
                    any = 1;
                }
                Fn[s] = add;
            }
            if (!__syncthreads_or(any))
                break;
            uint64_t *tmp = Fc;
            Fc = Fn;
            Fn = tmp;
        }
        for (int s = tid; s < N; s += bs)
            lat[s] ^= C[s];
        __syncthreads();
    }
    if (tid == 0 && w == 0) // once per run; no block reads it during the launch
        rec->sweeps = t0 + (uint32_t)nsteps;
    recount_column<D, J>(lat, jl, g, lat + N, rd, cur, w, Rlive, L, N, LL, mL);
}

// The sweep counter advances after the sweeps (a separate launch, so that no
// workgroup of the sweep reads a half-updated counter).
// ------------------------------------------------------------------ step 2: Q
// Energy levels h = (E + dN) / 4: all energies of a run share E mod 4, since a
// flip changes E by a multiple of 4.
__global__ void k_hist_prep(const PaRunDesc *__restrict__ runs)
{
    const PaRunDesc &rd = runs[blockIdx.x];
    for (int i = threadIdx.x; i < rd.H; i += blockDim.x)
        rd.dv.hist[i] = 0;
    if (threadIdx.x == 0) {
        rd.dv.rec->emin = INT_MAX;
        rd.dv.rec->emax = INT_MIN;
    }
}

__global__ __launch_bounds__(kThreads) void k_hist(const PaRunDesc *__restrict__ runs,
                                                   const PaBlk *__restrict__ map)
{
    extern __shared__ uint32_t lh[];
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    const int64_t R = (int64_t)rec->Rcur;
    const int64_t beg = (int64_t)b.idx * PA_HCHUNK;
    if (beg >= R || frozen(rec))
        return;
    const int H = rd.H, DN = rd.d * rd.N;
    const int32_t *E = rd.dv.E[rec->cur];
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        lh[i] = 0;
    __syncthreads();
    int64_t lo = INT_MAX, hi = INT_MIN;
    const int64_t end = beg + PA_HCHUNK < R ? beg + PA_HCHUNK : R;
    for (int64_t j = beg + threadIdx.x; j < end; j += blockDim.x) {
        const int32_t e = E[j];
        atomicAdd(&lh[(e + DN) >> 2], 1u);
        lo = e < lo ? e : lo;
        hi = e > hi ? e : hi;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        if (lh[i])
            atomicAdd(&rd.dv.hist[i], lh[i]);
    // one atomic per workgroup: the wave extremes meet in LDS first
    __shared__ int64_t s_lo[16], s_hi[16];
    lo = pa_wave_min_i64(lo);
    hi = pa_wave_max_i64(hi);
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            lo = s_lo[k] < lo ? s_lo[k] : lo;
            hi = s_hi[k] > hi ? s_hi[k] : hi;
        }
        atomicMin(&rec->emin, (int)lo);
        atomicMax(&rec->emax, (int)hi);
    }
}

__device__ __forceinline__ pa_u128 block_sum_u128(pa_u128 v, uint64_t *su)
{
    pa_u128 t = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t limb = (uint64_t)(v >> (32 * k)) & 0xFFFFFFFFull;
        t += (pa_u128)pa_block_sum_u64(limb, su) << (32 * k);
    }
    return t;
}

// One workgroup per run: weights per level above the lowest, the Q sum in a
// fixed order (contiguous chunk per thread, then the block's fixed tree), S
// and sum_h n_h W_h^2 exactly, ln Q and the Metropolis thresholds of the next
// beta.  A weighted population only gets dbeta and the thresholds here; its
// per-replica passes (k_rw_max, k_rw_sum, k_rw_final) do the rest.
__global__ __launch_bounds__(1024) void k_reweight(const PaRunDesc *__restrict__ runs, double beta_next)
{
    __shared__ uint64_t su[16 * 6];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const int DN = rd.d * rd.N;
    const double dbeta = beta_next - rec->beta;
    const int32_t emin = rec->emin, emax = rec->emax;
    // the resampling that follows starts with clean tile flags, tickets and status
    const int64_t ntiles = 2 * pa_tiles_per_sum(rd.cap);
    for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x)
        rd.dv.tiles[t].word = 0ull;
    const int hmin = (emin + DN) >> 2, hmax = (emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    if (rec->weighted) {
        __syncthreads(); // every thread has read the record before thread 0 writes it
        // the level histogram is not needed any more: back to zero for the next build
        for (int k = threadIdx.x; k < nlev; k += blockDim.x)
            rd.dv.hist[hmin + k] = 0;
        if (threadIdx.x == 0) {
            rec->emin = INT_MAX;
            rec->emax = INT_MIN;
            rec->ticket[0] = rec->ticket[1] = 0u;
            rec->status = 0;
            rec->skip = 0;
            rec->keep = 0;
            rec->wemin = emin;
            rec->dbeta = dbeta;
            rec->beta_next = beta_next;
            rec->S = 0;
            rec->Q2[0] = rec->Q2[1] = 0;
            rec->xmag = ~0ull;
            rec->Tn[0] = pa_threshold(beta_next, 4);
            rec->Tn[1] = pa_threshold(beta_next, 8);
            rec->Tn[2] = pa_threshold(beta_next, 12);
        }
        return;
    }
    const int chunk = (nlev + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = (int)threadIdx.x * chunk;
    const int hi = lo + chunk < nlev ? lo + chunk : nlev;
    double q = 0.0;
    uint64_t s = 0;
    pa_u128 s2 = 0;
    for (int k = lo; k < hi; ++k) {
        const uint32_t n = rd.dv.hist[hmin + k];
        const double wv = pa_exp(-(dbeta * (double)(4 * k)));
        const uint64_t W = (uint64_t)floor(ldexp(wv, 40));
        rd.dv.wtab[k] = W;
        q = q + (double)n * wv;
        s += (uint64_t)n * W;
        s2 += (pa_u128)((uint64_t)n * W) * W;
    }
    // one exchange through LDS for all block sums: Q (a double, the waves'
    // butterfly totals added in wave order, so the same bits every run), S and
    // the four 32-bit limbs of sum n W^2 (a limb's block total stays below 2^42)
    uint64_t x[6] = {s, (uint64_t)s2 & 0xFFFFFFFFull, (uint64_t)(s2 >> 32) & 0xFFFFFFFFull,
                     (uint64_t)(s2 >> 64) & 0xFFFFFFFFull, (uint64_t)(s2 >> 96),
                     (uint64_t)__double_as_longlong(pa_wave_sum_f64(q))};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        x[i] = pa_wave_sum_u64(x[i]);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i)
            su[wave * 6 + i] = x[i];
    __syncthreads(); // also: every level has been read
    double Q = 0.0;
    uint64_t t[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nwaves; ++k) {
#pragma unroll
        for (int i = 0; i < 5; ++i)
            t[i] += su[k * 6 + i];
        Q = Q + __longlong_as_double((long long)su[k * 6 + 5]);
    }
    const uint64_t S = t[0];
    const pa_u128 S2 = (pa_u128)t[1] + ((pa_u128)t[2] << 32) + ((pa_u128)t[3] << 64) + ((pa_u128)t[4] << 96);
    // back to zero for the next build of the level histogram
    for (int k = threadIdx.x; k < nlev; k += blockDim.x)
        rd.dv.hist[hmin + k] = 0;
    // the record's new values, the exponentials on separate lanes
    if (threadIdx.x == 0) {
        rec->emin = INT_MAX;
        rec->emax = INT_MIN;
        rec->ticket[0] = rec->ticket[1] = 0u;
        rec->status = 0;
        rec->skip = 0;
        rec->keep = 0;
        rec->wemin = emin;
        rec->qsum = Q;
        rec->S = S;
        rec->Q2[0] = (uint64_t)S2;
        rec->Q2[1] = (uint64_t)(S2 >> 64);
        rec->dbeta = dbeta;
        rec->beta_next = beta_next;
        rec->lnQ = -dbeta * (double)emin + log(Q / (double)rec->Rcur);
    } else if (threadIdx.x < 4) {
        rec->Tn[threadIdx.x - 1] = pa_threshold(beta_next, 4 * (int)threadIdx.x);
    }
}

// ------------------------------------------------------------------ adaptive step
// Overlap of the population with its reweighting by dbeta, with the integer
// weights the resampling uses: W_h = floor(2^40 pa_exp(-dbeta 4(h - hmin)))
// per energy level, S = sum_h n_h W_h, and
//   alpha = sum_h n_h min(S, R W_h) / (R S)
// exactly (integer sums, so any order gives the same numbers).  The bisection
// keeps the largest dbeta in [0, dbeta_max] with 2^32 num >= A R S, A the
// target overlap in units of 2^-32.
__device__ __forceinline__ double u128_to_double(pa_u128 x)
{
    return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}

struct Overlap {
    pa_u128 num, den;
};

__device__ Overlap rule_overlap(const uint32_t *__restrict__ hist, int hmin, int nlev, uint64_t R, double dbeta,
                                uint64_t *wcache, uint64_t *su)
{
    const int chunk = (nlev + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = (int)threadIdx.x * chunk;
    const int hi = lo + chunk < nlev ? lo + chunk : nlev;
    uint64_t s = 0;
    for (int k = lo; k < hi; ++k) {
        const uint64_t W = pa_weight(dbeta, 4 * k);
        if (k < kRuleCache)
            wcache[k] = W;
        s += (uint64_t)hist[hmin + k] * W;
    }
    const uint64_t S = pa_block_sum_u64(s, su);
    pa_u128 a = 0;
    for (int k = lo; k < hi; ++k) {
        const uint64_t W = k < kRuleCache ? wcache[k] : pa_weight(dbeta, 4 * k);
        const uint64_t RW = R * W;
        a += (pa_u128)hist[hmin + k] * (RW < S ? RW : S);
    }
    Overlap o;
    o.num = block_sum_u128(a, su);
    o.den = (pa_u128)R * S;
    return o;
}

__device__ __forceinline__ bool qualifies(const Overlap &o, uint64_t A) { return (o.num << 32) >= (pa_u128)A * o.den; }

__global__ __launch_bounds__(kRuleThreads) void k_rule(const PaRunDesc *__restrict__ runs, double alpha_star,
                                                       double dbeta_max, int iterations, int bisect)
{
    __shared__ uint64_t su[16];
    __shared__ uint64_t wcache[kRuleCache];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const int DN = rd.d * rd.N;
    const int hmin = (rec->emin + DN) >> 2, hmax = (rec->emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    const uint64_t R = rec->Rcur;
    const uint64_t A = (uint64_t)rint(ldexp(alpha_star, 32));
    const Overlap top = rule_overlap(rd.dv.hist, hmin, nlev, R, dbeta_max, wcache, su);
    double best = dbeta_max;
    Overlap obest = top;
    if (bisect && !qualifies(top, A)) {
        double lo = 0.0, hi = dbeta_max;
        obest.num = obest.den = 1; // alpha(0) = 1
        for (int it = 0; it < iterations; ++it) {
            const double mid = 0.5 * (lo + hi);
            const Overlap om = rule_overlap(rd.dv.hist, hmin, nlev, R, mid, wcache, su);
            if (qualifies(om, A)) {
                lo = mid;
                obest = om;
            } else {
                hi = mid;
            }
        }
        best = lo;
    }
    if (threadIdx.x == 0) {
        rec->rule_dbeta = best;
        rec->rule_alpha = u128_to_double(obest.num) / u128_to_double(obest.den);
    }
}

// Inputs of the learned step model from the energy histogram (moments in
// float64, fixed chunks and tree), the record's ln Q history and the family
// entropy of the latest observables: beta, <E>/N, sd(E)/sqrt(N), skewness,
// ln Q_{i-2..i}/N, S_f / ln R.
__global__ __launch_bounds__(kRuleThreads) void k_features(const PaRunDesc *__restrict__ runs)
{
    __shared__ double sd[16];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const int DN = rd.d * rd.N;
    const int32_t emin = rec->emin;
    const int hmin = (emin + DN) >> 2, hmax = (rec->emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    const double R = (double)rec->Rcur;
    const int chunk = (nlev + (int)blockDim.x - 1) / (int)blockDim.x;
    const int lo = (int)threadIdx.x * chunk;
    const int hi = lo + chunk < nlev ? lo + chunk : nlev;
    double s1 = 0.0;
    for (int k = lo; k < hi; ++k)
        s1 = s1 + (double)rd.dv.hist[hmin + k] * (double)(emin + 4 * k);
    const double mean = pa_block_sum_f64(s1, sd) / R;
    double s2 = 0.0, s3 = 0.0;
    for (int k = lo; k < hi; ++k) {
        const double dx = (double)(emin + 4 * k) - mean, n = (double)rd.dv.hist[hmin + k];
        s2 = s2 + n * dx * dx;
        s3 = s3 + n * dx * dx * dx;
    }
    const double var = pa_block_sum_f64(s2, sd) / R;
    const double m3 = pa_block_sum_f64(s3, sd) / R;
    if (threadIdx.x == 0) {
        const double N = (double)rd.N;
        rec->feat[0] = (float)rec->beta;
        rec->feat[1] = (float)(mean / N);
        rec->feat[2] = (float)(sqrt(var) / sqrt(N));
        rec->feat[3] = (float)(var > 0.0 ? m3 / (var * sqrt(var)) : 0.0);
        rec->feat[4] = (float)(rec->lnq_hist[0] / N);
        rec->feat[5] = (float)(rec->lnq_hist[1] / N);
        rec->feat[6] = (float)(rec->lnq_hist[2] / N);
        rec->feat[7] = (float)(R > 1.0 ? rec->S_f / log(R) : 0.0);
    }
}

// The learned proposal is kept if it passes the exact overlap check;
// otherwise the bisection of the rule decides (fallback).
// The learned step's exact check: the model's proposal c (clamped to
// dbeta_max) is kept only where alpha >= alpha*.  With refine > 0 it seeds a
// short search instead of being taken as it is: if c qualifies, the bracket
// [c, min(bracket c, dbeta_max)] (whose top is taken if it qualifies), else
// [c / bracket, c] if its bottom qualifies, is halved `refine` times keeping
// the lower end qualified.  Where neither applies (or c <= 0) the rule itself
// decides: the bisection of k_rule over [0, dbeta_max] (the fallback).
// Every value returned has alpha >= alpha*, tested exactly.
__global__ __launch_bounds__(kRuleThreads) void k_check_candidate(const PaRunDesc *__restrict__ runs,
                                                                  double alpha_star, double dbeta_max, int iterations,
                                                                  double bracket, int refine)
{
    __shared__ uint64_t su[16];
    __shared__ uint64_t wcache[kRuleCache];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const int DN = rd.d * rd.N;
    const int hmin = (rec->emin + DN) >> 2, hmax = (rec->emax + DN) >> 2;
    const int nlev = hmax - hmin + 1;
    const uint64_t R = rec->Rcur;
    const uint64_t A = (uint64_t)rint(ldexp(alpha_star, 32));
    const double cand = rec->cand_dbeta;
    auto overlap = [&](double db) { return rule_overlap(rd.dv.hist, hmin, nlev, R, db, wcache, su); };
    auto publish = [&](double db, const Overlap &o, uint32_t fb) {
        if (threadIdx.x == 0) {
            rec->rule_dbeta = db;
            rec->rule_alpha = u128_to_double(o.num) / u128_to_double(o.den);
            rec->fallback = fb;
        }
    };
    if (cand > 0.0) {
        const Overlap oc = overlap(cand);
        const bool ok = qualifies(oc, A);
        if (ok && (refine == 0 || cand >= dbeta_max)) {
            publish(cand, oc, 0u);
            return;
        }
        if (refine > 0) {
            double lo = cand, hi = cand;
            Overlap olo = oc;
            bool bracketed = false;
            if (ok) {
                hi = bracket * cand < dbeta_max ? bracket * cand : dbeta_max;
                const Overlap oh = overlap(hi);
                if (qualifies(oh, A)) {
                    publish(hi, oh, 0u);
                    return;
                }
                bracketed = true;
            } else {
                lo = cand / bracket;
                olo = overlap(lo);
                bracketed = qualifies(olo, A);
            }
            if (bracketed) {
                for (int it = 0; it < refine; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    const Overlap om = overlap(mid);
                    if (qualifies(om, A)) {
                        lo = mid;
                        olo = om;
                    } else {
                        hi = mid;
                    }
                }
                publish(lo, olo, 0u);
                return;
            }
        }
    }
    const Overlap top = overlap(dbeta_max);
    double best = dbeta_max;
    Overlap obest = top;
    if (!qualifies(top, A)) {
        double lo = 0.0, hi = dbeta_max;
        obest.num = obest.den = 1;
        for (int it = 0; it < iterations; ++it) {
            const double mid = 0.5 * (lo + hi);
            const Overlap om = overlap(mid);
            if (qualifies(om, A)) {
                lo = mid;
                obest = om;
            } else {
                hi = mid;
            }
        }
        best = lo;
    }
    publish(best, obest, 1u);
}

// ------------------------------------------------------------------ resampling
__device__ __forceinline__ uint64_t weight_of(int32_t e, int DN, int hmin, const uint64_t *wtab)
{
    return wtab[((e + DN) >> 2) - hmin];
}

// Per-replica resampling kernels: chunk b.idx of run b.run, replicas
// [idx*CHUNK, ...) below the pre-resampling size.
struct RepCtx {
    const PaRunDesc *rd;
    PaRecord *rec;
    int64_t beg, end;
};

__device__ __forceinline__ bool rep_ctx(const PaRunDesc *runs, const PaBlk *map, RepCtx *c)
{
    const PaBlk b = map[blockIdx.x];
    c->rd = runs + b.run;
    c->rec = c->rd->dv.rec;
    const int64_t R = (int64_t)c->rec->Rcur;
    c->beg = (int64_t)b.idx * PA_CHUNK;
    c->end = c->beg + PA_CHUNK < R ? c->beg + PA_CHUNK : R;
    return c->beg < R && !frozen(c->rec);
}

// The kernels of a resampling proper: idle when a conditional resampling
// decided to keep the population.
__device__ __forceinline__ bool rs_ctx(const PaRunDesc *runs, const PaBlk *map, RepCtx *c)
{
    return rep_ctx(runs, map, c) && !c->rec->keep;
}

// Integer weight of replica j for the resampling: per energy level for a
// uniform population, per replica (k_rw_sum) for a weighted one.
__device__ __forceinline__ uint64_t rep_weight(const RepCtx &c, bool wt, const int32_t *E, int64_t j, int DN,
                                               int hmin)
{
    return wt ? c.rd->dv.Wj[j] : weight_of(E[j], DN, hmin, c.rd->dv.wtab);
}

// ------------------------------------------------------------------ weighted populations
// Sec. 3 allows keeping the population, with importance weights, while their
// variance is small.  Replica j then carries a log-weight lw_j <= 0 (largest
// 0) and weighs exp(lw_j - dbeta E_j) at the next beta.  With
//   x_j = lw_j + (-(dbeta (E_j - E_min)))   (every x_j <= 0)
// and m = min_j |x_j| (so max_j x_j = -m), the integer weights are
// W_j = floor(2^40 pa_exp(x_j + m)) and
//   ln Q = -dbeta E_min - m + ln sum_j exp(x_j + m) - ln sum_j exp(lw_j),
// Eq. (1) for weighted replicas.  A uniform population is the case lw = 0
// (x_j is then the argument of its per-level weights and m = 0).
__device__ __forceinline__ double wx(const PaDev &dv, const PaRecord *rec, int cur, bool wt, int64_t j)
{
    const double g = (double)(dv.E[cur][j] - rec->wemin);
    const double lw = wt ? dv.lw[j] : 0.0;
    return lw + (-(rec->dbeta * g));
}

__device__ __forceinline__ double xmag_value(const PaRecord *rec) { return __longlong_as_double((long long)rec->xmag); }

// m: the smallest |x_j| (IEEE bits of non-negative doubles order as integers).
__global__ __launch_bounds__(kThreads) void k_rw_max(const PaRunDesc *__restrict__ runs,
                                                     const PaBlk *__restrict__ map)
{
    RepCtx c;
    if (!rep_ctx(runs, map, &c) || !c.rec->weighted)
        return;
    const PaDev &dv = c.rd->dv;
    const int cur = c.rec->cur;
    int64_t mag = INT64_MAX;
    for (int64_t j = c.beg + threadIdx.x; j < c.end; j += blockDim.x) {
        const int64_t b = __double_as_longlong(wx(dv, c.rec, cur, true, j)) & INT64_MAX;
        mag = b < mag ? b : mag;
    }
    mag = pa_wave_min_i64(mag);
    if ((threadIdx.x & 63) == 0)
        atomicMin(&c.rec->xmag, (unsigned long long)mag);
}

// Per-replica integer weights, S and sum W^2 exactly (order-free atomics),
// and per chunk the fixed-order sums of pa_exp(x_j + m) and pa_exp(lw_j).
__global__ __launch_bounds__(kThreads) void k_rw_sum(const PaRunDesc *__restrict__ runs,
                                                     const PaBlk *__restrict__ map)
{
    __shared__ double sd[16];
    __shared__ uint64_t su[16];
    RepCtx c;
    if (!rep_ctx(runs, map, &c) || !c.rec->weighted)
        return;
    const PaDev &dv = c.rd->dv;
    const int cur = c.rec->cur;
    const double m = xmag_value(c.rec);
    uint64_t s = 0;
    pa_u128 s2 = 0;
    double q = 0.0, l = 0.0;
    for (int64_t j = c.beg + threadIdx.x; j < c.end; j += blockDim.x) {
        const double wv = pa_exp(wx(dv, c.rec, cur, true, j) + m);
        const uint64_t W = (uint64_t)floor(ldexp(wv, 40));
        dv.Wj[j] = W;
        s += W;
        s2 += (pa_u128)W * W;
        q = q + wv;
        l = l + pa_exp(dv.lw[j]);
    }
    s = pa_block_sum_u64(s, su);
    s2 = block_sum_u128(s2, su);
    q = pa_block_sum_f64(q, sd);
    l = pa_block_sum_f64(l, sd);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&c.rec->S, (unsigned long long)s);
        const unsigned long long lo = (uint64_t)s2, hi = (uint64_t)(s2 >> 64);
        const unsigned long long old = atomicAdd(&c.rec->Q2[0], lo);
        atomicAdd(&c.rec->Q2[1], hi + (old + lo < old ? 1ull : 0ull));
        const int64_t chunks = (c.rd->cap + PA_CHUNK - 1) / PA_CHUNK, k = c.beg / PA_CHUNK;
        dv.wpart[k] = q;
        dv.wpart[chunks + k] = l;
    }
}

// ln Q of a weighted population from the chunk sums in chunk order.
__global__ __launch_bounds__(kThreads) void k_rw_final(const PaRunDesc *__restrict__ runs)
{
    __shared__ double sd[16];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec) || !rec->weighted)
        return;
    const int64_t chunks = (rd.cap + PA_CHUNK - 1) / PA_CHUNK;
    const int nlive = (int)(((int64_t)rec->Rcur + PA_CHUNK - 1) / PA_CHUNK);
    double q = 0.0, l = 0.0;
    for (int k = threadIdx.x; k < nlive; k += blockDim.x) {
        q = q + rd.dv.wpart[k];
        l = l + rd.dv.wpart[chunks + k];
    }
    q = pa_block_sum_f64(q, sd);
    l = pa_block_sum_f64(l, sd);
    if (threadIdx.x == 0) {
        rec->qsum = q;
        rec->lnQ = ((-rec->dbeta * (double)rec->wemin - xmag_value(rec)) + log(q)) - log(l);
    }
}

// Conditional resampling: resample only if the effective sample size of the
// step's weights, ESS = S^2 / sum_j W_j^2, is below kappa R_cur.  Decided
// exactly as 2^16 S^2 < kq R_cur sum_j W_j^2 (kq = kappa 2^16) on 192-bit
// integers: S^2 < 2^128, sum W^2 < 2^104, kq R_cur < 2^41.
__global__ void k_cond_decide(const PaRunDesc *__restrict__ runs, uint32_t kq)
{
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (threadIdx.x != 0 || frozen(rec))
        return;
    const uint64_t S = rec->S;
    const pa_u128 S2 = (pa_u128)S * S;
    const uint64_t a0 = (uint64_t)(S2 << 16), a1 = (uint64_t)((S2 << 16) >> 64), a2 = (uint64_t)(S2 >> 112);
    const uint64_t f = (uint64_t)kq * rec->Rcur;
    const pa_u128 p0 = (pa_u128)rec->Q2[0] * f, p1 = (pa_u128)rec->Q2[1] * f;
    const pa_u128 mid = (p0 >> 64) + (pa_u128)(uint64_t)p1;
    const uint64_t r0 = (uint64_t)p0, r1 = (uint64_t)mid, r2 = (uint64_t)(p1 >> 64) + (uint64_t)(mid >> 64);
    const bool resample = a2 != r2 ? a2 < r2 : (a1 != r1 ? a1 < r1 : a0 < r0);
    rec->keep = resample ? 0u : 1u;
    if (!resample)
        rec->Rnew = rec->Rcur; // the capacity and extinction checks see the kept size
}


// Sampling variance, Eq. (5): each chunk sums (r_j - tauhat_j)^2 over its
// replicas in a fixed order (per thread, then the block's fixed tree) into
// partial[chunk]; k_commit adds the partials in chunk order.
__device__ __forceinline__ double sv_term(uint32_t r, uint64_t W, double S, double Rt)
{
    const double tau = ((double)W / S) * Rt;
    const double dlt = (double)r - tau;
    return dlt * dlt;
}

__device__ __forceinline__ void sv_store(const RepCtx &c, double acc, double *sd)
{
    const double t = pa_block_sum_f64(acc, sd);
    if (threadIdx.x == 0)
        c.rd->dv.partial[c.beg / PA_CHUNK] = t;
}

// Poisson by inversion: tauhat = R W / S; tauhat > 32 is cut into
// ceil(tauhat/32) equal pieces, piece p using u from Philox(j, p, i, RS_POIS<<28).
__device__ __forceinline__ uint32_t poisson_copies(const PaRunDesc &rd, uint64_t W, uint64_t S, uint64_t Rt,
                                                   int64_t j, uint32_t step)
{
    const double tau = ((double)W / (double)S) * (double)Rt;
    uint32_t m = 1;
    if (tau > 32.0)
        m = (uint32_t)ceil(tau / 32.0);
    const double mu = tau / (double)m;
    uint32_t tot = 0;
    for (uint32_t p = 0; p < m; ++p) {
        const pa_philox_out o = pa_philox(rd.seed, rd.run_id, (uint32_t)j, p, step, PA_PURPOSE_RS_POIS << 28);
        const double u = ((double)(o.x0 >> 5) * 67108864.0 + (double)(o.x1 >> 6)) * (1.0 / 9007199254740992.0);
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
    return tot;
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

// Multinomial: U_k = floor(r S / 2^128), r = 128 bits of Philox(k, 0, i,
// RS_MULT<<28), k < R; the box of replica j is [C_{j-1}, C_j).  The chunks of
// the map cover the draws k (capacity >= R).
__global__ __launch_bounds__(kThreads) void k_counts_multinomial(const PaRunDesc *__restrict__ runs,
                                                                 const PaBlk *__restrict__ map)
{
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    const int64_t Rt = rd.R0, Rprev = (int64_t)rec->Rcur;
    const int64_t beg = (int64_t)b.idx * PA_CHUNK;
    if (beg >= Rt || frozen(rec) || rec->keep)
        return;
    const int64_t end = beg + PA_CHUNK < Rt ? beg + PA_CHUNK : Rt;
    const uint64_t S = rec->S;
    const uint32_t step = rec->step + 1;
    const uint64_t *C = rd.dv.C;
    for (int64_t k = beg + threadIdx.x; k < end; k += blockDim.x) {
        const pa_philox_out o = pa_philox(rd.seed, rd.run_id, (uint32_t)k, 0u, step, PA_PURPOSE_RS_MULT << 28);
        const uint64_t lo = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
        const uint64_t hi = (uint64_t)o.x2 | ((uint64_t)o.x3 << 32);
        const pa_u128 A = (pa_u128)lo * S, B = (pa_u128)hi * S;
        const uint64_t U = (uint64_t)((B + (A >> 64)) >> 64);
        int64_t a = 0, z = Rprev - 1;
        while (a < z) {
            const int64_t mid = a + ((z - a) >> 1);
            if (C[mid] > U)
                z = mid;
            else
                a = mid + 1;
        }
        atomicAdd(&rd.dv.r[a], 1u);
    }
}

// Sampling variance of the multinomial scheme (its copy numbers are complete
// only after k_counts_multinomial).
__global__ __launch_bounds__(kThreads) void k_sv_partial(const PaRunDesc *__restrict__ runs,
                                                          const PaBlk *__restrict__ map)
{
    __shared__ double sd[16];
    RepCtx c;
    if (!rs_ctx(runs, map, &c))
        return;
    const PaRunDesc &rd = *c.rd;
    const bool wt = c.rec->weighted != 0u;
    const int DN = rd.d * rd.N;
    const int hmin = (c.rec->wemin + DN) >> 2;
    const double S = (double)c.rec->S, Rt = (double)rd.R0;
    const int32_t *E = rd.dv.E[c.rec->cur];
    double acc = 0.0;
    for (int64_t j = c.beg + threadIdx.x; j < c.end; j += blockDim.x)
        acc = acc + sv_term(rd.dv.r[j], rep_weight(c, wt, E, j, DN, hmin), S, Rt);
    sv_store(c, acc, sd);
}

// Decoupled look-back (Merrill & Garland 2016), run by a tile's first wave:
// the tile publishes its aggregate, looks back over up to 64 preceding tiles
// at once (one flag per lane; the nearest tile with an inclusive prefix ends
// the look-back, the aggregates of the tiles after it add up), then
// publishes its own inclusive prefix.  Returns the exclusive prefix in every
// lane of the wave.  The workgroups of a run take their tile index from the
// run's own atomic ticket, so every tile a tile waits on (same run, lower
// index) belongs to a workgroup that is already running; a wait past the
// spin limit sets the run's timeout status and gives up (the resampling is
// then not applied).
__device__ __forceinline__ unsigned long long tile_lookback(PaScanTile *tiles, uint32_t tile,
                                                            unsigned long long agg, PaRecord *rec)
{
    const int lane = threadIdx.x & 63;
    unsigned long long *me = &tiles[tile].word;
    unsigned long long excl = 0;
    if (lane == 0) // tile 0's aggregate is its inclusive prefix
        __hip_atomic_store(me, (tile == 0 ? PA_TILE_INCL : PA_TILE_AGG) | agg, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (tile == 0)
        return 0;
    int64_t top = (int64_t)tile - 1; // the window: tiles top - lane
    uint32_t spins = 0;
    for (;;) {
        const int64_t p = top - lane;
        unsigned long long word = PA_TILE_INCL; // before tile 0: an inclusive prefix of 0
        if (p >= 0)
            word = __hip_atomic_load(&tiles[p].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t f = (uint32_t)(word >> 62);
        const unsigned long long val = word & PA_TILE_VALUE;
        const uint64_t inc = __ballot(f == 2u), pending = __ballot(f == 0u);
        const int first = inc ? __ffsll((long long)inc) - 1 : 64;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull); // lanes 0..first
        if (pending & need) { // a tile the prefix needs has not published yet
            if (++spins > (1u << 26)) {
                if (lane == 0)
                    atomicOr(&rec->status, PA_ST_SCAN_TIMEOUT);
                break; // gave up; the status bit is set
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += pa_wave_sum_u64(((need >> lane) & 1ull) ? val : 0ull);
        if (first < 64)
            break;
        top -= 64;
    }
    // a prefix too wide for the word stays unpublished: later tiles then
    // add this tile's aggregate themselves
    if (lane == 0 && excl + agg <= PA_TILE_VALUE)
        __hip_atomic_store(me, PA_TILE_INCL | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// Exclusive prefix of each thread's `run` within the workgroup (waves by
// shuffles, then the waves' totals through LDS); *agg: the workgroup total.
template <int THREADS>
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long run, unsigned long long *s_wave,
                                                              unsigned long long *agg)
{
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
    unsigned long long wave_off = 0, a = 0;
    for (int k = 0; k < THREADS / 64; ++k) {
        if (k < wave)
            wave_off += s_wave[k];
        a += s_wave[k];
    }
    *agg = a;
    return wave_off + incl - run;
}

// The ancestor map from a replica's copy number r and exclusive offset P:
// anc[P + k] = j for k < r (kept below the capacity; a resampling that
// overflows is not applied).
__device__ __forceinline__ void write_ancestors(uint32_t *anc, unsigned long long P, uint32_t r, int64_t j,
                                                int64_t cap)
{
    for (unsigned long long d = P; d < P + r && d < (unsigned long long)cap; ++d)
        anc[d] = (uint32_t)j;
}

// Multinomial copy numbers' exclusive prefix sum, written only as the
// ancestor map: each run's first Rcur copy numbers (entries past Rcur count
// as 0), PA_SCAN_ITEMS consecutive ones per thread, tiles of PA_SCAN_TILE.
__global__ __launch_bounds__(PA_SCAN_THREADS) void k_scan_counts(const PaRunDesc *__restrict__ runs,
                                                                 const PaBlk *__restrict__ map)
{
    static_assert(PA_SCAN_ITEMS % 4 == 0, "items of a thread are whole 16-byte vectors");
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_wave[PA_SCAN_THREADS / 64];
    __shared__ unsigned long long s_excl;
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec) || rec->keep)
        return; // every tile of a frozen (or kept) run returns: none waits
    if (threadIdx.x == 0)
        s_tile = atomicAdd(&rec->ticket[1], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t n = (int64_t)rec->Rcur;
    const int64_t ntiles = (rd.cap + PA_SCAN_TILE - 1) / PA_SCAN_TILE;
    PaScanTile *tiles = rd.dv.tiles + pa_tiles_per_sum(rd.cap);
    const int64_t base = (int64_t)tile * PA_SCAN_TILE + (int64_t)threadIdx.x * PA_SCAN_ITEMS;
    alignas(16) uint32_t v[PA_SCAN_ITEMS];
    if (base + PA_SCAN_ITEMS <= n) {
#pragma unroll
        for (int k = 0; k < PA_SCAN_ITEMS / 4; ++k)
            reinterpret_cast<uint4 *>(v)[k] = reinterpret_cast<const uint4 *>(rd.dv.r + base)[k];
    } else {
#pragma unroll
        for (int k = 0; k < PA_SCAN_ITEMS; ++k)
            v[k] = base + k < n ? rd.dv.r[base + k] : 0u;
    }
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < PA_SCAN_ITEMS; ++k)
        run += v[k];
    unsigned long long agg;
    const unsigned long long thread_excl = block_excl_scan<PA_SCAN_THREADS>(run, s_wave, &agg);
    if ((threadIdx.x >> 6) == 0) {
        const unsigned long long excl = tile_lookback(tiles, tile, agg, rec);
        if ((threadIdx.x & 63) == 0) {
            s_excl = excl;
            if ((int64_t)tile == ntiles - 1)
                rec->Rnew = excl + agg;
        }
    }
    __syncthreads();
    unsigned long long acc = s_excl + thread_excl;
#pragma unroll
    for (int k = 0; k < PA_SCAN_ITEMS; ++k) {
        if (base + k < n)
            write_ancestors(rd.dv.anc, acc, v[k], base + k, rd.cap);
        acc += v[k];
    }
}

// The chunk sums of the sampling-variance terms: a wave's slots are one
// chunk when it holds PA_CHUNK of them (ITEMS = 16), else the tile is one
// chunk (ITEMS = 4: block sum).  The barriers it contains (or adds) publish
// what the first wave wrote to LDS before.
template <int ITEMS>
__device__ __forceinline__ void store_chunk_sv(const PaRunDesc &rd, uint32_t tile, double sv, double *sd)
{
    constexpr int kTile = kThreads * ITEMS;
    if (64 * ITEMS == PA_CHUNK) {
        const double t = pa_wave_sum_f64(sv);
        const int64_t chunk = (int64_t)tile * (kTile / PA_CHUNK) + (threadIdx.x >> 6);
        if ((threadIdx.x & 63) == 0 && chunk * PA_CHUNK < rd.cap)
            rd.dv.partial[chunk] = t;
        __syncthreads();
    } else {
        static_assert(64 * ITEMS == PA_CHUNK || kTile == PA_CHUNK, "chunks of whole waves or whole tiles");
        const double t = pa_block_sum_f64(sv, sd);
        if (threadIdx.x == 0)
            rd.dv.partial[tile] = t;
    }
}

// Integer weights and their inclusive prefix sums C in one pass: tile t (the
// run's ticket order) holds replica slots [T t, T (t + 1)), T = kThreads
// ITEMS = pa_counts_tile(cap), ITEMS consecutive ones per thread; each weight
// is taken from the replica's energy level (or a weighted population's own)
// as the tile is loaded.  MULTINOMIAL: writes C and returns the copy numbers
// to zero for the draws.  SYSTEMATIC: writes no C but each replica's copy
// range [N(C_{j-1}), N(C_j)) straight into the ancestor map (the points
// below C_{j-1} are the copies of the replicas before j), the new size
// N(C_{R-1}) and the sampling variance per chunk.
constexpr int PA_SCAN_SYSTEMATIC = 0, PA_SCAN_MULTINOMIAL = 1;
template <int MODE, int ITEMS>
__device__ __forceinline__ void weights_scan_tile(const PaRunDesc &rd, PaRecord *rec, uint32_t tile,
                                                  unsigned long long *s_wave, unsigned long long *s_excl,
                                                  double *sd)
{
    constexpr int kTile = kThreads * ITEMS;
    const int64_t n = (int64_t)rec->Rcur;
    const int64_t ntiles = (rd.cap + kTile - 1) / kTile;
    PaScanTile *tiles = rd.dv.tiles;
    const int64_t base = (int64_t)tile * kTile + (int64_t)threadIdx.x * ITEMS;
    const bool whole = base + ITEMS <= n; // the thread's slots are all live
    const bool wt = rec->weighted != 0u;
    const int DN = rd.d * rd.N;
    const int hmin = (rec->wemin + DN) >> 2;
    const int32_t *E = rd.dv.E[rec->cur];
    uint64_t v[ITEMS];
    if (whole && !wt) {
        alignas(16) int32_t e[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS / 4; ++k)
            reinterpret_cast<uint4 *>(e)[k] = reinterpret_cast<const uint4 *>(E + base)[k];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            v[k] = weight_of(e[k], DN, hmin, rd.dv.wtab);
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            v[k] = base + k < n ? (wt ? rd.dv.Wj[base + k] : weight_of(E[base + k], DN, hmin, rd.dv.wtab)) : 0ull;
    }
    if (MODE == PA_SCAN_MULTINOMIAL) {
        if (whole) {
#pragma unroll
            for (int k = 0; k < ITEMS / 4; ++k)
                reinterpret_cast<uint4 *>(rd.dv.r + base)[k] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int k = 0; k < ITEMS; ++k)
                if (base + k < n)
                    rd.dv.r[base + k] = 0u;
        }
    }
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        run += v[k];
    unsigned long long agg;
    const unsigned long long thread_excl = block_excl_scan<kThreads>(run, s_wave, &agg);
    if ((threadIdx.x >> 6) == 0) {
        const unsigned long long excl = tile_lookback(tiles, tile, agg, rec);
        if ((threadIdx.x & 63) == 0) {
            *s_excl = excl;
            if ((int64_t)tile == ntiles - 1)
                rec->Ctot = excl + agg;
        }
    }
    if (MODE == PA_SCAN_MULTINOMIAL) {
        __syncthreads();
        unsigned long long acc = *s_excl + thread_excl;
        alignas(16) uint64_t o[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            acc += v[k];
            o[k] = acc;
        }
        if (whole) {
#pragma unroll
            for (int k = 0; k < ITEMS / 2; ++k)
                reinterpret_cast<uint4 *>(rd.dv.C + base)[k] = reinterpret_cast<const uint4 *>(o)[k];
        } else {
            for (int k = 0; k < ITEMS; ++k)
                if (base + k < n)
                    rd.dv.C[base + k] = o[k];
        }
        return;
    }
    // systematic: N(c) = #points (k + U/2^32) S/R below c, k < R
    __syncthreads();
    const uint64_t S = rec->S, Rt = (uint64_t)rd.R0;
    const uint32_t U = pa_philox(rd.seed, rd.run_id, 0u, 0u, rec->step + 1, PA_PURPOSE_RS_SYS << 28).x0;
    unsigned long long acc = *s_excl + thread_excl;
    uint64_t lo = sys_below(acc, Rt, S, U); // N(C_{base-1}); N(0) = 0
    double sv = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t j = base + k;
        if (j < n) {
            acc += v[k];
            const uint64_t hi = sys_below(acc, Rt, S, U);
            for (uint64_t d = lo; d < hi; ++d)
                rd.dv.anc[d] = (uint32_t)j;
            if (j == n - 1)
                rec->Rnew = hi; // N(S) = Rt: the size is kept
            sv = sv + sv_term((uint32_t)(hi - lo), v[k], (double)S, (double)Rt);
            lo = hi;
        }
    }
    store_chunk_sv<ITEMS>(rd, tile, sv, sd);
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_weights_scan(const PaRunDesc *__restrict__ runs,
                                                           const PaBlk *__restrict__ map)
{
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_wave[kThreads / 64];
    __shared__ unsigned long long s_excl;
    __shared__ double sd[16];
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec) || rec->keep)
        return; // every tile of a frozen (or kept) run returns: none waits
    if (threadIdx.x == 0)
        s_tile = atomicAdd(&rec->ticket[0], 1u);
    __syncthreads();
    static_assert(kThreads * 16 == 4096 && kThreads * 4 == 1024, "the tiles of pa_counts_tile");
    if (pa_counts_tile(rd.cap) == 4096)
        weights_scan_tile<MODE, 16>(rd, rec, s_tile, s_wave, &s_excl, sd);
    else
        weights_scan_tile<MODE, 4>(rd, rec, s_tile, s_wave, &s_excl, sd);
}

// Nearest-integer (SCHEME 2: floor(tauhat) + [u S < (R W mod S) 2^32], u =
// x0 of Philox(j, 0, i, RS_NI<<28)) or Poisson (SCHEME 1) copy numbers drawn
// and summed in one pass: tile t (the run's ticket order) holds replica slots
// [T t, T (t + 1)), T = kThreads ITEMS = pa_counts_tile(cap), ITEMS
// consecutive ones per thread.  Each thread draws its replicas' copy
// numbers, the workgroup sums them, the look-back gives the tile's offset,
// and the ancestor map is written from it.  The sampling-variance terms of
// chunk c (PA_CHUNK slots) go to partial[c].
template <int SCHEME, int ITEMS>
__device__ __forceinline__ void counts_scan_tile(const PaRunDesc &rd, PaRecord *rec, uint32_t *s_tile,
                                                 unsigned long long *s_wave, unsigned long long *s_excl,
                                                 double *sd)
{
    constexpr int kTile = kThreads * ITEMS;
    const uint32_t tile = *s_tile;
    const int64_t n = (int64_t)rec->Rcur;
    const int64_t ntiles = (rd.cap + kTile - 1) / kTile;
    PaScanTile *tiles = rd.dv.tiles + pa_tiles_per_sum(rd.cap);
    const int64_t base = (int64_t)tile * kTile + (int64_t)threadIdx.x * ITEMS;
    const bool wt = rec->weighted != 0u;
    const int DN = rd.d * rd.N;
    const int hmin = (rec->wemin + DN) >> 2;
    const uint64_t S = rec->S, Rt = (uint64_t)rd.R0;
    const uint32_t step = rec->step + 1;
    const int32_t *E = rd.dv.E[rec->cur];
    alignas(16) int32_t e[ITEMS];
    if (base + ITEMS <= n && !wt) {
#pragma unroll
        for (int k = 0; k < ITEMS / 4; ++k)
            reinterpret_cast<uint4 *>(e)[k] = reinterpret_cast<const uint4 *>(E + base)[k];
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            e[k] = (!wt && base + k < n) ? E[base + k] : 0;
    }
    uint32_t r[ITEMS];
    double sv = 0.0;
    unsigned long long run = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t j = base + k;
        r[k] = 0;
        if (j >= n)
            continue;
        const uint64_t W = wt ? rd.dv.Wj[j] : weight_of(e[k], DN, hmin, rd.dv.wtab);
        if (SCHEME == 2) {
            const uint64_t a = Rt * W;
            const uint64_t qt = a / S;
            const uint64_t rho = a - qt * S;
            const pa_philox_out o = pa_philox(rd.seed, rd.run_id, (uint32_t)j, 0u, step, PA_PURPOSE_RS_NI << 28);
            const bool extra = ((pa_u128)o.x0 * S) < ((pa_u128)rho << 32);
            r[k] = (uint32_t)qt + (extra ? 1u : 0u);
        } else {
            r[k] = poisson_copies(rd, W, S, Rt, j, step);
        }
        sv = sv + sv_term(r[k], W, (double)S, (double)Rt);
        run += r[k];
    }
    unsigned long long agg;
    const unsigned long long thread_excl = block_excl_scan<kThreads>(run, s_wave, &agg);
    if ((threadIdx.x >> 6) == 0) {
        const unsigned long long excl = tile_lookback(tiles, tile, agg, rec);
        if ((threadIdx.x & 63) == 0) {
            *s_excl = excl;
            if ((int64_t)tile == ntiles - 1)
                rec->Rnew = excl + agg;
        }
    }
    store_chunk_sv<ITEMS>(rd, tile, sv, sd);
    unsigned long long acc = *s_excl + thread_excl;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (base + k < n)
            write_ancestors(rd.dv.anc, acc, r[k], base + k, rd.cap);
        acc += r[k];
    }
}

template <int SCHEME>
__global__ __launch_bounds__(kThreads) void k_counts_scan(const PaRunDesc *__restrict__ runs,
                                                          const PaBlk *__restrict__ map)
{
    __shared__ uint32_t s_tile;
    __shared__ unsigned long long s_wave[kThreads / 64];
    __shared__ unsigned long long s_excl;
    __shared__ double sd[16];
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec) || rec->keep)
        return; // every tile of a frozen (or kept) run returns: none waits
    if (threadIdx.x == 0)
        s_tile = atomicAdd(&rec->ticket[1], 1u);
    __syncthreads();
    static_assert(kThreads * 16 == 4096 && kThreads * 4 == 1024, "the tiles of pa_counts_tile");
    if (pa_counts_tile(rd.cap) == 4096)
        counts_scan_tile<SCHEME, 16>(rd, rec, &s_tile, s_wave, &s_excl, sd);
    else
        counts_scan_tile<SCHEME, 4>(rd, rec, &s_tile, s_wave, &s_excl, sd);
}

// A new resampling starts with a clean status (a frozen run stays frozen),
// cleared tile flags for both prefix sums (weights, copy numbers) and their
// tile tickets.  The reweighting prepares its resampling the same way; this
// launch serves a resampling retried after a failed one.
__global__ void k_resample_prep(const PaRunDesc *__restrict__ runs)
{
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    const int64_t ntiles = 2 * pa_tiles_per_sum(rd.cap);
    for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x)
        rd.dv.tiles[t].word = 0ull;
    if (threadIdx.x == 0) {
        rec->ticket[0] = rec->ticket[1] = 0u;
        if (!frozen(rec)) {
            rec->status = 0;
            rec->skip = 0;
            rec->keep = 0;
        }
    }
}

// Capacity and extinction: a resampling that would not fit (or leave no
// replica), a non-finite ln Q or an unfinished prefix sum is not applied.
// Every kernel after the copy-number scan evaluates this from the same record
// fields, so they agree without a separate pass; k_commit records it.
__device__ __forceinline__ uint32_t resample_status(const PaRecord *rec, int64_t cap)
{
    const uint64_t Rn = rec->Rnew;
    uint32_t st = rec->status & PA_ST_SCAN_TIMEOUT;
    if (Rn > (uint64_t)cap)
        st |= PA_ST_CAPACITY;
    if (Rn == 0)
        st |= PA_ST_EXTINCT;
    const double q = rec->lnQ;
    if (!(q == q) || q - q != 0.0)
        st |= PA_ST_NONFINITE;
    return st;
}

// ------------------------------------------------------------------ apply

// A resampled population's energies, magnetisations and labels, from their
// ancestors into the other buffer (before the commit swaps the buffers).  Its
// spins follow later (PaRecord::gather): in the next sweep's column load, or
// in k_gather_spins when something else reads them first.
__global__ __launch_bounds__(kThreads) void k_gather_meta(const PaRunDesc *__restrict__ runs,
                                                          const PaBlk *__restrict__ map)
{
    const PaBlk blk = map[blockIdx.x];
    const PaRunDesc &rd = runs[blk.run];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec) || rec->keep || resample_status(rec, rd.cap) != 0u)
        return;
    const int64_t Rnew = (int64_t)rec->Rnew;
    const int64_t beg = (int64_t)blk.idx * PA_CHUNK, end = beg + PA_CHUNK < Rnew ? beg + PA_CHUNK : Rnew;
    const int cur = rec->cur;
    for (int64_t d = beg + threadIdx.x; d < end; d += blockDim.x) {
        const uint32_t a = rd.dv.anc[d];
        rd.dv.E[cur ^ 1][d] = rd.dv.E[cur][a];
        rd.dv.M[cur ^ 1][d] = rd.dv.M[cur][a];
        rd.dv.label[cur ^ 1][d] = rd.dv.label[cur][a];
    }
}

// Word column w of a resampled population from its ancestors.  PRE: before
// the commit swaps the buffers, from the current buffer into the other one,
// with the energies, magnetisations and labels (every run's spins move now).
// Otherwise: after the commit, the spins a resampling left for the sweeps
// (PaRecord::gather), from the other buffer into the current one.
template <bool PRE>
__global__ __launch_bounds__(kThreads) void k_gather_spins(const PaRunDesc *__restrict__ runs,
                                                           const PaBlk *__restrict__ map)
{
    __shared__ uint64_t g_mask[64];
    __shared__ uint32_t g_word[64];
    __shared__ int g_shift[64];
    __shared__ int s_ngroups;
    // an output word takes bits of the source words its ancestors lie in, the
    // same words as its neighbours: neighbouring words go to one XCD
    const PaBlk blk = map[xcd_contiguous(blockIdx.x, gridDim.x)];
    const PaRunDesc &rd = runs[blk.run];
    PaRecord *rec = rd.dv.rec;
    const int64_t R = PRE ? (int64_t)rec->Rnew : (int64_t)rec->Rcur;
    const uint32_t w = blk.idx;
    if (frozen(rec) || (int64_t)w * 64 >= R)
        return;
    if (PRE ? (rec->keep || resample_status(rec, rd.cap) != 0u) : rec->gather == 0u)
        return;
    const int N = rd.N;
    const int cur = rec->cur;
    const int from = PRE ? cur : cur ^ 1;
    if (PRE && threadIdx.x < 64) { // the replicas' energies, magnetisations and labels
        const int64_t d = 64 * (int64_t)w + threadIdx.x;
        if (d < R) {
            const uint32_t a = rd.dv.anc[d];
            rd.dv.E[cur ^ 1][d] = rd.dv.E[cur][a];
            rd.dv.M[cur ^ 1][d] = rd.dv.M[cur][a];
            rd.dv.label[cur ^ 1][d] = rd.dv.label[cur][a];
        }
    }
    const GatherGroups G = {g_mask, g_word, g_shift, &s_ngroups};
    gather_groups(rd.dv.anc, w, R, G);
    __syncthreads();
    __attribute__((address_space(1))) pa_u64x2 *dst =
        (__attribute__((address_space(1))) pa_u64x2 *)(rd.dv.spins[from ^ 1] + (size_t)w * N);
    gather_sites(rd.dv.spins[from], N, G, [&](int p, pa_u64x2 v) { dst[p] = v; });
}

// A kept population takes its new log-weights x_j + m (m = 0 if it was uniform).
__global__ __launch_bounds__(kThreads) void k_keep(const PaRunDesc *__restrict__ runs,
                                                   const PaBlk *__restrict__ map)
{
    RepCtx c;
    if (!rep_ctx(runs, map, &c) || !c.rec->keep || resample_status(c.rec, c.rd->cap) != 0u)
        return;
    const PaDev &dv = c.rd->dv;
    const int cur = c.rec->cur;
    const bool wt = c.rec->weighted != 0u;
    const double m = wt ? xmag_value(c.rec) : 0.0;
    for (int64_t j = c.beg + threadIdx.x; j < c.end; j += blockDim.x)
        dv.lw[j] = wx(dv, c.rec, cur, wt, j) + m;
}

// Completes an applied resampling: SV (Eq. (5)) from the partials in fixed
// order, ln Z_hat += ln Q (Eq. (7)), the new beta and its thresholds, the
// buffer swap and the step count.  A kept population advances the same way
// with its members in place, its new log-weights and SV = 0 (nothing drawn).
// spins_moved: the spins were gathered before the commit (k_gather_spins<true>).
__global__ __launch_bounds__(kThreads) void k_commit(const PaRunDesc *__restrict__ runs, int freeze,
                                                     int spins_moved)
{
    __shared__ double sd[16];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const uint32_t st = resample_status(rec, rd.cap);
    __syncthreads(); // every thread has read the status before thread 0 writes it
    if (st != 0u) {
        if (threadIdx.x == 0) {
            rec->skip = 1;
            rec->status = freeze ? (st | PA_ST_FROZEN) : st;
            rec->gather = 0;
        }
        return;
    }
    if (rec->keep) {
        if (threadIdx.x == 0) {
            rec->gather = 0;
            rec->sv = 0.0;
            rec->lnZ = rec->lnZ + rec->lnQ;
            rec->lnq_hist[0] = rec->lnq_hist[1];
            rec->lnq_hist[1] = rec->lnq_hist[2];
            rec->lnq_hist[2] = rec->lnQ;
            rec->T[0] = rec->Tn[0];
            rec->T[1] = rec->Tn[1];
            rec->T[2] = rec->Tn[2];
            rec->Rprev = rec->Rcur;
            rec->beta = rec->beta_next;
            rec->step += 1;
            rec->sweeps = 0;
            rec->weighted = 1;
        }
        return;
    }
    const int64_t Rprev = (int64_t)rec->Rcur;
    const int nlive = (int)((Rprev + PA_CHUNK - 1) / PA_CHUNK);
    double v = 0.0;
    for (int k = threadIdx.x; k < nlive; k += blockDim.x)
        v = v + rd.dv.partial[k];
    const double t = pa_block_sum_f64(v, sd);
    if (threadIdx.x == 0) {
        rec->sv = t / (double)Rprev;
        rec->lnZ = rec->lnZ + rec->lnQ;
        rec->lnq_hist[0] = rec->lnq_hist[1];
        rec->lnq_hist[1] = rec->lnq_hist[2];
        rec->lnq_hist[2] = rec->lnQ;
        rec->T[0] = rec->Tn[0];
        rec->T[1] = rec->Tn[1];
        rec->T[2] = rec->Tn[2];
        rec->Rprev = (uint64_t)Rprev;
        rec->Rcur = rec->Rnew;
        rec->cur ^= 1;
        rec->gather = spins_moved ? 0 : 1; // else the spins wait in the other buffer
        rec->beta = rec->beta_next;
        rec->step += 1;
        rec->sweeps = 0;
        rec->weighted = 0;
        rec->resamplings += 1;
    }
}

// ------------------------------------------------------------------ step 4: observables
// Counters of the level histogram a block of the observables pass keeps in
// LDS: its energies' levels, from its lowest; a wider spread (high
// temperatures, large lattices) goes to the run's histogram directly.
constexpr int kObsLevels = 2048;

__global__ __launch_bounds__(kThreads) void k_obs_rep(const PaRunDesc *__restrict__ runs,
                                                      const PaBlk *__restrict__ map, int build_hist)
{
    __shared__ uint64_t su[16 * 5];
    __shared__ double sd[16 * PA_WPARTS];
    __shared__ uint32_t lh[kObsLevels];
    __shared__ int s_lo[kThreads / 64], s_hi[kThreads / 64];
    // PA_HCHUNK replica slots per workgroup (four chunks): fewer workgroups
    // merge their level counts and sums into the run's, on the same addresses
    RepCtx c;
    {
        const PaBlk b = map[blockIdx.x];
        c.rd = runs + b.run;
        c.rec = c.rd->dv.rec;
        const int64_t R = (int64_t)c.rec->Rcur;
        c.beg = (int64_t)b.idx * PA_HCHUNK;
        c.end = c.beg + PA_HCHUNK < R ? c.beg + PA_HCHUNK : R;
        if (c.beg >= R || frozen(c.rec))
            return;
    }
    const PaDev &dv = c.rd->dv;
    const int cur = c.rec->cur;
    const int DN = c.rd->d * c.rd->N;
    // the level histogram of the population (for the next reweighting, the
    // step rule and the step model): the block's energy range first, then
    // per-block counts in LDS merged with one atomic per populated level
    int hlo = 0, nlh = 0;
    if (build_hist) {
        int64_t lo = INT_MAX, hi = INT_MIN;
        for (int64_t d = c.beg + threadIdx.x; d < c.end; d += blockDim.x) {
            const int64_t e = dv.E[cur][d];
            lo = e < lo ? e : lo;
            hi = e > hi ? e : hi;
        }
        lo = pa_wave_min_i64(lo);
        hi = pa_wave_max_i64(hi);
        if ((threadIdx.x & 63) == 0) {
            s_lo[threadIdx.x >> 6] = (int)lo;
            s_hi[threadIdx.x >> 6] = (int)hi;
        }
        __syncthreads();
        int blo = s_lo[0], bhi = s_hi[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            blo = s_lo[k] < blo ? s_lo[k] : blo;
            bhi = s_hi[k] > bhi ? s_hi[k] : bhi;
        }
        hlo = (blo + DN) >> 2;
        nlh = ((bhi + DN) >> 2) - hlo + 1;
        if (nlh <= kObsLevels)
            for (int k = threadIdx.x; k < nlh; k += blockDim.x)
                lh[k] = 0;
        if (threadIdx.x == 0) {
            atomicMin(&c.rec->emin, blo);
            atomicMax(&c.rec->emax, bhi);
        }
        __syncthreads();
    }
    uint64_t sE = 0, sE2 = 0, sA = 0, sM2 = 0, sE3 = 0; // sE3: int64 bits (|sum| < 2^63 per block)
    const int lane = threadIdx.x & 63;
    // a weighted population: sums of w, wE, wE^2, wE^3, w|M|, wM^2, w^2 with w = pa_exp(lw)
    const bool wt = c.rec->weighted != 0u;
    double ws[PA_WPARTS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    static_assert(PA_HCHUNK % PA_CHUNK == 0 && PA_CHUNK % kThreads == 0, "whole chunks of whole passes");
    const int64_t chunks = (c.rd->cap + PA_CHUNK - 1) / PA_CHUNK;
    // kPre passes' loads are issued before the first pass's atomics (which
    // the compiler would not let later loads pass); a slot past the end loads
    // the last slot again and is not counted
    constexpr int kPre = 4;
    for (int64_t base0 = c.beg; base0 < c.end; base0 += kPre * (int64_t)blockDim.x) {
        int32_t pe[kPre], pm[kPre];
        uint32_t pl[kPre];
        double plw[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int64_t d = base0 + k * (int64_t)blockDim.x + threadIdx.x;
            const int64_t dc = d < c.end ? d : c.end - 1;
            pe[k] = dv.E[cur][dc];
            pm[k] = dv.M[cur][dc];
            pl[k] = dv.label[cur][dc];
            plw[k] = wt ? dv.lw[dc] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int64_t base = base0 + k * (int64_t)blockDim.x;
            if (base >= c.end)
                break;
            const int64_t d = base + threadIdx.x;
            const bool valid = d < c.end;
            uint32_t lab = 0xFFFFFFFFu;
            if (valid) {
                const int64_t e = pe[k], m = pm[k];
                if (build_hist) {
                    const int h = ((int)e + DN) >> 2;
                    if (nlh <= kObsLevels)
                        atomicAdd(&lh[h - hlo], 1u);
                    else
                        atomicAdd(&dv.hist[h], 1u);
                }
                sE += (uint64_t)e;
                sE2 += (uint64_t)(e * e);
                sE3 += (uint64_t)(e * e * e);
                sA += (uint64_t)(m < 0 ? -m : m);
                sM2 += (uint64_t)(m * m);
                lab = pl[k];
                if (wt) {
                    const double w = pa_exp(plw[k]), ef = (double)e, mf = (double)(m < 0 ? -m : m);
                    ws[0] = ws[0] + w;
                    ws[1] = ws[1] + w * ef;
                    ws[2] = ws[2] + w * (ef * ef);
                    ws[3] = ws[3] + w * (ef * ef * ef);
                    ws[4] = ws[4] + w * mf;
                    ws[5] = ws[5] + w * (mf * mf);
                    ws[6] = ws[6] + w * w;
                }
            }
            // family counts: one atomic per run of equal labels in the wave (the
            // resampling keeps copies adjacent, so runs are long)
            const uint32_t prev = (uint32_t)__shfl_up((int)lab, 1, 64);
            const bool start = valid && (lane == 0 || lab != prev);
            const uint64_t sm = __ballot(start), vm = __ballot(valid);
            if (start) {
                const uint64_t above = lane == 63 ? 0ull : ((sm | ~vm) & ~((2ull << lane) - 1ull));
                const int stop = above ? __ffsll((long long)above) - 1 : 64;
                atomicAdd(&dv.fam[lab], (uint32_t)(stop - lane));
            }
            // a weighted population's sums per chunk of PA_CHUNK slots, in the
            // fixed order of the block sum
            if (wt && ((base + (int64_t)blockDim.x) % PA_CHUNK == 0 || base + (int64_t)blockDim.x >= c.end)) {
                pa_block_sum_f64x(ws, sd);
                if (threadIdx.x == 0)
#pragma unroll
                    for (int f = 0; f < PA_WPARTS; ++f)
                        dv.wpart[f * chunks + base / PA_CHUNK] = ws[f];
#pragma unroll
                for (int f = 0; f < PA_WPARTS; ++f)
                    ws[f] = 0.0;
            }
        }
    }
    uint64_t sums[5] = {sE, sE2, sA, sM2, sE3};
    pa_block_sum_u64x(sums, su); // (its barriers also end the LDS counting)
    sE = sums[0];
    sE2 = sums[1];
    sA = sums[2];
    sM2 = sums[3];
    sE3 = sums[4];
    if (build_hist && nlh <= kObsLevels)
        for (int k = threadIdx.x; k < nlh; k += blockDim.x)
            if (lh[k])
                atomicAdd(&dv.hist[hlo + k], lh[k]);
    if (threadIdx.x == 0) {
        // 128-bit add of the block's signed sum: low word, then the high word
        // with the carry out of the low word (order-free, hence exact)
        const unsigned long long lo = sE3, hi = (long long)sE3 < 0 ? ~0ull : 0ull;
        const unsigned long long old = atomicAdd(&c.rec->accE3[0], lo);
        atomicAdd(&c.rec->accE3[1], hi + (old + lo < old ? 1ull : 0ull));
        atomicAdd(&c.rec->accE, (unsigned long long)sE);
        atomicAdd(&c.rec->accE2, (unsigned long long)sE2);
        atomicAdd(&c.rec->accAbsM, (unsigned long long)sA);
        atomicAdd(&c.rec->accM2, (unsigned long long)sM2);
    }
}

// Family statistics over PA_HCHUNK family slots per workgroup: sum of c^2,
// the number of families and sum of c ln c (partial[block], in the block's
// fixed order; k_obs_final adds them in block order); the counts return to
// zero for the next pass.
__global__ __launch_bounds__(kThreads) void k_obs_fam(const PaRunDesc *__restrict__ runs,
                                                      const PaBlk *__restrict__ map)
{
    __shared__ uint64_t su[16 * 2];
    __shared__ double sd[16];
    const PaBlk b = map[blockIdx.x];
    const PaRunDesc &rd = runs[b.run];
    PaRecord *rec = rd.dv.rec;
    if (frozen(rec))
        return;
    const int64_t beg = (int64_t)b.idx * PA_HCHUNK;
    const int64_t end = beg + PA_HCHUNK < rd.R0 ? beg + PA_HCHUNK : rd.R0;
    uint64_t c2 = 0, nf = 0;
    double cl = 0.0;
    // four passes' loads before their stores (a slot past the end loads the
    // last slot again and is not counted)
    constexpr int kPre = 4;
    for (int64_t f0 = beg; f0 < end; f0 += kPre * (int64_t)blockDim.x) {
        uint32_t pc[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int64_t f = f0 + k * (int64_t)blockDim.x + threadIdx.x;
            pc[k] = rd.dv.fam[f < end ? f : end - 1];
        }
#pragma unroll
        for (int k = 0; k < kPre; ++k) {
            const int64_t f = f0 + k * (int64_t)blockDim.x + threadIdx.x;
            const uint64_t c = pc[k];
            if (f < end && c) {
                c2 += c * c;
                rd.dv.fam[f] = 0;
                nf += 1;
                cl = cl + (double)c * log((double)c);
            }
        }
    }
    uint64_t sums[2] = {c2, nf};
    pa_block_sum_u64x(sums, su);
    cl = pa_block_sum_f64(cl, sd);
    if (threadIdx.x == 0) {
        atomicAdd(&rec->accC2, (unsigned long long)sums[0]);
        atomicAdd(&rec->accFam, (unsigned long long)sums[1]);
        rd.dv.partial[b.idx] = cl;
    }
}

// A signed 128-bit integer (two's complement words) to double: magnitude
// from its two non-negative words, so no cancellation between them.
__device__ __forceinline__ double i128_to_double(unsigned long long lo, unsigned long long hi)
{
    const bool neg = (long long)hi < 0;
    if (neg) {
        lo = ~lo + 1ull;
        hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    }
    const double m = (double)hi * 18446744073709551616.0 + (double)lo;
    return neg ? -m : m;
}

// Averages of step 4 and the family statistics: rho_t = sum_k c_k^2 / R
// (Eq. (6) with n_k = c_k / R), S_f = ln R - (1/R) sum_k c_k ln c_k.  A
// weighted population reports weighted averages sum_j w_j O_j / sum_j w_j and
// ESS = (sum w)^2 / sum w^2 (the integer sums and family statistics stay
// those of the members).  In a batched anneal the row of temperature point
// `point` is written too.
__global__ __launch_bounds__(kThreads) void k_obs_final(const PaRunDesc *__restrict__ runs, PaStepRecord *steprec,
                                                        int npoints, int point)
{
    __shared__ double sd[16];
    const PaRunDesc &rd = runs[blockIdx.x];
    PaRecord *rec = rd.dv.rec;
    const bool fz = frozen(rec);
    const bool wt = !fz && rec->weighted != 0u;
    const int nparts = (int)((rd.R0 + PA_HCHUNK - 1) / PA_HCHUNK); // k_obs_fam's workgroups
    double v = 0.0;
    if (!fz)
        for (int k = threadIdx.x; k < nparts; k += blockDim.x)
            v = v + rd.dv.partial[k];
    const double t = pa_block_sum_f64(v, sd);
    double ws[PA_WPARTS];
    if (wt) {
        const int64_t chunks = (rd.cap + PA_CHUNK - 1) / PA_CHUNK;
        const int nlive = (int)(((int64_t)rec->Rcur + PA_CHUNK - 1) / PA_CHUNK);
        for (int f = 0; f < PA_WPARTS; ++f) {
            double a = 0.0;
            for (int k = threadIdx.x; k < nlive; k += blockDim.x)
                a = a + rd.dv.wpart[f * chunks + k];
            ws[f] = pa_block_sum_f64(a, sd);
        }
    }
    if (threadIdx.x != 0)
        return;
    if (!fz) {
        rec->sumE = rec->accE;
        rec->sumE2 = rec->accE2;
        rec->sumAbsM = rec->accAbsM;
        rec->sumM2 = rec->accM2;
        rec->sumC2 = rec->accC2;
        rec->families = rec->accFam;
        rec->accE = rec->accE2 = rec->accAbsM = rec->accM2 = rec->accC2 = rec->accFam = 0;
        rec->sumE3[0] = rec->accE3[0];
        rec->sumE3[1] = rec->accE3[1];
        rec->accE3[0] = rec->accE3[1] = 0;
        const double n = (double)rd.N, r = (double)rec->Rcur;
        rec->e3 = i128_to_double(rec->sumE3[0], rec->sumE3[1]) / (n * n * n * r);
        rec->sumClnC = t;
        rec->e = (double)(long long)rec->sumE / (n * r);
        rec->e2 = (double)(long long)rec->sumE2 / (n * n * r);
        rec->abs_m = (double)(long long)rec->sumAbsM / (n * r);
        rec->m2 = (double)(long long)rec->sumM2 / (n * n * r);
        rec->rho_t = (double)rec->sumC2 / r;
        rec->S_f = log(r) - t / r;
        rec->ess = r;
        if (wt) {
            rec->e = ws[1] / ws[0] / n;
            rec->e2 = ws[2] / ws[0] / (n * n);
            rec->e3 = ws[3] / ws[0] / (n * n * n);
            rec->abs_m = ws[4] / ws[0] / n;
            rec->m2 = ws[5] / ws[0] / (n * n);
            rec->ess = ws[0] * ws[0] / ws[6];
        }
    }
    if (steprec) {
        PaStepRecord *o = steprec + (size_t)blockIdx.x * npoints + point;
        o->beta = rec->beta;
        o->lnQ = point > 0 ? rec->lnQ : 0.0;
        o->lnZ = rec->lnZ;
        o->sv = rec->sv;
        o->e = rec->e;
        o->e2 = rec->e2;
        o->abs_m = rec->abs_m;
        o->m2 = rec->m2;
        o->rho_t = rec->rho_t;
        o->S_f = rec->S_f;
        o->R = (long long)rec->Rcur;
        o->sumE = (long long)rec->sumE;
        o->sumE2 = (long long)rec->sumE2;
        o->sumAbsM = (long long)rec->sumAbsM;
        o->sumM2 = (long long)rec->sumM2;
        o->sumC2 = (long long)rec->sumC2;
        o->families = (long long)rec->families;
        o->status = rec->status;
    }
}

// ------------------------------------------------------------------ overlap
// Pairs replica d of run a with replica d of run b: per word column, the
// bit-sliced count of differing sites per replica, then q-histogram entry
// N - count.
__global__ __launch_bounds__(kThreads) void k_overlap(const PaRunDesc *__restrict__ A,
                                                      const PaRunDesc *__restrict__ B, unsigned long long *hist)
{
    __shared__ uint64_t red[kThreads / 64][16];
    const uint32_t w = blockIdx.x;
    const PaRecord *ra = A->dv.rec, *rb = B->dv.rec;
    const int64_t R = ra->Rcur < rb->Rcur ? (int64_t)ra->Rcur : (int64_t)rb->Rcur;
    if ((int64_t)w * 64 >= R)
        return;
    const int N = A->N;
    const uint64_t *a = A->dv.spins[ra->cur] + (size_t)w * N;
    const uint64_t *b = B->dv.spins[rb->cur] + (size_t)w * N;
    uint64_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t c16[16];
    // up to 64 sites per thread with 256 threads and N <= 16384: fits 8 planes
    for (int s = threadIdx.x; s < N; s += 2 * blockDim.x) {
        const int t = s + blockDim.x;
        vadd2_at<0>(v, a[s] ^ b[s], t < N ? a[t] ^ b[t] : 0ull);
    }
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

// Free-energy-weighted combination of runs (Eqs. (9)-(10)): for group g, the
// runs m with group_of[m] == g in index order; l_m = ln R_i^(m) + ln Z_hat_i^(m),
// omega_m = exp(l_m - l_max) / sum exp(l - l_max); ln Z of the pooled
// population = l_max + ln sum exp(l - l_max) - ln sum R^(m); moments are
// weighted averages and c, chi follow Eqs. (11)-(12).
__global__ void k_combine(const PaStepRecord *__restrict__ steprec, int npoints, int point,
                          const int32_t *__restrict__ group_of, int nruns, int ngroups, const int32_t *__restrict__ Ns,
                          double *__restrict__ out /* [ngroups][PA_COMBINE_FIELDS] */)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups)
        return;
    double lmax = -INFINITY, Rsum = 0.0;
    int n = 0, N = 0;
    for (int m = 0; m < nruns; ++m) {
        if (group_of[m] != g)
            continue;
        const PaStepRecord &r = steprec[(size_t)m * npoints + point];
        if (r.status & PA_ST_FROZEN)
            continue;
        const double l = log((double)r.R) + r.lnZ;
        lmax = l > lmax ? l : lmax;
        Rsum = Rsum + (double)r.R;
        N = Ns[m];
        ++n;
    }
    double den = 0.0, e = 0.0, e2 = 0.0, am = 0.0, m2 = 0.0, w2 = 0.0, beta = 0.0;
    double cn = 0.0, chn = 0.0, ep = 0.0, cp = 0.0, chp = 0.0; // naive weighted and plain means
    for (int m = 0; m < nruns && n > 0; ++m) {
        if (group_of[m] != g)
            continue;
        const PaStepRecord &r = steprec[(size_t)m * npoints + point];
        if (r.status & PA_ST_FROZEN)
            continue;
        den = den + exp(log((double)r.R) + r.lnZ - lmax);
        beta = r.beta;
    }
    for (int m = 0; m < nruns && n > 0; ++m) {
        if (group_of[m] != g)
            continue;
        const PaStepRecord &r = steprec[(size_t)m * npoints + point];
        if (r.status & PA_ST_FROZEN)
            continue;
        const double om = exp(log((double)r.R) + r.lnZ - lmax) / den;
        e = e + om * r.e;
        e2 = e2 + om * r.e2;
        am = am + om * r.abs_m;
        m2 = m2 + om * r.m2;
        w2 = w2 + om * om;
        const double c_m = beta * beta * (double)N * (r.e2 - r.e * r.e); // the run's own c and chi
        const double chi_m = beta * (double)N * (r.m2 - r.abs_m * r.abs_m);
        cn = cn + om * c_m;
        chn = chn + om * chi_m;
        ep = ep + r.e;
        cp = cp + c_m;
        chp = chp + chi_m;
    }
    double *o = out + (size_t)g * PA_COMBINE_FIELDS;
    o[0] = n > 0 ? lmax + log(den) - log(Rsum) : NAN;
    o[1] = e;
    o[2] = e2;
    o[3] = am;
    o[4] = m2;
    o[5] = beta * beta * (double)N * (e2 - e * e);
    o[6] = beta * (double)N * (m2 - am * am);
    o[7] = n > 0 ? 1.0 / w2 : 0.0;
    o[8] = (double)n;
    o[9] = beta;
    o[10] = cn;
    o[11] = chn;
    o[12] = n > 0 ? ep / (double)n : NAN;
    o[13] = n > 0 ? cp / (double)n : NAN;
    o[14] = n > 0 ? chp / (double)n : NAN;
}

// Imported state: thresholds of its beta and the scalars.
__global__ void k_set_beta(const PaRunDesc *__restrict__ runs, double beta, double lnZ, uint32_t step,
                           uint32_t sweeps, uint64_t R)
{
    PaRecord *rec = runs[blockIdx.x].dv.rec;
    if (threadIdx.x == 0) {
        rec->T[0] = pa_threshold(beta, 4);
        rec->T[1] = pa_threshold(beta, 8);
        rec->T[2] = pa_threshold(beta, 12);
        rec->beta = beta;
        rec->lnZ = lnZ;
        rec->step = step;
        rec->sweeps = sweeps;
        rec->Rcur = R;
        rec->sv = 0.0;
        rec->status = 0;
        rec->skip = 0;
        rec->weighted = 0;
        rec->keep = 0;
        rec->gather = 0;
    }
}

// Metropolis thresholds of every run set to those of `beta` (the autotuner
// times sweeps at a temperature of the anneal; the populations are drawn
// again afterwards).
__global__ void k_tune_beta(const PaRunDesc *__restrict__ runs, double beta)
{
    PaRecord *rec = runs[blockIdx.x].dv.rec;
    if (threadIdx.x == 0) {
        rec->T[0] = pa_threshold(beta, 4);
        rec->T[1] = pa_threshold(beta, 8);
        rec->T[2] = pa_threshold(beta, 12);
    }
}

// Generator throughput probe: Metropolis-purpose counters as the sweep forms
// them, three independent chains per thread, outputs folded into one word.
__global__ __launch_bounds__(kThreads) void k_philox_probe(uint32_t *__restrict__ out, int iters)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int i = 0; i < iters; ++i) {
        pa_philox_out o[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
            o[q] = pa_philox(1u, 2u, t, (uint32_t)i, 7u, (PA_PURPOSE_METRO << 28) | (uint32_t)q);
#pragma unroll
        for (int q = 0; q < 3; ++q)
            acc ^= o[q].x0 ^ o[q].x1 ^ o[q].x2 ^ o[q].x3;
    }
    out[t] = acc;
}

// Whether group g's sweeps take in the spins a resampling left in the other
// buffer (their column load gathers them) or a k_gather_spins pass of the
// resampling moves them: the gather in the load keeps the workgroup off the
// VALU for longer, which the other resident workgroups hide only when each
// SIMD holds four sweep waves (measured: 3D L = 10 and the uneven batch gain
// 2-6 %, 3D L = 16 at 256 lanes, three waves per SIMD, loses 1.3 %).  A
// function of the group's workgroup size, which the host keeps fixed between
// a resampling and the sweep after it.
bool sweep_gathers(const PaBatchView &v, int g)
{
    constexpr int kLdsPerCu = 163840, kWavesPerCu = 16; // gfx950 LDS; four waves per SIMD (<= 128 VGPRs)
    const int threads = v.gthreads[g], w = threads / 64;
    int blocks = (int)(kLdsPerCu / pa_sweep_lds_bytes(v.gN[g], v.gd[g], threads, v.gJ[g] != 0));
    if (blocks > kWavesPerCu / w)
        blocks = kWavesPerCu / w;
    return blocks * w >= kWavesPerCu;
}

hipError_t sweep_launch(const PaBatchView &v, int g, int theta, int threads, uint32_t t0, hipStream_t st,
                        int gather)
{
    if (v.gncol[g] == 0)
        return hipSuccess;
    const size_t lds = pa_sweep_lds_bytes(v.gN[g], v.gd[g], threads, v.gJ[g] != 0);
    if (gather && !sweep_gathers(v, g)) // gathered after the resampling
        gather = 0;
    if (v.gd[g] == 3)
        return pa_sweep3_launch(v.runs, v.gcol[g], v.gncol[g], threads, lds, st, v.gJ[g] != 0, theta, t0, gather);
    if (v.gJ[g])
        k_sweep<2, true><<<v.gncol[g], threads, lds, st>>>(v.runs, v.gcol[g], theta, t0, gather);
    else
        k_sweep<2, false><<<v.gncol[g], threads, lds, st>>>(v.runs, v.gcol[g], theta, t0, gather);
    return hipGetLastError();
}

} // namespace

// ====================================================================== launchers
size_t pa_sweep_lds_bytes(int N, int d, int threads, bool J)
{
    return (size_t)N * 8 + (size_t)(threads / 64) * kQueue * (3 * 8 + 4) +
           (size_t)(d == 2 ? ttab_words<2>() : ttab_words<3>()) * 4 +
           (J ? (((size_t)N + 7) & ~(size_t)7) : 0);
}

size_t pa_cluster_lds_bytes(int N, bool J)
{
    const size_t nw = kClusterThreads / 64, nred = (size_t)3 * N > 32 * nw ? (size_t)3 * N : 32 * nw;
    return ((size_t)N + nred) * 8 + nw * kClusterQueue * (8 + 4) + (J ? (((size_t)N + 7) & ~(size_t)7) : 0);
}

hipError_t pa_b_cluster(const PaBatchView &v, int nsteps, uint32_t t0)
{
    for (int g = 0; g < v.ngroups; ++g) {
        if (v.gncol[g] == 0)
            continue;
        const size_t lds = pa_cluster_lds_bytes(v.gN[g], v.gJ[g] != 0);
        if (v.gd[g] == 2 && v.gJ[g])
            k_cluster<2, true><<<v.gncol[g], kClusterThreads, lds, v.stream>>>(v.runs, v.gcol[g], nsteps, t0);
        else if (v.gd[g] == 2)
            k_cluster<2, false><<<v.gncol[g], kClusterThreads, lds, v.stream>>>(v.runs, v.gcol[g], nsteps, t0);
        else if (v.gJ[g])
            k_cluster<3, true><<<v.gncol[g], kClusterThreads, lds, v.stream>>>(v.runs, v.gcol[g], nsteps, t0);
        else
            k_cluster<3, false><<<v.gncol[g], kClusterThreads, lds, v.stream>>>(v.runs, v.gcol[g], nsteps, t0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t pa_query_lds(int *max_lds)
{
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess)
        *max_lds = v;
    return e;
}

hipError_t pa_b_init(const PaBatchView &v)
{
    k_init_rec<<<v.nruns, 64, 0, v.stream>>>(v.runs);
    k_hist_prep<<<v.nruns, kThreads, 0, v.stream>>>(v.runs);
    k_init_spins<<<v.ncol, kThreads, 0, v.stream>>>(v.runs, v.col);
    k_init_labels<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
    hipError_t e = hipGetLastError();
    for (int g = 0; g < v.ngroups && e == hipSuccess; ++g)
        e = sweep_launch(v, g, 0, v.gthreads[g], 0u, v.stream, 0);
    return e;
}

hipError_t pa_b_sweep_group(const PaBatchView &v, int g, int theta, int threads)
{
    return sweep_launch(v, g, theta, threads, 0u, v.stream, 0);
}

hipError_t pa_b_gather(const PaBatchView &v)
{
    for (int g = 0; g < v.ngroups; ++g)
        if (v.gncol[g] && sweep_gathers(v, g))
            k_gather_spins<false><<<v.gncol[g], kThreads, 0, v.stream>>>(v.runs, v.gcol[g]);
    return hipGetLastError();
}

hipError_t pa_b_sweep(const PaBatchView &v, int theta, uint32_t t0, int gather)
{
    hipError_t e = hipSuccess;
    if (v.ngroups < 2 || !v.fork) {
        for (int g = 0; g < v.ngroups && e == hipSuccess; ++g)
            e = sweep_launch(v, g, theta, v.gthreads[g], t0, v.stream, gather);
        return e;
    }
    // the groups are independent: each on its own stream, so that one group's
    // last partly filled round of workgroups overlaps the others' work
    e = hipEventRecord(v.fork, v.stream);
    for (int g = 0; g < v.ngroups && e == hipSuccess; ++g) {
        e = hipStreamWaitEvent(v.gstream[g], v.fork, 0);
        if (e == hipSuccess)
            e = sweep_launch(v, g, theta, v.gthreads[g], t0, v.gstream[g], gather);
        if (e == hipSuccess)
            e = hipEventRecord(v.join[g], v.gstream[g]);
    }
    for (int g = 0; g < v.ngroups && e == hipSuccess; ++g)
        e = hipStreamWaitEvent(v.stream, v.join[g], 0);
    return e;
}

// The level histogram of the current populations, from the state the host
// tracks: valid (nothing to do), zero (build it) or stale (clear, then build).
static hipError_t hist_launch(const PaBatchView &v, int state)
{
    if (state == PA_HIST_VALID)
        return hipSuccess;
    if (state == PA_HIST_STALE)
        k_hist_prep<<<v.nruns, kThreads, 0, v.stream>>>(v.runs);
    k_hist<<<v.nhrep, kThreads, (size_t)v.maxH * 4, v.stream>>>(v.runs, v.hrep);
    return hipGetLastError();
}


hipError_t pa_b_reweight(const PaBatchView &v, double beta_next, int hist_state)
{
    hipError_t e = hist_launch(v, hist_state);
    if (e != hipSuccess)
        return e;
    k_reweight<<<v.nruns, 1024, 0, v.stream>>>(v.runs, beta_next);
    if (v.weights) { // runs that may hold a weighted population
        k_rw_max<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
        k_rw_sum<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
        k_rw_final<<<v.nruns, kThreads, 0, v.stream>>>(v.runs);
    }
    return hipGetLastError();
}

hipError_t pa_b_rule(const PaBatchView &v, double alpha_star, double dbeta_max, int iterations, int bisect,
                     int hist_state)
{
    hipError_t e = hist_launch(v, hist_state);
    if (e != hipSuccess)
        return e;
    k_rule<<<v.nruns, kRuleThreads, 0, v.stream>>>(v.runs, alpha_star, dbeta_max, iterations, bisect);
    return hipGetLastError();
}

hipError_t pa_b_features(const PaBatchView &v, int hist_state)
{
    hipError_t e = hist_launch(v, hist_state);
    if (e != hipSuccess)
        return e;
    k_features<<<v.nruns, kRuleThreads, 0, v.stream>>>(v.runs);
    return hipGetLastError();
}

// after pa_b_features and the model's proposal (the histogram is current)
hipError_t pa_b_check_candidate(const PaBatchView &v, double alpha_star, double dbeta_max, int iterations,
                                double bracket, int refine)
{
    k_check_candidate<<<v.nruns, kRuleThreads, 0, v.stream>>>(v.runs, alpha_star, dbeta_max, iterations, bracket,
                                                              refine);
    return hipGetLastError();
}

// Launches per scheme (after the reweighting): nearest integer and Poisson
// draw the copy numbers and sum them into the ancestor map in one pass;
// systematic sums the weights and writes the ancestor map from each
// replica's closed-form copy range in the same pass; multinomial sums the
// weights, draws, adds the sampling variance and sums the copy numbers.
// Then the energies, magnetisations and labels move to the ancestors' order
// and the commit swaps the buffers; the spins follow at once for groups whose
// sweeps do not gather them, else in the next sweep or pa_b_gather.
hipError_t pa_b_resample(const PaBatchView &v, int scheme, int freeze, int kq, bool prepped)
{
    hipError_t e;
    if (!prepped)
        k_resample_prep<<<v.nruns, kThreads, 0, v.stream>>>(v.runs);
    if (kq >= 0)
        k_cond_decide<<<v.nruns, 64, 0, v.stream>>>(v.runs, (uint32_t)kq);
    switch (scheme) {
    case 2:
        k_counts_scan<2><<<v.ncrep, kThreads, 0, v.stream>>>(v.runs, v.crep);
        break;
    case 1:
        k_counts_scan<1><<<v.ncrep, kThreads, 0, v.stream>>>(v.runs, v.crep);
        break;
    case 3:
    case 0:
        if (scheme == 3) {
            k_weights_scan<PA_SCAN_SYSTEMATIC><<<v.ncrep, kThreads, 0, v.stream>>>(v.runs, v.crep);
        } else {
            k_weights_scan<PA_SCAN_MULTINOMIAL><<<v.ncrep, kThreads, 0, v.stream>>>(v.runs, v.crep);
            k_counts_multinomial<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
            k_sv_partial<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
            k_scan_counts<<<v.ntile, PA_SCAN_THREADS, 0, v.stream>>>(v.runs, v.tile);
        }
        break;
    default:
        return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // with no group whose sweeps gather, every spin moves now in the same pass
    // as the energies, magnetisations and labels; otherwise those move now and
    // the spins of the other groups right after the commit
    bool any = false;
    for (int g = 0; g < v.ngroups; ++g)
        any = any || (v.gncol[g] && sweep_gathers(v, g));
    if (any)
        k_gather_meta<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
    else
        k_gather_spins<true><<<v.ncol, kThreads, 0, v.stream>>>(v.runs, v.col);
    if (kq >= 0)
        k_keep<<<v.nrep, kThreads, 0, v.stream>>>(v.runs, v.rep);
    k_commit<<<v.nruns, kThreads, 0, v.stream>>>(v.runs, freeze, any ? 0 : 1);
    for (int g = 0; any && g < v.ngroups; ++g)
        if (v.gncol[g] && !sweep_gathers(v, g))
            k_gather_spins<false><<<v.gncol[g], kThreads, 0, v.stream>>>(v.runs, v.gcol[g]);
    return hipGetLastError();
}

hipError_t pa_b_observables(const PaBatchView &v, int point, int hist_state)
{
    if (hist_state == PA_HIST_STALE)
        k_hist_prep<<<v.nruns, kThreads, 0, v.stream>>>(v.runs);
    k_obs_rep<<<v.nhrep, kThreads, 0, v.stream>>>(v.runs, v.hrep, hist_state != PA_HIST_VALID);
    k_obs_fam<<<v.nfam, kThreads, 0, v.stream>>>(v.runs, v.fam);
    k_obs_final<<<v.nruns, kThreads, 0, v.stream>>>(v.runs, point >= 0 ? v.steprec : nullptr, v.npoints,
                                                    point);
    return hipGetLastError();
}

hipError_t pa_b_set_beta(const PaBatchView &v, double beta, double lnZ, uint32_t step, uint32_t sweeps,
                         uint64_t R)
{
    k_set_beta<<<v.nruns, 64, 0, v.stream>>>(v.runs, beta, lnZ, step, sweeps, R);
    return hipGetLastError();
}

hipError_t pa_b_tune_beta(const PaBatchView &v, double beta)
{
    k_tune_beta<<<v.nruns, 64, 0, v.stream>>>(v.runs, beta);
    return hipGetLastError();
}

hipError_t pa_launch_combine(const PaBatchView &v, int point, const int32_t *group_of, int ngroups,
                             const int32_t *Ns, double *out)
{
    k_combine<<<(ngroups + 63) / 64, 64, 0, v.stream>>>(v.steprec, v.npoints, point, group_of, (int)v.nruns,
                                                        ngroups, Ns, out);
    return hipGetLastError();
}

hipError_t pa_launch_philox_probe(uint32_t *out, int64_t nthreads, int iters, hipStream_t st)
{
    k_philox_probe<<<(unsigned)(nthreads / kThreads), kThreads, 0, st>>>(out, iters);
    return hipGetLastError();
}

hipError_t pa_launch_overlap(const PaRunDesc *a, const PaRunDesc *b, int N, uint32_t ncols_a,
                             unsigned long long *hist, hipStream_t st)
{
    k_fill_u32<<<grid_for((int64_t)(N + 1) * 2), kThreads, 0, st>>>(reinterpret_cast<uint32_t *>(hist),
                                                                     (int64_t)(N + 1) * 2, 0u);
    k_overlap<<<ncols_a, kThreads, 0, st>>>(a, b, hist);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free overlap
// The overlap histogram of pa_overlap_noalloc lives in this file-scope device
// array instead of a run's workspace: PA_NOALLOC_HIST_MAX counters (the
// largest lattice's N + 1), 128 KiB per device, held until the process ends.
// Every call on a device shares that device's copy.  In host code `scratch`
// names a host-side stand-in, never the device memory: the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is passed to kernels.
static __device__ __align__(256) unsigned long long scratch[PA_NOALLOC_HIST_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
} // namespace

hipError_t pa_noalloc_scratch(int device, unsigned long long **out)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess)
            return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess)
            return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess)
                e = e2;
        }
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned long long *>(g_scratch_ptr[device]);
    return hipSuccess;
}
