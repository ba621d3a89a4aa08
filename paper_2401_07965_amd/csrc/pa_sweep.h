// The sweep kernel and what it shares with the other kernels of the hot
// path, for gfx950 (MI355X): included by pa_kernels.hip (2D sweeps and every
// other kernel) and by pa_sweep3.hip (3D sweeps, compiled with their own
// scheduling flags).  Spins are multi-spin coded: bit b of word [w][s] is
// replica 64w+b at site s, 1 meaning sigma = -1.
#pragma once
#include "pa_device.h"
#include "pa_internal.h"

#include <type_traits>

namespace {

constexpr int kThreads = 256;
constexpr int kSweepMaxThreads = 768;
constexpr int kRuleThreads = 1024;
constexpr int kRuleCache = 4096; // levels whose weights stay in LDS between the two sums

__device__ __forceinline__ bool frozen(const PaRecord *rec) { return (rec->status & PA_ST_FROZEN) != 0u; }

// Workgroups of a launch go to the 8 XCDs in turn (block b to XCD b mod 8).
// This permutation hands each XCD one contiguous range of [0, n), so blocks
// that read neighbouring data share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n)
{
    const uint32_t x = b & 7u, k = b >> 3, q = n >> 3, r = n & 7u;
    return (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + k;
}

// Workgroup-uniform values read from device memory, kept in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x)
{
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | (uint64_t)uni((uint32_t)x);
}

// ------------------------------------------------------------------ step 3: sweeps
constexpr int kXor3 = PA_T3(PA_A ^ PA_B ^ PA_C);
constexpr int kMaj = PA_T3((PA_A & PA_B) | (PA_A & PA_C) | (PA_B & PA_C));

// Adds the masks a and b at plane P of a bit-sliced count (one full adder,
// then the carry rippled up to plane 7).
template <int P>
__device__ __forceinline__ void vadd2_at(uint64_t c[8], uint64_t a, uint64_t b)
{
    uint64_t x = pa_bop3<kMaj>(c[P], a, b);
    c[P] = pa_bop3<kXor3>(c[P], a, b);
#pragma unroll
    for (int k = P + 1; k < 8; ++k) {
        const uint64_t t = c[k] & x;
        c[k] ^= x;
        x = t;
    }
}

// The value of lane l ^ M, for the butterfly levels below (all lanes active).
// Levels 1 and 2 are quad permutations; from level 4 on, each lane's value
// is its group's sum so far, so any partner in the other half of the next
// larger group will do: the mirrors within 8 and 16 lanes stand in for xor 4
// and xor 8.  xor 16 is a swizzle within 32 lanes, xor 32 a lane permute.
template <int M>
__device__ __forceinline__ uint32_t xlane(uint32_t v)
{
    if (M == 1)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false); // quad_perm 1,0,3,2
    if (M == 2)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false); // quad_perm 2,3,0,1
    if (M == 4)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false); // row_half_mirror
    if (M == 8)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false); // row_mirror
    if (M == 16)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F); // and 0x1F, xor 0x10
    return (uint32_t)__shfl_xor((int)v, 32, 64);
}

// One butterfly level: adds the partner's count.  Counts are below
// 2^(8 + LV) before level LV (per-lane counts below 2^8), so only those
// planes move and the carry lands in plane 8 + LV.
template <int LV, int M>
__device__ __forceinline__ void vsum_level(uint64_t c[16])
{
    uint64_t carry = 0;
#pragma unroll
    for (int k = 0; k < 8 + LV; ++k) {
        const uint64_t o = ((uint64_t)xlane<M>((uint32_t)(c[k] >> 32)) << 32) | xlane<M>((uint32_t)c[k]);
        const uint64_t sum = pa_bop3<kXor3>(c[k], o, carry);
        carry = pa_bop3<kMaj>(c[k], o, carry);
        c[k] = sum;
    }
    c[8 + LV] = carry;
}

// Sum of the bit-sliced counters of all 64 lanes: planes 0..7 in (counts
// below 2^8, planes 8..15 zero), the 16-plane wave total out in every lane.
__device__ __forceinline__ void wave_vsum16(uint64_t c[16])
{
    vsum_level<0, 1>(c);
    vsum_level<1, 2>(c);
    vsum_level<2, 4>(c);
    vsum_level<3, 8>(c);
    vsum_level<4, 16>(c);
    vsum_level<5, 32>(c);
}

// All-ones if bit k of jb is set (one signed bit-field extract; both halves alike).
__device__ __forceinline__ uint64_t jbit(uint32_t jb, int k)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)jb, (uint32_t)k, 1u);
    return ((uint64_t)m << 32) | m;
}

// Unsatisfied-bond mask of a bond between words S and n: S ^ n, inverted for
// an antiferromagnetic coupling (bit k of jb).
template <bool J>
__device__ __forceinline__ uint64_t bond(uint64_t S, uint64_t n, uint32_t jb, int k)
{
    if (!J)
        return S ^ n;
    return pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>(S, n, jbit(jb, k));
}

// Bit-plane decision of u < T for the undecided replicas of one word: plane
// pair q of Philox(s, w, i, METRO<<28 | t<<8 | q) gives bits 31-2q and 30-2q of
// every replica's uniform; a replica is decided at the first bit where u and
// its class threshold differ (accepted if u has 0 there).
struct PlaneCtx {
    uint32_t seed, run_id, w, step, t;
    uint32_t t4, t8, t12;
};

// All-ones if bit b of the threshold t is set (one signed bit-field extract;
// both halves alike).
__device__ __forceinline__ uint64_t tbit(uint32_t t, int b)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)t, (uint32_t)b, 1u);
    return ((uint64_t)m << 32) | m;
}

// The threshold bit on one plane of every undecided replica, from the
// classes' bits t4, t8, t12 on that plane (masks).  The undecided replicas
// all belong to the drawing classes, which are disjoint, so on them
// Tp = m4 ? t4 : t8 in 2D and m4 ? t4 : (m8 ? t8 : t12) in 3D; the value on
// other replicas is never used.
template <int D>
__device__ __forceinline__ uint64_t plane_threshold_m(uint64_t m4, uint64_t m8, uint64_t t4, uint64_t t8,
                                                      uint64_t t12)
{
    constexpr int kSel = PA_T3((PA_A & PA_B) | (~PA_A & PA_C));
    const uint64_t t = D == 2 ? t8 : pa_bop3<kSel>(m8, t8, t12);
    return pa_bop3<kSel>(m4, t4, t);
}

// The same on plane (bit) b.  `last` is the last class's bit (T8_b in 2D,
// T12_b in 3D) as a mask, passed in so that it can come from a vector
// register: one instruction takes at most one scalar operand.
template <int D>
__device__ __forceinline__ uint64_t plane_threshold(const PlaneCtx &pc, int b, uint64_t m4, uint64_t m8,
                                                    uint64_t last)
{
    return plane_threshold_m<D>(m4, m8, tbit(pc.t4, b), D == 2 ? last : tbit(pc.t8, b), last);
}

// A threshold-bit mask (0 or all-ones) as a 64-bit mask.
__device__ __forceinline__ uint64_t dup32(uint32_t m) { return ((uint64_t)m << 32) | m; }

// One plane: returns the replicas accepted on it (u has 0, the threshold 1);
// those where u and the threshold agree stay undecided.
__device__ __forceinline__ uint64_t plane_step(uint64_t P, uint64_t Tp, uint64_t &und)
{
    const uint64_t a = pa_bop3<PA_T3(PA_A & ~PA_B & PA_C)>(und, P, Tp);
    und = pa_bop3<PA_T3(PA_A & ~(PA_B ^ PA_C))>(und, P, Tp);
    return a;
}

__device__ __forceinline__ pa_philox_out metro_philox(const PlaneCtx &pc, uint32_t s, uint32_t q)
{
    return pa_philox(pc.seed, pc.run_id, s, pc.w, pc.step, (PA_PURPOSE_METRO << 28) | (pc.t << 8) | q);
}

// The products shared by a site's plane pairs (one share per site and sweep
// for its inline pairs).
__device__ __forceinline__ pa_philox_shared metro_share(const PlaneCtx &pc, uint32_t s)
{
    return pa_philox_share(pc.seed, pc.run_id, s, pc.w, pc.step);
}

// A plane pair given its two planes' thresholds T0, T1.  The undecided set
// comes in as uin (its complement if INV) and leaves in und.
template <bool INV>
__device__ __forceinline__ void pair_core(const pa_philox_out &o, uint64_t T0, uint64_t T1, uint64_t uin,
                                          uint64_t &und, uint64_t &acc)
{
    const uint64_t P0 = (uint64_t)o.x0 | ((uint64_t)o.x1 << 32);
    const uint64_t P1 = (uint64_t)o.x2 | ((uint64_t)o.x3 << 32);
    uint64_t a0;
    if (INV) {
        a0 = pa_bop3<PA_T3(~PA_A & ~PA_B & PA_C)>(uin, P0, T0);
        und = pa_bop3<PA_T3(~PA_A & ~(PA_B ^ PA_C))>(uin, P0, T0);
    } else {
        und = uin;
        a0 = plane_step(P0, T0, und);
    }
    const uint64_t a1 = plane_step(P1, T1, und);
    acc = pa_bop3<PA_T3(PA_A | PA_B | PA_C)>(acc, a0, a1);
}

// Plane pair q; last0, last1: the last class's threshold bits on its planes.
template <int D, bool INV = false>
__device__ __forceinline__ void apply_pair(const PlaneCtx &pc, const pa_philox_out &o, uint32_t q, uint64_t m4,
                                           uint64_t m8, uint64_t last0, uint64_t last1, uint64_t uin,
                                           uint64_t &und, uint64_t &acc)
{
    const int b0 = 31 - 2 * (int)q;
    pair_core<INV>(o, plane_threshold<D>(pc, b0, m4, m8, last0), plane_threshold<D>(pc, b0 - 1, m4, m8, last1),
                   uin, und, acc);
}

// Plane pair q of a queued item: the threshold bits come from the launch's
// table, tt[ttab_stride<D>() q + 2 c + j] = class c's bit on plane j of pair q as
// a mask (classes dE = 4, 8 and, in 3D, 12).
template <int D>
constexpr int ttab_stride() { return D == 2 ? 4 : 8; }

template <int D>
__device__ __forceinline__ void apply_pair_queued(const uint32_t *tt, const pa_philox_out &o, uint32_t q,
                                                  uint64_t m4, uint64_t m8, uint64_t &und, uint64_t &acc)
{
    const uint4 a = *reinterpret_cast<const uint4 *>(tt + ttab_stride<D>() * q);
    if (D == 2) {
        pair_core<false>(o, plane_threshold_m<D>(m4, m8, dup32(a.x), dup32(a.z), 0ull),
                         plane_threshold_m<D>(m4, m8, dup32(a.y), dup32(a.w), 0ull), und, und, acc);
    } else {
        const uint2 b = *reinterpret_cast<const uint2 *>(tt + ttab_stride<D>() * q + 4);
        pair_core<false>(o, plane_threshold_m<D>(m4, m8, dup32(a.x), dup32(a.z), dup32(b.x)),
                         plane_threshold_m<D>(m4, m8, dup32(a.y), dup32(a.w), dup32(b.y)), und, und, acc);
    }
}

// Per-wave queue of word-sites whose replicas are still undecided after the
// first kInlinePairs plane pairs: they are compacted into full 64-lane
// batches (one plane pair per batch) instead of keeping the wave waiting for
// its slowest lane.  Results are the same: each site's planes are the same
// Philox outputs, taken in the same order.
constexpr int kInlinePairs = 3;
constexpr int kQueue = 128; // per wave; never more than 127 items are live
// threshold-bit table: 16 plane pairs x (2 classes in 2D, 3 in 3D, padded to 4) x 2 planes
template <int D>
constexpr int ttab_words() { return 16 * ttab_stride<D>(); }

struct WaveQueue {
    uint32_t *sq;  // site | next pair << 16
    uint64_t *und, *m4, *m8; // m8: 3D only
    const uint32_t *tt;      // threshold-bit masks per plane pair (apply_pair_queued)
};

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Appends this lane's item if `has`; returns the new item count (wave-uniform).
template <int D>
__device__ __forceinline__ uint32_t queue_push(const WaveQueue &Q, uint32_t head, uint32_t cnt, bool has,
                                               uint32_t sq, uint64_t und, uint64_t m4, uint64_t m8)
{
    const uint64_t bal = __ballot(has);
    if (has) {
        const uint32_t slot = (head + cnt + (uint32_t)__popcll(bal & lanemask_lt())) & (kQueue - 1);
        Q.sq[slot] = sq;
        Q.und[slot] = und;
        Q.m4[slot] = m4;
        if (D == 3)
            Q.m8[slot] = m8;
    }
    __builtin_amdgcn_wave_barrier();
    return cnt + (uint32_t)__popcll(bal);
}

// One plane pair for up to 64 queued items; the still undecided go back.
// calls: the wave's Philox evaluations (wave-uniform), n per pass.
template <int D>
__device__ __forceinline__ void queue_pass(const WaveQueue &Q, const PlaneCtx &pc, uint64_t *lat, uint32_t &head,
                                           uint32_t &cnt, uint32_t &calls)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t n = cnt < 64u ? cnt : 64u;
    const bool act = lane < n;
    uint32_t sq = 0;
    uint64_t und = 0, m4 = 0, m8 = 0;
    if (act) {
        const uint32_t slot = (head + lane) & (kQueue - 1);
        sq = Q.sq[slot];
        und = Q.und[slot];
        m4 = Q.m4[slot];
        if (D == 3)
            m8 = Q.m8[slot];
    }
    __builtin_amdgcn_wave_barrier();
    head += n;
    cnt -= n;
    const uint32_t s = sq & 0xFFFFu, q = sq >> 16;
    calls += n;
    if (act) {
        uint64_t acc = 0;
        apply_pair_queued<D>(Q.tt, metro_philox(pc, s, q), q, m4, m8, und, acc);
        lat[s] ^= acc;
    }
    const bool again = act && und != 0 && q + 1 < 16;
    cnt = queue_push<D>(Q, head, cnt, again, s | ((q + 1) << 16), und, m4, m8);
}

// The last items of a colour: up to 64 at a time, each lane taking its
// item's remaining plane pairs in turn until the item is decided, with no
// requeueing (the site passes leave fewer than 64, so this is one batch).
// calls: this lane's Philox evaluations.
template <int D>
__device__ __forceinline__ void queue_drain(const WaveQueue &Q, const PlaneCtx &pc, uint64_t *lat, uint32_t &head,
                                            uint32_t &cnt, uint32_t &calls)
{
    const uint32_t lane = threadIdx.x & 63;
    while (cnt > 0u) {
        const uint32_t n = cnt < 64u ? cnt : 64u;
        const bool act = lane < n;
        uint32_t sq = 0;
        uint64_t und = 0, m4 = 0, m8 = 0;
        if (act) {
            const uint32_t slot = (head + lane) & (kQueue - 1);
            sq = Q.sq[slot];
            und = Q.und[slot];
            m4 = Q.m4[slot];
            if (D == 3)
                m8 = Q.m8[slot];
        }
        __builtin_amdgcn_wave_barrier();
        head += n;
        cnt -= n;
        const uint32_t s = sq & 0xFFFFu;
        uint64_t acc = 0;
        for (uint32_t q = sq >> 16; und != 0 && q < 16u; ++q) {
            apply_pair_queued<D>(Q.tt, metro_philox(pc, s, q), q, m4, m8, und, acc);
            ++calls;
        }
        if (act)
            lat[s] ^= acc;
    }
}

// Recount of a column after its updates: each replica's unsatisfied-bond
// count U and number of down spins, bit-sliced (forward bonds once each, two
// sites per pass added with full adders, then a wave butterfly and the waves'
// partial counts in red[32 per wave]): E = 2U - dN, M = N - 2 n_down.  Also
// writes the lattice back to g.  Per-lane counts stay below 2^8: at most
// ceil(N / blockDim) sites per lane, d bonds each (the launch checks).
template <int D, bool J>
__device__ __forceinline__ void recount_column(const uint64_t *lat, const uint8_t *jl, uint64_t *g, uint64_t *red,
                                               const PaRunDesc &rd, int cur, uint32_t w, int64_t Rlive, int L,
                                               int N, int LL, uint32_t mL)
{
    const int tid = threadIdx.x, bs = blockDim.x;
    uint64_t ve[8] = {0, 0, 0, 0, 0, 0, 0, 0}, vm[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = tid; s < N; s += 2 * bs) {
        uint64_t S[2] = {0, 0}, e[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = s + h * bs;
            if (h == 0 || t < N) {
                const int row = (int)__umulhi((uint32_t)t, mL);
                const int x = t - row * L;
                const int z = (D == 2) ? 0 : (int)__umulhi((uint32_t)row, mL);
                const int y = row - z * L;
                const uint32_t jb = J ? (uint32_t)jl[t] : 0u;
                S[h] = lat[t];
                e[h][0] = bond<J>(S[h], lat[x == L - 1 ? t - (L - 1) : t + 1], jb, 0);
                e[h][1] = bond<J>(S[h], lat[y == L - 1 ? t - L * (L - 1) : t + L], jb, 1);
                if (D == 3)
                    e[h][2] = bond<J>(S[h], lat[z == L - 1 ? t - LL * (L - 1) : t + LL], jb, 2);
                g[t] = S[h];
            }
        }
        if (D == 2) {
            const uint64_t k1 = pa_bop3<kMaj>(ve[0], e[0][0], e[0][1]);
            ve[0] = pa_bop3<kXor3>(ve[0], e[0][0], e[0][1]);
            const uint64_t k2 = pa_bop3<kMaj>(ve[0], e[1][0], e[1][1]);
            ve[0] = pa_bop3<kXor3>(ve[0], e[1][0], e[1][1]);
            vadd2_at<1>(ve, k1, k2);
        } else {
            // each site's three bonds as sum + 2 carry, then plane by plane
            const uint64_t sA = pa_bop3<kXor3>(e[0][0], e[0][1], e[0][2]);
            const uint64_t cA = pa_bop3<kMaj>(e[0][0], e[0][1], e[0][2]);
            const uint64_t sB = pa_bop3<kXor3>(e[1][0], e[1][1], e[1][2]);
            const uint64_t cB = pa_bop3<kMaj>(e[1][0], e[1][1], e[1][2]);
            const uint64_t k1 = pa_bop3<kMaj>(ve[0], sA, sB);
            ve[0] = pa_bop3<kXor3>(ve[0], sA, sB);
            const uint64_t k2 = pa_bop3<kMaj>(ve[1], cA, cB);
            ve[1] = pa_bop3<kXor3>(ve[1], cA, cB);
            const uint64_t k3 = ve[1] & k1;
            ve[1] ^= k1;
            vadd2_at<2>(ve, k2, k3);
        }
        vadd2_at<0>(vm, S[0], S[1]);
    }
    // the two bit-sliced counts reduced one after the other (fewer live registers)
    const int wave = tid >> 6, lane = tid & 63, nw = bs >> 6;
    {
        uint64_t c[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            c[k] = k < 8 ? ve[k] : 0;
        wave_vsum16(c);
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 16; ++k)
                red[wave * 32 + k] = c[k];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            c[k] = k < 8 ? vm[k] : 0;
        wave_vsum16(c);
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 16; ++k)
                red[wave * 32 + 16 + k] = c[k];
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t U = 0, nd = 0;
        for (int v = 0; v < nw; ++v)
            for (int k = 0; k < 16; ++k) {
                U += (uint32_t)((red[v * 32 + k] >> lane) & 1u) << k;
                nd += (uint32_t)((red[v * 32 + 16 + k] >> lane) & 1u) << k;
            }
        const int64_t r = 64 * (int64_t)w + lane;
        if (r < Rlive) {
            rd.dv.E[cur][r] = 2 * (int32_t)U - D * N;
            rd.dv.M[cur][r] = N - 2 * (int32_t)nd;
        }
    }
}

// The theta sweeps of one column in LDS.  ALL: every energy-change class has
// a threshold strictly between 0 and 2^32 (the usual case), so no class is
// decided without random bits.
struct SweepGeom {
    int L, N, half, nh, LL;
    uint32_t mhalf, mL; // ceil(2^32 / half), ceil(2^32 / L)
};

// Site k of colour c (k < N/2): row = y + L z = k div (L/2), x = 2 (k mod L/2)
// + (y + z + c) mod 2.  Colour-c sites are independent and each one's random
// bits are keyed by its site index, so the order in which lanes visit them
// does not change any result.  FIX: the workgroup size is a multiple of L
// (2D) or L^2 (3D), so from one iteration to the next a lane's site moves by
// 2 * blockDim sites along y (2D) or z (3D) and its other coordinates stay:
// their neighbour offsets are computed once per colour.
// zp: the number of leading inline plane pairs on which every drawing class's
// threshold has 0 bits (their planes lie above the largest threshold): there
// a differing bit can only reject, so such a pair decides as und &= ~(P0 | P1).
// ZU (3D, FIX): every wave's sites share their z in each pass (L^2 / 2 colour
// sites per z plane, a multiple of 64), so the z neighbours' offsets are
// wave-uniform: +-L^2, or across the periodic boundary when the wave's
// plane is the last or the first.
// Returns the Philox evaluations, summed over the wave's lanes.
template <int D, bool J, bool ALL, bool FIX, bool ZU = false>
__device__ __forceinline__ uint32_t sweep_columns(uint64_t *lat, const uint8_t *jl, const SweepGeom &G, PlaneCtx pc,
                                                  const WaveQueue &Q, int theta, uint32_t t0, uint64_t sure4,
                                                  uint64_t sure8, uint64_t sure12, uint64_t draw4, uint64_t draw8,
                                                  uint64_t draw12, int zp)
{
    const int L = G.L, N = G.N, half = G.half, nh = G.nh, LL = G.LL;
    const uint32_t mhalf = G.mhalf, mL = G.mL;
    const int tid = threadIdx.x, bs = blockDim.x;
    // FIX: stride of the coordinate that moves (y in 2D, z in 3D); a step
    // across the periodic boundary along it is a step modulo N
    const uint32_t vst = D == 2 ? (uint32_t)L : (uint32_t)LL;
    // the last class's threshold bits on the inline planes, kept in vector
    // registers for the whole launch
    uint32_t tl[2 * kInlinePairs];
#pragma unroll
    for (int i = 0; i < 2 * kInlinePairs; ++i) {
        tl[i] = (uint32_t)__builtin_amdgcn_sbfe((int)(D == 2 ? pc.t8 : pc.t12), 31u - (uint32_t)i, 1u);
        asm volatile("" : "+v"(tl[i]));
    }
    // Philox evaluations: the wave's count of site and queue passes
    // (wave-uniform) and this lane's count of its end-of-colour items
    uint32_t wcalls = 0, calls = 0;
    for (int tt = 0; tt < theta; ++tt) {
        pc.t = t0 + (uint32_t)tt;
        for (int c = 0; c < 2; ++c) {
            uint32_t head = 0, cnt = 0;
            int sf = 0, oxp = 0, oxm = 0, oyp = 0, oym = 0;
            if (FIX) { // the lane's first site, and the offsets that stay
                const int row = half > 1 ? (int)__umulhi((uint32_t)tid, mhalf) : tid;
                const int m = tid - row * half;
                const int z = (D == 2) ? 0 : (int)__umulhi((uint32_t)row, mL);
                const int y = row - z * L;
                const int x = 2 * m + ((y + z + c) & 1);
                sf = x + L * row;
                oxp = x == L - 1 ? -(L - 1) : 1;
                oxm = x == 0 ? L - 1 : -1;
                oyp = y == L - 1 ? -L * (L - 1) : L;
                oym = y == 0 ? L * (L - 1) : -L;
            }
            // one pass over bs sites of the colour; RAGGED: some lanes have no
            // site (only the last pass, when bs does not divide N/2)
            auto pass = [&](const int kb, auto ragged) {
                constexpr bool RAGGED = decltype(ragged)::value;
                const int k = kb + tid;
                // a lane without a site (RAGGED) keeps und = 0 and always =
                // ~0: no pair, no push
                uint64_t und = 0, m4 = 0, m8 = 0, always = ~0ull, acc = 0, S = 0;
                uint32_t s = 0;
                if (!RAGGED || k < nh) {
                    uint64_t n0, n1, n2, n3, n4 = 0, n5 = 0;
                    if (FIX) {
                        s = (uint32_t)sf;
                        n0 = lat[sf + oxp];
                        n1 = lat[sf + oxm];
                        uint64_t nu, nd;
                        if (ZU) { // the wave's z plane decides both offsets
                            const int s0 = __builtin_amdgcn_readfirstlane(sf);
                            const uint64_t *ps = lat + sf;
                            nu = ps[s0 >= N - LL ? LL - N : LL];
                            nd = ps[s0 < LL ? N - LL : -LL];
                        } else {
                            // (s +- vst) mod N as the unsigned smaller of the two candidates
                            const uint32_t up = (uint32_t)sf + vst, dn = (uint32_t)sf - vst;
                            nu = lat[min(up, up - (uint32_t)N)];
                            nd = lat[min(dn, dn + (uint32_t)N)];
                        }
                        if (D == 2) {
                            n2 = nu;
                            n3 = nd;
                        } else {
                            n2 = lat[sf + oyp];
                            n3 = lat[sf + oym];
                            n4 = nu;
                            n5 = nd;
                        }
                    } else {
                        const int row = half > 1 ? (int)__umulhi((uint32_t)k, mhalf) : k; // row = y + L z
                        const int m = k - row * half;
                        const int z = (D == 2) ? 0 : (int)__umulhi((uint32_t)row, mL);
                        const int y = row - z * L;
                        const int x = 2 * m + ((y + z + c) & 1);
                        s = (uint32_t)(x + L * row);
                        n0 = lat[x == L - 1 ? s - (L - 1) : s + 1];
                        n1 = lat[x == 0 ? s + (L - 1) : s - 1];
                        n2 = lat[y == L - 1 ? s - L * (L - 1) : s + L];
                        n3 = lat[y == 0 ? s + L * (L - 1) : s - L];
                        if (D == 3) {
                            n4 = lat[z == L - 1 ? s - LL * (L - 1) : s + LL];
                            n5 = lat[z == 0 ? s + LL * (L - 1) : s - LL];
                        }
                    }
                    const uint32_t jb = J ? (uint32_t)jl[s] : 0u;
                    S = lat[s];
                    // a_k: bond k unsatisfied (S ^ neighbour ^ [J = -1])
                    const uint64_t a0 = bond<J>(S, n0, jb, 0), a1 = bond<J>(S, n1, jb, D);
                    const uint64_t a2 = bond<J>(S, n2, jb, 1), a3 = bond<J>(S, n3, jb, D + 1);
                    // u = number of unsatisfied bonds among 2d; dE = 4(d - u)
                    uint64_t m12;
                    if (D == 2) {
                        // pair sums s and carries c of (a0, a1) and (a2, a3); without
                        // couplings S cancels from the sums and each carry is one
                        // three-input operation on S and the neighbours
                        constexpr int kBoth = PA_T3((PA_A ^ PA_B) & (PA_A ^ PA_C));
                        const uint64_t s0 = J ? a0 ^ a1 : n0 ^ n1, s1 = J ? a2 ^ a3 : n2 ^ n3;
                        const uint64_t c0 = J ? a0 & a1 : pa_bop3<kBoth>(S, n0, n1);
                        const uint64_t c1 = J ? a2 & a3 : pa_bop3<kBoth>(S, n2, n3);
                        const uint64_t cc = c0 | c1;
                        always = pa_bop3<PA_T3(PA_A | (PA_B & PA_C))>(cc, s0, s1); // u >= 2
                        m4 = pa_bop3<PA_T3((PA_A ^ PA_B) & ~PA_C)>(s0, s1, cc);    // u == 1
                        m8 = pa_bop3<PA_T3(~(PA_A | PA_B | PA_C))>(s0, s1, cc);    // u == 0
                        m12 = 0;
                    } else {
                        const uint64_t a4 = bond<J>(S, n4, jb, 2), a5 = bond<J>(S, n5, jb, 5);
                        // three-bond sums and carries, then u = 2 (cA + cB + lc) + ls
                        const uint64_t sA = pa_bop3<kXor3>(a0, a1, a2), cA = pa_bop3<kMaj>(a0, a1, a2);
                        const uint64_t sB = pa_bop3<kXor3>(a3, a4, a5), cB = pa_bop3<kMaj>(a3, a4, a5);
                        const uint64_t ls = sA ^ sB, lc = sA & sB;
                        const uint64_t maj = pa_bop3<kMaj>(cA, cB, lc);  // cA + cB + lc >= 2
                        const uint64_t odd = pa_bop3<kXor3>(cA, cB, lc); // ... is odd
                        const uint64_t none = pa_bop3<PA_T3(~(PA_A | PA_B | PA_C))>(cA, cB, lc);
                        always = pa_bop3<PA_T3(PA_A | (PA_B & PA_C))>(maj, odd, ls); // u >= 3
                        m4 = pa_bop3<PA_T3(~PA_A & PA_B & ~PA_C)>(maj, odd, ls);     // u == 2
                        m8 = none & ls;                                               // u == 1
                        m12 = none & ~ls;                                             // u == 0
                    }
                    if (ALL) { // every class draws: the rest of the word (~always) is undecided
                        acc = always;
                    } else {
                        acc = always | (m4 & sure4) | (m8 & sure8) | (m12 & sure12);
                        und = (m4 & draw4) | (m8 & draw8) | (m12 & draw12);
                    }
                }
                // the first kInlinePairs plane pairs of the site: their Philox
                // calls in lockstep (independent chains), then the decisions;
                // the wave counts each pair's evaluations by a ballot
                const bool need = ALL ? always != ~0ull : und != 0;
                const uint64_t needing = __ballot(need);
                wcalls += (uint32_t)__popcll(needing);
                // branch for the wave, not the lane: a lane that needs no pair
                // has und = 0 (always = ~0) and its decisions change nothing,
                // and the pair counts below stay wave-uniform
                if (needing != 0ull) {
                    pa_philox_out o[kInlinePairs];
                    pa_philox_k<kInlinePairs>(pc.seed, pc.run_id, metro_share(pc, s), pc.w, pc.step,
                                              (PA_PURPOSE_METRO << 28) | (pc.t << 8), o);
                    // keep the calls together (the compiler would otherwise move
                    // each into the branch of its pair, one chain at a time)
#pragma unroll
                    for (int k = 0; k < kInlinePairs; ++k)
                        asm volatile("" : "+v"(o[k].x0), "+v"(o[k].x1), "+v"(o[k].x2), "+v"(o[k].x3));
                    const uint64_t l0 = ((uint64_t)tl[0] << 32) | tl[0], l1 = ((uint64_t)tl[1] << 32) | tl[1];
                    if (zp > 0) { // nothing accepts on these planes
                        const uint64_t P0 = (uint64_t)o[0].x0 | ((uint64_t)o[0].x1 << 32);
                        const uint64_t P1 = (uint64_t)o[0].x2 | ((uint64_t)o[0].x3 << 32);
                        und = ALL ? pa_bop3<PA_T3(~(PA_A | PA_B | PA_C))>(always, P0, P1)
                                  : pa_bop3<PA_T3(PA_A & ~(PA_B | PA_C))>(und, P0, P1);
                    } else if (ALL) {
                        apply_pair<D, true>(pc, o[0], 0u, m4, m8, l0, l1, always, und, acc);
                    } else {
                        apply_pair<D>(pc, o[0], 0u, m4, m8, l0, l1, und, und, acc);
                    }
                    // a decided lane's pairs change nothing (und = 0)
#pragma unroll
                    for (int k = 1; k < kInlinePairs; ++k) {
                        wcalls += (uint32_t)__popcll(__ballot(und != 0));
                        if (k < zp) {
                            const uint64_t P0 = (uint64_t)o[k].x0 | ((uint64_t)o[k].x1 << 32);
                            const uint64_t P1 = (uint64_t)o[k].x2 | ((uint64_t)o[k].x3 << 32);
                            und = pa_bop3<PA_T3(PA_A & ~(PA_B | PA_C))>(und, P0, P1);
                        } else {
                            apply_pair<D>(pc, o[k], (uint32_t)k, m4, m8, ((uint64_t)tl[2 * k] << 32) | tl[2 * k],
                                          ((uint64_t)tl[2 * k + 1] << 32) | tl[2 * k + 1], und, und, acc);
                        }
                    }
                }
                if (!RAGGED || k < nh)
                    lat[s] = S ^ acc;
                // an item still undecided has taken all inline pairs
                cnt = queue_push<D>(Q, head, cnt, und != 0, s | ((uint32_t)kInlinePairs << 16), und, m4, m8);
                while (cnt >= 64u)
                    queue_pass<D>(Q, pc, lat, head, cnt, wcalls);
            };
            int kb = 0;
            for (; kb + bs <= nh; kb += bs, sf += 2 * bs)
                pass(kb, std::false_type{});
            if (kb < nh)
                pass(kb, std::true_type{});
            queue_drain<D>(Q, pc, lat, head, cnt, calls);
            __syncthreads();
        }
    }

    return calls + ((threadIdx.x & 63) == 0 ? __builtin_amdgcn_readfirstlane(wcalls) : 0u);
}

// n elements from global memory into LDS.  A lane issues R loads before its
// first store, so that they are in flight together: rounds of 8, then of 4,
// while whole rounds remain, then rounds of 2 (lanes past the end load the
// last element again and store nothing).  No load is under a branch, which
// would make each one wait for the one before.
template <typename T, int R>
__device__ __forceinline__ int stage_rounds(T *dst, const __attribute__((address_space(1))) T *src, int n, int b0,
                                            bool whole)
{
    const int tid = threadIdx.x, bs = blockDim.x;
    for (; whole ? b0 + R * bs <= n : b0 < n; b0 += R * bs) {
        T v[R];
#pragma unroll
        for (int k = 0; k < R; ++k)
            v[k] = src[whole ? b0 + tid + k * bs : min(b0 + tid + k * bs, n - 1)];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = b0 + tid + k * bs;
            if (whole || i < n)
                dst[i] = v[k];
        }
    }
    return b0;
}

template <typename T>
__device__ __forceinline__ void stage_to_lds(T *dst, const __attribute__((address_space(1))) T *src, int n)
{
    int b0 = stage_rounds<T, 8>(dst, src, n, 0, true);
    b0 = stage_rounds<T, 4>(dst, src, n, b0, true);
    stage_rounds<T, 2>(dst, src, n, b0, false);
}

// A column's N words (16 bytes per load) and, with couplings, its N bond
// masks (4 bytes per load) into LDS.  N is a multiple of 4 (L even); g is
// 32-byte and jm 256-byte aligned.
template <bool J>
__device__ __forceinline__ void load_column(uint64_t *lat, uint8_t *jl, const uint64_t *g, const uint8_t *jm,
                                            int N)
{
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    stage_to_lds<u64x2>(reinterpret_cast<u64x2 *>(lat), (const __attribute__((address_space(1))) u64x2 *)g,
                        N >> 1);
    if (J)
        stage_to_lds<uint32_t>(reinterpret_cast<uint32_t *>(jl),
                               (const __attribute__((address_space(1))) uint32_t *)jm, N >> 2);
}

// Destination word column w takes the bits of its 64 ancestors.  Bit b comes
// from bit (a_b & 63) of source word a_b >> 6, i.e. from that word shifted by
// delta_b = (a_b & 63) - b.  Bits sharing (source word, delta) form one group:
// one shift, mask and or per group per site.  Ancestors are non-decreasing, so
// delta moves by one per dropped or repeated replica and a column has few
// groups (fewer than its runs of consecutive ancestors), listed in order of
// source word.  The group lists live in LDS.
struct GatherGroups {
    uint64_t *mask; // [64]
    uint32_t *word; // [64]
    int *shift;     // [64]
    int *n;         // [1]
};

// Wave 0 lists the groups of destination word w (replicas 64 w + b below R,
// ancestors anc); the caller synchronises the workgroup before they are read.
__device__ __forceinline__ void gather_groups(const uint32_t *anc, uint32_t w, int64_t R, const GatherGroups &G)
{
    if (threadIdx.x >= 64)
        return;
    const int b = threadIdx.x;
    const int64_t d = 64 * (int64_t)w + b;
    const bool valid = d < R;
    const uint32_t a = valid ? anc[d] : 0u;
    const uint32_t q = a >> 6;
    const int dl = (int)(a & 63u) - b;
    uint64_t rem = __ballot(valid);
    int ng = 0;
    while (rem) { // wave-uniform: one group per pass, led by the lowest remaining lane
        const int l = __ffsll((long long)rem) - 1;
        const uint32_t ql = (uint32_t)__shfl((int)q, l, 64);
        const int dll = __shfl(dl, l, 64);
        const uint64_t m = __ballot(valid && q == ql && dl == dll);
        if (b == 0) {
            G.word[ng] = ql;
            G.shift[ng] = dll;
            G.mask[ng] = m;
        }
        rem &= ~m;
        ++ng;
    }
    if (b == 0)
        *G.n = ng;
}

typedef uint64_t pa_u64x2 __attribute__((ext_vector_type(2)));

// Every thread: the destination word's sites from the source words (column
// sw at src + sw N), kP site pairs at a time with one 16-byte load each, in
// flight together (a lane past the end loads the last pair again and stores
// nothing: no load under a branch); store(p, v) keeps site pair p.
template <typename Store>
__device__ __forceinline__ void gather_sites(const uint64_t *src, int N, const GatherGroups &G, Store store)
{
    typedef const __attribute__((address_space(1))) pa_u64x2 g_u64x2;
    constexpr int kP = 4;
    const int ng = uni(*G.n);
    const int nt = (int)blockDim.x;
    const int np = N >> 1; // N is a multiple of 4 (L even)
    g_u64x2 *src2 = (g_u64x2 *)src;
    for (int p0 = threadIdx.x; p0 < np; p0 += kP * nt) {
        pa_u64x2 out[kP], v[kP];
#pragma unroll
        for (int k = 0; k < kP; ++k) {
            out[k] = pa_u64x2{0ull, 0ull};
            v[k] = out[k];
        }
        uint32_t last = 0xFFFFFFFFu;
        for (int i = 0; i < ng; ++i) {
            const uint32_t sw = uni(G.word[i]);
            if (sw != last) {
#pragma unroll
                for (int k = 0; k < kP; ++k)
                    v[k] = src2[(size_t)sw * np + min(p0 + k * nt, np - 1)];
                last = sw;
            }
            const int sh = uni(G.shift[i]);
            const uint64_t mask = uni64(G.mask[i]);
            if (sh >= 0) {
#pragma unroll
                for (int k = 0; k < kP; ++k) {
                    out[k].x = pa_bop3<PA_T3((PA_A & PA_B) | PA_C)>(v[k].x >> sh, mask, out[k].x);
                    out[k].y = pa_bop3<PA_T3((PA_A & PA_B) | PA_C)>(v[k].y >> sh, mask, out[k].y);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kP; ++k) {
                    out[k].x = pa_bop3<PA_T3((PA_A & PA_B) | PA_C)>(v[k].x << -sh, mask, out[k].x);
                    out[k].y = pa_bop3<PA_T3((PA_A & PA_B) | PA_C)>(v[k].y << -sh, mask, out[k].y);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kP; ++k) {
            const int p = p0 + k * nt;
            if (p < np)
                store(p, out[k]);
        }
    }
}

// One workgroup = one word column w (64 replicas) of one run; the lattice
// stays in LDS for all theta sweeps, then each replica's unsatisfied-bond
// count U and number of down spins are counted bit-sliced: E = 2U - dN,
// M = N - 2 n_down.  theta = 0 only measures.  J: the run has +-J couplings
// (per-site bond masks in LDS); without, every bond is ferromagnetic.
template <int D, bool J>
__global__ __launch_bounds__(kSweepMaxThreads) void k_sweep(const PaRunDesc *__restrict__ runs,
                                                            const PaBlk *__restrict__ map, int theta, uint32_t t0,
                                                            int gather)
{
    // dynamic LDS: lattice [N] u64 | queues [waves][3][kQueue] u64 | queue sites [waves][kQueue] u32 |
    // threshold-bit table [16][4 or 8] u32 | jmask [N]
    extern __shared__ uint64_t lat[];
    const PaBlk blk = map[blockIdx.x];
    const PaRunDesc &rd = runs[blk.run];
    PaRecord *rec = rd.dv.rec;
    const uint32_t w = blk.idx;
    const int64_t Rlive = (int64_t)rec->Rcur;
    if ((int64_t)w * 64 >= Rlive || frozen(rec))
        return;
    const int L = uni(rd.L), N = uni(rd.N);
    const int cur = uni(rec->cur);
    const uint32_t step = uni(rec->step);
    const int tid = threadIdx.x, bs = blockDim.x, nwaves = bs >> 6;
    uint64_t *qbase = lat + N + (size_t)(tid >> 6) * 3 * kQueue;
    uint32_t *qsites = reinterpret_cast<uint32_t *>(lat + N + (size_t)nwaves * 3 * kQueue);
    uint32_t *ttab = qsites + (size_t)nwaves * kQueue;
    uint8_t *jl = reinterpret_cast<uint8_t *>(ttab + ttab_words<D>());
    uint64_t *g = rd.dv.spins[cur] + (size_t)w * N;
    const uint64_t T4 = uni64(rec->T[0]), T8 = uni64(rec->T[1]), T12 = uni64(rec->T[2]);
    if (tid < 16) { // the threshold-bit masks of plane pair tid
        const uint32_t b0 = 31u - 2u * (uint32_t)tid;
        const uint32_t t[3] = {(uint32_t)T4, (uint32_t)T8, (uint32_t)T12};
#pragma unroll
        for (int c = 0; c < (D == 2 ? 2 : 3); ++c) {
            ttab[ttab_stride<D>() * tid + 2 * c] = (uint32_t)__builtin_amdgcn_sbfe((int)t[c], b0, 1u);
            ttab[ttab_stride<D>() * tid + 2 * c + 1] = (uint32_t)__builtin_amdgcn_sbfe((int)t[c], b0 - 1u, 1u);
        }
    }
    if (gather && uni(rec->gather) != 0u) {
        // the column of a resampled population, gathered from the other
        // buffer into LDS (the group lists in wave 0's queue space, unused
        // until the sweeps)
        uint64_t *gq = lat + N;
        uint32_t *gw = reinterpret_cast<uint32_t *>(gq + 64);
        const GatherGroups G = {gq, gw, reinterpret_cast<int *>(gw + 64), reinterpret_cast<int *>(gw + 128)};
        gather_groups(rd.dv.anc, w, Rlive, G);
        __syncthreads();
        pa_u64x2 *dst = reinterpret_cast<pa_u64x2 *>(lat);
        gather_sites(rd.dv.spins[cur ^ 1], N, G, [&](int p, pa_u64x2 v) { dst[p] = v; });
        if (J)
            stage_to_lds<uint32_t>(reinterpret_cast<uint32_t *>(jl),
                                   (const __attribute__((address_space(1))) uint32_t *)rd.dv.jmask, N >> 2);
    } else {
        load_column<J>(lat, jl, g, rd.dv.jmask, N);
    }
    __syncthreads();

    const uint64_t two32 = 1ull << 32;
    // classes whose threshold is 2^32 accept outright, those at 0 never accept
    const uint64_t sure4 = T4 >= two32 ? ~0ull : 0ull, sure8 = T8 >= two32 ? ~0ull : 0ull,
                   sure12 = T12 >= two32 ? ~0ull : 0ull;
    const uint64_t draw4 = (T4 > 0 && T4 < two32) ? ~0ull : 0ull,
                   draw8 = (T8 > 0 && T8 < two32) ? ~0ull : 0ull,
                   draw12 = (T12 > 0 && T12 < two32) ? ~0ull : 0ull;
    const int half = L >> 1, nh = N >> 1, LL = L * L;
    // floor(n / half) and floor(n / L) as one high multiply by ceil(2^32 / d):
    // exact for n d < 2^32, and here n < 2^14, d <= 2^13
    const uint32_t mhalf = half > 1 ? uni((uint32_t)(((1ull << 32) + (uint64_t)half - 1) / (uint64_t)half)) : 0u;
    const uint32_t mL = uni((uint32_t)(((1ull << 32) + (uint64_t)L - 1) / (uint64_t)L));
    PlaneCtx pc;
    pc.seed = uni(rd.seed);
    pc.run_id = uni(rd.run_id);
    pc.w = w;
    pc.step = step;
    pc.t4 = (uint32_t)T4;
    pc.t8 = (uint32_t)T8;
    pc.t12 = (uint32_t)T12;
    const WaveQueue Q = {qsites + (size_t)(tid >> 6) * kQueue, qbase, qbase + kQueue, qbase + 2 * kQueue, ttab};
    const SweepGeom G = {L, N, half, nh, LL, mhalf, mL};
    const bool all_draw = draw4 != 0 && draw8 != 0 && (D == 2 || draw12 != 0);
    const bool fix = bs % (D == 2 ? L : LL) == 0;
    // leading planes on which every drawing class's threshold bit is 0: the
    // leading zeros of their thresholds' or (each drawing threshold is < 2^32)
    const uint32_t tor = (uint32_t)((T4 & draw4) | (T8 & draw8) | (D == 3 ? (T12 & draw12) : 0ull));
    const int zp = uni(min(kInlinePairs, (tor ? (int)__builtin_clz(tor) : 32) / 2));
    // 3D fixed-axis walk with every wave inside one z plane per pass
    const bool zu = D == 3 && fix && (LL / 2) % 64 == 0;
    uint32_t calls;
    if (all_draw && zu)
        calls = sweep_columns<D, J, true, true, D == 3>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4,
                                                        draw8, draw12, zp);
    else if (all_draw && fix)
        calls = sweep_columns<D, J, true, true>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4, draw8,
                                                draw12, zp);
    else if (all_draw)
        calls = sweep_columns<D, J, true, false>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4, draw8,
                                                 draw12, zp);
    else if (zu)
        calls = sweep_columns<D, J, false, true, D == 3>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4,
                                                         draw8, draw12, zp);
    else if (fix)
        calls = sweep_columns<D, J, false, true>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4, draw8,
                                                 draw12, zp);
    else
        calls = sweep_columns<D, J, false, false>(lat, jl, G, pc, Q, theta, t0, sure4, sure8, sure12, draw4, draw8,
                                                  draw12, zp);

    // after the sweeps the queue region is free: per-wave partial counts of the measurement
    if (theta > 0) {
        const uint64_t tot = pa_wave_sum_u64(calls);
        if ((tid & 63) == 0)
            atomicAdd(&rec->philox_calls, (unsigned long long)tot);
        if (tid == 0)
            atomicAdd(&rec->site_updates, (unsigned long long)theta * (unsigned long long)N);
        if (tid == 0 && w == 0) { // once per run; no block reads these during the launch
            rec->sweeps = t0 + (uint32_t)theta;
            rec->attempts += (unsigned long long)theta * (unsigned long long)N * (unsigned long long)Rlive;
        }
    }
    recount_column<D, J>(lat, jl, g, lat + N, rd, cur, w, Rlive, L, N, LL, mL);
}

} // namespace

// Launches k_sweep<3, J> (defined in pa_sweep3.hip).
hipError_t pa_sweep3_launch(const PaRunDesc *runs, const PaBlk *map, int nblocks, int threads, size_t lds,
                            hipStream_t st, bool J, int theta, uint32_t t0, int gather);
