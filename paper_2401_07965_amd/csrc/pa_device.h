// Device-side building blocks of the population-annealing library (gfx950).
//
// * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), the counter-based
//   generator every random decision of the method draws from.
// * pa_exp: the exponential used wherever exp() decides something (Metropolis
//   thresholds, resampling weights, Poisson probabilities): Cody-Waite
//   reduction by ln 2 and a degree-13 Taylor polynomial in Horner form, every
//   double operation rounded on its own (the library is built with
//   -ffp-contract=off), so its bits are fixed by IEEE-754 alone.
// * 128-bit helpers for the exact integer resampling arithmetic and the
//   fixed-order wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 pa_u128;

// Counter purpose codes, held in bits 31..28 of counter word 3.
#define PA_PURPOSE_INIT 1u
#define PA_PURPOSE_METRO 2u
#define PA_PURPOSE_RS_NI 4u
#define PA_PURPOSE_RS_POIS 5u
#define PA_PURPOSE_RS_MULT 6u
#define PA_PURPOSE_RS_SYS 7u
#define PA_PURPOSE_WSEED 8u
#define PA_PURPOSE_WBOND 9u

struct pa_philox_out {
    uint32_t x0, x1, x2, x3;
};

// gfx950 three-input bitwise operation (v_bitop3_b32): bit i of the result is
// bit (a_i b_i c_i) (a the most significant) of the 8-bit table.  A table is
// written as the wanted function applied to the columns a = 0xF0, b = 0xCC,
// c = 0xAA, e.g. PA_T3(PA_A ^ PA_B ^ PA_C) for a three-way xor.
#define PA_A 0xF0
#define PA_B 0xCC
#define PA_C 0xAA
#define PA_T3(f) ((f) & 0xFF)

template <int TT>
__device__ __forceinline__ uint32_t pa_bop3(uint32_t a, uint32_t b, uint32_t c)
{
    return (uint32_t)__builtin_amdgcn_bitop3_b32((int)a, (int)b, (int)c, TT);
}

template <int TT>
__device__ __forceinline__ uint64_t pa_bop3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = pa_bop3<TT>((uint32_t)a, (uint32_t)b, (uint32_t)c);
    const uint32_t hi = pa_bop3<TT>((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Philox4x32-10: ten rounds of (x0,x1,x2,x3) -> (hi(B x2) ^ x1 ^ k0, lo(B x2),
// hi(A x0) ^ x3 ^ k1, lo(A x0)) with A = 0xD2511F53, B = 0xCD9E8D57 and the key
// advanced by (0x9E3779B9, 0xBB67AE85) between rounds.  The callers vary x0
// per lane and keep x1..x3 and the key common to a wavefront, so the first
// rounds keep plain xors that let common words meet in scalar registers
// (round 2's x3 is lo(A x0) of a common x0); from the third round on every
// word varies per lane and each output takes one three-way xor.
// Calls that differ in x3 alone share two products: the first round's
// A x0 (a0), and the third round's B x2, whose x2 = hi(A y0) ^ lo(A x0) ^ k1'
// (y0 = hi(B x2) ^ x1 ^ k0 of the first round, k1' the second round's key)
// does not involve x3 (b2).
struct pa_philox_shared {
    uint64_t a0, b2;
};

__device__ __forceinline__ pa_philox_shared pa_philox_share(uint32_t k0, uint32_t k1, uint32_t x0, uint32_t x1,
                                                            uint32_t x2)
{
    const uint64_t a0 = (uint64_t)0xD2511F53u * x0;
    const uint32_t y0 = (uint32_t)(((uint64_t)0xCD9E8D57u * x2) >> 32) ^ x1 ^ k0;
    const uint32_t x2r2 = (uint32_t)(((uint64_t)0xD2511F53u * y0) >> 32) ^ (uint32_t)a0 ^ (k1 + 0xBB67AE85u);
    return {a0, (uint64_t)0xCD9E8D57u * x2r2};
}

__device__ __forceinline__ pa_philox_out pa_philox_with(uint32_t k0, uint32_t k1, const pa_philox_shared &sh,
                                                        uint32_t x1, uint32_t x2, uint32_t x3)
{
    uint32_t x0 = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = round == 0 ? sh.a0 : (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = round == 2 ? sh.b2 : (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0, y2;
        if (round < 2) {
            y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
            y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        } else if (round == 2) {
            y0 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p1 >> 32), x1, k0);
            y2 = (uint32_t)(p0 >> 32) ^ (x3 ^ k1);
        } else {
            y0 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p1 >> 32), x1, k0);
            y2 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p0 >> 32), x3, k1);
        }
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {x0, x1, x2, x3};
}

// K calls that differ in x3 alone, x3 = x3b | k for k < K, their rounds
// taken in lockstep so that the K independent chains interleave.
template <int K>
__device__ __forceinline__ void pa_philox_k(uint32_t k0, uint32_t k1, const pa_philox_shared &sh, uint32_t x1in,
                                            uint32_t x2in, uint32_t x3b, pa_philox_out out[K])
{
    uint32_t x0[K], x1[K], x2[K], x3[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        x0[k] = 0;
        x1[k] = x1in;
        x2[k] = x2in;
        x3[k] = x3b | (uint32_t)k;
    }
#pragma unroll
    for (int round = 0; round < 10; ++round) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t p0 = round == 0 ? sh.a0 : (uint64_t)0xD2511F53u * x0[k];
            const uint64_t p1 = round == 2 ? sh.b2 : (uint64_t)0xCD9E8D57u * x2[k];
            uint32_t y0, y2;
            if (round < 2) {
                y0 = (uint32_t)(p1 >> 32) ^ x1[k] ^ k0;
                y2 = (uint32_t)(p0 >> 32) ^ x3[k] ^ k1;
            } else if (round == 2) {
                y0 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p1 >> 32), x1[k], k0);
                y2 = (uint32_t)(p0 >> 32) ^ (x3[k] ^ k1);
            } else {
                y0 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p1 >> 32), x1[k], k0);
                y2 = pa_bop3<PA_T3(PA_A ^ PA_B ^ PA_C)>((uint32_t)(p0 >> 32), x3[k], k1);
            }
            x1[k] = (uint32_t)p1;
            x3[k] = (uint32_t)p0;
            x0[k] = y0;
            x2[k] = y2;
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        out[k] = {x0[k], x1[k], x2[k], x3[k]};
}

__device__ __forceinline__ pa_philox_out pa_philox(uint32_t k0, uint32_t k1, uint32_t x0, uint32_t x1,
                                                   uint32_t x2, uint32_t x3)
{
    return pa_philox_with(k0, k1, pa_philox_share(k0, k1, x0, x1, x2), x1, x2, x3);
}

// 1/n! rounded to nearest, n = 0..13 (n! is exact in double).
__device__ __forceinline__ double pa_inv_fact(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k)
        f *= (double)k;
    return 1.0 / f;
}

// exp(x) for x in [-700, 0]; 0 below -700 and for NaN.
__device__ __forceinline__ double pa_exp(double x)
{
    if (!(x >= -700.0))
        return 0.0;
    const double inv_ln2 = 0x1.71547652b82fep+0; // 1/ln 2, nearest double
    const double ln2_hi = 0x1.62e42fee00000p-1;  // ln 2 cut to 32 significant bits
    const double ln2_lo = 0x1.a39ef35793c76p-33; // ln 2 - ln2_hi, nearest double
    const double k = rint(x * inv_ln2);
    const double r = (x - k * ln2_hi) - k * ln2_lo;
    constexpr double c2 = 1.0 / 2.0, c3 = 1.0 / 6.0, c4 = 1.0 / 24.0, c5 = 1.0 / 120.0,
                     c6 = 1.0 / 720.0, c7 = 1.0 / 5040.0, c8 = 1.0 / 40320.0,
                     c9 = 1.0 / 362880.0, c10 = 1.0 / 3628800.0, c11 = 1.0 / 39916800.0,
                     c12 = 1.0 / 479001600.0, c13 = 1.0 / 6227020800.0;
    double p = c13;
    p = p * r + c12;
    p = p * r + c11;
    p = p * r + c10;
    p = p * r + c9;
    p = p * r + c8;
    p = p * r + c7;
    p = p * r + c6;
    p = p * r + c5;
    p = p * r + c4;
    p = p * r + c3;
    p = p * r + c2;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

// Metropolis threshold T(dE) = min(2^32, floor(2^32 pa_exp(-beta dE))): a move
// that raises the energy by dE is taken iff the replica's 32-bit uniform u < T.
__device__ __forceinline__ uint64_t pa_threshold(double beta, int dE)
{
    const double p = pa_exp(-(beta * (double)dE));
    uint64_t T = (uint64_t)floor(ldexp(p, 32));
    return T > (1ull << 32) ? (1ull << 32) : T;
}

// Integer resampling weight of an energy gap g = E - E_min >= 0:
// floor(2^40 pa_exp(-dbeta g)), at most 2^40.
__device__ __forceinline__ uint64_t pa_weight(double dbeta, int32_t gap)
{
    return (uint64_t)floor(ldexp(pa_exp(-(dbeta * (double)gap)), 40));
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ uint64_t pa_shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double pa_shfl_xor_f64(double v, int m)
{
    return __longlong_as_double((long long)pa_shfl_xor_u64((uint64_t)__double_as_longlong(v), m));
}

// Butterfly sum over the 64 lanes of a wavefront: the same pairing in every
// call, so a double result is the same bits on every run.
__device__ __forceinline__ double pa_wave_sum_f64(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v = v + pa_shfl_xor_f64(v, m);
    return v;
}

__device__ __forceinline__ uint64_t pa_wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += pa_shfl_xor_u64(v, m);
    return v;
}

__device__ __forceinline__ int64_t pa_wave_min_i64(int64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const int64_t o = (int64_t)pa_shfl_xor_u64((uint64_t)v, m);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int64_t pa_wave_max_i64(int64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const int64_t o = (int64_t)pa_shfl_xor_u64((uint64_t)v, m);
        v = o > v ? o : v;
    }
    return v;
}

// Block-wide fixed-order double sum (blockDim.x a multiple of 64, <= 1024):
// wave butterflies, then the wave totals in wave order.  Every thread gets it.
__device__ __forceinline__ double pa_block_sum_f64(double v, double *lds /* >= 16 */)
{
    v = pa_wave_sum_f64(v);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nwaves; ++k)
        t = t + lds[k];
    __syncthreads();
    return t;
}

__device__ __forceinline__ uint64_t pa_block_sum_u64(uint64_t v, uint64_t *lds /* >= 16 */)
{
    v = pa_wave_sum_u64(v);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        lds[wave] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int k = 0; k < nwaves; ++k)
        t += lds[k];
    __syncthreads();
    return t;
}

// K block-wide double sums with one exchange through LDS, each in the fixed
// order of pa_block_sum_f64 (wave tree, then the waves in order).
template <int K>
__device__ __forceinline__ void pa_block_sum_f64x(double (&v)[K], double *lds /* >= 16 K */)
{
#pragma unroll
    for (int i = 0; i < K; ++i)
        v[i] = pa_wave_sum_f64(v[i]);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < K; ++i)
            lds[wave * K + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double t = 0.0;
        for (int k = 0; k < nwaves; ++k)
            t = t + lds[k * K + i];
        v[i] = t;
    }
    __syncthreads();
}

// K block-wide uint64 sums with one exchange through LDS (exact, so any order).
template <int K>
__device__ __forceinline__ void pa_block_sum_u64x(uint64_t (&v)[K], uint64_t *lds /* >= 16 K */)
{
#pragma unroll
    for (int i = 0; i < K; ++i)
        v[i] = pa_wave_sum_u64(v[i]);
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < K; ++i)
            lds[wave * K + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint64_t t = 0;
        for (int k = 0; k < nwaves; ++k)
            t += lds[k * K + i];
        v[i] = t;
    }
    __syncthreads();
}
