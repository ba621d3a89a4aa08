// The learned temperature-step model on gfx950: an 8 -> 64 -> 64 -> 1 tanh
// network that proposes ln(dbeta) from population statistics.  Training in
// float32 (forward/backward per sample, then one thread per parameter summing
// its gradient over the samples in a fixed order, then Adam), inference in
// bfloat16 (weights and layer inputs rounded to bfloat16, float32 sums).
// Parameter vector: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
#include "pa_device.h"
#include "pa_internal.h"

namespace {

constexpr int kH = PA_MLP_HIDDEN;
constexpr int oW1 = 0, ob1 = oW1 + kH * 8, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
static_assert(ob3 + 1 == PA_MLP_PARAMS, "parameter layout");

// float32 -> nearest bfloat16 (ties to even), kept in a float
__device__ __forceinline__ float bf16r(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// One thread per sample: forward pass and the backward pass down to the
// pre-activations; activations and their error signals go to global memory
// for the per-parameter gradient sums.
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const float *__restrict__ P, const PaMlpNorm *__restrict__ nm,
                                                    const float *__restrict__ X, const float *__restrict__ Y, int n,
                                                    float *__restrict__ Xn, float *__restrict__ H1,
                                                    float *__restrict__ H2, float *__restrict__ D1,
                                                    float *__restrict__ D2, float *__restrict__ dY,
                                                    float *__restrict__ r2)
{
    __shared__ float sp[PA_MLP_PARAMS];
    for (int k = threadIdx.x; k < PA_MLP_PARAMS; k += blockDim.x)
        sp[k] = P[k];
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float x[8];
    for (int k = 0; k < 8; ++k) {
        x[k] = (X[i * 8 + k] - nm->x_mean[k]) / nm->x_std[k];
        Xn[i * 8 + k] = x[k];
    }
    const float yn = (Y[i] - nm->y_mean) / nm->y_std;
    float *h1 = H1 + (size_t)i * kH, *h2 = H2 + (size_t)i * kH;
    for (int a = 0; a < kH; ++a) {
        float z = sp[ob1 + a];
        for (int k = 0; k < 8; ++k)
            z += sp[oW1 + a * 8 + k] * x[k];
        h1[a] = tanhf(z);
    }
    float yh = sp[ob3];
    for (int a = 0; a < kH; ++a) {
        float z = sp[ob2 + a];
        for (int b = 0; b < kH; ++b)
            z += sp[oW2 + a * kH + b] * h1[b];
        const float h = tanhf(z);
        h2[a] = h;
        yh += sp[oW3 + a] * h;
    }
    const float res = yh - yn;
    const float dy = res / (float)n;
    dY[i] = dy;
    r2[i] = res * res;
    float *d2 = D2 + (size_t)i * kH, *d1 = D1 + (size_t)i * kH;
    for (int a = 0; a < kH; ++a)
        d2[a] = dy * sp[oW3 + a] * (1.0f - h2[a] * h2[a]);
    for (int b = 0; b < kH; ++b) {
        float s = 0.0f;
        for (int a = 0; a < kH; ++a)
            s += d2[a] * sp[oW2 + a * kH + b];
        d1[b] = s * (1.0f - h1[b] * h1[b]);
    }
}

// One thread per parameter: its gradient as a sum over the samples in order;
// then (adam != 0) one Adam step, t counting from 1.
__global__ __launch_bounds__(256) void k_mlp_update(float *__restrict__ P, float *__restrict__ Mm,
                                                    float *__restrict__ Vv, float *__restrict__ G,
                                                    const float *__restrict__ Xn, const float *__restrict__ H1,
                                                    const float *__restrict__ H2, const float *__restrict__ D1,
                                                    const float *__restrict__ D2, const float *__restrict__ dY, int n,
                                                    int adam, int t, float lr)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= PA_MLP_PARAMS)
        return;
    float g = 0.0f;
    if (p < ob1) {
        const int a = (p - oW1) / 8, k = (p - oW1) % 8;
        for (int i = 0; i < n; ++i)
            g += D1[(size_t)i * kH + a] * Xn[i * 8 + k];
    } else if (p < oW2) {
        const int a = p - ob1;
        for (int i = 0; i < n; ++i)
            g += D1[(size_t)i * kH + a];
    } else if (p < ob2) {
        const int a = (p - oW2) / kH, b = (p - oW2) % kH;
        for (int i = 0; i < n; ++i)
            g += D2[(size_t)i * kH + a] * H1[(size_t)i * kH + b];
    } else if (p < oW3) {
        const int a = p - ob2;
        for (int i = 0; i < n; ++i)
            g += D2[(size_t)i * kH + a];
    } else if (p < ob3) {
        const int a = p - oW3;
        for (int i = 0; i < n; ++i)
            g += dY[i] * H2[(size_t)i * kH + a];
    } else {
        for (int i = 0; i < n; ++i)
            g += dY[i];
    }
    G[p] = g;
    if (adam) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float m = b1 * Mm[p] + (1.0f - b1) * g;
        const float v = b2 * Vv[p] + (1.0f - b2) * g * g;
        Mm[p] = m;
        Vv[p] = v;
        const float mh = m / (1.0f - powf(b1, (float)t));
        const float vh = v / (1.0f - powf(b2, (float)t));
        P[p] = P[p] - lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void k_mlp_loss(const float *__restrict__ r2, int n, double *loss)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i)
            s += (double)r2[i];
        *loss = 0.5 * s / (double)n;
    }
}

// bfloat16 inference of one feature vector by one wave: lane a owns hidden
// unit a of both layers; the output sum runs over a in order on lane 0.
__device__ float mlp_infer_wave(const float *__restrict__ P, const PaMlpNorm *__restrict__ nm, const float *f,
                                float *h1s, float *h2s)
{
    const int a = threadIdx.x & 63;
    float x[8];
    for (int k = 0; k < 8; ++k)
        x[k] = bf16r((f[k] - nm->x_mean[k]) / nm->x_std[k]);
    float z = bf16r(P[ob1 + a]);
    for (int k = 0; k < 8; ++k)
        z += bf16r(P[oW1 + a * 8 + k]) * x[k];
    h1s[a] = bf16r(tanhf(z));
    __syncthreads();
    z = bf16r(P[ob2 + a]);
    for (int b = 0; b < kH; ++b)
        z += bf16r(P[oW2 + a * kH + b]) * h1s[b];
    h2s[a] = bf16r(tanhf(z));
    __syncthreads();
    float y = bf16r(P[ob3]);
    for (int b = 0; b < kH; ++b)
        y += bf16r(P[oW3 + b]) * h2s[b];
    return y;
}

__device__ __forceinline__ double to_dbeta(float yhat, const PaMlpNorm *nm) { return exp((double)yhat * nm->y_std + nm->y_mean); }

// Standalone inference: one 64-lane workgroup per feature vector.
__global__ __launch_bounds__(64) void k_mlp_predict(const float *__restrict__ P, const PaMlpNorm *__restrict__ nm,
                                                   const float *__restrict__ X, int n, float *__restrict__ out)
{
    __shared__ float h1s[kH], h2s[kH];
    const int i = blockIdx.x;
    if (i >= n)
        return;
    const float y = mlp_infer_wave(P, nm, X + (size_t)i * 8, h1s, h2s);
    if (threadIdx.x == 0)
        out[i] = (float)to_dbeta(y, nm);
}

// Inference for every run of a batch from the features in its record; the
// proposal is clamped to (0, dbeta_max] and stored for the exact check.
__global__ __launch_bounds__(64) void k_mlp_propose(const PaRunDesc *__restrict__ runs, const float *__restrict__ P,
                                                   const PaMlpNorm *__restrict__ nm, double dbeta_max)
{
    __shared__ float h1s[kH], h2s[kH];
    PaRecord *rec = runs[blockIdx.x].dv.rec;
    if (rec->status & PA_ST_FROZEN)
        return;
    float f[8];
    for (int k = 0; k < 8; ++k)
        f[k] = rec->feat[k];
    const float y = mlp_infer_wave(P, nm, f, h1s, h2s);
    if (threadIdx.x == 0) {
        double d = to_dbeta(y, nm);
        if (!(d > 0.0))
            d = 0.0;
        rec->cand_dbeta = d < dbeta_max ? d : dbeta_max;
    }
}

} // namespace

hipError_t pa_mlp_launch_grad(const PaMlpDev &m, int n, int adam, int t, float lr)
{
    const int blocks = (n + 255) / 256;
    k_mlp_fwdbwd<<<blocks, 256, 0, m.stream>>>(m.P, m.norm, m.X, m.Y, n, m.Xn, m.H1, m.H2, m.D1, m.D2, m.dY, m.r2);
    k_mlp_update<<<(PA_MLP_PARAMS + 255) / 256, 256, 0, m.stream>>>(m.P, m.M, m.V, m.G, m.Xn, m.H1, m.H2, m.D1,
                                                                    m.D2, m.dY, n, adam, t, lr);
    k_mlp_loss<<<1, 64, 0, m.stream>>>(m.r2, n, m.loss);
    return hipGetLastError();
}

hipError_t pa_mlp_launch_predict(const PaMlpDev &m, const float *X, int n, float *out)
{
    k_mlp_predict<<<n, 64, 0, m.stream>>>(m.P, m.norm, X, n, out);
    return hipGetLastError();
}

hipError_t pa_mlp_launch_propose(const PaBatchView &v, const PaMlpDev &m, double dbeta_max)
{
    k_mlp_propose<<<v.nruns, 64, 0, v.stream>>>(v.runs, m.P, m.norm, dbeta_max);
    return hipGetLastError();
}
