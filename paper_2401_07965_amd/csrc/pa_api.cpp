// Host side of the C ABI declared in include/pa.h: argument checks, the
// per-run state machine (init -> [reweight -> resample] -> sweep ...), the
// layout of the caller's device workspace, and the few small device-to-host
// copies each step needs (ln Q, the new population size, averages).
#include "pa.h"
#include "pa_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

struct pa_ctx {
    PaLaunch lp;
    PaDev dv;
    int cur = 0;         // which ping-pong buffer holds the population
    int64_t Rcur = 0;    // replicas in the population
    double beta = 0.0;   // current inverse temperature
    uint32_t step = 0;   // temperature index i
    uint32_t sweeps = 0; // sweeps done at step i
    uint64_t sweeps_total = 0;
    bool reweighted = false;
    double beta_next = 0.0;
    PaRecord *hrec = nullptr; // pinned host copy of the device record
    std::string err;
};

namespace {

thread_local std::string g_init_err;
bool g_kernels_configured = false;
int g_max_lds = 0;

constexpr int64_t kMaxCapacity = (1ll << 24) - 64; // R W_j < 2^64 for W_j <= 2^40
constexpr int kMaxSites = 16384;                  // LDS and 8-plane counters per thread

pa_status fail(pa_ctx *c, pa_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_init_err = msg;
    return s;
}

pa_status hip_fail(pa_ctx *c, hipError_t e, const char *where)
{
    return fail(c, PA_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

int64_t default_capacity(int64_t R)
{
    int64_t cs = (int64_t)std::sqrt((double)R);
    while (cs * cs < R)
        ++cs;
    while (cs > 0 && (cs - 1) * (cs - 1) >= R)
        --cs;
    const int64_t c = R + 8 * cs + 64;
    return (c + 63) / 64 * 64;
}

struct Geometry {
    int d, L, N, H;
    int64_t R, cap, W;
};

pa_status check_config(const pa_config *cfg, Geometry *g, std::string *msg)
{
    if (!cfg) {
        *msg = "config is NULL";
        return PA_E_INVAL;
    }
    if (cfg->dim != 2 && cfg->dim != 3) {
        *msg = "dim must be 2 or 3";
        return PA_E_INVAL;
    }
    if (cfg->L < 2 || (cfg->L & 1)) {
        *msg = "L must be even and >= 2 (checkerboard sweeps)";
        return PA_E_INVAL;
    }
    int64_t N = 1;
    for (int k = 0; k < cfg->dim; ++k)
        N *= cfg->L;
    if (N > kMaxSites) {
        *msg = "L^dim must not exceed 16384";
        return PA_E_INVAL;
    }
    if (cfg->R < 1) {
        *msg = "R must be >= 1";
        return PA_E_INVAL;
    }
    const int64_t cap = cfg->capacity ? cfg->capacity : default_capacity(cfg->R);
    if (cap < cfg->R || cap > kMaxCapacity) {
        *msg = "capacity must satisfy R <= capacity < 2^24 - 64";
        return PA_E_INVAL;
    }
    g->d = cfg->dim;
    g->L = cfg->L;
    g->N = (int)N;
    g->H = cfg->dim * (int)N / 2 + 1;
    g->R = cfg->R;
    g->cap = cap;
    g->W = (cap + 63) / 64;
    return PA_OK;
}

// Carves the workspace (base may be null to only measure it).
uint64_t carve(const Geometry &g, char *base, PaDev *dv)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    const uint64_t words = (uint64_t)g.W * g.N;
    const uint64_t slots = (uint64_t)g.W * 64;
    PaDev d{};
    for (int k = 0; k < 2; ++k) {
        d.spins[k] = (uint64_t *)take(words * 8);
        d.E[k] = (int32_t *)take(slots * 4);
        d.M[k] = (int32_t *)take(slots * 4);
        d.label[k] = (uint32_t *)take(slots * 4);
    }
    d.jmask = (uint8_t *)take((uint64_t)g.N);
    d.hist = (uint32_t *)take((uint64_t)g.H * 4);
    d.wtab = (uint64_t *)take((uint64_t)g.H * 8);
    d.r = (uint32_t *)take(slots * 4);
    d.P = (uint32_t *)take(slots * 4);
    d.anc = (uint32_t *)take(slots * 4);
    d.C = (uint64_t *)take(slots * 8);
    d.qhist = (unsigned long long *)take((uint64_t)(g.N + 1) * 8);
    d.tiles = (PaScanTile *)take((uint64_t)((slots + PA_SCAN_TILE - 1) / PA_SCAN_TILE) * sizeof(PaScanTile));
    d.ticket = (uint32_t *)take(4);
    d.fam = (uint32_t *)take((uint64_t)g.R * 4);
    d.partial = (double *)take(PA_RED_BLOCKS * 8);
    d.rec = (PaRecord *)take(sizeof(PaRecord));
    if (dv)
        *dv = d;
    return off;
}

pa_status fetch_record(pa_ctx *c, const char *where)
{
    hipError_t e = hipMemcpyAsync(c->hrec, c->dv.rec, sizeof(PaRecord), hipMemcpyDeviceToHost, c->lp.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c->lp.stream);
    if (e != hipSuccess)
        return hip_fail(c, e, where);
    return PA_OK;
}

} // namespace

extern "C" {

pa_status pa_required_bytes(const pa_config *cfg, uint64_t *bytes)
{
    Geometry g;
    std::string msg;
    pa_status s = check_config(cfg, &g, &msg);
    if (s != PA_OK)
        return fail(nullptr, s, msg);
    if (!bytes)
        return fail(nullptr, PA_E_INVAL, "bytes is NULL");
    *bytes = carve(g, nullptr, nullptr);
    return PA_OK;
}

pa_status pa_init(const pa_config *cfg, void *workspace, uint64_t workspace_bytes, void *stream, pa_ctx **out)
{
    if (!out)
        return fail(nullptr, PA_E_INVAL, "out is NULL");
    *out = nullptr;
    Geometry g;
    std::string msg;
    pa_status s = check_config(cfg, &g, &msg);
    if (s != PA_OK)
        return fail(nullptr, s, msg);
    const uint64_t need = carve(g, nullptr, nullptr);
    if (!workspace || workspace_bytes < need)
        return fail(nullptr, PA_E_INVAL, "workspace missing or smaller than pa_required_bytes");
    if (((uintptr_t)workspace & 255u) != 0)
        return fail(nullptr, PA_E_INVAL, "workspace must be 256-byte aligned");

    // couplings -> per-site masks of the 2d incident bonds
    std::vector<uint8_t> jm((size_t)g.N, 0);
    if (cfg->couplings) {
        for (int64_t s0 = 0; s0 < g.N; ++s0) {
            int64_t stride = 1;
            for (int mu = 0; mu < g.d; ++mu) {
                const int8_t J = cfg->couplings[s0 * g.d + mu];
                if (J != 1 && J != -1)
                    return fail(nullptr, PA_E_INVAL, "couplings must be +1 or -1");
                if (J == -1) {
                    const int64_t x = (s0 / stride) % g.L;
                    const int64_t s1 = s0 + ((x + 1) % g.L - x) * stride;
                    jm[(size_t)s0] |= (uint8_t)(1u << mu);
                    jm[(size_t)s1] |= (uint8_t)(1u << (g.d + mu));
                }
                stride *= g.L;
            }
        }
    }

    pa_ctx *c = new (std::nothrow) pa_ctx;
    if (!c)
        return fail(nullptr, PA_E_NOMEM, "out of host memory");
    hipError_t e;
    if (!g_kernels_configured) {
        if ((e = pa_configure_kernels(&g_max_lds)) != hipSuccess) {
            delete c;
            return hip_fail(nullptr, e, "kernel attributes");
        }
        g_kernels_configured = true;
    }
    if (pa_sweep_lds_bytes(g.N) > (size_t)g_max_lds || (size_t)g.H * 4 > (size_t)g_max_lds) {
        delete c;
        return fail(nullptr, PA_E_INVAL, "lattice too large for the workgroup LDS of this device");
    }
    if ((e = hipHostMalloc((void **)&c->hrec, sizeof(PaRecord), hipHostMallocDefault)) != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "pinned record");
    }
    carve(g, (char *)workspace, &c->dv);
    c->lp.d = g.d;
    c->lp.L = g.L;
    c->lp.N = g.N;
    c->lp.H = g.H;
    c->lp.seed = cfg->seed;
    c->lp.run_id = cfg->run_id;
    c->lp.R0 = g.R;
    c->lp.cap = g.cap;
    c->lp.stream = (hipStream_t)stream;
    c->Rcur = g.R;

    std::memset(c->hrec, 0, sizeof(PaRecord));
    c->hrec->lnZ = (double)g.N * std::log(2.0); // Z_0 = 2^N at beta_0 = 0
    for (int k = 0; k < 3; ++k)
        c->hrec->T[k] = c->hrec->Tn[k] = 1ull << 32; // beta = 0 accepts every move
    e = hipMemcpyAsync(c->dv.rec, c->hrec, sizeof(PaRecord), hipMemcpyHostToDevice, c->lp.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->dv.jmask, jm.data(), jm.size(), hipMemcpyHostToDevice, c->lp.stream);
    if (e == hipSuccess)
        e = pa_launch_init(c->lp, c->dv, 0);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c->lp.stream);
    if (e != hipSuccess) {
        hip_fail(nullptr, e, "pa_init");
        (void)hipHostFree(c->hrec);
        delete c;
        return PA_E_DEVICE;
    }
    *out = c;
    return PA_OK;
}

pa_status pa_sweep(pa_ctx *c, int32_t theta)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (theta < 0)
        return fail(c, PA_E_INVAL, "theta must be >= 0");
    if ((uint64_t)c->sweeps + (uint64_t)theta > (1u << 20))
        return fail(c, PA_E_INVAL, "more than 2^20 sweeps at one temperature");
    if (theta == 0)
        return PA_OK;
    hipError_t e = pa_launch_sweep(c->lp, c->dv, c->cur, c->Rcur, c->step, c->sweeps, theta);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_sweep");
    c->sweeps += (uint32_t)theta;
    c->sweeps_total += (uint64_t)theta;
    return PA_OK;
}

pa_status pa_reweight(pa_ctx *c, double beta_next, double *lnQ_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!std::isfinite(beta_next) || beta_next < c->beta)
        return fail(c, PA_E_INVAL, "beta_next must be finite and >= the current beta");
    const double dbeta = beta_next - c->beta;
    hipError_t e = pa_launch_reweight(c->lp, c->dv, c->cur, c->Rcur, dbeta, beta_next);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_reweight");
    pa_status s = fetch_record(c, "pa_reweight");
    if (s != PA_OK)
        return s;
    if (!std::isfinite(c->hrec->lnQ)) {
        c->reweighted = false;
        return fail(c, PA_E_NONFINITE, "ln Q is not finite");
    }
    c->reweighted = true;
    c->beta_next = beta_next;
    if (lnQ_out)
        *lnQ_out = c->hrec->lnQ;
    return PA_OK;
}

pa_status pa_resample(pa_ctx *c, pa_resampler scheme, int64_t *R_new_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if ((int)scheme < 0 || (int)scheme > 3)
        return fail(c, PA_E_INVAL, "unknown resampling scheme");
    if (!c->reweighted)
        return fail(c, PA_E_STATE, "pa_resample needs a pa_reweight first");
    const int64_t Rprev = c->Rcur, Rt = c->lp.R0;
    const uint32_t step = c->step + 1;
    hipError_t e = pa_launch_counts(c->lp, c->dv, c->cur, Rprev, Rt, (int)scheme, step);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_resample counts");
    pa_status s = fetch_record(c, "pa_resample");
    if (s != PA_OK)
        return s;
    if (c->hrec->err)
        return fail(c, PA_E_DEVICE, "prefix-sum look-back timed out");
    const int64_t Rnew = (int64_t)c->hrec->Rnew;
    if (Rnew > c->lp.cap)
        return fail(c, PA_E_CAPACITY, "resampled population exceeds the capacity");
    if (Rnew == 0)
        return fail(c, PA_E_EXTINCT, "resampled population is empty");
    e = pa_launch_apply(c->lp, c->dv, c->cur, Rprev, Rnew);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_resample apply");
    c->cur ^= 1;
    c->Rcur = Rnew;
    c->beta = c->beta_next;
    c->step = step;
    c->sweeps = 0;
    c->reweighted = false;
    if (R_new_out)
        *R_new_out = Rnew;
    return PA_OK;
}

pa_status pa_observables(pa_ctx *c, pa_obs *out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!out)
        return fail(c, PA_E_INVAL, "out is NULL");
    hipError_t e = pa_launch_observables(c->lp, c->dv, c->cur, c->Rcur);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_observables");
    pa_status s = fetch_record(c, "pa_observables");
    if (s != PA_OK)
        return s;
    const PaRecord &r = *c->hrec;
    out->R = c->Rcur;
    out->beta = c->beta;
    out->sum_E = (int64_t)r.sumE;
    out->sum_E2 = (int64_t)r.sumE2;
    out->sum_absM = (int64_t)r.sumAbsM;
    out->sum_M2 = (int64_t)r.sumM2;
    out->sum_c2 = (int64_t)r.sumC2;
    out->families = (int64_t)r.families;
    out->e = r.e;
    out->e2 = r.e2;
    out->abs_m = r.abs_m;
    out->m2 = r.m2;
    out->rho_t = r.rho_t;
    out->S_f = r.S_f;
    out->sv = r.sv;
    return PA_OK;
}

pa_status pa_free_energy(pa_ctx *c, double *lnZ_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!lnZ_out)
        return fail(c, PA_E_INVAL, "lnZ_out is NULL");
    pa_status s = fetch_record(c, "pa_free_energy");
    if (s != PA_OK)
        return s;
    *lnZ_out = c->hrec->lnZ;
    return PA_OK;
}

pa_status pa_export_state(pa_ctx *c, pa_host_state *st)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!st)
        return fail(c, PA_E_INVAL, "state is NULL");
    pa_status s = fetch_record(c, "pa_export_state");
    if (s != PA_OK)
        return s;
    const int64_t R = c->Rcur;
    const int k = c->cur;
    hipError_t e = hipSuccess;
    if (st->spins)
        e = hipMemcpy(st->spins, c->dv.spins[k], (size_t)((R + 63) / 64) * c->lp.N * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->energy)
        e = hipMemcpy(st->energy, c->dv.E[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->magnetization)
        e = hipMemcpy(st->magnetization, c->dv.M[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->label)
        e = hipMemcpy(st->label, c->dv.label[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_export_state");
    st->R = R;
    st->step = c->step;
    st->sweeps = c->sweeps;
    st->beta = c->beta;
    st->lnZ = c->hrec->lnZ;
    return PA_OK;
}

pa_status pa_import_state(pa_ctx *c, const pa_host_state *st)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!st || !st->spins || !st->energy || !st->magnetization || !st->label)
        return fail(c, PA_E_INVAL, "state and all four arrays are required");
    if (st->R < 1 || st->R > c->lp.cap)
        return fail(c, PA_E_INVAL, "state R must be in [1, capacity]");
    if (!std::isfinite(st->beta) || st->beta < 0.0 || !std::isfinite(st->lnZ))
        return fail(c, PA_E_INVAL, "beta and lnZ must be finite, beta >= 0");
    if (st->sweeps > (1u << 20))
        return fail(c, PA_E_INVAL, "sweeps out of range");
    const int N = c->lp.N, DN = c->lp.d * c->lp.N;
    for (int64_t j = 0; j < st->R; ++j) {
        if ((int64_t)st->label[j] >= c->lp.R0)
            return fail(c, PA_E_INVAL, "label out of range");
        const int32_t E = st->energy[j], M = st->magnetization[j];
        if (E < -DN || E > DN || ((E + DN) & 1) || M < -N || M > N)
            return fail(c, PA_E_INVAL, "energy or magnetisation out of range");
    }
    const int64_t R = st->R;
    const int k = c->cur;
    hipError_t e = hipMemcpy(c->dv.spins[k], st->spins, (size_t)((R + 63) / 64) * N * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->dv.E[k], st->energy, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->dv.M[k], st->magnetization, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c->dv.label[k], st->label, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = pa_launch_set_beta(c->lp, c->dv, st->beta, st->lnZ);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c->lp.stream);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_import_state");
    c->Rcur = R;
    c->step = st->step;
    c->sweeps = st->sweeps;
    c->beta = st->beta;
    c->reweighted = false;
    return PA_OK;
}

pa_status pa_overlap(pa_ctx *a, pa_ctx *b, int64_t *hist_out)
{
    if (!a || !b)
        return fail(a, PA_E_INVAL, "ctx is NULL");
    if (!hist_out)
        return fail(a, PA_E_INVAL, "hist_out is NULL");
    if (a->lp.d != b->lp.d || a->lp.L != b->lp.L)
        return fail(a, PA_E_INVAL, "runs on different lattices");
    const int64_t R = a->Rcur < b->Rcur ? a->Rcur : b->Rcur;
    const int N = a->lp.N;
    hipError_t e = hipStreamSynchronize(b->lp.stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(a->dv.qhist, 0, (size_t)(N + 1) * 8, a->lp.stream);
    if (e == hipSuccess)
        e = pa_launch_overlap(a->lp, a->dv.spins[a->cur], b->dv.spins[b->cur], R, a->dv.qhist);
    std::vector<unsigned long long> h((size_t)N + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), a->dv.qhist, h.size() * 8, hipMemcpyDeviceToHost, a->lp.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(a->lp.stream);
    if (e != hipSuccess)
        return hip_fail(a, e, "pa_overlap");
    for (int k = 0; k <= N; ++k)
        hist_out[k] = (int64_t)h[(size_t)k];
    return PA_OK;
}

pa_status pa_step_alpha(pa_ctx *c, double dbeta, double *alpha_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!alpha_out || !std::isfinite(dbeta) || dbeta < 0.0)
        return fail(c, PA_E_INVAL, "dbeta must be finite and >= 0; alpha_out non-NULL");
    hipError_t e = pa_launch_rule(c->lp, c->dv, c->cur, c->Rcur, 0.0, dbeta, 0, 0);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_step_alpha");
    pa_status s = fetch_record(c, "pa_step_alpha");
    if (s != PA_OK)
        return s;
    *alpha_out = c->hrec->rule_alpha;
    return PA_OK;
}

pa_status pa_step_rule(pa_ctx *c, double alpha_star, double dbeta_max, int32_t iterations, double *dbeta_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!dbeta_out || !(alpha_star > 0.0 && alpha_star < 1.0) || !std::isfinite(dbeta_max) || dbeta_max <= 0.0 ||
        iterations < 1 || iterations > 200)
        return fail(c, PA_E_INVAL, "need 0 < alpha_star < 1, dbeta_max > 0, 1 <= iterations <= 200");
    hipError_t e = pa_launch_rule(c->lp, c->dv, c->cur, c->Rcur, alpha_star, dbeta_max, iterations, 1);
    if (e != hipSuccess)
        return hip_fail(c, e, "pa_step_rule");
    pa_status s = fetch_record(c, "pa_step_rule");
    if (s != PA_OK)
        return s;
    *dbeta_out = c->hrec->rule_dbeta;
    return PA_OK;
}

pa_status pa_get_counters(pa_ctx *c, pa_counters *out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!out)
        return fail(c, PA_E_INVAL, "out is NULL");
    pa_status s = fetch_record(c, "pa_get_counters");
    if (s != PA_OK)
        return s;
    out->philox_calls = c->hrec->philox_calls;
    out->site_updates = c->hrec->site_updates;
    out->sweeps = c->sweeps_total;
    return PA_OK;
}

void pa_destroy(pa_ctx *c)
{
    if (!c)
        return;
    if (c->hrec)
        (void)hipHostFree(c->hrec);
    delete c;
}

const char *pa_last_error(const pa_ctx *c) { return c ? c->err.c_str() : g_init_err.c_str(); }

} // extern "C"
