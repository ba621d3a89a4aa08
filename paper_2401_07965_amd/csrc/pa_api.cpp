// Host side of the C ABI declared in include/pa.h: argument checks, the
// layout of the caller's device workspace, the block maps of a batch, the
// per-run state machine of the single-run calls, the batched anneal (with
// optional capture of the whole anneal in one HIP graph) and the autotuner.
// A single run (pa_ctx) is a batch of one.
#include "pa.h"
#include "pa_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <string>
#include <utility>
#include <vector>

namespace {

thread_local std::string g_init_err;
int g_max_lds = 0;

constexpr int64_t kMaxCapacity = (1ll << 24) - 64; // R W_j < 2^64 for W_j <= 2^40
constexpr int kMaxSites = 16384;                  // LDS and 8-plane counters per thread
constexpr int kMaxRuns = 65536;

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
    int J; // 1: couplings given (+-J bonds), 0: ferromagnet
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
        *msg = "capacity must satisfy R <= capacity <= 2^24 - 64";
        return PA_E_INVAL;
    }
    g->d = cfg->dim;
    g->L = cfg->L;
    g->J = cfg->couplings ? 1 : 0;
    g->N = (int)N;
    g->H = cfg->dim * (int)N / 2 + 1;
    g->R = cfg->R;
    g->cap = cap;
    g->W = (cap + 63) / 64;
    return PA_OK;
}

// Sweep workgroup sizes: 64..768 lanes, at most 255 unsatisfied bonds per
// lane for the measurement's 8-plane counters.
constexpr int kSweepMaxLanes = 768;
bool sweep_threads_ok(int N, int d, int t)
{
    return t >= 64 && t <= kSweepMaxLanes && t % 64 == 0 && (int64_t)((N + t - 1) / t) * d <= 255;
}

constexpr int kLdsPerCu = 163840; // gfx950: 160 KiB of LDS per CU

// Default sweep workgroup size, by a score: resident sweep waves per CU
// (limited by the LDS of the lattice and queues and by whole workgroups of
// waves) times the fraction of lanes busy over a colour's sites (N/2 sites in
// rounds of t lanes).  Waves are counted up to 4 per SIMD (what the sweep's
// registers allow) for workgroups of one or two waves and up to 3 for larger
// ones: measured, 3D L = 8 and 10 sweep 3-13 % faster with 16 resident waves
// of 128-lane workgroups than with 12 of 64 lanes, while larger workgroups
// gain nothing from a fourth wave per SIMD (their waves meet at the end of
// every colour).  The smaller size wins ties.  Autotuning refines it for
// batches.
int default_sweep_threads(int N, int d, bool J)
{
    const int lds_max = g_max_lds ? g_max_lds : kLdsPerCu;
    const int nh = N / 2;
    int best = 0;
    double best_score = -1.0;
    for (int t = 64; t <= 768; t += 64) {
        const size_t lds = pa_sweep_lds_bytes(N, d, t, J);
        if (!sweep_threads_ok(N, d, t) || lds > (size_t)lds_max)
            continue;
        const int w = t / 64;
        const int cap = 4 * (w <= 2 ? 4 : 3); // waves per CU counted
        int blocks = (int)(kLdsPerCu / lds);
        if (blocks > cap / w)
            blocks = cap / w;
        const int waves = blocks * w;
        const int rounds = (nh + t - 1) / t;
        const double score = waves * ((double)nh / ((double)rounds * t));
        if (score > best_score + 1e-9) {
            best_score = score;
            best = t;
        }
    }
    return best ? best : 768; // none fits: rejected by the LDS check of the batch set-up
}

uint64_t round256(uint64_t b) { return (b + 255) / 256 * 256; }

// Buffers of one run (base may be null to only measure them).
uint64_t carve_run(const Geometry &g, char *base, PaDev *dv)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += round256(bytes);
        return p;
    };
    const uint64_t words = (uint64_t)g.W * g.N;
    const uint64_t slots = (uint64_t)g.W * 64;
    const uint64_t chunks = (uint64_t)((g.cap + PA_CHUNK - 1) / PA_CHUNK);
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
    d.anc = (uint32_t *)take(slots * 4);
    d.C = (uint64_t *)take(slots * 8);
    d.qhist = (unsigned long long *)take((uint64_t)(g.N + 1) * 8);
    // tile flags of the two prefix sums of a resampling (weights, copy numbers)
    d.tiles = (PaScanTile *)take((uint64_t)(2 * pa_tiles_per_sum(g.cap)) * sizeof(PaScanTile));
    d.partial = (double *)take(chunks * 8);
    d.fam = (uint32_t *)take((uint64_t)g.R * 4);
    d.lw = (double *)take(slots * 8);
    d.Wj = (uint64_t *)take(slots * 8);
    d.wpart = (double *)take(chunks * PA_WPARTS * 8);
    d.rec = (PaRecord *)take(sizeof(PaRecord));
    if (dv)
        *dv = d;
    return off;
}

} // namespace

// A batch of independent runs sharing one workspace and one stream.
struct Batch {
    int M = 0;
    std::vector<Geometry> geo;
    std::vector<PaRunDesc> hdesc;
    std::vector<std::vector<uint8_t>> jmask;
    PaBatchView v{};
    PaRunDesc *ddesc = nullptr;
    int32_t *dgroup = nullptr, *dNs = nullptr;
    double *dcomb = nullptr;
    PaRecord *hrec = nullptr; // pinned host copies of the M device records
    int max_points = 0;
    std::string err;
    // host bookkeeping of the single-run calls
    double beta = 0.0, beta_next = 0.0;
    uint64_t sweeps_total = 0;
    uint32_t sweeps = 0;
    bool reweighted = false;
    int anneal_points = 0;
    // launch bookkeeping: the state of the runs' level histograms (PA_HIST_*:
    // the observables pass builds them from zero, so do the step rule and the
    // reweighting when they find them not valid; the reweighting clears them
    // after use); the latest launch was a reweighting, which also prepared the
    // resampling's flags and status
    int hist_state = PA_HIST_STALE;
    bool rs_prepped = false;
    // a resampling was launched since the last sweep: its spins may still be
    // in the other buffer (the device record says whether), taken in by the
    // next sweep or gathered before anything else reads them
    bool gather_pending = false;
    // the latest anneal captured as a HIP graph, replayed while the anneal's
    // arguments (schedule, theta, scheme) and the groups' workgroup sizes stay
    // the same
    hipGraphExec_t anneal_exec = nullptr;
    std::vector<double> anneal_betas;
    int anneal_theta = -1, anneal_scheme = -1;
    std::vector<int> anneal_threads;
    int anneal_end_hist = PA_HIST_STALE; // bookkeeping after the captured anneal
    bool anneal_end_rs = false;
    bool anneal_end_gather = false;
};

namespace {

// Launch wrappers that keep the bookkeeping above.
hipError_t launch_init(Batch *b)
{
    hipError_t e = pa_b_init(b->v); // clears the histograms
    b->hist_state = PA_HIST_ZERO;
    b->rs_prepped = false;
    b->gather_pending = false;
    return e;
}

// The spins of a resampling that no sweep has taken in yet, gathered before
// anything other than a sweep reads them.
hipError_t settle_spins(Batch *b)
{
    if (!b->gather_pending)
        return hipSuccess;
    b->gather_pending = false;
    return pa_b_gather(b->v);
}

hipError_t launch_reweight(Batch *b, double beta_next)
{
    hipError_t e = pa_b_reweight(b->v, beta_next, b->hist_state);
    b->hist_state = PA_HIST_ZERO;
    b->rs_prepped = true;
    return e;
}

hipError_t launch_resample(Batch *b, int scheme, int freeze, int kq)
{
    hipError_t e = settle_spins(b); // the ancestors below are of the populations as they are now
    if (e == hipSuccess)
        e = pa_b_resample(b->v, scheme, freeze, kq, b->rs_prepped);
    b->gather_pending = true;
    b->rs_prepped = false;
    if (b->hist_state == PA_HIST_VALID) // a histogram of the replaced population
        b->hist_state = PA_HIST_STALE;
    return e;
}

// The observables pass also builds the level histogram unless it is valid.
hipError_t launch_observables(Batch *b, int point)
{
    hipError_t e = pa_b_observables(b->v, point, b->hist_state);
    b->hist_state = PA_HIST_VALID;
    b->rs_prepped = false;
    return e;
}

// Sweeps (cluster updates: cluster != 0) of every run change the energies.
hipError_t launch_updates(Batch *b, int n, uint32_t t0, int cluster)
{
    hipError_t e = hipSuccess;
    if (cluster) {
        e = settle_spins(b);
        if (e == hipSuccess)
            e = pa_b_cluster(b->v, n, t0);
    } else {
        e = pa_b_sweep(b->v, n, t0, b->gather_pending ? 1 : 0);
        b->gather_pending = false;
    }
    if (b->hist_state == PA_HIST_VALID)
        b->hist_state = PA_HIST_STALE;
    return e;
}

// The step rule and the learned step build the histogram when it is not valid.
void histogram_built(Batch *b)
{
    b->hist_state = PA_HIST_VALID;
    b->rs_prepped = false;
}

// An imported population: the histogram describes another one.
void population_replaced(Batch *b)
{
    b->hist_state = PA_HIST_STALE;
    b->rs_prepped = false;
    b->gather_pending = false;
}

} // namespace

struct pa_ctx {
    Batch b;
};

struct pa_batch {
    Batch b;
};

struct pa_mlp {
    PaMlpDev d{};
    int max_samples = 0;
    int n = 0;     // samples set
    int t = 0;     // Adam steps taken
    std::string err;
};

namespace {

pa_status fail(Batch *b, pa_status s, const std::string &msg)
{
    if (b)
        b->err = msg;
    else
        g_init_err = msg;
    return s;
}

pa_status hip_fail(Batch *b, hipError_t e, const char *where)
{
    return fail(b, PA_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Whole layout of a batch: tables first, then each run's buffers.
struct Tables {
    std::vector<PaBlk> rep, hrep, crep, fam, col, tile;
    std::vector<std::vector<PaBlk>> gcol;
    std::vector<int> gd, gN, gJ, gthreads;
};

uint64_t layout(const std::vector<Geometry> &geo, int max_points, char *base, Batch *b, Tables *t)
{
    const int M = (int)geo.size();
    Tables tb;
    std::map<std::tuple<int, int, int>, int> group_of_shape;
    std::vector<int> run_group(M);
    for (int m = 0; m < M; ++m) {
        const Geometry &g = geo[m];
        for (int64_t c = 0; c < (g.cap + PA_CHUNK - 1) / PA_CHUNK; ++c)
            tb.rep.push_back({(uint32_t)m, (uint32_t)c});
        for (int64_t c = 0; c < (g.cap + PA_HCHUNK - 1) / PA_HCHUNK; ++c)
            tb.hrep.push_back({(uint32_t)m, (uint32_t)c});
        for (int64_t c = 0; c < (g.cap + pa_counts_tile(g.cap) - 1) / pa_counts_tile(g.cap); ++c)
            tb.crep.push_back({(uint32_t)m, (uint32_t)c});
        for (int64_t c = 0; c < (g.R + PA_HCHUNK - 1) / PA_HCHUNK; ++c)
            tb.fam.push_back({(uint32_t)m, (uint32_t)c});
        for (int64_t w = 0; w < g.W; ++w)
            tb.col.push_back({(uint32_t)m, (uint32_t)w});
        for (int64_t k = 0; k < (g.cap + PA_SCAN_TILE - 1) / PA_SCAN_TILE; ++k)
            tb.tile.push_back({(uint32_t)m, (uint32_t)k});
        const auto key = std::make_tuple(g.d, g.L, g.J);
        auto it = group_of_shape.find(key);
        if (it == group_of_shape.end()) {
            it = group_of_shape.emplace(key, (int)tb.gcol.size()).first;
            tb.gcol.emplace_back();
            tb.gd.push_back(g.d);
            tb.gN.push_back(g.N);
            tb.gJ.push_back(g.J);
            tb.gthreads.push_back(default_sweep_threads(g.N, g.d, g.J != 0));
        }
        for (int64_t w = 0; w < g.W; ++w)
            tb.gcol[it->second].push_back({(uint32_t)m, (uint32_t)w});
    }
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += round256(bytes);
        return p;
    };
    char *p_desc = take(sizeof(PaRunDesc) * (uint64_t)M);
    char *p_rep = take(sizeof(PaBlk) * tb.rep.size());
    char *p_hrep = take(sizeof(PaBlk) * tb.hrep.size());
    char *p_crep = take(sizeof(PaBlk) * tb.crep.size());
    char *p_fam = take(sizeof(PaBlk) * tb.fam.size());
    char *p_col = take(sizeof(PaBlk) * tb.col.size());
    char *p_tile = take(sizeof(PaBlk) * tb.tile.size());
    std::vector<char *> p_g;
    for (auto &gc : tb.gcol)
        p_g.push_back(take(sizeof(PaBlk) * gc.size()));
    char *p_steprec = take(sizeof(PaStepRecord) * (uint64_t)M * (uint64_t)(max_points > 0 ? max_points : 0));
    char *p_group = take(4ull * M);
    char *p_Ns = take(4ull * M);
    char *p_comb = take(8ull * PA_COMBINE_FIELDS * M);
    std::vector<PaDev> devs(M);
    for (int m = 0; m < M; ++m) {
        char *rb = take(0); // current offset
        const uint64_t n = carve_run(geo[m], rb, &devs[m]);
        off += n;
    }
    if (b) {
        b->M = M;
        b->geo = geo;
        b->hdesc.resize(M);
        int maxH = 0;
        for (int m = 0; m < M; ++m) {
            PaRunDesc &d = b->hdesc[m];
            d.d = geo[m].d;
            d.L = geo[m].L;
            d.N = geo[m].N;
            d.H = geo[m].H;
            d.R0 = geo[m].R;
            d.cap = geo[m].cap;
            d.dv = devs[m];
            maxH = geo[m].H > maxH ? geo[m].H : maxH;
        }
        b->ddesc = (PaRunDesc *)p_desc;
        PaBatchView &v = b->v;
        v.runs = (const PaRunDesc *)p_desc;
        v.nruns = (uint32_t)M;
        v.rep = (const PaBlk *)p_rep;
        v.nrep = (uint32_t)tb.rep.size();
        v.hrep = (const PaBlk *)p_hrep;
        v.nhrep = (uint32_t)tb.hrep.size();
        v.crep = (const PaBlk *)p_crep;
        v.ncrep = (uint32_t)tb.crep.size();
        v.fam = (const PaBlk *)p_fam;
        v.nfam = (uint32_t)tb.fam.size();
        v.col = (const PaBlk *)p_col;
        v.ncol = (uint32_t)tb.col.size();
        v.tile = (const PaBlk *)p_tile;
        v.ntile = (uint32_t)tb.tile.size();
        v.maxH = maxH;
        v.ngroups = (int)tb.gcol.size();
        for (int g = 0; g < v.ngroups; ++g) {
            v.gcol[g] = (const PaBlk *)p_g[g];
            v.gncol[g] = (uint32_t)tb.gcol[g].size();
            v.gd[g] = tb.gd[g];
            v.gN[g] = tb.gN[g];
            v.gJ[g] = tb.gJ[g];
            v.gthreads[g] = tb.gthreads[g];
        }
        v.steprec = (PaStepRecord *)p_steprec;
        v.npoints = max_points;
        b->dgroup = (int32_t *)p_group;
        b->dNs = (int32_t *)p_Ns;
        b->dcomb = (double *)p_comb;
        b->max_points = max_points;
    }
    if (t)
        *t = std::move(tb);
    return off;
}

pa_status check_batch(const pa_config *cfgs, int32_t nruns, int32_t max_points, std::vector<Geometry> *geo,
                      std::string *msg)
{
    if (!cfgs || nruns < 1 || nruns > kMaxRuns) {
        *msg = "need 1 <= nruns <= 65536 configurations";
        return PA_E_INVAL;
    }
    if (max_points < 0 || max_points > 1000000) {
        *msg = "max_points out of range";
        return PA_E_INVAL;
    }
    geo->resize(nruns);
    std::map<std::tuple<int, int, int>, int> shapes;
    for (int m = 0; m < nruns; ++m) {
        pa_status s = check_config(&cfgs[m], &(*geo)[m], msg);
        if (s != PA_OK) {
            *msg = "run " + std::to_string(m) + ": " + *msg;
            return s;
        }
        shapes[std::make_tuple(cfgs[m].dim, cfgs[m].L, cfgs[m].couplings ? 1 : 0)] = 1;
    }
    if ((int)shapes.size() > PA_MAX_GROUPS) {
        *msg = "at most 16 groups of (lattice shape, couplings given or not) per batch";
        return PA_E_INVAL;
    }
    return PA_OK;
}

// couplings -> per-site masks of the 2d incident bonds
pa_status coupling_masks(const pa_config &cfg, const Geometry &g, std::vector<uint8_t> *jm, std::string *msg)
{
    jm->assign((size_t)g.N, 0);
    if (!cfg.couplings)
        return PA_OK;
    for (int64_t s0 = 0; s0 < g.N; ++s0) {
        int64_t stride = 1;
        for (int mu = 0; mu < g.d; ++mu) {
            const int8_t J = cfg.couplings[s0 * g.d + mu];
            if (J != 1 && J != -1) {
                *msg = "couplings must be +1 or -1";
                return PA_E_INVAL;
            }
            if (J == -1) {
                const int64_t x = (s0 / stride) % g.L;
                const int64_t s1 = s0 + ((x + 1) % g.L - x) * stride;
                (*jm)[(size_t)s0] |= (uint8_t)(1u << mu);
                (*jm)[(size_t)s1] |= (uint8_t)(1u << (g.d + mu));
            }
            stride *= g.L;
        }
    }
    return PA_OK;
}

void free_batch(Batch *b);

pa_status make_batch(const pa_config *cfgs, int32_t nruns, int32_t max_points, void *workspace, uint64_t bytes,
                     void *stream, Batch *b)
{
    std::vector<Geometry> geo;
    std::string msg;
    pa_status s = check_batch(cfgs, nruns, max_points, &geo, &msg);
    if (s != PA_OK)
        return fail(nullptr, s, msg);
    const uint64_t need = layout(geo, max_points, nullptr, nullptr, nullptr);
    if (!workspace || bytes < need)
        return fail(nullptr, PA_E_INVAL, "workspace missing or smaller than the required bytes");
    if (((uintptr_t)workspace & 255u) != 0)
        return fail(nullptr, PA_E_INVAL, "workspace must be 256-byte aligned");
    hipError_t e;
    if (g_max_lds == 0 && (e = pa_query_lds(&g_max_lds)) != hipSuccess)
        return hip_fail(nullptr, e, "device query");
    for (const Geometry &g : geo)
        if (pa_sweep_lds_bytes(g.N, g.d, default_sweep_threads(g.N, g.d, g.J != 0), g.J != 0) > (size_t)g_max_lds ||
            (size_t)g.H * 4 > (size_t)g_max_lds)
            return fail(nullptr, PA_E_INVAL, "lattice too large for the workgroup LDS of this device");
    b->jmask.resize(nruns);
    for (int m = 0; m < nruns; ++m)
        if ((s = coupling_masks(cfgs[m], geo[m], &b->jmask[m], &msg)) != PA_OK)
            return fail(nullptr, s, "run " + std::to_string(m) + ": " + msg);
    Tables t;
    layout(geo, max_points, (char *)workspace, b, &t);
    for (int m = 0; m < nruns; ++m) {
        b->hdesc[m].seed = cfgs[m].seed;
        b->hdesc[m].run_id = cfgs[m].run_id;
    }
    b->v.stream = (hipStream_t)stream;
    if ((e = hipHostMalloc((void **)&b->hrec, sizeof(PaRecord) * (size_t)nruns, hipHostMallocDefault)) !=
        hipSuccess)
        return hip_fail(nullptr, e, "pinned records");
    if (b->v.ngroups > 1) { // side streams (default priority) and events for the groups' sweeps
        e = hipEventCreateWithFlags(&b->v.fork, hipEventDisableTiming);
        for (int g = 0; g < b->v.ngroups && e == hipSuccess; ++g) {
            e = hipStreamCreateWithFlags(&b->v.gstream[g], hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&b->v.join[g], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            free_batch(b);
            return hip_fail(nullptr, e, "group streams");
        }
    }
    const hipStream_t st = b->v.stream;
    auto up = [&](const void *dst, const void *src, size_t n) {
        if (e == hipSuccess && n)
            e = hipMemcpyAsync(const_cast<void *>(dst), src, n, hipMemcpyHostToDevice, st);
    };
    e = hipSuccess;
    up(b->ddesc, b->hdesc.data(), sizeof(PaRunDesc) * nruns);
    up(b->v.rep, t.rep.data(), sizeof(PaBlk) * t.rep.size());
    up(b->v.hrep, t.hrep.data(), sizeof(PaBlk) * t.hrep.size());
    up(b->v.crep, t.crep.data(), sizeof(PaBlk) * t.crep.size());
    up(b->v.fam, t.fam.data(), sizeof(PaBlk) * t.fam.size());
    up(b->v.col, t.col.data(), sizeof(PaBlk) * t.col.size());
    up(b->v.tile, t.tile.data(), sizeof(PaBlk) * t.tile.size());
    for (int g = 0; g < b->v.ngroups; ++g)
        up(b->v.gcol[g], t.gcol[g].data(), sizeof(PaBlk) * t.gcol[g].size());
    for (int m = 0; m < nruns; ++m)
        up(b->hdesc[m].dv.jmask, b->jmask[m].data(), b->jmask[m].size());
    if (e == hipSuccess)
        e = launch_init(b);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(nullptr, e, "batch set-up");
    }
    return PA_OK;
}

pa_status fetch_records(Batch *b, const char *where)
{
    hipError_t e = hipSuccess;
    for (int m = 0; m < b->M && e == hipSuccess; ++m)
        e = hipMemcpyAsync(b->hrec + m, b->hdesc[m].dv.rec, sizeof(PaRecord), hipMemcpyDeviceToHost, b->v.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(b->v.stream);
    if (e != hipSuccess)
        return hip_fail(b, e, where);
    return PA_OK;
}

pa_status status_error(Batch *b, uint32_t st)
{
    if (st & PA_ST_SCAN_TIMEOUT)
        return fail(b, PA_E_DEVICE, "prefix-sum look-back timed out");
    if (st & PA_ST_NONFINITE)
        return fail(b, PA_E_NONFINITE, "ln Q is not finite");
    if (st & PA_ST_CAPACITY)
        return fail(b, PA_E_CAPACITY, "resampled population exceeds the capacity");
    if (st & PA_ST_EXTINCT)
        return fail(b, PA_E_EXTINCT, "resampled population is empty");
    return PA_OK;
}

// Records of a single run once its stream has drained.  A run frozen by a
// deferred pa_resample reports the failure that froze it.
pa_status ctx_records(Batch *b, const char *where)
{
    pa_status s = fetch_records(b, where);
    if (s != PA_OK)
        return s;
    if (b->hrec[0].status & PA_ST_FROZEN)
        return status_error(b, b->hrec[0].status);
    return PA_OK;
}

// The overlap rule and the learned step read the energy histogram, which
// describes a uniform population only.
pa_status need_uniform(Batch *b, const char *where)
{
    if (!b->v.weights)
        return PA_OK;
    pa_status s = ctx_records(b, where);
    if (s != PA_OK)
        return s;
    if (b->hrec[0].weighted)
        return fail(b, PA_E_STATE,
                    std::string(where) + " needs a uniform population: a kept step left weights (resample first)");
    return PA_OK;
}

pa_status export_run(Batch *b, int m, pa_host_state *st)
{
    const hipError_t eg = settle_spins(b);
    if (eg != hipSuccess)
        return hip_fail(b, eg, "export");
    pa_status s = fetch_records(b, "export");
    if (s != PA_OK)
        return s;
    const PaRecord &r = b->hrec[m];
    const PaRunDesc &d = b->hdesc[m];
    const int64_t R = (int64_t)r.Rcur;
    const int k = r.cur;
    hipError_t e = hipSuccess;
    if (st->spins)
        e = hipMemcpy(st->spins, d.dv.spins[k], (size_t)((R + 63) / 64) * d.N * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->energy)
        e = hipMemcpy(st->energy, d.dv.E[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->magnetization)
        e = hipMemcpy(st->magnetization, d.dv.M[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && st->label)
        e = hipMemcpy(st->label, d.dv.label[k], (size_t)R * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(b, e, "export");
    st->R = R;
    st->step = r.step;
    st->sweeps = r.sweeps;
    st->beta = r.beta;
    st->lnZ = r.lnZ;
    return PA_OK;
}

void drop_anneal_graph(Batch *b)
{
    if (b->anneal_exec)
        (void)hipGraphExecDestroy(b->anneal_exec);
    b->anneal_exec = nullptr;
    b->anneal_betas.clear();
    b->anneal_theta = b->anneal_scheme = -1;
    b->anneal_threads.clear();
}

void free_batch(Batch *b)
{
    drop_anneal_graph(b);
    if (b->hrec)
        (void)hipHostFree(b->hrec);
    b->hrec = nullptr;
    for (int g = 0; g < PA_MAX_GROUPS; ++g) {
        if (b->v.gstream[g])
            (void)hipStreamDestroy(b->v.gstream[g]);
        if (b->v.join[g])
            (void)hipEventDestroy(b->v.join[g]);
        b->v.gstream[g] = nullptr;
        b->v.join[g] = nullptr;
    }
    if (b->v.fork)
        (void)hipEventDestroy(b->v.fork);
    b->v.fork = nullptr;
}

} // namespace

extern "C" {

// ====================================================================== single run
pa_status pa_required_bytes(const pa_config *cfg, uint64_t *bytes)
{
    std::vector<Geometry> geo;
    std::string msg;
    pa_status s = check_batch(cfg, 1, 0, &geo, &msg);
    if (s != PA_OK)
        return fail(nullptr, s, msg);
    if (!bytes)
        return fail(nullptr, PA_E_INVAL, "bytes is NULL");
    *bytes = layout(geo, 0, nullptr, nullptr, nullptr);
    return PA_OK;
}

pa_status pa_init(const pa_config *cfg, void *workspace, uint64_t workspace_bytes, void *stream, pa_ctx **out)
{
    if (!out)
        return fail(nullptr, PA_E_INVAL, "out is NULL");
    *out = nullptr;
    pa_ctx *c = new (std::nothrow) pa_ctx;
    if (!c)
        return fail(nullptr, PA_E_NOMEM, "out of host memory");
    pa_status s = make_batch(cfg, 1, 0, workspace, workspace_bytes, stream, &c->b);
    if (s != PA_OK) {
        delete c;
        return s;
    }
    *out = c;
    return PA_OK;
}

pa_status pa_sweep(pa_ctx *c, int32_t theta)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (theta < 0)
        return fail(b, PA_E_INVAL, "theta must be >= 0");
    if ((uint64_t)b->sweeps + (uint64_t)theta > (1u << 20))
        return fail(b, PA_E_INVAL, "more than 2^20 sweeps at one temperature");
    if (theta == 0)
        return PA_OK;
    hipError_t e = launch_updates(b, theta, b->sweeps, 0);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_sweep");
    b->sweeps += (uint32_t)theta;
    b->sweeps_total += (uint64_t)theta;
    return PA_OK;
}

pa_status pa_cluster(pa_ctx *c, int32_t nsteps)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (nsteps < 0)
        return fail(b, PA_E_INVAL, "nsteps must be >= 0");
    if ((uint64_t)b->sweeps + (uint64_t)nsteps > (1u << 20))
        return fail(b, PA_E_INVAL, "more than 2^20 sweeps and cluster updates at one temperature");
    for (int g = 0; g < b->v.ngroups; ++g)
        if (pa_cluster_lds_bytes(b->v.gN[g], b->v.gJ[g] != 0) > (size_t)g_max_lds)
            return fail(b, PA_E_INVAL, "lattice too large for cluster updates (LDS of one workgroup)");
    if (nsteps == 0)
        return PA_OK;
    hipError_t e = launch_updates(b, nsteps, b->sweeps, 1);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_cluster");
    b->sweeps += (uint32_t)nsteps;
    b->sweeps_total += (uint64_t)nsteps;
    return PA_OK;
}

pa_status pa_reweight(pa_ctx *c, double beta_next, double *lnQ_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!std::isfinite(beta_next) || beta_next < b->beta)
        return fail(b, PA_E_INVAL, "beta_next must be finite and >= the current beta");
    hipError_t e = launch_reweight(b, beta_next);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_reweight");
    if (!lnQ_out) { // deferred: a non-finite ln Q is caught by the resampling
        b->reweighted = true;
        b->beta_next = beta_next;
        return PA_OK;
    }
    pa_status s = ctx_records(b, "pa_reweight");
    if (s != PA_OK)
        return s;
    if (!std::isfinite(b->hrec[0].lnQ)) {
        b->reweighted = false;
        return fail(b, PA_E_NONFINITE, "ln Q is not finite");
    }
    b->reweighted = true;
    b->beta_next = beta_next;
    if (lnQ_out)
        *lnQ_out = b->hrec[0].lnQ;
    return PA_OK;
}

pa_status pa_resample(pa_ctx *c, pa_resampler scheme, int64_t *R_new_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if ((int)scheme < 0 || (int)scheme > 3)
        return fail(b, PA_E_INVAL, "unknown resampling scheme");
    if (!b->reweighted)
        return fail(b, PA_E_STATE, "pa_resample needs a pa_reweight first");
    const bool deferred = R_new_out == nullptr;
    hipError_t e = launch_resample(b, (int)scheme, deferred ? 1 : 0, -1);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_resample");
    if (deferred) { // a failure freezes the run; the next synchronising call reports it
        b->beta = b->beta_next;
        b->sweeps = 0;
        b->reweighted = false;
        return PA_OK;
    }
    pa_status s = ctx_records(b, "pa_resample");
    if (s != PA_OK)
        return s;
    if (b->hrec[0].skip)
        return status_error(b, b->hrec[0].status);
    b->beta = b->beta_next;
    b->sweeps = 0;
    b->reweighted = false;
    if (R_new_out)
        *R_new_out = (int64_t)b->hrec[0].Rcur;
    return PA_OK;
}

pa_status pa_resample_conditional(pa_ctx *c, pa_resampler scheme, double kappa, int64_t *R_new_out,
                                  int32_t *resampled_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if ((int)scheme < 0 || (int)scheme > 3)
        return fail(b, PA_E_INVAL, "unknown resampling scheme");
    if (!(kappa >= 0.0 && kappa <= 1.0))
        return fail(b, PA_E_INVAL, "kappa must lie in [0, 1]");
    if (!b->reweighted)
        return fail(b, PA_E_STATE, "pa_resample_conditional needs a pa_reweight first");
    // From now on the reweighting runs the per-replica passes a weighted
    // population needs.  This step's population is still uniform (only a step
    // of this call can keep one), so its reweighting is complete already.
    b->v.weights = true;
    const int kq = (int)std::floor(kappa * 65536.0 + 0.5);
    const bool deferred = R_new_out == nullptr && resampled_out == nullptr;
    hipError_t e = launch_resample(b, (int)scheme, deferred ? 1 : 0, kq);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_resample_conditional");
    if (deferred) {
        b->beta = b->beta_next;
        b->sweeps = 0;
        b->reweighted = false;
        return PA_OK;
    }
    pa_status s = ctx_records(b, "pa_resample_conditional");
    if (s != PA_OK)
        return s;
    if (b->hrec[0].skip)
        return status_error(b, b->hrec[0].status);
    b->beta = b->beta_next;
    b->sweeps = 0;
    b->reweighted = false;
    if (R_new_out)
        *R_new_out = (int64_t)b->hrec[0].Rcur;
    if (resampled_out)
        *resampled_out = b->hrec[0].keep ? 0 : 1;
    return PA_OK;
}

pa_status pa_log_weights(pa_ctx *c, double *out, int32_t *weighted_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!out)
        return fail(b, PA_E_INVAL, "out is NULL");
    pa_status s = fetch_records(b, "pa_log_weights");
    if (s != PA_OK)
        return s;
    const PaRecord &r = b->hrec[0];
    const int64_t R = (int64_t)r.Rcur;
    if (r.weighted) {
        hipError_t e = hipMemcpy(out, b->hdesc[0].dv.lw, (size_t)R * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return hip_fail(b, e, "pa_log_weights");
    } else {
        std::fill(out, out + R, 0.0);
    }
    if (weighted_out)
        *weighted_out = r.weighted ? 1 : 0;
    return PA_OK;
}

pa_status pa_observables(pa_ctx *c, pa_obs *out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    hipError_t e = launch_observables(b, -1);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_observables");
    if (!out)
        return PA_OK;
    pa_status s = ctx_records(b, "pa_observables");
    if (s != PA_OK)
        return s;
    const PaRecord &r = b->hrec[0];
    out->R = (int64_t)r.Rcur;
    out->beta = r.beta;
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
    out->sum_E3_hi = (int64_t)r.sumE3[1];
    out->sum_E3_lo = (uint64_t)r.sumE3[0];
    out->e3 = r.e3;
    out->ess = r.ess;
    out->weighted = r.weighted ? 1 : 0;
    out->pad = 0;
    return PA_OK;
}

pa_status pa_free_energy(pa_ctx *c, double *lnZ_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!lnZ_out)
        return fail(b, PA_E_INVAL, "lnZ_out is NULL");
    pa_status s = ctx_records(b, "pa_free_energy");
    if (s != PA_OK)
        return s;
    *lnZ_out = b->hrec[0].lnZ;
    return PA_OK;
}

pa_status pa_export_state(pa_ctx *c, pa_host_state *st)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    if (!st)
        return fail(&c->b, PA_E_INVAL, "state is NULL");
    return export_run(&c->b, 0, st);
}

pa_status pa_import_state(pa_ctx *c, const pa_host_state *st)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    const PaRunDesc &d = b->hdesc[0];
    if (!st || !st->spins || !st->energy || !st->magnetization || !st->label)
        return fail(b, PA_E_INVAL, "state and all four arrays are required");
    if (st->R < 1 || st->R > d.cap)
        return fail(b, PA_E_INVAL, "state R must be in [1, capacity]");
    if (!std::isfinite(st->beta) || st->beta < 0.0 || !std::isfinite(st->lnZ))
        return fail(b, PA_E_INVAL, "beta and lnZ must be finite, beta >= 0");
    if (st->sweeps > (1u << 20))
        return fail(b, PA_E_INVAL, "sweeps out of range");
    const int N = d.N, DN = d.d * d.N;
    for (int64_t j = 0; j < st->R; ++j) {
        if ((int64_t)st->label[j] >= d.R0)
            return fail(b, PA_E_INVAL, "label out of range");
        const int32_t E = st->energy[j], M = st->magnetization[j];
        if (E < -DN || E > DN || ((E + DN) & 1) || M < -N || M > N)
            return fail(b, PA_E_INVAL, "energy or magnetisation out of range");
    }
    pa_status s = fetch_records(b, "pa_import_state");
    if (s != PA_OK)
        return s;
    const int64_t R = st->R;
    const int k = b->hrec[0].cur;
    hipError_t e = hipMemcpy(d.dv.spins[k], st->spins, (size_t)((R + 63) / 64) * N * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d.dv.E[k], st->energy, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d.dv.M[k], st->magnetization, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d.dv.label[k], st->label, (size_t)R * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = pa_b_set_beta(b->v, st->beta, st->lnZ, st->step, st->sweeps, (uint64_t)R);
    population_replaced(b);
    if (e == hipSuccess)
        e = hipStreamSynchronize(b->v.stream);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_import_state");
    b->beta = st->beta;
    b->sweeps = st->sweeps;
    b->reweighted = false;
    return PA_OK;
}

pa_status pa_philox_probe(void *out, int64_t nthreads, int32_t iters, void *stream)
{
    if (!out || nthreads < 256 || nthreads % 256 || nthreads > (1 << 24) || iters < 1)
        return fail(nullptr, PA_E_INVAL, "need out, nthreads a multiple of 256 in [256, 2^24], iters >= 1");
    const hipError_t e = pa_launch_philox_probe((uint32_t *)out, nthreads, iters, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(nullptr, e, "pa_philox_probe");
    return PA_OK;
}

pa_status pa_overlap(pa_ctx *a, pa_ctx *c2, int64_t *hist_out)
{
    if (!a || !c2)
        return fail(a ? &a->b : nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *A = &a->b, *B = &c2->b;
    if (!hist_out)
        return fail(A, PA_E_INVAL, "hist_out is NULL");
    if (A->hdesc[0].d != B->hdesc[0].d || A->hdesc[0].L != B->hdesc[0].L)
        return fail(A, PA_E_INVAL, "runs on different lattices");
    const int N = A->hdesc[0].N;
    hipError_t e = settle_spins(B);
    if (e == hipSuccess)
        e = settle_spins(A);
    if (e == hipSuccess)
        e = hipStreamSynchronize(B->v.stream);
    if (e == hipSuccess)
        e = pa_launch_overlap(A->ddesc, B->ddesc, N, A->v.ncol, A->hdesc[0].dv.qhist, A->v.stream);
    std::vector<unsigned long long> h((size_t)N + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), A->hdesc[0].dv.qhist, h.size() * 8, hipMemcpyDeviceToHost, A->v.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(A->v.stream);
    if (e != hipSuccess)
        return hip_fail(A, e, "pa_overlap");
    for (int k = 0; k <= N; ++k)
        hist_out[k] = (int64_t)h[(size_t)k];
    return PA_OK;
}

pa_status pa_overlap_noalloc(pa_ctx *a, pa_ctx *c2, int64_t *hist_out)
{
    if (!a || !c2)
        return fail(a ? &a->b : nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *A = &a->b, *B = &c2->b;
    if (!hist_out)
        return fail(A, PA_E_INVAL, "hist_out is NULL");
    if (A->hdesc[0].d != B->hdesc[0].d || A->hdesc[0].L != B->hdesc[0].L)
        return fail(A, PA_E_INVAL, "runs on different lattices");
    const int N = A->hdesc[0].N;
    if (N + 1 > PA_NOALLOC_HIST_MAX)
        return fail(A, PA_E_INVAL, "N + 1 exceeds the allocation-free histogram's " +
                                       std::to_string(PA_NOALLOC_HIST_MAX) + " counters");
    // the device of run a's stream holds the histogram this call uses
    int dev = 0;
    hipError_t e = A->v.stream ? hipStreamGetDevice(A->v.stream, &dev) : hipGetDevice(&dev);
    unsigned long long *hist = nullptr;
    if (e == hipSuccess)
        e = pa_noalloc_scratch(dev, &hist);
    if (e == hipSuccess)
        e = settle_spins(B);
    if (e == hipSuccess)
        e = settle_spins(A);
    if (e == hipSuccess)
        e = hipStreamSynchronize(B->v.stream);
    if (e == hipSuccess) // the fill kernel clears the N + 1 counters this call uses
        e = pa_launch_overlap(A->ddesc, B->ddesc, N, A->v.ncol, hist, A->v.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hist_out, hist, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, A->v.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(A->v.stream);
    if (e != hipSuccess)
        return hip_fail(A, e, "pa_overlap_noalloc");
    return PA_OK;
}

pa_status pa_step_alpha(pa_ctx *c, double dbeta, double *alpha_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!alpha_out || !std::isfinite(dbeta) || dbeta < 0.0)
        return fail(b, PA_E_INVAL, "dbeta must be finite and >= 0; alpha_out non-NULL");
    pa_status u = need_uniform(b, "pa_step_alpha");
    if (u != PA_OK)
        return u;
    hipError_t e = pa_b_rule(b->v, 0.0, dbeta, 0, 0, b->hist_state);
    histogram_built(b);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_step_alpha");
    pa_status s = ctx_records(b, "pa_step_alpha");
    if (s != PA_OK)
        return s;
    *alpha_out = b->hrec[0].rule_alpha;
    return PA_OK;
}

pa_status pa_step_rule(pa_ctx *c, double alpha_star, double dbeta_max, int32_t iterations, double *dbeta_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!dbeta_out || !(alpha_star > 0.0 && alpha_star < 1.0) || !std::isfinite(dbeta_max) || dbeta_max <= 0.0 ||
        iterations < 1 || iterations > 200)
        return fail(b, PA_E_INVAL, "need 0 < alpha_star < 1, dbeta_max > 0, 1 <= iterations <= 200");
    pa_status u = need_uniform(b, "pa_step_rule");
    if (u != PA_OK)
        return u;
    hipError_t e = pa_b_rule(b->v, alpha_star, dbeta_max, iterations, 1, b->hist_state);
    histogram_built(b);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_step_rule");
    pa_status s = ctx_records(b, "pa_step_rule");
    if (s != PA_OK)
        return s;
    *dbeta_out = b->hrec[0].rule_dbeta;
    return PA_OK;
}

pa_status pa_get_counters(pa_ctx *c, pa_counters *out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!out)
        return fail(b, PA_E_INVAL, "out is NULL");
    pa_status s = ctx_records(b, "pa_get_counters");
    if (s != PA_OK)
        return s;
    out->philox_calls = b->hrec[0].philox_calls;
    out->site_updates = b->hrec[0].site_updates;
    out->sweeps = b->sweeps_total;
    out->spin_attempts = b->hrec[0].attempts;
    out->resamplings = b->hrec[0].resamplings;
    return PA_OK;
}

void pa_destroy(pa_ctx *c)
{
    if (!c)
        return;
    free_batch(&c->b);
    delete c;
}

const char *pa_last_error(const pa_ctx *c) { return c ? c->b.err.c_str() : g_init_err.c_str(); }

// ====================================================================== batches
pa_status pa_batch_required_bytes(const pa_config *cfgs, int32_t nruns, int32_t max_points, uint64_t *bytes)
{
    std::vector<Geometry> geo;
    std::string msg;
    pa_status s = check_batch(cfgs, nruns, max_points, &geo, &msg);
    if (s != PA_OK)
        return fail(nullptr, s, msg);
    if (!bytes)
        return fail(nullptr, PA_E_INVAL, "bytes is NULL");
    *bytes = layout(geo, max_points, nullptr, nullptr, nullptr);
    return PA_OK;
}

pa_status pa_batch_create(const pa_config *cfgs, int32_t nruns, int32_t max_points, void *workspace,
                          uint64_t workspace_bytes, void *stream, pa_batch **out)
{
    if (!out)
        return fail(nullptr, PA_E_INVAL, "out is NULL");
    *out = nullptr;
    pa_batch *p = new (std::nothrow) pa_batch;
    if (!p)
        return fail(nullptr, PA_E_NOMEM, "out of host memory");
    pa_status s = make_batch(cfgs, nruns, max_points, workspace, workspace_bytes, stream, &p->b);
    if (s != PA_OK) {
        delete p;
        return s;
    }
    *out = p;
    return PA_OK;
}

pa_status pa_batch_tune(pa_batch *p, int32_t theta, double beta, int32_t *threads_out, float *ms_out)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (theta < 1 || theta > 64)
        return fail(b, PA_E_INVAL, "theta must be in [1, 64]");
    if (!std::isfinite(beta) || beta < 0.0)
        return fail(b, PA_E_INVAL, "beta must be finite and >= 0");
    // Each candidate sweeps the current populations with the thresholds of
    // `beta`; the populations are re-initialised afterwards (initial sampling
    // is deterministic), so tuning leaves no trace.  Every candidate gives the
    // same bits by construction.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = settle_spins(b);
    if (e == hipSuccess)
        e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e == hipSuccess)
        e = pa_b_tune_beta(b->v, beta);
    for (int g = 0; g < b->v.ngroups && e == hipSuccess; ++g) {
        float best = 1e30f;
        int best_t = b->v.gthreads[g];
        for (int t = 64; t <= kSweepMaxLanes && e == hipSuccess; t += 64) {
            if (ms_out)
                ms_out[g * (kSweepMaxLanes / 64) + t / 64 - 1] = -1.0f;
            if (!sweep_threads_ok(b->v.gN[g], b->v.gd[g], t) ||
                pa_sweep_lds_bytes(b->v.gN[g], b->v.gd[g], t, b->v.gJ[g] != 0) > (size_t)g_max_lds)
                continue;
            e = pa_b_sweep_group(b->v, g, theta, t); // warm-up
            if (e == hipSuccess)
                e = hipEventRecord(e0, b->v.stream);
            if (e == hipSuccess)
                e = pa_b_sweep_group(b->v, g, theta, t);
            if (e == hipSuccess)
                e = hipEventRecord(e1, b->v.stream);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms_out)
                ms_out[g * (kSweepMaxLanes / 64) + t / 64 - 1] = ms;
            if (e == hipSuccess && ms < best) {
                best = ms;
                best_t = t;
            }
        }
        b->v.gthreads[g] = best_t;
        if (threads_out)
            threads_out[g] = best_t;
    }
    if (e == hipSuccess)
        e = launch_init(b);
    if (e == hipSuccess)
        e = hipStreamSynchronize(b->v.stream);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_batch_tune");
    return PA_OK;
}

pa_status pa_batch_set_threads(pa_batch *p, int32_t group, int32_t threads)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (group < 0 || group >= b->v.ngroups)
        return fail(b, PA_E_INVAL, "no such group");
    if (!sweep_threads_ok(b->v.gN[group], b->v.gd[group], threads) ||
        pa_sweep_lds_bytes(b->v.gN[group], b->v.gd[group], threads, b->v.gJ[group] != 0) > (size_t)g_max_lds)
        return fail(b, PA_E_INVAL, "workgroup size not usable for this group (64..768 lanes in steps of 64, "
                                   "within the LDS and the per-lane site bound)");
    // the size decides which kernel gathers a resampling's spins: none may be
    // left for the next sweep across the change
    const hipError_t e = settle_spins(b);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_batch_set_threads");
    b->v.gthreads[group] = threads;
    return PA_OK;
}

pa_status pa_batch_groups(pa_batch *p, int32_t *ngroups, int32_t *threads)
{
    if (!p || !ngroups)
        return fail(p ? &p->b : nullptr, PA_E_INVAL, "NULL argument");
    *ngroups = p->b.v.ngroups;
    if (threads)
        for (int g = 0; g < p->b.v.ngroups; ++g)
            threads[g] = p->b.v.gthreads[g];
    return PA_OK;
}

pa_status pa_batch_anneal(pa_batch *p, const double *betas, int32_t npoints, int32_t theta, pa_resampler scheme,
                          int32_t use_graph)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (!betas || npoints < 1 || npoints > b->max_points)
        return fail(b, PA_E_INVAL, "need 1 <= npoints <= max_points of pa_batch_create");
    if (betas[0] != 0.0)
        return fail(b, PA_E_INVAL, "the anneal starts at beta_0 = 0");
    for (int i = 1; i < npoints; ++i)
        if (!std::isfinite(betas[i]) || betas[i] < betas[i - 1])
            return fail(b, PA_E_INVAL, "betas must be finite and non-decreasing");
    if (theta < 0 || theta > (1 << 20))
        return fail(b, PA_E_INVAL, "theta out of range");
    if ((int)scheme < 0 || (int)scheme > 3)
        return fail(b, PA_E_INVAL, "unknown resampling scheme");
    const hipStream_t st = b->v.stream;
    const std::vector<double> sched(betas, betas + npoints);
    const std::vector<int> threads(b->v.gthreads, b->v.gthreads + b->v.ngroups);
    hipError_t e = hipSuccess;
    if (use_graph && b->anneal_exec && b->anneal_betas == sched && b->anneal_theta == theta &&
        b->anneal_scheme == (int)scheme && b->anneal_threads == threads) {
        // the same anneal as the captured one: replay it (every kernel's
        // arguments, the block maps and the workspace are unchanged; the
        // anneal starts with the initial sampling, so no earlier state enters)
        e = hipGraphLaunch(b->anneal_exec, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return hip_fail(b, e, "pa_batch_anneal (replay)");
        b->hist_state = b->anneal_end_hist; // as the captured anneal left the bookkeeping
        b->rs_prepped = b->anneal_end_rs;
        b->gather_pending = b->anneal_end_gather;
        b->anneal_points = npoints;
        return PA_OK;
    }
    if (use_graph)
        drop_anneal_graph(b);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (use_graph)
        e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess)
        e = launch_init(b);
    if (e == hipSuccess)
        e = launch_observables(b, 0);
    for (int i = 1; i < npoints && e == hipSuccess; ++i) {
        e = launch_reweight(b, betas[i]);
        if (e == hipSuccess)
            e = launch_resample(b, (int)scheme, 1, -1);
        if (e == hipSuccess && theta > 0)
            e = launch_updates(b, theta, 0u, 0); // every run was just resampled
        if (e == hipSuccess)
            e = launch_observables(b, i);
    }
    if (use_graph) {
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (e == hipSuccess)
            e = e2;
        if (e == hipSuccess)
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess)
            e = hipGraphLaunch(exec, st);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (graph)
        (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        return hip_fail(b, e, "pa_batch_anneal");
    }
    if (exec) { // kept for replays of the same anneal
        b->anneal_end_hist = b->hist_state;
        b->anneal_end_rs = b->rs_prepped;
        b->anneal_end_gather = b->gather_pending;
        b->anneal_exec = exec;
        b->anneal_betas = sched;
        b->anneal_theta = theta;
        b->anneal_scheme = (int)scheme;
        b->anneal_threads = threads;
    }
    b->anneal_points = npoints;
    return PA_OK;
}

pa_status pa_batch_records(pa_batch *p, pa_step_record *out)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (!out || b->anneal_points == 0)
        return fail(b, PA_E_STATE, "no anneal recorded");
    static_assert(sizeof(pa_step_record) == sizeof(PaStepRecord), "record layout");
    std::vector<PaStepRecord> all((size_t)b->M * b->max_points);
    hipError_t e = hipMemcpy(all.data(), b->v.steprec, all.size() * sizeof(PaStepRecord), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_batch_records");
    for (int m = 0; m < b->M; ++m)
        std::memcpy(out + (size_t)m * b->anneal_points, all.data() + (size_t)m * b->max_points,
                    sizeof(PaStepRecord) * (size_t)b->anneal_points);
    return PA_OK;
}

pa_status pa_batch_export_run(pa_batch *p, int32_t run, pa_host_state *st)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (!st || run < 0 || run >= b->M)
        return fail(b, PA_E_INVAL, "bad run index or NULL state");
    return export_run(b, run, st);
}

pa_status pa_batch_overlap(pa_batch *p, int32_t run_a, int32_t run_b, int64_t *hist_out)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (!hist_out || run_a < 0 || run_a >= b->M || run_b < 0 || run_b >= b->M)
        return fail(b, PA_E_INVAL, "bad run index or NULL hist_out");
    const PaRunDesc &da = b->hdesc[run_a], &db = b->hdesc[run_b];
    if (da.d != db.d || da.L != db.L)
        return fail(b, PA_E_INVAL, "runs on different lattices");
    const int N = da.N;
    hipError_t e = settle_spins(b);
    if (e == hipSuccess)
        e = pa_launch_overlap(b->ddesc + run_a, b->ddesc + run_b, N, (uint32_t)b->geo[run_a].W, da.dv.qhist,
                              b->v.stream);
    std::vector<unsigned long long> h((size_t)N + 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), da.dv.qhist, h.size() * 8, hipMemcpyDeviceToHost, b->v.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(b->v.stream);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_batch_overlap");
    for (int k = 0; k <= N; ++k)
        hist_out[k] = (int64_t)h[(size_t)k];
    return PA_OK;
}

pa_status pa_batch_combine(pa_batch *p, const int32_t *group_of_run, int32_t ngroups, int32_t point,
                           pa_combined *out)
{
    if (!p)
        return fail(nullptr, PA_E_INVAL, "batch is NULL");
    Batch *b = &p->b;
    if (!group_of_run || !out || ngroups < 1 || ngroups > b->M)
        return fail(b, PA_E_INVAL, "need group_of_run, out and 1 <= ngroups <= nruns");
    if (b->anneal_points == 0 || point < 0 || point >= b->anneal_points)
        return fail(b, PA_E_INVAL, "point outside the recorded anneal");
    std::vector<int32_t> Ns(b->M);
    for (int m = 0; m < b->M; ++m) {
        if (group_of_run[m] < -1 || group_of_run[m] >= ngroups)
            return fail(b, PA_E_INVAL, "group index out of range (-1 = no group)");
        Ns[m] = b->hdesc[m].N;
    }
    PaBatchView v = b->v;
    v.npoints = b->max_points;
    hipError_t e = hipMemcpyAsync(b->dgroup, group_of_run, 4ull * b->M, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dNs, Ns.data(), 4ull * b->M, hipMemcpyHostToDevice, v.stream);
    if (e == hipSuccess)
        e = pa_launch_combine(v, point, b->dgroup, ngroups, b->dNs, b->dcomb);
    std::vector<double> h((size_t)ngroups * PA_COMBINE_FIELDS);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), b->dcomb, h.size() * 8, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(v.stream);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_batch_combine");
    for (int g = 0; g < ngroups; ++g) {
        const double *o = h.data() + (size_t)g * PA_COMBINE_FIELDS;
        out[g].lnZ = o[0];
        out[g].e = o[1];
        out[g].e2 = o[2];
        out[g].abs_m = o[3];
        out[g].m2 = o[4];
        out[g].c = o[5];
        out[g].chi = o[6];
        out[g].n_eff = o[7];
        out[g].runs = (int32_t)o[8];
        out[g].beta = o[9];
        out[g].c_naive = o[10];
        out[g].chi_naive = o[11];
        out[g].e_plain = o[12];
        out[g].c_plain = o[13];
        out[g].chi_plain = o[14];
    }
    return PA_OK;
}

void pa_batch_destroy(pa_batch *p)
{
    if (!p)
        return;
    free_batch(&p->b);
    delete p;
}

const char *pa_batch_last_error(const pa_batch *p) { return p ? p->b.err.c_str() : g_init_err.c_str(); }

// ====================================================================== learned step
static uint64_t mlp_layout(int max_samples, char *base, PaMlpDev *d)
{
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += round256(bytes);
        return p;
    };
    const uint64_t n = (uint64_t)max_samples, h = PA_MLP_HIDDEN;
    PaMlpDev m{};
    m.P = (float *)take(4ull * PA_MLP_PARAMS);
    m.M = (float *)take(4ull * PA_MLP_PARAMS);
    m.V = (float *)take(4ull * PA_MLP_PARAMS);
    m.G = (float *)take(4ull * PA_MLP_PARAMS);
    m.norm = (PaMlpNorm *)take(sizeof(PaMlpNorm));
    m.X = (float *)take(4 * n * 8);
    m.Y = (float *)take(4 * n);
    m.Xn = (float *)take(4 * n * 8);
    m.H1 = (float *)take(4 * n * h);
    m.H2 = (float *)take(4 * n * h);
    m.D1 = (float *)take(4 * n * h);
    m.D2 = (float *)take(4 * n * h);
    m.dY = (float *)take(4 * n);
    m.r2 = (float *)take(4 * n);
    m.loss = (double *)take(8);
    m.pred = (float *)take(4 * n);
    if (d)
        *d = m;
    return off;
}

static pa_status mfail(pa_mlp *m, pa_status s, const std::string &msg)
{
    if (m)
        m->err = msg;
    else
        g_init_err = msg;
    return s;
}

pa_status pa_mlp_required_bytes(int32_t max_samples, uint64_t *bytes)
{
    if (max_samples < 1 || max_samples > (1 << 22) || !bytes)
        return mfail(nullptr, PA_E_INVAL, "need 1 <= max_samples <= 2^22 and bytes");
    *bytes = mlp_layout(max_samples, nullptr, nullptr);
    return PA_OK;
}

pa_status pa_mlp_create(int32_t max_samples, const float *params, const pa_mlp_norm *norm, void *workspace,
                        uint64_t bytes, void *stream, pa_mlp **out)
{
    if (!out)
        return mfail(nullptr, PA_E_INVAL, "out is NULL");
    *out = nullptr;
    if (max_samples < 1 || max_samples > (1 << 22) || !params || !norm)
        return mfail(nullptr, PA_E_INVAL, "need 1 <= max_samples <= 2^22, params and norm");
    for (int k = 0; k < 8; ++k)
        if (!(norm->x_std[k] > 0.0f) || !std::isfinite(norm->x_mean[k]))
            return mfail(nullptr, PA_E_INVAL, "feature scales must be positive and finite");
    if (!(norm->y_std > 0.0f) || !std::isfinite(norm->y_mean))
        return mfail(nullptr, PA_E_INVAL, "target scale must be positive and finite");
    if (!workspace || bytes < mlp_layout(max_samples, nullptr, nullptr) || ((uintptr_t)workspace & 255u))
        return mfail(nullptr, PA_E_INVAL, "workspace missing, too small or not 256-byte aligned");
    pa_mlp *m = new (std::nothrow) pa_mlp;
    if (!m)
        return mfail(nullptr, PA_E_NOMEM, "out of host memory");
    mlp_layout(max_samples, (char *)workspace, &m->d);
    m->d.stream = (hipStream_t)stream;
    m->max_samples = max_samples;
    static_assert(sizeof(pa_mlp_norm) == sizeof(PaMlpNorm), "norm layout");
    std::vector<float> zeros(PA_MLP_PARAMS, 0.0f);
    hipError_t e = hipMemcpyAsync(m->d.P, params, 4ull * PA_MLP_PARAMS, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d.M, zeros.data(), 4ull * PA_MLP_PARAMS, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d.V, zeros.data(), 4ull * PA_MLP_PARAMS, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d.norm, norm, sizeof(PaMlpNorm), hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess) {
        delete m;
        return mfail(nullptr, PA_E_DEVICE, std::string("pa_mlp_create: ") + hipGetErrorString(e));
    }
    *out = m;
    return PA_OK;
}

pa_status pa_mlp_set_data(pa_mlp *m, const float *X, const float *y, int32_t n)
{
    if (!m)
        return mfail(nullptr, PA_E_INVAL, "model is NULL");
    if (!X || !y || n < 1 || n > m->max_samples)
        return mfail(m, PA_E_INVAL, "need X, y and 1 <= n <= max_samples");
    hipError_t e = hipMemcpyAsync(m->d.X, X, 4ull * 8 * n, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d.Y, y, 4ull * n, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess)
        return mfail(m, PA_E_DEVICE, std::string("pa_mlp_set_data: ") + hipGetErrorString(e));
    m->n = n;
    return PA_OK;
}

pa_status pa_mlp_gradient(pa_mlp *m, float *grad_out, double *loss_out)
{
    if (!m)
        return mfail(nullptr, PA_E_INVAL, "model is NULL");
    if (m->n == 0)
        return mfail(m, PA_E_STATE, "no training data set");
    hipError_t e = pa_mlp_launch_grad(m->d, m->n, 0, 1, 0.0f);
    if (e == hipSuccess && grad_out)
        e = hipMemcpyAsync(grad_out, m->d.G, 4ull * PA_MLP_PARAMS, hipMemcpyDeviceToHost, m->d.stream);
    if (e == hipSuccess && loss_out)
        e = hipMemcpyAsync(loss_out, m->d.loss, 8, hipMemcpyDeviceToHost, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess)
        return mfail(m, PA_E_DEVICE, std::string("pa_mlp_gradient: ") + hipGetErrorString(e));
    return PA_OK;
}

pa_status pa_mlp_train(pa_mlp *m, int32_t epochs, float lr, double *loss_out)
{
    if (!m)
        return mfail(nullptr, PA_E_INVAL, "model is NULL");
    if (m->n == 0)
        return mfail(m, PA_E_STATE, "no training data set");
    if (epochs < 1 || !(lr > 0.0f))
        return mfail(m, PA_E_INVAL, "need epochs >= 1 and lr > 0");
    hipError_t e = hipSuccess;
    for (int k = 0; k < epochs && e == hipSuccess; ++k)
        e = pa_mlp_launch_grad(m->d, m->n, 1, ++m->t, lr);
    // the loss after the last update
    if (e == hipSuccess && loss_out)
        e = pa_mlp_launch_grad(m->d, m->n, 0, 1, 0.0f);
    if (e == hipSuccess && loss_out)
        e = hipMemcpyAsync(loss_out, m->d.loss, 8, hipMemcpyDeviceToHost, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess)
        return mfail(m, PA_E_DEVICE, std::string("pa_mlp_train: ") + hipGetErrorString(e));
    return PA_OK;
}

pa_status pa_mlp_params(pa_mlp *m, float *out)
{
    if (!m || !out)
        return mfail(m, PA_E_INVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(out, m->d.P, 4ull * PA_MLP_PARAMS, hipMemcpyDeviceToHost, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess)
        return mfail(m, PA_E_DEVICE, std::string("pa_mlp_params: ") + hipGetErrorString(e));
    return PA_OK;
}

pa_status pa_mlp_predict(pa_mlp *m, const float *X, int32_t n, float *dbeta_out)
{
    if (!m)
        return mfail(nullptr, PA_E_INVAL, "model is NULL");
    if (!X || !dbeta_out || n < 1 || n > m->max_samples)
        return mfail(m, PA_E_INVAL, "need X, out and 1 <= n <= max_samples");
    // the data slot holds the inputs; a later pa_mlp_set_data is needed to train again
    hipError_t e = hipMemcpyAsync(m->d.X, X, 4ull * 8 * n, hipMemcpyHostToDevice, m->d.stream);
    if (e == hipSuccess)
        e = pa_mlp_launch_predict(m->d, m->d.X, n, m->d.pred);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dbeta_out, m->d.pred, 4ull * n, hipMemcpyDeviceToHost, m->d.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(m->d.stream);
    if (e != hipSuccess)
        return mfail(m, PA_E_DEVICE, std::string("pa_mlp_predict: ") + hipGetErrorString(e));
    m->n = 0;
    return PA_OK;
}

pa_status pa_features(pa_ctx *c, float *out8)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!out8)
        return fail(b, PA_E_INVAL, "out is NULL");
    pa_status u = need_uniform(b, "pa_features");
    if (u != PA_OK)
        return u;
    hipError_t e = pa_b_features(b->v, b->hist_state);
    histogram_built(b);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_features");
    pa_status s = ctx_records(b, "pa_features");
    if (s != PA_OK)
        return s;
    std::memcpy(out8, b->hrec[0].feat, sizeof(float) * 8);
    return PA_OK;
}

pa_status pa_step_learned(pa_ctx *c, pa_mlp *m, double alpha_star, double dbeta_max, int32_t iterations,
                          double bracket, int32_t refine, double *dbeta_out, int32_t *fallback_out,
                          double *proposal_out)
{
    if (!c)
        return fail(nullptr, PA_E_INVAL, "ctx is NULL");
    Batch *b = &c->b;
    if (!m || !dbeta_out || !(alpha_star > 0.0 && alpha_star < 1.0) || !std::isfinite(dbeta_max) ||
        dbeta_max <= 0.0 || iterations < 1 || iterations > 200 || !std::isfinite(bracket) || bracket < 1.0 ||
        refine < 0 || refine > 64)
        return fail(b, PA_E_INVAL, "need a model, 0 < alpha_star < 1, dbeta_max > 0, 1 <= iterations <= 200, "
                                   "bracket >= 1, 0 <= refine <= 64");
    pa_status u = need_uniform(b, "pa_step_learned");
    if (u != PA_OK)
        return u;
    if (m->d.stream != b->v.stream) {
        hipError_t e = hipStreamSynchronize(m->d.stream);
        if (e != hipSuccess)
            return hip_fail(b, e, "pa_step_learned");
    }
    hipError_t e = pa_b_features(b->v, b->hist_state);
    histogram_built(b);
    if (e == hipSuccess)
        e = pa_mlp_launch_propose(b->v, m->d, dbeta_max);
    if (e == hipSuccess)
        e = pa_b_check_candidate(b->v, alpha_star, dbeta_max, iterations, bracket, refine);
    if (e != hipSuccess)
        return hip_fail(b, e, "pa_step_learned");
    pa_status s = ctx_records(b, "pa_step_learned");
    if (s != PA_OK)
        return s;
    *dbeta_out = b->hrec[0].rule_dbeta;
    if (fallback_out)
        *fallback_out = (int32_t)b->hrec[0].fallback;
    if (proposal_out)
        *proposal_out = b->hrec[0].cand_dbeta;
    return PA_OK;
}

void pa_mlp_destroy(pa_mlp *m) { delete m; }

const char *pa_mlp_last_error(const pa_mlp *m) { return m ? m->err.c_str() : g_init_err.c_str(); }

} // extern "C"
