// smc_host.cpp -- host driver of libsmc: validation, device memory, tile choice,
// the stage loop and the C ABI declared in include/smc.h.
//
// Per tempering stage the host issues two launches for every group at once
// (k_stage: one workgroup per group; k_move: every chain of every group) and
// reads back the groups' small state blocks to learn which K have finished.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "host_common.hpp"

namespace smc {

// ------------------------------------------------------------------ kernel table

static KernelTable g_table;
static std::once_flag g_table_once;

const KernelTable& kernels() {
    std::call_once(g_table_once, [] {
        std::memset(&g_table, 0, sizeof(g_table));
        register_kernels_00(g_table);
        register_kernels_01(g_table);
        register_kernels_10(g_table);
        register_kernels_11(g_table);
        register_kernels_xps(g_table);
        register_kernels_xrd(g_table);
    });
    return g_table;
}

// ------------------------------------------------------------------ validation

static bool prior_ok(const smc_prior& p) {
    if (!std::isfinite(p.a) || !std::isfinite(p.b)) return false;
    switch (p.kind) {
    case SMC_PRIOR_UNIFORM: return p.a < p.b;
    case SMC_PRIOR_GAMMA: return p.a > 0.0 && p.b > 0.0;
    case SMC_PRIOR_NORMAL: return p.b > 0.0;
    case SMC_PRIOR_FIXED: return true;
    default: return false;
    }
}

int params_per_peak(int peak_kind) { return peak_kind == SMC_PEAK_GAUSS ? 3 : (peak_kind == SMC_PEAK_PVOIGT ? 4 : 9); }
int params_bg(int bg_kind) {
    return bg_kind == SMC_BG_NONE ? 0 : (bg_kind == SMC_BG_CONST ? 1 : (bg_kind == SMC_BG_XRD ? 4 : 2));
}

smc_prior component_prior(const smc_problem& p, int K, int j) {
    const int np = params_per_peak(p.peak_kind);
    if (j < K * np) {
        const int k = j / np, q = j % np;
        return p.peak_prior_k ? p.peak_prior_k[k * SMC_MAX_PEAK_PARAMS + q] : p.peak_prior[q];
    }
    return p.bg_prior[j - K * np];
}

smc_status validate(const smc_problem* p, const smc_options* o) {
    if (!p || !o) return SMC_EINVAL;
    if (p->n_points < 1 || !p->x || !p->y) return SMC_EINVAL;
    if (p->peak_kind < SMC_PEAK_GAUSS || p->peak_kind > SMC_PEAK_XRD) return SMC_EINVAL;
    if (p->bg_kind < SMC_BG_NONE || p->bg_kind > SMC_BG_XRD) return SMC_EINVAL;
    if ((p->peak_kind == SMC_PEAK_XRD) != (p->bg_kind == SMC_BG_XRD)) return SMC_EINVAL;
    if (p->peak_kind == SMC_PEAK_XRD) {
        // the XRD powder profile: Poisson counts, reference positions, 0 < 2theta < 180
        if (p->noise_kind != SMC_NOISE_POISSON || !p->mu_ref || p->n_points > kMaxXrdPoints) return SMC_EINVAL;
        for (int k = 0; k < p->k_max; ++k)
            if (!std::isfinite(p->mu_ref[k])) return SMC_EINVAL;
        for (int i = 0; i < p->n_points; ++i)
            if (!(p->x[i] > 0.0 && p->x[i] < 180.0)) return SMC_EINVAL;
    }
    if (p->noise_kind < SMC_NOISE_GAUSS || p->noise_kind > SMC_NOISE_HETERO) return SMC_EINVAL;
    if (p->peak_kind != SMC_PEAK_XRD && p->n_points > kMaxPoints) return SMC_EINVAL;
    if (p->noise_kind == SMC_NOISE_GAUSS && !(p->sigma > 0.0 && std::isfinite(p->sigma))) return SMC_EINVAL;
    if (xps_model(*p)) {
        // the XPS model form: pseudo-Voigt peaks, Shirley background, heteroscedastic noise
        if (p->bg_kind != SMC_BG_SHIRLEY || p->noise_kind != SMC_NOISE_HETERO || p->peak_kind != SMC_PEAK_PVOIGT)
            return SMC_EINVAL;
        if (p->n_points < 2 || p->n_points > kMaxXpsPoints) return SMC_EINVAL;
        for (int i = 1; i < p->n_points; ++i)
            if (!(static_cast<float>(p->x[i]) > static_cast<float>(p->x[i - 1]))) return SMC_EINVAL;
        double ssum = 0.0;
        for (double v : p->noise_s) {
            if (!(v >= 0.0 && std::isfinite(v))) return SMC_EINVAL;
            ssum += v;
        }
        if (!(ssum > 0.0)) return SMC_EINVAL;
    }
    if (p->k_min < 1 || p->k_min > p->k_max || p->k_max > kMaxK) return SMC_EINVAL;
    for (int i = 0; i < p->n_points; ++i) {
        if (!std::isfinite(p->x[i]) || !std::isfinite(p->y[i])) return SMC_EINVAL;
        if (p->noise_kind == SMC_NOISE_POISSON && p->y[i] < 0.0) return SMC_EINVAL;
    }
    const int np = params_per_peak(p->peak_kind);
    for (int q = 0; q < np; ++q)
        if (!p->peak_prior_k && !prior_ok(p->peak_prior[q])) return SMC_EINVAL;
    if (p->peak_prior_k)
        for (int k = 0; k < p->k_max; ++k)
            for (int q = 0; q < np; ++q)
                if (!prior_ok(p->peak_prior_k[k * SMC_MAX_PEAK_PARAMS + q])) return SMC_EINVAL;
    for (int q = 0; q < params_bg(p->bg_kind); ++q)
        if (!prior_ok(p->bg_prior[q])) return SMC_EINVAL;
    if (o->n_particles < 2 || o->n_moves < 1) return SMC_EINVAL;
    if (o->waste_free && (o->n_particles % o->n_moves) != 0) return SMC_EINVAL;
    // device tables index component-major particle arrays with 32-bit offsets
    const int64_t dmax = static_cast<int64_t>(p->k_max) * np + params_bg(p->bg_kind);
    if (dmax * o->n_particles > INT32_MAX) return SMC_EINVAL;
    if (!(o->ess_frac > 0.0 && o->ess_frac < 1.0)) return SMC_EINVAL;
    if (o->bisect_iters < 1 || o->bisect_iters > 200 || o->max_stages < 1) return SMC_EINVAL;
    if (o->lanes_per_chain != 0 && o->lanes_per_chain != 16 && o->lanes_per_chain != 32 &&
        o->lanes_per_chain != 64 && o->lanes_per_chain != 128 && o->lanes_per_chain != 256 &&
        o->lanes_per_chain != 512)
        return SMC_EINVAL;
    if ((o->lanes_per_chain == 128 || o->lanes_per_chain == 512) && p->peak_kind != SMC_PEAK_XRD) return SMC_EINVAL;
    return SMC_OK;
}

bool xps_model(const smc_problem& p) { return p.bg_kind == SMC_BG_SHIRLEY || p.noise_kind == SMC_NOISE_HETERO; }

double energy_constant(const smc_problem& p) {
    if (p.noise_kind == SMC_NOISE_GAUSS)
        return 0.5 * p.n_points * std::log(2.0 * M_PI * p.sigma * p.sigma);
    if (p.noise_kind == SMC_NOISE_HETERO) return 0.5 * p.n_points * std::log(2.0 * M_PI);
    double c = 0.0;
    for (int i = 0; i < p.n_points; ++i) {
        const double y = static_cast<float>(p.y[i]);
        c += y + std::lgamma(y + 1.0) - (y > 0.0 ? y * std::log(y) : 0.0);
    }
    return c;
}

DevPrior dev_prior(const smc_prior& p) {
    DevPrior d;
    d.kind = p.kind;
    d.a = static_cast<float>(p.a);
    d.b = static_cast<float>(p.b);
    d.c = 0.0f;
    d.lo = d.a;
    d.hi = d.a;
    if (p.kind == SMC_PRIOR_UNIFORM) d.hi = d.b;
    if (p.kind == SMC_PRIOR_GAMMA) {
        d.c = static_cast<float>(p.a - 1.0);
        d.lo = 0.0f;
        d.hi = __builtin_inff();
    }
    if (p.kind == SMC_PRIOR_NORMAL) {
        d.c = static_cast<float>(1.0 / (2.0 * p.b * p.b));
        d.lo = -__builtin_inff();
        d.hi = __builtin_inff();
    }
    return d;
}

// ------------------------------------------------------------------ tile choice

// Deterministic tile rule, a function of the group shape only (N and the chain
// count of the launch): the smallest lane count whose points fit the register
// budget (<= 32 points per lane) and that still gives >= 2 waves per SIMD
// (2048 waves on 256 CUs); otherwise the largest lane count that fits.
Tile choose_tile(const smc_problem& p, int64_t chains, int forced_lanes) {
    const int n_points = p.n_points;
    Tile t{};
    if (xps_model(p)) {
        // one wavefront per chain group, at most 16 points per lane (the Shirley scan runs
        // across the lanes of one wavefront)
        int best = -1;
        for (int li = 0; li < kNumLaneCfg; ++li) {
            const int lc = kLaneOrder[li], lanes = kLanesOf[lc];
            if (lanes > 64 || (forced_lanes && lanes != forced_lanes)) continue;
            if ((n_points + lanes - 1) / lanes > 16) continue;
            if (!forced_lanes && best >= 0 && kLanesOf[best] >= n_points) break;
            best = lc;
            if (chains * lanes / 64 >= 2048) break;
        }
        if (best < 0) return t;
        const int rows = (n_points + kLanesOf[best] - 1) / kLanesOf[best];
        int pi = 0;
        while (kPplOf[pi] < rows) ++pi;
        if (n_points <= ppl_before(kPplOf[pi]) * kLanesOf[best]) return t;
        return Tile{best, pi, kLanesOf[best], kPplOf[pi], true};
    }
    // Preference: chains inside one wavefront with at most 16 points per lane (the move
    // kernel keeps 4+ waves per SIMD there), then up to 32 points per lane (2-3 waves),
    // then four or eight wavefronts per chain (a cross-wave LDS reduction per proposal).
    // Within a class the smallest lane count that still gives 2048 wavefronts, never more
    // lanes than points beyond the smallest configuration; only configurations the model
    // family has kernels for.
    // The XRD profile holds more per point (tan, y and two shapes) and its move kernel needs
    // several waves per SIMD to hide its transcendental latency: one-wavefront chains only
    // up to 8 points per lane (3+ waves), then 128 lanes up to 8 points per lane, then 256 or
    // 512 lanes (whole runs at P = 250000: N = 1000 216 ms at 128 x 8 against 242 at 256 x 4
    // and 251 at 64 x 16; N = 600 130 ms at 128 x 5 against 172 at 256 x 3 and 133 at 64 x 10;
    // N = 1500, 2000 and 2560 6-16% slower at 128 lanes than at 256).
    const bool xrd = p.peak_kind == SMC_PEAK_XRD;
    const int max_rows = xrd ? 20 : kPplOf[kNumPpl - 1];
    const int row_limits[3] = {xrd ? 8 : 16, xrd ? 8 : max_rows, max_rows};
    int best = -1;
    for (int cls = 0; cls < 3 && best < 0; ++cls) {
        for (int li = 0; li < kNumLaneCfg; ++li) {
            const int lc = kLaneOrder[li], lanes = kLanesOf[lc];
            if (forced_lanes ? lanes != forced_lanes : ((cls < 2) != (lanes <= 64))) continue;
            if (!kernels().move[p.peak_kind][p.noise_kind][lc][0]) continue;
            const int rows = (n_points + lanes - 1) / lanes;
            if (rows > (forced_lanes ? max_rows : row_limits[cls])) continue;
            if (!forced_lanes && lanes == 128 && rows > 8) continue;
            if (!forced_lanes && best >= 0 && kLanesOf[best] >= n_points) break;
            best = lc;
            if (chains * lanes / 64 >= 2048) break;
        }
    }
    if (best < 0) return t;  // the lane count cannot hold N points in the register budget
    const int lanes = kLanesOf[best];
    const int rows = (n_points + lanes - 1) / lanes;
    int pi = 0;
    while (kPplOf[pi] < rows) ++pi;
    // the kernels take the rows before ppl_before(PPL) as free of padding
    if (n_points <= ppl_before(kPplOf[pi]) * lanes) return t;
    t.lc = best;
    t.pi = pi;
    t.lanes = lanes;
    t.ppl = kPplOf[pi];
    t.valid = true;
    return t;
}

bool tile_has_kernels(const smc_problem& p, const Tile& t) {
    return t.valid && kernels().move[p.peak_kind][p.noise_kind][t.lc][t.pi] &&
           kernels().energy[p.peak_kind][p.noise_kind][t.lc][t.pi];
}

// Cross-wave reduction slots (two per wavefront of a chain, double-buffered) and the
// two evaluation counters.
static size_t reduce_floats(const Tile& t) { return 2 * static_cast<size_t>(t.lanes > 64 ? t.lanes / 64 : 1) + 2; }

size_t move_lds_bytes(const Tile& t, int d, int peak_kind, int noise_kind) {
    const int cpw = tile_chains_per_wg(t);
    size_t b = sizeof(DevPrior) * d + sizeof(float) * (static_cast<size_t>(cpw) * 4 * d + reduce_floats(t));
    const int sb = move_shape_lds_bytes(peak_kind, noise_kind, t.ppl, t.lanes);
    if (sb > 0) b = ((b + 7) & ~static_cast<size_t>(7)) + static_cast<size_t>(sb) * tile_threads(t) * t.ppl;
    const int ib = move_iw_lds_bytes(peak_kind, t.ppl, t.lanes);
    if (ib > 0) b = ((b + 7) & ~static_cast<size_t>(7)) + static_cast<size_t>(ib) * tile_threads(t) * t.ppl;
    return b;
}

size_t energy_lds_bytes(const Tile& t, int d) {
    const int cpw = tile_chains_per_wg(t);
    return sizeof(float) * (static_cast<size_t>(cpw) * d + reduce_floats(t));
}

// Work items: groups in the given order, each split into workgroups of
// tile_chains_per_wg chains.
void build_work(const std::vector<int>& groups, const std::vector<int>& chains_of, const Tile& t,
                std::vector<MoveWork>& out) {
    const int cpw = tile_chains_per_wg(t);
    for (int g : groups) {
        const int nc = chains_of[g];
        for (int c0 = 0; c0 < nc; c0 += cpw) out.push_back(MoveWork{g, c0, std::min(cpw, nc - c0), 0});
    }
}

hipError_t launch_tiled(const void* fn, const Tile& t, int n_work, size_t lds, const GroupDesc* groups,
                        const MoveWork* work, hipStream_t s) {
    if (n_work <= 0) return hipSuccess;
    void* args[] = {&groups, &work};
    return hipLaunchKernel(fn, dim3(static_cast<unsigned>(n_work)), dim3(static_cast<unsigned>(tile_threads(t))), args,
                           lds, s);
}

// ------------------------------------------------------------------ device arena

void* Arena::take(size_t bytes) {
    const size_t off = (used + 255) & ~static_cast<size_t>(255);
    if (off + bytes > size) return nullptr;
    used = off + bytes;
    return static_cast<char*>(base) + off;
}

}  // namespace smc

using namespace smc;

// ------------------------------------------------------------------ context

// Stages that smc_run puts into the stream between two reads of the group states.
constexpr int kStagesPerRead = 4;

struct smc_ctx {
    Spectrum spec;                   // owned copy of the problem
    smc_options opt{};
    int kmin = 0, kmax = 0, ng = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* dmem = nullptr;
    Arena arena;
    GroupDesc* d_groups = nullptr;
    MoveWork* d_work = nullptr;
    MoveWork* d_init_work = nullptr;
    GroupState* d_states = nullptr;
    std::vector<GroupDesc> groups;   // host copies (device pointers inside)
    std::vector<GroupState> states;  // host mirror
    Tile tile{};
    int n_work = 0, n_init_work = 0;
    std::vector<int> work_off, work_cnt;  // per group: its range of move work items
    size_t lds_move = 0, lds_energy = 0;
    double econst = 0.0;
    bool finished = false;
    uint64_t stage0_evals = 0;
    // optional HIP-event timing of the launches: one (start, end) pair per move launch
    // (ev[2b], ev[2b + 1]) and per stage launch (ev[2 kStagesPerRead + 2b], ...) between
    // two reads of the group states
    hipEvent_t ev[4 * kStagesPerRead] = {};
    int n_ev_move = 0, n_ev_stage = 0;
    double move_ms = 0.0, stage_ms = 0.0;
    int64_t move_launches = 0, stage_launches = 0;
};

extern "C" void smc_default_options(smc_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_particles = 4096;
    o->n_moves = 16;
    o->waste_free = 1;
    o->bisect_iters = 50;
    o->max_stages = 1000;
    o->ess_frac = 0.5;
    o->seed = 0;
}

extern "C" int32_t smc_dim(const smc_problem* p, int32_t K) {
    if (!p || K < 0) return -1;
    return K * params_per_peak(p->peak_kind) + params_bg(p->bg_kind);
}

extern "C" smc_status smc_energy_constant(const smc_problem* p, double* c) {
    if (!p || !c || p->n_points < 1 || !p->y) return SMC_EINVAL;
    *c = energy_constant(*p);
    return SMC_OK;
}

extern "C" const char* smc_strerror(smc_status s) {
    switch (s) {
    case SMC_OK: return "success";
    case SMC_EINVAL: return "invalid argument";
    case SMC_ENOMEM: return "out of memory";
    case SMC_EDEVICE: return "HIP device error (or no gfx950 device)";
    case SMC_ENUMERIC: return "numerical failure (NaN energy, all energies infinite, or stage cap reached)";
    case SMC_ESTATE: return "invalid state for this call";
    case SMC_EBUDGET: return "request exceeds the memory budget";
    case SMC_EAGAIN: return "not ready";
    default: return "unknown status";
    }
}

static smc_status ctx_fail(smc_ctx* c, smc_status s) {
    smc_free(c);
    return s;
}

// Describe and allocate the groups of one spectrum (used by smc_init and the batch / server paths).
namespace smc {

size_t group_bytes(int d, int P, int M, int max_stages) {
    auto al = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    const size_t dd = std::max(d, 1);
    return al(sizeof(float) * dd * P) + al(sizeof(float) * P) + al(sizeof(float) * dd * M) + al(sizeof(float) * M) +
           al(sizeof(unsigned long long) * P) + al(sizeof(double) * dd) + al(sizeof(float) * dd) +
           al(sizeof(uint32_t) * dd) + al(sizeof(DevPrior) * dd) + al(sizeof(double) * kTraceCols * max_stages) +
           stage_scratch_bytes(P);
}

// Scratch of the stage kernels: chunk partial sums [2][nchunk][kStagePartVals], the search
// state [2] and the chunk totals [nchunk].
size_t stage_scratch_bytes(int P) {
    auto al = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    const size_t nchunk = (static_cast<size_t>(P) + kStageChunk - 1) / kStageChunk;
    return al(sizeof(double) * 2 * nchunk * kStagePartVals) + al(sizeof(StageNewton) * 2) +
           al(sizeof(unsigned long long) * nchunk);
}

bool carve_stage_scratch(Arena& a, int P, GroupDesc& g) {
    g.nchunk = (P + kStageChunk - 1) / kStageChunk;
    g.part = static_cast<double*>(a.take(sizeof(double) * 2 * g.nchunk * kStagePartVals));
    g.nst = static_cast<StageNewton*>(a.take(sizeof(StageNewton) * 2));
    g.ctot = static_cast<unsigned long long*>(a.take(sizeof(unsigned long long) * g.nchunk));
    return g.part && g.nst && g.ctot;
}

size_t spectrum_bytes(const smc_problem& p, const smc_options& o) {
    const int P = o.n_particles, M = o.waste_free ? P / o.n_moves : P;
    size_t b = 2 * ((sizeof(float) * p.n_points + 255) & ~static_cast<size_t>(255)) + 256 + sizeof(float) * p.k_max;
    for (int K = p.k_min; K <= p.k_max; ++K) {
        const int d = K * params_per_peak(p.peak_kind) + params_bg(p.bg_kind);
        b += group_bytes(d, P, M, o.max_stages) + sizeof(GroupDesc) + sizeof(GroupState) + 512;
    }
    return b;
}

void model_consts(const smc_problem& p, int K, GroupDesc& g) {
    g.n = p.n_points;
    g.K = K;
    g.np = params_per_peak(p.peak_kind);
    g.nbg = params_bg(p.bg_kind);
    g.d = K * g.np + g.nbg;
    g.peak_kind = p.peak_kind;
    g.bg_kind = p.bg_kind;
    g.noise_kind = p.noise_kind;
    g.inv2s2 = p.noise_kind == SMC_NOISE_GAUSS ? static_cast<float>(1.0 / (2.0 * p.sigma * p.sigma)) : 0.0f;
    for (int q = 0; q < 3; ++q)
        g.hn[q] = p.noise_kind == SMC_NOISE_HETERO ? static_cast<float>(p.noise_s[q] * p.noise_s[q]) : 0.0f;
}

// Fill descriptors for K = k_min..k_max of one spectrum, carving buffers from `arena`.
// Host-side prior tables are uploaded through `staging` (device pointer, host vector pairs).
bool describe_spectrum(const Spectrum& sp, const smc_options& o, Arena& arena, GroupState* d_states_base,
                       int first_state, std::vector<GroupDesc>& out, std::vector<PendingCopy>& copies) {
    const smc_problem& p = sp.prob;
    const int P = o.n_particles, M = o.waste_free ? P / o.n_moves : P;
    float* dx = static_cast<float*>(arena.take(sizeof(float) * p.n_points));
    float* dy = static_cast<float*>(arena.take(sizeof(float) * p.n_points));
    if (!dx || !dy) return false;
    copies.push_back(PendingCopy{dx, sp.xf.data(), sizeof(float) * p.n_points});
    copies.push_back(PendingCopy{dy, sp.yf.data(), sizeof(float) * p.n_points});
    float* dmu = nullptr;
    if (!sp.mref_f.empty()) {
        dmu = static_cast<float*>(arena.take(sizeof(float) * sp.mref_f.size()));
        if (!dmu) return false;
        copies.push_back(PendingCopy{dmu, sp.mref_f.data(), sizeof(float) * sp.mref_f.size()});
    }
    int si = first_state;
    for (int K = p.k_min; K <= p.k_max; ++K, ++si) {
        GroupDesc g{};
        model_consts(p, K, g);
        g.x = dx;
        g.mu_ref = dmu;
        g.y = dy;
        g.P = P;
        g.M = M;
        g.n_moves = o.n_moves;
        g.waste_free = o.waste_free;
        const size_t dd = std::max(g.d, 1);
        g.theta = static_cast<float*>(arena.take(sizeof(float) * dd * P));
        g.energy = static_cast<float*>(arena.take(sizeof(float) * P));
        g.start = static_cast<float*>(arena.take(sizeof(float) * dd * M));
        g.start_e = static_cast<float*>(arena.take(sizeof(float) * M));
        g.cdf = static_cast<unsigned long long*>(arena.take(sizeof(unsigned long long) * P));
        g.lambda = static_cast<double*>(arena.take(sizeof(double) * dd));
        g.step = static_cast<float*>(arena.take(sizeof(float) * dd));
        g.acc = static_cast<uint32_t*>(arena.take(sizeof(uint32_t) * dd));
        DevPrior* pri = static_cast<DevPrior*>(arena.take(sizeof(DevPrior) * dd));
        g.trace = static_cast<double*>(arena.take(sizeof(double) * kTraceCols * o.max_stages));
        if (!g.theta || !g.energy || !g.start || !g.start_e || !g.cdf || !g.lambda || !g.step || !g.acc || !pri ||
            !g.trace || !carve_stage_scratch(arena, P, g))
            return false;
        g.prior = pri;
        g.st = d_states_base + si;
        g.rho = o.ess_frac;
        g.bisect_iters = o.bisect_iters;
        g.max_stages = o.max_stages;
        g.key0 = static_cast<uint32_t>(o.seed);
        g.key1 = static_cast<uint32_t>(o.seed >> 32) ^ p.uid;
        g.kidx = K - p.k_min;
        out.push_back(g);
    }
    return true;
}

void Spectrum::assign(const smc_problem& p) {
    prob = p;
    x.assign(p.x, p.x + p.n_points);
    y.assign(p.y, p.y + p.n_points);
    xf.resize(p.n_points);
    yf.resize(p.n_points);
    for (int i = 0; i < p.n_points; ++i) {
        xf[i] = static_cast<float>(x[i]);
        yf[i] = static_cast<float>(y[i]);
    }
    prob.x = x.data();
    prob.y = y.data();
    if (p.peak_prior_k) {
        ppk.assign(p.peak_prior_k, p.peak_prior_k + SMC_MAX_PEAK_PARAMS * p.k_max);
        prob.peak_prior_k = ppk.data();
    } else {
        ppk.clear();
    }
    mref.clear();
    mref_f.clear();
    if (p.mu_ref) {
        mref.assign(p.mu_ref, p.mu_ref + p.k_max);
        for (double v : mref) mref_f.push_back(static_cast<float>(v));
        prob.mu_ref = mref.data();
    }
}

// Upload the per-group prior tables and initial lambda / state values.
hipError_t upload_group_tables(const Spectrum& sp, const std::vector<GroupDesc>& gs, size_t first, size_t count,
                               hipStream_t s, std::vector<std::vector<char>>& keep) {
    for (size_t gi = first; gi < first + count; ++gi) {
        const GroupDesc& g = gs[gi];
        std::vector<char> buf(sizeof(DevPrior) * std::max(g.d, 1) + sizeof(double) * std::max(g.d, 1));
        DevPrior* pri = reinterpret_cast<DevPrior*>(buf.data());
        double* lam = reinterpret_cast<double*>(buf.data() + sizeof(DevPrior) * std::max(g.d, 1));
        for (int j = 0; j < g.d; ++j) {
            pri[j] = dev_prior(component_prior(sp.prob, g.K, j));
            lam[j] = 1.0;
        }
        keep.push_back(std::move(buf));
        const std::vector<char>& b = keep.back();
        hipError_t e = hipMemcpyAsync(const_cast<DevPrior*>(g.prior), b.data(), sizeof(DevPrior) * g.d,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(g.lambda, b.data() + sizeof(DevPrior) * std::max(g.d, 1), sizeof(double) * g.d,
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemsetAsync(g.acc, 0, sizeof(uint32_t) * std::max(g.d, 1), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bool device_ok() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

}  // namespace smc

// Stage 0 of every group: prior draws and their energies.
static smc_status stage0(smc_ctx* c) {
    const int P = c->opt.n_particles;
    for (int gi = 0; gi < c->ng; ++gi)
        if (launch_draw(c->d_groups, gi, static_cast<int64_t>(c->groups[gi].d) * P, c->stream) != hipSuccess)
            return SMC_EDEVICE;
    const void* efn = kernels().energy[c->spec.prob.peak_kind][c->spec.prob.noise_kind][c->tile.lc][c->tile.pi];
    if (launch_tiled(efn, c->tile, c->n_init_work, c->lds_energy, c->d_groups, c->d_init_work, c->stream) != hipSuccess)
        return SMC_EDEVICE;
    c->stage0_evals = static_cast<uint64_t>(P) * c->ng;
    return SMC_OK;
}

extern "C" smc_status smc_init(smc_ctx** out, const smc_problem* prob, const smc_options* opt) {
    if (!out) return SMC_EINVAL;
    *out = nullptr;
    smc_status st = validate(prob, opt);
    if (st != SMC_OK) return st;
    if (!device_ok()) return SMC_EDEVICE;

    smc_ctx* c = new (std::nothrow) smc_ctx();
    if (!c) return SMC_ENOMEM;
    c->spec.assign(*prob);
    c->opt = *opt;
    c->kmin = prob->k_min;
    c->kmax = prob->k_max;
    c->ng = c->kmax - c->kmin + 1;
    c->econst = energy_constant(c->spec.prob);
    if (opt->hip_stream) {
        c->stream = static_cast<hipStream_t>(opt->hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return ctx_fail(c, SMC_EDEVICE);
        c->own_stream = true;
    }

    const int P = opt->n_particles, M = opt->waste_free ? P / opt->n_moves : P;
    // tiles: one tile for all groups of the spectrum (same N); work ordered heaviest K first
    const int64_t chains = static_cast<int64_t>(c->ng) * M;
    c->tile = choose_tile(*prob, chains, opt->lanes_per_chain);
    if (!tile_has_kernels(*prob, c->tile)) return ctx_fail(c, SMC_EINVAL);
    std::vector<int> order(c->ng), chains_m(c->ng, M), chains_p(c->ng, P);
    for (int i = 0; i < c->ng; ++i) order[i] = c->ng - 1 - i;
    std::vector<MoveWork> work, init_work;
    c->work_off.assign(c->ng, 0);
    c->work_cnt.assign(c->ng, 0);
    for (int gi : order) {
        const size_t before = work.size();
        build_work(std::vector<int>{gi}, chains_m, c->tile, work);
        c->work_off[gi] = static_cast<int>(before);
        c->work_cnt[gi] = static_cast<int>(work.size() - before);
    }
    build_work(order, chains_p, c->tile, init_work);
    c->n_work = static_cast<int>(work.size());
    c->n_init_work = static_cast<int>(init_work.size());

    const size_t bytes = spectrum_bytes(c->spec.prob, *opt) + 4096 + 512 * 4 +
                         sizeof(GroupDesc) * c->ng + sizeof(GroupState) * c->ng +
                         sizeof(MoveWork) * (work.size() + init_work.size());
    if (hipMalloc(&c->dmem, bytes) != hipSuccess) return ctx_fail(c, SMC_ENOMEM);
    c->arena = Arena{c->dmem, bytes, 0};
    c->d_groups = static_cast<GroupDesc*>(c->arena.take(sizeof(GroupDesc) * c->ng));
    c->d_states = static_cast<GroupState*>(c->arena.take(sizeof(GroupState) * c->ng));
    std::vector<PendingCopy> copies;
    if (!c->d_groups || !c->d_states || !describe_spectrum(c->spec, *opt, c->arena, c->d_states, 0, c->groups, copies))
        return ctx_fail(c, SMC_ENOMEM);
    c->d_work = static_cast<MoveWork*>(c->arena.take(sizeof(MoveWork) * work.size()));
    c->d_init_work = static_cast<MoveWork*>(c->arena.take(sizeof(MoveWork) * init_work.size()));
    if (!c->d_work || !c->d_init_work) return ctx_fail(c, SMC_ENOMEM);
    int dmax = 1;
    for (const GroupDesc& g : c->groups) dmax = std::max(dmax, g.d);
    c->lds_move = move_lds_bytes(c->tile, dmax, prob->peak_kind, prob->noise_kind);
    c->lds_energy = energy_lds_bytes(c->tile, dmax);

    c->states.assign(c->ng, GroupState{});
    std::vector<std::vector<char>> keep;
    hipStream_t s = c->stream;
    bool ok = hipMemcpyAsync(c->d_groups, c->groups.data(), sizeof(GroupDesc) * c->ng, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(c->d_states, c->states.data(), sizeof(GroupState) * c->ng, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(c->d_work, work.data(), sizeof(MoveWork) * work.size(), hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(c->d_init_work, init_work.data(), sizeof(MoveWork) * init_work.size(),
                             hipMemcpyHostToDevice, s) == hipSuccess;
    for (const PendingCopy& pc : copies)
        ok = ok && hipMemcpyAsync(pc.dst, pc.src, pc.bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && upload_group_tables(c->spec, c->groups, 0, c->groups.size(), s, keep) == hipSuccess;
    if (!ok) return ctx_fail(c, SMC_EDEVICE);

    if (opt->profile)
        for (hipEvent_t& e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) return ctx_fail(c, SMC_EDEVICE);
    st = stage0(c);
    if (st != SMC_OK) return ctx_fail(c, st);
    if (hipStreamSynchronize(s) != hipSuccess) return ctx_fail(c, SMC_EDEVICE);
    *out = c;
    return SMC_OK;
}

extern "C" smc_status smc_reset(smc_ctx* c, uint64_t seed) {
    if (!c) return SMC_EINVAL;
    c->opt.seed = seed;
    for (GroupDesc& g : c->groups) {
        g.key0 = static_cast<uint32_t>(seed);
        g.key1 = static_cast<uint32_t>(seed >> 32) ^ c->spec.prob.uid;
    }
    c->states.assign(c->ng, GroupState{});
    std::vector<std::vector<char>> keep;
    hipStream_t s = c->stream;
    if (hipMemcpyAsync(c->d_groups, c->groups.data(), sizeof(GroupDesc) * c->ng, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(c->d_states, c->states.data(), sizeof(GroupState) * c->ng, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        upload_group_tables(c->spec, c->groups, 0, c->groups.size(), s, keep) != hipSuccess)
        return SMC_EDEVICE;
    c->finished = false;
    c->n_ev_move = c->n_ev_stage = 0;   // event pairs of a run that ended in an error are dropped
    smc_status st = stage0(c);
    if (st != SMC_OK) return st;
    return hipStreamSynchronize(s) == hipSuccess ? SMC_OK : SMC_EDEVICE;
}

extern "C" smc_status smc_evaluations(const smc_ctx* c, uint64_t* n) {
    if (!c || !n) return SMC_EINVAL;
    uint64_t t = c->stage0_evals;
    for (const GroupState& s : c->states) t += s.evals;
    *n = t;
    return SMC_OK;
}

extern "C" smc_status smc_evaluation_kinds(const smc_ctx* c, uint64_t* out) {
    if (!c || !out) return SMC_EINVAL;
    uint64_t all = 0, linear = 0;
    for (const GroupState& s : c->states) {
        all += s.evals;
        linear += s.evals_linear;
    }
    out[0] = c->stage0_evals;
    out[1] = all - linear;
    out[2] = linear;
    return SMC_OK;
}

extern "C" smc_status smc_profile(const smc_ctx* c, double* out) {
    if (!c || !out) return SMC_EINVAL;
    if (!c->opt.profile) return SMC_ESTATE;
    out[0] = c->move_ms;
    out[1] = static_cast<double>(c->move_launches);
    out[2] = c->stage_ms;
    out[3] = static_cast<double>(c->stage_launches);
    return SMC_OK;
}

static void collect_events(smc_ctx* c, int moves, int stages);

static int max_stage(const smc_ctx* c) {
    int m = 0;
    for (const GroupState& s : c->states) m = std::max(m, static_cast<int>(s.stage));
    return m;
}

// Read the group states back.  With profiling, the timed launches since the last read are
// collected: all of them when `before` < 0, else only the launches in which some group had
// work, as many as the largest stage count advanced from `before` (a move launch did work
// iff some group advanced a stage before it).
static smc_status read_states(smc_ctx* c, int before = -1) {
    if (hipMemcpyAsync(c->states.data(), c->d_states, sizeof(GroupState) * c->ng, hipMemcpyDeviceToHost, c->stream) !=
        hipSuccess)
        return SMC_EDEVICE;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SMC_EDEVICE;
    if (c->opt.profile) {
        const int real = before < 0 ? kStagesPerRead : std::max(0, max_stage(c) - before);
        collect_events(c, std::min(real, c->n_ev_move), std::min(real, c->n_ev_stage));
    }
    return SMC_OK;
}

// Launch wrappers that bracket the launch with HIP events when profiling.
static hipError_t timed_stage(smc_ctx* c, const GroupDesc* groups, int n) {
    const bool prof = c->opt.profile && c->n_ev_stage < kStagesPerRead;
    hipEvent_t* ev = c->ev + 2 * kStagesPerRead + 2 * c->n_ev_stage;
    if (prof && hipEventRecord(ev[0], c->stream) != hipSuccess) return hipErrorUnknown;
    int dmax = 1;
    for (const GroupDesc& g : c->groups) dmax = std::max(dmax, g.d);
    const int P = c->opt.n_particles, M = c->opt.waste_free ? P / c->opt.n_moves : P;
    hipError_t e = launch_stage(StageLaunch{groups, n, P, M, dmax}, c->stream);
    if (prof && e == hipSuccess) {
        e = hipEventRecord(ev[1], c->stream);
        ++c->n_ev_stage;
    }
    return e;
}

static hipError_t timed_move(smc_ctx* c, const void* fn, int n_work, const MoveWork* work) {
    const bool prof = c->opt.profile && c->n_ev_move < kStagesPerRead;
    hipEvent_t* ev = c->ev + 2 * c->n_ev_move;
    if (prof && hipEventRecord(ev[0], c->stream) != hipSuccess) return hipErrorUnknown;
    hipError_t e = launch_tiled(fn, c->tile, n_work, c->lds_move, c->d_groups, work, c->stream);
    if (prof && e == hipSuccess) {
        e = hipEventRecord(ev[1], c->stream);
        ++c->n_ev_move;
    }
    return e;
}

static void collect_events(smc_ctx* c, int moves, int stages) {
    float ms = 0.0f;
    for (int b = 0; b < moves; ++b)
        if (hipEventElapsedTime(&ms, c->ev[2 * b], c->ev[2 * b + 1]) == hipSuccess) {
            c->move_ms += ms;
            ++c->move_launches;
        }
    const hipEvent_t* es = c->ev + 2 * kStagesPerRead;
    for (int b = 0; b < stages; ++b)
        if (hipEventElapsedTime(&ms, es[2 * b], es[2 * b + 1]) == hipSuccess) {
            c->stage_ms += ms;
            ++c->stage_launches;
        }
    c->n_ev_move = c->n_ev_stage = 0;
}

static const void* move_fn(const smc_ctx* c) {
    return kernels().move[c->spec.prob.peak_kind][c->spec.prob.noise_kind][c->tile.lc][c->tile.pi];
}

// Plain comparator: the first unfinished K advances by one stage with its own launches.
static smc_status step_plain(smc_ctx* c, int32_t* all_done) {
    int gi = 0;
    while (gi < c->ng && (c->states[gi].done || c->states[gi].beta >= 1.0)) ++gi;
    if (gi < c->ng) {
        if (timed_stage(c, c->d_groups + gi, 1) != hipSuccess) return SMC_EDEVICE;
        if (timed_move(c, move_fn(c), c->work_cnt[gi], c->d_work + c->work_off[gi]) != hipSuccess)
            return SMC_EDEVICE;
        smc_status st = read_states(c);
        if (st != SMC_OK) return st;
        if (c->states[gi].status != SMC_OK) return c->states[gi].status;
        if (c->states[gi].beta >= 1.0) {
            if (timed_stage(c, c->d_groups + gi, 1) != hipSuccess) return SMC_EDEVICE;
            st = read_states(c);
            if (st != SMC_OK) return st;
        }
    }
    bool done = true;
    for (const GroupState& s : c->states) done = done && (s.done || s.beta >= 1.0);
    c->finished = done;
    if (all_done) *all_done = done ? 1 : 0;
    return SMC_OK;
}

extern "C" smc_status smc_step(smc_ctx* c, int32_t* all_done) {
    if (!c) return SMC_EINVAL;
    if (c->finished) {
        if (all_done) *all_done = 1;
        return SMC_OK;
    }
    if (c->opt.plain) return step_plain(c, all_done);
    if (timed_stage(c, c->d_groups, c->ng) != hipSuccess) return SMC_EDEVICE;
    if (timed_move(c, move_fn(c), c->n_work, c->d_work) != hipSuccess) return SMC_EDEVICE;
    smc_status st = read_states(c);
    if (st != SMC_OK) return st;
    bool done = true;
    for (const GroupState& s : c->states) {
        if (s.status != SMC_OK) return s.status;
        done = done && (s.done || s.beta >= 1.0);
    }
    if (done) {
        // one more stage launch records the final acceptance and marks the groups done
        if (timed_stage(c, c->d_groups, c->ng) != hipSuccess) return SMC_EDEVICE;
        st = read_states(c);
        if (st != SMC_OK) return st;
        c->finished = true;
    }
    if (all_done) *all_done = done ? 1 : 0;
    return SMC_OK;
}

// The whole run: kStagesPerRead stages (stage pipeline + move) go into the stream before
// each read of the group states, so the host's round trip and launch work overlap the
// device's.  A stage launched after a group has finished does nothing for it (every
// stage and move kernel returns at once for a done group), so the states are those of
// one stage per read.
extern "C" smc_status smc_run(smc_ctx* c) {
    if (!c) return SMC_EINVAL;
    if (c->opt.plain) {
        int32_t done = 0;
        while (!done) {
            smc_status st = smc_step(c, &done);
            if (st != SMC_OK) return st;
        }
        return SMC_OK;
    }
    while (!c->finished) {
        const int before = max_stage(c);
        for (int b = 0; b < kStagesPerRead; ++b) {
            if (timed_stage(c, c->d_groups, c->ng) != hipSuccess) return SMC_EDEVICE;
            if (timed_move(c, move_fn(c), c->n_work, c->d_work) != hipSuccess) return SMC_EDEVICE;
        }
        smc_status st = read_states(c, before);
        if (st != SMC_OK) return st;
        bool done = true, marked = true;
        for (const GroupState& s : c->states) {
            if (s.status != SMC_OK) return s.status;
            done = done && (s.done || s.beta >= 1.0);
            marked = marked && s.done;
        }
        if (done) {
            if (!marked) {
                // one more stage launch records the final acceptance and marks the groups done
                if (timed_stage(c, c->d_groups, c->ng) != hipSuccess) return SMC_EDEVICE;
                st = read_states(c);
                if (st != SMC_OK) return st;
            }
            c->finished = true;
        }
    }
    return SMC_OK;
}

extern "C" smc_status smc_log_evidence(const smc_ctx* c, double* logz, int32_t cap) {
    if (!c || !logz) return SMC_EINVAL;
    const int n = std::min(cap, c->ng);
    bool all = true;
    for (int i = 0; i < n; ++i) {
        const GroupState& s = c->states[i];
        logz[i] = s.logz - s.beta * c->econst;
        all = all && s.beta >= 1.0;
    }
    return all ? SMC_OK : SMC_ESTATE;
}

extern "C" smc_status smc_stage_info(const smc_ctx* c, int32_t K, int32_t* stage, double* beta, double* logz,
                                     double* ess) {
    if (!c || K < c->kmin || K > c->kmax) return SMC_EINVAL;
    const GroupState& s = c->states[K - c->kmin];
    if (stage) *stage = s.stage;
    if (beta) *beta = s.beta;
    if (logz) *logz = s.logz - s.beta * c->econst;
    if (ess) *ess = s.ess;
    return SMC_OK;
}

extern "C" smc_status smc_trace(const smc_ctx* c, int32_t K, double* beta, double* ess, double* logz, double* accept,
                                int32_t cap, int32_t* n) {
    if (!c || K < c->kmin || K > c->kmax) return SMC_EINVAL;
    const GroupDesc& g = c->groups[K - c->kmin];
    const GroupState& s = c->states[K - c->kmin];
    const int ns = std::min(s.stage, std::min(cap, c->opt.max_stages));
    std::vector<double> tr(static_cast<size_t>(kTraceCols) * std::max(ns, 1));
    if (ns > 0 && hipMemcpy(tr.data(), g.trace, sizeof(double) * kTraceCols * ns, hipMemcpyDeviceToHost) != hipSuccess)
        return SMC_EDEVICE;
    for (int i = 0; i < ns; ++i) {
        const double* r = tr.data() + i * kTraceCols;
        if (beta) beta[i] = r[0];
        if (ess) ess[i] = r[2];
        if (logz) logz[i] = r[4] - r[0] * c->econst;
        if (accept) accept[i] = r[5];
    }
    if (n) *n = ns;
    return SMC_OK;
}

extern "C" smc_status smc_particles(const smc_ctx* c, int32_t K, float* theta_soa, float* energy, int64_t cap) {
    if (!c || K < c->kmin || K > c->kmax) return SMC_EINVAL;
    const GroupDesc& g = c->groups[K - c->kmin];
    const int64_t need = static_cast<int64_t>(g.d) * g.P;
    if (theta_soa) {
        if (cap < need) return SMC_EINVAL;
        if (need > 0 && hipMemcpy(theta_soa, g.theta, sizeof(float) * need, hipMemcpyDeviceToHost) != hipSuccess)
            return SMC_EDEVICE;
    }
    if (energy && hipMemcpy(energy, g.energy, sizeof(float) * g.P, hipMemcpyDeviceToHost) != hipSuccess)
        return SMC_EDEVICE;
    return SMC_OK;
}

extern "C" smc_status smc_posterior_summary(smc_ctx* c, int32_t K, const double* probs, int32_t n_probs,
                                            int32_t relabel, double* mean, double* quant) {
    if (!c || K < c->kmin || K > c->kmax) return SMC_EINVAL;
    const int gi = K - c->kmin;
    if (c->states[gi].beta < 1.0) return SMC_ESTATE;
    const GroupDesc& g = c->groups[gi];
    if (relabel && g.peak_kind == SMC_PEAK_XRD) return SMC_EINVAL;   // XRD peaks carry their own mu_ref
    const int n_peaks = relabel ? K : 0;
    return posterior_summary(g.theta, g.d, g.P, n_peaks, g.np, probs, n_probs, mean, quant, c->stream);
}

extern "C" smc_status smc_posterior_k(const smc_ctx* c, double* out, int32_t cap) {
    if (!c || !out || cap < 1) return SMC_EINVAL;
    const int n = std::min(cap, c->ng);
    std::vector<double> lz(n);
    const smc_status st = smc_log_evidence(c, lz.data(), n);
    if (st != SMC_OK) return st;
    double m = -INFINITY;
    for (double v : lz) m = std::max(m, v);
    if (!std::isfinite(m)) return SMC_ENUMERIC;
    double sum = 0.0;
    for (double v : lz) sum += std::exp(v - m);
    for (int i = 0; i < n; ++i) out[i] = std::exp(lz[i] - m) / sum;
    return SMC_OK;
}

extern "C" void smc_free(smc_ctx* c) {
    if (!c) return;
    // teardown: errors here have nowhere to go
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->dmem) (void)hipFree(c->dmem);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// ------------------------------------------------------------------ tile tuner
//
// Times the move kernel of every lane configuration that has kernels for the problem's
// model family and holds its N points, on this device, and keeps the fastest per problem
// shape.  Each candidate runs `stages` tempering stages of the problem itself (stage 0
// included) with HIP-event profiling; the cost is the move time per particle*point
// evaluation, so candidates that take slightly different trajectories compare fairly.

namespace {

struct TuneKey {
    int32_t peak, bg, noise, n, k_min, k_max, P, n_moves, waste_free, stages, device;
    bool operator<(const TuneKey& o) const {
        return std::tie(peak, bg, noise, n, k_min, k_max, P, n_moves, waste_free, stages, device) <
               std::tie(o.peak, o.bg, o.noise, o.n, o.k_min, o.k_max, o.P, o.n_moves, o.waste_free, o.stages,
                        o.device);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int32_t, double>> g_tune_cache;

}  // namespace

extern "C" smc_status smc_tune_lanes(const smc_problem* prob, const smc_options* opt, int32_t stages,
                                     int32_t* lanes_out, double* ns_per_eval_out) {
    if (!prob || !opt || !lanes_out || stages < 1 || stages > 64) return SMC_EINVAL;
    smc_options base = *opt;
    base.lanes_per_chain = 0;
    const smc_status vst = validate(prob, &base);
    if (vst != SMC_OK) return vst;
    if (!device_ok()) return SMC_EDEVICE;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return SMC_EDEVICE;
    const TuneKey key{prob->peak_kind, prob->bg_kind, prob->noise_kind, prob->n_points, prob->k_min, prob->k_max,
                      opt->n_particles, opt->n_moves, opt->waste_free, stages, device};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *lanes_out = it->second.first;
            if (ns_per_eval_out) *ns_per_eval_out = it->second.second;
            return SMC_OK;
        }
    }
    int32_t best = 0;
    double best_ns = INFINITY;
    for (int lc = 0; lc < kNumLaneCfg; ++lc) {
        smc_options o = base;
        o.lanes_per_chain = kLanesOf[lc];
        o.profile = 1;
        if (validate(prob, &o) != SMC_OK) continue;   // a lane count this family does not run
        smc_ctx* c = nullptr;
        smc_status st = smc_init(&c, prob, &o);
        if (st == SMC_EINVAL) continue;               // no tile holds N at this lane count
        if (st != SMC_OK) return st;
        uint64_t e0 = 0, e1 = 0;
        double prof[4] = {0.0, 0.0, 0.0, 0.0};
        int32_t done = 0;
        st = smc_evaluations(c, &e0);
        for (int s = 0; s < stages && st == SMC_OK && !done; ++s) st = smc_step(c, &done);
        if (st == SMC_OK) st = smc_profile(c, prof);
        if (st == SMC_OK) st = smc_evaluations(c, &e1);
        smc_free(c);
        if (st != SMC_OK) return st;
        if (e1 <= e0 || prof[1] < 1.0) continue;
        const double ns = prof[0] * 1e6 / (static_cast<double>(e1 - e0) * prob->n_points);
        if (ns < best_ns) {
            best_ns = ns;
            best = kLanesOf[lc];
        }
    }
    if (best == 0) return SMC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best, best_ns};
    }
    *lanes_out = best;
    if (ns_per_eval_out) *ns_per_eval_out = best_ns;
    return SMC_OK;
}
