// hooks.cpp -- per-kernel entry points: the production kernels run on caller
// buffers, so each step of the sampler can be compared with the reference on
// identical inputs.  Temporary descriptors live in a small device block that
// is released before returning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "host_common.hpp"

using namespace smc;

namespace {

struct Scratch {
    void* mem = nullptr;
    ~Scratch() {
        if (mem) (void)hipFree(mem);
    }
};

// Descriptor of one group whose particle buffers belong to the caller.
struct HookGroup {
    Scratch scratch;
    GroupDesc* d_group = nullptr;
    GroupState* d_state = nullptr;
    MoveWork* d_work = nullptr;
    int n_work = 0;
    Tile tile{};
    GroupDesc g{};
    Spectrum sp;
};

smc_status make_hook_group(HookGroup& h, const smc_problem* prob, int K, int P, int M, int n_moves, int waste_free,
                           int chains, int lanes, double beta, int stage, uint64_t seed, hipStream_t s) {
    smc_options o;
    smc_default_options(&o);
    o.n_particles = P;
    o.n_moves = n_moves;
    o.waste_free = waste_free;
    o.lanes_per_chain = lanes;
    o.seed = seed;
    o.max_stages = 1;
    if ((prob->peak_prior_k || prob->mu_ref) && K > prob->k_max) return SMC_EINVAL;
    smc_problem p = *prob;
    p.k_min = p.k_max = K;
    smc_status st = validate(&p, &o);
    if (st != SMC_OK) return st;
    if (!device_ok()) return SMC_EDEVICE;
    h.sp.assign(p);
    h.sp.prob.k_min = h.sp.prob.k_max = K;
    h.tile = choose_tile(p, chains, lanes);
    if (!tile_has_kernels(p, h.tile)) return SMC_EINVAL;

    std::vector<MoveWork> work;
    build_work(std::vector<int>{0}, std::vector<int>{chains}, h.tile, work);
    h.n_work = static_cast<int>(work.size());
    const int d = K * params_per_peak(p.peak_kind) + params_bg(p.bg_kind);
    const size_t bytes = 4 * 4096 + sizeof(MoveWork) * work.size() + sizeof(DevPrior) * std::max(d, 1) +
                         sizeof(double) * std::max(d, 1) + sizeof(float) * std::max(d, 1) * 2 +
                         2 * sizeof(float) * p.n_points + sizeof(unsigned long long) * std::max(P, 1) +
                         sizeof(double) * kTraceCols + sizeof(float) * std::max(K, 1) + 8192;
    if (hipMalloc(&h.scratch.mem, bytes) != hipSuccess) return SMC_ENOMEM;
    Arena a{h.scratch.mem, bytes, 0};
    h.d_group = static_cast<GroupDesc*>(a.take(sizeof(GroupDesc)));
    h.d_state = static_cast<GroupState*>(a.take(sizeof(GroupState)));
    h.d_work = static_cast<MoveWork*>(a.take(sizeof(MoveWork) * work.size()));
    float* dx = static_cast<float*>(a.take(sizeof(float) * p.n_points));
    float* dy = static_cast<float*>(a.take(sizeof(float) * p.n_points));
    DevPrior* pri = static_cast<DevPrior*>(a.take(sizeof(DevPrior) * std::max(d, 1)));
    double* lam = static_cast<double*>(a.take(sizeof(double) * std::max(d, 1)));
    unsigned long long* cdf = static_cast<unsigned long long*>(a.take(sizeof(unsigned long long) * std::max(P, 1)));
    double* trace = static_cast<double*>(a.take(sizeof(double) * kTraceCols));
    float* dmu = h.sp.mref_f.empty() ? nullptr : static_cast<float*>(a.take(sizeof(float) * K));
    if (!h.d_group || !h.d_state || !h.d_work || !dx || !dy || !pri || !lam || !cdf || !trace) return SMC_ENOMEM;
    if (!h.sp.mref_f.empty() && !dmu) return SMC_ENOMEM;

    GroupDesc& g = h.g;
    model_consts(p, K, g);
    g.x = dx;
    g.mu_ref = dmu;
    g.y = dy;
    g.prior = pri;
    g.P = P;
    g.M = M;
    g.n_moves = n_moves;
    g.waste_free = waste_free;
    g.cdf = cdf;
    g.lambda = lam;
    g.st = h.d_state;
    g.trace = trace;
    g.rho = 0.5;
    g.bisect_iters = 50;
    g.max_stages = 1;
    g.key0 = static_cast<uint32_t>(seed);
    g.key1 = static_cast<uint32_t>(seed >> 32) ^ p.uid;

    std::vector<DevPrior> hp(std::max(d, 1));
    for (int j = 0; j < d; ++j) hp[j] = dev_prior(component_prior(h.sp.prob, K, j));
    GroupState gs{};
    gs.beta = beta;
    gs.stage = stage;
    if (hipMemcpyAsync(dx, h.sp.xf.data(), sizeof(float) * p.n_points, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(dy, h.sp.yf.data(), sizeof(float) * p.n_points, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(pri, hp.data(), sizeof(DevPrior) * std::max(d, 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        (dmu && hipMemcpyAsync(dmu, h.sp.mref_f.data(), sizeof(float) * K, hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(h.d_state, &gs, sizeof(GroupState), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h.d_work, work.data(), sizeof(MoveWork) * work.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SMC_EDEVICE;
    return SMC_OK;
}

smc_status upload_desc(HookGroup& h, hipStream_t s) {
    if (hipMemcpyAsync(h.d_group, &h.g, sizeof(GroupDesc), hipMemcpyHostToDevice, s) != hipSuccess) return SMC_EDEVICE;
    return SMC_OK;
}

smc_status finish(hipStream_t s) { return hipStreamSynchronize(s) == hipSuccess ? SMC_OK : SMC_EDEVICE; }

}  // namespace

extern "C" smc_status smc_kernel_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, uint32_t* out, int64_t n,
                                        void* stream) {
    if (n < 0 || (n > 0 && (!ctr || !out))) return SMC_EINVAL;
    if (n == 0) return SMC_OK;
    if (!device_ok()) return SMC_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (launch_philox(ctr, key0, key1, out, n, s) != hipSuccess) return SMC_EDEVICE;
    return finish(s);
}

extern "C" smc_status smc_kernel_init(const smc_problem* prob, int32_t K, int32_t P, uint64_t seed, float* theta_soa,
                                      float* energy, int32_t lanes_per_chain, void* stream) {
    if (!prob || K < 1 || P < 1 || !theta_soa || !energy) return SMC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HookGroup h;
    smc_status st = make_hook_group(h, prob, K, P, P, 1, 0, P, lanes_per_chain, 0.0, 0, seed, s);
    if (st != SMC_OK) return st;
    h.g.theta = theta_soa;
    h.g.energy = energy;
    if ((st = upload_desc(h, s)) != SMC_OK) return st;
    if (launch_draw(h.d_group, 0, static_cast<int64_t>(h.g.d) * P, s) != hipSuccess) return SMC_EDEVICE;
    const void* fn = kernels().energy[h.g.peak_kind][h.g.noise_kind][h.tile.lc][h.tile.pi];
    if (launch_tiled(fn, h.tile, h.n_work, energy_lds_bytes(h.tile, h.g.d), h.d_group, h.d_work, s) != hipSuccess)
        return SMC_EDEVICE;
    return finish(s);
}

extern "C" smc_status smc_kernel_energy(const smc_problem* prob, int32_t K, const float* theta_soa, int64_t n_theta,
                                        float* energy, int32_t lanes_per_chain, void* stream) {
    if (!prob || K < 1 || n_theta < 1 || n_theta > (1 << 30) || !theta_soa || !energy) return SMC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HookGroup h;
    const int n = static_cast<int>(n_theta);
    smc_status st = make_hook_group(h, prob, K, n, n, 1, 0, n, lanes_per_chain, 0.0, 0, 0, s);
    if (st != SMC_OK) return st;
    h.g.theta = const_cast<float*>(theta_soa);
    h.g.energy = energy;
    if ((st = upload_desc(h, s)) != SMC_OK) return st;
    const void* fn = kernels().energy[h.g.peak_kind][h.g.noise_kind][h.tile.lc][h.tile.pi];
    if (launch_tiled(fn, h.tile, h.n_work, energy_lds_bytes(h.tile, h.g.d), h.d_group, h.d_work, s) != hipSuccess)
        return SMC_EDEVICE;
    return finish(s);
}

// One stand-alone group for the stage hooks: state, trace row, CDF and stage scratch.
namespace {
struct StageHook {
    Scratch scratch;
    GroupDesc* d_group = nullptr;
    GroupDesc g{};
};

smc_status make_stage_hook(StageHook& h, int P, int M, double beta, double rho, int iters, hipStream_t s) {
    const size_t bytes = 2 * 4096 + sizeof(GroupDesc) + sizeof(GroupState) + sizeof(double) * kTraceCols +
                         sizeof(unsigned long long) * P + stage_scratch_bytes(P) + 4096;
    if (hipMalloc(&h.scratch.mem, bytes) != hipSuccess) return SMC_ENOMEM;
    Arena a{h.scratch.mem, bytes, 0};
    h.d_group = static_cast<GroupDesc*>(a.take(sizeof(GroupDesc)));
    GroupState* st = static_cast<GroupState*>(a.take(sizeof(GroupState)));
    GroupDesc& g = h.g;
    g.trace = static_cast<double*>(a.take(sizeof(double) * kTraceCols));
    g.cdf = static_cast<unsigned long long*>(a.take(sizeof(unsigned long long) * P));
    if (!h.d_group || !st || !g.trace || !g.cdf || !carve_stage_scratch(a, P, g)) return SMC_ENOMEM;
    g.P = P;
    g.M = M;
    g.n_moves = 1;
    g.st = st;
    g.rho = rho;
    g.bisect_iters = iters;
    g.max_stages = 1;
    GroupState gs{};
    gs.beta = beta;
    if (hipMemcpyAsync(st, &gs, sizeof(gs), hipMemcpyHostToDevice, s) != hipSuccess) return SMC_EDEVICE;
    return SMC_OK;
}
}  // namespace

extern "C" smc_status smc_kernel_ess_bisect(const float* energy, int32_t P, double beta, double rho, int32_t iters,
                                            double* out, void* stream) {
    if (!energy || !out || P < 1 || !(beta >= 0.0 && beta < 1.0) || !(rho > 0.0 && rho < 1.0) || iters < 1 ||
        iters > 200)
        return SMC_EINVAL;
    if (!device_ok()) return SMC_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageHook h;
    smc_status st = make_stage_hook(h, P, 1, beta, rho, iters, s);
    if (st != SMC_OK) return st;
    h.g.energy = const_cast<float*>(energy);
    if (hipMemcpyAsync(h.d_group, &h.g, sizeof(GroupDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_search_hook(h.d_group, P, s) != hipSuccess)
        return SMC_EDEVICE;
    GroupState gs{};
    StageNewton fin{};
    if (hipMemcpyAsync(&gs, h.g.st, sizeof(gs), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&fin, h.g.nst + stage_final_parity(), sizeof(fin), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SMC_EDEVICE;
    if (gs.status != SMC_OK || fin.phase != kPhaseDone) {
        out[0] = __builtin_nan("");
        return SMC_ENUMERIC;
    }
    out[0] = gs.delta;
    out[1] = gs.ess;
    out[2] = gs.lse;
    out[3] = fin.emin;
    return SMC_OK;
}

extern "C" smc_status smc_kernel_resample(const double* weights, int32_t P, int32_t M, uint32_t r, int32_t* ancestors,
                                          void* stream) {
    if (!weights || !ancestors || P < 1 || M < 1) return SMC_EINVAL;
    if (!device_ok()) return SMC_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageHook h;
    smc_status st = make_stage_hook(h, P, M, 0.0, 0.5, 50, s);
    if (st != SMC_OK) return st;
    if (hipMemcpyAsync(h.g.cdf, weights, sizeof(double) * P, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h.d_group, &h.g, sizeof(GroupDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_resample_hook(h.d_group, P, M, r, ancestors, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return SMC_EDEVICE;
    return SMC_OK;
}

extern "C" smc_status smc_kernel_move(const smc_problem* prob, int32_t K, const float* start_soa, const float* start_e,
                                      int32_t M, int32_t n, int32_t waste_free, double beta, uint64_t seed,
                                      uint32_t stage, const float* step, float* out_soa, float* out_e, uint32_t* acc,
                                      int32_t lanes_per_chain, void* stream) {
    if (!prob || K < 1 || M < 1 || n < 1 || !start_soa || !start_e || !step || !out_soa || !out_e || !acc ||
        !(beta >= 0.0 && beta <= 1.0))
        return SMC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int P = waste_free ? M * n : M;
    HookGroup h;
    smc_status st = make_hook_group(h, prob, K, P, M, n, waste_free ? 1 : 0, M, lanes_per_chain, beta,
                                    static_cast<int>(stage), seed, s);
    if (st != SMC_OK) return st;
    h.g.start = const_cast<float*>(start_soa);
    h.g.start_e = const_cast<float*>(start_e);
    h.g.theta = out_soa;
    h.g.energy = out_e;
    h.g.step = const_cast<float*>(step);
    h.g.acc = acc;
    if ((st = upload_desc(h, s)) != SMC_OK) return st;
    const void* fn = kernels().move[h.g.peak_kind][h.g.noise_kind][h.tile.lc][h.tile.pi];
    if (launch_tiled(fn, h.tile, h.n_work, move_lds_bytes(h.tile, h.g.d, h.g.peak_kind, h.g.noise_kind), h.d_group, h.d_work, s) != hipSuccess)
        return SMC_EDEVICE;
    return finish(s);
}

extern "C" smc_status smc_kernel_step_sizes(const smc_problem* prob, int32_t K, const float* start_soa, int32_t M,
                                            int32_t n_moves, double* lambda, uint32_t* acc, float* step,
                                            void* stream) {
    if (!prob || K < 1 || M < 1 || n_moves < 1 || !start_soa || !lambda || !acc || !step) return SMC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HookGroup h;
    smc_status st = make_hook_group(h, prob, K, M, M, n_moves, 0, M, 0, 0.0, 1, 0, s);
    if (st != SMC_OK) return st;
    h.g.start = const_cast<float*>(start_soa);
    h.g.lambda = lambda;
    h.g.acc = acc;
    h.g.step = step;
    if ((st = upload_desc(h, s)) != SMC_OK) return st;
    if (launch_steps_hook(h.d_group, h.g.d, s) != hipSuccess) return SMC_EDEVICE;
    return finish(s);
}

extern "C" smc_status smc_kernel_summary(const float* theta, int32_t d, int32_t P, int32_t n_peaks, int32_t np,
                                         const double* probs, int32_t n_probs, double* mean, double* quant,
                                         void* hip_stream) {
    return posterior_summary(theta, d, P, n_peaks, np, probs, n_probs, mean, quant,
                             static_cast<hipStream_t>(hip_stream));
}
