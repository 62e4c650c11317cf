// host_common.hpp -- declarations shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "kernel_table.hpp"
#include "smc_types.hpp"

namespace smc {

constexpr int kMaxK = 64;
constexpr int kMaxXpsPoints = 1024;   // XPS model form: 64 lanes x 16 points
constexpr int kMaxXrdPoints = 10240;  // XRD powder profile: 512 lanes x 20 points
constexpr int kMaxPoints = 8192;      // Gaussian / pseudo-Voigt families: 256 lanes x 32 points

struct Tile {
    int lc, pi, lanes, ppl;
    bool valid;
};

// Threads per workgroup of the move / energy kernels: 256 (several chains of up to 256
// lanes), or one chain of more lanes.
inline int tile_threads(const Tile& t) { return t.lanes > 64 ? t.lanes : 256; }
inline int tile_chains_per_wg(const Tile& t) { return tile_threads(t) / t.lanes; }

struct Arena {
    void* base;
    size_t size;
    size_t used;
    void* take(size_t bytes);
};

// 0-based sample ranks of the requested quantiles, passed to the summary kernel by value.
struct SummaryRanks {
    int32_t n;
    int32_t r[SMC_MAX_PROBS];
};

struct PendingCopy {
    void* dst;
    const void* src;
    size_t bytes;
};

// Owned copy of one problem, with FP32 images of the data.
struct Spectrum {
    smc_problem prob{};
    std::vector<double> x, y;
    std::vector<float> xf, yf;
    std::vector<smc_prior> ppk;
    std::vector<double> mref;        // XRD reference positions
    std::vector<float> mref_f;
    void assign(const smc_problem& p);
};

const KernelTable& kernels();
int params_per_peak(int peak_kind);
int params_bg(int bg_kind);
smc_prior component_prior(const smc_problem& p, int K, int j);
smc_status validate(const smc_problem* p, const smc_options* o);
double energy_constant(const smc_problem& p);
DevPrior dev_prior(const smc_prior& p);
bool xps_model(const smc_problem& p);
void model_consts(const smc_problem& p, int K, GroupDesc& g);
Tile choose_tile(const smc_problem& p, int64_t chains, int forced_lanes);
bool tile_has_kernels(const smc_problem& p, const Tile& t);
size_t move_lds_bytes(const Tile& t, int d, int peak_kind, int noise_kind);
size_t energy_lds_bytes(const Tile& t, int d);
void build_work(const std::vector<int>& groups, const std::vector<int>& chains_of, const Tile& t,
                std::vector<MoveWork>& out);
hipError_t launch_tiled(const void* fn, const Tile& t, int n_work, size_t lds, const GroupDesc* groups,
                        const MoveWork* work, hipStream_t s);
size_t group_bytes(int d, int P, int M, int max_stages);
size_t spectrum_bytes(const smc_problem& p, const smc_options& o);
bool describe_spectrum(const Spectrum& sp, const smc_options& o, Arena& arena, GroupState* d_states_base,
                       int first_state, std::vector<GroupDesc>& out, std::vector<PendingCopy>& copies);
hipError_t upload_group_tables(const Spectrum& sp, const std::vector<GroupDesc>& gs, size_t first, size_t count,
                               hipStream_t s, std::vector<std::vector<char>>& keep);
bool device_ok();

// launchers defined in stage.hip
struct StageLaunch {
    const GroupDesc* groups;  // device array of n_groups descriptors
    int n_groups, max_p, max_m, max_d;
};
hipError_t launch_stage(const StageLaunch& L, hipStream_t s);
hipError_t launch_search_hook(const GroupDesc* group, int P, hipStream_t s);
hipError_t launch_resample_hook(const GroupDesc* group, int P, int M, uint32_t r, int32_t* anc, hipStream_t s);
hipError_t launch_steps_hook(const GroupDesc* group, int d, hipStream_t s);
int stage_final_parity();
size_t stage_scratch_bytes(int P);
bool carve_stage_scratch(Arena& a, int P, GroupDesc& g);
hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_draw(const GroupDesc* groups, int group, int64_t n_draws, hipStream_t s);
hipError_t launch_draw_items(const GroupDesc* groups, const MoveWork* items, int n_items, hipStream_t s);

// summary.hip
hipError_t launch_relabel(const float* in, float* out, int P, int d, int n_peaks, int np, hipStream_t s);
hipError_t launch_summary(const float* theta, int P, int d, const SummaryRanks& ranks, double* mean, float* quant,
                          hipStream_t s);
smc_status posterior_summary(const float* theta, int d, int P, int n_peaks, int np, const double* probs,
                             int n_probs, double* mean, double* quant, hipStream_t s);

}  // namespace smc
