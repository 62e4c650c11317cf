// smc_types.hpp -- data layout shared by the host driver and the kernels.
//
// One "group" is the SMC sampler of one (spectrum, K) pair: its particles,
// adaptation state and tempering state live in device memory and are described
// by a GroupDesc.  All kernels index groups through a device array of
// descriptors, so one launch can serve any mix of spectra and peak counts.
#pragma once

#include <stdint.h>

#include "smc.h"

namespace smc {

enum { kPurposeInit = 1, kPurposeResample = 2, kPurposeMove = 3 };

// Prior of one component in FP32 with the constant its log-density ratio needs:
// gamma: c = shape - 1 (a = shape, b = rate); normal: c = 1 / (2 sd^2) (a = mean, b = sd);
// uniform: a = lo, b = hi; fixed: a = value.  The support is the open interval (lo, hi):
// (a, b) uniform, (0, +inf) gamma, (-inf, +inf) normal (so NaN and infinities fall outside).
struct DevPrior {
    int32_t kind;
    float a, b, c;
    float lo, hi;
};
constexpr int kPriorFloats = static_cast<int>(sizeof(DevPrior) / sizeof(float));   // LDS floats per prior

// Tempering state of a group (device resident).
struct GroupState {
    double beta;      // inverse temperature of the particles' current target
    double logz;      // running log Z without the likelihood's constant
    double delta, ess, lse;
    int32_t stage;    // stages completed (0 = prior draws only)
    int32_t done;     // 1 once the final move at beta = 1 has run
    int32_t status;   // SMC_OK or SMC_ENUMERIC
    int32_t pad;
    unsigned long long evals;         // likelihood evaluations of Metropolis proposals
    unsigned long long evals_linear;  // of which a linear coefficient changed (cached shapes)
};

constexpr int kTraceCols = 6;  // beta, delta, ess, lse, logz, acceptance

// Points per lane of the move / energy tiles.  A tile of PPL points per lane serves the N
// with ceil(N / lanes) in (ppl_before(PPL), PPL]: its first ppl_before(PPL) rows of points
// are full for every such N, only the rows after them can hold padding.
constexpr int kNumPpl = 16;
constexpr int kPplOf[kNumPpl] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32};
constexpr int ppl_before(int ppl) {
    int b = 0;
    for (int i = 0; i < kNumPpl; ++i)
        if (kPplOf[i] < ppl) b = kPplOf[i];
    return b;
}

// The stage kernels split each group's P particles into chunks of kStageChunk.
constexpr int kStageChunk = 4096;
constexpr int kStagePartVals = 6;  // partial sums per chunk

// State of the temperature search of one stage (double-buffered by launch parity).
enum { kPhaseH = 0, kPhaseNewton = 1, kPhaseDone = 2, kPhaseFail = 3 };
struct StageNewton {
    double x, L, U, delta, emin, target, lt, mean, var, nfin;
    unsigned long long Q;   // total of the quantised weights
    int32_t phase, iter;
};

struct GroupDesc {
    // model
    int32_t n, K, d, np, nbg, peak_kind, bg_kind, noise_kind;
    float inv2s2;               // 1 / (2 sigma^2) for Gaussian noise
    int32_t pad0;
    float hn[3];                // s0^2, s1^2, s2^2 of heteroscedastic noise
    int32_t pad2;
    const float* x;             // [n]
    const float* y;             // [n]
    const DevPrior* prior;      // [d]
    // particles
    int32_t P, M, n_moves, waste_free;
    float* theta;               // [d][P]
    float* energy;              // [P]
    float* start;               // [d][M] resampled start states of the move
    float* start_e;             // [M]
    unsigned long long* cdf;    // [P] integer CDF scratch
    double* lambda;             // [d] step-size multipliers
    float* step;                // [d] random-walk scales of the current stage
    uint32_t* acc;              // [d] accepted proposals of the last move
    GroupState* st;
    double* trace;              // [max_stages][kTraceCols]
    double rho;
    int32_t bisect_iters, max_stages;
    uint32_t key0, key1;
    int32_t kidx, pad1;
    // stage-kernel scratch
    double* part;               // [2][nchunk][kStagePartVals] chunk partial sums
    StageNewton* nst;           // [2] temperature-search state
    unsigned long long* ctot;   // [nchunk] integer weight totals, then their exclusive prefix
    int32_t nchunk, pad3;
    const float* mu_ref;        // XRD peaks: reference positions [K]
};

// Waves per SIMD the register allocator is asked to leave room for.  The cached
// point state grows with PPL (x, D and the shapes: one for a Gaussian peak, two
// for a pseudo-Voigt peak; y too and the deviance's temporaries for Poisson
// counts); these limits are the largest that compile without spilling on gfx950
// (pseudo-Voigt with Poisson counts at 32 points per lane spills a few words).  A chain
// of several wavefronts (the cross-wave reduction) needs a few more registers: one wave
// less where the limit is 4 or 5.
constexpr int move_min_waves(int peak, int noise, int points, int wpc) {
    int w = 2;
    if (noise == SMC_NOISE_GAUSS) {
        if (peak == SMC_PEAK_GAUSS) w = points <= 16 ? 5 : (points <= 20 ? 4 : (points <= 24 ? 3 : 2));
        else w = points <= 10 ? 5 : (points <= 16 ? 4 : (points <= 20 ? 3 : 2));
    } else if (peak == SMC_PEAK_GAUSS) {
        w = points <= 8 ? 5 : (points <= 14 ? 4 : (points <= 20 ? 3 : 2));
    } else {
        w = points <= 7 ? 5 : (points <= 12 ? 4 : (points <= 16 ? 3 : 2));
    }
    return wpc > 1 && w >= 4 ? w - 1 : w;
}

// The XPS (Shirley) and XRD move kernels, by points per lane.
constexpr int xps_min_waves(int points) { return points <= 5 ? 4 : (points <= 8 ? 3 : 2); }
constexpr int xrd_min_waves(int points) { return points <= 6 ? 4 : (points <= 14 ? 3 : 2); }

// Bytes of LDS per lane and point where a move kernel keeps the shapes of the current
// proposal (an accepted shape proposal then copies them instead of evaluating them again):
// 4 (one shape: Gaussian peak) or 8 (two: pseudo-Voigt, XRD), or 0 where the workgroups
// that the kernel's register budget lets run on one CU would need more than 128 KB of the
// CU's 160 KB for them (a 256-thread workgroup is one wave per SIMD; 512 threads two).
constexpr int move_shape_lds_bytes(int peak_kind, int noise_kind, int ppl, int lanes) {
    const int threads = lanes > 64 ? lanes : 256;
    const int wpc = lanes > 64 ? lanes / 64 : 1;
    const int waves = peak_kind == SMC_PEAK_XRD ? xrd_min_waves(ppl)
                      : noise_kind == SMC_NOISE_HETERO ? xps_min_waves(ppl)
                                                       : move_min_waves(peak_kind, noise_kind, ppl, wpc);
    const int wgs = waves * 256 / threads > 1 ? waves * 256 / threads : 1;
    const int b = peak_kind == SMC_PEAK_GAUSS ? 4 : 8;
    return wgs * threads * ppl * b <= 131072 ? b : 0;
}

// Bytes of LDS per lane and point where the XRD move kernel keeps the reciprocal of each
// count from 10 to 16 points per lane (registers hold them up to 8; at 20 the kernel is at
// its register limit and the LDS reads cost more spills than the v_rcp they replace: 2%
// slower): 4, or 0 where the workgroups its register budget lets run on one CU would need
// more than 128 KB for them and the shapes together.
constexpr int move_iw_lds_bytes(int peak_kind, int ppl, int lanes) {
    if (peak_kind != SMC_PEAK_XRD || ppl <= 8 || ppl > 16) return 0;
    const int threads = lanes > 64 ? lanes : 256;
    const int waves = xrd_min_waves(ppl);
    const int wgs = waves * 256 / threads > 1 ? waves * 256 / threads : 1;
    const int sb = move_shape_lds_bytes(peak_kind, SMC_NOISE_POISSON, ppl, lanes);
    return wgs * threads * ppl * (sb + 4) <= 131072 ? 4 : 0;
}

// One workgroup of the move / energy kernels: chains [chain0, chain0 + nchains) of a group.
struct MoveWork {
    int32_t group, chain0, nchains, pad;
};

}  // namespace smc
