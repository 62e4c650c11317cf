// stage.hip -- the per-stage bookkeeping of the tempered SMC sampler, entirely on the
// device, as a pipeline of chunk-parallel launches (described below, before the kernels):
//
//   1. step-size multipliers lambda_j from the previous move's acceptance;
//   2. the next inverse-temperature increment delta from the ESS of the incremental
//      weights w_i = exp(-delta E_i) (Eq. smc_incremental_weight), defined by bisection;
//   3. log-sum-exp, ESS and the evidence increment LSE - ln P
//      (Eq. smc_marginal_likelihood), all in FP64;
//   4. systematic resampling of M ancestors on weights quantised to 2^-52
//      (integer CDF, 128-bit positions, so the ancestors are exact);
//   5. gather of the ancestors into the move's start buffer and the
//      random-walk scales s_j = lambda_j * sd_j over the resampled states.
// Plus the small kernels behind the per-kernel hooks, which run the same kernels.
#include <algorithm>

#include "host_common.hpp"
#include "smc_device.hpp"

namespace smc {

// FP64 sums and minima over the 64 lanes of a wavefront (the stage kernels), the same bits
// in every lane: each 64-bit exchange is two 32-bit DPP moves inside 16-lane rows, then the
// permlane swaps across rows and halves (VALU only; a shuffle through ds_bpermute costs an
// LDS round trip per step).
template <int CTRL>
__device__ __forceinline__ double dpp_swap64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b)), CTRL, 0xF, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(b >> 32)), CTRL, 0xF, 0xF, false));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// The two values of v that a permlane swap pairs (rows 2r and 2r+1 for the 16-lane swap,
// the two halves for the 32-lane one), in the same order in every lane; the empty asm keeps
// the compiler from folding the pair (see swap_sum).
template <bool HALVES>
__device__ __forceinline__ void swap_pair64(double v, double& a, double& b) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = static_cast<unsigned>(u), hi = static_cast<unsigned>(u >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (HALVES) {
        const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = pl[0]; l1 = pl[1]; h0 = ph[0]; h1 = ph[1];
    } else {
        const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = pl[0]; l1 = pl[1]; h0 = ph[0]; h1 = ph[1];
    }
    asm volatile("" : "+v"(l0), "+v"(l1), "+v"(h0), "+v"(h1));
    a = __builtin_bit_cast(double, (static_cast<uint64_t>(h0) << 32) | l0);
    b = __builtin_bit_cast(double, (static_cast<uint64_t>(h1) << 32) | l1);
}

__device__ __forceinline__ double wave_sum64(double v) {
    v += dpp_swap64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_swap64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_swap64<0x141>(v);  // row_half_mirror
    v += dpp_swap64<0x140>(v);  // row_mirror
    double a, b;
    swap_pair64<false>(v, a, b);
    v = a + b;
    swap_pair64<true>(v, a, b);
    return a + b;
}

__device__ __forceinline__ double wave_min64(double v) {
    v = fmin(v, dpp_swap64<0xB1>(v));
    v = fmin(v, dpp_swap64<0x4E>(v));
    v = fmin(v, dpp_swap64<0x141>(v));
    v = fmin(v, dpp_swap64<0x140>(v));
    double a, b;
    swap_pair64<false>(v, a, b);
    v = fmin(a, b);
    swap_pair64<true>(v, a, b);
    return fmin(a, b);
}

// Inclusive prefix sum of a 64-bit integer over the 64 lanes of a wavefront (exact): shifts
// by 1, 2, 4, 8 lanes inside each 16-lane row, then each row total broadcast into the rows
// after it (DPP row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).  Lanes that a
// shift or a row mask leaves out receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(v)), CTRL, ROWS, 0xF, false));
    const uint32_t hi = static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(v >> 32)), CTRL, ROWS, 0xF, false));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    v += dpp_u64<0x111, 0xF>(v);   // row_shr:1
    v += dpp_u64<0x112, 0xF>(v);   // row_shr:2
    v += dpp_u64<0x114, 0xF>(v);   // row_shr:4
    v += dpp_u64<0x118, 0xF>(v);   // row_shr:8
    v += dpp_u64<0x142, 0xA>(v);   // row_bcast:15
    v += dpp_u64<0x143, 0xC>(v);   // row_bcast:31
    return v;
}

constexpr int kStageThreads = 1024;
constexpr int kStageWaves = kStageThreads / 64;

struct StageShared {
    double red[4][kStageWaves];
    unsigned long long scan[kStageWaves];
    unsigned long long total;
};

// Sums of up to four FP64 values over the workgroup; every thread receives the same bits.
template <int NV>
__device__ inline void block_sum(double* v, StageShared& sh) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum64(v[q]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) sh.red[q][w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int k = 0; k < kStageWaves; ++k) s += sh.red[q][k];
        v[q] = s;
    }
}

// Weight sums at increment delta, with a_i = E_i - min E and w_i = exp(-delta a_i):
// s[0] = sum w, s[1] = sum w^2, and with NV = 4 also s[2] = sum a w, s[3] = sum a w^2.
template <int NV>
__device__ inline void weight_sums(const float* E, int P, double emin, double delta, double* s, StageShared& sh) {
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = 0.0;
    for (int i = threadIdx.x; i < P; i += kStageThreads) {
        const double a = static_cast<double>(E[i]) - emin;
        const double w = exp(-delta * a);
        s[0] += w;
        s[1] += w * w;
        if constexpr (NV == 4) {
            const double aw = w > 0.0 ? a * w : 0.0;
            s[2] += aw;
            s[3] += aw * w;
        }
    }
    block_sum<NV>(s, sh);
}

struct BisectOut {
    double delta, ess, lse, emin, s1;
    int ok;
};

// The next increment, defined as the result of `iters` halvings of [0, 1 - beta]
// that keep the low end where ESS >= rho P (all of 1 - beta if ESS there already
// qualifies; the final high end if no tested point qualified).
//
// The halvings are replayed, not evaluated one by one.  g(delta) = ln ESS(delta) -
// ln(rho P) is non-increasing (the weights exp(-delta a) concentrate as delta
// grows), so Newton's method on g, kept inside a bracket [L, U] with g(L) >= 0 >
// g(U) and started from the small-delta expansion ESS/P ~ 1/(1 + delta^2 Var E),
// converges to the root r in a few passes (g' = 2 (sum a w^2 / sum w^2 - sum a w /
// sum w) comes from the same pass).  Each halving then keeps the low end iff its
// midpoint is <= r.  This reproduces the halvings except where the FP64 rounding
// of the weight sums decides ESS(mid) >= rho P, which is equally true of any
// implementation of them.  Without convergence (not seen) the midpoints are
// evaluated one by one.
__device__ inline BisectOut bisect(const float* E, int P, double beta, double rho, int iters, StageShared& sh) {
    BisectOut o;
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // NaN flag, finite count, sum E, sum E^2 (finite E)
    double emin = __builtin_inf();
    for (int i = threadIdx.x; i < P; i += kStageThreads) {
        const float e = E[i];
        if (__builtin_isnan(e)) v[0] = 1.0;
        if (__builtin_isfinite(e)) {
            const double x = static_cast<double>(e);
            v[1] += 1.0;
            v[2] += x;
            v[3] += x * x;
        }
        emin = fmin(emin, static_cast<double>(e));
    }
    emin = wave_min64(emin);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh.red[3][threadIdx.x >> 6] = emin;  // read before block_sum reuses red
    __syncthreads();
    {
        double m = sh.red[3][0];
        for (int k = 1; k < kStageWaves; ++k) m = fmin(m, sh.red[3][k]);
        emin = m;
    }
    block_sum<4>(v, sh);
    const bool nan = v[0] != 0.0;
    const double nfin = v[1];
    o.emin = emin;
    o.ok = !nan && emin < __builtin_inf();
    if (!o.ok) {
        o.delta = o.ess = o.lse = o.s1 = 0.0;
        return o;
    }
    const double target = rho * static_cast<double>(P);
    const double H = 1.0 - beta;
    double s[4];
    weight_sums<2>(E, P, emin, H, s, sh);
    double delta;
    if (s[0] * s[0] / s[1] >= target) {
        delta = H;
    } else if (nfin < target) {
        // ESS(delta) <= number of finite energies < rho P for every delta > 0: every halving
        // keeps the high end, which ends at H / 2^iters (exact in FP64)
        double hi = H;
        for (int it = 0; it < iters; ++it) hi = 0.5 * (0.0 + hi);
        delta = hi;
        weight_sums<2>(E, P, emin, delta, s, sh);
    } else {
        const double lt = log(target);
        const double mean = v[2] / nfin;
        const double var = fmax(v[3] / nfin - mean * mean, 0.0);
        double L = 0.0, U = H;
        double x = var > 0.0 ? sqrt((1.0 / rho - 1.0) / var) : 0.5 * H;
        if (!(x > L && x < U)) x = 0.5 * H;
        double r = -1.0;
        for (int it = 0; it < 40; ++it) {
            weight_sums<4>(E, P, emin, x, s, sh);
            const double g = 2.0 * log(s[0]) - log(s[1]) - lt;
            const double gp = 2.0 * (s[3] / s[1] - s[2] / s[0]);
            if (g >= 0.0) L = x;
            else U = x;
            const bool newton = gp < 0.0;
            const double step = newton ? -g / gp : 0.0;
            if (newton && fabs(step) <= 4e-16 * x) {
                r = fmin(fmax(x + step, L), U);
                break;
            }
            if (U - L <= 1e-15 * U) {
                r = 0.5 * (L + U);
                break;
            }
            double xn = x + step;
            if (!newton || !(xn > L && xn < U)) xn = L > 0.0 ? sqrt(L * U) : 0.125 * U;
            x = xn;
        }
        double lo = 0.0, hi = H;
        for (int it = 0; it < iters; ++it) {
            const double mid = 0.5 * (lo + hi);
            bool keep_low;
            if (r >= 0.0) {
                keep_low = mid <= r;
            } else {
                weight_sums<2>(E, P, emin, mid, s, sh);
                keep_low = s[0] * s[0] / s[1] >= target;
            }
            if (keep_low) lo = mid;
            else hi = mid;
        }
        delta = lo > 0.0 ? lo : hi;
        weight_sums<2>(E, P, emin, delta, s, sh);
    }
    o.delta = delta;
    o.ess = s[0] * s[0] / s[1];
    o.lse = -delta * emin + log(s[0]);
    o.s1 = s[0];
    return o;
}

// floor((m 2^32 + r) Q / (M 2^32)) with a 128-bit product and base-2^32 long division.
__device__ inline unsigned long long position(uint32_t m, uint32_t r, unsigned long long Q, uint32_t M) {
    const unsigned long long a = (static_cast<unsigned long long>(m) << 32) | r;
    const unsigned long long lo = a * Q;
    const unsigned long long hi = __umul64hi(a, Q);
    // (hi:lo) >> 32 as three 32-bit limbs, most significant first
    const unsigned long long l2 = hi >> 32, l1 = hi & 0xffffffffull, l0 = lo >> 32;
    unsigned long long rem = l2 % M;
    unsigned long long x = (rem << 32) | l1;
    const unsigned long long q1 = x / M;
    rem = x % M;
    x = (rem << 32) | l0;
    const unsigned long long q0 = x / M;
    return (q1 << 32) + q0;
}

// First j with cdf[j] > pos.
__device__ inline int ancestor(const unsigned long long* cdf, int P, unsigned long long pos) {
    int lo = 0, hi = P - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > pos) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// ==================================================================== stage pipeline
//
// One stage of all groups runs as a short sequence of launches over (group, chunk)
// workgroups of kChunkThreads threads, each chunk kStageChunk particles, so a stage of
// one group uses as many CUs as it has chunks.  The launch boundaries order the steps;
// every reduction over chunks is done in chunk order, redundantly by each workgroup
// that needs it, so all of them see the same bits:
//   stats   per chunk: NaN flag, finite count, sum E, sum E^2, min E; chunk 0 also applies
//           the step-size multipliers of the last move and ends finished groups;
//   search  kNewtonLaunches launches: reduce the previous launch's chunk sums, advance the
//           temperature search (ESS at 1 - beta, then the bracketed Newton iteration of
//           bisect()), and form the chunk sums at the next trial increment;
//   finish  one workgroup per group that the search left unconverged: bisect() in full;
//   weights w_i = exp(-delta (E_i - min E)), kept in the CDF buffer, and their chunk sums;
//   evidence + quantise: ESS, LSE, log Z, trace (chunk 0), then q_i = floor(w_i 2^52 / sum w)
//           with an inclusive scan inside the chunk and the chunk's total;
//   offsets exclusive prefix of the chunk totals (one workgroup per group);
//   resample the ancestor of each of the M positions (search over chunk offsets, then
//           inside the chunk) and the gather of its state into the move's start buffer;
//   steps   the random-walk scale of each component over the resampled states.

constexpr int kChunkThreads = 256;
constexpr int kChunkWaves = kChunkThreads / 64;
constexpr int kPerThread = kStageChunk / kChunkThreads;
constexpr int kNewtonLaunches = 10;

__device__ inline StageNewton* nst_buf(const GroupDesc& g, int parity) { return g.nst + (parity & 1); }
__device__ inline double* part_buf(const GroupDesc& g, int parity) {
    return g.part + static_cast<size_t>(parity & 1) * g.nchunk * kStagePartVals;
}

// Sum of NV doubles over the chunk workgroup (fixed order); the result in every thread.
template <int NV>
__device__ inline void chunk_block_sum(double* v, double (*red)[kChunkWaves]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum64(v[q]);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q][w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kChunkWaves; ++k) s += red[q][k];
        v[q] = s;
    }
}

// Reduce the chunk partials parts[c][0..NV) over c = 0..nchunk-1: thread t adds chunks
// t, t + 256, ... in order, then the fixed block tree.  Value NV-1 is a minimum when
// MIN_LAST is set.
template <int NV, bool MIN_LAST>
__device__ inline void reduce_parts(const double* parts, int nchunk, double* out, double (*red)[kChunkWaves]) {
    if (nchunk == 1) {
        // one chunk: what the tree below returns for it (its partials plus zeros, or the
        // minimum with +inf), without the block reduction
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] = (MIN_LAST && q == NV - 1) ? fmin(__builtin_inf(), parts[q]) : 0.0 + parts[q];
        return;
    }
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = (MIN_LAST && q == NV - 1) ? __builtin_inf() : 0.0;
    for (int c = threadIdx.x; c < nchunk; c += kChunkThreads) {
        const double* p = parts + static_cast<size_t>(c) * kStagePartVals;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            if (MIN_LAST && q == NV - 1) v[q] = fmin(v[q], p[q]);
            else v[q] += p[q];
        }
    }
    if constexpr (MIN_LAST) {
        double m = v[NV - 1];
        m = wave_min64(m);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = m;
        __syncthreads();
        m = red[0][0];
#pragma unroll
        for (int k = 1; k < kChunkWaves; ++k) m = fmin(m, red[0][k]);
        v[NV - 1] = 0.0;
        chunk_block_sum<NV>(v, red);
        v[NV - 1] = m;
    } else {
        chunk_block_sum<NV>(v, red);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = v[q];
}

// Weight sums of this workgroup's chunk at increment x (NV = 2: sum w, sum w^2; NV = 4
// also sum a w, sum a w^2 with a = E - emin); optionally keeps w_i in `keep`.
template <int NV>
__device__ inline void chunk_weight_sums(const float* E, int i0, int i1, double emin, double x, double* out,
                                         double* keep, double (*red)[kChunkWaves]) {
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
#pragma unroll 4
    for (int k = 0; k < kPerThread; ++k) {
        const int i = i0 + k * kChunkThreads + static_cast<int>(threadIdx.x);
        if (i < i1) {
            const double a = static_cast<double>(E[i]) - emin;
            const double w = exp(-x * a);
            v[0] += w;
            v[1] += w * w;
            if constexpr (NV == 4) {
                const double aw = w > 0.0 ? a * w : 0.0;
                v[2] += aw;
                v[3] += aw * w;
            }
            if (keep) keep[i] = w;
        }
    }
    chunk_block_sum<NV>(v, red);
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = v[q];
}

// One step of the temperature search from the sums at the last trial point (same rules
// as bisect()).  it == 0: `sums` are the stats {NaN flag, finite count, sum E, sum E^2, min E}.
__device__ inline StageNewton search_step(const GroupDesc& g, StageNewton s, const double* sums, int it,
                                          double beta) {
    const int P = g.P;
    if (it == 0) {
        s = StageNewton{};
        s.nfin = sums[1];
        s.emin = sums[4];
        if (sums[0] != 0.0 || !(s.emin < __builtin_inf())) {
            s.phase = kPhaseFail;
            return s;
        }
        s.mean = sums[2] / s.nfin;
        s.var = fmax(sums[3] / s.nfin - s.mean * s.mean, 0.0);
        s.target = g.rho * static_cast<double>(P);
        s.lt = log(s.target);
        s.U = 1.0 - beta;
        s.x = s.U;
        s.phase = kPhaseH;
        return s;
    }
    const double H = 1.0 - beta;
    if (s.phase == kPhaseH) {
        if (sums[0] * sums[0] / sums[1] >= s.target) {
            s.delta = H;
            s.phase = kPhaseDone;
        } else if (s.nfin < s.target) {
            double hi = H;
            for (int k = 0; k < g.bisect_iters; ++k) hi = 0.5 * (0.0 + hi);
            s.delta = hi;
            s.phase = kPhaseDone;
        } else {
            s.L = 0.0;
            s.U = H;
            double x = s.var > 0.0 ? sqrt((1.0 / g.rho - 1.0) / s.var) : 0.5 * H;
            if (!(x > s.L && x < s.U)) x = 0.5 * H;
            s.x = x;
            s.iter = 0;
            s.phase = kPhaseNewton;
        }
        return s;
    }
    if (s.phase != kPhaseNewton) return s;
    const double x = s.x;
    const double gv = 2.0 * log(sums[0]) - log(sums[1]) - s.lt;
    const double gp = 2.0 * (sums[3] / sums[1] - sums[2] / sums[0]);
    if (gv >= 0.0) s.L = x;
    else s.U = x;
    const bool newton = gp < 0.0;
    const double step = newton ? -gv / gp : 0.0;
    double r = -1.0;
    if (newton && fabs(step) <= 4e-16 * x) r = fmin(fmax(x + step, s.L), s.U);
    else if (s.U - s.L <= 1e-15 * s.U) r = 0.5 * (s.L + s.U);
    if (r >= 0.0) {
        double lo = 0.0, hi = H;
        for (int k = 0; k < g.bisect_iters; ++k) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= r) lo = mid;
            else hi = mid;
        }
        s.delta = lo > 0.0 ? lo : hi;
        s.phase = kPhaseDone;
        return s;
    }
    double xn = x + step;
    if (!newton || !(xn > s.L && xn < s.U)) xn = s.L > 0.0 ? sqrt(s.L * s.U) : 0.125 * s.U;
    s.x = xn;
    ++s.iter;
    return s;
}

// chunk index range of workgroup (group, c)
__device__ inline void chunk_range(const GroupDesc& g, int c, int& i0, int& i1) {
    i0 = c * kStageChunk;
    i1 = min(g.P, i0 + kStageChunk);
}

// Step-size adaptation after a move (one workgroup, thread j for component j):
// lambda_j <- clamp(lambda_j exp(acc_j - 0.44), 0.01, 10) with acc_j the acceptance rate of
// component j over the move's M n proposals, the counters cleared, and the stage's mean
// acceptance over the free components into the trace.  Before the first move (stage 0) only
// the counters are cleared.
__device__ inline void st_adapt(const GroupDesc& g, int stage_prev, double (*red)[kChunkWaves]) {
    if (stage_prev > 0) {
        const double props = static_cast<double>(g.M) * g.n_moves;
        double v[2] = {0.0, 0.0};   // sum of acceptance rates, free components
        for (int j = threadIdx.x; j < g.d; j += kChunkThreads) {
            if (g.prior[j].kind == SMC_PRIOR_FIXED) continue;
            const double a = g.acc[j] / props;
            v[0] += a;
            v[1] += 1.0;
            g.lambda[j] = fmin(10.0, fmax(0.01, g.lambda[j] * exp(a - 0.44)));
            g.acc[j] = 0u;
        }
        chunk_block_sum<2>(v, red);
        if (threadIdx.x == 0 && stage_prev <= g.max_stages)
            g.trace[(stage_prev - 1) * kTraceCols + 5] = v[1] > 0.0 ? v[0] / v[1] : 0.0;
    } else {
        for (int j = threadIdx.x; j < g.d; j += kChunkThreads) g.acc[j] = 0u;
    }
}

__device__ inline void st_stats(const GroupDesc* __restrict__ groups, int gi, int c) {
    const GroupDesc& g = groups[gi];
    GroupState* st = g.st;
    if (c >= g.nchunk || st->done) return;
    __shared__ double red[kStagePartVals][kChunkWaves];
    if (c == 0) {
        // step sizes adapt to the last move; end finished groups
        const int stage_prev = st->stage;
        st_adapt(g, stage_prev, red);
        if (threadIdx.x == 0 && (st->beta >= 1.0 || stage_prev >= g.max_stages)) {
            if (st->beta < 1.0) st->status = SMC_ENUMERIC;
            st->done = 1;
        }
    }
    int i0, i1;
    chunk_range(g, c, i0, i1);
    double v[5] = {0.0, 0.0, 0.0, 0.0, __builtin_inf()};
#pragma unroll 4
    for (int k = 0; k < kPerThread; ++k) {
        const int i = i0 + k * kChunkThreads + static_cast<int>(threadIdx.x);
        if (i < i1) {
            const float e = g.energy[i];
            if (__builtin_isnan(e)) v[0] = 1.0;
            if (__builtin_isfinite(e)) {
                const double x = static_cast<double>(e);
                v[1] += 1.0;
                v[2] += x;
                v[3] += x * x;
            }
            v[4] = fmin(v[4], static_cast<double>(e));
        }
    }
    double m = v[4];
    m = wave_min64(m);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[5][threadIdx.x >> 6] = m;
    chunk_block_sum<4>(v, red);
    if (threadIdx.x == 0) {
        m = red[5][0];
#pragma unroll
        for (int k = 1; k < kChunkWaves; ++k) m = fmin(m, red[5][k]);
        double* out = part_buf(g, 0) + static_cast<size_t>(c) * kStagePartVals;
        for (int q = 0; q < 4; ++q) out[q] = v[q];
        out[4] = m;
    }
}

__global__ void __launch_bounds__(kChunkThreads) k_st_stats(const GroupDesc* __restrict__ groups, int maxch) {
    st_stats(groups, blockIdx.x / maxch, blockIdx.x % maxch);
}

__device__ inline void st_search(const GroupDesc* __restrict__ groups, int gi, int c, int it) {
    const GroupDesc& g = groups[gi];
    GroupState* st = g.st;
    if (c >= g.nchunk || st->done) return;
    __shared__ double red[kStagePartVals][kChunkWaves];
    __shared__ StageNewton s_nst;
    StageNewton prev{};
    if (it > 0) {
        prev = *nst_buf(g, it);
        if (prev.phase == kPhaseDone || prev.phase == kPhaseFail) {
            if (c == 0 && threadIdx.x == 0) *nst_buf(g, it + 1) = prev;
            return;
        }
    }
    double sums[5];
    if (it == 0) reduce_parts<5, true>(part_buf(g, 0), g.nchunk, sums, red);
    else reduce_parts<4, false>(part_buf(g, it), g.nchunk, sums, red);
    if (threadIdx.x == 0) {
        const StageNewton ns = search_step(g, prev, sums, it, st->beta);
        s_nst = ns;
        if (c == 0) {
            *nst_buf(g, it + 1) = ns;
            if (ns.phase == kPhaseFail) {
                st->status = SMC_ENUMERIC;
                st->done = 1;
            }
        }
    }
    __syncthreads();
    const StageNewton ns = s_nst;
    if (ns.phase != kPhaseH && ns.phase != kPhaseNewton) return;
    int i0, i1;
    chunk_range(g, c, i0, i1);
    double out[4];
    if (ns.phase == kPhaseH) {
        chunk_weight_sums<2>(g.energy, i0, i1, ns.emin, ns.x, out, nullptr, red);
        out[2] = out[3] = 0.0;
    } else {
        chunk_weight_sums<4>(g.energy, i0, i1, ns.emin, ns.x, out, nullptr, red);
    }
    if (threadIdx.x == 0) {
        double* p = part_buf(g, it + 1) + static_cast<size_t>(c) * kStagePartVals;
        for (int q = 0; q < 4; ++q) p[q] = out[q];
    }
}

__global__ void __launch_bounds__(kChunkThreads) k_st_search(const GroupDesc* __restrict__ groups, int maxch, int it) {
    st_search(groups, blockIdx.x / maxch, blockIdx.x % maxch, it);
}

// Groups whose search did not converge within the launches: the full search in one
// workgroup (bisect() from the start; rare: 4 of 125 stages of the N = 201, P = 512
// three-Gaussian runs, 50-100 us each, an idle launch of ~5 us otherwise).
__global__ void __launch_bounds__(kStageThreads) k_st_finish(const GroupDesc* __restrict__ groups) {
    const GroupDesc& g = groups[blockIdx.x];
    GroupState* st = g.st;
    if (st->done) return;
    StageNewton* fin = nst_buf(g, kNewtonLaunches);
    if (fin->phase == kPhaseDone) return;
    __shared__ StageShared sh;
    const BisectOut b = bisect(g.energy, g.P, st->beta, g.rho, g.bisect_iters, sh);
    if (threadIdx.x == 0) {
        if (!b.ok) {
            fin->phase = kPhaseFail;
            st->status = SMC_ENUMERIC;
            st->done = 1;
        } else {
            fin->delta = b.delta;
            fin->emin = b.emin;
            fin->phase = kPhaseDone;
        }
    }
}

__device__ inline void st_weights(const GroupDesc* __restrict__ groups, int gi, int c) {
    const GroupDesc& g = groups[gi];
    if (c >= g.nchunk || g.st->done) return;
    __shared__ double red[kStagePartVals][kChunkWaves];
    const StageNewton fin = *nst_buf(g, kNewtonLaunches);
    int i0, i1;
    chunk_range(g, c, i0, i1);
    double out[2];
    chunk_weight_sums<2>(g.energy, i0, i1, fin.emin, fin.delta, out, reinterpret_cast<double*>(g.cdf), red);
    if (threadIdx.x == 0) {
        double* p = part_buf(g, 0) + static_cast<size_t>(c) * kStagePartVals;
        p[0] = out[0];
        p[1] = out[1];
    }
}

__global__ void __launch_bounds__(kChunkThreads) k_st_weights(const GroupDesc* __restrict__ groups, int maxch) {
    st_weights(groups, blockIdx.x / maxch, blockIdx.x % maxch);
}

// Evidence update (chunk 0) and the quantised weights with their scan inside the chunk.
// With unit_sum set the weights in the CDF buffer are taken as already normalised.
__device__ inline void st_quantise(const GroupDesc* __restrict__ groups, int gi, int c, int unit_sum) {
    const GroupDesc& g = groups[gi];
    GroupState* st = g.st;
    if (c >= g.nchunk || st->done) return;
    __shared__ double red[kStagePartVals][kChunkWaves];
    __shared__ unsigned long long s_scan[kChunkWaves];
    double sums[2];
    if (unit_sum) {
        sums[0] = 1.0;
        sums[1] = 1.0;
    } else {
        reduce_parts<2, false>(part_buf(g, 0), g.nchunk, sums, red);
    }
    const double s1 = sums[0];
    if (c == 0 && threadIdx.x == 0 && !unit_sum) {
        const StageNewton fin = *nst_buf(g, kNewtonLaunches);
        const double delta = fin.delta, beta = st->beta;
        double beta_new = (delta == 1.0 - beta) ? 1.0 : beta + delta;
        if (beta_new > 1.0) beta_new = 1.0;
        const double ess = s1 * s1 / sums[1];
        const double lse = -delta * fin.emin + log(s1);
        const int stage = st->stage + 1;
        st->logz += lse - log(static_cast<double>(g.P));
        st->beta = beta_new;
        st->delta = delta;
        st->ess = ess;
        st->lse = lse;
        st->stage = stage;
        if (stage <= g.max_stages) {
            double* tr = g.trace + (stage - 1) * kTraceCols;
            tr[0] = beta_new;
            tr[1] = delta;
            tr[2] = ess;
            tr[3] = lse;
            tr[4] = st->logz;
            tr[5] = 0.0;
        }
    }
    // thread t owns the kPerThread consecutive weights t*kPerThread.. of the chunk
    int i0, i1;
    chunk_range(g, c, i0, i1);
    const double* w = reinterpret_cast<const double*>(g.cdf);
    unsigned long long q[kPerThread];
    unsigned long long local = 0;
    const int base = i0 + static_cast<int>(threadIdx.x) * kPerThread;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int i = base + k;
        q[k] = i < i1 ? static_cast<unsigned long long>(floor(w[i] / s1 * 4503599627370496.0)) : 0ull;
        local += q[k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long incl = wave_incl_scan_u64(local);
    __syncthreads();   // every weight of the chunk read before any is overwritten
    if (lane == 63) s_scan[wv] = incl;
    __syncthreads();
    unsigned long long run = incl - local;
#pragma unroll
    for (int k = 0; k < kChunkWaves; ++k)
        if (k < wv) run += s_scan[k];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const int i = base + k;
        run += q[k];
        if (i < i1) g.cdf[i] = run;
    }
    if (threadIdx.x == kChunkThreads - 1) {
        unsigned long long tot = 0;
#pragma unroll
        for (int k = 0; k < kChunkWaves; ++k) tot += s_scan[k];
        g.ctot[c] = tot;
    }
}

__global__ void __launch_bounds__(kChunkThreads) k_st_quantise(const GroupDesc* __restrict__ groups, int maxch,
                                                               int unit_sum) {
    st_quantise(groups, blockIdx.x / maxch, blockIdx.x % maxch, unit_sum);
}

// Exclusive prefix of the chunk totals, in place, and their grand total Q (kept in the
// final search state).
__device__ inline void st_offsets(const GroupDesc* __restrict__ groups, int gi) {
    const GroupDesc& g = groups[gi];
    if (g.st->done) return;
    __shared__ unsigned long long s_scan[kChunkWaves];
    __shared__ unsigned long long s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c0 = 0; c0 < g.nchunk; c0 += kChunkThreads) {
        const int c = c0 + static_cast<int>(threadIdx.x);
        const unsigned long long v = c < g.nchunk ? g.ctot[c] : 0ull;
        const unsigned long long incl = wave_incl_scan_u64(v);
        if (lane == 63) s_scan[wv] = incl;
        __syncthreads();
        unsigned long long off = s_carry + incl - v;
#pragma unroll
        for (int k = 0; k < kChunkWaves; ++k)
            if (k < wv) off += s_scan[k];
        if (c < g.nchunk) g.ctot[c] = off;
        __syncthreads();
        if (threadIdx.x == kChunkThreads - 1) s_carry = off + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) nst_buf(g, kNewtonLaunches)->Q = s_carry;
}

__global__ void __launch_bounds__(kChunkThreads) k_st_offsets(const GroupDesc* __restrict__ groups) {
    st_offsets(groups, blockIdx.x);
}

// Ancestor of position m and the gather of its state.  r_fixed >= 0 replaces the drawn
// uniform (hook).  anc (optional) receives the ancestors.
__device__ inline void st_resample(const GroupDesc* __restrict__ groups, int gi, int mb, int64_t r_fixed,
                                   int32_t* __restrict__ anc) {
    const GroupDesc& g = groups[gi];
    GroupState* st = g.st;
    const int m = mb * kChunkThreads + static_cast<int>(threadIdx.x);
    if (st->done || m >= g.M) return;
    const StageNewton fin = *nst_buf(g, kNewtonLaunches);
    const unsigned long long Q = fin.Q;
    const uint32_t r = r_fixed >= 0 ? static_cast<uint32_t>(r_fixed)
                                    : draw(g.key0, g.key1, 0u, static_cast<uint32_t>(st->stage), 0u,
                                           static_cast<uint32_t>(g.K), kPurposeResample).x;
    const unsigned long long pos = position(static_cast<uint32_t>(m), r, Q, static_cast<uint32_t>(g.M));
    // chunk: the first c whose end (offset of c + 1, or Q) exceeds pos
    int lo = 0, hi = g.nchunk - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const unsigned long long end = mid + 1 < g.nchunk ? g.ctot[mid + 1] : Q;
        if (end > pos) hi = mid;
        else lo = mid + 1;
    }
    const unsigned long long rel = pos - g.ctot[lo];
    int i0, i1;
    chunk_range(g, lo, i0, i1);
    int a = i0 + ancestor(g.cdf + i0, i1 - i0, rel);
    if (anc) anc[m] = a;
    if (g.theta) {
        g.start_e[m] = g.energy[a];
        for (int j = 0; j < g.d; ++j) g.start[(size_t)j * g.M + m] = g.theta[(size_t)j * g.P + a];
    }
}

__global__ void __launch_bounds__(kChunkThreads) k_st_resample(const GroupDesc* __restrict__ groups, int mblocks,
                                                               int64_t r_fixed, int32_t* __restrict__ anc) {
    st_resample(groups, blockIdx.x / mblocks, blockIdx.x % mblocks, r_fixed, anc);
}

// Random-walk scales s_j = lambda_j * sd_j over the resampled states: one 256-thread
// workgroup per (group, component) (a fixed shape, so every path sums in the same order
// and gives the same bits), two passes (the mean, then the squared deviations) in FP64 with
// four accumulators per thread to keep several loads in flight.
__device__ inline void st_steps(const GroupDesc* __restrict__ groups, int gi, int j) {
    __shared__ double red[1][kChunkWaves];
    const GroupDesc& g = groups[gi];
    if (g.st->done || j >= g.d) return;
    if (g.prior[j].kind == SMC_PRIOR_FIXED) {
        if (threadIdx.x == 0) g.step[j] = 0.0f;
        return;
    }
    const int M = g.M;
    const float* col = g.start + (size_t)j * M;
    constexpr int kStride = 4 * kChunkThreads;
    double acc4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m0 = threadIdx.x; m0 < M; m0 += kStride)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (m0 + kChunkThreads * u < M) acc4[u] += col[m0 + kChunkThreads * u];
    double v[1] = {(acc4[0] + acc4[1]) + (acc4[2] + acc4[3])};
    chunk_block_sum<1>(v, red);
    const double mean = v[0] / M;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc4[u] = 0.0;
    for (int m0 = threadIdx.x; m0 < M; m0 += kStride)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (m0 + kChunkThreads * u < M) {
                const double dd = col[m0 + kChunkThreads * u] - mean;
                acc4[u] += dd * dd;
            }
    v[0] = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    chunk_block_sum<1>(v, red);
    const double sd = sqrt(v[0] / M);
    const double fl = 1e-12 * (fabs(mean) + 1.0);
    if (threadIdx.x == 0) g.step[j] = static_cast<float>(g.lambda[j] * (sd > fl ? sd : fl));
}

__global__ void __launch_bounds__(kChunkThreads) k_st_steps(const GroupDesc* __restrict__ groups, int dmax) {
    st_steps(groups, blockIdx.x / dmax, blockIdx.x % dmax);
}

// Hook: the adaptation of st_stats on its own (one group, stage index > 0).
__global__ void __launch_bounds__(kChunkThreads) k_st_adapt(const GroupDesc* __restrict__ groups) {
    __shared__ double red[kStagePartVals][kChunkWaves];
    st_adapt(groups[0], groups[0].st->stage, red);
}

// ------------------------------------------------------------ single-chunk stages
// Groups of at most kStageChunk particles (one chunk) and at most kStageChunk resampled
// positions: the steps above up to the resampling, in one workgroup per group, as the
// bodies of the launches they replace, run one after another with a barrier between them
// (the writes of one are the reads of the next, within the workgroup).  Every body sums in
// the order of its own launch, so the results are those of the chunk-parallel launches bit
// for bit; the stage costs four launches instead of seventeen (the step sizes keep their
// own launch, one workgroup per component).
// The passes of st_search for a group of one chunk, inside its workgroup: the search state
// and the weight sums stay in the workgroup (LDS and registers) between passes instead of
// going through the global buffers that separate launches need, and the passes stop once the
// search has ended.  The same steps on the same sums (a one-chunk reduction of the partials
// is the partial plus zero), so the same bits; the final state goes where k_st_finish and the
// weights read it.
__device__ inline void st_search_one_chunk(const GroupDesc* __restrict__ groups, int gi) {
    const GroupDesc& g = groups[gi];
    GroupState* st = g.st;
    if (st->done) return;
    __shared__ double red[kStagePartVals][kChunkWaves];
    __shared__ StageNewton s_nst;
    double sums[5];
    reduce_parts<5, true>(part_buf(g, 0), 1, sums, red);
    StageNewton ns{};
    int i0, i1;
    chunk_range(g, 0, i0, i1);
    for (int it = 0; it < kNewtonLaunches; ++it) {
        if (threadIdx.x == 0) {
            ns = search_step(g, ns, sums, it, st->beta);
            s_nst = ns;
            if (ns.phase == kPhaseFail) {
                st->status = SMC_ENUMERIC;
                st->done = 1;
            }
        }
        __syncthreads();
        ns = s_nst;
        if (ns.phase != kPhaseH && ns.phase != kPhaseNewton) break;
        if (it + 1 == kNewtonLaunches) break;   // no pass left to use the sums
        double out[4];
        if (ns.phase == kPhaseH) {
            chunk_weight_sums<2>(g.energy, i0, i1, ns.emin, ns.x, out, nullptr, red);
            out[2] = out[3] = 0.0;
        } else {
            chunk_weight_sums<4>(g.energy, i0, i1, ns.emin, ns.x, out, nullptr, red);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) sums[q] = 0.0 + out[q];
    }
    if (threadIdx.x == 0) *nst_buf(g, kNewtonLaunches) = ns;
}

__global__ void __launch_bounds__(kChunkThreads) k_st_pre1(const GroupDesc* __restrict__ groups) {
    st_stats(groups, blockIdx.x, 0);
    __syncthreads();
    st_search_one_chunk(groups, blockIdx.x);
}

__global__ void __launch_bounds__(kChunkThreads) k_st_post1(const GroupDesc* __restrict__ groups, int mblocks) {
    st_weights(groups, blockIdx.x, 0);
    __syncthreads();
    st_quantise(groups, blockIdx.x, 0, 0);
    __syncthreads();
    st_offsets(groups, blockIdx.x);
    __syncthreads();
    for (int mb = 0; mb < mblocks; ++mb) st_resample(groups, blockIdx.x, mb, int64_t{-1}, nullptr);
}

// ------------------------------------------------------------------ hook kernels

__global__ void k_philox(const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1, uint4* __restrict__ out, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox(ctr[i], k0, k1);
}

// Stage 0 draws: one thread per (particle, component).
__global__ void k_draw(const GroupDesc* __restrict__ groups, int group) {
    const GroupDesc& g = groups[group];
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(g.P) * g.d) return;
    const int j = static_cast<int>(t / g.P), i = static_cast<int>(t % g.P);
    g.theta[(size_t)j * g.P + i] = prior_draw(g.prior[j], g.key0, g.key1, static_cast<uint32_t>(g.K),
                                              static_cast<uint32_t>(i), static_cast<uint32_t>(j));
}

// Stage-0 draws of many groups: each work item is a run of <= 256 consecutive draws
// (linear index j * P + i) of one group.
__global__ void k_draw_items(const GroupDesc* __restrict__ groups, const MoveWork* __restrict__ items) {
    const MoveWork w = items[blockIdx.x];
    if (static_cast<int>(threadIdx.x) >= w.nchains) return;
    const GroupDesc& g = groups[w.group];
    const int64_t t = static_cast<int64_t>(w.chain0) + threadIdx.x;
    const int j = static_cast<int>(t / g.P), i = static_cast<int>(t % g.P);
    g.theta[(size_t)j * g.P + i] = prior_draw(g.prior[j], g.key0, g.key1, static_cast<uint32_t>(g.K),
                                              static_cast<uint32_t>(i), static_cast<uint32_t>(j));
}

// ------------------------------------------------------------------ launchers

hipError_t launch_draw_items(const GroupDesc* groups, const MoveWork* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_draw_items, dim3(static_cast<unsigned>(n_items)), dim3(256), 0, s, groups, items);
    return hipGetLastError();
}


hipError_t launch_stage(const StageLaunch& L, hipStream_t s) {
    if (L.n_groups <= 0) return hipSuccess;
    const int maxch = (L.max_p + kStageChunk - 1) / kStageChunk;
    if (maxch == 1 && L.max_m <= kStageChunk) {
        const dim3 ng(static_cast<unsigned>(L.n_groups));
        hipLaunchKernelGGL(k_st_pre1, ng, dim3(kChunkThreads), 0, s, L.groups);
        hipLaunchKernelGGL(k_st_finish, ng, dim3(kStageThreads), 0, s, L.groups);
        hipLaunchKernelGGL(k_st_post1, ng, dim3(kChunkThreads), 0, s, L.groups,
                           (L.max_m + kChunkThreads - 1) / kChunkThreads);
        const int dmax = std::max(L.max_d, 1);
        hipLaunchKernelGGL(k_st_steps, dim3(L.n_groups * dmax), dim3(kChunkThreads), 0, s, L.groups, dmax);
        return hipGetLastError();
    }
    const dim3 nb(static_cast<unsigned>(L.n_groups * maxch));
    hipLaunchKernelGGL(k_st_stats, nb, dim3(kChunkThreads), 0, s, L.groups, maxch);
    for (int it = 0; it < kNewtonLaunches; ++it)
        hipLaunchKernelGGL(k_st_search, nb, dim3(kChunkThreads), 0, s, L.groups, maxch, it);
    hipLaunchKernelGGL(k_st_finish, dim3(L.n_groups), dim3(kStageThreads), 0, s, L.groups);
    hipLaunchKernelGGL(k_st_weights, nb, dim3(kChunkThreads), 0, s, L.groups, maxch);
    hipLaunchKernelGGL(k_st_quantise, nb, dim3(kChunkThreads), 0, s, L.groups, maxch, 0);
    hipLaunchKernelGGL(k_st_offsets, dim3(L.n_groups), dim3(kChunkThreads), 0, s, L.groups);
    const int mblocks = (L.max_m + kChunkThreads - 1) / kChunkThreads;
    hipLaunchKernelGGL(k_st_resample, dim3(L.n_groups * mblocks), dim3(kChunkThreads), 0, s, L.groups, mblocks,
                       int64_t{-1}, static_cast<int32_t*>(nullptr));
    const int dmax = std::max(L.max_d, 1);
    hipLaunchKernelGGL(k_st_steps, dim3(L.n_groups * dmax), dim3(kChunkThreads), 0, s, L.groups, dmax);
    return hipGetLastError();
}

hipError_t launch_search_hook(const GroupDesc* group, int P, hipStream_t s) {
    const int maxch = (P + kStageChunk - 1) / kStageChunk;
    hipLaunchKernelGGL(k_st_stats, dim3(maxch), dim3(kChunkThreads), 0, s, group, maxch);
    for (int it = 0; it < kNewtonLaunches; ++it)
        hipLaunchKernelGGL(k_st_search, dim3(maxch), dim3(kChunkThreads), 0, s, group, maxch, it);
    hipLaunchKernelGGL(k_st_finish, dim3(1), dim3(kStageThreads), 0, s, group);
    hipLaunchKernelGGL(k_st_weights, dim3(maxch), dim3(kChunkThreads), 0, s, group, maxch);
    hipLaunchKernelGGL(k_st_quantise, dim3(maxch), dim3(kChunkThreads), 0, s, group, maxch, 0);
    return hipGetLastError();
}

hipError_t launch_resample_hook(const GroupDesc* group, int P, int M, uint32_t r, int32_t* anc, hipStream_t s) {
    const int maxch = (P + kStageChunk - 1) / kStageChunk;
    hipLaunchKernelGGL(k_st_quantise, dim3(maxch), dim3(kChunkThreads), 0, s, group, maxch, 1);
    hipLaunchKernelGGL(k_st_offsets, dim3(1), dim3(kChunkThreads), 0, s, group);
    const int mblocks = (M + kChunkThreads - 1) / kChunkThreads;
    hipLaunchKernelGGL(k_st_resample, dim3(mblocks), dim3(kChunkThreads), 0, s, group, mblocks, int64_t{r}, anc);
    return hipGetLastError();
}

hipError_t launch_steps_hook(const GroupDesc* group, int d, hipStream_t s) {
    hipLaunchKernelGGL(k_st_adapt, dim3(1), dim3(kChunkThreads), 0, s, group);
    hipLaunchKernelGGL(k_st_steps, dim3(std::max(d, 1)), dim3(kChunkThreads), 0, s, group, std::max(d, 1));
    return hipGetLastError();
}

// Index of the final temperature-search state (read by the hooks).
int stage_final_parity() { return kNewtonLaunches & 1; }

hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(ctr), k0, k1, reinterpret_cast<uint4*>(out), n);
    return hipGetLastError();
}



hipError_t launch_draw(const GroupDesc* groups, int group, int64_t n_draws, hipStream_t s) {
    if (n_draws <= 0) return hipSuccess;
    const int64_t blocks = (n_draws + 255) / 256;
    hipLaunchKernelGGL(k_draw, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, groups, group);
    return hipGetLastError();
}

}  // namespace smc
