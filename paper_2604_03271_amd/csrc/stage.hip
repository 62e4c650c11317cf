// stage.hip -- the per-stage bookkeeping of the tempered SMC sampler, one
// workgroup of 1024 threads per (spectrum, K) group, entirely on the device:
//
//   1. step-size multipliers lambda_j from the previous move's acceptance;
//   2. the next inverse-temperature increment delta by bisection on the ESS of
//      the incremental weights w_i = exp(-delta E_i) (Eq. smc_incremental_weight);
//   3. log-sum-exp, ESS and the evidence increment LSE - ln P
//      (Eq. smc_marginal_likelihood), all in FP64;
//   4. systematic resampling of M ancestors on weights quantised to 2^-52
//      (integer CDF, 128-bit positions, so the ancestors are exact);
//   5. gather of the ancestors into the move's start buffer and the
//      random-walk scales s_j = lambda_j * sd_j over the resampled states.
// Plus the small kernels behind the per-kernel hooks, which reuse the same
// device functions.
#include "smc_device.hpp"

namespace smc {

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
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], o, 64);
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
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) emin = fmin(emin, __shfl_xor(emin, off, 64));
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

// Quantise normalised weights to q_i = floor(W_i 2^52) and write the inclusive
// prefix sums to cdf.  Returns Q = sum q_i (same value in every thread).
template <class WeightFn>
__device__ inline unsigned long long quantise_scan(WeightFn weight, int P, unsigned long long* cdf, StageShared& sh) {
    const int chunk = (P + kStageThreads - 1) / kStageThreads;
    const int c0 = min(P, static_cast<int>(threadIdx.x) * chunk), c1 = min(P, c0 + chunk);
    unsigned long long local = 0;
    for (int i = c0; i < c1; ++i) {
        const unsigned long long q = static_cast<unsigned long long>(floor(weight(i) * 4503599627370496.0));
        cdf[i] = q;
        local += q;
    }
    // exclusive scan of the per-thread sums: inside each wave, then over waves
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    __syncthreads();
    if (lane == 63) sh.scan[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int q = 0; q < kStageWaves; ++q) {
            const unsigned long long v = sh.scan[q];
            sh.scan[q] = run;
            run += v;
        }
        sh.total = run;
    }
    __syncthreads();
    unsigned long long run = sh.scan[w] + incl - local;
    for (int i = c0; i < c1; ++i) {
        run += cdf[i];
        cdf[i] = run;
    }
    const unsigned long long Q = sh.total;
    __syncthreads();
    return Q;
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

__global__ void __launch_bounds__(kStageThreads) k_stage(const GroupDesc* __restrict__ groups) {
    const GroupDesc& g = groups[blockIdx.x];
    GroupState* st = g.st;
    __shared__ StageShared sh;
    __shared__ int s_done;
    if (st->done) return;
    const int d = g.d, P = g.P, M = g.M;
    const int stage_prev = st->stage;

    // 1. lambda_j <- clamp(lambda_j exp(acc_j - 0.44), 0.01, 10) after a move
    if (stage_prev > 0 && threadIdx.x == 0) {
        const double props = static_cast<double>(M) * g.n_moves;
        double acc_sum = 0.0;
        int nfree = 0;
        for (int j = 0; j < d; ++j) {
            if (g.prior[j].kind == SMC_PRIOR_FIXED) continue;
            const double a = g.acc[j] / props;
            acc_sum += a;
            ++nfree;
            g.lambda[j] = fmin(10.0, fmax(0.01, g.lambda[j] * exp(a - 0.44)));
        }
        if (stage_prev <= g.max_stages) g.trace[(stage_prev - 1) * kTraceCols + 5] = nfree ? acc_sum / nfree : 0.0;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += kStageThreads) g.acc[j] = 0u;

    if (threadIdx.x == 0) s_done = st->beta >= 1.0 || stage_prev >= g.max_stages;
    __syncthreads();
    if (s_done) {
        if (threadIdx.x == 0) {
            if (st->beta < 1.0) st->status = SMC_ENUMERIC;
            st->done = 1;
        }
        return;
    }
    const int stage = stage_prev + 1;
    const double beta = st->beta;

    // 2-3. temperature, weights, evidence
    const BisectOut b = bisect(g.energy, P, beta, g.rho, g.bisect_iters, sh);
    if (!b.ok) {
        if (threadIdx.x == 0) {
            st->status = SMC_ENUMERIC;
            st->done = 1;
        }
        return;
    }
    double beta_new = (b.delta == 1.0 - beta) ? 1.0 : beta + b.delta;
    if (beta_new > 1.0) beta_new = 1.0;
    const double s1 = b.s1, emin = b.emin, delta = b.delta;

    // 4. resampling
    const float* E = g.energy;
    const unsigned long long Q = quantise_scan(
        [=](int i) { return exp(-delta * (static_cast<double>(E[i]) - emin)) / s1; }, P, g.cdf, sh);
    const uint32_t r = draw(g.key0, g.key1, 0u, static_cast<uint32_t>(stage), 0u, static_cast<uint32_t>(g.K),
                            kPurposeResample).x;
    for (int m = threadIdx.x; m < M; m += kStageThreads) {
        const int a = ancestor(g.cdf, P, position(static_cast<uint32_t>(m), r, Q, static_cast<uint32_t>(M)));
        g.start_e[m] = E[a];
        for (int j = 0; j < d; ++j) g.start[(size_t)j * M + m] = g.theta[(size_t)j * P + a];
    }
    __syncthreads();

    // 5. step sizes over the resampled states (one wave per component)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int j = w; j < d; j += kStageWaves) {
        if (g.prior[j].kind == SMC_PRIOR_FIXED) {
            if (lane == 0) g.step[j] = 0.0f;
            continue;
        }
        const float* col = g.start + (size_t)j * M;
        double sum = 0.0;
        for (int m = lane; m < M; m += 64) sum += col[m];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        const double mean = sum / M;
        double ss = 0.0;
        for (int m = lane; m < M; m += 64) {
            const double c = col[m] - mean;
            ss += c * c;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
        const double sd = sqrt(ss / M);
        const double fl = 1e-12 * (fabs(mean) + 1.0);
        if (lane == 0) g.step[j] = static_cast<float>(g.lambda[j] * (sd > fl ? sd : fl));
    }

    if (threadIdx.x == 0) {
        st->logz += b.lse - log(static_cast<double>(P));
        st->beta = beta_new;
        st->delta = delta;
        st->ess = b.ess;
        st->lse = b.lse;
        st->stage = stage;
        double* tr = g.trace + (stage - 1) * kTraceCols;
        tr[0] = beta_new;
        tr[1] = delta;
        tr[2] = b.ess;
        tr[3] = b.lse;
        tr[4] = st->logz;
        tr[5] = 0.0;
    }
}

// ------------------------------------------------------------------ hook kernels

__global__ void k_philox(const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1, uint4* __restrict__ out, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox(ctr[i], k0, k1);
}

__global__ void __launch_bounds__(kStageThreads) k_bisect_hook(const float* __restrict__ E, int P, double beta, double rho,
                                                              int iters, double* __restrict__ out) {
    __shared__ StageShared sh;
    const BisectOut b = bisect(E, P, beta, rho, iters, sh);
    if (threadIdx.x == 0) {
        out[0] = b.ok ? b.delta : __builtin_nan("");
        out[1] = b.ess;
        out[2] = b.lse;
        out[3] = b.emin;
    }
}

__global__ void __launch_bounds__(kStageThreads) k_resample_hook(const double* __restrict__ W, int P, int M, uint32_t r,
                                                                unsigned long long* __restrict__ cdf,
                                                                int32_t* __restrict__ anc) {
    __shared__ StageShared sh;
    const unsigned long long Q = quantise_scan([=](int i) { return W[i]; }, P, cdf, sh);
    for (int m = threadIdx.x; m < M; m += kStageThreads)
        anc[m] = ancestor(cdf, P, position(static_cast<uint32_t>(m), r, Q, static_cast<uint32_t>(M)));
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


hipError_t launch_stage(const GroupDesc* groups, int n_groups, hipStream_t s) {
    hipLaunchKernelGGL(k_stage, dim3(n_groups), dim3(kStageThreads), 0, s, groups);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, int64_t n, hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(ctr), k0, k1, reinterpret_cast<uint4*>(out), n);
    return hipGetLastError();
}

hipError_t launch_bisect_hook(const float* E, int P, double beta, double rho, int iters, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_bisect_hook, dim3(1), dim3(kStageThreads), 0, s, E, P, beta, rho, iters, out);
    return hipGetLastError();
}

hipError_t launch_resample_hook(const double* W, int P, int M, uint32_t r, unsigned long long* cdf, int32_t* anc,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_resample_hook, dim3(1), dim3(kStageThreads), 0, s, W, P, M, r, cdf, anc);
    return hipGetLastError();
}

hipError_t launch_draw(const GroupDesc* groups, int group, int64_t n_draws, hipStream_t s) {
    if (n_draws <= 0) return hipSuccess;
    const int64_t blocks = (n_draws + 255) / 256;
    hipLaunchKernelGGL(k_draw, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, groups, group);
    return hipGetLastError();
}

}  // namespace smc
