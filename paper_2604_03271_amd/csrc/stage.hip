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
    double red[2][kStageWaves];
    unsigned long long scan[kStageWaves];
    unsigned long long total;
};

// Sum of two FP64 values over the workgroup; every thread receives the same bits.
__device__ inline double2 block_sum2(double a, double b, StageShared& sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh.red[0][w] = a;
        sh.red[1][w] = b;
    }
    __syncthreads();
    double s = 0.0, t = 0.0;
    for (int q = 0; q < kStageWaves; ++q) {
        s += sh.red[0][q];
        t += sh.red[1][q];
    }
    return make_double2(s, t);
}

__device__ inline double block_min(double v, int& any_nan, StageShared& sh) {
    int nan_flag = any_nan;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v = fmin(v, __shfl_xor(v, o, 64));
        nan_flag |= __shfl_xor(nan_flag, o, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh.red[0][w] = v;
        sh.red[1][w] = nan_flag;
    }
    __syncthreads();
    double m = sh.red[0][0];
    int nf = 0;
    for (int q = 0; q < kStageWaves; ++q) {
        m = fmin(m, sh.red[0][q]);
        nf |= sh.red[1][q] != 0.0;
    }
    any_nan = nf;
    return m;
}

// S1 = sum exp(-delta a_i), S2 = sum exp(-delta a_i)^2 with a_i = E_i - min E.
__device__ inline double2 weight_sums(const float* E, int P, double emin, double delta, StageShared& sh) {
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < P; i += kStageThreads) {
        const double w = exp(-delta * (static_cast<double>(E[i]) - emin));
        s1 += w;
        s2 += w * w;
    }
    return block_sum2(s1, s2, sh);
}

struct BisectOut {
    double delta, ess, lse, emin;
    int ok;
};

// Next increment: all of 1 - beta if ESS there >= rho P, else `iters` halvings of
// [0, 1 - beta] keeping the low end; the high end if no tested point qualified.
__device__ inline BisectOut bisect(const float* E, int P, double beta, double rho, int iters, StageShared& sh) {
    BisectOut o;
    int nan = 0;
    double emin = __builtin_inf();
    for (int i = threadIdx.x; i < P; i += kStageThreads) {
        const float e = E[i];
        nan |= __builtin_isnan(e);
        emin = fmin(emin, static_cast<double>(e));
    }
    emin = block_min(emin, nan, sh);
    o.emin = emin;
    o.ok = !nan && emin < __builtin_inf();
    if (!o.ok) {
        o.delta = o.ess = o.lse = 0.0;
        return o;
    }
    const double target = rho * static_cast<double>(P);
    double hi = 1.0 - beta;
    double2 s = weight_sums(E, P, emin, hi, sh);
    double delta;
    if (s.x * s.x / s.y >= target) {
        delta = hi;
    } else {
        double lo = 0.0;
        for (int it = 0; it < iters; ++it) {
            const double mid = 0.5 * (lo + hi);
            const double2 t = weight_sums(E, P, emin, mid, sh);
            if (t.x * t.x / t.y >= target) lo = mid;
            else hi = mid;
        }
        delta = lo > 0.0 ? lo : hi;
        s = weight_sums(E, P, emin, delta, sh);
    }
    o.delta = delta;
    o.ess = s.x * s.x / s.y;
    o.lse = -delta * emin + log(s.x);
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
    if (stage_prev > 0) {
        const double props = static_cast<double>(M) * g.n_moves;
        double acc_sum = 0.0;
        int nfree = 0;
        for (int j = 0; j < d; ++j) {
            if (g.prior[j].kind == SMC_PRIOR_FIXED) continue;
            const double a = g.acc[j] / props;
            acc_sum += a;
            ++nfree;
            if (threadIdx.x == 0) g.lambda[j] = fmin(10.0, fmax(0.01, g.lambda[j] * exp(a - 0.44)));
        }
        if (threadIdx.x == 0 && stage_prev <= g.max_stages)
            g.trace[(stage_prev - 1) * kTraceCols + 5] = nfree ? acc_sum / nfree : 0.0;
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
    const double2 s = weight_sums(g.energy, P, b.emin, b.delta, sh);
    const double s1 = s.x;
    const double emin = b.emin, delta = b.delta;

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

// ------------------------------------------------------------------ launchers

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
