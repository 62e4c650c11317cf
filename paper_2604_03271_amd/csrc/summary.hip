// summary.hip -- posterior summaries of one candidate K from its final particle
// population (Sec. III: posterior means and the endpoints of the 95% / 99%
// credible intervals).
//
// After the final move at beta = 1 the P particles are an equally weighted
// posterior sample.  Per component the mean is an FP64 sum; each quantile q is
// the sample value of rank ceil(q P) (inverse empirical CDF), found exactly by
// a four-pass radix select on order-preserving 32-bit keys: every pass builds a
// 256-bin histogram in LDS of the next key byte among the values that share
// the already fixed upper bytes, one histogram per requested rank.  The values
// are read four times from HBM and nothing is sorted or copied to the host.
//
// The prior is exchangeable in the peaks, so per-peak summaries need one
// labelling: the relabel kernel writes a copy of the population with each
// particle's peaks in non-decreasing centre order (ties keep index order).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "host_common.hpp"

namespace smc {
namespace {

constexpr int kSumThreads = 1024;
constexpr int kSumWaves = kSumThreads / 64;

// IEEE-754 bits -> unsigned key with the same order (NaN excluded).
__device__ __forceinline__ uint32_t order_key(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// One thread per particle.  The rank of peak k is the number of peaks whose
// centre is smaller, or equal with a smaller index, so the ranks are a
// permutation and the copy is a stable sort by centre.
__global__ __launch_bounds__(256) void k_relabel(const float* __restrict__ in, float* __restrict__ out, int P,
                                                 int d, int n_peaks, int np) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const size_t sP = static_cast<size_t>(P);
    for (int k = 0; k < n_peaks; ++k) {
        const float mu = in[(static_cast<size_t>(k) * np + 1) * sP + i];
        int rank = 0;
        for (int k2 = 0; k2 < n_peaks; ++k2) {
            const float m2 = in[(static_cast<size_t>(k2) * np + 1) * sP + i];
            rank += (m2 < mu || (m2 == mu && k2 < k)) ? 1 : 0;
        }
        for (int q = 0; q < np; ++q)
            out[(static_cast<size_t>(rank) * np + q) * sP + i] = in[(static_cast<size_t>(k) * np + q) * sP + i];
    }
    for (int j = n_peaks * np; j < d; ++j) out[static_cast<size_t>(j) * sP + i] = in[static_cast<size_t>(j) * sP + i];
}

// One workgroup per component; ranks.r[t] (0-based) for t < ranks.n <= SMC_MAX_PROBS.
__global__ __launch_bounds__(kSumThreads) void k_summary(const float* __restrict__ theta, int P, int d,
                                                         SummaryRanks ranks, double* __restrict__ mean,
                                                         float* __restrict__ quant) {
    __shared__ uint32_t hist[SMC_MAX_PROBS][256];
    __shared__ uint32_t prefix[SMC_MAX_PROBS];
    __shared__ int32_t rem[SMC_MAX_PROBS];
    __shared__ double red[kSumWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x;
    const int nt = ranks.n;
    const float* col = theta + static_cast<size_t>(j) * P;
    if (tid < nt) {
        prefix[tid] = 0u;
        rem[tid] = ranks.r[tid];
    }
    double s = 0.0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        const int nh = pass == 0 ? 1 : nt;   // the first byte's histogram serves every rank
        for (int i = tid; i < nh * 256; i += kSumThreads) hist[i >> 8][i & 255] = 0u;
        __syncthreads();
        uint32_t pre[SMC_MAX_PROBS];
#pragma unroll
        for (int t = 0; t < SMC_MAX_PROBS; ++t) pre[t] = t < nt ? prefix[t] : 0u;
        for (int i = tid; i < P; i += kSumThreads) {
            const float v = col[i];
            const uint32_t key = order_key(v);
            const uint32_t bin = (key >> shift) & 255u;
            if (pass == 0) {
                s += static_cast<double>(v);
                atomicAdd(&hist[0][bin], 1u);
            } else {
                const uint32_t hi = key >> (shift + 8);
#pragma unroll
                for (int t = 0; t < SMC_MAX_PROBS; ++t)
                    if (t < nt && hi == pre[t]) atomicAdd(&hist[t][bin], 1u);
            }
        }
        __syncthreads();
        // wave t locates rank t: lane l owns bins 4l..4l+3
        if (wave < nt) {
            const uint32_t* h = hist[pass == 0 ? 0 : wave];
            const uint32_t c0 = h[4 * lane], c1 = h[4 * lane + 1], c2 = h[4 * lane + 2], c3 = h[4 * lane + 3];
            const uint32_t own = c0 + c1 + c2 + c3;
            uint32_t incl = own;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t o = __shfl_up(incl, off, 64);
                if (lane >= off) incl += o;
            }
            const uint32_t excl = incl - own;
            const uint32_t r = static_cast<uint32_t>(rem[wave]);
            const uint32_t p0 = prefix[wave];
            if (excl <= r && r < incl) {
                uint32_t b = 0, before = excl;
                if (r >= before + c0) {
                    before += c0;
                    b = 1;
                    if (r >= before + c1) {
                        before += c1;
                        b = 2;
                        if (r >= before + c2) {
                            before += c2;
                            b = 3;
                        }
                    }
                }
                prefix[wave] = (p0 << 8) | (4u * lane + b);
                rem[wave] = static_cast<int32_t>(r - before);
            }
        }
        __syncthreads();
    }
    // FP64 block sum for the mean
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kSumWaves; ++w) t += red[w];
        mean[j] = t / static_cast<double>(P);
    }
    if (tid < nt) quant[static_cast<size_t>(tid) * d + j] = key_value(prefix[tid]);
}

}  // namespace

hipError_t launch_relabel(const float* in, float* out, int P, int d, int n_peaks, int np, hipStream_t s) {
    hipLaunchKernelGGL(k_relabel, dim3((P + 255) / 256), dim3(256), 0, s, in, out, P, d, n_peaks, np);
    return hipGetLastError();
}

hipError_t launch_summary(const float* theta, int P, int d, const SummaryRanks& ranks, double* mean, float* quant,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_summary, dim3(d), dim3(kSumThreads), 0, s, theta, P, d, ranks, mean, quant);
    return hipGetLastError();
}

// Host side of both summary entry points: ranks, device scratch, launches, copies.
smc_status posterior_summary(const float* theta, int d, int P, int n_peaks, int np, const double* probs,
                             int n_probs, double* mean, double* quant, hipStream_t s) {
    if (!theta || d < 1 || P < 1 || !mean || n_probs < 0 || n_probs > SMC_MAX_PROBS) return SMC_EINVAL;
    if (n_probs > 0 && (!probs || !quant)) return SMC_EINVAL;
    if (n_peaks < 0 || (n_peaks > 0 && (np < 2 || n_peaks * np > d))) return SMC_EINVAL;
    if (static_cast<int64_t>(d) * P > INT32_MAX) return SMC_EINVAL;
    SummaryRanks ranks{};
    ranks.n = n_probs;
    for (int t = 0; t < n_probs; ++t) {
        const double q = probs[t];
        if (!(q >= 0.0 && q <= 1.0)) return SMC_EINVAL;
        double r = std::ceil(q * static_cast<double>(P));
        r = r < 1.0 ? 1.0 : (r > P ? static_cast<double>(P) : r);
        ranks.r[t] = static_cast<int32_t>(r) - 1;
    }
    if (!device_ok()) return SMC_EDEVICE;
    const size_t relabel_bytes = n_peaks > 0 ? sizeof(float) * static_cast<size_t>(d) * P : 0;
    const size_t mean_off = (relabel_bytes + 255) & ~size_t(255);
    const size_t quant_off = mean_off + ((sizeof(double) * d + 255) & ~size_t(255));
    const size_t total = quant_off + sizeof(float) * static_cast<size_t>(SMC_MAX_PROBS) * d;
    char* buf = nullptr;
    if (hipMalloc(&buf, total) != hipSuccess) return SMC_ENOMEM;
    smc_status st = SMC_OK;
    const float* src = theta;
    std::vector<float> q32(static_cast<size_t>(n_probs) * d);
    if (n_peaks > 0) {
        if (launch_relabel(theta, reinterpret_cast<float*>(buf), P, d, n_peaks, np, s) != hipSuccess)
            st = SMC_EDEVICE;
        src = reinterpret_cast<const float*>(buf);
    }
    double* d_mean = reinterpret_cast<double*>(buf + mean_off);
    float* d_quant = reinterpret_cast<float*>(buf + quant_off);
    if (st == SMC_OK && launch_summary(src, P, d, ranks, d_mean, d_quant, s) != hipSuccess) st = SMC_EDEVICE;
    if (st == SMC_OK && hipMemcpyAsync(mean, d_mean, sizeof(double) * d, hipMemcpyDeviceToHost, s) != hipSuccess)
        st = SMC_EDEVICE;
    if (st == SMC_OK && n_probs > 0 &&
        hipMemcpyAsync(q32.data(), d_quant, sizeof(float) * q32.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = SMC_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) st = SMC_EDEVICE;
    (void)hipFree(buf);
    if (st == SMC_OK)
        for (size_t i = 0; i < q32.size(); ++i) quant[i] = q32[i];
    return st;
}

}  // namespace smc
