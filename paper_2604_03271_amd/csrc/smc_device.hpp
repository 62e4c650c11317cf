// smc_device.hpp -- device-side building blocks of the gfx950 SMC sampler.
//
// Everything here runs on the GPU.  FP32 is used for the forward model
// (Eq. forward_model with the Gaussian basis of Eq. spectral_forward_model or
// the pseudo-Voigt basis of Eq. xps_forward_model), the energies and the
// Metropolis decisions; FP64 only in the stage kernel (weights, ESS, evidence).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smc_types.hpp"

namespace smc {

constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLog2e = 1.442695040888963407f;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds, each two
// 32x32->64 products of counter words 0 and 2 with the published multipliers,
// XOR of the high halves with words 1/3 and the round key, and a Weyl key
// schedule with the published increments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint4 draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                      uint32_t K, uint32_t purpose) {
    return philox(make_uint4(c0, c1, c2, (K << 8) | purpose), k0, k1);
}

// (r + 1/2) / 2^32 rounded to FP32: in (0, 1].
__device__ __forceinline__ float u01(uint32_t r) {
    return __builtin_fmaf(static_cast<float>(r), 0x1.0p-32f, 0x1.0p-33f);
}

__device__ __forceinline__ float fast_ln(float v) { return __builtin_amdgcn_logf(v) * kLn2; }

// Box-Muller, cosine branch; v_cos_f32 takes its argument in revolutions.
__device__ __forceinline__ float box_muller(uint32_t r0, uint32_t r1) {
    const float rad = __builtin_sqrtf(-2.0f * fast_ln(u01(r0)));
    return rad * __builtin_amdgcn_cosf(u01(r1));
}

// Prior draw of one component (stage 0).  Uniform by inverse CDF, Normal by
// Box-Muller, Gamma by Marsaglia & Tsang (2000), shape < 1 boosted by u^(1/a).
__device__ inline float prior_draw(const DevPrior& pr, uint32_t k0, uint32_t k1, uint32_t K, uint32_t i,
                                   uint32_t j) {
    if (pr.kind == SMC_PRIOR_UNIFORM) {
        const uint4 r = draw(k0, k1, i, 0, 256u * j, K, kPurposeInit);
        return pr.a + (pr.b - pr.a) * u01(r.x);
    }
    if (pr.kind == SMC_PRIOR_NORMAL) {
        const uint4 r = draw(k0, k1, i, 0, 256u * j, K, kPurposeInit);
        return pr.a + pr.b * box_muller(r.x, r.y);
    }
    if (pr.kind == SMC_PRIOR_GAMMA) {
        const float shape = pr.a < 1.0f ? pr.a + 1.0f : pr.a;
        const float d = shape - 1.0f / 3.0f;
        const float c = 1.0f / __builtin_sqrtf(9.0f * d);
        for (uint32_t t = 0; t < 256u; ++t) {
            const uint4 r = draw(k0, k1, i, 0, 256u * j + t, K, kPurposeInit);
            const float z = box_muller(r.x, r.y);
            float v = 1.0f + c * z;
            if (v <= 0.0f) continue;
            v = v * v * v;
            if (fast_ln(u01(r.z)) < 0.5f * z * z + d - d * v + d * fast_ln(v)) {
                float g = d * v;
                if (pr.a < 1.0f) g *= __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(u01(r.w)) / pr.a);
                return g / pr.b;
            }
        }
        return pr.a / pr.b;
    }
    return pr.a;  // fixed
}

// A read-only table entry loaded through the constant address space: with an index that is
// the same in every lane the compiler issues scalar loads into scalar registers (the tables
// read this way are not written while a kernel runs).
template <typename T>
__device__ __forceinline__ T constant_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    using Word = const __attribute__((address_space(4))) uint32_t;
    Word* w = reinterpret_cast<Word*>(reinterpret_cast<uintptr_t>(p));
    uint32_t buf[sizeof(T) / 4];
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) buf[i] = w[i];
    return __builtin_bit_cast(T, buf);
}

// Inside the prior's support: the open interval (lo, hi) (uniform: (a, b); gamma: v > 0
// and finite; normal: finite).
__device__ __forceinline__ bool prior_in_support(const DevPrior& pr, float v) { return v > pr.lo && v < pr.hi; }

// ln p(new) - ln p(old) for one component inside its support.
__device__ __forceinline__ float prior_log_ratio(const DevPrior& pr, float vn, float vo) {
    if (pr.kind == SMC_PRIOR_GAMMA) {
        float r = -pr.b * (vn - vo);
        if (pr.c != 0.0f) r += pr.c * kLn2 * (__builtin_amdgcn_logf(vn) - __builtin_amdgcn_logf(vo));
        return r;
    }
    if (pr.kind == SMC_PRIOR_NORMAL) {
        const float dn = vn - pr.a, d0 = vo - pr.a;
        return (d0 * d0 - dn * dn) * pr.c;
    }
    return 0.0f;
}

// ---------------------------------------------------------------------------
// Peak profiles.  A peak's per-particle constants are hoisted out of the point
// loop (t = x - mu, evaluated exactly near the peak by Sterbenz's lemma):
//   Gaussian      A exp(-(b/2) t^2)                        = aG 2^(c t^2),
//                 c = -(b/2) log2 e, aG = A
//   pseudo-Voigt  A [eta e^(-ln2 t^2/s^2) + (1-eta) s^2/(s^2+t^2)] = aG 2^(-u) + aL / u,
//                 u = 1 + c t^2, c = 1/s^2, aG = 2 A eta, aL = A (1 - eta)
// (one fma forms u, which serves both shapes: 2^(-t^2/s^2) = 2 * 2^(-u) and
// s^2/(s^2 + t^2) = 1/u); background c0 + c1 x (constant background: c1 = 0).
// ---------------------------------------------------------------------------
struct PeakC {
    float mu, c, aG, aL;
};

template <int PK>
__device__ __forceinline__ PeakC peak_consts(const float* th) {
    PeakC q;
    q.mu = th[1];
    if constexpr (PK == SMC_PEAK_GAUSS) {
        q.c = -0.5f * kLog2e * th[2];
        q.aG = th[0];
        q.aL = 0.0f;
    } else {
        q.c = __builtin_amdgcn_rcpf(th[2] * th[2]);   // v_rcp (1 ulp): no IEEE division sequence per proposal
        q.aG = 2.0f * (th[0] * th[3]);
        q.aL = th[0] * (1.0f - th[3]);
    }
    return q;
}

// The constants of peak th with component Q replaced by v, from the constants qc of th itself:
// only the fields that depend on component Q are formed, each by the expression of
// peak_consts, so the result has the bits of peak_consts of the modified vector.
template <int PK, int Q>
__device__ __forceinline__ PeakC peak_consts_with(const PeakC& qc, const float* th, float v) {
    PeakC q = qc;
    if constexpr (Q == 1) {
        q.mu = v;
    } else if constexpr (PK == SMC_PEAK_GAUSS) {
        if constexpr (Q == 0) q.aG = v;
        else q.c = -0.5f * kLog2e * v;
    } else if constexpr (Q == 0) {
        q.aG = 2.0f * (v * th[3]);
        q.aL = v * (1.0f - th[3]);
    } else if constexpr (Q == 2) {
        q.c = __builtin_amdgcn_rcpf(v * v);
    } else {
        q.aG = 2.0f * (th[0] * v);
        q.aL = th[0] * (1.0f - v);
    }
    return q;
}

// Unit shapes of a peak at distance t from its centre: e (the exponential, in the
// units of aG) and, for a pseudo-Voigt peak, l (the Lorentzian, in the units of aL).
template <int PK>
__device__ __forceinline__ void peak_shapes(const PeakC& q, float t, float& e, float& l) {
    const float t2 = t * t;
    if constexpr (PK == SMC_PEAK_GAUSS) {
        e = __builtin_amdgcn_exp2f(q.c * t2);
        l = 0.0f;
    } else {
        const float u = __builtin_fmaf(t2, q.c, 1.0f);
        e = __builtin_amdgcn_exp2f(-u);
        l = __builtin_amdgcn_rcpf(u);
    }
}

template <int PK>
__device__ __forceinline__ float peak_eval(float x, const PeakC& q) {
    float e, l;
    peak_shapes<PK>(q, x - q.mu, e, l);
    if constexpr (PK == SMC_PEAK_GAUSS) return q.aG * e;
    else return __builtin_fmaf(q.aL, l, q.aG * e);
}

__device__ __forceinline__ PeakC bg_consts(const float* th, int nbg) {
    PeakC q{};
    q.aG = nbg > 0 ? th[0] : 0.0f;
    q.aL = nbg > 1 ? th[1] : 0.0f;
    return q;
}

__device__ __forceinline__ float bg_eval(float x, const PeakC& q) { return __builtin_fmaf(q.aL, x, q.aG); }

// Poisson deviance term of one point (Eq. xrd_poisson without its data-only part),
// f - y + y ln(y/f) = y g(f/y) with g(u) = u - 1 - ln u, added to acc.  Each point keeps
// w = count_w(y) and iw = 1/w, so the term takes a product, a subtraction, a log and two fmas:
// acc + w g(u), u = f iw.  Near the fit (u near 1) g is about (u-1)^2/2 but u - 1 is exact
// and the hardware log2 is accurate relative to its result, so the absolute error of the
// term is about |f - y| 2.4e-7 (the roundings of iw, of u and of ln u); the sum over points
// of such errors is far below the energies' 1e-5 relative tolerance.  A zero count is kept
// as w = 2^-40 (count_w): the term is then f - w (1 + ln(f/w)), within 1e-10 of the exact f,
// for any f below 2^88, where f iw would overflow.  f = 0 gives +inf (ln 0) and f < 0 NaN
// (ln of a negative number): poisson_energy maps a sum holding NaN to +inf once per energy.
// A padding point with y = f = 1 gives exactly 0.
constexpr float kZeroCountW = 0x1p-40f;

__device__ __forceinline__ float count_w(float y) { return y > 0.0f ? y : kZeroCountW; }

__device__ __forceinline__ float poisson_dev_acc(float acc, float w, float iw, float f) {
    const float u = f * iw;
    return __builtin_fmaf(w, __builtin_fmaf(-kLn2, __builtin_amdgcn_logf(u), u - 1.0f), acc);
}

// A sum of poisson_dev_acc terms as an energy: NaN (some model value <= 0) becomes +inf.
__device__ __forceinline__ float poisson_energy(float e) { return e == e ? e : __builtin_inff(); }

// ---------------------------------------------------------------------------
// Sum over the L consecutive lanes of a chain inside one wavefront.  Every step
// is a butterfly whose two operands are swapped between partner lanes, so all
// L lanes end with the same bits (IEEE addition is commutative); a whole
// wavefront ends in one scalar register.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_swap(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Across rows the gfx950 permlane swap (VALU, no LDS round trip) returns the even
// and the odd row of each pair of rows (16 lanes) in every lane; all lanes add them
// in the same order.
// The two results pass through an empty asm before they are added: this compiler
// otherwise folds the sum of the swap's two results into twice the first one (seen in
// the assembly as v_add_f32 vN, vN, vN after the swap), which is wrong.
__device__ __forceinline__ float swap_sum(unsigned a, unsigned b) {
    asm volatile("" : "+v"(a), "+v"(b));
    return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

__device__ __forceinline__ float row_pair_sum16(float v) {
    const unsigned w = __builtin_bit_cast(unsigned, v);
    const auto p = __builtin_amdgcn_permlane16_swap(w, w, false, false);
    return swap_sum(p[0], p[1]);
}

// v + (lane 15 of the row before) in rows 1 and 3, v elsewhere (one DPP add with a row mask;
// the lanes of the rows the mask leaves out keep their value, so the operand is tied to the
// result).  The s_nop gives the DPP read of v the wait states after the VALU write of v.
__device__ __forceinline__ float add_row_bcast15(float v) {
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf" : "+v"(v));
    return v;
}

// v + lane 31 in rows 2 and 3, v elsewhere.
__device__ __forceinline__ float add_row_bcast31(float v) {
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf" : "+v"(v));
    return v;
}

template <int L>
__device__ __forceinline__ float group_sum(float v) {
    v += dpp_swap<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_swap<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_swap<0x141>(v);  // row_half_mirror: quads of a half-row
    v += dpp_swap<0x140>(v);  // row_mirror: halves of a 16-lane row
    if constexpr (L == 32) v = row_pair_sum16(v);
    if constexpr (L == 64) {
        // a whole wavefront: the row sums added through DPP row broadcasts (row 1 += row 0,
        // row 3 += row 2, then rows 2-3 += lane 31), the total read from lane 63 into a
        // scalar register: one value for every lane, fewer instructions than two swaps
        v = add_row_bcast31(add_row_bcast15(v));
        v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
    }
    return v;
}

// Logical work item of block b in a launch of n blocks.  Consecutive workgroups go to
// the 8 XCDs in turn, each with its own L2, and neighbouring chains share cache lines of
// the component-major particle arrays, so items are dealt to the XCDs in chunks of
// `chunk` consecutive items (chunk c to XCD c mod 8): each XCD reads whole lines, and
// every group's chains still spread over all XCDs (the work list is ordered by group, so
// one contiguous range per XCD would give one XCD all of the heaviest group).  The
// ragged tail of fewer than 8 chunks keeps its order.  A bijection of [0, n).
__device__ __forceinline__ int xcd_block(int b, int n, int chunk) {
    constexpr int kXcds = 8;
    const int span = kXcds * chunk;
    if (b >= (n / span) * span) return b;
    const int x = b % kXcds, r = b / kXcds;
    return (x + kXcds * (r / chunk)) * chunk + r % chunk;
}

}  // namespace smc
