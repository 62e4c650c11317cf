// chain_xrd.hpp -- likelihood and Metropolis-Hastings kernels of the XRD powder
// profile of App. E (Eqs. xrd_forward_model, xrd_pvoigt, xrd_gauss, xrd_lorentz,
// xrd_sigma, xrd_omega, xrd_asym, xrd_bg) with Poisson counts (Eq. xrd_poisson).
//
// Peak k has nine parameters (A, shift, r, alpha, u, v, w, s, t) at the reference
// position mu_ref[k]: mu = mu_ref + shift, and at point x (degrees 2theta)
//   Sigma^2 = a^2 (u tan^2(x/2) - v tan(x/2) + w),  Omega = a (s sec(x/2) + t tan(x/2)),
// a = alpha for x >= mu and 1 below; G = exp(-4 ln2 (x - mu)^2 / Sigma^2) and
// L = 1 / (1 + 4 (x - mu)^2 / Omega^2); value A ((1 - r) G + r L).  The background
// (a, sigma_bg, r_bg, b) is a ((1 - r_bg) G_bg + r_bg L_bg) + b with both widths sigma_bg
// at position 0.  Layout and residual cache as in chain.hpp (lane r owns points r,
// r + LC, ...; D = model without the current term), plus tan(x/2) per point
// (sec(x/2) = sqrt(1 + tan^2(x/2)) for 0 < x < 180 degrees, formed when needed).
// The current term's shapes G, L are cached: a proposal of A or r (or of the
// background's a, r_bg, b) only forms the deviance from them; a proposal of a shift,
// asymmetry or width parameter (or sigma_bg) re-evaluates them.  So are the current
// peak's width factors at a = 1, W1 = 1 / (u tan^2 - v tan + w) and
// W2 = 1 / (s sec + t tan)^2: since Sigma^2 and Omega^2 both scale with a^2, a shift or
// asymmetry proposal forms G and L from them and 4 (x - mu)^2 / a^2 alone, a proposal of
// u, v or w forms W1 anew and one of s or t forms W2 anew.  Where a Caglioti argument is
// not positive the width is undefined and the energy is +inf.
#pragma once

#include "chain.hpp"

namespace smc {

struct XrdC {
    float mref, shift, ia4, u, v, w, s, t;  // shape (peak; ia4 = 4 / alpha^2); bg: s = 1 / sigma_bg^2
    float aG, aL, c0;                        // value = aG G + aL L + c0
};

// What a proposal of component q of a peak re-evaluates: nothing (A, r: linear), the shapes
// from the cached width factors (shift, alpha), W1 and the shapes (u, v, w) or W2 and the
// shapes (s, t).
enum XrdMode : int { kXrdLinear = 0, kXrdCachedW = 1, kXrdNewW1 = 2, kXrdNewW2 = 3 };
__host__ __device__ constexpr int xrd_peak_mode_c(int q) {
    return (q == 0 || q == 2) ? kXrdLinear : (q == 1 || q == 3) ? kXrdCachedW : q <= 6 ? kXrdNewW1 : kXrdNewW2;
}
__device__ __forceinline__ int xrd_peak_mode(int q) { return xrd_peak_mode_c(q); }

// Tiles whose move unrolls a peak's nine proposals (the component index, and with it the
// constants it changes, its linearity and its shape mode, known at compile time): those it
// leaves spill-free (up to 4 points per lane, 7 and 16) and 20 points per lane, where it spills
// a few words reloaded once per term and still measured 7-10% faster.  The others keep the
// run-time component loop.
template <int PPL>
constexpr bool kXrdUnroll = (PPL <= 8 && PPL != 6) || PPL == 10 || PPL == 12 || PPL == 14 || PPL == 16 || PPL == 20;

// Constants of peak k (th: its nine parameters) at reference position mref.
__device__ __forceinline__ XrdC xrd_peak_consts(const float* th, float mref) {
    XrdC q;
    q.mref = mref;
    q.shift = th[1];
    q.ia4 = 4.0f * __builtin_amdgcn_rcpf(th[3] * th[3]);
    q.u = th[4];
    q.v = th[5];
    q.w = th[6];
    q.s = th[7];
    q.t = th[8];
    q.aG = th[0] * (1.0f - th[2]);
    q.aL = th[0] * th[2];
    q.c0 = 0.0f;
    return q;
}

__device__ __forceinline__ XrdC xrd_bg_consts(const float* th) {
    XrdC q{};
    q.s = __builtin_amdgcn_rcpf(th[1] * th[1]);
    q.aG = th[0] * (1.0f - th[2]);
    q.aL = th[0] * th[2];
    q.c0 = th[3];
    return q;
}

// Components of a peak that enter its value linearly (A, r) and of the background (a, r_bg, b).
__device__ __forceinline__ bool xrd_linear(bool is_bg, int q) { return is_bg ? q != 1 : (q == 0 || q == 2); }

// IWL: the move kernel keeps the reciprocal counts in LDS (move_iw_lds_bytes).
template <int L, int WPC, int PPL, bool IWL = false>
struct XrdChain {
    static constexpr int LC = L * WPC;
    static constexpr int TPB = LC > 64 ? LC : 256;   // threads per workgroup (one multi-wavefront chain)
    // Width factors cached in registers: both up to 8 points per lane, neither at 12 and 14 (3
    // waves per SIMD there: with the unrolled proposals they would spill), W2 alone at 10, 16
    // and 20 (one of the two fits there; W2 is the dearer to form, a square root and two
    // reciprocals against one); a factor not cached is formed anew by every shape proposal.
    static constexpr bool kCW1 = PPL <= 8;
    static constexpr bool kCW2 = PPL <= 10 || PPL >= 16;
    // The reciprocal of every count (as count_w keeps it) held in registers up to 8 points
    // per lane, in LDS where IWL says so; otherwise each deviance term forms it (v_rcp).
    static constexpr bool kIW = PPL <= 8;
    float x[PPL], tn[PPL], w[PPL];
    float iw[kIW ? PPL : 1];
    const float* iwl = nullptr;   // IWL: this lane's reciprocal counts in LDS, stride LC
    float D[PPL];
    float S1[PPL], S2[PPL];
    float W1[PPL], W2[PPL];   // width factors of the current term when it is a peak
    bool wbad = false;        // some Caglioti argument of the current peak is not positive

    __device__ __forceinline__ void load_points(const GroupDesc& g, int lane) {
        constexpr float kHalfRad = 3.14159265358979f / 360.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int i = lane + p * LC;
            const bool ok = i < g.n;
            x[p] = ok ? g.x[i] : kFarX;
            w[p] = ok ? count_w(g.y[i]) : -1.0f;
            if constexpr (kIW) iw[p] = 1.0f / w[p];
            tn[p] = tanf(ok ? g.x[i] * kHalfRad : 0.0f);
        }
    }

    // IWL: the reciprocal counts into this lane's LDS area (read back only by this lane).
    __device__ __forceinline__ void keep_iw(float* dst) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) dst[p * LC] = 1.0f / w[p];
        iwl = dst;
    }

    // Width factors of a peak at point p (a = 1): W1 = 1 / Caglioti argument (`bad` collects
    // the points where that argument is not positive) and W2 = 1 / Omega0^2.
    __device__ __forceinline__ float peak_w1(const XrdC& q, int p, bool& bad) const {
        const float c = __builtin_fmaf(__builtin_fmaf(q.u, tn[p], -q.v), tn[p], q.w);
        bad |= !(c > 0.0f);
        return __builtin_amdgcn_rcpf(c);
    }

    __device__ __forceinline__ float peak_w2(const XrdC& q, int p) const {
        // sec(x/2) from an opaque copy of tan(x/2): hoisted out of the sweep loop it would
        // cost PPL more live registers.  The hardware square root (about 1 ulp, argument in
        // [1, 34) here) instead of the correctly rounded sequence, a dozen more instructions
        // per point of every width evaluation
        float tv = tn[p];
        asm volatile("" : "+v"(tv));
        const float sec = __builtin_amdgcn_sqrtf(__builtin_fmaf(tv, tv, 1.0f));
        const float om = __builtin_fmaf(q.s, sec, q.t * tn[p]);
        return __builtin_amdgcn_rcpf(om * om);
    }

    // Shapes of a peak at point p from its width factors: with z = 4 (x - mu)^2 / a^2,
    // G = 2^(-z W1) (= exp(-4 ln2 (x - mu)^2 / Sigma^2)) and L = 1 / (1 + z W2).
    __device__ __forceinline__ void peak_shape_w(const XrdC& q, int p, float w1, float w2, float& e,
                                                 float& l) const {
        // x - mu as (x - mu_ref) - shift: x - mu_ref is exact near the peak (both FP32,
        // within a factor of 2), so d carries no rounding of mu_ref + shift, which at
        // 2theta ~ 30 is ~1e-6 degrees, enough to move the energy of a narrow peak by
        // more than 1e-5 relative
        const float d = (x[p] - q.mref) - q.shift;
        const float z = d * d * (d >= 0.0f ? q.ia4 : 4.0f);
        e = __builtin_amdgcn_exp2f(-z * w1);
        l = __builtin_amdgcn_rcpf(__builtin_fmaf(z, w2, 1.0f));
    }

    // Shapes of a peak at point p, widths evaluated; `bad` collects undefined widths.
    __device__ __forceinline__ void peak_shape(const XrdC& q, int p, float& e, float& l, bool& bad) const {
        peak_shape_w(q, p, peak_w1(q, p, bad), peak_w2(q, p), e, l);
    }

    __device__ __forceinline__ void bg_shape(const XrdC& q, int p, float& e, float& l) const {
        float xv = x[p];   // opaque copy: 4 x^2 hoisted out of the sweep loop costs PPL registers
        asm volatile("" : "+v"(xv));
        const float z = 4.0f * xv * xv * q.s;   // 4 x^2 / sigma_bg^2
        e = __builtin_amdgcn_exp2f(-z);
        l = __builtin_amdgcn_rcpf(1.0f + z);
    }

    __device__ __forceinline__ void shape(bool is_bg, const XrdC& q, int p, float& e, float& l, bool& bad) const {
        if (is_bg) bg_shape(q, p, e, l);
        else peak_shape(q, p, e, l, bad);
    }

    __device__ __forceinline__ static float value(const XrdC& q, float e, float l) {
        return __builtin_fmaf(q.aL, l, __builtin_fmaf(q.aG, e, q.c0));
    }

    // The model at a point: the rest of the model Dp plus the term (a peak has no offset).
    template <bool BG>
    __device__ __forceinline__ static float model(float Dp, const XrdC& q, float e, float l) {
        return __builtin_fmaf(q.aL, l, __builtin_fmaf(q.aG, e, BG ? Dp + q.c0 : Dp));
    }

    // acc plus the deviance term of point p at model value f (poisson_dev_acc: a model
    // value <= 0 makes the sum +inf or NaN, which the energy maps to +inf).  Padding points
    // (x = kFarX), which only the rows from ppl_before(PPL) on hold (the tile rule), leave
    // acc as it is: the constant background keeps their model away from 1.
    __device__ __forceinline__ float dev(float acc, int p, float f) const {
        float iwp;
        if constexpr (kIW) {
            iwp = iw[p];
        } else if constexpr (IWL) {
            iwp = iwl[p * LC];
        } else {
            // formed at every use: the empty asm keeps the compiler from hoisting the
            // reciprocals out of the sweep loop into PPL more registers
            float wp = w[p];
            asm volatile("" : "+v"(wp));
            iwp = __builtin_amdgcn_rcpf(wp);
        }
        const float r = poisson_dev_acc(acc, w[p], iwp, f);
        if (p < ppl_before(PPL)) return r;
        return w[p] > 0.0f ? r : acc;
    }

    // Padding points contribute 0 (dev), and their shapes are never evaluated into anything
    // but that term.
    template <bool BG>
    __device__ __forceinline__ float partial_cached_t(const XrdC& q) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) acc = dev(acc, p, model<BG>(D[p], q, S1[p], S2[p]));
        return acc;
    }

    __device__ __forceinline__ float partial_cached(bool is_bg, const XrdC& q) const {
        return is_bg ? partial_cached_t<true>(q) : partial_cached_t<false>(q);
    }

    // A proposal's shapes at point p: the background's evaluated; a peak's from its width
    // factors, cached or (the one the proposal changes) formed anew.
    template <bool BG, int MODE>
    __device__ __forceinline__ void prop_shape(const XrdC& q, int p, float& e, float& l, bool& bad) const {
        if constexpr (BG) {
            bg_shape(q, p, e, l);
        } else {
            const float w1 = (MODE == kXrdNewW1 || !kCW1) ? peak_w1(q, p, bad) : W1[p];
            const float w2 = (MODE == kXrdNewW2 || !kCW2) ? peak_w2(q, p) : W2[p];
            peak_shape_w(q, p, w1, w2, e, l);
        }
    }

    // The lane's share of a shape proposal's energy; with STORE, the proposal's shapes are
    // left at sl[p * LC] (float2 units: this lane's entries of its chain's LDS area) for an
    // accept.  A proposal that keeps the Caglioti argument inherits its validity.
    template <bool BG, int MODE, bool STORE>
    __device__ __forceinline__ float partial_shape_t(const XrdC& q, float2* sl) const {
        float acc = 0.0f;
        bool bad = !BG && kCW1 && MODE != kXrdNewW1 && wbad;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            float e, l;
            prop_shape<BG, MODE>(q, p, e, l, bad);
            if constexpr (STORE) sl[p * LC] = make_float2(e, l);
            acc = dev(acc, p, model<BG>(D[p], q, e, l));
        }
        return bad ? __builtin_inff() : acc;
    }

    template <bool STORE>
    __device__ __forceinline__ float partial_shape(bool is_bg, int mode, const XrdC& q, float2* sl) const {
        if (is_bg) return partial_shape_t<true, kXrdCachedW, STORE>(q, sl);
        if (mode == kXrdCachedW) return partial_shape_t<false, kXrdCachedW, STORE>(q, sl);
        if (mode == kXrdNewW1) return partial_shape_t<false, kXrdNewW1, STORE>(q, sl);
        return partial_shape_t<false, kXrdNewW2, STORE>(q, sl);
    }

    __device__ __forceinline__ void load_shapes(const float2* sl) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const float2 v = sl[p * LC];
            S1[p] = v.x;
            S2[p] = v.y;
        }
    }

    // The current term's shapes (and, for a peak, its width factors) from its constants.
    __device__ __forceinline__ void set_shapes(bool is_bg, const XrdC& q) {
        if (is_bg) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) bg_shape(q, p, S1[p], S2[p]);
            return;
        }
        bool bad = false;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const float w1 = peak_w1(q, p, bad), w2 = peak_w2(q, p);
            if constexpr (kCW1) W1[p] = w1;
            if constexpr (kCW2) W2[p] = w2;
            peak_shape_w(q, p, w1, w2, S1[p], S2[p]);
        }
        wbad = bad;
    }

    // An accepted shape proposal becomes current: its shapes (from LDS when STORED) and the
    // width factor it changed.
    template <bool STORED>
    __device__ __forceinline__ void accept_shape(bool is_bg, int mode, const XrdC& q, const float2* sl) {
        if constexpr (!STORED) {
            set_shapes(is_bg, q);
            return;
        }
        load_shapes(sl);
        if (is_bg) return;
        if (kCW1 && mode == kXrdNewW1) {
            bool bad = false;
#pragma unroll
            for (int p = 0; p < PPL; ++p) W1[p] = peak_w1(q, p, bad);
            wbad = bad;
        } else if (kCW2 && mode == kXrdNewW2) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) W2[p] = peak_w2(q, p);
        }
    }

    // Term k joins the fixed part of the model in D (from its cached shapes, or evaluated).
    __device__ __forceinline__ void include_cached(const XrdC& q) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) D[p] += value(q, S1[p], S2[p]);
    }

    __device__ __forceinline__ bool include_eval(bool is_bg, const XrdC& q) {
        bool bad = false;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            float e, l;
            shape(is_bg, q, p, e, l, bad);
            D[p] += value(q, e, l);
        }
        return bad;
    }

    // Term k becomes current: its shapes cached and its value taken out of D.
    __device__ __forceinline__ void exclude(bool is_bg, const XrdC& q) {
        set_shapes(is_bg, q);
#pragma unroll
        for (int p = 0; p < PPL; ++p) D[p] -= value(q, S1[p], S2[p]);
    }

    __device__ __forceinline__ static XrdC term_consts(const GroupDesc& g, const float* th, int k) {
        return k < g.K ? xrd_peak_consts(th + k * g.np, g.mu_ref[k]) : xrd_bg_consts(th + g.K * g.np);
    }

    // Constants of term k with its component q replaced by vn, formed from the chain's
    // parameter vector in LDS (mref: the peak's reference position).
    __device__ __forceinline__ static XrdC term_consts_with(const GroupDesc& g, const float* th, int k, int q,
                                                            float vn, float mref) {
        if (k < g.K) {
            float t9[9];
            const float* b = th + k * 9;
#pragma unroll
            for (int u = 0; u < 9; ++u) t9[u] = u == q ? vn : b[u];
            return xrd_peak_consts(t9, mref);
        }
        float t4[4];
        const float* b = th + g.K * 9;
#pragma unroll
        for (int u = 0; u < 4; ++u) t4[u] = u == q ? vn : b[u];
        return xrd_bg_consts(t4);
    }

    // Rebuild D and the shapes of term 0 from th; the lane's share of the energy (+inf where
    // a width is undefined anywhere in the chain's points of this lane).
    __device__ __forceinline__ float rebuild(const GroupDesc& g, const float* th) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) D[p] = 0.0f;
        bool bad = false;
        for (int k = g.K; k >= 1; --k) bad |= include_eval(k == g.K, term_consts(g, th, k));
        const XrdC q0 = term_consts(g, th, 0);
        set_shapes(false, q0);
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) acc = dev(acc, p, model<false>(D[p], q0, S1[p], S2[p]));
        return (bad || wbad) ? __builtin_inff() : acc;
    }

    __device__ __forceinline__ void transition(const GroupDesc& g, const float* th, int from, int to) {
        include_cached(term_consts(g, th, from));
        exclude(to == g.K, term_consts(g, th, to));
    }
};

// Workgroups of TPB threads hold TPB / LC chains; XCD dealing in chunks of 16 chains,
// whole 64-byte lines of the component-major parameter arrays.
template <int L, int WPC, int PPL>
__global__ void __launch_bounds__(L* WPC > 64 ? L * WPC : 256) k_energy_xrd(const GroupDesc* __restrict__ groups,
                                                                             const MoveWork* __restrict__ work) {
    using CS = XrdChain<L, WPC, PPL>;
    constexpr int LC = CS::LC;
    constexpr int CPW = CS::TPB / LC;
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, 16 / CPW)];
    const GroupDesc& g = groups[w.group];
    extern __shared__ float lds[];
    const int slot = threadIdx.x / LC, lane = threadIdx.x % LC;
    const int d = g.d;
    float* th = lds + slot * d;
    float* red = lds + CPW * d;
    const bool active = slot < w.nchains;
    const int i = w.chain0 + slot;
    if (active)
        for (int j = lane; j < d; j += LC) th[j] = g.theta[(size_t)j * g.P + i];
    __syncthreads();
    if (!active) return;
    CS cs;
    cs.load_points(g, lane);
    int parity = 0;
    const float e = poisson_energy(chain_sum<L, WPC>(cs.rebuild(g, th), red, parity));
    if (lane == 0) g.energy[i] = e;
}


template <int L, int WPC, int PPL>
__global__ void __launch_bounds__(L* WPC > 64 ? L * WPC : 256, xrd_min_waves(PPL))
    k_move_xrd(const GroupDesc* __restrict__ groups, const MoveWork* __restrict__ work) {
    constexpr int kIB = move_iw_lds_bytes(SMC_PEAK_XRD, PPL, L * WPC);
    using CS = XrdChain<L, WPC, PPL, (kIB > 0)>;
    constexpr int LC = CS::LC;
    constexpr int TPB = CS::TPB;
    constexpr int CPW = TPB / LC;
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, 16 / CPW)];
    const GroupDesc& g = groups[w.group];
    GroupState* st = g.st;
    if (st->done) return;
    const int d = g.d;

    extern __shared__ float lds[];
    const int slot = threadIdx.x / LC, lane = threadIdx.x % LC;
    float* body = lds + kPriorFloats * d;
    float* th = body + slot * 3 * d;
    float* inc = th + d;
    float* lnu = inc + d;
    uint32_t* accc = reinterpret_cast<uint32_t*>(body + CPW * 3 * d);
    float* red = body + CPW * 3 * d + d;
    uint32_t* nevals = reinterpret_cast<uint32_t*>(red + 2 * WPC);
    // the proposal's shapes, [chain slot][point][lane] float2, 8-byte aligned after the above
    constexpr int kSB = move_shape_lds_bytes(SMC_PEAK_XRD, SMC_NOISE_POISSON, PPL, LC);
    float* shp_base = lds + ((kPriorFloats * d + CPW * 3 * d + d + 2 * WPC + 2 + 1) & ~1);
    float2* my_shp = reinterpret_cast<float2*>(shp_base) + (slot * PPL * LC + lane);
    // the reciprocal counts (kIB > 0), [chain slot][point][lane] float, after the shapes
    float* my_iw = shp_base + (kSB / 4) * CPW * PPL * LC + (slot * PPL * LC + lane);

    const bool active = slot < w.nchains;
    const int m = w.chain0 + slot;
    const int n = g.n_moves;
    const float beta = static_cast<float>(st->beta);
    const uint32_t stage = static_cast<uint32_t>(st->stage);
    const uint32_t K = static_cast<uint32_t>(g.K);

    for (int j = threadIdx.x; j < d; j += TPB) accc[j] = 0u;
    if (threadIdx.x < 2) nevals[threadIdx.x] = 0u;
    uint32_t my_shape = 0, my_linear = 0;
    float E = 0.0f;
    if (active) {
        for (int j = lane; j < d; j += LC) th[j] = g.start[(size_t)j * g.M + m];
        E = g.start_e[m];
    }
    CS cs;
    if (active) {
        cs.load_points(g, lane);
        if constexpr (kIB > 0) cs.keep_iw(my_iw);
    }
    const int kt = g.K + 1;
    int parity = 0;

    for (int t = 0; t < n; ++t) {
        __syncthreads();
        if (active) {
            for (int j = lane; j < d; j += LC) {
                const uint4 r = draw(g.key0, g.key1, (uint32_t)m, stage, (uint32_t)(t * d + j), K, kPurposeMove);
                inc[j] = g.step[j] * box_muller(r.x, r.y);
                lnu[j] = fast_ln(u01(r.z));
            }
        }
        __syncthreads();
        if (active) {
            if (t % kRebuildEvery == 0) E = poisson_energy(chain_sum<L, WPC>(cs.rebuild(g, th), red, parity));
            else cs.transition(g, th, kt - 1, 0);
            for (int k = 0; k < kt; ++k) {
                const bool is_bg = k == g.K;
                const int j0 = is_bg ? g.K * g.np : k * g.np;
                const int nq = is_bg ? g.nbg : g.np;
                if (k > 0) cs.transition(g, th, k - 1, k);
                // the current peak's reference position, read once per term (each proposal
                // forms its constants from the chain's parameter vector; keeping them all in
                // registers between proposals measured slower at 4 points per lane)
                const float mref = is_bg ? 0.0f : g.mu_ref[k];
                if constexpr (kXrdUnroll<PPL>) {
                    if (!is_bg) {
                        // one proposal of peak component QC (compile time)
                        auto propose = [&](auto qtag) {
                            constexpr int QC = decltype(qtag)::value;
                            constexpr int kMode = xrd_peak_mode_c(QC);
                            const int j = j0 + QC;
                            const DevPrior pr = constant_load(g.prior + j);
                            if (pr.kind == SMC_PRIOR_FIXED) return;
                            const float vo = th[j];
                            const float vn = vo + inc[j];
                            if (!chain_uniform<L>(prior_in_support(pr, vn))) return;
                            const XrdC qn = CS::term_consts_with(g, th, k, QC, vn, mref);
                            float part;
                            if constexpr (kMode == kXrdLinear) {
                                part = cs.template partial_cached_t<false>(qn);
                                ++my_linear;
                            } else {
                                part = cs.template partial_shape_t<false, kMode, (kSB > 0)>(qn, my_shp);
                                ++my_shape;
                            }
                            const float En = poisson_energy(chain_sum<L, WPC>(part, red, parity));
                            const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
                            if (chain_uniform<L>(lnu[j] < log_alpha)) {
                                E = En;
                                if constexpr (kMode != kXrdLinear) cs.template accept_shape<(kSB > 0)>(false, kMode, qn, my_shp);
                                th[j] = vn;
                                if (lane == 0) atomicAdd(&accc[j], 1u);
                            }
                        };
                        propose(std::integral_constant<int, 0>{});
                        propose(std::integral_constant<int, 1>{});
                        propose(std::integral_constant<int, 2>{});
                        propose(std::integral_constant<int, 3>{});
                        propose(std::integral_constant<int, 4>{});
                        propose(std::integral_constant<int, 5>{});
                        propose(std::integral_constant<int, 6>{});
                        propose(std::integral_constant<int, 7>{});
                        propose(std::integral_constant<int, 8>{});
                        continue;
                    }
                }
                for (int q = 0; q < nq; ++q) {
                    const int j = j0 + q;
                    const DevPrior pr = constant_load(g.prior + j);   // one component per chain: scalar loads
                    if (pr.kind == SMC_PRIOR_FIXED) continue;
                    const float vo = th[j];
                    const float vn = vo + inc[j];
                    if (!chain_uniform<L>(prior_in_support(pr, vn))) continue;
                    const XrdC qn = CS::term_consts_with(g, th, k, q, vn, mref);
                    const bool linear = xrd_linear(is_bg, q);
                    const int mode = is_bg ? kXrdCachedW : xrd_peak_mode(q);
                    float part;
                    if (linear) part = cs.partial_cached(is_bg, qn);
                    else part = cs.template partial_shape<(kSB > 0)>(is_bg, mode, qn, my_shp);
                    if (linear) ++my_linear;
                    else ++my_shape;
                    const float En = poisson_energy(chain_sum<L, WPC>(part, red, parity));
                    const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
                    if (chain_uniform<L>(lnu[j] < log_alpha)) {
                        E = En;
                        if (!linear) cs.template accept_shape<(kSB > 0)>(is_bg, mode, qn, my_shp);
                        th[j] = vn;
                        if (lane == 0) atomicAdd(&accc[j], 1u);
                    }
                }
            }
            const size_t out = g.waste_free ? (size_t)m * n + t : (size_t)m;
            if (g.waste_free || t == n - 1) {
                for (int j = lane; j < d; j += LC) g.theta[(size_t)j * g.P + out] = th[j];
                if (lane == 0) g.energy[out] = E;
            }
        }
    }
    if (active && lane == 0) {
        if (my_shape) atomicAdd(&nevals[0], my_shape);
        if (my_linear) atomicAdd(&nevals[1], my_linear);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += TPB)
        if (accc[j]) atomicAdd(&g.acc[j], accc[j]);
    if (threadIdx.x == 0 && (nevals[0] | nevals[1])) {
        atomicAdd(&g.st->evals, static_cast<unsigned long long>(nevals[0]) + nevals[1]);
        if (nevals[1]) atomicAdd(&g.st->evals_linear, static_cast<unsigned long long>(nevals[1]));
    }
}

}  // namespace smc
