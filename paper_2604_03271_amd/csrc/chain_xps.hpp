// chain_xps.hpp -- likelihood and Metropolis-Hastings kernels of the XPS model form
// of App. D: pseudo-Voigt peaks (Eq. xps_forward_model) on a dynamic Shirley
// background with heteroscedastic Gaussian noise sigma_i^2 = s0^2 f + s1^2 f^2 + s2^2.
//
// The Shirley background at point i is a + (b - a) C_i / C_N, with C_i the trapezoid
// integral of the model's peak sum from the first point: every change of a peak
// changes the background at every point through a prefix sum over the points.  So
// here lane r of a chain holds the contiguous points r*PPL .. r*PPL + PPL - 1, and
// a proposal's prefix sum is a sequential sum inside each lane plus one scan of
// the lane totals across the chain's lanes (DPP row shifts inside 16-lane rows,
// lane reads across rows).  Per point each lane keeps x, y, R = y - (peak sum), the
// current peak's shapes e and l, and C; a proposal of peak k forms the change d of
// its values (shapes re-evaluated for a centre or width, cached for an amplitude or
// a Gaussian fraction), the change of C by the scan, the new background and the
// noise terms.  A background proposal (a or b) needs no scan.  Moving to the next
// peak only evaluates its shapes.  The cache is rebuilt every kXpsRebuildEvery sweeps.
#pragma once

#include "chain.hpp"

namespace smc {

// The prefix integrals of the Shirley cache take more incremental updates per sweep than
// the plain residual cache, so they are rebuilt from the parameters more often.
constexpr int kXpsRebuildEvery = 4;

// Inclusive prefix of v over the L lanes of each chain inside one wavefront (L = 16,
// 32, 64; rows of 16 lanes), and the chain's total in every lane of the chain.
template <int L>
__device__ __forceinline__ float chain_scan(float v, float& total) {
    const int lane = threadIdx.x & 63, row = lane >> 4;
    float s = v;
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x111, 0xF, 0xF, true));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x112, 0xF, 0xF, true));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x114, 0xF, 0xF, true));
    s += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, s), 0x118, 0xF, 0xF, true));
    // row totals (lane 15 of each row); lanes of chains outside this wavefront's active
    // set may hold anything, but a chain only reads its own rows
    const float t0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 15));
    const float t1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 31));
    const float t2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 47));
    const float t3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 63));
    if constexpr (L == 16) {
        total = row == 0 ? t0 : (row == 1 ? t1 : (row == 2 ? t2 : t3));
        return s;
    } else if constexpr (L == 32) {
        const float lo = row < 2 ? t0 : t2;
        total = row < 2 ? t0 + t1 : t2 + t3;
        return (row & 1) ? s + lo : s;
    } else {
        total = ((t0 + t1) + t2) + t3;
        const float add = row == 0 ? 0.0f : (row == 1 ? t0 : (row == 2 ? t0 + t1 : (t0 + t1) + t2));
        return s + add;
    }
}

// Tiles whose move unrolls a peak's four proposals: 12 and 14 points per lane with 32 or 64
// lanes per chain, which run two waves per SIMD either way and stay spill-free (elsewhere the
// unrolled form costs a wave or spills).
template <int L, int PPL>
constexpr bool kXpsUnroll = (PPL == 12 || PPL == 14) && L >= 32;

// A chain's energy from its summed shares: NaN (a variance <= 0 somewhere) becomes +inf.
__device__ __forceinline__ float xps_energy(float e) { return e == e ? e : __builtin_inff(); }

template <int L, int PPL>
struct XpsChain {
    // Point widths x[p] - x[p - 1] (the lane's first point: minus the previous lane's last x)
    // kept in registers from 12 points per lane on, where the tile runs two waves per SIMD
    // anyway; below that they are formed at each use (keeping them would cost a wave).
    static constexpr bool kDX = PPL >= 12;
    float x[PPL];
    float dx[kDX ? PPL : 1];
    float y[PPL];
    float R[PPL];   // y - (sum of all peaks)
    float S1[PPL];  // current peak: exp2(c t^2)
    float S2[PPL];  // current peak: 1 / (s^2 + t^2)
    float C[PPL];   // twice the trapezoid integral of the peak sum from the first point
    float CN;       // its value at the last point (uniform over the chain)
    float xprev;    // x of the point before this lane's first point (own first x at the start)
    float x1, xspan;  // first point and x_N - x_1 (flat-limit background)
    int nvalid;     // points of this lane below N
    int lane;       // lane inside the chain
    bool whole;     // every lane of the wavefront holds all PPL of its points below N, or none

    // Points beyond N repeat the last x, so their trapezoid widths are 0, and are masked
    // out of the energy.
    __device__ __forceinline__ void load_points(const GroupDesc& g, int ln) {
        lane = ln;
        const int i0 = ln * PPL;
        nvalid = min(max(g.n - i0, 0), PPL);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int i = min(i0 + p, g.n - 1);
            x[p] = g.x[i];
            y[p] = i0 + p < g.n ? g.y[i] : 0.0f;
        }
        // the padding is whole lanes (N a multiple of PPL): the point loops then need no
        // per-point masks, and a lane without points drops its sums
        whole = __builtin_amdgcn_ballot_w64(nvalid != 0 && nvalid != PPL) == 0;
        xprev = ln == 0 ? x[0] : g.x[min(i0, g.n) - 1];
        if constexpr (kDX) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) dx[p] = x[p] - (p == 0 ? xprev : x[p - 1]);
        }
        x1 = g.x[0];
        xspan = g.x[g.n - 1] - g.x[0];
    }

    __device__ __forceinline__ void shape_at(const PeakC& q, int p, float& e, float& l) const {
        peak_shapes<SMC_PEAK_PVOIGT>(q, x[p] - q.mu, e, l);
    }

    __device__ __forceinline__ static float value(const PeakC& q, float e, float l) {
        return __builtin_fmaf(q.aL, l, q.aG * e);
    }

    __device__ __forceinline__ void set_shapes(const PeakC& q) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) shape_at(q, p, S1[p], S2[p]);
    }

    __device__ __forceinline__ void load_shapes(const float2* sl) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const float2 v = sl[p * L];
            S1[p] = v.x;
            S2[p] = v.y;
        }
    }

    // Twice the trapezoid increments of v over this lane's points, prefix-summed over the
    // chain into out (inclusive); returns the chain total.  Without kDX the point widths are
    // formed from copies of x that an empty asm makes opaque, so that the compiler does not
    // hoist them out of the sweep loop into PPL more live registers.
    __device__ __forceinline__ float integrate(const float* v, float* out) const {
        float vprev = __shfl_up(v[PPL - 1], 1, L);
        if (lane == 0) vprev = 0.0f;   // width 0 at the first point; keep NaN-free
        float w[PPL];
        if constexpr (kDX) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) w[p] = dx[p];
        } else {
            float xp = xprev;
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                float xs = x[p];
                asm volatile("" : "+v"(xs));
                w[p] = xs - xp;
                xp = xs;
            }
        }
        float run = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            run = __builtin_fmaf(w[p], vprev + v[p], run);
            out[p] = run;
            vprev = v[p];
        }
        float total;
        const float incl = chain_scan<L>(run, total);
        const float excl = incl - run;
#pragma unroll
        for (int p = 0; p < PPL; ++p) out[p] += excl;
        return total;
    }

    // The background a + (b - a) u_i with u_i = C_i / C_N, or (x_i - x_1) / (x_N - x_1) when
    // the peak sum has no area (the flat-peak limit), as B_i = C_i * w.kc + x_i * w.kx + w.k0
    // with the weights formed once per proposal: two fmas per point.
    struct BgWeights {
        float kc, kx, k0;
    };

    __device__ __forceinline__ BgWeights bg_weights(float cn, float a, float b) const {
        const float ba = b - a;
        if (cn > 0.0f) return BgWeights{ba * __builtin_amdgcn_rcpf(cn), 0.0f, a};
        const float s = ba * __builtin_amdgcn_rcpf(xspan);
        return BgWeights{0.0f, s, __builtin_fmaf(-x1, s, a)};
    }

    __device__ __forceinline__ float background(float Cp, const BgWeights& w, int p) const {
        return __builtin_fmaf(Cp, w.kc, __builtin_fmaf(x[p], w.kx, w.k0));
    }

    // No lane of the wavefront is in the flat-peak limit (kx = 0 everywhere): the background
    // is then C_i * kc + k0, the same value without the x term (x kx + k0 = k0 exactly).
    __device__ __forceinline__ static bool flat_free(const BgWeights& w) {
        return __builtin_amdgcn_ballot_w64(w.kx != 0.0f) == 0;
    }

    // Energy terms (without (N/2) ln 2 pi) of point p with residual r: ln of the variance
    // into accl, r^2 over the variance into accq.  A variance <= 0 (no likelihood there: energy +inf) makes
    // the sums NaN (the log of a negative number, or -inf + inf, or 0 * inf), which
    // xps_energy maps to +inf once per energy instead of a test per point.
    __device__ __forceinline__ static void noise_term(float r, float yp, const float* hn, float& accl, float& accq) {
        const float f = yp - r;
        const float v = __builtin_fmaf(__builtin_fmaf(hn[1], f, hn[0]), f, hn[2]);
        accl += __builtin_amdgcn_logf(v);
        accq = __builtin_fmaf(r * r, __builtin_amdgcn_rcpf(v), accq);
    }

    // The lane's energy share from its sums over points p < nvalid: every point when the
    // padding is whole lanes (a lane without points then returns 0), else a mask per point.
    template <typename Resid>
    __device__ __forceinline__ float energy_share(const float* hn, Resid resid) const {
        float accl = 0.0f, accq = 0.0f;
        if (whole) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) noise_term(resid(p), y[p], hn, accl, accq);
            if (nvalid == 0) accl = accq = 0.0f;
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p)
                if (p < nvalid) noise_term(resid(p), y[p], hn, accl, accq);
        }
        return 0.5f * __builtin_fmaf(kLn2, accl, accq);
    }

    // Energy share of the current state with background (a, b).
    __device__ __forceinline__ float partial_state(const float* hn, float a, float b) const {
        const BgWeights w = bg_weights(CN, a, b);
        if (flat_free(w)) return energy_share(hn, [&](int p) { return R[p] - __builtin_fmaf(C[p], w.kc, w.k0); });
        return energy_share(hn, [&](int p) { return R[p] - background(C[p], w, p); });
    }

    // Proposal changing the current peak from qo to qn: d = change of the peak's values,
    // dC = change of C, dCN = change of C_N.  Returns the energy share.
    // With kStore a shape proposal also leaves its shapes at sl[p * L] (float2 units: this
    // lane's entries of its chain's LDS area) for an accept.
    template <bool kShape, bool kStore = false>
    __device__ __forceinline__ float partial_peak(const PeakC& qo, const PeakC& qn, const float* hn, float a, float b,
                                                  float* d, float* dC, float& dCN, float2* sl = nullptr) const {
        // a linear proposal keeps the shapes: the change is (delta aG) e + (delta aL) l
        const float dG = qn.aG - qo.aG, dL = qn.aL - qo.aL;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if constexpr (kShape) {
                float e, l;
                shape_at(qn, p, e, l);
                if constexpr (kStore) sl[p * L] = make_float2(e, l);
                d[p] = value(qn, e, l) - value(qo, S1[p], S2[p]);
            } else {
                d[p] = __builtin_fmaf(dL, S2[p], dG * S1[p]);
            }
        }
        dCN = integrate(d, dC);
        const BgWeights w = bg_weights(CN + dCN, a, b);
        if (flat_free(w))
            return energy_share(hn, [&](int p) { return (R[p] - d[p]) - __builtin_fmaf(C[p] + dC[p], w.kc, w.k0); });
        return energy_share(hn, [&](int p) { return (R[p] - d[p]) - background(C[p] + dC[p], w, p); });
    }

    __device__ __forceinline__ void accept_peak(const float* d, const float* dC, float dCN) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            R[p] -= d[p];
            C[p] += dC[p];
        }
        CN += dCN;
    }

    // Rebuild R, C, C_N and the shapes of peak 0 from th; returns the energy share.
    __device__ __forceinline__ float rebuild(const GroupDesc& g, const float* th) {
        float sum[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) sum[p] = 0.0f;
        for (int k = g.K - 1; k >= 0; --k) {
            const PeakC q = peak_consts<SMC_PEAK_PVOIGT>(th + k * g.np);
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                float e, l;
                shape_at(q, p, e, l);
                sum[p] += value(q, e, l);
                if (k == 0) {
                    S1[p] = e;
                    S2[p] = l;
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) R[p] = y[p] - sum[p];
        CN = integrate(sum, C);
        const float* bg = th + g.K * g.np;
        return partial_state(g.hn, bg[0], bg[1]);
    }
};

// Energies of n parameter vectors (stage 0 and the energy hook), one chain per vector.
template <int L, int PPL>
__global__ void __launch_bounds__(256) k_energy_xps(const GroupDesc* __restrict__ groups,
                                                    const MoveWork* __restrict__ work) {
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, L / 16)];
    const GroupDesc& g = groups[w.group];
    extern __shared__ float lds[];
    const int slot = threadIdx.x / L, lane = threadIdx.x % L;
    const int d = g.d;
    float* th = lds + slot * d;
    const bool active = slot < w.nchains;
    const int i = w.chain0 + slot;
    if (active)
        for (int j = lane; j < d; j += L) th[j] = g.theta[(size_t)j * g.P + i];
    __syncthreads();
    if (!active) return;
    XpsChain<L, PPL> cs;
    cs.load_points(g, lane);
    const float e = xps_energy(group_sum<L>(cs.rebuild(g, th)));
    if (lane == 0) g.energy[i] = e;
}


// MH move of a tempering stage (same stream layout, output slots and counters as k_move).
template <int L, int PPL>
__global__ void __launch_bounds__(256, xps_min_waves(PPL)) k_move_xps(const GroupDesc* __restrict__ groups,
                                                                       const MoveWork* __restrict__ work) {
    constexpr int CPW = 256 / L;
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, L / 16)];
    const GroupDesc& g = groups[w.group];
    GroupState* st = g.st;
    if (st->done) return;
    const int d = g.d;

    extern __shared__ float lds[];
    const int slot = threadIdx.x / L, lane = threadIdx.x % L;
    float* body = lds + kPriorFloats * d;
    float* th = body + slot * 3 * d;
    float* inc = th + d;
    float* lnu = inc + d;
    uint32_t* accc = reinterpret_cast<uint32_t*>(body + CPW * 3 * d);
    uint32_t* nevals = reinterpret_cast<uint32_t*>(body + CPW * 3 * d + d + 2);   // [0] shape, [1] linear
    // the proposal's shapes, [chain slot][point][lane] float2, 8-byte aligned after the above
    constexpr int kSB = move_shape_lds_bytes(SMC_PEAK_PVOIGT, SMC_NOISE_HETERO, PPL, L);
    float2* my_shp = reinterpret_cast<float2*>(lds + ((kPriorFloats * d + CPW * 3 * d + d + 4 + 1) & ~1)) + (slot * PPL * L + lane);

    const bool active = slot < w.nchains;
    const int m = w.chain0 + slot;
    const int n = g.n_moves;
    const float beta = static_cast<float>(st->beta);
    const uint32_t stage = static_cast<uint32_t>(st->stage);
    const uint32_t K = static_cast<uint32_t>(g.K);
    const int np = g.np, jbg = g.K * g.np;

    for (int j = threadIdx.x; j < d; j += 256) accc[j] = 0u;
    if (threadIdx.x < 2) nevals[threadIdx.x] = 0u;
    uint32_t my_shape = 0, my_linear = 0;
    float E = 0.0f;
    if (active) {
        for (int j = lane; j < d; j += L) th[j] = g.start[(size_t)j * g.M + m];
        E = g.start_e[m];
    }
    XpsChain<L, PPL> cs;
    if (active) cs.load_points(g, lane);
    float dd[PPL], dC[PPL];

    for (int t = 0; t < n; ++t) {
        __syncthreads();
        if (active) {
            for (int j = lane; j < d; j += L) {
                const uint4 r = draw(g.key0, g.key1, (uint32_t)m, stage, (uint32_t)(t * d + j), K, kPurposeMove);
                inc[j] = g.step[j] * box_muller(r.x, r.y);
                lnu[j] = fast_ln(u01(r.z));
            }
        }
        __syncthreads();
        if (active) {
            if (t % kXpsRebuildEvery == 0) E = xps_energy(group_sum<L>(cs.rebuild(g, th)));
            else cs.set_shapes(peak_consts<SMC_PEAK_PVOIGT>(th));
            for (int k = 0; k <= g.K; ++k) {
                const bool is_bg = k == g.K;
                if (k > 0 && !is_bg) cs.set_shapes(peak_consts<SMC_PEAK_PVOIGT>(th + k * np));
                const int j0 = is_bg ? jbg : k * np;
                const int nq = is_bg ? g.nbg : np;
                if (kXpsUnroll<L, PPL> && !is_bg) {
                    // a peak's four proposals with the component index known at compile time:
                    // the changed constant alone is formed anew, and each proposal has one path
                    const PeakC qo = peak_consts<SMC_PEAK_PVOIGT>(th + j0);
                    PeakC qc = qo;
                    auto propose = [&](auto qtag) {
                        constexpr int Q = decltype(qtag)::value;
                        constexpr bool kLin = linear_component<SMC_PEAK_PVOIGT>(Q);
                        const int j = j0 + Q;
                        const DevPrior pr = constant_load(g.prior + j);
                        if (pr.kind == SMC_PRIOR_FIXED) return;
                        const float vo = th[j];
                        const float vn = vo + inc[j];
                        if (!chain_uniform<L>(prior_in_support(pr, vn))) return;
                        float dCN = 0.0f;
                        const PeakC qn = peak_consts_with<SMC_PEAK_PVOIGT, Q>(qc, th + j0, vn);
                        const float a = th[jbg], b = th[jbg + 1];
                        float part;
                        if constexpr (kLin) {
                            part = cs.template partial_peak<false>(qc, qn, g.hn, a, b, dd, dC, dCN);
                            ++my_linear;
                        } else {
                            part = cs.template partial_peak<true, (kSB > 0)>(qc, qn, g.hn, a, b, dd, dC, dCN, my_shp);
                            ++my_shape;
                        }
                        const float En = xps_energy(group_sum<L>(part));
                        const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
                        if (chain_uniform<L>(lnu[j] < log_alpha)) {
                            E = En;
                            cs.accept_peak(dd, dC, dCN);
                            if constexpr (!kLin) {
                                if constexpr (kSB > 0) cs.load_shapes(my_shp);
                                else cs.set_shapes(qn);
                            }
                            qc = qn;
                            th[j] = vn;
                            if (lane == 0) atomicAdd(&accc[j], 1u);
                        }
                    };
                    propose(std::integral_constant<int, 0>{});
                    propose(std::integral_constant<int, 1>{});
                    propose(std::integral_constant<int, 2>{});
                    propose(std::integral_constant<int, 3>{});
                    continue;
                }
                for (int q = 0; q < nq; ++q) {
                    const int j = j0 + q;
                    const DevPrior pr = constant_load(g.prior + j);   // one component per chain: scalar loads
                    if (pr.kind == SMC_PRIOR_FIXED) continue;
                    const float vo = th[j];
                    const float vn = vo + inc[j];
                    if (!chain_uniform<L>(prior_in_support(pr, vn))) continue;
                    float part, dCN = 0.0f;
                    PeakC qn{};
                    const bool linear = is_bg || linear_component<SMC_PEAK_PVOIGT>(q);
                    if (is_bg) {
                        const float a = q == 0 ? vn : th[jbg], b = q == 1 ? vn : th[jbg + 1];
                        part = cs.partial_state(g.hn, a, b);
                    } else {
                        float tmp[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) tmp[u] = u == q ? vn : th[j0 + u];
                        const PeakC qo = peak_consts<SMC_PEAK_PVOIGT>(th + j0);
                        qn = peak_consts<SMC_PEAK_PVOIGT>(tmp);
                        const float a = th[jbg], b = th[jbg + 1];
                        if (linear) part = cs.template partial_peak<false>(qo, qn, g.hn, a, b, dd, dC, dCN);
                        else part = cs.template partial_peak<true, (kSB > 0)>(qo, qn, g.hn, a, b, dd, dC, dCN, my_shp);
                    }
                    if (linear) ++my_linear;
                    else ++my_shape;
                    const float En = xps_energy(group_sum<L>(part));
                    const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
                    if (chain_uniform<L>(lnu[j] < log_alpha)) {
                        E = En;
                        if (!is_bg) {
                            cs.accept_peak(dd, dC, dCN);
                            if (!linear) {
                                if constexpr (kSB > 0) cs.load_shapes(my_shp);
                                else cs.set_shapes(qn);
                            }
                        }
                        th[j] = vn;
                        if (lane == 0) atomicAdd(&accc[j], 1u);
                    }
                }
            }
            const size_t out = g.waste_free ? (size_t)m * n + t : (size_t)m;
            if (g.waste_free || t == n - 1) {
                for (int j = lane; j < d; j += L) g.theta[(size_t)j * g.P + out] = th[j];
                if (lane == 0) g.energy[out] = E;
            }
        }
    }
    if (active && lane == 0) {
        if (my_shape) atomicAdd(&nevals[0], my_shape);
        if (my_linear) atomicAdd(&nevals[1], my_linear);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += 256)
        if (accc[j]) atomicAdd(&g.acc[j], accc[j]);
    if (threadIdx.x == 0 && (nevals[0] | nevals[1])) {
        atomicAdd(&g.st->evals, static_cast<unsigned long long>(nevals[0]) + nevals[1]);
        if (nevals[1]) atomicAdd(&g.st->evals_linear, static_cast<unsigned long long>(nevals[1]));
    }
}

}  // namespace smc
