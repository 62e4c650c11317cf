// chain.hpp -- the likelihood and Metropolis-Hastings kernels (templates).
//
// One Markov chain (one particle's trajectory) is held by LC = L * WPC lanes:
// L consecutive lanes of a wavefront (L = 16, 32, 64), or WPC = 4 whole
// wavefronts of one workgroup.  The chain's lanes split the N data points
// (lane r holds points r, r + LC, r + 2 LC, ...; PPL of them, in VGPRs), so a
// likelihood evaluation is PPL profile evaluations per lane followed by a
// butterfly reduction over the chain's lanes.  All lanes of a chain see the
// same reduced energy and therefore take the same Metropolis decision.
//
// Component-wise random-walk MH (Sec. II.B.4): one sweep updates the d
// components in order; a proposal only changes one term of the forward model
// (one peak, or the background), so every lane keeps, per point,
//   D = y - (model without the current term)   (Gaussian noise)
//   D = model without the current term          (Poisson counts)
// and the current peak's basis shapes at every point, t = x - mu: e = 2^(c t^2)
// for a Gaussian peak (value A e); e = 2^(-u) and l = 1/u with u = 1 + t^2/s^2 for a
// pseudo-Voigt peak (value 2 A eta e + A (1 - eta) l, which is
// A [eta e^(-ln2 t^2/s^2) + (1 - eta) s^2/(s^2 + t^2)]).  The background c0 + c1 x
// needs no cache.  Each term is linear in its remaining parameters, so a proposal
// of a centre or width re-evaluates the shapes (the transcendental work); a
// proposal of an amplitude, a Gaussian fraction or a background coefficient only
// forms the residual from the cached shapes.  Moving to the next term costs one
// shape evaluation.  D and the shapes are rebuilt from scratch every few
// sweeps, so rounding cannot accumulate.
#pragma once

#include <type_traits>

#include "smc_device.hpp"

namespace smc {

// Points beyond N (the tile holds LC * PPL >= N) are loaded with x = kFarX,
// where every peak profile underflows to 0 and the background is masked, and
// with y = 0 (Gaussian noise: residual 0) or y = 1 and a model of 1 (Poisson:
// deviance 0): they contribute exactly 0, so the point loops need no bounds.
constexpr float kFarX = 1.0e18f;

// The residual cache D and the shapes are rebuilt from the parameters every
// kRebuildEvery sweeps (and at every chain start), which bounds the rounding
// they accumulate through term-to-term updates: about 2(K+1) roundings of D per
// sweep, a random walk of ~7e-7 relative after 16 sweeps, far below the 1e-5
// energy tolerance (every 8 sweeps: 1-2% more time, every 4: 3-4%).
constexpr int kRebuildEvery = 16;

// Component q of a peak enters its term linearly: amplitude (both kinds) and
// Gaussian fraction (pseudo-Voigt).
template <int PK>
__host__ __device__ constexpr bool linear_component(int q) {
    return q == 0 || (PK == SMC_PEAK_PVOIGT && q == 3);
}

// A decision that every lane of a chain takes alike (its inputs have the same bits in all
// of them).  When a chain fills whole wavefronts the ballot of the active lanes is the
// decision of the wavefront, in scalar registers, so the branch on it is a scalar branch
// and what it guards needs no lane masks.
template <int L>
__device__ __forceinline__ bool chain_uniform(bool c) {
    if constexpr (L == 64) return __builtin_amdgcn_ballot_w64(c) != 0;
    else return c;
}

template <int PK, int NZ, int L, int WPC, int PPL>
struct ChainState {
    static constexpr int LC = L * WPC;
    static constexpr bool kPV = PK == SMC_PEAK_PVOIGT;
    static constexpr bool kGaussNoise = NZ == SMC_NOISE_GAUSS;
    float x[PPL];
    float w[kGaussNoise ? 1 : PPL];    // Poisson: the point's count as count_w keeps it
    float iw[kGaussNoise ? 1 : PPL];   // and its reciprocal
    float D[PPL];
    float S1[PPL];
    float S2[kPV ? PPL : 1];

    __device__ __forceinline__ void load_points(const GroupDesc& g, int lane) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int i = lane + p * LC;
            const bool ok = i < g.n;
            x[p] = ok ? g.x[i] : kFarX;
            if constexpr (!kGaussNoise) {
                w[p] = ok ? count_w(g.y[i]) : 1.0f;
                iw[p] = 1.0f / w[p];
            }
        }
    }

    // Constants of term k (peak k < K, background k == K) from the parameter vector th.
    __device__ __forceinline__ static PeakC term_consts(const GroupDesc& g, const float* th, int k) {
        return k < g.K ? peak_consts<PK>(th + k * g.np) : bg_consts(th + g.K * g.np, g.nbg);
    }

    // Unit shapes of a peak at point p.
    __device__ __forceinline__ void shape_at(const PeakC& q, int p, float& e, float& l) const {
        peak_shapes<PK>(q, x[p] - q.mu, e, l);
    }

    __device__ __forceinline__ float s2(int p) const {
        if constexpr (kPV) return S2[p];
        else return 0.0f;
    }

    // D + sg * (value of the peak with shapes e, l): sg = -1 takes the term out of the
    // Gaussian residual, +1 adds it to the Poisson model.
    __device__ __forceinline__ static float add_peak(float Dp, float sg, const PeakC& q, float e, float l) {
        float r = __builtin_fmaf(sg * q.aG, e, Dp);
        if constexpr (kPV) r = __builtin_fmaf(sg * q.aL, l, r);
        return r;
    }

    // The background at point p; 0 at padding points, which only the rows from
    // ppl_before(PPL) on can hold (the tile rule), so the rows before need no mask.
    __device__ __forceinline__ float bg_at(const PeakC& q, int p) const {
        if (p < ppl_before(PPL)) return bg_eval(x[p], q);
        return x[p] < 1.0e17f ? bg_eval(x[p], q) : 0.0f;
    }

    // acc plus the energy term of point p given the residual r (Gaussian) or the model
    // value f (Poisson).
    __device__ __forceinline__ float point_term(float acc, float rf, int p) const {
        if constexpr (kGaussNoise) return __builtin_fmaf(rf, rf, acc);
        else return poisson_dev_acc(acc, w[p], iw[p], rf);
    }

    static constexpr float kInclude = kGaussNoise ? -1.0f : 1.0f;

    // Energy share of the current term with constants q (its shapes cached): the current
    // state, or a proposal of a linear component of the current peak.
    __device__ __forceinline__ float partial_linear(const PeakC& q) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) acc = point_term(acc, add_peak(D[p], kInclude, q, S1[p], s2(p)), p);
        return acc;
    }

    // Energy share of a proposal that changes the current peak's centre or width.
    __device__ __forceinline__ float partial_shape(const PeakC& q) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            float e, l;
            shape_at(q, p, e, l);
            acc = point_term(acc, add_peak(D[p], kInclude, q, e, l), p);
        }
        return acc;
    }

    // Energy share of a background proposal (the background is the current term).
    __device__ __forceinline__ float partial_bg(const PeakC& q) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) acc = point_term(acc, __builtin_fmaf(kInclude, bg_at(q, p), D[p]), p);
        return acc;
    }

    // A centre or width proposal that also leaves its shapes at sl[p * LC] (this lane's
    // entries of its chain's LDS area: one float, or a float2 for a pseudo-Voigt peak).
    __device__ __forceinline__ float partial_shape_store(const PeakC& q, float* sl) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            float e, l;
            shape_at(q, p, e, l);
            if constexpr (kPV) reinterpret_cast<float2*>(sl)[p * LC] = make_float2(e, l);
            else sl[p * LC] = e;
            acc = point_term(acc, add_peak(D[p], kInclude, q, e, l), p);
        }
        return acc;
    }

    // An accepted proposal whose shapes partial_shape_store left in LDS.
    __device__ __forceinline__ void load_shapes(const float* sl) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if constexpr (kPV) {
                const float2 v = reinterpret_cast<const float2*>(sl)[p * LC];
                S1[p] = v.x;
                S2[p] = v.y;
            } else {
                S1[p] = sl[p * LC];
            }
        }
    }

    // An accepted centre or width: the cached shapes follow the new constants.
    __device__ __forceinline__ void accept_shape(const PeakC& q) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            float e, l;
            shape_at(q, p, e, l);
            S1[p] = e;
            if constexpr (kPV) S2[p] = l;
        }
    }

    // Term k with constants q joins the fixed part of the model held in D.
    __device__ __forceinline__ void include(bool is_bg, const PeakC& q, bool cached) {
        if (is_bg) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) D[p] = __builtin_fmaf(kInclude, bg_at(q, p), D[p]);
        } else if (cached) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) D[p] = add_peak(D[p], kInclude, q, S1[p], s2(p));
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                float e, l;
                shape_at(q, p, e, l);
                D[p] = add_peak(D[p], kInclude, q, e, l);
            }
        }
    }

    // Term k with constants q leaves the fixed part and becomes the current term.  The
    // background needs no shapes; clearing them there ends the previous peak's shapes on
    // both paths, so they are not kept alive beside the new ones.
    __device__ __forceinline__ void exclude(bool is_bg, const PeakC& q) {
        if (is_bg) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                D[p] = __builtin_fmaf(-kInclude, bg_at(q, p), D[p]);
                S1[p] = 0.0f;
                if constexpr (kPV) S2[p] = 0.0f;
            }
        } else {
            accept_shape(q);
#pragma unroll
            for (int p = 0; p < PPL; ++p) D[p] = add_peak(D[p], -kInclude, q, S1[p], s2(p));
        }
    }

    // Rebuild D and the shapes (current term = peak 0) from th; returns this lane's share of
    // the energy.
    __device__ __forceinline__ float rebuild(const GroupDesc& g, const float* th, int lane) {
        const int kt = g.K + (g.nbg > 0 ? 1 : 0);
        if constexpr (kGaussNoise) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const int i = lane + p * LC;
                D[p] = i < g.n ? g.y[i] : 0.0f;
            }
        } else {
            // a padding point's model stays 1 (its peaks underflow to 0, its background is
            // masked), equal to its count 1: its deviance term is exactly 0
#pragma unroll
            for (int p = 0; p < PPL; ++p) D[p] = lane + p * LC < g.n ? 0.0f : 1.0f;
        }
        for (int k = kt - 1; k >= 1; --k) include(k == g.K, term_consts(g, th, k), false);
        const PeakC q0 = term_consts(g, th, 0);
        accept_shape(q0);
        return partial_linear(q0);
    }

    // The current term moves from term `from` to term `to`.
    __device__ __forceinline__ void transition(const GroupDesc& g, const float* th, int from, int to) {
        include(from == g.K, term_consts(g, th, from), true);
        exclude(to == g.K, term_consts(g, th, to));
    }
};

// Reduce over the chain's lanes; WPC > 1 combines the wavefronts through LDS
// (double-buffered by call parity, one barrier per call).
template <int L, int WPC>
__device__ __forceinline__ float chain_sum(float v, float* red, int& parity) {
    v = group_sum<L>(v);
    if constexpr (WPC == 1) {
        return v;
    } else {
        const int w = threadIdx.x / 64;
        float* buf = red + parity * WPC;
        if ((threadIdx.x & 63) == 0) buf[w] = v;
        __syncthreads();
        float s = buf[0];
#pragma unroll
        for (int q = 1; q < WPC; ++q) s += buf[q];
        parity ^= 1;
        return s;
    }
}

// ---------------------------------------------------------------------------
// Energies of n parameter vectors (one chain slot per vector): stage 0 and the
// per-kernel energy hook.  theta_soa is [d][P] with P = g.P.
// ---------------------------------------------------------------------------
template <int PK, int NZ, int L, int WPC, int PPL>
__global__ void __launch_bounds__(256) k_energy(const GroupDesc* __restrict__ groups,
                                                const MoveWork* __restrict__ work) {
    using CS = ChainState<PK, NZ, L, WPC, PPL>;
    constexpr int LC = CS::LC;
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, LC / 16)];
    const GroupDesc& g = groups[w.group];
    extern __shared__ float lds[];
    const int slot = threadIdx.x / LC, lane = threadIdx.x % LC;
    const int d = g.d;
    float* th = lds + slot * d;
    float* red = lds + (256 / LC) * d;
    const bool active = slot < w.nchains;
    const int i = w.chain0 + slot;
    if (active)
        for (int j = lane; j < d; j += LC) th[j] = g.theta[(size_t)j * g.P + i];
    __syncthreads();
    if (!active) return;
    CS cs;
    cs.load_points(g, lane);
    int parity = 0;
    float e = chain_sum<L, WPC>(cs.rebuild(g, th, lane), red, parity);
    if (NZ == SMC_NOISE_GAUSS) e *= g.inv2s2;
    else e = poisson_energy(e);
    if (lane == 0) g.energy[i] = e;
}

// ---------------------------------------------------------------------------
// MH move of a tempering stage at the group's inverse temperature st->beta.
// Chain m starts from start[.][m]; standard mode writes its state after the
// last sweep to particle m, waste-free mode writes the state after sweep t to
// particle m * n + t (Sec. II.B.3).
// LDS: per chain slot theta[d], increment s_j z_j [d], ln u_j [d] and the chain's accept
// counters [d]; then the cross-wave reduction buffer (the prior table is read from global
// memory with scalar loads: every lane of a chain proposes the same component).

template <int PK, int NZ, int L, int WPC, int PPL>
__global__ void __launch_bounds__(256, move_min_waves(PK, NZ, PPL, WPC)) k_move(const GroupDesc* __restrict__ groups,
                                              const MoveWork* __restrict__ work) {
    using CS = ChainState<PK, NZ, L, WPC, PPL>;
    constexpr int LC = CS::LC;
    constexpr int CPW = 256 / LC;
    constexpr int NP = PK == SMC_PEAK_GAUSS ? 3 : 4;   // parameters of one peak
    const MoveWork w = work[xcd_block(blockIdx.x, gridDim.x, LC / 16)];
    const GroupDesc& g = groups[w.group];
    GroupState* st = g.st;
    if (st->done) return;
    const int d = g.d;
    if (d == 0) return;

    extern __shared__ float lds[];
    // a chain of whole wavefronts: its slot is the same in every lane (a scalar), so the
    // chain's addresses and control flow are scalar too
    const int slot = L == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / LC) : threadIdx.x / LC;
    const int lane = threadIdx.x % LC;
    float* body = lds;
    float* th = body + slot * 4 * d;
    float* inc = th + d;
    float* lnu = inc + d;
    uint32_t* accs = reinterpret_cast<uint32_t*>(lnu + d);   // this chain's accepted proposals [d]
    uint32_t* acc0 = reinterpret_cast<uint32_t*>(body + 3 * d);   // the first slot's
    float* red = body + CPW * 4 * d;
    uint32_t* nevals = reinterpret_cast<uint32_t*>(red + 2 * WPC);   // [0] shape, [1] linear
    // the proposal's shapes, [chain slot][point][lane], 8-byte aligned after the above
    constexpr int kSB = move_shape_lds_bytes(PK, NZ, PPL, LC);
    float* shp = lds + ((CPW * 4 * d + 2 * WPC + 2 + 1) & ~1);
    float* my_shp = shp + (kSB / 4) * (slot * PPL * LC + lane);

    const bool active = slot < w.nchains;
    const int m = w.chain0 + slot;
    const int n = g.n_moves;
    const float beta = static_cast<float>(st->beta);
    const uint32_t stage = static_cast<uint32_t>(st->stage);
    const uint32_t K = static_cast<uint32_t>(g.K);

    for (int j = threadIdx.x; j < CPW * d; j += 256) reinterpret_cast<uint32_t*>(body)[(j / d) * 4 * d + 3 * d + j % d] = 0u;
    if (threadIdx.x < 2) nevals[threadIdx.x] = 0u;
    uint32_t my_shape = 0, my_linear = 0;
    float E = 0.0f;
    if (active) {
        for (int j = lane; j < d; j += LC) th[j] = g.start[(size_t)j * g.M + m];
        E = g.start_e[m];
    }
    CS cs;
    if (active) cs.load_points(g, lane);
    const int kt = g.K + (g.nbg > 0 ? 1 : 0);
    int parity = 0;

    // One Metropolis-Hastings proposal of component j = j0 + q of the current term (peak or
    // background) whose constants are qc, from the state tk = th + j0 of that term.  Q >= 0:
    // a peak component known at compile time (the constants are updated field by field);
    // Q == kBgComp: a background coefficient; Q == kAnyComp: a peak component known at run time
    // (16-lane chains, four to a wavefront, where the unrolled form spills).  An accept updates
    // E, qc, the cached shapes and the state.
    constexpr int kBgComp = -1, kAnyComp = -2;
    bool any_bg = false;
    int nq_any = 0;
    auto propose = [&](auto qtag, int j0, int q, float* tk, PeakC& qc, const DevPrior& pr) {
        constexpr int Q = decltype(qtag)::value;
        constexpr bool kBg = Q == kBgComp;
        constexpr bool kAny = Q == kAnyComp;
        const int qi = Q < 0 ? q : Q;
        const int j = j0 + qi;
        if (pr.kind == SMC_PRIOR_FIXED) return;
        const float vo = tk[qi];
        const float vn = vo + inc[j];
        if (!chain_uniform<L>(prior_in_support(pr, vn))) return;
        PeakC qn;
        if constexpr (kBg) {
            qn = qc;
            if (qi == 0) qn.aG = vn;
            else qn.aL = vn;
        } else if constexpr (kAny) {
            float tmp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) tmp[u] = (u < nq_any) ? tk[u] : 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u == qi) tmp[u] = vn;
            qn = any_bg ? bg_consts(tmp, g.nbg) : peak_consts<PK>(tmp);
        } else {
            qn = peak_consts_with<PK, (Q < 0 ? 0 : Q)>(qc, tk, vn);
        }
        const bool linear = kBg || (kAny && any_bg) || linear_component<PK>(qi);
        float part;
        if (kBg || (kAny && any_bg)) {
            part = cs.partial_bg(qn);
        } else if (linear) {
            part = cs.partial_linear(qn);
        } else {
            if constexpr (kSB > 0) part = cs.partial_shape_store(qn, my_shp);
            else part = cs.partial_shape(qn);
        }
        if (linear) ++my_linear;
        else ++my_shape;
        float En = chain_sum<L, WPC>(part, red, parity);
        if (NZ == SMC_NOISE_GAUSS) En *= g.inv2s2;
        else En = poisson_energy(En);
        const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
        if (chain_uniform<L>(lnu[j] < log_alpha)) {
            E = En;
            if constexpr (!kAny) qc = qn;   // (kAny: the caller forms the constants again)
            if (!linear) {
                if constexpr (kSB > 0) cs.load_shapes(my_shp);
                else cs.accept_shape(qn);
            }
            tk[qi] = vn;
            if constexpr (L == 64) {
                if (lane == 0) ++accs[j];   // this chain's own counter: one lane writes it
            } else if (lane == 0) {
                atomicAdd(&acc0[j], 1u);    // chains sharing a wavefront share the first slot's counters
            }
        }
    };

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
            if (t % kRebuildEvery == 0) {
                E = chain_sum<L, WPC>(cs.rebuild(g, th, lane), red, parity);
                if (NZ == SMC_NOISE_GAUSS) E *= g.inv2s2;
                else E = poisson_energy(E);
            } else if (kt > 1) {
                cs.transition(g, th, kt - 1, 0);
            }
            if constexpr (L >= 32) {
            // the peaks, components in order (Sec. II.B.4); the current term's constants are
            // kept in qc and its shapes in the cache
            for (int k = 0; k < g.K; ++k) {
                float* tk = th + k * NP;
                // the priors (the same component in every lane: scalar loads), each read one
                // proposal ahead (the first two before the term switch) so that its load
                // overlaps the work before it
                const DevPrior* pk = g.prior + k * NP;
                const DevPrior p0 = constant_load(pk);
                const DevPrior p1 = constant_load(pk + 1);
                PeakC qc = peak_consts<PK>(tk);
                if (k > 0) cs.exclude(false, qc);
                propose(std::integral_constant<int, 0>{}, k * NP, 0, tk, qc, p0);
                const DevPrior p2 = constant_load(pk + 2);
                propose(std::integral_constant<int, 1>{}, k * NP, 1, tk, qc, p1);
                if constexpr (NP > 3) {
                    const DevPrior p3 = constant_load(pk + 3);
                    propose(std::integral_constant<int, 2>{}, k * NP, 2, tk, qc, p2);
                    propose(std::integral_constant<int, 3>{}, k * NP, 3, tk, qc, p3);
                } else {
                    propose(std::integral_constant<int, 2>{}, k * NP, 2, tk, qc, p2);
                }
                if (k + 1 < kt) cs.include(false, qc, true);
            }
            // the background coefficients
            if (g.nbg > 0) {
                float* tb = th + g.K * NP;
                PeakC qb = bg_consts(tb, g.nbg);
                cs.exclude(true, qb);
                for (int q = 0; q < g.nbg; ++q)
                    propose(std::integral_constant<int, kBgComp>{}, g.K * NP, q, tb, qb,
                            constant_load(g.prior + g.K * NP + q));
            }
            } else {
                PeakC unused{};
                for (int k = 0; k < kt; ++k) {
                    any_bg = k == g.K;
                    const int j0 = k * NP;
                    nq_any = any_bg ? g.nbg : NP;
                    if (k > 0) cs.transition(g, th, k - 1, k);
                    for (int q = 0; q < nq_any; ++q)
                        propose(std::integral_constant<int, kAnyComp>{}, j0, q, th + j0, unused, constant_load(g.prior + j0 + q));
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
    for (int j = threadIdx.x; j < d; j += 256) {
        uint32_t a = 0;
        for (int c = 0; c < CPW; ++c) a += reinterpret_cast<const uint32_t*>(body)[c * 4 * d + 3 * d + j];
        if (a) atomicAdd(&g.acc[j], a);
    }
    if (threadIdx.x == 0 && (nevals[0] | nevals[1])) {
        atomicAdd(&g.st->evals, static_cast<unsigned long long>(nevals[0]) + nevals[1]);
        if (nevals[1]) atomicAdd(&g.st->evals_linear, static_cast<unsigned long long>(nevals[1]));
    }
}

}  // namespace smc
