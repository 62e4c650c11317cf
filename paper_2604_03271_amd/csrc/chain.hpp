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
// and G = the current term's value.  A proposal then costs one profile
// evaluation per point; moving to the next term costs one more.  D and G are
// rebuilt from scratch every few sweeps, so rounding cannot accumulate.
#pragma once

#include "smc_device.hpp"

namespace smc {

template <int NZ>
__device__ __forceinline__ float point_term(float D, float g, float y) {
    if constexpr (NZ == SMC_NOISE_GAUSS) {
        const float r = D - g;
        return r * r;
    } else {
        return poisson_dev(y, D + g);
    }
}

// Points beyond N (the tile holds LC * PPL >= N) are loaded with x = kFarX,
// where every peak profile underflows to 0 and the background is masked, and
// with y = 0 (Gaussian noise) or y = -1 (Poisson, which the deviance term maps
// to 0): they contribute exactly 0, so the point loops need no bounds.
constexpr float kFarX = 1.0e18f;

// The residual cache D, G is rebuilt from the parameters every kRebuildEvery
// sweeps (and at every chain start), which bounds the rounding it accumulates
// through term-to-term updates to a few sweeps.
constexpr int kRebuildEvery = 4;

template <int PK, int NZ, int L, int WPC, int PPL>
struct ChainState {
    static constexpr int LC = L * WPC;
    float x[PPL];
    float y[NZ == SMC_NOISE_POISSON ? PPL : 1];
    float D[PPL];
    float G[PPL];
    float Gn[PPL];

    __device__ __forceinline__ void load_points(const GroupDesc& g, int lane) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int i = lane + p * LC;
            const bool ok = i < g.n;
            x[p] = ok ? g.x[i] : kFarX;
            if constexpr (NZ == SMC_NOISE_POISSON) y[p] = ok ? g.y[i] : -1.0f;
        }
    }

    // Constants of term k (peak k < K, background k == K) from the parameter vector th.
    __device__ __forceinline__ static PeakC term_consts(const GroupDesc& g, const float* th, int k) {
        return k < g.K ? peak_consts<PK>(th + k * g.np) : bg_consts(th + g.K * g.np, g.nbg);
    }

    __device__ __forceinline__ void eval_term(bool is_bg, const PeakC& q, float* out) const {
        if (is_bg) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) out[p] = x[p] < 1.0e17f ? bg_eval(x[p], q) : 0.0f;
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p) out[p] = peak_eval<PK>(x[p], q);
        }
    }

    // Sum of the per-point energy terms with the current term's values `gv`.
    __device__ __forceinline__ float partial(const float* gv) const {
        float acc = 0.0f;
#pragma unroll
        for (int p = 0; p < PPL; ++p) acc += point_term<NZ>(D[p], gv[p], NZ == SMC_NOISE_POISSON ? y[p] : 0.0f);
        return acc;
    }

    // Rebuild D and G (current term = term 0) from th; returns this lane's share of the energy.
    __device__ __forceinline__ float rebuild(const GroupDesc& g, const float* th, int lane) {
        const int kt = g.K + (g.nbg > 0 ? 1 : 0);
        if constexpr (NZ == SMC_NOISE_GAUSS) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const int i = lane + p * LC;
                D[p] = i < g.n ? g.y[i] : 0.0f;
            }
        } else {
#pragma unroll
            for (int p = 0; p < PPL; ++p) D[p] = 0.0f;
        }
        for (int k = kt - 1; k >= 1; --k) {
            eval_term(k == g.K, term_consts(g, th, k), Gn);
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                if constexpr (NZ == SMC_NOISE_GAUSS) D[p] -= Gn[p];
                else D[p] += Gn[p];
            }
        }
        eval_term(0 == g.K, term_consts(g, th, 0), G);
        return partial(G);
    }

    // Make term k current: D absorbs the old term's values and releases the new one's.
    __device__ __forceinline__ void advance(bool is_bg, const PeakC& q) {
        eval_term(is_bg, q, Gn);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if constexpr (NZ == SMC_NOISE_GAUSS) D[p] = (D[p] - G[p]) + Gn[p];
            else D[p] = (D[p] + G[p]) - Gn[p];
            G[p] = Gn[p];
        }
    }

    __device__ __forceinline__ void accept() {
#pragma unroll
        for (int p = 0; p < PPL; ++p) G[p] = Gn[p];
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
    const MoveWork w = work[blockIdx.x];
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
    if (lane == 0) g.energy[i] = e;
}

// ---------------------------------------------------------------------------
// MH move of a tempering stage at the group's inverse temperature st->beta.
// Chain m starts from start[.][m]; standard mode writes its state after the
// last sweep to particle m, waste-free mode writes the state after sweep t to
// particle m * n + t (Sec. II.B.3).
// LDS per chain slot: theta[d], increment s_j z_j [d], ln u_j [d]; then the
// per-component accept counters [d] and the cross-wave reduction buffer.
// ---------------------------------------------------------------------------
// Waves per SIMD the register allocator is asked to leave room for: the cached
// point state grows with PPL (x, D, G, Gn per point, and y for Poisson counts);
// these limits are the largest that compile without spilling on gfx950.
constexpr int move_min_waves(int noise, int points) {
    return noise == SMC_NOISE_GAUSS ? (points <= 12 ? 5 : (points <= 16 ? 4 : (points <= 20 ? 3 : 2)))
                                    : (points <= 8 ? 5 : (points <= 12 ? 4 : (points <= 16 ? 3 : 2)));
}

template <int PK, int NZ, int L, int WPC, int PPL>
__global__ void __launch_bounds__(256, move_min_waves(NZ, PPL)) k_move(const GroupDesc* __restrict__ groups,
                                              const MoveWork* __restrict__ work) {
    using CS = ChainState<PK, NZ, L, WPC, PPL>;
    constexpr int LC = CS::LC;
    constexpr int CPW = 256 / LC;
    const MoveWork w = work[blockIdx.x];
    const GroupDesc& g = groups[w.group];
    GroupState* st = g.st;
    if (st->done) return;
    const int d = g.d;
    if (d == 0) return;

    extern __shared__ float lds[];
    const int slot = threadIdx.x / LC, lane = threadIdx.x % LC;
    float* th = lds + slot * 3 * d;
    float* inc = th + d;
    float* lnu = inc + d;
    uint32_t* accc = reinterpret_cast<uint32_t*>(lds + CPW * 3 * d);
    float* red = lds + CPW * 3 * d + d;
    uint32_t* nevals = reinterpret_cast<uint32_t*>(red + 2 * WPC);

    const bool active = slot < w.nchains;
    const int m = w.chain0 + slot;
    const int n = g.n_moves;
    const float beta = static_cast<float>(st->beta);
    const uint32_t stage = static_cast<uint32_t>(st->stage);
    const uint32_t K = static_cast<uint32_t>(g.K);

    for (int j = threadIdx.x; j < d; j += 256) accc[j] = 0u;
    if (threadIdx.x == 0) *nevals = 0u;
    uint32_t my_evals = 0;
    float E = 0.0f;
    if (active) {
        for (int j = lane; j < d; j += LC) th[j] = g.start[(size_t)j * g.M + m];
        E = g.start_e[m];
    }
    CS cs;
    if (active) cs.load_points(g, lane);
    const int kt = g.K + (g.nbg > 0 ? 1 : 0);
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
            if (t % kRebuildEvery == 0) {
                E = chain_sum<L, WPC>(cs.rebuild(g, th, lane), red, parity);
                if (NZ == SMC_NOISE_GAUSS) E *= g.inv2s2;
            } else if (kt > 1) {
                cs.advance(0 == g.K, CS::term_consts(g, th, 0));
            }
            for (int k = 0; k < kt; ++k) {
                const bool is_bg = k == g.K;
                const int j0 = is_bg ? g.K * g.np : k * g.np;
                const int nq = is_bg ? g.nbg : g.np;
                if (k > 0) cs.advance(is_bg, CS::term_consts(g, th, k));
                for (int q = 0; q < nq; ++q) {
                    const int j = j0 + q;
                    const DevPrior pr = g.prior[j];
                    if (pr.kind == SMC_PRIOR_FIXED) continue;
                    const float vo = th[j];
                    const float vn = vo + inc[j];
                    if (!prior_in_support(pr, vn)) continue;
                    // constants of the term with component j replaced
                    float tmp[4];
                    const float* base = th + j0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) tmp[u] = (u < nq) ? base[u] : 0.0f;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (u == q) tmp[u] = vn;
                    const PeakC qn = is_bg ? bg_consts(tmp, g.nbg) : peak_consts<PK>(tmp);
                    ++my_evals;
                    cs.eval_term(is_bg, qn, cs.Gn);
                    float En = chain_sum<L, WPC>(cs.partial(cs.Gn), red, parity);
                    if (NZ == SMC_NOISE_GAUSS) En *= g.inv2s2;
                    const float log_alpha = -beta * (En - E) + prior_log_ratio(pr, vn, vo);
                    if (lnu[j] < log_alpha) {
                        E = En;
                        cs.accept();
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
    if (active && lane == 0 && my_evals) atomicAdd(nevals, my_evals);
    __syncthreads();
    for (int j = threadIdx.x; j < d; j += 256)
        if (accc[j]) atomicAdd(&g.acc[j], accc[j]);
    if (threadIdx.x == 0 && *nevals) atomicAdd(&g.st->evals, static_cast<unsigned long long>(*nevals));
}

}  // namespace smc
