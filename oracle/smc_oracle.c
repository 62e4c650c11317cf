/*
 * smc_oracle.c -- plain, slow, FP64 CPU reference of the tempered sequential
 * Monte Carlo sampler (SMCS) for Bayesian spectral deconvolution described in
 * Nabika, Hayashi & Okada, "GPU-Accelerated Sequential Monte Carlo for
 * Bayesian Spectral Analysis" (arXiv 2604.03271).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: the only things both sides agree on are the
 * published definition of the Philox4x32-10 counter-based generator and the
 * counter layout written down below.
 *
 * Everything is computed in double precision, one particle after another, in
 * the order the paper states the algorithm:
 *   - forward model, Eq. (forward_model) of Sec. II.A, with the Gaussian basis
 *     of Eq. (spectral_forward_model) (App. B) and the XPS pseudo-Voigt basis of
 *     Eq. (xps_forward_model) (App. D), plus a constant or linear baseline;
 *   - energy = negative log-likelihood: Gaussian noise with known sigma
 *     (App. B, including the normalising constant) or Poisson counts
 *     (Eq. (xrd_poisson), App. C, including ln y!);
 *   - tempered targets, Eq. (smc_tempered_sequence), incremental weights,
 *     Eq. (smc_incremental_weight), normalisation and resampling, and the
 *     evidence estimator, Eq. (smc_marginal_likelihood), all in Sec. II.B.2;
 *   - waste-free SMC, Sec. II.B.3;
 *   - component-wise random-walk Metropolis-Hastings, Sec. II.B.4.
 * Where the paper is silent (temperature rule, resampling scheme, step-size
 * rule, proposal law) the readings taken here are: ESS bisection towards
 * rho*P, systematic resampling on 2^-52 fixed-point weights,
 * s_j = lambda_j * sd_j with a multiplicative acceptance rule, and a Gaussian
 * random walk.
 *
 * Parity unpinned: the step-size rule (or_step_sizes, or_update_lambda; the
 * paper defers it to another work) and the waste-free bookkeeping of or_move
 * have no value of their own that the paper or a closed form fixes; they are
 * checked only through the evidence they produce (closed-form and quadrature
 * pins of whole runs).
 *
 * An optional OpenMP pragma runs independent particles on several threads;
 * every particle draws from its own counter-keyed stream and the reductions
 * stay sequential, so the results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "smc_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with
 * the published multipliers, XOR with the round key, and a Weyl-sequence key
 * schedule with the published increments.
 * ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream layout shared with the GPU side (a convention, not arithmetic):
 *   key      = (seed_lo, seed_hi ^ uid)
 *   counter  = (c0, c1, c2, K << 8 | purpose)
 *   INIT     : c0 = particle, c1 = 0,     c2 = 256*component + attempt
 *   RESAMPLE : c0 = 0,        c1 = stage, c2 = 0
 *   MOVE     : c0 = chain,    c1 = stage, c2 = sweep*d + component        */
enum { PURPOSE_INIT = 1, PURPOSE_RESAMPLE = 2, PURPOSE_MOVE = 3 };

static void draw4(const uint32_t key[2], uint32_t c0, uint32_t c1, uint32_t c2,
                  int K, int purpose, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, ((uint32_t)K << 8) | (uint32_t)purpose};
    or_philox4x32_10(ctr, key, out);
}

/* Uniform on (0,1): (r + 1/2) / 2^32. */
double or_u01(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* Box-Muller transform of two uniforms into one standard normal (cosine branch). */
double or_box_muller(uint32_t r0, uint32_t r1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = or_u01(r0), u1 = or_u01(r1);
    return sqrt(-2.0 * log(u0)) * cos(two_pi * u1);
}

/* ------------------------------------------------------------------------
 * Parameter layout for a model with K peaks:
 *   [peak 0 params][peak 1 params]...[peak K-1 params][background params]
 * Gaussian peak (App. B): (A, mu, b) with b a precision.
 * pseudo-Voigt peak (App. D): (A, mu, sigma, eta), sigma the half width at half
 * maximum, eta the Gaussian fraction.
 * Background: none; constant (b); linear (c0, c1) -> c0 + c1*x.
 * ------------------------------------------------------------------------ */
int or_params_per_peak(int peak_kind) { return peak_kind == OR_PEAK_GAUSS ? 3 : (peak_kind == OR_PEAK_PVOIGT ? 4 : 9); }
int or_params_bg(int bg_kind)
{
    return bg_kind == OR_BG_NONE ? 0 : (bg_kind == OR_BG_CONST ? 1 : (bg_kind == OR_BG_XRD ? 4 : 2));
}
/* (The Shirley background of App. D has two parameters too: the intensities a at the first
 * and b at the last data point.) */
int or_dim(const or_problem* p, int K) { return K * or_params_per_peak(p->peak_kind) + or_params_bg(p->bg_kind); }

/* Prior of component j for a model with K peaks. */
or_prior or_component_prior(const or_problem* p, int K, int j)
{
    int np = or_params_per_peak(p->peak_kind);
    if (j < K * np) {
        int k = j / np, q = j % np;
        if (p->peak_prior_k) return p->peak_prior_k[k * 9 + q];
        return p->peak_prior[q];
    }
    return p->bg_prior[j - K * np];
}

/* One Gaussian basis function, Eq. (spectral_forward_model): A exp(-(b/2)(x-mu)^2). */
double or_peak_gauss(double x, double A, double mu, double b)
{
    double t = x - mu;
    return A * exp(-0.5 * b * t * t);
}

/* One XPS pseudo-Voigt basis function, Eq. (xps_forward_model):
 * A [ eta exp(-(x-mu)^2 / (2 (sigma/sqrt(2 ln 2))^2)) + (1-eta) sigma^2/(sigma^2+(x-mu)^2) ]. */
double or_peak_pv(double x, double A, double mu, double sigma, double eta)
{
    double t = x - mu;
    double sg = sigma / sqrt(2.0 * log(2.0));        /* Gaussian standard deviation */
    double gauss = exp(-(t * t) / (2.0 * sg * sg));
    double lorentz = (sigma * sigma) / (sigma * sigma + t * t);
    return A * (eta * gauss + (1.0 - eta) * lorentz);
}

/* XRD pseudo-Voigt, Eqs. (xrd_pvoigt, xrd_gauss, xrd_lorentz): (1 - r) G + r L with
 * G = exp(-4 ln2 ((x - rho)/Sigma)^2) and L = 1 / (1 + 4 ((x - rho)/Omega)^2), Sigma and Omega
 * full widths at half maximum. */
double or_xrd_pv(double x, double rho, double Sigma, double Omega, double r)
{
    double zg = (x - rho) / Sigma, zl = (x - rho) / Omega;
    double G = exp(-4.0 * log(2.0) * zg * zg);
    double L = 1.0 / (1.0 + 4.0 * zl * zl);
    return (1.0 - r) * G + r * L;
}

/* One XRD peak, Eq. (xrd_forward_model) with Eqs. (xrd_sigma, xrd_omega, xrd_asym): the
 * parameters t = (A, shift, r, alpha, u, v, w, s, tl), position mu = mu_ref + shift, widths
 * Sigma(x) = a sqrt(u tan^2(x/2) - v tan(x/2) + w) and Omega(x) = a (s / cos(x/2) + tl tan(x/2)),
 * a = alpha for x >= mu and 1 below, x/2 converted from degrees to radians.  NaN where the
 * Caglioti argument is not positive (the width is undefined). */
double or_peak_xrd(double x, double mu_ref, const double* t)
{
    const double pi = 3.141592653589793238462643383279502884;
    double A = t[0], mu = mu_ref + t[1], r = t[2], alpha = t[3];
    double u = t[4], v = t[5], w = t[6], s = t[7], tl = t[8];
    double h = 0.5 * x * pi / 180.0;
    double tn = tan(h), sc = 1.0 / cos(h);
    double asym = x >= mu ? alpha : 1.0;
    double c = u * tn * tn - v * tn + w;
    if (!(c > 0.0)) return NAN;
    double Sigma = asym * sqrt(c);
    double Omega = asym * (s * sc + tl * tn);
    return A * or_xrd_pv(x, mu, Sigma, Omega, r);
}

/* Sum of the K basis functions at x. */
double or_peaks(const or_problem* p, int K, const double* theta, double x)
{
    int np = or_params_per_peak(p->peak_kind);
    double f = 0.0;
    for (int k = 0; k < K; ++k) {
        const double* t = theta + k * np;
        if (p->peak_kind == OR_PEAK_GAUSS) f += or_peak_gauss(x, t[0], t[1], t[2]);
        else if (p->peak_kind == OR_PEAK_PVOIGT) f += or_peak_pv(x, t[0], t[1], t[2], t[3]);
        else f += or_peak_xrd(x, p->mu_ref ? p->mu_ref[k] : 0.0, t);
    }
    return f;
}

/* Forward model, Eq. (forward_model): sum of K basis functions plus a pointwise baseline
 * (none, constant, linear).  The Shirley baseline depends on the whole grid: or_model. */
double or_forward(const or_problem* p, int K, const double* theta, double x)
{
    double f = or_peaks(p, K, theta, x);
    const double* bg = theta + K * or_params_per_peak(p->peak_kind);
    if (p->bg_kind == OR_BG_CONST) f += bg[0];
    else if (p->bg_kind == OR_BG_LINEAR) f += bg[0] + bg[1] * x;
    else if (p->bg_kind == OR_BG_SHIRLEY) f = NAN;
    else if (p->bg_kind == OR_BG_XRD) f += bg[0] * or_xrd_pv(x, 0.0, bg[1], bg[1], bg[2]) + bg[3];
    return f;
}

/* Dynamic Shirley background (App. D, after Shirley 1972 and Herrera-Gomez 2014): the
 * inelastic background at a point is proportional to the peak intensity integrated from
 * the first data point up to it, scaled so that it equals a at the first point and b at the
 * last:  B_i = a + (b - a) C_i / C_n,  C_1 = 0,
 *        C_i = C_{i-1} + (x_i - x_{i-1}) (peaks_{i-1} + peaks_i) / 2   (trapezoid rule),
 * with peaks the model's peak sum (the "dynamic" form: the fitted peaks, not the data).
 * With no peak area (C_n = 0) the limit of a flat peak sum is used: C_i / C_n = (x_i - x_1) /
 * (x_n - x_1).  x must increase. */
void or_shirley(const double* x, const double* peaks, int n, double a, double b, double* B)
{
    double C = 0.0;
    B[0] = 0.0;
    for (int i = 1; i < n; ++i) {
        C += (x[i] - x[i - 1]) * 0.5 * (peaks[i - 1] + peaks[i]);
        B[i] = C;
    }
    for (int i = 0; i < n; ++i) {
        double u = C > 0.0 ? B[i] / C : (n > 1 ? (x[i] - x[0]) / (x[n - 1] - x[0]) : 0.0);
        B[i] = a + (b - a) * u;
    }
}

/* The forward model at every data point into f [n]. */
void or_model(const or_problem* p, int K, const double* theta, double* f)
{
    if (p->bg_kind != OR_BG_SHIRLEY) {
        for (int i = 0; i < p->n; ++i) f[i] = or_forward(p, K, theta, p->x[i]);
        return;
    }
    double* peaks = (double*)malloc(sizeof(double) * (size_t)p->n);
    for (int i = 0; i < p->n; ++i) peaks[i] = or_peaks(p, K, theta, p->x[i]);
    const double* bg = theta + K * or_params_per_peak(p->peak_kind);
    or_shirley(p->x, peaks, p->n, bg[0], bg[1], f);
    for (int i = 0; i < p->n; ++i) f[i] += peaks[i];
    free(peaks);
}

/* Energy = negative log-likelihood -ln p(D|theta), with every constant kept.
 *   Gaussian noise (App. B, sigma known):  (N/2) ln(2 pi sigma^2) + sum (y-f)^2 / (2 sigma^2)
 *   Poisson counts (Eq. (xrd_poisson)):     sum [ f - y ln f + ln y! ],  +inf if some f <= 0
 *   heteroscedastic Gaussian noise (App. D): sigma_i^2 = s0^2 f_i + s1^2 f_i^2 + s2^2 and
 *     sum [ (1/2) ln(2 pi sigma_i^2) + (y_i - f_i)^2 / (2 sigma_i^2) ],  +inf if some
 *     sigma_i^2 <= 0 (the printed form lacks the 1/2 of the quadratic term; the Gaussian
 *     negative log-likelihood has it)
 * The paper writes the energies divided by N; the tempered likelihood p(D|theta)^beta
 * uses the undivided form. */
static double energy_hetero(const or_problem* p, const double* f)
{
    const double two_pi = 6.283185307179586476925286766559;
    const double a = p->noise_s[0] * p->noise_s[0], b = p->noise_s[1] * p->noise_s[1],
                 c = p->noise_s[2] * p->noise_s[2];
    double e = 0.0;
    for (int i = 0; i < p->n; ++i) {
        double s2 = a * f[i] + b * f[i] * f[i] + c;
        if (!(s2 > 0.0) || !isfinite(s2)) return INFINITY;
        double r = p->y[i] - f[i];
        e += 0.5 * log(two_pi * s2) + r * r / (2.0 * s2);
    }
    return e;
}

double or_energy(const or_problem* p, int K, const double* theta)
{
    const double two_pi = 6.283185307179586476925286766559;
    double e = 0.0;
    if (p->noise_kind == OR_NOISE_HETERO || p->bg_kind == OR_BG_SHIRLEY) {
        double* f = (double*)malloc(sizeof(double) * (size_t)p->n);
        or_model(p, K, theta, f);
        if (p->noise_kind == OR_NOISE_HETERO) {
            e = energy_hetero(p, f);
        } else if (p->noise_kind == OR_NOISE_GAUSS) {
            double s2 = p->sigma * p->sigma;
            for (int i = 0; i < p->n; ++i) e += (p->y[i] - f[i]) * (p->y[i] - f[i]) / (2.0 * s2);
            e += 0.5 * (double)p->n * log(two_pi * s2);
        } else {
            for (int i = 0; i < p->n && isfinite(e); ++i) {
                if (!(f[i] > 0.0)) e = INFINITY;
                else e += f[i] - p->y[i] * log(f[i]) + lgamma(p->y[i] + 1.0);
            }
        }
        free(f);
        return e;
    }
    if (p->noise_kind == OR_NOISE_GAUSS) {
        double s2 = p->sigma * p->sigma;
        for (int i = 0; i < p->n; ++i) {
            double r = p->y[i] - or_forward(p, K, theta, p->x[i]);
            e += r * r / (2.0 * s2);
        }
        e += 0.5 * (double)p->n * log(two_pi * s2);
    } else {
        for (int i = 0; i < p->n; ++i) {
            double f = or_forward(p, K, theta, p->x[i]);
            if (!(f > 0.0)) return INFINITY;   /* also NaN: a width undefined at this point */
            e += f - p->y[i] * log(f) + lgamma(p->y[i] + 1.0);
        }
    }
    return e;
}

/* ------------------------------------------------------------------------
 * Priors (Tables spectral_priors, xrd_priors, xps_priors): Uniform(lo, hi) on
 * the open interval, Gamma(shape, rate), Normal(mean, sd), Fixed(value).
 * ------------------------------------------------------------------------ */
int or_prior_in_support(or_prior pr, double v)
{
    switch (pr.kind) {
    case OR_PRIOR_UNIFORM: return v > pr.a && v < pr.b;
    case OR_PRIOR_GAMMA: return v > 0.0;
    case OR_PRIOR_NORMAL: return isfinite(v);
    default: return v == pr.a;
    }
}

double or_prior_logpdf(or_prior pr, double v)
{
    if (!or_prior_in_support(pr, v)) return -INFINITY;
    switch (pr.kind) {
    case OR_PRIOR_UNIFORM: return -log(pr.b - pr.a);
    case OR_PRIOR_GAMMA: return pr.a * log(pr.b) - lgamma(pr.a) + (pr.a - 1.0) * log(v) - pr.b * v;
    case OR_PRIOR_NORMAL: {
        double z = (v - pr.a) / pr.b;
        return -0.5 * z * z - log(pr.b) - 0.5 * log(6.283185307179586476925286766559);
    }
    default: return 0.0;
    }
}

/* Draw component j of particle i for a K-peak model from its prior.
 * Uniform: inverse CDF of one uniform.  Normal: one Box-Muller normal.
 * Gamma: Marsaglia & Tsang (ACM TOMS 26(3), 2000): with d = a' - 1/3 and
 * c = 1/sqrt(9d), accept v = (1 + c z)^3 > 0 when ln u < z^2/2 + d - d v + d ln v,
 * and return d v / rate; a shape a < 1 draws with a' = a + 1 and multiplies by
 * u'^(1/a).  Attempt t uses counter word 2 = 256 j + t (at most 256 attempts). */
double or_prior_draw(or_prior pr, const uint32_t key[2], int K, uint32_t i, uint32_t j)
{
    uint32_t r[4];
    switch (pr.kind) {
    case OR_PRIOR_UNIFORM:
        draw4(key, i, 0, 256u * j, K, PURPOSE_INIT, r);
        return pr.a + (pr.b - pr.a) * or_u01(r[0]);
    case OR_PRIOR_NORMAL:
        draw4(key, i, 0, 256u * j, K, PURPOSE_INIT, r);
        return pr.a + pr.b * or_box_muller(r[0], r[1]);
    case OR_PRIOR_GAMMA: {
        double shape = pr.a < 1.0 ? pr.a + 1.0 : pr.a;
        double d = shape - 1.0 / 3.0;
        double c = 1.0 / sqrt(9.0 * d);
        for (uint32_t t = 0; t < 256u; ++t) {
            draw4(key, i, 0, 256u * j + t, K, PURPOSE_INIT, r);
            double z = or_box_muller(r[0], r[1]);
            double v = 1.0 + c * z;
            if (v <= 0.0) continue;
            v = v * v * v;
            double u = or_u01(r[2]);
            if (log(u) < 0.5 * z * z + d - d * v + d * log(v)) {
                double g = d * v;
                if (pr.a < 1.0) g *= pow(or_u01(r[3]), 1.0 / pr.a);
                return g / pr.b;
            }
        }
        return pr.a / pr.b; /* 256 rejections in a row: probability far below 1e-300 */
    }
    default:
        return pr.a;
    }
}

/* ------------------------------------------------------------------------
 * Stage 0: P independent draws from the prior and their energies.
 * theta is [P][d] row-major.
 * ------------------------------------------------------------------------ */
void or_init(const or_problem* p, int K, int P, uint64_t seed, uint32_t uid,
             double* theta, double* energy)
{
    int d = or_dim(p, K);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ uid};
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < P; ++i) {
        double* th = theta + (size_t)i * d;
        for (int j = 0; j < d; ++j) th[j] = or_prior_draw(or_component_prior(p, K, j), key, K, (uint32_t)i, (uint32_t)j);
        energy[i] = or_energy(p, K, th);
    }
}

/* ------------------------------------------------------------------------
 * Incremental weights, normalisation and ESS (Sec. II.B.2).
 * For an increment delta of the inverse temperature the unnormalised weights
 * are w_i = exp(-delta E_i).  With a_i = E_i - min E they are computed as
 * exp(-delta a_i) and the shift is restored in the log-sum-exp:
 *   S1 = sum exp(-delta a_i),  S2 = sum exp(-delta a_i)^2,
 *   ESS = S1^2 / S2,  LSE = ln sum w_i = -delta min E + ln S1.
 * ------------------------------------------------------------------------ */
static double energy_min(const double* E, int P)
{
    double m = INFINITY;
    for (int i = 0; i < P; ++i)
        if (E[i] < m) m = E[i];
    return m;
}

double or_ess(const double* E, int P, double delta, double* lse)
{
    double emin = energy_min(E, P);
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < P; ++i) {
        double w = exp(-delta * (E[i] - emin));
        s1 += w;
        s2 += w * w;
    }
    if (lse) *lse = -delta * emin + log(s1);
    return s1 * s1 / s2;
}

/* Next increment of the inverse temperature: the whole remaining gap 1-beta if
 * the ESS there is still >= rho P; otherwise `iters` halvings of [0, 1-beta]
 * keeping the low end where ESS >= rho P.  If no tested point qualifies (only
 * possible when almost every energy is +inf) the final high end is taken so
 * that the ladder still moves. */
double or_next_delta(const double* E, int P, double beta, double rho, int iters)
{
    double hi = 1.0 - beta;
    double target = rho * (double)P;
    if (or_ess(E, P, hi, NULL) >= target) return hi;
    double lo = 0.0;
    for (int it = 0; it < iters; ++it) {
        double mid = 0.5 * (lo + hi);
        if (or_ess(E, P, mid, NULL) >= target) lo = mid;
        else hi = mid;
    }
    return lo > 0.0 ? lo : hi;
}

/* ------------------------------------------------------------------------
 * Systematic resampling on fixed-point weights.  q_i = floor(W_i 2^52),
 * C_i = q_0 + ... + q_i, Q = C_{P-1}; with one uniform U = r / 2^32 the M
 * positions are (m + U) Q / M, floored, and ancestor a_m is the first j with
 * C_j > position.  All integer, so the result does not depend on summation
 * order.
 * ------------------------------------------------------------------------ */
void or_resample(const double* W, int P, int M, uint32_t r, int32_t* anc)
{
    uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)P);
    uint64_t acc = 0;
    for (int i = 0; i < P; ++i) {
        acc += (uint64_t)floor(W[i] * 4503599627370496.0); /* 2^52 */
        C[i] = acc;
    }
    uint64_t Q = acc;
    int j = 0;
    for (int m = 0; m < M; ++m) {
        unsigned __int128 num = ((unsigned __int128)(((uint64_t)m << 32) | r)) * (unsigned __int128)Q;
        unsigned __int128 den = ((unsigned __int128)(uint64_t)M) << 32;
        uint64_t pos = (uint64_t)(num / den);
        while (j < P - 1 && !(C[j] > pos)) ++j;   /* positions increase with m */
        anc[m] = j;
    }
    free(C);
}

/* ------------------------------------------------------------------------
 * Component-wise random-walk Metropolis-Hastings (Sec. II.B.4): one sweep
 * updates the components in order j = 0..d-1; a fixed component is skipped.
 * Proposal theta'_j = theta_j + s_j z, z ~ N(0,1); a proposal outside the
 * prior's support is rejected without evaluating the likelihood; otherwise
 * it is accepted when ln u < -beta (E' - E) + ln p_j(theta'_j) - ln p_j(theta_j).
 * Counter word 2 = sweep*d + j, z from words (0,1), u from word 2.
 * ------------------------------------------------------------------------ */
static void mh_sweep(const or_problem* p, int K, int d, double beta, const uint32_t key[2],
                     uint32_t chain, uint32_t stage, uint32_t sweep, const double* step,
                     double* th, double* E, int32_t* acc, int64_t* n_eval)
{
    for (int j = 0; j < d; ++j) {
        or_prior pr = or_component_prior(p, K, j);
        if (pr.kind == OR_PRIOR_FIXED) continue;
        uint32_t r[4];
        draw4(key, chain, stage, sweep * (uint32_t)d + (uint32_t)j, K, PURPOSE_MOVE, r);
        double z = or_box_muller(r[0], r[1]);
        double u = or_u01(r[2]);
        double old = th[j];
        double prop = old + step[j] * z;
        if (!or_prior_in_support(pr, prop)) continue;
        th[j] = prop;
        *n_eval += 1;
        double Enew = or_energy(p, K, th);
        double log_alpha = -beta * (Enew - *E) + or_prior_logpdf(pr, prop) - or_prior_logpdf(pr, old);
        if (log(u) < log_alpha) {
            *E = Enew;
            acc[j] += 1;
        } else {
            th[j] = old;
        }
    }
}

/* Move the M start states (rows of `start`, energies `start_E`) with n sweeps at
 * inverse temperature beta; returns the number of likelihood evaluations.  Standard mode (waste_free = 0, M = P): particle i
 * keeps its state after the n-th sweep.  Waste-free mode (Sec. II.B.3, M = P/n):
 * every post-sweep state of chain m is kept, in slot m*n + t.
 * acc[j] returns the accepted count of component j over all chains and sweeps. */
int64_t or_move(const or_problem* p, int K, int M, int n, int waste_free, double beta,
                uint64_t seed, uint32_t uid, uint32_t stage, const double* step,
                const double* start, const double* start_E, double* out, double* out_E, int32_t* acc)
{
    int d = or_dim(p, K);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ uid};
    int32_t* acc_chain = (int32_t*)calloc((size_t)M * (size_t)(d > 0 ? d : 1), sizeof(int32_t));
    int64_t n_eval = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : n_eval)
    for (int m = 0; m < M; ++m) {
        double* th = (double*)malloc(sizeof(double) * (size_t)(d > 0 ? d : 1));
        memcpy(th, start + (size_t)m * d, sizeof(double) * (size_t)d);
        double E = start_E[m];
        for (int t = 0; t < n; ++t) {
            mh_sweep(p, K, d, beta, key, (uint32_t)m, stage, (uint32_t)t, step, th, &E, acc_chain + (size_t)m * d,
                     &n_eval);
            if (waste_free) {
                size_t slot = (size_t)m * n + t;
                memcpy(out + slot * d, th, sizeof(double) * (size_t)d);
                out_E[slot] = E;
            }
        }
        if (!waste_free) {
            memcpy(out + (size_t)m * d, th, sizeof(double) * (size_t)d);
            out_E[m] = E;
        }
        free(th);
    }
    for (int j = 0; j < d; ++j) {
        int32_t s = 0;
        for (int m = 0; m < M; ++m) s += acc_chain[(size_t)m * d + j];
        acc[j] = s;
    }
    free(acc_chain);
    return n_eval;
}

/* Threads an OpenMP region of the reference would use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later parallel loops (timing only; results do not depend on it). */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Step sizes (Sec. II.B.4; the paper defers the rule to another work, so this is
 * a reading, parity unpinned): s_j = lambda_j sd_j with sd_j the population
 * standard deviation of component j over the M resampled states, floored at
 * 1e-12 (|mean| + 1). */
void or_step_sizes(const double* theta, int M, int d, const double* lambda, double* step)
{
    for (int j = 0; j < d; ++j) {
        double mean = 0.0;
        for (int m = 0; m < M; ++m) mean += theta[(size_t)m * d + j];
        mean /= (double)M;
        double var = 0.0;
        for (int m = 0; m < M; ++m) {
            double c = theta[(size_t)m * d + j] - mean;
            var += c * c;
        }
        var /= (double)M;
        double sd = sqrt(var);
        double floor_sd = 1e-12 * (fabs(mean) + 1.0);
        step[j] = lambda[j] * (sd > floor_sd ? sd : floor_sd);
    }
}

/* lambda_j <- clamp(lambda_j exp(acc_j - 0.44), 0.01, 10), acc_j the acceptance
 * rate of component j in the stage just finished (a reading, parity unpinned). */
void or_update_lambda(double* lambda, const int32_t* acc, int d, double proposals)
{
    for (int j = 0; j < d; ++j) {
        double l = lambda[j] * exp((double)acc[j] / proposals - 0.44);
        lambda[j] = l < 0.01 ? 0.01 : (l > 10.0 ? 10.0 : l);
    }
}

/* ------------------------------------------------------------------------
 * Whole sampler for one candidate K (Sec. II.B.2-II.B.4):
 *   stage 0: draw from the prior (beta = 0, log Z = 0, lambda = 1);
 *   while beta < 1:
 *     choose delta (ESS bisection), w_i = exp(-delta E_i), log Z += LSE - ln P,
 *     resample M ancestors, step sizes from them, move them at beta + delta,
 *     update lambda from the move's acceptance, beta <- beta + delta.
 * The last move runs at beta = 1 and yields the posterior particles.
 * Returns 0, or a negative code: -1 bad options, -2 out of memory,
 * -3 numerical failure (NaN energy, or every energy +inf), -4 stage cap hit.
 * ------------------------------------------------------------------------ */
int or_run(const or_problem* p, int K, const or_options* o, or_result* res)
{
    int P = o->n_particles, n = o->n_moves;
    if (P <= 0 || n <= 0) return -1;
    if (o->waste_free && P % n != 0) return -1;
    int M = o->waste_free ? P / n : P;
    int d = or_dim(p, K);
    int dd = d > 0 ? d : 1;
    uint32_t key[2] = {(uint32_t)o->seed, (uint32_t)(o->seed >> 32) ^ o->uid};

    double* theta = (double*)malloc(sizeof(double) * (size_t)P * dd);
    double* E = (double*)malloc(sizeof(double) * (size_t)P);
    double* start = (double*)malloc(sizeof(double) * (size_t)M * dd);
    double* startE = (double*)malloc(sizeof(double) * (size_t)M);
    double* W = (double*)malloc(sizeof(double) * (size_t)P);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    double* lambda = (double*)malloc(sizeof(double) * (size_t)dd);
    double* step = (double*)malloc(sizeof(double) * (size_t)dd);
    int32_t* acc = (int32_t*)calloc((size_t)dd, sizeof(int32_t));
    if (!theta || !E || !start || !startE || !W || !anc || !lambda || !step || !acc) return -2;

    or_init(p, K, P, o->seed, o->uid, theta, E);
    for (int j = 0; j < d; ++j) lambda[j] = 1.0;
    double beta = 0.0, logZ = 0.0;
    int stage = 0, status = 0;

    while (beta < 1.0) {
        for (int i = 0; i < P; ++i)
            if (isnan(E[i])) { status = -3; goto done; }
        if (!(energy_min(E, P) < INFINITY)) { status = -3; goto done; }
        if (stage >= o->max_stages) { status = -4; goto done; }
        ++stage;

        double delta = or_next_delta(E, P, beta, o->ess_frac, o->bisect_iters);
        double beta_new = (delta == 1.0 - beta) ? 1.0 : beta + delta;
        if (beta_new > 1.0) beta_new = 1.0;

        double lse;
        double ess = or_ess(E, P, delta, &lse);
        logZ += lse - log((double)P);

        double emin = energy_min(E, P);
        double s1 = 0.0;
        for (int i = 0; i < P; ++i) s1 += exp(-delta * (E[i] - emin));
        for (int i = 0; i < P; ++i) W[i] = exp(-delta * (E[i] - emin)) / s1;

        uint32_t r[4];
        draw4(key, 0, (uint32_t)stage, 0, K, PURPOSE_RESAMPLE, r);
        or_resample(W, P, M, r[0], anc);
        for (int m = 0; m < M; ++m) {
            memcpy(start + (size_t)m * d, theta + (size_t)anc[m] * d, sizeof(double) * (size_t)d);
            startE[m] = E[anc[m]];
        }

        or_step_sizes(start, M, d, lambda, step);
        or_move(p, K, M, n, o->waste_free, beta_new, o->seed, o->uid, (uint32_t)stage, step,
                start, startE, theta, E, acc);
        or_update_lambda(lambda, acc, d, (double)M * (double)n);

        if (res && res->trace_cap > stage - 1) {
            int s = stage - 1;
            if (res->beta) res->beta[s] = beta_new;
            if (res->ess) res->ess[s] = ess;
            if (res->logz) res->logz[s] = logZ;
            if (res->accept) {
                double a = 0.0;
                int nfree = 0;
                for (int j = 0; j < d; ++j)
                    if (or_component_prior(p, K, j).kind != OR_PRIOR_FIXED) { a += acc[j]; ++nfree; }
                res->accept[s] = nfree ? a / ((double)nfree * M * n) : 0.0;
            }
        }
        beta = beta_new;
    }

done:
    if (res) {
        res->log_evidence = logZ;
        res->n_stages = stage;
        if (res->theta) memcpy(res->theta, theta, sizeof(double) * (size_t)P * d);
        if (res->energy) memcpy(res->energy, E, sizeof(double) * (size_t)P);
    }
    free(theta); free(E); free(start); free(startE); free(W); free(anc);
    free(lambda); free(step); free(acc);
    return status;
}

/* ------------------------------------------------------------------------
 * Posterior summaries (Sec. III: the posterior mean and the endpoints of the
 * 95% and 99% credible intervals; Sec. II.A: p(K|D) from the free energies).
 *
 * After the final move at beta = 1 the P particles are an equally weighted
 * sample of the posterior of one K.  For each component j:
 *   mean_j     = (1/P) sum_i theta_ij
 *   quantile_q = x_(r), r = max(1, ceil(q P)), x_(1) <= ... <= x_(P) the
 *                sorted sample: the smallest sample value whose empirical
 *                CDF reaches q (inverse of the empirical CDF).
 * A credible interval at level c is (quantile_{(1-c)/2}, quantile_{(1+c)/2}).
 *
 * The prior is exchangeable in the peaks, so the per-peak marginals are only
 * meaningful after the peaks of every particle are put in one order.  With
 * relabel > 0 each particle's relabel peaks (np parameters each, centre at
 * offset 1) are first sorted by centre; equal centres keep their index order.
 * theta is particle-major, [P][d].
 * ------------------------------------------------------------------------ */
static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

void or_relabel_by_centre(double* theta, int P, int d, int n_peaks, int np)
{
    (void)d;
    for (int i = 0; i < P; ++i) {
        double* t = theta + (size_t)i * d;
        /* stable insertion sort of the peak blocks by their centre */
        for (int k = 1; k < n_peaks; ++k) {
            double blk[8];
            memcpy(blk, t + k * np, sizeof(double) * (size_t)np);
            int m = k;
            while (m > 0 && t[(m - 1) * np + 1] > blk[1]) {
                memcpy(t + m * np, t + (m - 1) * np, sizeof(double) * (size_t)np);
                --m;
            }
            memcpy(t + m * np, blk, sizeof(double) * (size_t)np);
        }
    }
}

int or_posterior_summary(const double* theta_in, int P, int d, int relabel, int np,
                         const double* probs, int n_probs, double* mean, double* quant)
{
    if (P < 1 || d < 1 || n_probs < 0 || np < 2 || np > 8 || relabel * np > d) return -1;
    double* theta = (double*)malloc(sizeof(double) * (size_t)P * d);
    double* col = (double*)malloc(sizeof(double) * (size_t)P);
    if (!theta || !col) { free(theta); free(col); return -2; }
    memcpy(theta, theta_in, sizeof(double) * (size_t)P * d);
    if (relabel > 0) or_relabel_by_centre(theta, P, d, relabel, np);
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int i = 0; i < P; ++i) {
            col[i] = theta[(size_t)i * d + j];
            s += col[i];
        }
        mean[j] = s / (double)P;
        qsort(col, (size_t)P, sizeof(double), cmp_double);
        for (int q = 0; q < n_probs; ++q) {
            double r = ceil(probs[q] * (double)P);
            if (r < 1.0) r = 1.0;
            if (r > (double)P) r = (double)P;
            quant[(size_t)q * d + j] = col[(int)r - 1];
        }
    }
    free(theta); free(col);
    return 0;
}

/* p(K|D) for a uniform prior over the candidates: exp(log Z_K) normalised, by
 * the log-sum-exp of the log evidences (Eq. (free_energy_def): F = -log Z). */
void or_posterior_k(const double* logz, int n, double* out)
{
    double m = -INFINITY;
    for (int k = 0; k < n; ++k) if (logz[k] > m) m = logz[k];
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += exp(logz[k] - m);
    for (int k = 0; k < n; ++k) out[k] = exp(logz[k] - m) / s;
}
