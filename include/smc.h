/*
 * smc.h -- C ABI of libsmc, an MI355X (gfx950) tempered sequential Monte Carlo
 * sampler (SMCS) for Bayesian spectral deconvolution.
 *
 * Method: Nabika, Hayashi & Okada, "GPU-Accelerated Sequential Monte Carlo for
 * Bayesian Spectral Analysis", arXiv 2604.03271.  For every candidate peak
 * count K the library estimates the log evidence log Z_K = -F(K)
 * (Eq. free_energy_def) with a tempered SMC sampler (Sec. II.B.2, Eqs.
 * smc_tempered_sequence, smc_incremental_weight, smc_marginal_likelihood),
 * optionally waste-free (Sec. II.B.3), whose moves are component-wise
 * random-walk Metropolis-Hastings sweeps (Sec. II.B.4).  The forward model is a
 * sum of K Gaussian (Eq. spectral_forward_model) or XPS pseudo-Voigt
 * (Eq. xps_forward_model) peaks plus a baseline (Eq. forward_model), with
 * Gaussian noise of known sigma (App. B) or Poisson counts (Eq. xrd_poisson).
 *
 * Readings where the paper is silent: the next inverse temperature is chosen
 * by bisection so that the effective sample size of the incremental weights is
 * rho*P; resampling is systematic, on weights quantised to 2^-52 so that the
 * ancestors are exact integers; the random-walk scale of component j is
 * lambda_j times the standard deviation of that component over the resampled
 * particles, with lambda_j multiplied by exp(acceptance_j - 0.44) after every
 * stage and clamped to [0.01, 10].
 *
 * Precision: forward model, energies and Metropolis decisions in FP32;
 * log-weights, log-sum-exp, ESS, temperature bisection and log evidence in FP64.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed_lo, seed_hi ^ uid) and counter (c0, c1, c2, K << 8 | purpose):
 *   prior draw (purpose 1): c0 = particle, c1 = 0,     c2 = 256*component + attempt
 *   resampling (purpose 2): c0 = 0,        c1 = stage, c2 = 0   (uniform = word 0)
 *   move       (purpose 3): c0 = chain,    c1 = stage, c2 = sweep*d + component
 *
 * Parameter vector of a K-peak model: [peak 0][peak 1]...[peak K-1][background]
 * with (A, mu, b) per Gaussian peak (b a precision), (A, mu, sigma, eta) per
 * pseudo-Voigt peak (sigma the HWHM, eta the Gaussian fraction), and
 * background () | (b) | (c0, c1) meaning 0 | b | c0 + c1 x.
 * Particles are stored structure-of-arrays: theta[j * P + i].
 *
 * Conventions: every call returns smc_status (0 = success, negative = error);
 * no C++ exception crosses the ABI; callers own the buffers they pass; a
 * context owns its device memory until smc_free; a context is not thread-safe,
 * separate contexts are independent.  Host pointers are marked (host), device
 * pointers (device); device buffers may come from any allocator (PyTorch's
 * included) and stream arguments are hipStream_t values passed as void*.
 */
#ifndef SMC_H
#define SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t smc_status;
#define SMC_OK 0
#define SMC_EINVAL (-1)   /* invalid argument: NaN data, sigma <= 0, k_min > k_max, P % n != 0 in waste-free mode ... */
#define SMC_ENOMEM (-2)   /* a device or host allocation failed */
#define SMC_EDEVICE (-3)  /* a HIP call or kernel launch failed, or no gfx950 device */
#define SMC_ENUMERIC (-4) /* NaN energy, or every particle of some K has infinite energy */
#define SMC_ESTATE (-5)   /* call not valid in the current state (e.g. evidence of an unfinished run) */
#define SMC_EBUDGET (-6)  /* a served request can never fit the memory budget */
#define SMC_EAGAIN (-7)   /* server queue full / nothing ready yet */

enum { SMC_PEAK_GAUSS = 0, SMC_PEAK_PVOIGT = 1, SMC_PEAK_XRD = 2 };
enum { SMC_BG_NONE = 0, SMC_BG_CONST = 1, SMC_BG_LINEAR = 2, SMC_BG_SHIRLEY = 3, SMC_BG_XRD = 4 };
enum { SMC_NOISE_GAUSS = 0, SMC_NOISE_POISSON = 1, SMC_NOISE_HETERO = 2 };
enum { SMC_PRIOR_UNIFORM = 0, SMC_PRIOR_GAMMA = 1, SMC_PRIOR_NORMAL = 2, SMC_PRIOR_FIXED = 3 };

#define SMC_MAX_PEAK_PARAMS 9   /* parameters of one peak (XRD peaks have the most) */
#define SMC_MAX_BG_PARAMS 4     /* background parameters (XRD background has the most) */

/* Priors of the paper's tables (spectral_priors, xrd_priors, xps_priors):
 * UNIFORM(a = lo, b = hi) on the open interval, GAMMA(a = shape, b = rate),
 * NORMAL(a = mean, b = standard deviation), FIXED(a = value; not sampled). */
typedef struct {
    int32_t kind;
    double a, b;
} smc_prior;

/* One spectrum D = {x_i, y_i} and its model family (Sec. II.A).
 * Peaks: Gaussian (A, mu, b = precision; Eq. spectral_forward_model) or pseudo-Voigt
 * (A, mu, sigma = HWHM, eta = Gaussian fraction; Eq. xps_forward_model).  Backgrounds: none,
 * constant (c), linear (c0 + c1 x), or the dynamic Shirley background of App. D (a, b): the
 * trapezoid integral of the model's peak sum from the first point, scaled so that the
 * background is a at the first and b at the last point (x must increase).  Noise: Gaussian
 * with known sigma, Poisson counts (Eq. xrd_poisson), or heteroscedastic Gaussian with
 * sigma_i^2 = s0^2 f_i + s1^2 f_i^2 + s2^2 (App. D).  The Shirley background and the
 * heteroscedastic noise go together, with pseudo-Voigt peaks and N <= 1024 (the XPS model
 * form of App. D); other combinations of these two are SMC_EINVAL.
 * The XRD powder profile of App. E: peaks (A, shift, r, alpha, u, v, w, s, t) at reference
 * positions mu_ref (position = mu_ref + shift; Caglioti Gaussian width, sec/tan Lorentzian
 * width, asymmetry alpha above the position; x in degrees 2theta, 0 < x < 180) with the
 * pseudo-Voigt background (a, sigma_bg, r_bg, b) and Poisson counts, N <= 10240; XRD peaks and
 * the XRD background go together.  A parameter vector whose squared Caglioti width is not
 * positive, or whose Lorentzian width is zero, has no defined model and gets energy +inf
 * (it is never accepted). */
typedef struct {
    int32_t n_points;            /* N >= 1; at most 8192 for the Gaussian / pseudo-Voigt families
                                    (256 lanes x 32 points), 1024 (XPS form), 10240 (XRD) */
    const double* x;             /* (host) [N]; copied at init and rounded to FP32 */
    const double* y;             /* (host) [N]; Poisson counts must be >= 0 */
    int32_t peak_kind;           /* SMC_PEAK_* */
    int32_t bg_kind;             /* SMC_BG_* */
    int32_t noise_kind;          /* SMC_NOISE_* */
    double sigma;                /* noise standard deviation (Gaussian noise), > 0 */
    smc_prior peak_prior[SMC_MAX_PEAK_PARAMS];  /* prior of each peak parameter, shared by all peaks */
    smc_prior bg_prior[SMC_MAX_BG_PARAMS];      /* prior of each background parameter */
    const smc_prior* peak_prior_k; /* (host) optional [k_max][SMC_MAX_PEAK_PARAMS] per-peak priors; NULL = peak_prior */
    int32_t k_min, k_max;        /* candidate peak counts, 1 <= k_min <= k_max */
    uint32_t uid;                /* identity of the spectrum; part of the random-number key */
    double noise_s[3];           /* s0, s1, s2 >= 0 of the heteroscedastic noise (ignored otherwise) */
    const double* mu_ref;        /* (host) XRD peaks: reference positions [k_max], copied at init and
                                    rounded to FP32; NULL otherwise */
} smc_problem;

typedef struct {
    int32_t n_particles;   /* P per candidate K, >= 2, with P * dim(k_max) <= 2^31 - 1 */
    int32_t n_moves;       /* n: MCMC sweeps per stage (standard) or chain length (waste-free) */
    int32_t waste_free;    /* 1: resample P/n chains and keep every post-sweep state (needs P % n == 0) */
    int32_t bisect_iters;  /* halvings of the temperature bisection (paper reading: 50) */
    int32_t max_stages;    /* safety cap on tempering stages (e.g. 1000) */
    double ess_frac;       /* rho: target ESS fraction of the bisection (0 < rho < 1; 0.5) */
    uint64_t seed;         /* Philox key together with the problem's uid */
    int32_t lanes_per_chain; /* 0 = automatic; otherwise 16, 32, 64 or 256 lanes per chain, or 128 or 512 (XRD only) */
    int32_t plain;         /* 1 = one K at a time, one kernel per launch (the unbatched comparator) */
    int32_t profile;       /* 1 = time every stage / move launch with HIP events (see smc_profile) */
    void* hip_stream;      /* hipStream_t to run on; NULL = the library's own stream */
} smc_options;

typedef struct smc_ctx smc_ctx;

/* Fill *opt with the defaults (P = 4096, n = 16, waste-free, 50 halvings, rho = 0.5). */
void smc_default_options(smc_options* opt);

/* Validate the problem, copy the data to the device, allocate particle state for every
 * K in [k_min, k_max] and run stage 0 (prior draws and their energies, beta = 0).
 * *out receives a context owned by the caller (release with smc_free). */
smc_status smc_init(smc_ctx** out, const smc_problem* prob, const smc_options* opt);

/* One tempering stage of every unfinished K: temperature bisection, incremental weights,
 * log-evidence increment, systematic resampling, step sizes, and the MH move at the new
 * inverse temperature.  *all_done (may be NULL) becomes 1 once every K has made its final
 * move at beta = 1. */
smc_status smc_step(smc_ctx* ctx, int32_t* all_done);

/* Every stage until every K has reached beta = 1 (including its final move): the same
 * states, traces and log Z as calling smc_step until it reports all_done, bit for bit.  Four
 * stages go into the stream per read of the small per-K state (a stage launched after a K
 * has finished does nothing for it), so the host's round trip overlaps device work.  With
 * opt.profile the timed move launches are those in which some K still had work.  Errors as
 * smc_step (the first K whose status is not SMC_OK). */
smc_status smc_run(smc_ctx* ctx);

/* Start again from stage 0 on the resident data with a new seed (no allocation, no copy of
 * the spectrum): prior draws and their energies for every K, beta = 0, log Z = 0. */
smc_status smc_reset(smc_ctx* ctx, uint64_t seed);

/* Likelihood evaluations made so far over every K: one per particle at stage 0 plus one per
 * Metropolis proposal inside the prior's support.  Each evaluation covers all N points. */
smc_status smc_evaluations(const smc_ctx* ctx, uint64_t* n_evals);

/* The evaluations of smc_evaluations by kind, out (host) [3]: {stage-0 evaluations (every
 * term evaluated), proposals that changed a peak's centre or width (its basis shapes
 * re-evaluated at every point), proposals that changed a linear coefficient (amplitude,
 * Gaussian fraction, background; residuals formed from cached shapes)}. */
smc_status smc_evaluation_kinds(const smc_ctx* ctx, uint64_t* out);

/* With options.profile = 1: out (host) [4] = {total ms of move launches, number of move
 * launches, total ms of stage launches, number of stage launches}, measured with HIP events
 * on the context's stream.  Only launches in which some K still had work count (smc_run's
 * stages launched after every K finished do not); one move launch per stage. */
smc_status smc_profile(const smc_ctx* ctx, double* out);

/* Tile autotuner: runs `stages` (1..64) tempering stages of this problem with every lane
 * count its model family supports and that holds its N points (16, 32, 64, 256; 128 and 512 for
 * XRD), times the move kernel with HIP events, and writes the lane count with the least move
 * time per particle*point evaluation to *lanes_out (and that time, ns, to *ns_per_eval_out
 * if not NULL).  Pass it as options.lanes_per_chain.  Results are cached per process and
 * device by the problem's shape and the options' P, n and mode, so a second call with the
 * same shape returns at once.  Different lane counts split the points differently, so their
 * FP32 energies differ by rounding: the default rule (lanes_per_chain = 0) is the one that
 * gives the same bits on every machine.  Allocates and frees one context per candidate.
 * Errors: SMC_EINVAL (bad problem or options, no lane count fits), SMC_EDEVICE, SMC_ENOMEM. */
smc_status smc_tune_lanes(const smc_problem* prob, const smc_options* opt, int32_t stages, int32_t* lanes_out,
                          double* ns_per_eval_out);

/* log Z_K for K = k_min .. k_min + cap - 1 into logz (host, FP64), with every constant of
 * the likelihood included, so F(K) = -logz[K - k_min].  Returns SMC_ESTATE (and the partial
 * estimates) if some K has not finished. */
smc_status smc_log_evidence(const smc_ctx* ctx, double* logz, int32_t cap);

/* Current stage index, inverse temperature, running log Z and last ESS of candidate K. */
smc_status smc_stage_info(const smc_ctx* ctx, int32_t K, int32_t* stage, double* beta, double* logz,
                          double* ess);

/* Per-stage trace of candidate K (host arrays of length cap, any may be NULL): inverse
 * temperature after the stage, ESS of the incremental weights, running log Z, mean
 * acceptance of the stage's move.  *n receives the number of stages recorded. */
smc_status smc_trace(const smc_ctx* ctx, int32_t K, double* beta, double* ess, double* logz, double* accept,
                     int32_t cap, int32_t* n);

/* Copy candidate K's particles to host memory: theta_soa [d][P] FP32 (d = dimension of the
 * K-peak model) and energies [P] FP32 (negative log-likelihood without its theta-independent
 * constant).  cap is the capacity of theta_soa in floats. */
smc_status smc_particles(const smc_ctx* ctx, int32_t K, float* theta_soa, float* energy, int64_t cap);

/* ---------------- posterior summaries (Sec. III; Eq. (free_energy_def)) ---------------- */

#define SMC_MAX_PROBS 8

/* Summaries of candidate K from its final population (beta = 1, P equally weighted
 * particles), computed on the device.  For each component j of the K-peak model (d of them):
 *   mean[j]            = (1/P) sum_i theta_ij, summed in FP64;
 *   quant[t * d + j]   = the sample value of rank max(1, ceil(probs[t] * P)) in ascending order
 *                        (inverse empirical CDF), exact, for t < n_probs <= SMC_MAX_PROBS.
 * A credible interval at level c is (q_{(1-c)/2}, q_{(1+c)/2}): probs {0.025, 0.975} give the
 * 95% interval, {0.005, 0.995} the 99% one.  relabel != 0 first sorts every particle's peaks
 * by centre (stable), since the prior is exchangeable in the peaks and per-peak summaries
 * need one labelling; the stored particles are not changed.  XRD problems take relabel = 0:
 * their peak k belongs to the reference position mu_ref[k].  mean [d] and quant
 * [n_probs * d] are host arrays.  Allocates and frees a device buffer of d * P floats when
 * relabel != 0.  Errors: SMC_EINVAL (bad K, probabilities outside [0, 1], n_probs out of
 * range, NULL outputs, relabel != 0 on an XRD problem), SMC_ESTATE (K has not reached
 * beta = 1), SMC_EDEVICE. */
smc_status smc_posterior_summary(smc_ctx* ctx, int32_t K, const double* probs, int32_t n_probs, int32_t relabel,
                                 double* mean, double* quant);

/* p(K | D) for K = k_min .. k_min + cap - 1 under a uniform prior over the candidates:
 * exp(log Z_K) normalised by the log-sum-exp of the log evidences (F = -log Z), in FP64 on
 * the host.  SMC_ESTATE if some K has not finished. */
smc_status smc_posterior_k(const smc_ctx* ctx, double* out, int32_t cap);

/* Dimension d of the K-peak model of the problem. */
int32_t smc_dim(const smc_problem* prob, int32_t K);

/* The theta-independent part of the negative log-likelihood, added in FP64 to the FP32
 * energies: (N/2) ln(2 pi sigma^2) for Gaussian noise, sum_i [y_i - y_i ln y_i + ln y_i!]
 * for Poisson counts (the kernels evaluate sum_i [f_i - y_i + y_i ln(y_i/f_i)]). */
smc_status smc_energy_constant(const smc_problem* prob, double* c);

void smc_free(smc_ctx* ctx);
const char* smc_strerror(smc_status s);

/* ---------------- batched path ---------------- */

/* Run every (spectrum, K) group of n problems to beta = 1 together: all groups advance in
 * the same launches (captured once in a hipGraph and replayed), uneven N and K included.
 * logz_out (host) receives, for problem i, k_max_i - k_min_i + 1 values in order; problems
 * are concatenated in input order. */
smc_status smc_batch_run(const smc_problem* probs, int32_t n, const smc_options* opt, double* logz_out);

/* ---------------- served path (continuous batching) ---------------- */

typedef struct smc_server smc_server;

typedef struct {
    uint64_t request_id;
    smc_status status;
    int32_t k_min, k_max;
    double logz[32];        /* log Z for K = k_min .. k_max (at most 32 candidates) */
    int32_t best_k;         /* argmax_K log Z_K (uniform prior over K) */
    double latency_s;       /* submit -> result ready */
    int32_t n_stages;       /* max stage count over the request's K */
} smc_result;

/* A server owns a device work pool; requests are admitted while the particle state they
 * need fits mem_budget_bytes, join the pool at the next stage boundary and leave it when
 * every K is done.  defaults supplies P, n, mode, rho, seed and stream. */
smc_status smc_server_create(smc_server** out, uint64_t mem_budget_bytes, const smc_options* defaults);
/* Queue a request (the problem's arrays are copied) with its own options (NULL = the server's
 * defaults; the stream field is ignored).  SMC_EBUDGET if it can never fit the budget. */
smc_status smc_server_submit(smc_server* s, const smc_problem* prob, const smc_options* opt, uint64_t request_id);
/* Collect up to cap finished results, waiting at most wait_ms (0 = poll). */
smc_status smc_server_poll(smc_server* s, smc_result* out, int32_t cap, int32_t* n_out, int32_t wait_ms);
/* Bytes of device particle state a request of this problem would hold. */
uint64_t smc_server_request_bytes(const smc_problem* prob, const smc_options* opt);
void smc_server_destroy(smc_server* s);

/* ---------------- per-kernel hooks: the production kernels on caller buffers ---------------- */

/* Philox4x32-10 of n counters: ctr (device) [n][4], out (device) [n][4]. */
smc_status smc_kernel_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, uint32_t* out, int64_t n,
                             void* stream);

/* Stage 0 of candidate K on caller buffers: prior draws theta_soa (device) [d][P] and their
 * energies (device) [P], as smc_init does. */
smc_status smc_kernel_init(const smc_problem* prob, int32_t K, int32_t P, uint64_t seed,
                           float* theta_soa, float* energy, int32_t lanes_per_chain, void* stream);

/* Energies (negative log-likelihood without its constant, FP32) of n_theta parameter
 * vectors theta_soa (device) [d][n_theta] of the K-peak model, into energy (device). */
smc_status smc_kernel_energy(const smc_problem* prob, int32_t K, const float* theta_soa, int64_t n_theta,
                             float* energy, int32_t lanes_per_chain, void* stream);

/* Temperature bisection and weight statistics of energies (device) [P] at inverse
 * temperature beta: out (host) [4] = {delta, ESS(delta), log sum_i exp(-delta E_i), min E}. */
smc_status smc_kernel_ess_bisect(const float* energy, int32_t P, double beta, double rho, int32_t iters,
                                 double* out, void* stream);

/* Systematic resampling of M ancestors (device) [M] from normalised weights (device) [P]
 * with uniform r / 2^32 (integer-exact; see the reading above). */
smc_status smc_kernel_resample(const double* weights, int32_t P, int32_t M, uint32_t r, int32_t* ancestors,
                               void* stream);

/* For callers that cannot allocate device memory (code under stream capture, serving loops
 * and harnesses that forbid hipMalloc): smc_kernel_resample with the same kernels and the same
 * ancestors, whose scratch (descriptor, group state, integer CDF [P], chunk scratch) is a
 * static device array of the library, about 8.5 MB per GPU, held until the process ends, so
 * it calls no hipMalloc / hipFree.  P is limited to SMC_NOALLOC_MAX_P (SMC_EINVAL beyond).
 * Asynchronous: the work is queued on `stream` (NULL = the null stream) and the call
 * returns without waiting; ancestors (device) [M] are valid once that work completes.  Every
 * call on one GPU shares that GPU's array, so calls whose work overlaps on one GPU (other
 * streams, other host threads) race; calls queued on one stream are ordered. */
#define SMC_NOALLOC_MAX_P (1 << 20)
smc_status smc_kernel_resample_noalloc(const double* weights, int32_t P, int32_t M, uint32_t r,
                                       int32_t* ancestors, void* stream);

/* Posterior summary kernels on caller buffers: theta (device) [d][P] FP32 component-major,
 * optional relabelling of n_peaks peaks of np parameters (centre at offset 1; 0 = none),
 * outputs as for smc_posterior_summary (host).  The device scratch (d*P floats when
 * relabelling, plus the outputs) is allocated and freed inside.  hip_stream may be NULL. */
smc_status smc_kernel_summary(const float* theta, int32_t d, int32_t P, int32_t n_peaks, int32_t np,
                              const double* probs, int32_t n_probs, double* mean, double* quant, void* hip_stream);

/* Step-size adaptation and step sizes of candidate K (Sec. II.B.4; the rule itself is a
 * reading, stated at the top of this file), as one tempering stage computes them: first
 * lambda_j <- clamp(lambda_j exp(acc_j / (M n_moves) - 0.44), 0.01, 10) for every free
 * component j, with acc (device) [d] the accepted proposals of the last move (cleared to 0
 * on return); then step (device) [d] FP32 = lambda_j * sd_j, sd_j the FP64 population
 * standard deviation of component j over the M resampled states start_soa (device) [d][M]
 * (floored at 1e-12 (|mean_j| + 1)).  lambda (device) [d] FP64 is read and updated in place.
 * Components whose prior is FIXED keep their lambda and get step 0.  Errors: SMC_EINVAL
 * (NULL buffers, K, M or n_moves < 1, an invalid problem), SMC_ENOMEM, SMC_EDEVICE. */
smc_status smc_kernel_step_sizes(const smc_problem* prob, int32_t K, const float* start_soa, int32_t M,
                                 int32_t n_moves, double* lambda, uint32_t* acc, float* step, void* stream);

/* One MH move of candidate K at inverse temperature beta: M start states start_soa
 * (device) [d][M] with energies start_e [M], step sizes step (device) [d]; outputs
 * out_soa (device) [d][P] and out_e [P] with P = M*n (waste-free) or M (standard), and
 * per-component accepted counts acc (device) [d] (accumulated, not cleared). */
smc_status smc_kernel_move(const smc_problem* prob, int32_t K, const float* start_soa, const float* start_e,
                           int32_t M, int32_t n, int32_t waste_free, double beta, uint64_t seed, uint32_t stage,
                           const float* step, float* out_soa, float* out_e, uint32_t* acc, int32_t lanes_per_chain,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif
