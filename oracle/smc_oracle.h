/*
 * smc_oracle.h -- declarations of the FP64 CPU reference sampler (test
 * infrastructure only; see smc_oracle.c).  Not used by, and not sharing any
 * declaration with, the HIP library.
 */
#ifndef SMC_ORACLE_H
#define SMC_ORACLE_H
#include <stdint.h>

enum { OR_PEAK_GAUSS = 0, OR_PEAK_PVOIGT = 1, OR_PEAK_XRD = 2 };
enum { OR_BG_NONE = 0, OR_BG_CONST = 1, OR_BG_LINEAR = 2, OR_BG_SHIRLEY = 3, OR_BG_XRD = 4 };
enum { OR_NOISE_GAUSS = 0, OR_NOISE_POISSON = 1, OR_NOISE_HETERO = 2 };
enum { OR_PRIOR_UNIFORM = 0, OR_PRIOR_GAMMA = 1, OR_PRIOR_NORMAL = 2, OR_PRIOR_FIXED = 3 };

/* Uniform(a=lo, b=hi) | Gamma(a=shape, b=rate) | Normal(a=mean, b=sd) | Fixed(a=value) */
typedef struct {
    int32_t kind;
    double a, b;
} or_prior;

typedef struct {
    int32_t n;
    const double* x;
    const double* y;
    int32_t peak_kind, bg_kind, noise_kind;
    double sigma;
    or_prior peak_prior[9];       /* per peak parameter (up to 9: the XRD peak) */
    or_prior bg_prior[4];         /* per background parameter (up to 4: the XRD background) */
    const or_prior* peak_prior_k; /* optional [k][9] per-peak priors, NULL = peak_prior for all */
    double noise_s[3];            /* heteroscedastic noise: sigma0, sigma1, sigma2 */
    const double* mu_ref;         /* XRD peaks: reference positions [k_max] (degrees 2theta) */
} or_problem;

typedef struct {
    int32_t n_particles, n_moves, waste_free, bisect_iters, max_stages;
    double ess_frac;
    uint64_t seed;
    uint32_t uid;
} or_options;

typedef struct {
    double log_evidence;
    int32_t n_stages;
    int32_t trace_cap;
    double *beta, *ess, *logz, *accept; /* [trace_cap] per-stage trace, may be NULL */
    double *theta, *energy;             /* [P][d] and [P] final particles, may be NULL */
} or_result;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u01(uint32_t r);
double or_box_muller(uint32_t r0, uint32_t r1);

int or_params_per_peak(int peak_kind);
int or_params_bg(int bg_kind);
int or_dim(const or_problem* p, int K);
or_prior or_component_prior(const or_problem* p, int K, int j);
double or_peak_gauss(double x, double A, double mu, double b);
double or_peak_pv(double x, double A, double mu, double sigma, double eta);
double or_xrd_pv(double x, double rho, double Sigma, double Omega, double r);
double or_peak_xrd(double x, double mu_ref, const double* t);
double or_peaks(const or_problem* p, int K, const double* theta, double x);
double or_forward(const or_problem* p, int K, const double* theta, double x);
void or_shirley(const double* x, const double* peaks, int n, double a, double b, double* B);
void or_model(const or_problem* p, int K, const double* theta, double* f);
double or_energy(const or_problem* p, int K, const double* theta);

int or_prior_in_support(or_prior pr, double v);
double or_prior_logpdf(or_prior pr, double v);
double or_prior_draw(or_prior pr, const uint32_t key[2], int K, uint32_t i, uint32_t j);

void or_init(const or_problem* p, int K, int P, uint64_t seed, uint32_t uid, double* theta, double* energy);
double or_ess(const double* E, int P, double delta, double* lse);
double or_next_delta(const double* E, int P, double beta, double rho, int iters);
void or_resample(const double* W, int P, int M, uint32_t r, int32_t* anc);
int64_t or_move(const or_problem* p, int K, int M, int n, int waste_free, double beta,
                uint64_t seed, uint32_t uid, uint32_t stage, const double* step,
                const double* start, const double* start_E, double* out, double* out_E, int32_t* acc);
int or_num_threads(void);
void or_set_num_threads(int n);
void or_step_sizes(const double* theta, int M, int d, const double* lambda, double* step);
void or_update_lambda(double* lambda, const int32_t* acc, int d, double proposals);
int or_run(const or_problem* p, int K, const or_options* o, or_result* res);

void or_relabel_by_centre(double* theta, int P, int d, int n_peaks, int np);
int or_posterior_summary(const double* theta, int P, int d, int relabel, int np,
                         const double* probs, int n_probs, double* mean, double* quant);
void or_posterior_k(const double* logz, int n, double* out);

#endif
