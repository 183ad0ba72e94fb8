/*
 * smcgw.h - C ABI of the MI355X (gfx950) batched gravitational-wave
 * likelihood, adjoint gradient, NUTS and SMC library.
 *
 * Method: "The Sequential Monte Carlo goes NUTS: Boosting Gravitational-Wave
 * Inference" (arXiv:2601.02336).  Every entry point below names the passage
 * that defines what it computes.
 *
 * Conventions
 *   - Every function returns an int status: 0 = OK, > 0 = warning, < 0 = error
 *     (see SMCGW_* codes; smcgw_status_string() gives a message).  On an error
 *     no output has been written unless stated.
 *   - Batch arrays (theta, logl, grad, ancestors, per-particle outputs) are
 *     DEVICE pointers owned by the caller (e.g. torch tensors' data_ptr()).
 *     Set-up arrays (event data, PSD, detectors, bounds, target parameters)
 *     are HOST pointers; the library copies them.  The library never frees
 *     or allocates caller memory; the context owns its device tables and
 *     scratch, which grow on demand.
 *   - Work is enqueued asynchronously on the context's HIP stream.  Only
 *     functions documented as synchronising wait for the GPU.
 *   - Layouts: theta is row-major [P][D] float64 over the D sampled
 *     coordinates; the 11 source parameters are, in order,
 *     (chirp mass [Msun], q = m2/m1, chi1, chi2, d_L [Mpc], inclination,
 *     polarisation, right ascension, declination, t_c [s], phi_c).
 *     Event data are [n_det][N] interleaved complex float64, the PSD is
 *     [n_det][N] one-sided float64, f_j = f_low + j df, j = 0..N-1.
 *   - Reductions use a fixed order and no floating-point atomics, so results
 *     are bitwise reproducible for a given launch configuration.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef SMCGW_H
#define SMCGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status */
#define SMCGW_OK 0
#define SMCGW_WARN_FALLBACK 1       /* a fallback was used (e.g. diagonal mass matrix) */
#define SMCGW_ERR_INVALID (-1)      /* invalid argument / null pointer */
#define SMCGW_ERR_SHAPE (-2)        /* size out of the supported range */
#define SMCGW_ERR_HIP (-3)          /* a HIP runtime call failed */
#define SMCGW_ERR_OOM (-4)          /* device allocation failed */
#define SMCGW_ERR_NOT_INIT (-5)     /* no event / prior / target set */
#define SMCGW_ERR_STALL (-6)        /* tempering ladder cannot advance */

/* ------------------------------------------------------------ enums */
enum { SMCGW_PLAIN_FP64 = 0, SMCGW_MIXED = 1 };
enum { SMCGW_TARGET_GW = 0, SMCGW_TARGET_GAUSS = 1, SMCGW_TARGET_GAUSS_X_GAUSS = 2, SMCGW_TARGET_BIMODAL = 3 };
enum { SMCGW_BND_NONE = 0, SMCGW_BND_REFLECT = 1, SMCGW_BND_PERIODIC = 2 };
enum { SMCGW_PRIOR_FLAT = 0, SMCGW_PRIOR_UNIFORM = 1, SMCGW_PRIOR_LOGUNIFORM = 2, SMCGW_PRIOR_GAUSSIAN = 3 };

#define SMCGW_MAX_DET 4
#define SMCGW_MAX_DIM 16
#define SMCGW_MAX_DEPTH 12
#define SMCGW_MAX_EVENTS 64
#define SMCGW_MAX_BINS (1 << 24)   /* frequency bins of one event (its tables stay below 2 GiB) */

typedef struct smcgw_ctx smcgw_ctx;

/* One event: frequency grid, detector count, sidereal angle and the physical
 * constants (seconds per solar mass G Msun / c^3, metres per Mpc, c). */
typedef struct {
    double f_low, df;
    int32_t n_bins, n_det;
    double gmst;
    double t_sun, mpc_m, c_light;
    int32_t pn_order;                /* 0..7: highest half-PN order kept in the phase */
    int32_t reserved;
} smcgw_event_desc;

/* An L-shaped interferometer on a sphere: latitude, longitude, azimuths of
 * the two arms measured from local East towards North (radians), radius [m]. */
typedef struct {
    double lat, lon, az_x, az_y, radius;
} smcgw_detector;

/* Prior and boundary of one sampled coordinate (Sec. 5, "Boundary
 * conditions"): uniform / log-uniform on [lo, hi], Gaussian (lo = mean,
 * hi = sigma) or flat; reflective, periodic or no boundary. */
typedef struct {
    double lo, hi;
    int32_t bnd;
    int32_t prior;
} smcgw_bounds;

/* NUTS transition settings (Sec. 4). */
typedef struct {
    double step;           /* leapfrog step size epsilon */
    double beta;           /* temperature of the target L^beta pi (Sec. 3, Eq. 3) */
    double max_delta_h;    /* divergence threshold on H - H0 */
    int32_t max_depth;     /* maximum number of trajectory doublings (<= SMCGW_MAX_DEPTH) */
    int32_t uturn;         /* 1: stop at a U-turn; 0: always build to the depth limit */
    uint64_t seed;         /* Philox4x32-10 key */
    uint64_t iteration;    /* SMC iteration (part of the Philox counter) */
    int32_t chol_per_particle;   /* 0: chol is one [D][D] factor for all particles;
                                    1: chol is [P][D][D], one factor per particle
                                    (smcgw_local_metric) */
    int32_t reserved;            /* must be 0 */
    const double *beta_device;   /* non-NULL: beta is read from this device double when the
                                    kernel starts (e.g. written by
                                    smcgw_smc_reweight_resample_async), and `beta` is ignored */
    const double *state_device;  /* non-NULL: the particles are independent SMC runs of run_size
                                    consecutive particles each, run r with the device state
                                    state_device + r SMCGW_STATE_SIZE (see smcgw_smc_iteration):
                                    its temperature, iteration index (the Philox counter) and done
                                    flag replace beta / beta_device / iteration, run r draws with
                                    key seed + r and its particles' counters count from 0 within
                                    the run, a done run's particles are left untouched, and a shared
                                    factor (chol_per_particle = 0) is one [D][D] factor per run */
    int32_t run_size;            /* particles per run when state_device is set (P a multiple of it) */
    int32_t reserved2;           /* must be 0 */
} smcgw_nuts_params;

/* ------------------------------------------------------------ SMC state
 * Device-resident state of one SMC run (SMCGW_STATE_SIZE doubles), read and
 * updated on the device by smcgw_smc_iteration, so the host never touches
 * the temperature or the evidence:
 *   [SMCGW_ST_BETA]   beta_t, the temperature reached (0 before the first iteration)
 *   [SMCGW_ST_LOGZ]   log Z_t = sum of the increments so far (Sec. 3.1, Eq. 8), FP64
 *   [SMCGW_ST_DLOGZ]  the last increment log(Z_t / Z_{t-1}) (Sec. 3.1, Eq. 7)
 *   [SMCGW_ST_ITER]   index t of the last iteration (keys its resampling and transition streams)
 *   [SMCGW_ST_NEXT]   index of the next iteration (0 at the start)
 *   [SMCGW_ST_DONE]   1 once the run has ended: its last iteration mutated at beta = 1, or the
 *                     ladder stalled; every later iteration leaves the run untouched
 *   [SMCGW_ST_STALL]  1 when beta could not advance (the run ended without reaching 1)
 * A fresh run's state is all zeros.  Per-iteration record (SMCGW_HIST_SIZE
 * doubles per row, row t written by iteration t when t < history_cap):
 *   beta_t, log Z_t, log(Z_t / Z_{t-1}), leapfrog steps of the transition,
 *   summed tree depth, divergent transitions, 1 if the population covariance
 *   fell back to its diagonal, particles whose local metric fell back. */
#define SMCGW_STATE_SIZE 8
enum { SMCGW_ST_BETA = 0, SMCGW_ST_LOGZ = 1, SMCGW_ST_DLOGZ = 2, SMCGW_ST_ITER = 3, SMCGW_ST_NEXT = 4,
       SMCGW_ST_DONE = 5, SMCGW_ST_STALL = 6 };
#define SMCGW_HIST_SIZE 8
enum { SMCGW_H_BETA = 0, SMCGW_H_LOGZ = 1, SMCGW_H_DLOGZ = 2, SMCGW_H_LEAPFROG = 3, SMCGW_H_DEPTH = 4,
       SMCGW_H_DIVERGENT = 5, SMCGW_H_MM_FALLBACK = 6, SMCGW_H_METRIC_FALLBACKS = 7 };
#define SMCGW_MAX_RUNS 64

/* One SMC iteration of n_runs independent runs (Sec. 3 and Sec. 4): run r
 * owns particles [r P, (r+1) P) of the population arrays below (all device
 * arrays, sized for n_runs * P particles), its state state[r] and its record
 * history[r][history_cap]. */
typedef struct {
    int32_t n_runs, P, D;           /* runs, particles per run, sampled coordinates */
    int32_t precision;              /* SMCGW_PLAIN_FP64 or SMCGW_MIXED (likelihood inside NUTS) */
    double *theta, *logl, *grad;    /* [n_runs P][D], [n_runs P], [n_runs P][D]: population, updated in place */
    int32_t *ancestors;             /* [n_runs P]: indices within each run after resampling */
    int32_t *n_leapfrog;            /* [n_runs P]: leapfrog steps of each particle's last transition */
    int32_t *depth;                 /* [n_runs P] doublings of the last transition */
    uint8_t *divergent;             /* [n_runs P] */
    double *accept_stat;            /* [n_runs P] (may be NULL) */
    double *inv_mass, *chol;        /* [n_runs][D][D]: population covariance and its factor, per run */
    int32_t *mm_status;             /* [n_runs]: 1 when the covariance fell back to its diagonal */
    double *chol_pp;                /* [n_runs P][D][D] per-particle local metric factors, or NULL: the
                                       population metric */
    int32_t *metric_status;         /* [n_runs P] (local metric only) */
    double *state;                  /* [n_runs][SMCGW_STATE_SIZE] */
    double *history;                /* [n_runs][history_cap][SMCGW_HIST_SIZE] (may be NULL) */
    int32_t history_cap;
    int32_t max_depth;              /* NUTS depth limit */
    double alpha;                   /* ESS target fraction (Sec. 3, Eq. 6) */
    double shrink;                  /* diagonal shrinkage of the covariance */
    double step;                    /* leapfrog step */
    double max_delta_h;             /* divergence threshold on H - H0 */
    uint64_t seed;                  /* run r uses Philox key seed + r */
    int32_t uturn;                  /* 1: NUTS stops at a U-turn */
    int32_t nuts_form;              /* SMCGW_NUTS_PERSISTENT, or SMCGW_NUTS_SWEEPS: the plain comparison form
                                       (smcgw_nuts_step_sweeps; precision SMCGW_PLAIN_FP64, the call then
                                       synchronises and cannot be captured in a graph) */
} smcgw_smc_iter_desc;
enum { SMCGW_NUTS_PERSISTENT = 0, SMCGW_NUTS_SWEEPS = 1 };

/* Message for a status code (static storage). */
const char *smcgw_status_string(int status);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *ctx receives the handle. */
int smcgw_create(smcgw_ctx **ctx, int device, void *hip_stream);

/* Destroy a context and free everything it owns (synchronises). */
int smcgw_destroy(smcgw_ctx *ctx);

/* Change the stream later calls enqueue on. */
int smcgw_set_stream(smcgw_ctx *ctx, void *hip_stream);

/* Add an event: the data d(f) and PSD S_n(f) of Sec. 2, Eq. 2.  Builds the
 * frequency-major bin tables on the device: whitened data
 * 4 df conj(d)/S f^{-7/6}, the phase basis of every bin, <d|d> and
 * sum_j 4 df f^{-7/3}/S per detector.  data_reim [n_det][N][2], psd
 * [n_det][N] and dets [n_det] are host arrays; synchronises.  *event_id
 * receives the index used by smcgw_loglike_grad's event_of_particle.
 * SMCGW_ERR_SHAPE for N outside 1..SMCGW_MAX_BINS, n_det outside
 * 1..SMCGW_MAX_DET, more than SMCGW_MAX_EVENTS events, or a detector count
 * that differs from the events already added. */
int smcgw_add_event(smcgw_ctx *ctx, const smcgw_event_desc *ev, const double *data_reim, const double *psd,
                    const smcgw_detector *dets, int *event_id);

/* Relative-binning event (Zackay, Dai & Venumadhav 2018, arXiv:1806.08792;
 * the long-segment mitigation the paper names, Secs. 2 and 7).  The data sum
 * of the likelihood of Sec. 2, Eq. 2 is evaluated only at the bin edges: with
 * a fiducial parameter point theta0 (11 source parameters, host) the ratio
 * h / h0 is taken linear in f inside each bin, so the per-bin data collapse
 * into summary data per edge, built once here on the device over the full
 * grid.  <h|h> and <d|d> keep their values over every bin (|h|^2 of this
 * waveform does not depend on the phase).  Edges come from
 * smcgw_rb_edges(eps): eps is the allowed growth of the phase-difference
 * bound inside one bin (0.1: about 300 bins and logL errors of order 1e-2
 * near the fiducial point; 0.5: about 60 bins).  The event then serves every
 * entry point like one added with smcgw_add_event (smcgw_waveform returns
 * the strain at the edges).  Arguments as smcgw_add_event; *n_edges (may
 * be NULL) receives the edge count.  Synchronises. */
int smcgw_add_event_rb(smcgw_ctx *ctx, const smcgw_event_desc *ev, const double *data_reim, const double *psd,
                       const smcgw_detector *dets, const double *theta0, double eps, int *event_id, int *n_edges);

/* Relative-binning edges for a grid f_j = f_low + j df, j < n_bins (host
 * only, no context): the phase-difference bound
 *   dpsi(f) = 2 pi sum_k sgn(g_k) (f / f*_k)^g_k,  g = -5/3, -2/3, 1, 5/3, 7/3,
 * f*_k = f_low for negative and the last grid frequency for positive g_k, is
 * cut into B = ceil(growth / eps) steps of equal growth (at most n_bins - 1);
 * edge k (0 < k < B) is the first grid index where the bound has grown by k
 * steps, edge 0 is index 0 and edge B the last index; repeated indices are
 * dropped.  Writes the grid indices to edges [cap] and returns their count,
 * or a negative status. */
int smcgw_rb_edges(double f_low, double df, int n_bins, double eps, int32_t *edges, int cap);

/* Event of every particle for the sampler entry points: event_of_particle
 * [P] is a caller-owned DEVICE array that must stay valid while the
 * sampler runs (NULL: every particle uses event 0; indices outside the
 * added events are clamped).  All events of one context share the
 * detector count. */
int smcgw_set_event_map(smcgw_ctx *ctx, const int32_t *event_of_particle);

/* Which of the 11 source parameters are sampled: param_index[dim] gives the
 * source-parameter index of each sampled coordinate; fixed11[11] (host)
 * supplies the others.  Default: dim = 11, identity. */
int smcgw_set_param_map(smcgw_ctx *ctx, int dim, const int32_t *param_index, const double *fixed11);

/* Prior and boundaries of the dim sampled coordinates (host array). */
int smcgw_set_prior(smcgw_ctx *ctx, int dim, const smcgw_bounds *bounds);

/* Likelihood used by smcgw_nuts_step / smcgw_smc_reweight_resample:
 * SMCGW_TARGET_GW (the event likelihood of Sec. 2), or an analytic test
 * likelihood over dim coordinates: GAUSS logL = -|x|^2/2; GAUSS_X_GAUSS
 * normalised N(y; x, diag s^2) with params = y[dim], s[dim]; BIMODAL the
 * unweighted sum of two normalised isotropic Gaussians of App. A
 * (params = mu1[dim], mu2[dim], sigma).  params is a host array. */
int smcgw_set_target(smcgw_ctx *ctx, int kind, int dim, const double *params, int n_params);

/* Batched log-likelihood logL = -1/2 <d-h|d-h> (Sec. 2, Eq. 2) and its
 * gradient with respect to the dim sampled coordinates (hand-written
 * adjoint; the paper differentiates automatically, Sec. 5 "JAX
 * implementation").  theta [P][dim], logl [P], grad [P][dim] (NULL: forward
 * only) are device arrays; event_of_particle [P] (device, NULL = event 0)
 * picks each particle's event, so events of different lengths share one
 * launch (indices outside [0, events) are clamped).  precision: SMCGW_PLAIN_FP64 (FP64 throughout) or SMCGW_MIXED
 * (FP64 phase and argument reduction, FP32 trigonometry and per-bin
 * products, FP32 partial sums flushed into FP64 accumulators). */
int smcgw_loglike_grad(smcgw_ctx *ctx, int P, const int32_t *event_of_particle, const double *theta, double *logl,
                       double *grad, int precision);

/* The plain comparison form of smcgw_loglike_grad: logL of Sec. 2, Eq. 2 with
 * every per-bin quantity in FP64 (FP64 sin / cos, the per-bin |h|^2 written
 * out) and the gradient by forward-mode tangents, the derivatives with
 * respect to the 11 source parameters carried through every per-bin operation
 * as an automatic forward-mode differentiation computes them (the paper
 * differentiates automatically, Sec. 5 "JAX implementation").  Same
 * arguments, layouts and results as smcgw_loglike_grad (grad NULL: the value
 * only, the tangents are still carried).  Events added with
 * smcgw_add_event only (SMCGW_ERR_INVALID when a relative-binning event is
 * present). */
int smcgw_loglike_grad_tangent(smcgw_ctx *ctx, int P, const int32_t *event_of_particle, const double *theta,
                               double *logl, double *grad);

/* logL and its gradient of the context's current target (smcgw_set_target):
 * the event likelihood (as smcgw_loglike_grad with event_of_particle taken
 * from smcgw_set_event_map) or an analytic test likelihood.  theta [P][dim],
 * logl [P], grad [P][dim] are device arrays. */
int smcgw_target_loglike_grad(smcgw_ctx *ctx, int P, const double *theta, double *logl, double *grad,
                              int precision);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * likelihood and gradient of smcgw_loglike_grad, same arguments and results,
 * with its per-particle scratch (the 832 B coefficient block of each
 * particle) in a fixed device array of SMCGW_NOALLOC_MAX_P particles (13 MiB)
 * that each GPU holds from the first context on it until the process ends.
 * It calls no allocation, creates no event and does not synchronise.
 * SMCGW_ERR_SHAPE for P > SMCGW_NOALLOC_MAX_P.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race and must be serialised by the caller. */
#define SMCGW_NOALLOC_MAX_P 16384
int smcgw_loglike_grad_noalloc(smcgw_ctx *ctx, int P, const int32_t *event_of_particle, const double *theta,
                               double *logl, double *grad, int precision);

/* Projected detector strain h_d(f_j; theta) of event event_id for one point
 * of the 11 source parameters (theta11, host), written to the device array
 * h_reim [n_det][N][2].  Used to build injections. */
int smcgw_waveform(smcgw_ctx *ctx, int event_id, const double *theta11, double *h_reim);

/* Mass matrix from the particle population (Sec. 5, "Exploitation of local
 * geometry", read as the population covariance): inv_mass = cov(theta) with
 * the diagonal scaled by (1 + shrink), chol its lower Cholesky factor
 * (M^{-1} = chol chol^T).  theta [P][D], inv_mass [D][D], chol [D][D] are
 * device arrays.  status_device (device int32, may be NULL) receives 1 when
 * the covariance was not positive definite and a diagonal was used, else 0;
 * with it the call is asynchronous and returns SMCGW_OK.  Without it the
 * call synchronises and returns SMCGW_WARN_FALLBACK in that case. */
int smcgw_mass_matrix(smcgw_ctx *ctx, int P, int D, const double *theta, double shrink, double *inv_mass,
                      double *chol, int32_t *status_device);

/* Per-particle local metric (Sec. 5, "Exploitation of local geometry": at
 * the start of each SMC iteration every particle's mass matrix is set to the
 * Hessian of the tempered posterior at the particle and held fixed during
 * the mutation).  Read as the Gauss-Newton Hessian
 *   M_i = beta F(theta_i) + diag(prior precision),
 * F the Fisher matrix <dh/dtheta_k | dh/dtheta_l> of the event likelihood
 * (Sec. 2, Eq. 2) over the sampled coordinates (for an analytic test
 * likelihood, the exact Hessian of -log L), the prior precision
 * 12/(hi-lo)^2 (uniform), the inverse variance (log-uniform), 1/sigma^2
 * (Gaussian) or 0 (flat).  chol [P][D][D] receives the lower Cholesky
 * factor of M_i^{-1} (the layout smcgw_nuts_step takes with
 * chol_per_particle = 1); fisher [P][D][D] (may be NULL) receives F.  A
 * particle whose M_i or M_i^{-1} is not numerically positive definite gets
 * fallback_chol [D][D] (NULL: the identity) and status [P] = 1 (status may
 * be NULL; 0 otherwise).  All arrays are device arrays; beta in [0, 1], or
 * read from the device double beta_device when that is not NULL.
 * Needs a prior of dimension D and the GW target with a parameter map of
 * dimension D, or an analytic target of dimension D.  Asynchronous on the
 * context's stream. */
int smcgw_local_metric(smcgw_ctx *ctx, int P, int D, const double *theta, double beta, const double *beta_device,
                       const double *fallback_chol, double *chol, double *fisher, int32_t *status);

/* One No-U-Turn transition per particle (Sec. 4: momentum r ~ N(0, M),
 * Hamiltonian H = -log p_t + r^T M^{-1} r / 2, leapfrog Eqs. 11-13,
 * reflective / periodic boundaries of Sec. 5, a reflecting wall taken as the
 * specular reflection of the drift in the metric, which flips the crossing
 * coordinate's velocity and conserves the kinetic energy; multinomial
 * trajectory sampling with the generalised U-turn criterion).  theta [P][D], logl [P]
 * and grad [P][D] (device) hold the current point, its likelihood and the
 * likelihood gradient on entry and the selected point on exit.  chol [D][D]
 * (device) is the Cholesky factor of M^{-1}, or chol [P][D][D] one factor
 * per particle when params->chol_per_particle = 1.  max_depth_per_particle [P]
 * (device, NULL = params->max_depth) caps each tree.  work_hint [P]
 * (device) is a predicted leapfrog count per particle, for callers that know
 * it (e.g. forced depths): particles start in descending order of
 * floor(log2(hint)) so that the longest trees do not start last.  Without it
 * (NULL) the particles are dealt to the GPU's XCDs in stripes of 16
 * neighbouring indices, each XCD's slots taking their own stripes first and
 * the others' after, so that neighbouring particles, whose inputs and
 * outputs share cache lines, pass through one L2.  The hint changes only
 * the schedule; every output is the same with or without it.  Per-particle diagnostics (device, each may be NULL): doublings
 * done, leapfrog steps, divergence flag, mean acceptance statistic. */
int smcgw_nuts_step(smcgw_ctx *ctx, int P, int D, double *theta, double *logl, double *grad, const double *chol,
                    const smcgw_nuts_params *params, const int32_t *max_depth_per_particle,
                    const int32_t *work_hint, int precision, int32_t *depth, int32_t *n_leapfrog,
                    uint8_t *divergent, double *accept_stat);

/* The plain comparison form of smcgw_nuts_step: the same transition (tree,
 * random streams, decisions, outputs) advanced in lockstep sweeps, one
 * leapfrog step of every unfinished particle per sweep, with the likelihood
 * and gradient of smcgw_loglike_grad_tangent (FP64, forward-mode tangents).
 * A sweep is one launch of the tree step (one wavefront per particle) and
 * one batched likelihood launch over the particles still building their tree;
 * the tree states wait in device memory between sweeps.  Sweeps run in
 * groups of sweeps_per_group (1..64) captured once in a HIP graph (kept by the
 * context while the arguments stay the same) and replayed; after each group
 * the host reads the number of unfinished particles, so the call
 * synchronises, and it returns when that number is zero.  *n_sweeps_host
 * (may be NULL) receives the sweeps run.  Arguments as smcgw_nuts_step
 * (state_device / run_size included, no work hint); the GW target on events
 * added with smcgw_add_event only. */
int smcgw_nuts_step_sweeps(smcgw_ctx *ctx, int P, int D, double *theta, double *logl, double *grad,
                           const double *chol, const smcgw_nuts_params *params,
                           const int32_t *max_depth_per_particle, int32_t *depth, int32_t *n_leapfrog,
                           uint8_t *divergent, double *accept_stat, int sweeps_per_group, int *n_sweeps_host);

/* Reweighting, adaptive temperature and multinomial resampling of one SMC
 * iteration (Sec. 3, Eqs. 4-6): beta_next solves ESS(beta) = alpha P by
 * bisection on [beta_prev, 1] (beta_next = 1 when ESS(1) >= alpha P); the
 * evidence increment log(Z_t/Z_{t-1}) = log mean_i L_i^(beta_next-beta_prev)
 * (Sec. 3.1, Eq. 7) is accumulated in FP64.  Ancestors are drawn with
 * Philox uniforms keyed by (seed, iteration) and theta [P][D], logl [P],
 * grad [P][D] and carry [P] (device; grad and carry may be NULL) are gathered
 * in place; carry is any per-particle int32 payload that travels with the
 * particles (e.g. the last transition's leapfrog counts, as a work hint).
 * ancestors [P] (device) receives the indices.  Synchronises:
 * *beta_next_host and *dlogz_host are host scalars.  beta_prev = 1 is
 * allowed (beta_next = 1, a resample-only reweighting).  Returns
 * SMCGW_ERR_STALL when beta cannot advance. */
int smcgw_smc_reweight_resample(smcgw_ctx *ctx, int P, int D, double beta_prev, double alpha, uint64_t seed,
                                uint64_t iteration, double *theta, double *logl, double *grad, int32_t *carry,
                                int32_t *ancestors, double *beta_next_host, double *dlogz_host);

/* The same reweighting, temperature search and resampling without a host
 * synchronisation: out_device [2] (device) receives beta_next and the
 * evidence increment log(Z_t/Z_{t-1}).  The caller reads them back when it
 * needs them (e.g. through an event) and can queue the mass matrix and the
 * NUTS transition first, passing out_device as their beta_device, so the
 * device does not wait for the host between the steps of an iteration.
 * beta_next equal to beta_prev < 1 means the temperature could not advance
 * (the synchronous call's SMCGW_ERR_STALL). */
int smcgw_smc_reweight_resample_async(smcgw_ctx *ctx, int P, int D, double beta_prev, double alpha, uint64_t seed,
                                      uint64_t iteration, double *theta, double *logl, double *grad, int32_t *carry,
                                      int32_t *ancestors, double *out_device);

/* One whole SMC iteration of every run in desc, queued on the context's
 * stream without a host synchronisation (Sec. 3, Eqs. 3-8; Sec. 4; Sec. 5):
 *   1. per run: reweighting from beta_{t-1} = state[BETA] to beta_t by the
 *      bisection of smcgw_smc_reweight_resample, the evidence increment and
 *      the running log Z accumulated in FP64 in the state, multinomial
 *      resampling with the uniforms of iteration t = state[NEXT] (key
 *      seed + r) and the gather of theta, logl and grad;
 *   2. per run: the population covariance, its shrinkage and factor;
 *   3. with chol_pp: every particle's local metric at its run's beta_t, the
 *      run's population factor standing in where it is not positive definite;
 *   4. one persistent NUTS launch over all n_runs P particles at their runs'
 *      temperatures (iteration t, key seed + r), without a work hint (a
 *      particle's tree length hardly depends on its ancestor's);
 *   5. per run: the record row t (history).
 * A run whose state says done is left untouched, so the call may be queued
 * past the end of every run; the host reads state[DONE] when it needs to
 * know (e.g. through an event).  Allocates its scratch on the first call for
 * a shape (so a graph of it, smcgw_smc_graph_create, captures no
 * allocation).  Runs are independent: run r's results are bitwise those of
 * a one-run call with seed + r on its particles. */
int smcgw_smc_iteration(smcgw_ctx *ctx, const smcgw_smc_iter_desc *desc);

/* A HIP graph of smcgw_smc_iteration(ctx, desc), captured once on a private
 * stream (every pointer in desc is baked in) and replayed on the context's
 * stream.  Replays read the temperature, iteration index and done flag from
 * the device state, so one graph serves every iteration of the runs; replays
 * after every run is done change nothing.  *graph receives the handle. */
typedef struct smcgw_graph smcgw_graph;
int smcgw_smc_graph_create(smcgw_ctx *ctx, const smcgw_smc_iter_desc *desc, smcgw_graph **graph);
/* Replays the graph `count` times on the context's current stream (asynchronous). */
int smcgw_graph_launch(smcgw_graph *graph, int count);
int smcgw_graph_destroy(smcgw_graph *graph);

/* Persistent sampling (Karamanis & Seljak 2024, arXiv:2407.20722; the SMC
 * variant the paper names as future work, Sec. 7): every earlier population
 * stays in a pool.  The pool holds T populations of N points, population s
 * drawn from p_s = L^beta_s pi / Z_s (s = 0: the prior sample, beta_0 = 0,
 * log Z_0 = 0), and is read as draws of the mixture (1/T) sum_s p_s.  The
 * next temperature's weights over the pool are
 *   w_i(beta) = L_i^beta / ((1/T) sum_s L_i^beta_s / Z_s)
 * (the prior cancels); beta_next solves ESS(beta) = alpha N by the bisection
 * of smcgw_smc_reweight_resample over [beta_{T-1}, 1] (beta_next = 1 when
 * ESS(1) >= alpha N), the evidence is the pool mean of the weights,
 *   log Z(beta_next) = log((1 / (T N)) sum_i w_i(beta_next)),
 * and N ancestors are drawn from the pool with the Philox uniforms of
 * smcgw_smc_reweight_resample; theta [N][D], logl [N] and grad [N][D]
 * (device) receive the drawn points.  theta_pool [T*N][D], logl_pool [T*N]
 * and grad_pool [T*N][D] (device; grad_pool and grad both NULL or both set)
 * hold the pool, population s at rows s N .. s N + N - 1; betas_host [T] and
 * logz_host [T] (host) its temperatures and log evidences.  NaN or -inf
 * log L: weight zero.  ancestors [N] (device) receives pool indices.
 * Synchronises: *beta_next_host and *logz_next_host (log Z at beta_next,
 * not an increment) are host scalars.  Returns SMCGW_ERR_STALL when beta
 * cannot advance. */
int smcgw_ps_reweight_resample(smcgw_ctx *ctx, int T, int N, int D, const double *theta_pool,
                               const double *logl_pool, const double *grad_pool, const double *betas_host,
                               const double *logz_host, double alpha, uint64_t seed, uint64_t iteration,
                               double *theta, double *logl, double *grad, int32_t *ancestors, double *beta_next_host,
                               double *logz_next_host);

/* Sample recycling (Sec. 5, "Samples recycling"): the populations left by
 * the mutations of iterations t = 1..T are pooled and read as draws of the
 * mixture (1/T) sum_t p_t, with p_t = L^beta_t pi / Z_t normalised by the
 * evidence reached at iteration t.  Each pooled point gets the weight of the
 * final target against the mixture,
 *   log w = log L - log Z_T - log((1/T) sum_t L^beta_t / Z_t)
 * (NaN or -inf log L: weight zero), and rejection sampling keeps point i when
 * its Philox uniform (seed; index 0, particle i, iteration 0) is below
 * w_i / max w, giving i.i.d. draws of p_T.  logl [T][N] (device) holds the
 * log-likelihoods of the pooled points (pool index i = t N + n);
 * betas_host [T] and logz_host [T] (host) the temperatures and running log
 * evidence of the iterations.  logw [T*N] (device) receives the log weights,
 * kept [T*N] (device) the kept pool indices in increasing order, of which
 * there are *n_kept_host; *ess_host receives (sum w)^2 / sum w^2.
 * T*N must not exceed 2^31 - 1.  Synchronises. */
int smcgw_recycle(smcgw_ctx *ctx, int T, int N, const double *logl, const double *betas_host,
                  const double *logz_host, uint64_t seed, double *logw, int32_t *kept, int64_t *n_kept_host,
                  double *ess_host);

/* ------------------------------------------------------------ options
 * Launch-shape options of a context (chosen by the autotuner or by hand).
 *   SMCGW_OPT_NUTS_WAVES: wavefronts that share one particle's bin loop in the
 *     persistent NUTS kernel (2, 4, 6 or 8; 0 = the library default: 2 when
 *     no event of the context has more than 1024 padded bins, as with
 *     relative-binning events, else 4).
 *   SMCGW_OPT_NUTS_PRIORITY: 1 (default) raises the issue priority of a
 *     slot's wavefronts as its tree deepens, so the longest trajectories of
 *     a transition run ahead of the short ones that share their compute
 *     unit; 0 keeps every wavefront at the same priority.  Scheduling only:
 *     the outputs do not depend on it.
 *   SMCGW_OPT_NUTS_SLOTS_PER_CU: at most this many NUTS workgroups (slots)
 *     per compute unit in one launch (0, the default: as many as fit; values
 *     above what fits are clamped).  A caller that runs independent batches
 *     on several streams can give each launch a share of every compute unit,
 *     so that one launch's tail overlaps another's work.  Scheduling only:
 *     the outputs do not depend on it.  Accepts 0..64. */
enum { SMCGW_OPT_NUTS_WAVES = 0, SMCGW_OPT_NUTS_PRIORITY = 1, SMCGW_OPT_NUTS_SLOTS_PER_CU = 2 };
int smcgw_set_option(smcgw_ctx *ctx, int option, int64_t value);

/* Autotuner of the NUTS slot width: runs `trials` transitions of the given
 * batch (same arguments as smcgw_nuts_step, without diagnostics) for every
 * width 2, 4, 6 and 8 on device copies of theta / logl / grad, times each
 * launch with HIP events, and keeps the width with the shortest median time
 * (SMCGW_OPT_NUTS_WAVES).  The caller's arrays are not modified.  The width
 * changes the rounding order of the bin sums (not the method), so outputs
 * after tuning equal those of a run with that width set by hand.
 * Synchronises; *best_waves and times_ms[4] (host, may be NULL) receive the
 * choice and the median time of each width. */
int smcgw_autotune_nuts(smcgw_ctx *ctx, int P, int D, const double *theta, const double *logl, const double *grad,
                        const double *chol, const smcgw_nuts_params *params, int precision, int trials,
                        int *best_waves, double *times_ms);

/* ------------------------------------------------------------ timing
 * Kernel timing for measurement: HIP events are recorded on the context's
 * stream around every launch of the kernel classes whose bit is set in
 * class_mask (bit c = class c; 0 turns timing off).
 * smcgw_timing_read synchronises, returns the summed duration [ms] and the
 * launch count of one class since the last read, and resets that class.
 * The batched likelihood's epilogue runs inside its bin-loop kernel (class
 * BINS); class FINISH is kept for compatibility and records no launch. */
enum { SMCGW_KERNEL_BINS = 0, SMCGW_KERNEL_PREP = 1, SMCGW_KERNEL_FINISH = 2, SMCGW_KERNEL_NUTS = 3,
       SMCGW_KERNEL_SMC = 4, SMCGW_KERNEL_METRIC = 5, SMCGW_KERNEL_CLASSES = 6 };
int smcgw_timing_enable(smcgw_ctx *ctx, int class_mask);
int smcgw_timing_read(smcgw_ctx *ctx, int kernel_class, double *total_ms, int64_t *launches);
/* The same records one launch at a time, against a reference: ref_event is a
 * hipEvent_t (created with timing enabled, on this context's device) that the
 * caller has recorded before the launches; start_ms[k] / end_ms[k] (host,
 * cap entries each) receive launch k's start and end in ms after it.
 * Contexts that run on several streams of one device can share the reference
 * to find when their launches overlap.  Synchronises the context's stream and
 * the reference, consumes the class's records as smcgw_timing_read does and
 * sets *launches to their number; if that exceeds cap only the first cap are
 * written and SMCGW_ERR_SHAPE is returned. */
int smcgw_timing_intervals(smcgw_ctx *ctx, int kernel_class, void *ref_event, double *start_ms, double *end_ms,
                           int64_t cap, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* SMCGW_H */
