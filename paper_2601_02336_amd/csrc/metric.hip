// Per-particle local metric (arXiv:2601.02336, Sec. 5, "Exploitation of
// local geometry"): at the start of an SMC iteration every particle gets its
// own mass matrix, the Hessian of the tempered posterior's negative log
// density at the particle, held fixed during the mutation.  Read here as the
// Gauss-Newton form
//   M = beta F + diag(prior precision),
//   F_kl = <dh/dtheta_k | dh/dtheta_l> = sum_d sum_j w_dj Re(conj(dh_dj/dk) dh_dj/dl),
// which is positive semi-definite by construction and equals the expected
// Hessian of -log L.
//
// No bin loop per particle: with h_dj = P'_d a_j e^{-2 pi i Phi_dj},
// a_j = f_j^-7/6 / u_scale and Phi_dj = sum_a gamma_a g_a(f_j) a combination
// of the phase functions g (constant, the basis rows, f),
//   dh_dj/dk = a_j e^{-2 pi i Phi_dj} (D_dk - 2 pi i P'_d dPhi_dj/dk),
//   D_dk = dP'_d/dk,
// so
//   F_kl = sum_d [ W_d00 Re(conj D_dk D_dl)
//                + 2 pi (s_dk (W_d g_l)_0 + s_dl (W_d g_k)_0)
//                + 4 pi^2 |P'_d|^2 g_kd^T W_d g_ld ],
//   s_dk = Im(conj(D_dk) P'_d),  g_kd[a] = dgamma_a/dtheta_k (detector d),
// with W_d the per-event moments sum_j w_dj a_j^2 g_a(f_j) g_b(f_j) built once
// with the bin tables.  Then, per particle, the lower Cholesky factor of
// M^{-1} that the NUTS kernel takes.
#include "coeffs.h"
#include "common.h"
#include "context.h"

namespace smcgw {

constexpr int MET_THREADS = 128;   // two wavefronts per particle
constexpr int NPAIR = NPAR * (NPAR + 1) / 2;
static_assert(NPAIR <= MET_THREADS && NPAR * NGEO <= MET_THREADS, "one thread per pair and per Jacobian entry");

struct PrecDesc {
    double prec[MAXDIM];   // prior precision of each sampled coordinate
};

struct MetricShared {
    double cb[CB_SIZE];
    double W[MAXDET * NGEO * NGEO];
    double gam[NPAR][NGEO];   // d gamma_a / d theta_k for the current detector
    double wg[NPAR][NGEO];    // W_d gamma_k
    double dr[NPAR], di[NPAR], s[NPAR];
    double F[NPAR * NPAR];
    double M[MAXDIM * MAXDIM], R[MAXDIM * MAXDIM], Y[MAXDIM * MAXDIM];
    ExtAngles ang;
};

// Phase derivative of source parameter k on phase function a (cycles),
// detector d.  The phase is c_0 + sum_b c_{1+b} B_b(f) + f tau_d with
// c_0 containing -phi_c / (2 pi) and tau_d = t_c + delay_d(ra, dec).
__device__ __forceinline__ double phase_jac(const double* cb, int d, int k, int a) {
    if (k < 4) return a < NCOEF ? cb[CB_DC + 4 * a + k] : 0.0;
    if (a == 0) return k == P_PHIC ? -1.0 / TWO_PI : 0.0;
    if (a != NGEO - 1) return 0.0;
    return k == P_TC ? 1.0 : k == P_RA ? cb[CB_DTAU + 2 * d] : k == P_DEC ? cb[CB_DTAU + 2 * d + 1] : 0.0;
}

// Pair index e of the upper triangle (k <= l), row by row.
__device__ __forceinline__ void pair_of(int e, int& k, int& l) {
    k = 0;
    while (e >= NPAR - k) { e -= NPAR - k; ++k; }
    l = k + e;
}

// Lower Cholesky factor Lo of the D x D matrix A (row stride MAXDIM), one
// row per thread; false (uniform over the workgroup) when a pivot is not
// positive.  Each entry is formed in the textbook order: the matrix entry
// minus the products of the finished columns, k ascending.
__device__ bool block_cholesky(const double* A, double* Lo, int D, int tid) {
    for (int i = tid; i < MAXDIM * MAXDIM; i += MET_THREADS) Lo[i] = 0.0;
    __syncthreads();
    for (int j = 0; j < D; ++j) {
        double sjj = A[j * MAXDIM + j];
        for (int k = 0; k < j; ++k) sjj -= Lo[j * MAXDIM + k] * Lo[j * MAXDIM + k];
        if (!(sjj > 0.0)) return false;
        const double ljj = sqrt(sjj);
        if (tid > j && tid < D) {
            double t = A[tid * MAXDIM + j];
            for (int k = 0; k < j; ++k) t -= Lo[tid * MAXDIM + k] * Lo[j * MAXDIM + k];
            Lo[tid * MAXDIM + j] = t / ljj;
        }
        if (tid == j) Lo[j * MAXDIM + j] = ljj;
        __syncthreads();
    }
    return true;
}

// M = beta F + diag(prior precision) over the sampled coordinates (F with
// row stride fs, coordinate a of the sample being row idx[a]), then the lower
// Cholesky factor of M^{-1} into chol[p], or the fallback where M or the
// factor is not numerically positive definite.  The factor comes from the
// order-reversed matrix: with J the reversal permutation and J M J = R R^T,
// M^{-1} = (J R^-T J)(J R^-T J)^T and J R^-T J is lower triangular with a
// positive diagonal, so it is that factor; it needs one Cholesky and one
// triangular inverse.
__device__ void finish_metric(MetricShared& S, const double* F, int fs, const int* idx, int D, double beta,
                              const PrecDesc& pd,
                              const double* __restrict__ fallback, double* __restrict__ chol,
                              double* __restrict__ fisher, int32_t* __restrict__ status, int p, int tid) {
    // J M J (rows and columns in reverse order)
    for (int i = tid; i < MAXDIM * MAXDIM; i += MET_THREADS) {
        const int a = i / MAXDIM, b = i % MAXDIM;
        double v = 0.0;
        if (a < D && b < D) {
            const int ra = D - 1 - a, rb = D - 1 - b;
            const double f = F[idx[ra] * fs + idx[rb]];
            v = beta * f + (a == b ? pd.prec[ra] : 0.0);
            if (fisher) fisher[(size_t)p * D * D + ra * D + rb] = f;
        }
        S.M[i] = v;
    }
    __syncthreads();
    bool ok = block_cholesky(S.M, S.R, D, tid);
    if (ok) {
        // X = R^{-1}, thread c solving column c by forward substitution
        if (tid < D) {
            const int c = tid;
            for (int r = 0; r < D; ++r) {
                double v = (r == c) ? 1.0 : 0.0;
                for (int k = c; k < r; ++k) v -= S.R[r * MAXDIM + k] * S.Y[k * MAXDIM + c];
                S.Y[r * MAXDIM + c] = r < c ? 0.0 : v / S.R[r * MAXDIM + r];
            }
        }
        __syncthreads();
    }
    // factor L[i][j] = X[D-1-j][D-1-i]; a non-finite entry takes the fallback too
    bool bad_entry = false;
    if (ok)
        for (int i = tid; i < D * D; i += MET_THREADS) {
            const double v = S.Y[(D - 1 - i % D) * MAXDIM + (D - 1 - i / D)];
            bad_entry |= !isfinite(v);
        }
    ok = ok && !__syncthreads_or(bad_entry);
    for (int i = tid; i < D * D; i += MET_THREADS) {
        const int a = i / D, b = i % D;
        chol[(size_t)p * D * D + i] = ok ? S.Y[(D - 1 - b) * MAXDIM + (D - 1 - a)]
                                    : fallback ? fallback[i] : (a == b ? 1.0 : 0.0);
    }
    if (status && tid == 0) status[p] = ok ? 0 : 1;
}

// One workgroup of two wavefronts per particle.  The coefficient block is
// built as in the NUTS leaf: the intrinsic part with one tangent per lane on
// wavefront 0, the extrinsic part (shared sin / cos in parallel lanes, then
// one detector and tangent per lane) on wavefront 1.
__global__ __launch_bounds__(MET_THREADS) void local_metric_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                                  const int32_t* __restrict__ ev_of_p, ParamMap pm,
                                                                  PrecDesc pd, int P, const double* __restrict__ theta,
                                                                  double beta_host, const double* __restrict__ beta_dev,
                                                                  const double* __restrict__ fallback,
                                                                  double* __restrict__ chol, double* __restrict__ fisher,
                                                                  int32_t* __restrict__ status,
                                                                  const double* __restrict__ st, int run_size) {
    __shared__ MetricShared S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int p = blockIdx.x;
    const int D = pm.dim;
    // independent runs: particle p belongs to run p / run_size, whose state gives beta; a finished run is skipped
    const int run = st ? p / run_size : 0;
    if (st && st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_DONE] != 0.0) return;
    if (st && fallback) fallback += (size_t)run * D * D;
    const DevEvent& ev = evs[event_index(ev_of_p, p, n_events)];
    const int n_det = ev.n_det;

    for (int i = tid; i < n_det * NGEO * NGEO; i += MET_THREADS) S.W[i] = ev.wmom[i];
    if (wave == 0 && lane < 4) {
        double th[NPAR];
        expand_params(pm, theta + (size_t)p * D, th);
        prep_intrinsic_n<1>(ev, th, S.cb, lane, lane == 0);
    } else if (wave == 1) {
        double th[NPAR];
        if (lane <= 2 * MAXDET) expand_params(pm, theta + (size_t)p * D, th);
        if (lane < ANG_COUNT) {
            double sn, cs;
            sincos(extrinsic_angle(ev, th, lane), &sn, &cs);
            S.ang.sc[lane][0] = sn;
            S.ang.sc[lane][1] = cs;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane < 2 * MAXDET) {
            const ExtAngles ang = S.ang;
            const int k = lane / MAXDET;
            prep_extrinsic_det_n<1>(ev, th, ang, S.cb, lane - k * MAXDET, k, k == 0);
        } else if (lane == 2 * MAXDET) {
            prep_extrinsic_common(ev, th, S.cb);
        }
    }
    __syncthreads();
    const double amp = S.cb[CB_AMP];

    double acc = 0.0;   // F entry of pair tid (k <= l)
    for (int d = 0; d < n_det; ++d) {
        const double* W = S.W + d * NGEO * NGEO;
        const double qr = amp * S.cb[CB_PR + d], qi = amp * S.cb[CB_PI + d];
        if (tid < NPAR * NGEO) S.gam[tid / NGEO][tid % NGEO] = phase_jac(S.cb, d, tid / NGEO, tid % NGEO);
        if (tid < NPAR) {
            double xr = 0.0, xi = 0.0;
            if (tid == P_MC || tid == P_DL) {
                const double g = tid == P_MC ? S.cb[CB_DLNCA_MC] : S.cb[CB_DLNCA_DL];
                xr = g * qr;
                xi = g * qi;
            } else if (tid == P_IOTA || tid == P_PSI || tid == P_RA || tid == P_DEC) {
                const int m = tid == P_IOTA ? 0 : tid == P_PSI ? 1 : tid == P_RA ? 2 : 3;
                xr = amp * S.cb[CB_DPR + 4 * d + m];
                xi = amp * S.cb[CB_DPI + 4 * d + m];
            }
            S.dr[tid] = xr;
            S.di[tid] = xi;
            S.s[tid] = xr * qi - xi * qr;
        }
        __syncthreads();
        if (tid < NPAR * NGEO) {
            const int k = tid / NGEO, a = tid % NGEO;
            double v = 0.0;
            for (int b = 0; b < NGEO; ++b) v = fma(W[a * NGEO + b], S.gam[k][b], v);
            S.wg[k][a] = v;
        }
        __syncthreads();
        if (tid < NPAIR) {
            int k, l;
            pair_of(tid, k, l);
            double gwg = 0.0;
            for (int a = 0; a < NGEO; ++a) gwg = fma(S.gam[k][a], S.wg[l][a], gwg);
            acc += W[0] * (S.dr[k] * S.dr[l] + S.di[k] * S.di[l])
                 + TWO_PI * (S.s[k] * S.wg[l][0] + S.s[l] * S.wg[k][0])
                 + (4.0 * PI * PI) * (qr * qr + qi * qi) * gwg;
        }
        __syncthreads();
    }
    if (tid < NPAIR) {
        int k, l;
        pair_of(tid, k, l);
        S.F[k * NPAR + l] = acc;
        S.F[l * NPAR + k] = acc;
    }
    __syncthreads();

    const double beta = st ? st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_BETA] : beta_dev ? *beta_dev : beta_host;
    finish_metric(S, S.F, NPAR, pm.idx, D, beta, pd, fallback, chol, fisher, status, p, tid);
}

// The analytic test likelihoods take the exact Hessian of -log L as F: the
// identity (standard normal), diag(1 / sigma_l^2) (Gaussian likelihood), and
// for the unweighted sum of two isotropic Gaussians N(m1, s^2) + N(m2, s^2)
//   F = I / s^2 - r1 r2 (m1 - m2)(m1 - m2)^T / s^4,
// r_i the components' shares at the particle (the shares' mean of the
// components' Hessians less the shares' covariance of their gradients).
// Near a mode F is positive definite; across the saddle between the modes it
// is not, and the particle takes the fallback.  One workgroup per particle.
__global__ __launch_bounds__(MET_THREADS) void analytic_metric_kernel(TargetDesc tg, PrecDesc pd, int P,
                                                                     const double* __restrict__ theta,
                                                                     double beta_host, const double* __restrict__ beta_dev,
                                                                     const double* __restrict__ fallback,
                                                                     double* __restrict__ chol, double* __restrict__ fisher,
                                                                     int32_t* __restrict__ status,
                                                                     const double* __restrict__ st, int run_size) {
    __shared__ MetricShared S;
    __shared__ double F[MAXDIM * MAXDIM];
    __shared__ int idx[MAXDIM];
    const int tid = threadIdx.x;
    const int p = blockIdx.x;
    const int D = tg.dim;
    const int run = st ? p / run_size : 0;
    if (st && st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_DONE] != 0.0) return;
    if (st && fallback) fallback += (size_t)run * D * D;
    if (tid < MAXDIM) idx[tid] = tid;
    for (int e = tid; e < D * D; e += MET_THREADS) {
        const int k = e / D, l = e % D;
        double f = 0.0;
        if (tg.kind == SMCGW_TARGET_GAUSS) {
            f = k == l ? 1.0 : 0.0;
        } else if (tg.kind == SMCGW_TARGET_GAUSS_X_GAUSS) {
            const double sl = tg.params[D + k];
            f = k == l ? 1.0 / (sl * sl) : 0.0;
        } else {
            const double* x = theta + (size_t)p * D;
            const double* m1 = tg.params;
            const double* m2 = tg.params + D;
            const double sg = tg.params[2 * D], s2g = sg * sg;
            double s1 = 0.0, s2 = 0.0;
            for (int j = 0; j < D; ++j) {
                s1 += (x[j] - m1[j]) * (x[j] - m1[j]);
                s2 += (x[j] - m2[j]) * (x[j] - m2[j]);
            }
            const double r1 = 1.0 / (1.0 + exp(-0.5 * (s2 - s1) / s2g)), r2 = 1.0 - r1;
            f = (k == l ? 1.0 / s2g : 0.0) - r1 * r2 * (m1[k] - m2[k]) * (m1[l] - m2[l]) / (s2g * s2g);
        }
        F[k * MAXDIM + l] = f;
    }
    __syncthreads();
    const double beta = st ? st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_BETA] : beta_dev ? *beta_dev : beta_host;
    finish_metric(S, F, MAXDIM, idx, D, beta, pd, fallback, chol, fisher, status, p, tid);
}

// Prior precision of each sampled coordinate: 12 / (hi - lo)^2 (uniform),
// the inverse variance of the log-uniform density, 1 / sigma^2 (Gaussian),
// 0 (flat).
static PrecDesc prior_precision(const PriorDesc& pr) {
    PrecDesc pd;
    for (int k = 0; k < MAXDIM; ++k) {
        double v = 0.0;
        if (k < pr.dim) {
            const double lo = pr.lo[k], hi = pr.hi[k];
            if (pr.kind[k] == SMCGW_PRIOR_UNIFORM) {
                v = 12.0 / ((hi - lo) * (hi - lo));
            } else if (pr.kind[k] == SMCGW_PRIOR_LOGUNIFORM) {
                const double lr = std::log(hi / lo);
                const double m1 = (hi - lo) / lr, m2 = (hi * hi - lo * lo) / (2.0 * lr);
                v = 1.0 / (m2 - m1 * m1);
            } else if (pr.kind[k] == SMCGW_PRIOR_GAUSSIAN) {
                v = 1.0 / (hi * hi);
            }
        }
        pd.prec[k] = v;
    }
    return pd;
}

}  // namespace smcgw

namespace smcgw {
// Local metric of n_runs * run_size particles at their runs' temperatures
// (state st), the run's own population factor as the fallback.
static int metric_target_ok(smcgw_ctx* c, int D) {
    if (!c->prior_set) return SMCGW_ERR_NOT_INIT;
    if (c->target.kind == SMCGW_TARGET_GW) {
        if (c->events.empty()) return SMCGW_ERR_NOT_INIT;
        return c->prior.dim == D && c->pmap.dim == D ? SMCGW_OK : SMCGW_ERR_INVALID;
    }
    if (c->target.dim <= 0) return SMCGW_ERR_NOT_INIT;
    return c->prior.dim == D && c->target.dim == D ? SMCGW_OK : SMCGW_ERR_INVALID;
}

static int launch_metric(smcgw_ctx* c, int P, const double* theta, double beta, const double* beta_dev,
                         const double* fallback, double* chol, double* fisher, int32_t* status, const double* st,
                         int run_size) {
    const PrecDesc pd = prior_precision(c->prior);
    TimedLaunch tl(c, SMCGW_KERNEL_METRIC);
    if (c->target.kind == SMCGW_TARGET_GW)
        hipLaunchKernelGGL(local_metric_kernel, dim3(P), dim3(MET_THREADS), 0, c->stream, c->d_events,
                           (int)c->events.size(), c->ev_of_p, c->pmap, pd, P, theta, beta, beta_dev, fallback, chol,
                           fisher, status, st, run_size);
    else
        hipLaunchKernelGGL(analytic_metric_kernel, dim3(P), dim3(MET_THREADS), 0, c->stream, c->target, pd, P, theta,
                           beta, beta_dev, fallback, chol, fisher, status, st, run_size);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

int queue_local_metric(smcgw_ctx* c, int P, int D, const double* theta, const double* st, int run_size,
                       const double* fallback_runs, double* chol, int32_t* status) {
    const int rc = metric_target_ok(c, D);
    if (rc) return rc;
    return launch_metric(c, P, theta, 0.0, nullptr, fallback_runs, chol, nullptr, status, st, run_size);
}
}  // namespace smcgw

using namespace smcgw;

extern "C" int smcgw_local_metric(smcgw_ctx* c, int P, int D, const double* theta, double beta,
                                  const double* beta_device, const double* fallback_chol, double* chol, double* fisher,
                                  int32_t* status) {
    if (!c || P < 0 || D <= 0 || D > MAXDIM || (!beta_device && !(beta >= 0.0 && beta <= 1.0)) ||
        (P > 0 && (!theta || !chol)))
        return SMCGW_ERR_INVALID;
    const int rc = metric_target_ok(c, D);
    if (rc) return rc;
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    return launch_metric(c, P, theta, beta, beta_device, fallback_chol, chol, fisher, status, nullptr, P);
}
