// SMC kernels: adaptive tempering, evidence increment, multinomial
// resampling with gather (arXiv:2601.02336, Sec. 3, Eqs. 4-8) and the
// population mass matrix (Sec. 5, covariance reading of the metric).
//
// All reductions run inside one workgroup in a fixed order (no atomics), in
// FP64, so beta, the evidence increment and the ancestors are reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "context.h"
#include "philox.h"

using namespace smcgw;

namespace smcgw {

constexpr int SMC_THREADS = 1024;

// Fixed-order workgroup sum of one double per thread (result valid in all threads).
__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// log-likelihood with NaN mapped to -inf (zero weight)
__device__ __forceinline__ double ll_at(const double* logl, int i) {
    const double v = logl[i];
    return v == v ? v : -INFINITY;
}

// ESS of w_i = exp(db (logL_i - lmax)): (sum w)^2 / sum w^2.
__device__ double ess_at(const double* logl, int P, double db, double lmax, double* sh) {
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const double w = exp(db * (ll_at(logl, i) - lmax));
        s1 += w;
        s2 += w * w;
    }
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    return s1 * s1 / s2;
}

// One workgroup: beta_next by bisection, evidence increment, normalised
// weights and their inclusive prefix sum (fixed order).  out[0] = beta_next,
// out[1] = log(Z_t / Z_{t-1}).  Non-finite logL count as zero weight.
__global__ __launch_bounds__(SMC_THREADS) void reweight_kernel(const double* __restrict__ logl, int P,
                                                               double beta_prev, double alpha,
                                                               double* __restrict__ cum, double* __restrict__ out) {
    __shared__ double sh[SMC_THREADS];
    double lm = -INFINITY;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        if (isfinite(logl[i])) lm = fmax(lm, logl[i]);
    const double lmax = block_max(lm, sh);
    const double target = alpha * (double)P;
    double beta;
    if (ess_at(logl, P, 1.0 - beta_prev, lmax, sh) >= target) {
        beta = 1.0;
    } else {
        double lo = beta_prev, hi = 1.0;
        for (int it = 0; it < 100 && hi - lo > 1e-14; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (ess_at(logl, P, mid - beta_prev, lmax, sh) >= target) lo = mid; else hi = mid;
        }
        beta = lo;
    }
    const double db = beta - beta_prev;
    // log-sum-exp of db logL (max of db logL is db lmax for db >= 0)
    double s = 0.0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) s += exp(db * (ll_at(logl, i) - lmax));
    const double tot = block_sum(s, sh);
    const double lse = db * lmax + log(tot);
    // prefix sum: thread t owns the contiguous chunk [t*ch, (t+1)*ch)
    const int ch = (P + blockDim.x - 1) / blockDim.x;
    const int a = threadIdx.x * ch, b = min(P, a + ch);
    double loc = 0.0;
    for (int i = a; i < b; ++i) loc += exp(db * ll_at(logl, i) - lse);
    sh[threadIdx.x] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) { const double v = sh[t]; sh[t] = run; run += v; }
    }
    __syncthreads();
    double run = sh[threadIdx.x];
    for (int i = a; i < b; ++i) {
        run += exp(db * ll_at(logl, i) - lse);
        cum[i] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = beta;
        out[1] = lse - log((double)P);
        out[2] = cum[P - 1];
    }
}

// Ancestor of particle i: first k with cum_k / cum_{P-1} > u_i (last entry forced to 1).
__global__ __launch_bounds__(256) void ancestors_kernel(const double* __restrict__ cum, const double* __restrict__ out,
                                                        int P, uint64_t seed, uint64_t iteration,
                                                        int32_t* __restrict__ anc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    double u, u1;
    rng_uniform2(seed, 0u, (uint32_t)i, iteration, RNG_RESAMPLE, u, u1);
    const double total = out[2];
    int lo = 0, hi = P - 1;   // search the first index with normalised cum > u
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double c = (mid == P - 1) ? 1.0 : cum[mid] / total;
        if (c > u) hi = mid; else lo = mid + 1;
    }
    anc[i] = lo;
}

__global__ __launch_bounds__(256) void gather_kernel(const int32_t* __restrict__ anc, int P, int D,
                                                     const double* __restrict__ x, const double* __restrict__ ll,
                                                     const double* __restrict__ g, double* __restrict__ xo,
                                                     double* __restrict__ llo, double* __restrict__ go) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int a = anc[i];
    for (int k = 0; k < D; ++k) xo[(size_t)i * D + k] = x[(size_t)a * D + k];
    llo[i] = ll[a];
    if (g)
        for (int k = 0; k < D; ++k) go[(size_t)i * D + k] = g[(size_t)a * D + k];
}

__global__ __launch_bounds__(256) void copy_back_kernel(int P, int D, const double* __restrict__ xo,
                                                        const double* __restrict__ llo, const double* __restrict__ go,
                                                        double* __restrict__ x, double* __restrict__ ll,
                                                        double* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    for (int k = 0; k < D; ++k) x[(size_t)i * D + k] = xo[(size_t)i * D + k];
    ll[i] = llo[i];
    if (g)
        for (int k = 0; k < D; ++k) g[(size_t)i * D + k] = go[(size_t)i * D + k];
}

// Population mean and covariance (two passes, fixed order), diagonal
// shrinkage and Cholesky; status[0] = 1 when a diagonal fallback was used.
__global__ __launch_bounds__(256) void mass_matrix_kernel(const double* __restrict__ x, int P, int D, double shrink,
                                                          double* __restrict__ inv, double* __restrict__ L,
                                                          int* __restrict__ status) {
    __shared__ double sh[256];
    __shared__ double mu[MAXDIM];
    __shared__ double cov[MAXDIM * MAXDIM];
    __shared__ double l[MAXDIM * MAXDIM];
    for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < P; i += blockDim.x) s += x[(size_t)i * D + k];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) mu[k] = s / P;
    }
    __syncthreads();
    for (int a = 0; a < D; ++a)
        for (int b = 0; b <= a; ++b) {
            double s = 0.0;
            for (int i = threadIdx.x; i < P; i += blockDim.x)
                s += (x[(size_t)i * D + a] - mu[a]) * (x[(size_t)i * D + b] - mu[b]);
            s = block_sum(s, sh);
            if (threadIdx.x == 0) {
                const double v = s / (P - 1);
                cov[a * D + b] = v;
                cov[b * D + a] = v;
            }
        }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 0; k < D; ++k) cov[k * D + k] *= (1.0 + shrink);
    for (int i = 0; i < D * D; ++i) l[i] = 0.0;
    int bad = 0;
    for (int j = 0; j < D && !bad; ++j) {
        double s = cov[j * D + j];
        for (int k = 0; k < j; ++k) s -= l[j * D + k] * l[j * D + k];
        if (!(s > 0.0)) { bad = 1; break; }
        l[j * D + j] = sqrt(s);
        for (int i = j + 1; i < D; ++i) {
            double t = cov[i * D + j];
            for (int k = 0; k < j; ++k) t -= l[i * D + k] * l[j * D + k];
            l[i * D + j] = t / l[j * D + j];
        }
    }
    if (bad) {
        for (int i = 0; i < D * D; ++i) l[i] = 0.0;
        for (int k = 0; k < D; ++k) {
            double v = cov[k * D + k];
            if (!(v > 0.0)) v = 1.0;
            for (int b = 0; b < D; ++b) cov[k * D + b] = (b == k) ? v : 0.0;
            l[k * D + k] = sqrt(v);
        }
    }
    for (int i = 0; i < D * D; ++i) { inv[i] = cov[i]; L[i] = l[i]; }
    status[0] = bad;
}

// Analytic test likelihoods, one particle per lane (same definitions as the
// persistent NUTS kernel's).
__global__ __launch_bounds__(256) void analytic_loglike_kernel(int kind, int P, int D, const double* __restrict__ prm,
                                                               const double* __restrict__ x, double* __restrict__ logl,
                                                               double* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const double* xi = x + (size_t)i * D;
    double* gi = grad ? grad + (size_t)i * D : nullptr;
    double ll = 0.0;
    if (kind == SMCGW_TARGET_GAUSS) {
        for (int k = 0; k < D; ++k) { ll += -0.5 * xi[k] * xi[k]; if (gi) gi[k] = -xi[k]; }
    } else if (kind == SMCGW_TARGET_GAUSS_X_GAUSS) {
        for (int k = 0; k < D; ++k) {
            const double r = (prm[k] - xi[k]) / prm[D + k];
            ll += -0.5 * r * r - 0.5 * log(2.0 * PI * prm[D + k] * prm[D + k]);
            if (gi) gi[k] = r / prm[D + k];
        }
    } else {
        const double sg = prm[2 * D];
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < D; ++k) {
            s1 += (xi[k] - prm[k]) * (xi[k] - prm[k]);
            s2 += (xi[k] - prm[D + k]) * (xi[k] - prm[D + k]);
        }
        const double c = -0.5 * D * log(2.0 * PI * sg * sg);
        const double l1 = c - 0.5 * s1 / (sg * sg), l2 = c - 0.5 * s2 / (sg * sg);
        const double mx = fmax(l1, l2), w1 = exp(l1 - mx), w2 = exp(l2 - mx);
        ll = mx + log(w1 + w2);
        if (gi)
            for (int k = 0; k < D; ++k) gi[k] = (w1 * (prm[k] - xi[k]) + w2 * (prm[D + k] - xi[k])) / (sg * sg) / (w1 + w2);
    }
    logl[i] = ll;
}

// Scratch of the sampler entry points (device), grown on demand.
void* sampler_scratch(smcgw_ctx* c, size_t bytes) {
    if (bytes <= c->sampler_bytes) return c->d_sampler;
    hipFree(c->d_sampler);
    c->d_sampler = nullptr;
    c->sampler_bytes = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&c->d_sampler, cap) != hipSuccess) return nullptr;
    c->sampler_bytes = cap;
    return c->d_sampler;
}

double* pinned(smcgw_ctx* c) {
    if (!c->h_pinned && hipHostMalloc((void**)&c->h_pinned, 64 * sizeof(double)) != hipSuccess) c->h_pinned = nullptr;
    return c->h_pinned;
}

}  // namespace smcgw

extern "C" int smcgw_set_prior(smcgw_ctx* c, int dim, const smcgw_bounds* b) {
    if (!c || !b || dim <= 0 || dim > MAXDIM) return SMCGW_ERR_INVALID;
    PriorDesc p;
    std::memset(&p, 0, sizeof(p));
    p.dim = dim;
    for (int k = 0; k < dim; ++k) {
        if (b[k].bnd < 0 || b[k].bnd > 2 || b[k].prior < 0 || b[k].prior > 3) return SMCGW_ERR_INVALID;
        if ((b[k].bnd != SMCGW_BND_NONE || b[k].prior == SMCGW_PRIOR_UNIFORM || b[k].prior == SMCGW_PRIOR_LOGUNIFORM) &&
            !(b[k].hi > b[k].lo))
            return SMCGW_ERR_INVALID;
        if (b[k].prior == SMCGW_PRIOR_LOGUNIFORM && !(b[k].lo > 0.0)) return SMCGW_ERR_INVALID;
        if (b[k].prior == SMCGW_PRIOR_GAUSSIAN && !(b[k].hi > 0.0)) return SMCGW_ERR_INVALID;
        p.lo[k] = b[k].lo;
        p.hi[k] = b[k].hi;
        p.bnd[k] = b[k].bnd;
        p.kind[k] = b[k].prior;
    }
    c->prior = p;
    c->prior_set = true;
    return SMCGW_OK;
}

extern "C" int smcgw_set_target(smcgw_ctx* c, int kind, int dim, const double* params, int n_params) {
    if (!c || dim <= 0 || dim > MAXDIM) return SMCGW_ERR_INVALID;
    int need = 0;
    switch (kind) {
    case SMCGW_TARGET_GW: need = 0; break;
    case SMCGW_TARGET_GAUSS: need = 0; break;
    case SMCGW_TARGET_GAUSS_X_GAUSS: need = 2 * dim; break;
    case SMCGW_TARGET_BIMODAL: need = 2 * dim + 1; break;
    default: return SMCGW_ERR_INVALID;
    }
    if (n_params < need || (need > 0 && !params)) return SMCGW_ERR_INVALID;
    hipSetDevice(c->device);
    if (!c->d_target_params && hipMalloc(&c->d_target_params, 64 * sizeof(double)) != hipSuccess)
        return SMCGW_ERR_OOM;
    if (need > 0 &&
        (hipMemcpyAsync(c->d_target_params, params, need * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
         hipStreamSynchronize(c->stream)))
        return SMCGW_ERR_HIP;
    c->target.kind = kind;
    c->target.dim = dim;
    c->target.params = c->d_target_params;
    return SMCGW_OK;
}

extern "C" int smcgw_mass_matrix(smcgw_ctx* c, int P, int D, const double* theta, double shrink, double* inv_mass,
                                 double* chol) {
    if (!c || !theta || !inv_mass || !chol || P < 2 || D <= 0 || D > MAXDIM || !(shrink >= 0.0))
        return SMCGW_ERR_INVALID;
    hipSetDevice(c->device);
    int* st = (int*)sampler_scratch(c, 64);
    double* hp = pinned(c);
    if (!st || !hp) return SMCGW_ERR_OOM;
    hipLaunchKernelGGL(mass_matrix_kernel, dim3(1), dim3(256), 0, c->stream, theta, P, D, shrink, inv_mass, chol, st);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    if (hipMemcpyAsync(hp, st, sizeof(int), hipMemcpyDeviceToHost, c->stream) || hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    int s;
    std::memcpy(&s, hp, sizeof(int));
    return s ? SMCGW_WARN_FALLBACK : SMCGW_OK;
}

extern "C" int smcgw_smc_reweight_resample(smcgw_ctx* c, int P, int D, double beta_prev, double alpha, uint64_t seed,
                                           uint64_t iteration, double* theta, double* logl, double* grad,
                                           int32_t* ancestors, double* beta_next_host, double* dlogz_host) {
    if (!c || P < 1 || D <= 0 || D > MAXDIM || !theta || !logl || !ancestors || !beta_next_host || !dlogz_host)
        return SMCGW_ERR_INVALID;
    if (!(alpha > 0.0 && alpha <= 1.0) || !(beta_prev >= 0.0 && beta_prev <= 1.0)) return SMCGW_ERR_INVALID;
    hipSetDevice(c->device);
    const size_t off_cum = 64 * sizeof(double);
    const size_t off_x = off_cum + (size_t)P * sizeof(double);
    const size_t off_ll = off_x + (size_t)P * D * sizeof(double);
    const size_t off_g = off_ll + (size_t)P * sizeof(double);
    const size_t bytes = off_g + (size_t)P * D * sizeof(double);
    char* s = (char*)sampler_scratch(c, bytes);
    double* hp = pinned(c);
    if (!s || !hp) return SMCGW_ERR_OOM;
    double* out = (double*)s;
    double* cum = (double*)(s + off_cum);
    double* xo = (double*)(s + off_x);
    double* llo = (double*)(s + off_ll);
    double* go = (double*)(s + off_g);
    hipLaunchKernelGGL(reweight_kernel, dim3(1), dim3(SMC_THREADS), 0, c->stream, logl, P, beta_prev, alpha, cum, out);
    const dim3 g((P + 255) / 256), b(256);
    hipLaunchKernelGGL(ancestors_kernel, g, b, 0, c->stream, cum, out, P, seed, iteration, ancestors);
    hipLaunchKernelGGL(gather_kernel, g, b, 0, c->stream, ancestors, P, D, theta, logl, grad, xo, llo, go);
    hipLaunchKernelGGL(copy_back_kernel, g, b, 0, c->stream, P, D, xo, llo, go, theta, logl, grad);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    if (hipMemcpyAsync(hp, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    *beta_next_host = hp[0];
    *dlogz_host = hp[1];
    if (!(hp[0] > beta_prev) && beta_prev < 1.0) return SMCGW_ERR_STALL;
    return SMCGW_OK;
}

extern "C" int smcgw_target_loglike_grad(smcgw_ctx* c, int P, const double* theta, double* logl, double* grad,
                                         int precision) {
    if (!c || P < 0 || (P > 0 && (!theta || !logl))) return SMCGW_ERR_INVALID;
    if (precision != SMCGW_PLAIN_FP64 && precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (P == 0) return SMCGW_OK;
    hipSetDevice(c->device);
    if (c->target.kind == SMCGW_TARGET_GW) return ctx_loglike(c, P, c->ev_of_p, theta, logl, grad, precision);
    if (c->target.dim <= 0) return SMCGW_ERR_NOT_INIT;
    hipLaunchKernelGGL(analytic_loglike_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, c->target.kind, P,
                       c->target.dim, c->target.params, theta, logl, grad);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}
