// SMC kernels: adaptive tempering, evidence increment, multinomial
// resampling with gather (arXiv:2601.02336, Sec. 3, Eqs. 4-8), the
// population mass matrix (Sec. 5, covariance reading of the metric) and
// sample recycling (Sec. 5, "Samples recycling").
//
// All reductions run inside one workgroup in a fixed order (no atomics), in
// FP64, so beta, the evidence increment and the ancestors are reproducible.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "common.h"
#include "context.h"
#include "philox.h"

using namespace smcgw;

namespace smcgw {

constexpr int SMC_THREADS = 1024;
constexpr int SMC_WAVES = SMC_THREADS / 64;
// Bisection levels resolved per pass over the particles: every pass evaluates
// the ESS at all 2^RW_LEVELS - 1 midpoints the next RW_LEVELS bisection steps
// could visit (and, in the first pass, at beta = 1), so the walk down that
// subtree takes the sequential bisection's decisions.
constexpr int RW_LEVELS = 4;
constexpr int RW_CAND = 1 << RW_LEVELS;
constexpr int RW_THREADS = 512;   // 32 FP64 accumulators per thread need the larger register budget
// Per-run result block of the reweighting: beta_next, the evidence increment,
// the weight total, and whether the run's resampling is skipped.
constexpr int OUT_SIZE = 4;
constexpr int OUT_SKIP = 3;
constexpr double SKIP_NONE = 0.0, SKIP_DONE = 1.0, SKIP_STALL = 2.0;


// Workgroup sums of K values per thread: wavefront totals (one scattered
// reduction of all K values), then added in wavefront order.  tot[k] is valid
// in all threads after the call; red must hold K * (blockDim.x / 64) doubles.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* red, double* tot) {
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int idx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) idx[k] = k * nw;
    wave_totals_to<K>(v, idx, red + wave);
    __syncthreads();
    if ((int)threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x * nw + w];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max_total(v);
    if (lane == TOTAL_LANE) red[wave] = v;
    __syncthreads();
    double m = red[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

// log-likelihood with NaN mapped to -inf (zero weight)
__device__ __forceinline__ double ll_at(const double* logl, int i) {
    const double v = logl[i];
    return v == v ? v : -INFINITY;
}

// w = L^db / Lmax^db for e = logL - logLmax <= 0; db = 0 gives 1 for every
// particle (equal weights), also where L = 0.
__device__ __forceinline__ double incr_weight(double db, double e) { return db == 0.0 ? 1.0 : exp(db * e); }

// One workgroup: beta_next by bisection on the ESS, the evidence increment,
// normalised weights and their inclusive prefix sum (fixed order).
// out[0] = beta_next, out[1] = log(Z_t / Z_{t-1}), out[2] = cum[P-1].
// Non-finite logL count as zero weight.
// Persistent sampling passes lofs [P] (the log mixture density of every
// pooled point, see pool_logmix_kernel) and n_target (points per
// population): a point's weight at beta is then L^beta / mixture, written as
// exp(g_i + (beta - beta_prev) (logL_i - lmax)) with g_i = beta_prev logL_i -
// lofs_i - max_j(...), the ESS target is alpha n_target and out[1] is log Z
// at beta_next itself (the pool mean of the weights).  lofs = NULL is
// standard SMC (g_i = 0, n_target = P).
//
// Independent runs: run r = blockIdx.y takes logl + r P, cum + r P and
// out + r OUT_SIZE.  With a run state st (st + r SMCGW_STATE_SIZE), beta_prev
// is the state's temperature; a run that is done, or whose last iteration
// already mutated at beta = 1, gets out[OUT_SKIP] = SKIP_DONE and nothing
// else, and a ladder that cannot advance gets SKIP_STALL.
__global__ __launch_bounds__(RW_THREADS) void reweight_kernel(const double* __restrict__ logl, int P,
                                                              double beta_prev, double alpha,
                                                              const double* __restrict__ lofs, int n_target,
                                                              double* __restrict__ cum, double* __restrict__ out,
                                                              const double* __restrict__ st) {
    __shared__ double red[2 * RW_CAND * (RW_THREADS / 64)];
    __shared__ double tot[2 * RW_CAND];
    __shared__ double cand[2][RW_CAND];   // by pass parity: a wavefront may write the next pass's midpoints
                                          // while another still walks this pass's
    __shared__ double scan[RW_THREADS / 64 + 1];
    const int rix = blockIdx.y;   // run index
    logl += (size_t)rix * P;
    cum += (size_t)rix * P;
    out += (size_t)rix * OUT_SIZE;
    if (st) {
        st += (size_t)rix * SMCGW_STATE_SIZE;
        if (st[SMCGW_ST_DONE] != 0.0 || (st[SMCGW_ST_BETA] >= 1.0 && st[SMCGW_ST_NEXT] > 0.0)) {
            if (threadIdx.x == 0) out[OUT_SKIP] = SKIP_DONE;
            return;
        }
        beta_prev = st[SMCGW_ST_BETA];
    }
    double lm = -INFINITY, gm = -INFINITY;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const double l = ll_at(logl, i);
        lm = fmax(lm, l);
        if (lofs && l > -INFINITY) gm = fmax(gm, beta_prev * l - lofs[i]);
    }
    const double lmax = block_max(lm, red);
    if (!(lmax > -INFINITY)) {   // no particle with a finite likelihood: nothing to reweight
        for (int i = threadIdx.x; i < P; i += blockDim.x) cum[i] = 0.0;
        if (threadIdx.x == 0) {
            out[0] = beta_prev; out[1] = -INFINITY; out[2] = 0.0;
            out[OUT_SKIP] = st ? SKIP_STALL : SKIP_NONE;
        }
        return;
    }
    const double gmax = lofs ? block_max(gm, red) : 0.0;
    // base log weight of point i at beta_prev, relative to the largest (0 for standard SMC)
    auto base = [&](int i, double l) { return lofs ? beta_prev * l - lofs[i] - gmax : 0.0; };
    const double target = alpha * (double)(lofs ? n_target : P);
    // Each pass resolves RW_LEVELS bisection levels below [lo, hi].  The
    // midpoints those levels can visit are lo + k h, k = 1..15, h = (hi - lo)/16
    // (slot k); they are computed exactly as the sequential bisection computes
    // them (heap node n: children 2n below, 2n+1 above) and stored by node for
    // the walk.  A particle's weights on the grid are a geometric sequence,
    // w_k = exp((lo - beta_prev) e) exp(h e)^k, so a pass costs two exps per
    // particle.  Slot 0 of the first pass holds beta = 1.
    double lo = beta_prev, hi = 1.0, beta = -1.0;
    int it = 0;
    for (int pass = 0; beta < 0.0; ++pass) {
        double a[RW_CAND], b[RW_CAND], mid[RW_CAND];
        a[1] = lo; b[1] = hi;
#pragma unroll
        for (int n = 1; n < RW_CAND; ++n) {
            mid[n] = 0.5 * (a[n] + b[n]);
            if (2 * n + 1 < RW_CAND) {
                a[2 * n] = a[n]; b[2 * n] = mid[n];
                a[2 * n + 1] = mid[n]; b[2 * n + 1] = b[n];
            }
        }
        double* cnd = cand[pass & 1];
        if (threadIdx.x < RW_CAND) cnd[threadIdx.x] = threadIdx.x == 0 ? 1.0 : mid[threadIdx.x];
        const double h = (hi - lo) * (1.0 / RW_CAND);
        const double d0 = lo - beta_prev;
        double s[2 * RW_CAND];
#pragma unroll
        for (int n = 0; n < 2 * RW_CAND; ++n) s[n] = 0.0;
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            const double l = ll_at(logl, i);
            const double e = l - lmax;
            if (e == -INFINITY) continue;   // zero weight at every candidate (db > 0)
            const double g = base(i, l);
            if (pass == 0) {
                const double w1 = exp(g + (1.0 - beta_prev) * e);
                s[0] += w1;
                s[1] += w1 * w1;
            }
            const double r = exp(h * e);
            double w = exp(g + d0 * e);
#pragma unroll
            for (int k = 1; k < RW_CAND; ++k) {
                w *= r;
                s[2 * k] += w;
                s[2 * k + 1] += w * w;
            }
        }
        block_sums<2 * RW_CAND>(s, red, tot);
        if (pass == 0 && tot[0] * tot[0] / tot[1] >= target) { beta = 1.0; break; }
        int n = 1;
        for (int lev = 0; lev < RW_LEVELS; ++lev) {
            if (!(it < 100 && hi - lo > 1e-14)) { beta = lo; break; }
            const int k = (2 * (n - (1 << lev)) + 1) << (RW_LEVELS - 1 - lev);   // grid slot of node n
            if (tot[2 * k] * tot[2 * k] / tot[2 * k + 1] >= target) { lo = cnd[n]; n = 2 * n + 1; }
            else { hi = cnd[n]; n = 2 * n; }
            ++it;
        }
    }
    const double db = beta - beta_prev;
    // weight of point i at beta relative to db lmax + gmax (zero for a non-finite logL)
    auto weight = [&](int i) {
        const double l = ll_at(logl, i);
        if (!lofs) return incr_weight(db, l - lmax);
        return l > -INFINITY ? exp(base(i, l) + db * (l - lmax)) : 0.0;
    };
    // log-sum-exp of the log weights (max of db logL is db lmax for db >= 0)
    double s1[1] = {0.0};
    for (int i = threadIdx.x; i < P; i += blockDim.x) s1[0] += weight(i);
    block_sums<1>(s1, red, tot);
    const double lse = db * lmax + gmax + log(tot[0]);
    // inclusive prefix sum: thread t owns the contiguous chunk [t*ch, (t+1)*ch)
    const int ch = (P + blockDim.x - 1) / blockDim.x;
    const int lo_i = threadIdx.x * ch, hi_i = min(P, lo_i + ch);
    double loc = 0.0;
    const double inv_tot = 1.0 / tot[0];   // normalised weight: exp(db (logL - lmax)) / sum
    for (int i = lo_i; i < hi_i; ++i) loc += weight(i) * inv_tot;
    // exclusive scan of the chunk totals: lanes (shuffle ladder), then wavefronts
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { scan[w] = run; run += red[w]; }
        scan[blockDim.x >> 6] = run;
    }
    __syncthreads();
    double ex = __shfl_up(inc, 1);
    if (lane == 0) ex = 0.0;
    double run = scan[wave] + ex;
    for (int i = lo_i; i < hi_i; ++i) {
        run += weight(i) * inv_tot;
        cum[i] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = beta;
        out[1] = lse - log((double)P);
        out[2] = cum[P - 1];
        out[OUT_SKIP] = (st && !(beta > beta_prev) && beta_prev < 1.0) ? SKIP_STALL : SKIP_NONE;
    }
}

// Ancestor of particle i: first k with cum_k / cum_{P-1} > u_i (last entry forced to 1).
// Run r = blockIdx.y draws n_draw ancestors among its P weights with key
// seed + r and, with a run state, the iteration index state[NEXT].
__global__ __launch_bounds__(256) void ancestors_kernel(const double* __restrict__ cum, const double* __restrict__ out,
                                                        int P, int n_draw, uint64_t seed, uint64_t iteration,
                                                        int32_t* __restrict__ anc, const double* __restrict__ st) {
    const int run = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    out += (size_t)run * OUT_SIZE;
    if (i >= n_draw || out[OUT_SKIP] != SKIP_NONE) return;
    cum += (size_t)run * P;
    anc += (size_t)run * n_draw;
    if (st) iteration = (uint64_t)st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_NEXT];
    double u, u1;
    rng_uniform2(seed + (uint64_t)run, 0u, (uint32_t)i, iteration, RNG_RESAMPLE, u, u1);
    const double total = out[2];
    int lo = 0, hi = P - 1;   // search the first index with normalised cum > u
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double c = (mid == P - 1) ? 1.0 : cum[mid] / total;
        if (c > u) hi = mid; else lo = mid + 1;
    }
    anc[i] = lo;
}

// Gather of run r = blockIdx.y: P particles drawn from its n_src candidates
// (n_src = P for standard SMC, the pool for persistent sampling).
__global__ __launch_bounds__(256) void gather_kernel(const int32_t* __restrict__ anc, int P, int D, int n_src,
                                                     const double* __restrict__ x, const double* __restrict__ ll,
                                                     const double* __restrict__ g, const int32_t* __restrict__ cy,
                                                     double* __restrict__ xo, double* __restrict__ llo,
                                                     double* __restrict__ go, int32_t* __restrict__ cyo,
                                                     const double* __restrict__ out) {
    const int run = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P || out[(size_t)run * OUT_SIZE + OUT_SKIP] != SKIP_NONE) return;
    const size_t src = (size_t)run * n_src + anc[(size_t)run * P + i], dst = (size_t)run * P + i;
    for (int k = 0; k < D; ++k) xo[dst * D + k] = x[src * D + k];
    llo[dst] = ll[src];
    if (g)
        for (int k = 0; k < D; ++k) go[dst * D + k] = g[src * D + k];
    if (cy) cyo[dst] = cy[src];
}

__global__ __launch_bounds__(256) void copy_back_kernel(int P, int D, const double* __restrict__ xo,
                                                        const double* __restrict__ llo, const double* __restrict__ go,
                                                        const int32_t* __restrict__ cyo, double* __restrict__ x,
                                                        double* __restrict__ ll, double* __restrict__ g,
                                                        int32_t* __restrict__ cy, const double* __restrict__ out) {
    const int run = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P || out[(size_t)run * OUT_SIZE + OUT_SKIP] != SKIP_NONE) return;
    const size_t j = (size_t)run * P + i;
    for (int k = 0; k < D; ++k) x[j * D + k] = xo[j * D + k];
    ll[j] = llo[j];
    if (g)
        for (int k = 0; k < D; ++k) g[j * D + k] = go[j * D + k];
    if (cy) cy[j] = cyo[j];
}

// Run states after the reweighting (one thread per run): the temperature,
// the increment and the running log evidence log Z_t = log Z_{t-1} +
// log(Z_t / Z_{t-1}) in FP64 (Sec. 3.1, Eq. 8), the iteration index, and the
// first three entries of the record row t.  A skipped run is marked done
// (stalled when the temperature could not advance).
__global__ void state_update_kernel(const double* __restrict__ out, int n_runs, double* __restrict__ st,
                                    double* __restrict__ hist, int hist_cap) {
    const int r = threadIdx.x;
    if (r >= n_runs) return;
    const double* o = out + (size_t)r * OUT_SIZE;
    double* s = st + (size_t)r * SMCGW_STATE_SIZE;
    if (o[OUT_SKIP] != SKIP_NONE) {
        if (o[OUT_SKIP] == SKIP_STALL) s[SMCGW_ST_STALL] = 1.0;
        s[SMCGW_ST_DONE] = 1.0;
        return;
    }
    const double t = s[SMCGW_ST_NEXT];
    s[SMCGW_ST_BETA] = o[0];
    s[SMCGW_ST_DLOGZ] = o[1];
    s[SMCGW_ST_LOGZ] += o[1];
    s[SMCGW_ST_ITER] = t;
    s[SMCGW_ST_NEXT] = t + 1.0;
    if (hist && t < (double)hist_cap) {
        double* h = hist + ((size_t)r * hist_cap + (size_t)t) * SMCGW_HIST_SIZE;
        h[SMCGW_H_BETA] = o[0];
        h[SMCGW_H_LOGZ] = s[SMCGW_ST_LOGZ];
        h[SMCGW_H_DLOGZ] = o[1];
    }
}

// Covariance entries (a, b), b <= a < MAXDIM, in row order (a compile-time table).
constexpr int MM_ENTRIES = MAXDIM * (MAXDIM + 1) / 2;
struct TriTable {
    int a[MM_ENTRIES], b[MM_ENTRIES];
    constexpr TriTable() : a(), b() {
        int e = 0;
        for (int i = 0; i < MAXDIM; ++i)
            for (int j = 0; j <= i; ++j) { a[e] = i; b[e] = j; ++e; }
    }
};
constexpr TriTable TRI{};

// Population covariance in one pass over the particles, shifted by the first
// particle x_0 (the mean of the shifted values is small, so the one-pass
// form keeps its accuracy): per block of MMB particles, in particle order,
//   s_k = sum_i (x_ik - x_0k),  s_ab = sum_i (x_ia - x_0a)(x_ib - x_0b),
// one thread per sum; the block's rows are staged in LDS.
constexpr int MMB = 64;
constexpr int MM_SUMS = MAXDIM + MM_ENTRIES;
constexpr int MM_THREADS = 256;
static_assert(MM_SUMS <= MM_THREADS, "one thread per sum");

// A run whose state says done (st, nullable) is skipped.
__device__ __forceinline__ bool run_is_done(const double* st, int run) {
    return st && st[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_DONE] != 0.0;
}

// Run r = blockIdx.y covers particles [r P, (r+1) P); its block partials go
// to part + r gridDim.x MM_SUMS.
__global__ __launch_bounds__(MM_THREADS) void mm_partial_kernel(const double* __restrict__ x, int P, int D,
                                                                double* __restrict__ part,
                                                                const double* __restrict__ st) {
    __shared__ double xs[MMB * MAXDIM];
    __shared__ double x0[MAXDIM];
    const int run = blockIdx.y;
    if (run_is_done(st, run)) return;
    x += (size_t)run * P * D;
    part += (size_t)run * gridDim.x * MM_SUMS;
    const int blk = blockIdx.x;
    const int i0 = blk * MMB, n = min(MMB, P - i0);
    for (int t = threadIdx.x; t < n * D; t += blockDim.x) xs[t] = x[(size_t)i0 * D + t];
    if ((int)threadIdx.x < D) x0[threadIdx.x] = x[threadIdx.x];
    __syncthreads();
    const int e = threadIdx.x;
    if (e >= MM_SUMS) return;
    double s = 0.0;
    if (e < MAXDIM) {
        if (e < D)
            for (int i = 0; i < n; ++i) s += xs[i * D + e] - x0[e];
    } else {
        const int a = TRI.a[e - MAXDIM], b = TRI.b[e - MAXDIM];
        if (a < D)
            for (int i = 0; i < n; ++i) s += (xs[i * D + a] - x0[a]) * (xs[i * D + b] - x0[b]);
    }
    part[(size_t)blk * MM_SUMS + e] = s;
}

// Block partials summed in block order, covariance (s_ab - s_a s_b / P) / (P - 1),
// diagonal shrinkage and Cholesky; status[0] = 1 when a diagonal fallback
// was used.
// One workgroup per run (blockIdx.x): inv, L + run D D, status + run.
__global__ __launch_bounds__(MM_THREADS) void mm_finish_kernel(const double* __restrict__ part, int nblk, int P,
                                                               int D, double shrink, double* __restrict__ inv,
                                                               double* __restrict__ L, int* __restrict__ status,
                                                               const double* __restrict__ st) {
    __shared__ double tot[MM_SUMS];
    __shared__ double cov[MAXDIM * MAXDIM];
    __shared__ double l[MAXDIM * MAXDIM];
    __shared__ int bad;
    const int run = blockIdx.x;
    if (run_is_done(st, run)) return;
    part += (size_t)run * nblk * MM_SUMS;
    inv += (size_t)run * D * D;
    L += (size_t)run * D * D;
    status += run;
    if ((int)threadIdx.x < MM_SUMS) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * MM_SUMS + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < MM_ENTRIES; e += blockDim.x) {
        const int a = TRI.a[e], b = TRI.b[e];
        if (a < D) {
            const double v = (tot[MAXDIM + e] - tot[a] * tot[b] / P) / (P - 1);
            cov[a * D + b] = v;
            cov[b * D + a] = v;
        }
    }
    __syncthreads();
    // Cholesky on wavefront 0, one row per lane: column j needs the finished
    // columns < j of rows j and i, read from LDS.
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    if (lane < D) cov[lane * D + lane] *= (1.0 + shrink);
    for (int i = lane; i < D * D; i += 64) l[i] = 0.0;
    if (lane == 0) bad = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < D; ++j) {
        double sjj = cov[j * D + j];
        for (int k = 0; k < j; ++k) sjj -= l[j * D + k] * l[j * D + k];
        if (!(sjj > 0.0)) { if (lane == 0) bad = 1; break; }   // uniform: every lane computes sjj
        const double ljj = sqrt(sjj);
        if (lane > j && lane < D) {
            double t = cov[lane * D + j];
            for (int k = 0; k < j; ++k) t -= l[lane * D + k] * l[j * D + k];
            l[lane * D + j] = t / ljj;
        }
        if (lane == j) l[j * D + j] = ljj;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (bad) {
        for (int i = lane; i < D * D; i += 64) l[i] = 0.0;
        __builtin_amdgcn_wave_barrier();
        if (lane < D) {
            double v = cov[lane * D + lane];
            if (!(v > 0.0)) v = 1.0;
            for (int b = 0; b < D; ++b) cov[lane * D + b] = (b == lane) ? v : 0.0;
            l[lane * D + lane] = sqrt(v);
        }
        __builtin_amdgcn_wave_barrier();
    }
    for (int i = lane; i < D * D; i += 64) { inv[i] = cov[i]; L[i] = l[i]; }
    if (lane == 0) status[0] = bad;
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

// Record row t = state[ITER] of run r = blockIdx.x after its transition:
// leapfrog steps, summed depth, divergent transitions (fixed-order sums over
// the run's particles), the covariance fallback flag and the local metric's
// fallbacks.  A run that was done before this iteration is skipped.
constexpr int REC_THREADS = 256;
__global__ __launch_bounds__(REC_THREADS) void record_kernel(int P, const int32_t* __restrict__ nlf,
                                                             const int32_t* __restrict__ depth,
                                                             const uint8_t* __restrict__ div,
                                                             const int32_t* __restrict__ mm_status,
                                                             const int32_t* __restrict__ metric_status,
                                                             const double* __restrict__ st, double* __restrict__ hist,
                                                             int hist_cap) {
    __shared__ double red[4 * (REC_THREADS / 64)];
    __shared__ double tot[4];
    const int run = blockIdx.x;
    const double* s = st + (size_t)run * SMCGW_STATE_SIZE;
    if (s[SMCGW_ST_DONE] != 0.0 || !(s[SMCGW_ST_ITER] < (double)hist_cap)) return;
    const size_t base = (size_t)run * P;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        v[0] += (double)nlf[base + i];
        v[1] += (double)depth[base + i];
        v[2] += (double)div[base + i];
        if (metric_status) v[3] += (double)metric_status[base + i];
    }
    block_sums<4>(v, red, tot);
    if (threadIdx.x == 0) {
        double* h = hist + ((size_t)run * hist_cap + (size_t)s[SMCGW_ST_ITER]) * SMCGW_HIST_SIZE;
        h[SMCGW_H_LEAPFROG] = tot[0];
        h[SMCGW_H_DEPTH] = tot[1];
        h[SMCGW_H_DIVERGENT] = tot[2];
        h[SMCGW_H_METRIC_FALLBACKS] = tot[3];
        h[SMCGW_H_MM_FALLBACK] = mm_status ? (double)mm_status[run] : 0.0;
    }
}

// log((1/T) sum_t L^beta_t / Z_t) for one point of log-likelihood l.
__device__ __forceinline__ double log_mixture(double l, const double* betas, const double* logz, int T) {
    double m = -INFINITY;
    for (int t = 0; t < T; ++t) m = fmax(m, betas[t] * l - logz[t]);
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += exp(betas[t] * l - logz[t] - m);
    return m + log(s) - log((double)T);
}

// Sample recycling (Sec. 5, "Samples recycling").  The populations left by
// the mutations of iterations t = 1..T form a pool read as draws of the
// mixture (1/T) sum_t p_t, p_t = L^beta_t pi / Z_t.  Point i's weight for the
// final target against the mixture is
//   log w_i = log L_i - log Z_T - log((1/T) sum_t L_i^beta_t / Z_t),
// one lane per point (the prior cancels; NaN or -inf log L: weight zero).
__global__ __launch_bounds__(256) void recycle_weights_kernel(const double* __restrict__ logl, int n, int T,
                                                              const double* __restrict__ bz,
                                                              double* __restrict__ logw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = logl[i];
    if (!(l > -INFINITY)) {
        logw[i] = -INFINITY;
        return;
    }
    logw[i] = l - bz[2 * T - 1] - log_mixture(l, bz, bz + T, T);
}

// Log mixture density of the pool at every point (persistent sampling):
// lofs_i = log((1/T) sum_t L_i^beta_t / Z_t); entries of non-finite logL are
// not used.
__global__ __launch_bounds__(256) void pool_logmix_kernel(const double* __restrict__ logl, int n, int T,
                                                          const double* __restrict__ bz, double* __restrict__ lofs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double l = logl[i];
    lofs[i] = l > -INFINITY ? log_mixture(l, bz, bz + T, T) : 0.0;
}

// Rejection sampling over the pool in one workgroup: point i is kept when
// its Philox uniform (index 0, particle i, iteration 0, purpose RECYCLE) is
// below w_i / max w.  Thread t owns the contiguous chunk [t ch, (t+1) ch), so
// the kept indices come out in increasing order after an exclusive scan of
// the per-thread counts.  out[0] = kept count, out[1] = Kish ESS
// (sum w)^2 / sum w^2, out[2] = max log w.
__global__ __launch_bounds__(SMC_THREADS) void recycle_select_kernel(const double* __restrict__ logw, int n,
                                                                     uint64_t seed, int32_t* __restrict__ kept,
                                                                     double* __restrict__ out) {
    __shared__ double red[2 * SMC_WAVES];
    __shared__ double tot[2];
    __shared__ int cnt[SMC_THREADS + 1];
    const int tid = threadIdx.x;
    const int ch = (n + SMC_THREADS - 1) / SMC_THREADS;
    const int i0 = min(n, tid * ch), i1 = min(n, i0 + ch);
    double m = -INFINITY;
    for (int i = i0; i < i1; ++i) m = fmax(m, logw[i]);
    const double wmax = block_max(m, red);
    const bool any = wmax > -INFINITY;
    double v[2] = {0.0, 0.0};
    int k = 0;
    if (any)
        for (int i = i0; i < i1; ++i) {
            const double w = exp(logw[i] - wmax);
            v[0] += w;
            v[1] += w * w;
            double u, u1;
            rng_uniform2(seed, 0u, (uint32_t)i, 0, RNG_RECYCLE, u, u1);
            k += u < w ? 1 : 0;
        }
    block_sums<2>(v, red, tot);
    cnt[tid] = k;
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int t = 0; t < SMC_THREADS; ++t) {
            const int c = cnt[t];
            cnt[t] = s;
            s += c;
        }
        cnt[SMC_THREADS] = s;
    }
    __syncthreads();
    int o = cnt[tid];
    if (any)
        for (int i = i0; i < i1; ++i) {
            double u, u1;
            rng_uniform2(seed, 0u, (uint32_t)i, 0, RNG_RECYCLE, u, u1);
            if (u < exp(logw[i] - wmax)) kept[o++] = i;
        }
    if (tid == 0) {
        out[0] = (double)cnt[SMC_THREADS];
        out[1] = tot[1] > 0.0 ? tot[0] * tot[0] / tot[1] : 0.0;
        out[2] = wmax;
    }
}

// out[0..1] (beta_next, evidence increment) into the caller's device buffer.
__global__ void export_pair_kernel(const double* __restrict__ out, double* __restrict__ dst) {
    if (threadIdx.x < 2) dst[threadIdx.x] = out[threadIdx.x];
}

// Scratch of the sampler entry points (device), grown on demand.
void* sampler_scratch(smcgw_ctx* c, size_t bytes) {
    if (bytes <= c->sampler_bytes) return c->d_sampler;
    (void)hipFree(c->d_sampler);
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
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
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
                                 double* chol, int32_t* status_device) {
    if (!c || !theta || !inv_mass || !chol || P < 2 || D <= 0 || D > MAXDIM || !(shrink >= 0.0))
        return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    int* st = status_device;
    double* hp = nullptr;
    if (!st) {
        st = (int*)sampler_scratch(c, 64);
        hp = pinned(c);
        if (!st || !hp) return SMCGW_ERR_OOM;
    }
    const int nblk = (P + MMB - 1) / MMB;
    if (mm_reserve(c, 1, P) != SMCGW_OK) return SMCGW_ERR_OOM;
    hipLaunchKernelGGL(mm_partial_kernel, dim3(nblk), dim3(MM_THREADS), 0, c->stream, theta, P, D, c->d_mm,
                       (const double*)nullptr);
    hipLaunchKernelGGL(mm_finish_kernel, dim3(1), dim3(MM_THREADS), 0, c->stream, (const double*)c->d_mm, nblk, P, D,
                       shrink, inv_mass, chol, st, (const double*)nullptr);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    if (status_device) return SMCGW_OK;
    if (hipMemcpyAsync(hp, st, sizeof(int), hipMemcpyDeviceToHost, c->stream) || hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    int s;
    std::memcpy(&s, hp, sizeof(int));
    return s ? SMCGW_WARN_FALLBACK : SMCGW_OK;
}

namespace smcgw {
// Reweighting, temperature search, resampling and gather of n_runs runs of P
// particles on the context's stream (run r: particles [r P, (r+1) P)); out
// (device, [n_runs][OUT_SIZE]) holds beta_next, the evidence increment, the
// weight total and the skip flag of each run when the queued work has run.
// With run states st, beta_prev and the iteration index come from them and
// state_update_kernel advances them (and fills the record rows in hist).
int queue_reweight_resample(smcgw_ctx* c, int n_runs, int P, int D, double beta_prev, double alpha, uint64_t seed,
                            uint64_t iteration, double* theta, double* logl, double* grad, int32_t* carry,
                            int32_t* ancestors, double* st, double* hist, int hist_cap, double** out_dev) {
    if (!c || n_runs < 1 || P < 1 || D <= 0 || D > MAXDIM || !theta || !logl || !ancestors) return SMCGW_ERR_INVALID;
    if (!(alpha > 0.0 && alpha <= 1.0) || !(beta_prev >= 0.0 && beta_prev <= 1.0)) return SMCGW_ERR_INVALID;
    if ((size_t)n_runs * P > (size_t)INT32_MAX) return SMCGW_ERR_SHAPE;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    const size_t n = (size_t)n_runs * P;
    const size_t off_cum = 64 * sizeof(double) * ((n_runs * OUT_SIZE + 63) / 64);
    const size_t off_x = off_cum + n * sizeof(double);
    const size_t off_ll = off_x + n * D * sizeof(double);
    const size_t off_g = off_ll + n * sizeof(double);
    const size_t off_cy = off_g + n * D * sizeof(double);
    const size_t bytes = off_cy + n * sizeof(int32_t);
    char* s = (char*)sampler_scratch(c, bytes);
    if (!s) return SMCGW_ERR_OOM;
    double* out = (double*)s;
    double* cum = (double*)(s + off_cum);
    double* xo = (double*)(s + off_x);
    double* llo = (double*)(s + off_ll);
    double* go = (double*)(s + off_g);
    int32_t* cyo = (int32_t*)(s + off_cy);
    hipLaunchKernelGGL(reweight_kernel, dim3(1, n_runs), dim3(RW_THREADS), 0, c->stream, logl, P, beta_prev, alpha,
                       (const double*)nullptr, P, cum, out, (const double*)st);
    const dim3 g((P + 255) / 256, n_runs), b(256);
    hipLaunchKernelGGL(ancestors_kernel, g, b, 0, c->stream, cum, out, P, P, seed, iteration, ancestors,
                       (const double*)st);
    hipLaunchKernelGGL(gather_kernel, g, b, 0, c->stream, ancestors, P, D, P, theta, logl, grad, carry, xo, llo, go,
                       cyo, (const double*)out);
    hipLaunchKernelGGL(copy_back_kernel, g, b, 0, c->stream, P, D, xo, llo, go, cyo, theta, logl, grad, carry,
                       (const double*)out);
    if (st)
        hipLaunchKernelGGL(state_update_kernel, dim3(1), dim3(SMCGW_MAX_RUNS), 0, c->stream, (const double*)out,
                           n_runs, st, hist, hist_cap);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    *out_dev = out;
    return SMCGW_OK;
}

size_t reweight_scratch_bytes(int n_runs, int P, int D) {
    const size_t n = (size_t)n_runs * P;
    return 64 * sizeof(double) * ((n_runs * OUT_SIZE + 63) / 64) + n * (2 * D + 2) * sizeof(double) +
           n * sizeof(int32_t);
}

// Block partials of the population covariance for n_runs runs of P particles.
int mm_reserve(smcgw_ctx* c, int n_runs, int P) {
    const int nblk = (P + MMB - 1) / MMB;
    const size_t need = (size_t)n_runs * nblk * MM_SUMS * sizeof(double);
    if (need <= c->mm_bytes) return SMCGW_OK;
    (void)hipFree(c->d_mm);
    c->d_mm = nullptr;
    c->mm_bytes = 0;
    if (hipMalloc(&c->d_mm, need) != hipSuccess) return SMCGW_ERR_OOM;
    c->mm_bytes = need;
    return SMCGW_OK;
}

// Covariance, shrinkage and factor of every run (run r: particles [r P, (r+1) P),
// inv, chol + r D D, status + r); runs whose state says done are skipped.
int queue_mass_matrix_runs(smcgw_ctx* c, int n_runs, int P, int D, const double* theta, double shrink, double* inv,
                           double* chol, int32_t* status, const double* st) {
    const int nblk = (P + MMB - 1) / MMB;
    if ((size_t)n_runs * nblk * MM_SUMS * sizeof(double) > c->mm_bytes) return SMCGW_ERR_INVALID;
    hipLaunchKernelGGL(mm_partial_kernel, dim3(nblk, n_runs), dim3(MM_THREADS), 0, c->stream, theta, P, D, c->d_mm,
                       st);
    hipLaunchKernelGGL(mm_finish_kernel, dim3(n_runs), dim3(MM_THREADS), 0, c->stream, (const double*)c->d_mm, nblk, P,
                       D, shrink, inv, chol, status, st);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

// Record rows of every run after its transition.
int queue_record(smcgw_ctx* c, int n_runs, int P, const int32_t* nlf, const int32_t* depth, const uint8_t* div,
                 const int32_t* mm_status, const int32_t* metric_status, const double* st, double* hist,
                 int hist_cap) {
    hipLaunchKernelGGL(record_kernel, dim3(n_runs), dim3(REC_THREADS), 0, c->stream, P, nlf, depth, div, mm_status,
                       metric_status, st, hist, hist_cap);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

static int reweight_resample(smcgw_ctx* c, int P, int D, double beta_prev, double alpha, uint64_t seed,
                             uint64_t iteration, double* theta, double* logl, double* grad, int32_t* carry,
                             int32_t* ancestors, double** out_dev) {
    return queue_reweight_resample(c, 1, P, D, beta_prev, alpha, seed, iteration, theta, logl, grad, carry, ancestors,
                                   nullptr, nullptr, 0, out_dev);
}
}  // namespace smcgw

extern "C" int smcgw_smc_reweight_resample(smcgw_ctx* c, int P, int D, double beta_prev, double alpha, uint64_t seed,
                                           uint64_t iteration, double* theta, double* logl, double* grad,
                                           int32_t* carry, int32_t* ancestors, double* beta_next_host,
                                           double* dlogz_host) {
    if (!beta_next_host || !dlogz_host) return SMCGW_ERR_INVALID;
    double* out = nullptr;
    int rc = reweight_resample(c, P, D, beta_prev, alpha, seed, iteration, theta, logl, grad, carry, ancestors, &out);
    if (rc) return rc;
    double* hp = pinned(c);
    if (!hp) return SMCGW_ERR_OOM;
    if (hipMemcpyAsync(hp, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    *beta_next_host = hp[0];
    *dlogz_host = hp[1];
    if (!(hp[0] > beta_prev) && beta_prev < 1.0) return SMCGW_ERR_STALL;
    return SMCGW_OK;
}

extern "C" int smcgw_smc_reweight_resample_async(smcgw_ctx* c, int P, int D, double beta_prev, double alpha,
                                                 uint64_t seed, uint64_t iteration, double* theta, double* logl,
                                                 double* grad, int32_t* carry, int32_t* ancestors,
                                                 double* out_device) {
    if (!out_device) return SMCGW_ERR_INVALID;
    double* out = nullptr;
    int rc = reweight_resample(c, P, D, beta_prev, alpha, seed, iteration, theta, logl, grad, carry, ancestors, &out);
    if (rc) return rc;
    hipLaunchKernelGGL(export_pair_kernel, dim3(1), dim3(64), 0, c->stream, out, out_device);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

extern "C" int smcgw_target_loglike_grad(smcgw_ctx* c, int P, const double* theta, double* logl, double* grad,
                                         int precision) {
    if (!c || P < 0 || (P > 0 && (!theta || !logl))) return SMCGW_ERR_INVALID;
    if (precision != SMCGW_PLAIN_FP64 && precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    if (c->target.kind == SMCGW_TARGET_GW) return ctx_loglike(c, P, c->ev_of_p, theta, logl, grad, precision);
    if (c->target.dim <= 0) return SMCGW_ERR_NOT_INIT;
    hipLaunchKernelGGL(analytic_loglike_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, c->target.kind, P,
                       c->target.dim, c->target.params, theta, logl, grad);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

extern "C" int smcgw_recycle(smcgw_ctx* c, int T, int N, const double* logl, const double* betas_host,
                             const double* logz_host, uint64_t seed, double* logw, int32_t* kept,
                             int64_t* n_kept_host, double* ess_host) {
    if (!c || T < 1 || N < 1 || (int64_t)T * N > INT32_MAX || !logl || !betas_host || !logz_host || !logw || !kept ||
        !n_kept_host || !ess_host)
        return SMCGW_ERR_INVALID;
    for (int t = 0; t < T; ++t)
        if (!(betas_host[t] >= 0.0 && betas_host[t] <= 1.0) || !std::isfinite(logz_host[t])) return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    const int n = T * N;
    char* s = (char*)sampler_scratch(c, 64 * sizeof(double) + 2 * (size_t)T * sizeof(double));
    double* hp = pinned(c);
    if (!s || !hp) return SMCGW_ERR_OOM;
    double* out = (double*)s;
    double* bz = out + 64;
    if (hipMemcpyAsync(bz, betas_host, T * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(bz + T, logz_host, T * sizeof(double), hipMemcpyHostToDevice, c->stream))
        return SMCGW_ERR_HIP;
    hipLaunchKernelGGL(recycle_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, logl, n, T, bz, logw);
    hipLaunchKernelGGL(recycle_select_kernel, dim3(1), dim3(SMC_THREADS), 0, c->stream, logw, n, seed, kept, out);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    if (hipMemcpyAsync(hp, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    *n_kept_host = (int64_t)hp[0];
    *ess_host = hp[1];
    return SMCGW_OK;
}

extern "C" int smcgw_ps_reweight_resample(smcgw_ctx* c, int T, int N, int D, const double* theta_pool,
                                          const double* logl_pool, const double* grad_pool, const double* betas_host,
                                          const double* logz_host, double alpha, uint64_t seed, uint64_t iteration,
                                          double* theta, double* logl, double* grad, int32_t* ancestors,
                                          double* beta_next_host, double* logz_next_host) {
    if (!c || T < 1 || N < 1 || D <= 0 || D > MAXDIM || (int64_t)T * N > INT32_MAX || !theta_pool || !logl_pool ||
        !betas_host || !logz_host || !theta || !logl || !ancestors || !beta_next_host || !logz_next_host ||
        ((grad_pool == nullptr) != (grad == nullptr)))
        return SMCGW_ERR_INVALID;
    if (!(alpha > 0.0 && alpha <= 1.0)) return SMCGW_ERR_INVALID;
    for (int t = 0; t < T; ++t)
        if (!(betas_host[t] >= 0.0 && betas_host[t] <= 1.0) || !std::isfinite(logz_host[t])) return SMCGW_ERR_INVALID;
    const double beta_prev = betas_host[T - 1];
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    const int n = T * N;
    const size_t off_bz = 64 * sizeof(double);
    const size_t off_lofs = off_bz + 2 * (size_t)T * sizeof(double);
    const size_t off_cum = off_lofs + (size_t)n * sizeof(double);
    const size_t off_x = off_cum + (size_t)n * sizeof(double);
    const size_t off_ll = off_x + (size_t)N * D * sizeof(double);
    const size_t off_g = off_ll + (size_t)N * sizeof(double);
    const size_t bytes = off_g + (size_t)N * D * sizeof(double);
    char* s = (char*)sampler_scratch(c, bytes);
    double* hp = pinned(c);
    if (!s || !hp) return SMCGW_ERR_OOM;
    double* out = (double*)s;
    double* bz = (double*)(s + off_bz);
    double* lofs = (double*)(s + off_lofs);
    double* cum = (double*)(s + off_cum);
    double* xo = (double*)(s + off_x);
    double* llo = (double*)(s + off_ll);
    double* go = (double*)(s + off_g);
    if (hipMemcpyAsync(bz, betas_host, T * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(bz + T, logz_host, T * sizeof(double), hipMemcpyHostToDevice, c->stream))
        return SMCGW_ERR_HIP;
    hipLaunchKernelGGL(pool_logmix_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, logl_pool, n, T, bz, lofs);
    hipLaunchKernelGGL(reweight_kernel, dim3(1), dim3(RW_THREADS), 0, c->stream, logl_pool, n, beta_prev, alpha,
                       (const double*)lofs, N, cum, out, (const double*)nullptr);
    const dim3 g((N + 255) / 256), b(256);
    hipLaunchKernelGGL(ancestors_kernel, g, b, 0, c->stream, cum, out, n, N, seed, iteration, ancestors,
                       (const double*)nullptr);
    hipLaunchKernelGGL(gather_kernel, g, b, 0, c->stream, ancestors, N, D, n, theta_pool, logl_pool, grad_pool,
                       (const int32_t*)nullptr, xo, llo, go, (int32_t*)nullptr, (const double*)out);
    hipLaunchKernelGGL(copy_back_kernel, g, b, 0, c->stream, N, D, xo, llo, go, (const int32_t*)nullptr, theta, logl,
                       grad, (int32_t*)nullptr, (const double*)out);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    if (hipMemcpyAsync(hp, out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return SMCGW_ERR_HIP;
    *beta_next_host = hp[0];
    *logz_next_host = hp[1];
    if (!(hp[0] > beta_prev) && beta_prev < 1.0) return SMCGW_ERR_STALL;
    return SMCGW_OK;
}
