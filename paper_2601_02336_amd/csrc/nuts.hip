// Persistent No-U-Turn kernel (arXiv:2601.02336, Sec. 4 and Sec. 5).
//
// One NUTS transition per particle: momentum r ~ N(0, M) with M^{-1} = L L^T,
// Hamiltonian H = -log p_t(x) + r^T M^{-1} r / 2 with p_t ~ L^beta pi (Sec. 3,
// Eq. 3), leapfrog steps (Eqs. 11-13) mapped back into the prior box by the
// reflective / periodic boundaries of Sec. 5, trajectory doubling in a random
// direction until the generalised U-turn criterion fires or the depth limit
// is reached (Hoffman & Gelman 2014; multinomial variant of Betancourt 2017,
// App. A): uniform progressive sampling inside each new subtree, biased
// progressive sampling when it is merged, divergence when H - H0 exceeds a
// threshold.
//
// Execution: each workgroup owns one particle slot at a time and pulls the
// next particle index from an atomic queue when its transition ends, so trees
// of uneven depth keep every slot busy until the queue drains.  Wavefront 0
// runs the tree logic with one coordinate per lane (lanes 0..D-1); for the
// gravitational-wave target every leaf's likelihood is evaluated by all
// wavefronts of the workgroup: prologue on two lanes, the bin loop split into
// interleaved blocks across the wavefronts, FP64 epilogue on wavefront 0.
// Random numbers come from Philox4x32-10 with counter (index, particle,
// iteration, purpose), so every decision can be replayed.
#include <algorithm>
#include <cstring>
#include <vector>

#include "binloop.h"
#include "coeffs.h"
#include "common.h"
#include "context.h"
#include "philox.h"

namespace smcgw {

struct NutsArgs {
    int P, D;
    double* theta;
    double* logl;
    double* grad;
    const double* chol;
    double step, beta, max_dh;
    int max_depth, uturn;
    uint64_t seed, iteration;
    const int32_t* md_per_p;
    int32_t* depth_out;
    int32_t* nlf_out;
    uint8_t* div_out;
    double* acc_out;
    const DevEvent* events;
    int n_events;
    const int32_t* ev_of_p;
    int* queue;
    const int32_t* order;   // start order of the particles (NULL: index order)
    int priority;           // raise wavefront priority with the tree depth
    int chol_pp;            // chol holds one [D][D] factor per particle
    const double* beta_dev; // beta from device memory (NULL: the value above)
    const double* state;    // independent runs' states (NULL: one run with the values above)
    int run_size;           // particles per run when state is set
};

constexpr int MAX_WAVES = 8;
// Wavefronts per SIMD the register budget is sized for (4: 128 VGPRs, 3: 168,
// 2: 256).
constexpr int NUTS_WAVES_PER_SIMD = 3;
constexpr int MAXD1 = SMCGW_MAX_DEPTH + 1;

// Per-detector terms of a leaf's epilogue (see leaf_finish).
enum { FD_LL = 0, FD_DLN, FD_GP, FD_T = FD_GP + 4, FD_RA, FD_DEC, FD_SIZE };

struct NutsShared {
    double L[MAXDIM * MAXDIM];
    double LT[MAXDIM * MAXDIM];                  // transpose of L
    double Minv[MAXDIM * MAXDIM];
    double vec[MAXDIM], red[2][MAXDIM];          // cross-lane exchange of wavefront 0
    double pred[MAXDIM];                         // cross-lane exchange of the auxiliary wavefront
    ExtAngles ang;                               // extrinsic transcendentals of the leaf in flight
    double utr[2][MAXD1][MAXDIM];                // U-turn dot-product terms of every level
    double cb[CB_SIZE];
    double mom[MAX_WAVES][MOM_SIZE];
    double fin_phase[4], fin_det[MAXDET][FD_SIZE], fin_g[NPAR + 1];   // epilogue terms of the leaf
    double th[NPAR];
    double left[5][MAXDIM], right[5][MAXDIM];   // x, r, g (grad log p_t), gl (grad logL), v = M^{-1} r
    double prop[2][MAXDIM], sprop[2][MAXDIM];    // x, gl
    double ck_rho[MAXD1][MAXDIM], ck_v[MAXD1][MAXDIM];   // U-turn checkpoints: prefix sum, first velocity
    double end_ll[2], end_lp[2];                 // logL, log p_t of left / right
    double plo[MAXDIM], phi[MAXDIM];             // prior / boundary description
    double pnorm[MAXDIM];                        // log normalising constant of each coordinate's prior
    int pbnd[MAXDIM], pkind[MAXDIM];
    int pidx[MAXDIM];                            // sampled coordinate -> source parameter
    double pfixed[NPAR];
    DevEvent ev;                                 // event of the current particle
    int p;
    int cmd;
};
static_assert(sizeof(DevEvent) % 8 == 0, "the event descriptor is copied in 8-byte words");

enum { CMD_EVAL = 0, CMD_DONE = 1 };

// log(e^a + e^b) = m + log(e^{a-m} + e^{b-m}) with m = max(a, b); the term of
// the larger argument is exp(0) = 1 exactly, so one exp suffices.
__device__ __forceinline__ double log_add_exp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = fmax(a, b);
    return m + log(1.0 + exp(fmin(a, b) - m));
}

// Cross-lane operations of wavefront 0 over the coordinate lanes 0..D-1, done
// through LDS: each lane writes its value, then every lane reads all MAXDIM
// entries (zero beyond D) and combines them in the same fixed order, so all
// lanes obtain bitwise identical results.  LDS accesses of one wavefront
// complete in issue order, so no barrier is needed between the write and the
// reads.

// Sum over the coordinate lanes of v.
__device__ __forceinline__ double dim_sum_at(double* red, int D, int lane, double v) {
    if (lane < MAXDIM) red[lane] = (lane < D) ? v : 0.0;
    __builtin_amdgcn_wave_barrier();
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < MAXDIM; ++m) s += red[m];
    __builtin_amdgcn_wave_barrier();
    return s;
}

__device__ __forceinline__ double dim_sum(NutsShared& S, int D, int lane, double v) {
    return dim_sum_at(S.red[0], D, lane, v);
}

// Two sums at once.
__device__ __forceinline__ void dim_sum2(NutsShared& S, int D, int lane, double a, double b, double& sa, double& sb) {
    if (lane < MAXDIM) {
        S.red[0][lane] = (lane < D) ? a : 0.0;
        S.red[1][lane] = (lane < D) ? b : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int m = 0; m < MAXDIM; ++m) { x += S.red[0][m]; y += S.red[1][m]; }
    __builtin_amdgcn_wave_barrier();
    sa = x;
    sb = y;
}

// (M^{-1} v) for this lane's coordinate.
__device__ __forceinline__ double minv_apply(NutsShared& S, int D, int lane, double v) {
    if (lane < MAXDIM) S.vec[lane] = (lane < D) ? v : 0.0;
    __builtin_amdgcn_wave_barrier();
    const int row = lane < D ? lane : 0;
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < MAXDIM; ++m) acc = fma(S.Minv[row * MAXDIM + m], S.vec[m], acc);
    __builtin_amdgcn_wave_barrier();
    return lane < D ? acc : 0.0;
}

// Normalised log prior of this lane's coordinate and its derivative.
__device__ __forceinline__ double log_prior_lane(const NutsShared& S, int k, double x, double& g) {
    g = 0.0;
    const double lo = S.plo[k], hi = S.phi[k];
    switch (S.pkind[k]) {
    case SMCGW_PRIOR_UNIFORM:
        return (x < lo || x > hi) ? -INFINITY : S.pnorm[k];
    case SMCGW_PRIOR_LOGUNIFORM:
        if (x < lo || x > hi) return -INFINITY;
        g = -1.0 / x;
        return -log(x) + S.pnorm[k];
    case SMCGW_PRIOR_GAUSSIAN: {
        const double r = (x - lo) / hi;
        g = -r / hi;
        return -0.5 * r * r + S.pnorm[k];
    }
    default:
        return 0.0;
    }
}

// The drift x += eps M^{-1} r of one leapfrog step inside the prior box
// (Sec. 4, Eq. 12; Sec. 5, Eqs. 15-18), one coordinate per lane of wavefront
// 0, v = M^{-1} r on entry.  The drift runs at velocity v until the first
// reflective coordinate k reaches its wall (the earliest over the lanes,
// lowest k on ties); there the momentum is reflected in the metric,
//   r_k -> r_k - 2 v_k / (M^{-1})_kk,   v -> v - 2 v_k / (M^{-1})_kk M^{-1} e_k,
// which reverses v_k and keeps the kinetic energy, and the drift goes on for
// the rest of the step.  With a diagonal metric this is the fold of the
// coordinate and the flip of its momentum component; for any metric the step
// stays reversible and volume preserving.  Periodic coordinates wrap at the
// end.  A step that meets no wall costs one ballot.
__device__ __forceinline__ void drift_lane(NutsShared& S, int D, int lane, double eps, double& x, double& r,
                                           double v) {
    const bool dl = lane < D;
    const int kk = dl ? lane : 0;
    const bool refl = dl && S.pbnd[kk] == SMCGW_BND_REFLECT;
    const double lo = S.plo[kk], hi = S.phi[kk];
    double rem = 1.0;   // fraction of the step left
    for (int it = 0; it < 64; ++it) {
        const double u = eps * v;
        double fr = 2.0, wall = 0.0;   // fraction of the step at which this coordinate meets its wall
        if (refl && u != 0.0) {
            wall = u > 0.0 ? hi : lo;
            fr = fmax((wall - x) / u, 0.0);
        }
        const bool hit = fr < rem;
        if (__ballot(hit) == 0) {
            if (dl) x = fma(rem * eps, v, x);
            break;
        }
        if (lane < MAXDIM) S.red[0][lane] = hit ? fr : 2.0;
        __builtin_amdgcn_wave_barrier();
        double fmin = 2.0;
        int kmin = 0;
#pragma unroll
        for (int m = 0; m < MAXDIM; ++m) {
            const double f = S.red[0][m];
            if (f < fmin) { fmin = f; kmin = m; }
        }
        __builtin_amdgcn_wave_barrier();
        if (dl) x = lane == kmin ? wall : fma(fmin * eps, v, x);
        rem -= fmin;
        const double vk = __shfl(v, kmin, 64);
        const double c = 2.0 * vk / S.Minv[kmin * MAXDIM + kmin];
        if (lane == kmin) r -= c;
        if (dl) v = fma(-c, S.Minv[kk * MAXDIM + kmin], v);
    }
    if (dl && S.pbnd[kk] == SMCGW_BND_PERIODIC) {
        const double w = hi - lo;
        for (int it = 0; it < 64 && (x < lo || x >= hi); ++it) x = (x >= hi) ? x - w : x + w;
    }
}

// Analytic likelihoods (one coordinate per lane of wavefront 0).
template <int TK>
__device__ __forceinline__ double analytic_loglike(NutsShared& S, const TargetDesc& t, int D, int lane, double x,
                                                   double& gl) {
    const bool dl = lane < D;
    if (TK == SMCGW_TARGET_GAUSS) {
        gl = dl ? -x : 0.0;
        return -0.5 * dim_sum(S, D, lane, x * x);
    } else if (TK == SMCGW_TARGET_GAUSS_X_GAUSS) {
        const double y = dl ? t.params[lane] : 0.0, s = dl ? t.params[D + lane] : 1.0;
        const double r = (y - x) / s;
        gl = dl ? r / s : 0.0;
        return dim_sum(S, D, lane, -0.5 * r * r - 0.5 * log(2.0 * PI * s * s));
    } else {
        const double m1 = dl ? t.params[lane] : 0.0, m2 = dl ? t.params[D + lane] : 0.0, sg = t.params[2 * D];
        double s1, s2;
        dim_sum2(S, D, lane, (x - m1) * (x - m1), (x - m2) * (x - m2), s1, s2);
        const double c = -0.5 * D * log(2.0 * PI * sg * sg);
        const double l1 = c - 0.5 * s1 / (sg * sg), l2 = c - 0.5 * s2 / (sg * sg);
        const double mx = fmax(l1, l2);
        const double w1 = exp(l1 - mx), w2 = exp(l2 - mx);
        gl = dl ? (w1 * (m1 - x) + w2 * (m2 - x)) / (sg * sg) / (w1 + w2) : 0.0;
        return mx + log(w1 + w2);
    }
}

// Tree state of the slot's current transition (LDS; wavefront 0 only).
//
// Leaf pipeline: once the likelihood of leaf k is known, `advance` completes
// its momentum and moves to leaf k+1 on the assumption that the tree goes on
// (the position of the next leaf does not depend on the multinomial sampling
// or the U-turn checks).  `bookkeep` then takes those decisions for leaf k on
// wavefront 0 while the other wavefronts already run leaf k+1's prologue; if
// the tree stops, that prologue is discarded.  Every quantity is the one the
// plain sequential algorithm computes.
struct NutsState {
    double x[MAXDIM], r[MAXDIM];                         // the leaf in flight: position, half-step momentum
    double rho[MAXDIM], srho[MAXDIM];                    // momentum sums of the tree / subtree
    double gl_new[MAXDIM];                               // likelihood gradient of the leaf in flight
    double rec[4][MAXDIM];                               // finished leaf: x, r, g (grad log p_t), gl
    double pgp[MAXDIM];                                  // prior gradient at the leaf in flight
    double plp;                                          // log prior at the leaf in flight
    double ul[2][2];                                     // log u and log(1 - u) of the leaf uniforms, by leaf index parity
    double dtab_u[MAXD1];                                // log of the merge uniform of each doubling
    int dtab_dir[MAXD1];                                 // direction of each doubling
    double h0, logw, sub_logw, uacc, acc_sum, eps, prop_ll, sprop_ll, ll_new, rec_ll, rec_lp;
    int first, stop, j, n, nleaves, depth, nlf, div, dir, md, inflight;
    uint32_t leafc;
    // the particle's run: temperature, Philox key and iteration, particle index within the run
    double beta;
    uint64_t seed, iter;
    uint32_t pid;
};

// Direction and merge uniform of doubling j (Philox stream DOUBLING).
__device__ __forceinline__ void doubling_draw(const NutsState& T, int j, int& dir, double& uacc) {
    double ud0, ud1;
    rng_uniform2(T.seed, (uint32_t)j, T.pid, T.iter, RNG_DOUBLING, ud0, ud1);
    dir = (ud0 < 0.5) ? -1 : 1;
    uacc = ud1;
}

// Start a transition of particle p (wavefront 0): momentum, H0, tree of one point.
__device__ __noinline__ void start_transition(NutsShared& S, NutsState& T, const NutsArgs& a, int p, int lane) {
    const int D = a.D;
    const bool dl = lane < D;
    const int kk = dl ? lane : 0;
    const double x = dl ? a.theta[(size_t)p * D + lane] : 0.0;
    const double gl = dl ? a.grad[(size_t)p * D + lane] : 0.0;
    const double ll = a.logl[p];
    double gp;
    const double lpr = dim_sum(S, D, lane, dl ? log_prior_lane(S, kk, x, gp) : 0.0);
    if (!dl) gp = 0.0;
    const double beta = T.beta;
    const double lp = beta * ll + lpr;
    const double g = beta * gl + gp;
    // r = L^{-T} z with z ~ N(0, I) from Box-Muller on Philox uniform pairs.
    double u0, u1;
    rng_uniform2(T.seed, (uint32_t)(lane >> 1), T.pid, T.iter, RNG_MOMENTUM, u0, u1);
    const double rad = sqrt(-2.0 * log(1.0 - u0));
    const double z = (lane & 1) ? rad * sin(2.0 * PI * u1) : rad * cos(2.0 * PI * u1);
    double accz = dl ? z : 0.0, r = 0.0;
    for (int i = D - 1; i >= 0; --i) {
        const double ri = __shfl(accz, i, 64) / S.L[i * MAXDIM + i];
        if (lane == i) r = ri;
        if (lane < i) accz = fma(-S.L[i * MAXDIM + lane], ri, accz);
    }
    if (!dl) r = 0.0;
    const double v = minv_apply(S, D, lane, r);
    const double h0 = -lp + 0.5 * dim_sum(S, D, lane, r * v);
    if (dl) {
        S.left[0][lane] = x; S.left[1][lane] = r; S.left[2][lane] = g; S.left[3][lane] = gl; S.left[4][lane] = v;
        S.right[0][lane] = x; S.right[1][lane] = r; S.right[2][lane] = g; S.right[3][lane] = gl; S.right[4][lane] = v;
        S.prop[0][lane] = x; S.prop[1][lane] = gl;
        T.rho[lane] = r;
        T.srho[lane] = 0.0;
    }
    const int md = a.md_per_p ? min(a.md_per_p[p], SMCGW_MAX_DEPTH) : a.max_depth;
    // every doubling's draws at once, one per lane (the merge uniform as its
    // log: the merge test u < W_sub / W becomes log u < log W_sub - log W)
    if (lane < md) {
        int dj;
        double uj;
        doubling_draw(T, lane, dj, uj);
        T.dtab_dir[lane] = dj;
        T.dtab_u[lane] = log(uj);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int dir0 = md > 0 ? T.dtab_dir[0] : 1;
    const double ua0 = md > 0 ? T.dtab_u[0] : 0.0;
    if (lane == 0) {
        S.end_ll[0] = S.end_ll[1] = ll;
        S.end_lp[0] = S.end_lp[1] = lp;
        T.prop_ll = ll;
        T.h0 = h0;
        T.logw = 0.0;
        T.acc_sum = 0.0;
        T.first = 1;
        T.stop = 0;
        T.j = 0;
        T.n = 0;
        T.nleaves = 1;
        T.sub_logw = -INFINITY;
        T.depth = 0;
        T.nlf = 0;
        T.div = 0;
        T.leafc = 0;
        T.md = md;
        T.dir = dir0;
        T.uacc = ua0;
    }
}

// Complete the leaf in flight (momentum full step with its gradient) into the
// record for `bookkeep`, then take the leapfrog step to the next leaf: the
// next one in the current subtree, else the first leaf of the next doubling
// from the tree end on its side.  Returns CMD_DONE when no leaf follows (the
// depth limit, or no doubling at all).
template <int TK>
__device__ __noinline__ int advance(NutsShared& S, NutsState& T, const NutsArgs& a, int lane) {
    const int D = a.D;
    const bool dl = lane < D;
    const int kk = dl ? lane : 0;
    // Every tree-state value the step may need is read up front, both tree ends
    // included, so the LDS round trips overlap instead of following the branches.
    const int first = T.first, n = T.n, nleaves = T.nleaves, j = T.j, md = T.md, dcur = T.dir;
    const double ll = T.ll_new, plp = T.plp, eps_prev = T.eps, beta = T.beta;
    const double gl = T.gl_new[kk], xf = T.x[kk], pg = T.pgp[kk], rh = T.r[kk];
    const double lx = S.left[0][kk], lr = S.left[1][kk], lg = S.left[2][kk];
    const double rx = S.right[0][kk], rr = S.right[1][kk], rg = S.right[2][kk];
    const int dnext = T.dtab_dir[min(j + 1, MAXD1 - 1)];
    double xs, rs, gs;   // start point of the next leapfrog step
    int dir;
    if (first) {
        if (md < 1) return CMD_DONE;
        xs = dl ? lx : 0.0;
        rs = dl ? lr : 0.0;
        gs = dl ? lg : 0.0;
        dir = dcur;
    } else {
        const double x = dl ? xf : 0.0;
        const double lp = beta * ll + plp;
        const double g = dl ? beta * gl + pg : 0.0;
        const double r = dl ? fma(0.5 * eps_prev, g, rh) : 0.0;
        if (dl) { T.rec[0][lane] = x; T.rec[1][lane] = r; T.rec[2][lane] = g; T.rec[3][lane] = gl; }
        if (lane == 0) { T.rec_ll = ll; T.rec_lp = lp; }
        if (n + 1 < nleaves) {
            xs = x; rs = r; gs = g;
            dir = dcur;
        } else if (j + 1 < md) {
            dir = dnext;
            if (dir == dcur) {
                xs = x; rs = r; gs = g;
            } else {
                xs = dl ? (dir > 0 ? rx : lx) : 0.0;
                rs = dl ? (dir > 0 ? rr : lr) : 0.0;
                gs = dl ? (dir > 0 ? rg : lg) : 0.0;
            }
        } else {
            return CMD_DONE;
        }
    }
    if (lane == 0) T.inflight = first ? 0 : T.nlf + 1;   // leaf index of the next leaf
    const double eps = dir * a.step;
    double r = dl ? fma(0.5 * eps, gs, rs) : 0.0;
    const double v = minv_apply(S, D, lane, r);
    double x = dl ? xs : 0.0;
    drift_lane(S, D, lane, eps, x, r, v);
    __builtin_amdgcn_wave_barrier();
    if (dl) { T.x[lane] = x; T.r[lane] = r; }
    if (lane == 0) T.eps = eps;
    if (TK == SMCGW_TARGET_GW) {
        if (lane < NPAR) S.th[lane] = S.pfixed[lane];
        __builtin_amdgcn_wave_barrier();
        if (dl) S.th[S.pidx[lane]] = x;
    }
    return CMD_EVAL;
}

// Work on the leaf in flight that `bookkeep` does not wait for (run on an
// otherwise idle wavefront): its amplitude entries of the coefficient block,
// the log prior and its gradient at its position (used by the next
// `advance`) and the uniform of its progressive sampling step (leaf index =
// leaves booked before it, the Philox LEAF counter).
template <int TK>
__device__ __noinline__ void aux_in_flight(const DevEvent* ev, NutsShared& S, NutsState& T, const NutsArgs& a, int p,
                                           int lane) {
    if (TK == SMCGW_TARGET_GW && lane == 0) prep_extrinsic_common(*ev, S.th, S.cb);
    const int D = a.D;
    const bool dl = lane < D;
    double gp;
    const double lpr = dim_sum_at(S.pred, D, lane, dl ? log_prior_lane(S, lane, T.x[lane], gp) : 0.0);
    if (dl) T.pgp[lane] = gp;
    const int idx = T.inflight;
    double ul0, ul1;
    rng_uniform2(T.seed, (uint32_t)idx, T.pid, T.iter, RNG_LEAF, ul0, ul1);
    // The progressive sampling test u < w / (W + w) is taken as log u + log W < log(1 - u) + log w: lanes 0
    // and 1 take the two logs at once.
    const double lu = log(lane == 0 ? ul0 : 1.0 - ul0);
    const double lu0 = __shfl(lu, 0, 64), lu1 = __shfl(lu, 1, 64);
    if (lane == 0) { T.plp = lpr; T.ul[idx & 1][0] = lu0; T.ul[idx & 1][1] = lu1; }
}

// Decisions for the finished leaf (wavefront 0): energy, divergence,
// progressive sampling, U-turn checks of the nodes it completes, the merge
// when its subtree is complete, and the set-up of the next doubling.  Sets
// T.stop when the transition ends here.
__device__ __noinline__ void bookkeep(NutsShared& S, NutsState& T, const NutsArgs& a, int p, int lane) {
    if (T.first) {
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) T.first = 0;
        return;
    }
    const int D = a.D;
    const bool dl = lane < D;
    const double x = dl ? T.rec[0][lane] : 0.0;
    const double r = dl ? T.rec[1][lane] : 0.0;
    const double g = dl ? T.rec[2][lane] : 0.0;
    const double gl = dl ? T.rec[3][lane] : 0.0;
    const double ll = T.rec_ll, lp = T.rec_lp;
    const double v = minv_apply(S, D, lane, r);   // velocity of this leaf: energy and every U-turn check
    const int j = T.j, n = T.n;
    const double h0 = T.h0;
    const double dh = -lp + 0.5 * dim_sum(S, D, lane, r * v) - h0;
    const bool finite = (dh == dh) && dh != INFINITY && dh != -INFINITY;
    double sub_logw = T.sub_logw;
    // Both exponentials of the leaf in one evaluation: lane 0 the log-add term e^{min - max} of the subtree
    // weight update, lane 1 the acceptance term e^{-dh}.
    const double lw = -dh;
    const double lmax = fmax(sub_logw, lw), lmin = fmin(sub_logw, lw);
    const double ee = exp(lane == 0 ? lmin - lmax : -dh);
    const double e_add = __shfl(ee, 0, 64), e_acc = __shfl(ee, 1, 64);
    double acc_sum = T.acc_sum + (finite ? fmin(1.0, e_acc) : 0.0);
    double srho = dl ? T.srho[lane] : 0.0;
    double sprop_ll = T.sprop_ll;
    uint32_t leafc = T.leafc;
    bool ok = true;
    int div = T.div;
    if (!finite || dh > a.max_dh) {
        div = 1;
        ok = false;
    } else {
        // this leaf opens the nodes of levels 1 .. ls (n a multiple of 2^l)
        const int ls = n == 0 ? j : min(j, __builtin_ctz((unsigned)n));
        if (dl)
            for (int l = 1; l <= ls; ++l) { S.ck_rho[l][lane] = srho; S.ck_v[l][lane] = v; }
        srho += r;
        // uniform drawn while this leaf was in flight: accept with probability w / (W + w)
        const double lu0 = T.ul[leafc & 1][0], lu1 = T.ul[leafc & 1][1];
        ++leafc;
        const double nlw = sub_logw == -INFINITY ? lw : lmax + log(1.0 + e_add);
        if (lu0 + sub_logw < lu1 + lw) {
            if (dl) { S.sprop[0][lane] = x; S.sprop[1][lane] = gl; }
            sprop_ll = ll;
        }
        sub_logw = nlw;
        if (a.uturn && j > 0 && ((n + 1) & 1) == 0) {
            // nodes completed by this leaf: level l covers leaves n+1-2^l .. n and
            // needs rho.v_first > 0 and rho.v_last > 0.  All levels at once: the
            // coordinate lanes write their terms, lane l sums level l in
            // coordinate order.
            // levels 1 .. lc complete here, lc = min(j, trailing zeros of n + 1)
            const int lc = min(j, __builtin_ctz((unsigned)(n + 1)));
            __builtin_amdgcn_wave_barrier();
            if (dl)
                for (int l = 1; l <= lc; ++l) {
                    const double nr = srho - S.ck_rho[l][lane];
                    S.utr[0][l][lane] = nr * S.ck_v[l][lane];
                    S.utr[1][l][lane] = nr * v;
                }
            __builtin_amdgcn_wave_barrier();
            bool fail = false;
            if (lane >= 1 && lane <= lc) {
                // all MAXDIM entries read at once, those beyond D masked to zero
                double sa = 0.0, sb = 0.0;
#pragma unroll
                for (int m = 0; m < MAXDIM; ++m) {
                    const bool in = m < D;
                    sa += in ? S.utr[0][lane][m] : 0.0;
                    sb += in ? S.utr[1][lane][m] : 0.0;
                }
                fail = !(sa > 0.0 && sb > 0.0);
            }
            if (__ballot(fail) != 0) ok = false;
            __builtin_amdgcn_wave_barrier();
        }
    }
    int depth = T.depth, jn = j, nn = n, dir = T.dir;
    double logw = T.logw, prop_ll = T.prop_ll, uacc = T.uacc;
    bool stop = false;
    if (!ok) {
        stop = true;
    } else if (n + 1 == T.nleaves) {
        depth = j + 1;
        __builtin_amdgcn_wave_barrier();
        if (uacc < sub_logw - logw) {   // uacc holds the log of the merge uniform
            if (dl) { S.prop[0][lane] = S.sprop[0][lane]; S.prop[1][lane] = S.sprop[1][lane]; }
            prop_ll = sprop_ll;
        }
        logw = log_add_exp(logw, sub_logw);
        const double rho = (dl ? T.rho[lane] : 0.0) + srho;
        const int side = dir > 0 ? 1 : 0;
        if (dl) {
            double (*E)[MAXDIM] = side ? S.right : S.left;
            E[0][lane] = x; E[1][lane] = r; E[2][lane] = g; E[3][lane] = gl; E[4][lane] = v;
            T.rho[lane] = rho;
        }
        if (lane == 0) { S.end_ll[side] = ll; S.end_lp[side] = lp; }
        __builtin_amdgcn_wave_barrier();
        if (a.uturn) {
            const double vl = dl ? S.left[4][lane] : 0.0, vr = dl ? S.right[4][lane] : 0.0;
            double sa, sb;
            dim_sum2(S, D, lane, rho * vl, rho * vr, sa, sb);
            stop = !(sa > 0.0 && sb > 0.0);
        }
        if (!stop && j + 1 >= T.md) stop = true;   // depth limit
        if (!stop) {
            // next doubling j + 1
            jn = j + 1;
            nn = 0;
            dir = T.dtab_dir[jn];
            uacc = T.dtab_u[jn];
            srho = 0.0;
            sub_logw = -INFINITY;
        }
    } else {
        nn = n + 1;
    }
    if (dl) T.srho[lane] = srho;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        T.acc_sum = acc_sum; T.sub_logw = sub_logw; T.sprop_ll = sprop_ll; T.leafc = leafc;
        T.div = div; T.stop = stop ? 1 : 0; T.depth = depth; T.j = jn; T.n = nn; T.logw = logw; T.prop_ll = prop_ll;
        T.dir = dir; T.uacc = uacc;
        T.nleaves = 1 << jn;
        T.nlf = T.nlf + 1;
    }
}

__device__ __noinline__ void write_outputs(NutsShared& S, NutsState& T, const NutsArgs& a, int p, int lane) {
    const int D = a.D;
    __builtin_amdgcn_wave_barrier();
    if (lane < D) {
        a.theta[(size_t)p * D + lane] = S.prop[0][lane];
        a.grad[(size_t)p * D + lane] = S.prop[1][lane];
    }
    if (lane == 0) {
        a.logl[p] = T.prop_ll;
        if (a.depth_out) a.depth_out[p] = T.depth;
        if (a.nlf_out) a.nlf_out[p] = T.nlf;
        if (a.div_out) a.div_out[p] = (uint8_t)T.div;
        if (a.acc_out) a.acc_out[p] = T.nlf > 0 ? T.acc_sum / T.nlf : 0.0;
    }
}

// Issue priority of the slot's wavefronts while doubling j runs: a tree that
// has reached 2^3, 2^4, 2^5 leaves outranks the shallower trees sharing its
// SIMDs, so the transitions that decide when the launch ends go first.
__device__ __forceinline__ void tree_priority(int j) {
    if (j >= 5) __builtin_amdgcn_s_setprio(3);
    else if (j == 4) __builtin_amdgcn_s_setprio(2);
    else if (j == 3) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Prologue pieces of one leaf (kept out of line so their registers do not
// constrain the bin loop).
__device__ __noinline__ void leaf_prep_intrinsic(const DevEvent* ev, NutsShared& S, int lane) {
    prep_intrinsic_n<1>(*ev, S.th, S.cb, lane, lane == 0);
}

// Extrinsic prologue on one wavefront: lanes 0-3 take one sin / cos each (in
// parallel), then lane d (d < MAXDET) builds detector d with its ra
// derivatives and lane MAXDET + d the dec derivatives of the same detector
// (one tangent per lane keeps each lane's chain short).  The amplitude is
// computed on the auxiliary wavefront.
__device__ __noinline__ void leaf_prep_extrinsic(const DevEvent* ev, NutsShared& S, int lane) {
    if (lane < ANG_COUNT) {
        double sn, cs;
        sincos(extrinsic_angle(*ev, S.th, lane), &sn, &cs);
        S.ang.sc[lane][0] = sn;
        S.ang.sc[lane][1] = cs;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < 2 * MAXDET) {
        const ExtAngles ang = S.ang;
        const int k = lane / MAXDET;
        prep_extrinsic_det_n<1>(*ev, S.th, ang, S.cb, lane - k * MAXDET, k, k == 0);
    }
}

// Epilogue of one leaf (wavefront 0): sum the wavefronts' moments, then logL
// and its gradient (the algebra of finish_particle) spread over lanes, so the
// chain is a few dependent steps instead of one lane's whole epilogue:
//   lanes 0..3        the phase part of d logL / d(Mc, q, chi1, chi2): a dot
//                     product of the basis moments with the prologue's Jacobian;
//   lanes 4..4+n_det  detector d's terms of logL, of d logL / d ln C_A, of the
//                     projection derivatives and of the arrival-time terms;
//   lanes 0..NPAR     one gradient component each, summing the detector terms in
//                     detector order; lane FIN_LL_LANE the log-likelihood.
constexpr int FIN_LL_LANE = NPAR;

template <int NDET, int WAVES>
__device__ __noinline__ void leaf_finish(const DevEvent* ev, NutsShared& S, NutsState& T, int D, int lane) {
    // wavefront totals of the moments, in wavefront order, into S.mom[0]
    if (lane < MOM_SIZE) {
        double s = S.mom[0][lane];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) s += S.mom[w][lane];
        S.mom[0][lane] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const double* c = S.cb;
    const double* m = S.mom[0];
    if (lane < 4) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NCOEF; ++b) s += c[CB_DC + 4 * b + lane] * m[MOM_G + b];
        S.fin_phase[lane] = TWO_PI * s;
    } else if (lane < 4 + NDET) {
        const int d = lane - 4;
        const double amp = c[CB_AMP];
        const double pr = c[CB_PR + d] * amp, pi = c[CB_PI + d] * amp;
        const double zr = m[MOM_ZR + d], zi = m[MOM_ZI + d], h = ev->hnorm[d];
        const double re = pr * zr - pi * zi;
        const double p2 = pr * pr + pi * pi;
        double* o = S.fin_det[d];
        o[FD_LL] = re - 0.5 * p2 * h;
        o[FD_DLN] = re - p2 * h;
        const double ar = zr - h * pr, ai = -zi - h * pi;   // dlogL / d(Re P', Im P')
#pragma unroll
        for (int k = 0; k < 4; ++k) o[FD_GP + k] = amp * (ar * c[CB_DPR + 4 * d + k] + ai * c[CB_DPI + 4 * d + k]);
        const double t = m[MOM_T + d];
        o[FD_T] = t;
        o[FD_RA] = TWO_PI * t * c[CB_DTAU + 2 * d];
        o[FD_DEC] = TWO_PI * t * c[CB_DTAU + 2 * d + 1];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // every lane sums the detector terms in detector order (broadcast reads, no
    // divergence) and keeps the component of its own index: gradient component
    // q on lane q, logL on FIN_LL_LANE
    double sum[FD_SIZE];
#pragma unroll
    for (int f = 0; f < FD_SIZE; ++f) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < NDET; ++d) s += S.fin_det[d][f];
        sum[f] = s;
    }
    const double g_mc = S.fin_phase[0] + sum[FD_DLN] * c[CB_DLNCA_MC];
    const double g_dl = sum[FD_DLN] * c[CB_DLNCA_DL];
    const double g_ra = sum[FD_RA] + sum[FD_GP + 2];
    const double g_dec = sum[FD_DEC] + sum[FD_GP + 3];
    const double g_tc = TWO_PI * sum[FD_T];
    const double ll = -0.5 * ev->dd + sum[FD_LL];
    double v = ll;
    v = lane == P_MC ? g_mc : v;
    v = lane == P_Q ? S.fin_phase[1] : v;
    v = lane == P_CHI1 ? S.fin_phase[2] : v;
    v = lane == P_CHI2 ? S.fin_phase[3] : v;
    v = lane == P_DL ? g_dl : v;
    v = lane == P_IOTA ? sum[FD_GP + 0] : v;
    v = lane == P_PSI ? sum[FD_GP + 1] : v;
    v = lane == P_RA ? g_ra : v;
    v = lane == P_DEC ? g_dec : v;
    v = lane == P_TC ? g_tc : v;
    v = lane == P_PHIC ? -m[MOM_G + 0] : v;
    if (lane <= FIN_LL_LANE) S.fin_g[lane] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < D) T.gl_new[lane] = S.fin_g[S.pidx[lane]];
    if (lane == 0) T.ll_new = ll;
}

// The Cholesky factor L of M^{-1} ([D][D], row-major) into LDS, zero-padded
// to MAXDIM; derive_metric then forms M^{-1} = L L^T and L^T from it (every
// thread a share of the entries; the caller's barrier orders them).
__device__ __forceinline__ void load_factor(NutsShared& S, const double* chol, int D, int tid) {
    for (int i = tid; i < MAXDIM * MAXDIM; i += blockDim.x) {
        const int r = i / MAXDIM, c = i % MAXDIM;
        S.L[i] = (r < D && c < D) ? chol[r * D + c] : 0.0;
    }
}

__device__ __noinline__ void derive_metric(NutsShared& S, int D, int tid) {
    for (int i = tid; i < MAXDIM * MAXDIM; i += blockDim.x) {
        const int r = i / MAXDIM, c = i % MAXDIM;
        double s = 0.0;
        for (int m = 0; m < D; ++m) s = fma(S.L[r * MAXDIM + m], S.L[c * MAXDIM + m], s);
        S.Minv[i] = s;
        S.LT[i] = S.L[c * MAXDIM + r];
    }
}

// Particle queues of a launch without a work hint.  The particles are dealt
// in stripes of STRIPE neighbouring indices, stripe g to queue g mod N_QUEUES,
// one queue per XCD: a slot takes the next particle of its own XCD's queue
// and, once that is drained, of the others in turn.  Neighbouring particles,
// whose inputs and outputs share cache lines, then pass through one XCD's L2
// instead of leaving partly written lines in several.  A queue is drained for
// good once a fetch runs past P (its particle indices only grow), so every
// slot leaves after at most N_QUEUES empty fetches.
constexpr int N_QUEUES = 8;
constexpr int STRIPE = 16;

__device__ __forceinline__ int striped_particle(int queue, int k) {
    return ((k / STRIPE) * N_QUEUES + queue) * STRIPE + k % STRIPE;
}

template <int NDET, int PREC, int TK, int WAVES>
__global__ __launch_bounds__(WAVES * 64, (WAVES == 1 ? 2 : NUTS_WAVES_PER_SIMD)) void nuts_kernel(NutsArgs a, PriorDesc pri, ParamMap pm,
                                                                             TargetDesc tgt) {
    __shared__ NutsShared S;
    __shared__ NutsState T;
    __shared__ NutsArgs A;   // the arguments as the out-of-line tree steps read them (LDS, not a stack copy)
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int D = a.D;

    // one factor for the whole launch; per-run factors are loaded when a particle's run changes
    const bool run_factor = !a.chol_pp && a.state;
    if (!a.chol_pp && !a.state) load_factor(S, a.chol, D, tid);
    if (tid == 0) {
        A = a;
        if (a.beta_dev) A.beta = *a.beta_dev;
        // once per launch on one lane: kept rolled, so the logs are not copied out per coordinate
#pragma unroll 1
        for (int k = 0; k < MAXDIM; ++k) {
            S.plo[k] = pri.lo[k]; S.phi[k] = pri.hi[k]; S.pbnd[k] = pri.bnd[k]; S.pkind[k] = pri.kind[k];
            S.pidx[k] = pm.idx[k];
            const double lo = pri.lo[k], hi = pri.hi[k];
            S.pnorm[k] = k >= D ? 0.0
                       : pri.kind[k] == SMCGW_PRIOR_UNIFORM ? -log(hi - lo)
                       : pri.kind[k] == SMCGW_PRIOR_LOGUNIFORM ? -log(log(hi / lo))
                       : pri.kind[k] == SMCGW_PRIOR_GAUSSIAN ? -0.5 * log(2.0 * PI * hi * hi) : 0.0;
        }
        for (int k = 0; k < NPAR; ++k) S.pfixed[k] = pm.fixed[k];
    }
    __syncthreads();
    if (!a.chol_pp && !a.state) {
        derive_metric(S, D, tid);
        __syncthreads();
    }

    int ev_cached = -1;    // event whose descriptor S.ev holds
    int run_cached = -1;   // run whose factor S.L holds (per-run factors)
    // this slot's XCD (hardware register XCC_ID) and the queues it has seen drained
    const int home = (int)(__builtin_amdgcn_s_getreg((31 << 11) | 20) & (N_QUEUES - 1));
    unsigned drained = 0;
    for (;;) {
        if (tid == 0) {
            if (a.order) {
                const int q = __hip_atomic_fetch_add(a.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                S.p = q < a.P ? a.order[q] : a.P;
            } else {
                int next = a.P;
                for (int t = 0; t < N_QUEUES; ++t) {
                    const int x = (home + t) & (N_QUEUES - 1);
                    if (drained & (1u << x)) continue;
                    const int k = __hip_atomic_fetch_add(a.queue + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int cand = striped_particle(x, k);
                    if (cand < a.P) {
                        next = cand;
                        break;
                    }
                    drained |= 1u << x;
                }
                S.p = next;
            }
        }
        __syncthreads();
        const int p = __builtin_amdgcn_readfirstlane(S.p);
        if (p >= a.P) break;
        // the particle's run (uniform over the workgroup)
        const int run = a.state ? p / a.run_size : 0;
        if (a.state && a.state[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_DONE] != 0.0) {
            __syncthreads();   // every thread has read S.p before thread 0 pulls the next particle
            continue;          // a finished run's particles are left untouched
        }
        if (tid == 0) {
            if (a.state) {
                const double* st = a.state + (size_t)run * SMCGW_STATE_SIZE;
                T.beta = st[SMCGW_ST_BETA];
                T.iter = (uint64_t)st[SMCGW_ST_ITER];
                T.seed = a.seed + (uint64_t)run;
                T.pid = (uint32_t)(p - run * a.run_size);
            } else {
                T.beta = A.beta;
                T.iter = a.iteration;
                T.seed = a.seed;
                T.pid = (uint32_t)p;
            }
        }
        if (run_factor && run != run_cached) {   // the previous transition's readers are past a barrier
            load_factor(S, a.chol + (size_t)run * D * D, D, tid);
            __syncthreads();
            derive_metric(S, D, tid);
            run_cached = run;
        }
        __syncthreads();   // T's run values and the factor are visible to every wavefront
        // The particle's event descriptor is copied into LDS (all threads, ordered
        // before its first use by the barrier that follows advance), so the
        // leaf's serial phases read it without a round trip to the L2.
        const DevEvent* ev = &S.ev;
        if (TK == SMCGW_TARGET_GW) {
            const int e = __builtin_amdgcn_readfirstlane(event_index(a.ev_of_p, p, a.n_events));
            if (e != ev_cached) {   // uniform over the workgroup
                const unsigned long long* src = (const unsigned long long*)(a.events + e);
                unsigned long long* dst = (unsigned long long*)&S.ev;
                for (int i = tid; i < (int)(sizeof(DevEvent) / 8); i += blockDim.x) dst[i] = src[i];
                ev_cached = e;
            }
        }
        if (a.chol_pp) {   // the particle's own metric (the previous transition's readers are past a barrier)
            load_factor(S, a.chol + (size_t)p * D * D, D, tid);
            __syncthreads();
            derive_metric(S, D, tid);
            __syncthreads();
        }
        if (wave == 0) start_transition(S, T, A, p, lane);

        // Wavefronts of the leaf prologue: intrinsic and extrinsic parts on
        // wavefronts 1 and 2 while wavefront 0 books the previous leaf (both on
        // wavefront 1 when the slot has two).
        constexpr int W_INTR = WAVES > 1 ? 1 : 0;
        constexpr int W_EXTR = WAVES > 2 ? 2 : W_INTR;
        constexpr int W_AUX = WAVES > 3 ? 3 : 0;
        for (;;) {
            if (wave == 0) {
                const int cmd = advance<TK>(S, T, A, lane);
                if (lane == 0) S.cmd = cmd;
            }
            __syncthreads();
            const int cmd = __builtin_amdgcn_readfirstlane(S.cmd);
            if (wave == 0) bookkeep(S, T, A, p, lane);
            if (wave == W_AUX && cmd == CMD_EVAL) aux_in_flight<TK>(ev, S, T, A, p, lane);
            if (TK == SMCGW_TARGET_GW && cmd == CMD_EVAL) {
                if (wave == W_INTR && lane < 4) leaf_prep_intrinsic(ev, S, lane);
                if (wave == W_EXTR && lane < 8) leaf_prep_extrinsic(ev, S, lane);
            }
            __syncthreads();
            if (cmd == CMD_DONE || __builtin_amdgcn_readfirstlane(T.stop)) break;
            if (a.priority) tree_priority(__builtin_amdgcn_readfirstlane(T.j));

            if (TK == SMCGW_TARGET_GW) {
                {
                    const BinCoef k = load_coef(S.cb);
                    if (PREC == SMCGW_MIXED)
                        bins_mixed_wave<NDET>(ev, k, wave, WAVES, S.mom[wave]);
                    else
                        bins_fp64_wave<NDET>(ev, k, wave, WAVES, S.mom[wave]);
                }
                __syncthreads();
                if (wave == 0) leaf_finish<NDET, WAVES>(ev, S, T, D, lane);
            } else if (wave == 0) {
                double gl;
                const double ll = analytic_loglike<TK>(S, tgt, D, lane, lane < D ? T.x[lane] : 0.0, gl);
                if (lane < D) T.gl_new[lane] = gl;
                if (lane == 0) T.ll_new = ll;
            }
        }
        if (a.priority) __builtin_amdgcn_s_setprio(0);
        if (wave == 0) write_outputs(S, T, A, p, lane);
        __syncthreads();
    }
}

// Start order from a work hint: particles sorted by descending bucket
// floor(log2(hint)) + 1 (0 for hint <= 0), stable in the particle index.
// One workgroup; thread t owns the contiguous index chunk [t*ch, (t+1)*ch).
// Four wavefronts (one per SIMD) fit in the registers of a single NUTS slot,
// so the kernel starts as soon as one slot of a co-running launch frees.
constexpr int ORDER_THREADS = 256;
constexpr int ORDER_BUCKETS = 16;

__device__ __forceinline__ int hint_bucket(int32_t h) { return h <= 0 ? 0 : min(ORDER_BUCKETS - 1, 32 - __clz(h)); }

__global__ __launch_bounds__(ORDER_THREADS) void order_kernel(const int32_t* __restrict__ hint, int P,
                                                              int32_t* __restrict__ order) {
    __shared__ int wsum[ORDER_THREADS / 64][ORDER_BUCKETS];
    __shared__ int base[ORDER_THREADS / 64][ORDER_BUCKETS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ch = (P + ORDER_THREADS - 1) / ORDER_THREADS;
    const int lo = min(P, tid * ch), hi = min(P, lo + ch);
    int cnt[ORDER_BUCKETS];
#pragma unroll
    for (int k = 0; k < ORDER_BUCKETS; ++k) cnt[k] = 0;
    for (int i = lo; i < hi; ++i) {
        const int b = hint_bucket(hint[i]);
#pragma unroll
        for (int k = 0; k < ORDER_BUCKETS; ++k) cnt[k] += (b == k);
    }
    // exclusive offsets of this thread inside each bucket: lanes, then wavefronts
    int off[ORDER_BUCKETS];
#pragma unroll
    for (int k = 0; k < ORDER_BUCKETS; ++k) {
        int inc = cnt[k];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        off[k] = inc - cnt[k];
        if (lane == 63) wsum[wave][k] = inc;
    }
    __syncthreads();
    if (tid == 0) {   // bucket starts in descending bucket order, then wavefront order inside a bucket
        int start = 0;
        for (int k = ORDER_BUCKETS - 1; k >= 0; --k) {
            for (int w = 0; w < ORDER_THREADS / 64; ++w) {
                base[w][k] = start;
                start += wsum[w][k];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ORDER_BUCKETS; ++k) off[k] += base[wave][k];
    for (int i = lo; i < hi; ++i) {
        const int b = hint_bucket(hint[i]);
        int pos = 0;
#pragma unroll
        for (int k = 0; k < ORDER_BUCKETS; ++k) {
            if (b == k) { pos = off[k]; ++off[k]; }
        }
        order[pos] = i;
    }
}

__global__ void zero_queues_kernel(int* q) {
    if (threadIdx.x < N_QUEUES) q[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ lockstep sweeps
// The plain comparison form of the transition: the same tree, random streams
// and decisions as nuts_kernel, but advanced one leapfrog step per particle per
// sweep.  A sweep is one launch of nuts_sweep_kernel (one wavefront per
// particle: the tree step that books the leaf just evaluated and moves to the
// next one) and one batched likelihood launch over the particles still
// building their tree; the tree state waits in global memory between sweeps.

// A particle's tree between sweeps.
struct SweepState {
    NutsState T;
    double left[5][MAXDIM], right[5][MAXDIM];
    double prop[2][MAXDIM], sprop[2][MAXDIM];
    double ck_rho[MAXD1][MAXDIM], ck_v[MAXD1][MAXDIM];
    double end_ll[2], end_lp[2];
    int phase;
    int pad;
};
static_assert(sizeof(NutsState) % 8 == 0 && sizeof(SweepState) % 8 == 0, "copied in 8-byte words");
enum { SW_START = 0, SW_RUN = 1, SW_DONE = 2 };

__device__ __forceinline__ void copy_words(void* dst, const void* src, size_t bytes, int lane) {
    unsigned long long* d = (unsigned long long*)dst;
    const unsigned long long* s = (const unsigned long long*)src;
    for (size_t i = lane; i < bytes / 8; i += 64) d[i] = s[i];
}

// Tree state between LDS and the particle's record.
__device__ __forceinline__ void sweep_save(SweepState& G, const NutsShared& S, const NutsState& T, int lane) {
    copy_words(&G.T, &T, sizeof(NutsState), lane);
    copy_words(G.left, S.left, sizeof(S.left), lane);
    copy_words(G.right, S.right, sizeof(S.right), lane);
    copy_words(G.prop, S.prop, sizeof(S.prop), lane);
    copy_words(G.sprop, S.sprop, sizeof(S.sprop), lane);
    copy_words(G.ck_rho, S.ck_rho, sizeof(S.ck_rho), lane);
    copy_words(G.ck_v, S.ck_v, sizeof(S.ck_v), lane);
    copy_words(G.end_ll, S.end_ll, sizeof(S.end_ll), lane);
    copy_words(G.end_lp, S.end_lp, sizeof(S.end_lp), lane);
}

__device__ __forceinline__ void sweep_load(const SweepState& G, NutsShared& S, NutsState& T, int lane) {
    copy_words(&T, &G.T, sizeof(NutsState), lane);
    copy_words(S.left, G.left, sizeof(S.left), lane);
    copy_words(S.right, G.right, sizeof(S.right), lane);
    copy_words(S.prop, G.prop, sizeof(S.prop), lane);
    copy_words(S.sprop, G.sprop, sizeof(S.sprop), lane);
    copy_words(S.ck_rho, G.ck_rho, sizeof(S.ck_rho), lane);
    copy_words(S.ck_v, G.ck_v, sizeof(S.ck_v), lane);
    copy_words(S.end_ll, G.end_ll, sizeof(S.end_ll), lane);
    copy_words(S.end_lp, G.end_lp, sizeof(S.end_lp), lane);
}

// Every particle starts its transition; the next-position rows hold the
// current points until the first sweep replaces them.
__global__ __launch_bounds__(256) void sweep_init_kernel(SweepState* __restrict__ st, uint8_t* __restrict__ active,
                                                         const double* __restrict__ theta, double* __restrict__ x_next,
                                                         int P, int D) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    st[p].phase = SW_START;
    active[p] = 1;
    for (int k = 0; k < D; ++k) x_next[(size_t)p * D + k] = theta[(size_t)p * D + k];
}

// One tree step of particle p = blockIdx.x: the transition's start on the
// first sweep, else the booking of the leaf whose likelihood ll_in / gl_in
// the batched likelihood has just computed; then either the next leaf's
// position (x_next, active = 1) or the transition's outputs (active = 0).
// The tree steps are out-of-line functions shared with nuts_kernel, and a
// function's register budget is the loosest of its callers': the occupancy
// bound here matches nuts_kernel's so the shared steps keep its budget.
__global__ __launch_bounds__(64, NUTS_WAVES_PER_SIMD) void nuts_sweep_kernel(NutsArgs a, PriorDesc pri, ParamMap pm,
                                                        SweepState* __restrict__ st,
                                                        const double* __restrict__ ll_in,
                                                        const double* __restrict__ gl_in,
                                                        double* __restrict__ x_next, uint8_t* __restrict__ active) {
    __shared__ NutsShared S;
    __shared__ NutsState T;
    __shared__ NutsArgs A;
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const int D = a.D;
    SweepState& G = st[p];
    const int phase = __builtin_amdgcn_readfirstlane(G.phase);
    if (phase == SW_DONE) return;
    const int run = a.state ? p / a.run_size : 0;
    if (a.state && a.state[(size_t)run * SMCGW_STATE_SIZE + SMCGW_ST_DONE] != 0.0) {
        if (lane == 0) { G.phase = SW_DONE; active[p] = 0; }   // a finished run's particles are left untouched
        return;
    }
    const double* chol = a.chol_pp ? a.chol + (size_t)p * D * D : a.state ? a.chol + (size_t)run * D * D : a.chol;
    load_factor(S, chol, D, lane);
    if (lane == 0) {
        A = a;
        if (a.beta_dev) A.beta = *a.beta_dev;
#pragma unroll 1
        for (int k = 0; k < MAXDIM; ++k) {
            S.plo[k] = pri.lo[k]; S.phi[k] = pri.hi[k]; S.pbnd[k] = pri.bnd[k]; S.pkind[k] = pri.kind[k];
            S.pidx[k] = pm.idx[k];
            const double lo = pri.lo[k], hi = pri.hi[k];
            S.pnorm[k] = k >= D ? 0.0
                       : pri.kind[k] == SMCGW_PRIOR_UNIFORM ? -log(hi - lo)
                       : pri.kind[k] == SMCGW_PRIOR_LOGUNIFORM ? -log(log(hi / lo))
                       : pri.kind[k] == SMCGW_PRIOR_GAUSSIAN ? -0.5 * log(2.0 * PI * hi * hi) : 0.0;
        }
        for (int k = 0; k < NPAR; ++k) S.pfixed[k] = pm.fixed[k];
    }
    __syncthreads();
    derive_metric(S, D, lane);
    if (phase == SW_START) {
        if (lane == 0) {
            if (a.state) {
                const double* rs = a.state + (size_t)run * SMCGW_STATE_SIZE;
                T.beta = rs[SMCGW_ST_BETA];
                T.iter = (uint64_t)rs[SMCGW_ST_ITER];
                T.seed = a.seed + (uint64_t)run;
                T.pid = (uint32_t)(p - run * a.run_size);
            } else {
                T.beta = A.beta;
                T.iter = a.iteration;
                T.seed = a.seed;
                T.pid = (uint32_t)p;
            }
        }
        __syncthreads();
        start_transition(S, T, A, p, lane);
    } else {
        sweep_load(G, S, T, lane);
        __syncthreads();
        if (lane < D) T.gl_new[lane] = gl_in[(size_t)p * D + lane];
        if (lane == 0) T.ll_new = ll_in[p];
    }
    __syncthreads();
    const int cmd = advance<SMCGW_TARGET_GW>(S, T, A, lane);
    bookkeep(S, T, A, p, lane);
    __syncthreads();
    if (cmd == CMD_DONE || __builtin_amdgcn_readfirstlane(T.stop)) {
        write_outputs(S, T, A, p, lane);
        if (lane == 0) { G.phase = SW_DONE; active[p] = 0; }
        return;
    }
    aux_in_flight<SMCGW_TARGET_GW>(a.events + event_index(a.ev_of_p, p, a.n_events), S, T, A, p, lane);
    __syncthreads();
    if (lane < D) x_next[(size_t)p * D + lane] = T.x[lane];
    sweep_save(G, S, T, lane);
    if (lane == 0) { G.phase = SW_RUN; active[p] = 1; }
}

// Particles still building their tree (one workgroup).
__global__ __launch_bounds__(256) void sweep_count_kernel(const uint8_t* __restrict__ active, int P,
                                                          int* __restrict__ count) {
    __shared__ int part[256];
    int n = 0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) n += active[i];
    part[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int t = 0; t < 256; ++t) s += part[t];
        *count = s;
    }
}

}  // namespace smcgw

using namespace smcgw;

namespace {

template <class K>
int launch_persistent(smcgw_ctx* c, K kernel, int block, const NutsArgs& a, const PriorDesc& pri, const ParamMap& pm,
                      const TargetDesc& t) {
    auto it = c->resident.find((const void*)kernel);
    if (it == c->resident.end()) {
        int dev_cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
            return SMCGW_ERR_HIP;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        it = c->resident.emplace((const void*)kernel, std::make_pair(dev_cus, per_cu)).first;
    }
    int per_cu = it->second.second;
    if (c->nuts_slots_per_cu > 0) per_cu = std::min(per_cu, c->nuts_slots_per_cu);
    const int grid = std::max(1, std::min(a.P, it->second.first * per_cu));
    hipLaunchKernelGGL(zero_queues_kernel, dim3(1), dim3(N_QUEUES), 0, c->stream, a.queue);
    {
        TimedLaunch tl(c, SMCGW_KERNEL_NUTS);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, c->stream, a, pri, pm, t);
    }
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

template <int NDET, int W>
int launch_gw_w(smcgw_ctx* c, int precision, const NutsArgs& a, const PriorDesc& pri, const ParamMap& pm,
                const TargetDesc& t) {
    if (precision == SMCGW_MIXED)
        return launch_persistent(c, nuts_kernel<NDET, SMCGW_MIXED, SMCGW_TARGET_GW, W>, W * 64, a, pri, pm, t);
    return launch_persistent(c, nuts_kernel<NDET, SMCGW_PLAIN_FP64, SMCGW_TARGET_GW, W>, W * 64, a, pri, pm, t);
}

// Slot width when none is set: the bin loop splits an event into blocks of
// TABLE_PAD bins, one wavefront per block, so when no event of the context has
// more than two blocks (relative-binning events) wider slots add wavefronts
// that hold only prologue roles; two-wavefront slots give every compute unit
// twice the particles in flight instead.  Otherwise four.
int default_nuts_waves(const smcgw_ctx* c) {
    int blocks = 0;
    for (const DevEvent& e : c->events) blocks = std::max(blocks, e.n_pad / TABLE_PAD);
    return blocks <= 2 ? 2 : 4;
}

template <int NDET>
int launch_gw(smcgw_ctx* c, int precision, const NutsArgs& a, const PriorDesc& pri, const ParamMap& pm,
              const TargetDesc& t) {
    switch (c->nuts_waves ? c->nuts_waves : default_nuts_waves(c)) {
    case 2: return launch_gw_w<NDET, 2>(c, precision, a, pri, pm, t);
    case 6: return launch_gw_w<NDET, 6>(c, precision, a, pri, pm, t);
    case 8: return launch_gw_w<NDET, 8>(c, precision, a, pri, pm, t);
    default: return launch_gw_w<NDET, 4>(c, precision, a, pri, pm, t);
    }
}

}  // namespace

// The work-queue counter and the start-order buffer for P particles.
int smcgw::nuts_reserve(smcgw_ctx* c, int P, bool hint) {
    if (!c->d_queue && hipMalloc(&c->d_queue, 256) != hipSuccess) return SMCGW_ERR_OOM;
    if (hint && P > c->order_cap) {
        (void)hipFree(c->d_order);
        c->d_order = nullptr;
        c->order_cap = 0;
        if (hipMalloc(&c->d_order, (size_t)P * sizeof(int32_t)) != hipSuccess) return SMCGW_ERR_OOM;
        c->order_cap = P;
    }
    return SMCGW_OK;
}

extern "C" int smcgw_nuts_step(smcgw_ctx* c, int P, int D, double* theta, double* logl, double* grad,
                               const double* chol, const smcgw_nuts_params* prm,
                               const int32_t* max_depth_per_particle, const int32_t* work_hint, int precision,
                               int32_t* depth, int32_t* n_leapfrog, uint8_t* divergent, double* accept_stat) {
    if (!c || !prm || P < 0 || D <= 0 || D > MAXDIM || (P > 0 && (!theta || !logl || !grad || !chol)))
        return SMCGW_ERR_INVALID;
    if (precision != SMCGW_PLAIN_FP64 && precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (prm->max_depth < 0 || prm->max_depth > SMCGW_MAX_DEPTH || !(prm->step > 0.0) ||
        (!prm->beta_device && !(prm->beta >= 0.0)) ||
        !(prm->max_delta_h > 0.0) || (prm->chol_per_particle != 0 && prm->chol_per_particle != 1) ||
        prm->reserved != 0 || prm->reserved2 != 0)
        return SMCGW_ERR_INVALID;
    if (prm->state_device && (prm->run_size < 1 || P % prm->run_size != 0 || P / prm->run_size > SMCGW_MAX_RUNS))
        return SMCGW_ERR_INVALID;
    if (!c->prior_set || c->prior.dim != D) return SMCGW_ERR_NOT_INIT;
    const int kind = c->target.kind;
    if (kind == SMCGW_TARGET_GW) {
        if (c->events.empty() || c->pmap.dim != D) return SMCGW_ERR_NOT_INIT;
    } else if (c->target.dim != D) {
        return SMCGW_ERR_NOT_INIT;
    }
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    if (nuts_reserve(c, P, work_hint != nullptr) != SMCGW_OK) return SMCGW_ERR_OOM;
    if (work_hint) {
        hipLaunchKernelGGL(order_kernel, dim3(1), dim3(ORDER_THREADS), 0, c->stream, work_hint, P, c->d_order);
        if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    }
    NutsArgs a;
    a.P = P;
    a.D = D;
    a.theta = theta;
    a.logl = logl;
    a.grad = grad;
    a.chol = chol;
    a.step = prm->step;
    a.beta = prm->beta;
    a.max_dh = prm->max_delta_h;
    a.max_depth = prm->max_depth;
    a.uturn = prm->uturn ? 1 : 0;
    a.seed = prm->seed;
    a.iteration = prm->iteration;
    a.md_per_p = max_depth_per_particle;
    a.depth_out = depth;
    a.nlf_out = n_leapfrog;
    a.div_out = divergent;
    a.acc_out = accept_stat;
    a.events = c->d_events;
    a.n_events = (int)c->events.size();
    a.ev_of_p = c->ev_of_p;
    a.queue = (int*)c->d_queue;
    a.order = work_hint ? c->d_order : nullptr;
    a.priority = c->nuts_priority;
    a.chol_pp = prm->chol_per_particle;
    a.beta_dev = prm->beta_device;
    a.state = prm->state_device;
    a.run_size = prm->state_device ? prm->run_size : P;
    const TargetDesc t = c->target;
    switch (kind) {
    case SMCGW_TARGET_GW:
        switch (c->n_det) {
        case 1: return launch_gw<1>(c, precision, a, c->prior, c->pmap, t);
        case 2: return launch_gw<2>(c, precision, a, c->prior, c->pmap, t);
        case 3: return launch_gw<3>(c, precision, a, c->prior, c->pmap, t);
        case 4: return launch_gw<4>(c, precision, a, c->prior, c->pmap, t);
        default: return SMCGW_ERR_SHAPE;
        }
    case SMCGW_TARGET_GAUSS:
        return launch_persistent(c, nuts_kernel<1, SMCGW_PLAIN_FP64, SMCGW_TARGET_GAUSS, 1>, 64, a, c->prior,
                                 c->pmap, t);
    case SMCGW_TARGET_GAUSS_X_GAUSS:
        return launch_persistent(c, nuts_kernel<1, SMCGW_PLAIN_FP64, SMCGW_TARGET_GAUSS_X_GAUSS, 1>, 64, a, c->prior,
                                 c->pmap, t);
    case SMCGW_TARGET_BIMODAL:
        return launch_persistent(c, nuts_kernel<1, SMCGW_PLAIN_FP64, SMCGW_TARGET_BIMODAL, 1>, 64, a, c->prior,
                                 c->pmap, t);
    default:
        return SMCGW_ERR_INVALID;
    }
}

extern "C" int smcgw_autotune_nuts(smcgw_ctx* c, int P, int D, const double* theta, const double* logl,
                                   const double* grad, const double* chol, const smcgw_nuts_params* prm, int precision,
                                   int trials, int* best_waves, double* times_ms) {
    if (!c || !prm || P < 1 || D <= 0 || D > MAXDIM || !theta || !logl || !grad || !chol || trials < 1 || trials > 16)
        return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    const size_t nx = (size_t)P * D * sizeof(double), nl = (size_t)P * sizeof(double);
    double *x = nullptr, *l = nullptr, *g = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SMCGW_OK;
    if (hipMalloc(&x, nx) != hipSuccess || hipMalloc(&l, nl) != hipSuccess || hipMalloc(&g, nx) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = SMCGW_ERR_OOM;
    const int widths[4] = {2, 4, 6, 8};
    double med[4] = {0.0, 0.0, 0.0, 0.0};
    const int saved = c->nuts_waves;
    for (int w = 0; w < 4 && rc == SMCGW_OK; ++w) {
        c->nuts_waves = widths[w];
        float t[16];
        for (int k = 0; k < trials && rc == SMCGW_OK; ++k) {
            if (hipMemcpyAsync(x, theta, nx, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
                hipMemcpyAsync(l, logl, nl, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
                hipMemcpyAsync(g, grad, nx, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
                hipEventRecord(e0, c->stream) != hipSuccess) {
                rc = SMCGW_ERR_HIP;
                break;
            }
            rc = smcgw_nuts_step(c, P, D, x, l, g, chol, prm, nullptr, nullptr, precision, nullptr, nullptr, nullptr,
                                 nullptr);
            if (rc != SMCGW_OK) break;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t[k], e0, e1) != hipSuccess)
                rc = SMCGW_ERR_HIP;
        }
        if (rc == SMCGW_OK) {
            std::sort(t, t + trials);
            med[w] = t[trials / 2];
        }
    }
    int best = saved;
    if (rc == SMCGW_OK) {
        int bi = 0;
        for (int w = 1; w < 4; ++w)
            if (med[w] < med[bi]) bi = w;
        best = widths[bi];
        if (best_waves) *best_waves = best;
        if (times_ms)
            for (int w = 0; w < 4; ++w) times_ms[w] = med[w];
    }
    c->nuts_waves = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(l);
    (void)hipFree(g);
    return rc;
}

namespace {

// Scratch of the sweep form: tree states [P], next positions [P][D], their
// logL [P] and gradients [P][D], active flags [P] and the active count.
struct SweepScratch {
    SweepState* st;
    double *x_next, *ll, *gl;
    uint8_t* active;
    int* count;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int sweep_reserve(smcgw_ctx* c, int P, int D, SweepScratch& s) {
    const size_t b_st = align256((size_t)P * sizeof(SweepState));
    const size_t b_x = align256((size_t)P * D * sizeof(double));
    const size_t b_ll = align256((size_t)P * sizeof(double));
    const size_t b_act = align256((size_t)P);
    const size_t need = b_st + 2 * b_x + b_ll + b_act + 256;
    if (need > c->sweep_bytes) {
        c->sweep_free();
        if (hipMalloc(&c->d_sweep, need) != hipSuccess) return SMCGW_ERR_OOM;
        c->sweep_bytes = need;
    }
    char* base = (char*)c->d_sweep;
    s.st = (SweepState*)base;
    s.x_next = (double*)(base + b_st);
    s.ll = (double*)(base + b_st + b_x);
    s.gl = (double*)(base + b_st + b_x + b_ll);
    s.active = (uint8_t*)(base + b_st + 2 * b_x + b_ll);
    s.count = (int*)(base + b_st + 2 * b_x + b_ll + b_act);
    return SMCGW_OK;
}

// One group of sweeps and the active count, on the context's stream.
int queue_sweep_group(smcgw_ctx* c, const NutsArgs& a, const SweepScratch& s, int sweeps) {
    for (int k = 0; k < sweeps; ++k) {
        {
            TimedLaunch tl(c, SMCGW_KERNEL_NUTS);
            hipLaunchKernelGGL(nuts_sweep_kernel, dim3(a.P), dim3(64), 0, c->stream, a, c->prior, c->pmap, s.st,
                               (const double*)s.ll, (const double*)s.gl, s.x_next, s.active);
        }
        if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
        const int rc = queue_loglike_tangent(c, a.P, c->ev_of_p, s.x_next, s.active, s.ll, s.gl);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(sweep_count_kernel, dim3(1), dim3(256), 0, c->stream, (const uint8_t*)s.active, a.P, s.count);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

}  // namespace

extern "C" int smcgw_nuts_step_sweeps(smcgw_ctx* c, int P, int D, double* theta, double* logl, double* grad,
                                      const double* chol, const smcgw_nuts_params* prm,
                                      const int32_t* max_depth_per_particle, int32_t* depth, int32_t* n_leapfrog,
                                      uint8_t* divergent, double* accept_stat, int sweeps_per_group,
                                      int* n_sweeps_host) {
    if (!c || !prm || P < 0 || D <= 0 || D > MAXDIM || (P > 0 && (!theta || !logl || !grad || !chol)) ||
        sweeps_per_group < 1 || sweeps_per_group > 64)
        return SMCGW_ERR_INVALID;
    if (prm->max_depth < 0 || prm->max_depth > SMCGW_MAX_DEPTH || !(prm->step > 0.0) ||
        (!prm->beta_device && !prm->state_device && !(prm->beta >= 0.0)) || !(prm->max_delta_h > 0.0) ||
        (prm->chol_per_particle != 0 && prm->chol_per_particle != 1) || prm->reserved != 0 || prm->reserved2 != 0)
        return SMCGW_ERR_INVALID;
    if (prm->state_device && (prm->run_size < 1 || P % prm->run_size != 0 || P / prm->run_size > SMCGW_MAX_RUNS))
        return SMCGW_ERR_INVALID;
    if (!c->prior_set || c->prior.dim != D || c->target.kind != SMCGW_TARGET_GW || c->events.empty() ||
        c->pmap.dim != D)
        return SMCGW_ERR_NOT_INIT;
    if (!tangent_supported(c)) return SMCGW_ERR_INVALID;
    if (n_sweeps_host) *n_sweeps_host = 0;
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    SweepScratch s;
    int rc = tangent_reserve(c, P);
    if (rc == SMCGW_OK) rc = sweep_reserve(c, P, D, s);
    int* hp = (int*)pinned(c);
    if (rc) return rc;
    if (!hp) return SMCGW_ERR_OOM;
    NutsArgs a{};
    a.P = P;
    a.D = D;
    a.theta = theta;
    a.logl = logl;
    a.grad = grad;
    a.chol = chol;
    a.step = prm->step;
    a.beta = prm->beta;
    a.max_dh = prm->max_delta_h;
    a.max_depth = prm->max_depth;
    a.uturn = prm->uturn ? 1 : 0;
    a.seed = prm->seed;
    a.iteration = prm->iteration;
    a.md_per_p = max_depth_per_particle;
    a.depth_out = depth;
    a.nlf_out = n_leapfrog;
    a.div_out = divergent;
    a.acc_out = accept_stat;
    a.events = c->d_events;
    a.n_events = (int)c->events.size();
    a.ev_of_p = c->ev_of_p;
    a.chol_pp = prm->chol_per_particle;
    a.beta_dev = prm->beta_device;
    a.state = prm->state_device;
    a.run_size = prm->state_device ? prm->run_size : P;
    hipLaunchKernelGGL(sweep_init_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, s.st, s.active,
                       (const double*)theta, s.x_next, P, D);
    if (hipGetLastError() != hipSuccess) return SMCGW_ERR_HIP;
    // the group graph is captured once for these arguments and replayed
    std::vector<unsigned char> key(sizeof(NutsArgs) + sizeof(PriorDesc) + sizeof(ParamMap) + 3 * sizeof(int));
    unsigned char* kp = key.data();
    std::memcpy(kp, &a, sizeof(a));
    std::memcpy(kp + sizeof(a), &c->prior, sizeof(PriorDesc));
    std::memcpy(kp + sizeof(a) + sizeof(PriorDesc), &c->pmap, sizeof(ParamMap));
    const int extra[3] = {sweeps_per_group, c->n_det, (int)(c->timing_mask != 0)};
    std::memcpy(kp + sizeof(a) + sizeof(PriorDesc) + sizeof(ParamMap), extra, sizeof(extra));
    if (key != c->sweep_key || !c->sweep_exec) {
        if (c->sweep_exec) (void)hipGraphExecDestroy(c->sweep_exec);
        if (c->sweep_graph) (void)hipGraphDestroy(c->sweep_graph);
        c->sweep_exec = nullptr;
        c->sweep_graph = nullptr;
        c->sweep_key.clear();
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SMCGW_ERR_HIP;
        const hipStream_t saved = c->stream;
        const unsigned saved_mask = c->timing_mask;
        c->stream = cap;
        c->timing_mask = 0;   // no timing events inside the graph
        bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        hipGraph_t g = nullptr;
        if (ok) {
            rc = queue_sweep_group(c, a, s, sweeps_per_group);
            ok = hipStreamEndCapture(cap, &g) == hipSuccess && rc == SMCGW_OK;
        }
        c->stream = saved;
        c->timing_mask = saved_mask;
        (void)hipStreamDestroy(cap);
        if (ok) ok = hipGraphInstantiate(&c->sweep_exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            if (g) (void)hipGraphDestroy(g);
            c->sweep_exec = nullptr;
            return rc ? rc : SMCGW_ERR_HIP;
        }
        c->sweep_graph = g;
        c->sweep_key = key;
    }
    // every transition ends within 2^max_depth sweeps (one leaf per sweep, the start included)
    const int md = max_depth_per_particle ? SMCGW_MAX_DEPTH : prm->max_depth;
    const long limit = (1L << md) + 1;
    long sweeps = 0;
    for (;;) {
        if (hipGraphLaunch(c->sweep_exec, c->stream) != hipSuccess) return SMCGW_ERR_HIP;
        sweeps += sweeps_per_group;
        if (hipMemcpyAsync(hp, s.count, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return SMCGW_ERR_HIP;
        if (*hp == 0) break;
        if (sweeps > limit + sweeps_per_group) return SMCGW_ERR_HIP;
    }
    if (n_sweeps_host) *n_sweeps_host = (int)sweeps;
    return SMCGW_OK;
}
