// Per-wavefront bin loop of the likelihood and its FP64 epilogue, shared by
// the batched likelihood kernels and the persistent NUTS kernel.
//
// A wavefront walks blocks of TABLE_PAD bins (its 64 lanes stride the bins of
// a block, TABLE_PAD/64 bins per lane) starting at block `blk0` with stride
// `blk_step`; the per-bin tables are read coalesced and shared by every
// particle.  Moments (see likelihood.hip) are returned wave-summed in FP64:
// every lane holds the totals of the blocks the wavefront visited.
#pragma once

#include "common.h"

namespace smcgw {

constexpr int BIN_KB = TABLE_PAD / 64;   // bins per lane per block (FP32 partials flushed per block)

// Wave-uniform per-particle values the bin loop needs (from the coefficient block).
struct BinCoef {
    double c[NCOEF];
    double tau[MAXDET];
    double pr[MAXDET], pi[MAXDET];
};

__device__ __forceinline__ double uniform_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sin(2 pi x), cos(2 pi x) for |x| <= 1/2 on the hardware transcendental unit
// (v_sin_f32 / v_cos_f32 take their argument in revolutions).
__device__ __forceinline__ void sincos_rev_hw(float x, float& s, float& c) {
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
}

// Coefficients of one particle from a coefficient block in any address space.
__device__ __forceinline__ BinCoef load_coef(const double* cb) {
    BinCoef k;
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) k.c[b] = uniform_d(cb[CB_C + b]);
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) {
        k.tau[d] = uniform_d(cb[CB_TAU + d]);
        k.pr[d] = uniform_d(cb[CB_PR + d]);
        k.pi[d] = uniform_d(cb[CB_PI + d]);
    }
    return k;
}

// Chunk cursor of a wavefront: 64-bin chunks of the blocks blk0, blk0 + step, ...
struct ChunkCursor {
    int blk, s;   // block and chunk within the block (0 .. BIN_KB-1)
    __device__ __forceinline__ int bin(int lane) const { return blk * TABLE_PAD + 64 * s + lane; }
    __device__ __forceinline__ bool advance(int blk_step, int nblk) {
        if (++s == BIN_KB) { s = 0; blk += blk_step; }
        return blk < nblk;
    }
};

// MIXED: FP64 phase and argument reduction, FP32 sin/cos, complex products and
// per-lane partial sums (flushed into FP64 once per block), FP64 basis moments.
// The table entries of the next chunk are loaded while the current one is
// computed.
template <int NDET>
__device__ __forceinline__ void bins_mixed_wave(const DevEvent* __restrict__ ev, const BinCoef& k, int blk0,
                                                int blk_step, double mom[MOM_SIZE]) {
    const int lane = threadIdx.x & 63;
    const int npad = ev->n_pad;
    const int nblk = npad / TABLE_PAD;
    const double* __restrict__ fwl = ev->fwl;
    const float2* __restrict__ u = ev->u32;
    float pr[NDET], pim[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { pr[d] = (float)k.pr[d]; pim[d] = (float)k.pi[d]; }
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];
    float zr[NDET], zi[NDET], tq[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { Zr[d] = 0.0; Zi[d] = 0.0; T[d] = 0.0; zr[d] = 0.f; zi[d] = 0.f; tq[d] = 0.f; }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) G[b] = 0.0;
    ChunkCursor cur{blk0, 0};
    bool more = blk0 < nblk;
    double nf = 0.0, nw = 0.0, nl = 0.0;
    float2 nu[NDET];
    if (more) {
        const int j = cur.bin(lane);
        nf = fwl[(size_t)ROW_F * npad + j];
        nw = fwl[(size_t)ROW_W * npad + j];
        nl = fwl[(size_t)ROW_LN * npad + j];
#pragma unroll
        for (int d = 0; d < NDET; ++d) nu[d] = u[(size_t)d * npad + j];
    }
    while (more) {
        const double f = nf, w = nw, lnf = nl;
        float2 uu[NDET];
#pragma unroll
        for (int d = 0; d < NDET; ++d) uu[d] = nu[d];
        const bool flush = (cur.s == BIN_KB - 1);
        more = cur.advance(blk_step, nblk);
        if (more) {
            const int j = cur.bin(lane);
            nf = fwl[(size_t)ROW_F * npad + j];
            nw = fwl[(size_t)ROW_W * npad + j];
            nl = fwl[(size_t)ROW_LN * npad + j];
#pragma unroll
            for (int d = 0; d < NDET; ++d) nu[d] = u[(size_t)d * npad + j];
        }
        double B[NBASIS];
        basis_rows(f, w, lnf, B);
        double ph = k.c[0];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) ph = fma(k.c[1 + b], B[b], ph);
        const float ff = (float)f;
        float psib;
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const double phd = fma(f, k.tau[d], ph);
            const float x = (float)(phd - rint(phd));
            float sn, cs;
            sincos_rev_hw(x, sn, cs);
            const float sr = fmaf(uu[d].x, cs, uu[d].y * sn);    // u e^{-2 pi i x}
            const float si = fmaf(uu[d].y, cs, -uu[d].x * sn);
            zr[d] += sr;
            zi[d] += si;
            const float q = fmaf(pr[d], si, pim[d] * sr);
            psib = (d == 0) ? q : psib + q;
            tq[d] = fmaf(q, ff, tq[d]);
        }
        const double pb = (double)psib;
        G[0] += pb;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(pb, B[b], G[1 + b]);
        if (flush) {
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                Zr[d] += zr[d]; Zi[d] += zi[d]; T[d] += tq[d];
                zr[d] = 0.f; zi[d] = 0.f; tq[d] = 0.f;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MOM_SIZE; ++i) mom[i] = 0.0;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        mom[MOM_ZR + d] = wave_sum(Zr[d] + zr[d]);
        mom[MOM_ZI + d] = wave_sum(Zi[d] + zi[d]);
        mom[MOM_T + d] = wave_sum(T[d] + tq[d]);
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) mom[MOM_G + b] = wave_sum(G[b]);
}

// PLAIN_FP64: the same algebra in FP64 throughout.
template <int NDET>
__device__ __forceinline__ void bins_fp64_wave(const DevEvent* __restrict__ ev, const BinCoef& k, int blk0,
                                               int blk_step, double mom[MOM_SIZE]) {
    const int lane = threadIdx.x & 63;
    const int npad = ev->n_pad;
    const int nblk = npad / TABLE_PAD;
    const double* __restrict__ fwl = ev->fwl;
    const double2* __restrict__ u = ev->u64;
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { Zr[d] = 0.0; Zi[d] = 0.0; T[d] = 0.0; }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) G[b] = 0.0;
    ChunkCursor cur{blk0, 0};
    bool more = blk0 < nblk;
    double nf = 0.0, nw = 0.0, nl = 0.0;
    double2 nu[NDET];
    if (more) {
        const int j = cur.bin(lane);
        nf = fwl[(size_t)ROW_F * npad + j];
        nw = fwl[(size_t)ROW_W * npad + j];
        nl = fwl[(size_t)ROW_LN * npad + j];
#pragma unroll
        for (int d = 0; d < NDET; ++d) nu[d] = u[(size_t)d * npad + j];
    }
    while (more) {
        const double f = nf, w = nw, lnf = nl;
        double2 uu[NDET];
#pragma unroll
        for (int d = 0; d < NDET; ++d) uu[d] = nu[d];
        more = cur.advance(blk_step, nblk);
        if (more) {
            const int j = cur.bin(lane);
            nf = fwl[(size_t)ROW_F * npad + j];
            nw = fwl[(size_t)ROW_W * npad + j];
            nl = fwl[(size_t)ROW_LN * npad + j];
#pragma unroll
            for (int d = 0; d < NDET; ++d) nu[d] = u[(size_t)d * npad + j];
        }
        double B[NBASIS];
        basis_rows(f, w, lnf, B);
        double ph = k.c[0];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) ph = fma(k.c[1 + b], B[b], ph);
        double psib;
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const double phd = fma(f, k.tau[d], ph);
            const double x = phd - rint(phd);
            double sn, cs;
            sincospi(2.0 * x, &sn, &cs);
            const double sr = fma(uu[d].x, cs, uu[d].y * sn);
            const double si = fma(uu[d].y, cs, -uu[d].x * sn);
            Zr[d] += sr;
            Zi[d] += si;
            const double q = fma(k.pr[d], si, k.pi[d] * sr);
            psib = (d == 0) ? q : psib + q;
            T[d] = fma(q, f, T[d]);
        }
        G[0] += psib;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(psib, B[b], G[1 + b]);
    }
#pragma unroll
    for (int i = 0; i < MOM_SIZE; ++i) mom[i] = 0.0;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        mom[MOM_ZR + d] = wave_sum(Zr[d]);
        mom[MOM_ZI + d] = wave_sum(Zi[d]);
        mom[MOM_T + d] = wave_sum(T[d]);
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) mom[MOM_G + b] = wave_sum(G[b]);
}

template <int NDET>
__device__ __forceinline__ void bins_wave(int precision, const DevEvent* ev, const BinCoef& k, int blk0, int blk_step,
                                          double mom[MOM_SIZE]) {
    if (precision == SMCGW_MIXED)
        bins_mixed_wave<NDET>(ev, k, blk0, blk_step, mom);
    else
        bins_fp64_wave<NDET>(ev, k, blk0, blk_step, mom);
}

// logL and its gradient with respect to the 11 source parameters from the
// moments and the prologue's Jacobians (FP64, one lane).
__device__ __forceinline__ double finish_particle(const DevEvent& ev, const double* c, const double* m,
                                                  double g[NPAR]) {
    double ll = -0.5 * ev.dd;
    double dlnca = 0.0, sum_t = 0.0;
    double gp[4] = {0.0, 0.0, 0.0, 0.0};   // iota, psi, ra, dec through P'_d
    for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
    for (int d = 0; d < ev.n_det; ++d) {
        const double pr = c[CB_PR + d], pi = c[CB_PI + d];
        const double zr = m[MOM_ZR + d], zi = m[MOM_ZI + d], h = ev.hnorm[d];
        const double re = pr * zr - pi * zi;
        const double p2 = pr * pr + pi * pi;
        ll += re - 0.5 * p2 * h;
        dlnca += re - p2 * h;
        const double ar = zr - h * pr, ai = -zi - h * pi;   // dlogL / d(Re P', Im P')
#pragma unroll
        for (int k = 0; k < 4; ++k) gp[k] += ar * c[CB_DPR + 4 * d + k] + ai * c[CB_DPI + 4 * d + k];
        const double t = m[MOM_T + d];
        sum_t += t;
        g[P_RA] += TWO_PI * t * c[CB_DTAU + 2 * d];
        g[P_DEC] += TWO_PI * t * c[CB_DTAU + 2 * d + 1];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double s = 0.0;
        for (int b = 0; b < NCOEF; ++b) s += c[CB_DC + 4 * b + k] * m[MOM_G + b];
        g[k] = TWO_PI * s;   // Mc, q, chi1, chi2 through the phase
    }
    g[P_MC] += dlnca * c[CB_DLNCA_MC];
    g[P_DL] = dlnca * c[CB_DLNCA_DL];
    g[P_IOTA] = gp[0];
    g[P_PSI] = gp[1];
    g[P_RA] += gp[2];
    g[P_DEC] += gp[3];
    g[P_TC] = TWO_PI * sum_t;
    g[P_PHIC] = -m[MOM_G + 0];
    return ll;
}

}  // namespace smcgw
