// Batched GW log-likelihood and hand-written adjoint gradient.
//
// logL = -1/2 <d-h|d-h>, <a|b> = 4 Re sum_j a_j* b_j / S_j df (arXiv:2601.02336,
// Sec. 2, Eq. 2), expanded as
//   logL = -<d|d>/2 + sum_d [ Re(P'_d Z_d) - |P'_d|^2 H_d / 2 ],
//   Z_d  = sum_j u_dj e^{-2 pi i Phi_dj},   u_dj = 4 df conj(d_dj) f_j^-7/6 / S_dj,
// with P'_d = C_A P_d the per-particle amplitude and projection and Phi_dj the
// phase in cycles.  The adjoint of Z_d with respect to Phi_dj is
//   dlogL/dPhi_dj = 2 pi q_dj,  q_dj = Im(P'_d u_dj e^{-2 pi i Phi_dj}),
// so the gradient needs only the bin moments
//   G_b = sum_j psibar_j B_b(f_j),  psibar_j = sum_d q_dj,   T_d = sum_j q_dj f_j,
// accumulated in the same pass as Z_d; the epilogue chains them through the
// prologue's Jacobians.
//
// Kernels:
//   prep   (one lane per particle): coefficient block, FP64.
//   bins   (one wavefront per particle): lanes stride the frequency bins, the
//          shared per-bin tables are read coalesced and each lane keeps its own
//          partial sums; a wavefront shuffle tree reduces them in FP64.
//   finish (one lane per particle): logL and the gradient, FP64.
#include "common.h"
#include "coeffs.h"

namespace smcgw {

constexpr int BINS_WAVES = 4;          // wavefronts (particles) per workgroup
constexpr int BINS_KB = TABLE_PAD / 64; // bins per lane between FP32 -> FP64 flushes

__global__ __launch_bounds__(256) void prep_kernel(const DevEvent* __restrict__ evs, const int32_t* __restrict__ ev_of_p,
                                                   ParamMap pm, int P, const double* __restrict__ theta,
                                                   double* __restrict__ cb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double th[NPAR];
    expand_params(pm, theta + (size_t)p * pm.dim, th);
    const DevEvent& ev = evs[ev_of_p ? ev_of_p[p] : 0];
    double* c = cb + (size_t)p * CB_SIZE;
    prep_intrinsic(ev, th, c);
    prep_extrinsic(ev, th, c);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sin(2 pi x), cos(2 pi x) for |x| <= 1/2 with the hardware transcendental
// unit (v_sin_f32 / v_cos_f32 take their argument in revolutions).
__device__ __forceinline__ void sincos_rev_hw(float x, float& s, float& c) {
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
}

// MIXED precision bin loop: FP64 phase and argument reduction, FP32 sin/cos,
// complex products and partial sums (flushed into FP64 every BINS_KB bins per
// lane), FP64 phase-basis moments.
template <int NDET>
__global__ __launch_bounds__(256) void bins_mixed_kernel(const DevEvent* __restrict__ evs,
                                                         const int32_t* __restrict__ ev_of_p, int P,
                                                         const double* __restrict__ cb, double* __restrict__ mom) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * BINS_WAVES + wave;
    if (p >= P) return;
    const int e = ev_of_p ? __builtin_amdgcn_readfirstlane(ev_of_p[p]) : 0;
    const DevEvent* ev = evs + e;
    const int npad = ev->n_pad;
    const double* __restrict__ basis = ev->basis;
    const double* __restrict__ freq = ev->freq;
    const float2* __restrict__ u = ev->u32;
    const double* c = cb + (size_t)p * CB_SIZE;
    double cc[NCOEF];
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) cc[b] = c[CB_C + b];
    double tau[NDET];
    float pr[NDET], pim[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        tau[d] = c[CB_TAU + d];
        pr[d] = (float)c[CB_PR + d];
        pim[d] = (float)c[CB_PI + d];
    }
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { Zr[d] = 0.0; Zi[d] = 0.0; T[d] = 0.0; }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) G[b] = 0.0;

    for (int jb = 0; jb < npad; jb += 64 * BINS_KB) {
        float zr[NDET], zi[NDET], tq[NDET];
#pragma unroll
        for (int d = 0; d < NDET; ++d) { zr[d] = 0.f; zi[d] = 0.f; tq[d] = 0.f; }
#pragma unroll 2
        for (int k = 0; k < BINS_KB; ++k) {
            const int j = jb + 64 * k + lane;
            double B[NBASIS];
#pragma unroll
            for (int b = 0; b < NBASIS; ++b) B[b] = basis[(size_t)b * npad + j];
            const double f = freq[j];
            double ph = cc[0];
#pragma unroll
            for (int b = 0; b < NBASIS; ++b) ph = fma(cc[1 + b], B[b], ph);
            const float ff = (float)f;
            float psib = 0.f;
#pragma unroll
            for (int d = 0; d < NDET; ++d) {
                const double phd = fma(f, tau[d], ph);
                const float x = (float)(phd - rint(phd));
                float sn, cs;
                sincos_rev_hw(x, sn, cs);
                const float2 uu = u[(size_t)d * npad + j];
                // s = u e^{-2 pi i x}
                const float sr = fmaf(uu.x, cs, uu.y * sn);
                const float si = fmaf(uu.y, cs, -uu.x * sn);
                zr[d] += sr;
                zi[d] += si;
                const float q = fmaf(pr[d], si, pim[d] * sr);
                psib += q;
                tq[d] = fmaf(q, ff, tq[d]);
            }
            const double pb = (double)psib;
            G[0] += pb;
#pragma unroll
            for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(pb, B[b], G[1 + b]);
        }
#pragma unroll
        for (int d = 0; d < NDET; ++d) { Zr[d] += zr[d]; Zi[d] += zi[d]; T[d] += tq[d]; }
    }
    double* m = mom + (size_t)p * MOM_SIZE;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double a = wave_sum(Zr[d]), b2 = wave_sum(Zi[d]), t = wave_sum(T[d]);
        if (lane == 0) { m[MOM_ZR + d] = a; m[MOM_ZI + d] = b2; m[MOM_T + d] = t; }
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) {
        const double g = wave_sum(G[b]);
        if (lane == 0) m[MOM_G + b] = g;
    }
}

// PLAIN_FP64 bin loop: the same algebra with FP64 throughout.
template <int NDET>
__global__ __launch_bounds__(256) void bins_fp64_kernel(const DevEvent* __restrict__ evs,
                                                        const int32_t* __restrict__ ev_of_p, int P,
                                                        const double* __restrict__ cb, double* __restrict__ mom) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * BINS_WAVES + wave;
    if (p >= P) return;
    const int e = ev_of_p ? __builtin_amdgcn_readfirstlane(ev_of_p[p]) : 0;
    const DevEvent* ev = evs + e;
    const int npad = ev->n_pad;
    const double* __restrict__ basis = ev->basis;
    const double* __restrict__ freq = ev->freq;
    const double2* __restrict__ u = ev->u64;
    const double* c = cb + (size_t)p * CB_SIZE;
    double cc[NCOEF];
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) cc[b] = c[CB_C + b];
    double tau[NDET], pr[NDET], pim[NDET];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { tau[d] = c[CB_TAU + d]; pr[d] = c[CB_PR + d]; pim[d] = c[CB_PI + d]; }
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];
#pragma unroll
    for (int d = 0; d < NDET; ++d) { Zr[d] = 0.0; Zi[d] = 0.0; T[d] = 0.0; }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) G[b] = 0.0;
    for (int j = lane; j < npad; j += 64) {
        double B[NBASIS];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) B[b] = basis[(size_t)b * npad + j];
        const double f = freq[j];
        double ph = cc[0];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) ph = fma(cc[1 + b], B[b], ph);
        double psib = 0.0;
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const double phd = fma(f, tau[d], ph);
            const double x = phd - rint(phd);
            double sn, cs;
            sincospi(2.0 * x, &sn, &cs);
            const double2 uu = u[(size_t)d * npad + j];
            const double sr = fma(uu.x, cs, uu.y * sn);
            const double si = fma(uu.y, cs, -uu.x * sn);
            Zr[d] += sr;
            Zi[d] += si;
            const double q = fma(pr[d], si, pim[d] * sr);
            psib += q;
            T[d] = fma(q, f, T[d]);
        }
        G[0] += psib;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(psib, B[b], G[1 + b]);
    }
    double* m = mom + (size_t)p * MOM_SIZE;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const double a = wave_sum(Zr[d]), b2 = wave_sum(Zi[d]), t = wave_sum(T[d]);
        if (lane == 0) { m[MOM_ZR + d] = a; m[MOM_ZI + d] = b2; m[MOM_T + d] = t; }
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) {
        const double g = wave_sum(G[b]);
        if (lane == 0) m[MOM_G + b] = g;
    }
}

// logL and its gradient from the moments and the prologue's Jacobians.
__device__ __forceinline__ double finish_particle(const DevEvent& ev, const double* c, const double* m, double g[NPAR]) {
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

__global__ __launch_bounds__(256) void finish_kernel(const DevEvent* __restrict__ evs, const int32_t* __restrict__ ev_of_p,
                                                     ParamMap pm, int P, const double* __restrict__ cb,
                                                     const double* __restrict__ mom, double* __restrict__ logl,
                                                     double* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const DevEvent& ev = evs[ev_of_p ? ev_of_p[p] : 0];
    double g[NPAR];
    const double ll = finish_particle(ev, cb + (size_t)p * CB_SIZE, mom + (size_t)p * MOM_SIZE, g);
    logl[p] = ll;
    if (grad)
        for (int k = 0; k < pm.dim; ++k) grad[(size_t)p * pm.dim + k] = g[pm.idx[k]];
}

// Projected strain of one parameter point (FP64), h_reim [n_det][N][2].
__global__ __launch_bounds__(256) void waveform_kernel(const DevEvent* __restrict__ evs, int e,
                                                       const double* __restrict__ c, double* __restrict__ h, int n,
                                                       int n_det) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const DevEvent& ev = evs[e];
    const double f = ev.freq[j];
    double ph = c[CB_C];
    for (int b = 0; b < NBASIS; ++b) ph = fma(c[CB_C + 1 + b], ev.basis[(size_t)b * ev.n_pad + j], ph);
    const double a = pow(f, -7.0 / 6.0) / ev.u_scale;
    for (int d = 0; d < n_det; ++d) {
        const double phd = fma(f, c[CB_TAU + d], ph);
        const double x = phd - rint(phd);
        double sn, cs;
        sincospi(2.0 * x, &sn, &cs);
        const double pr = c[CB_PR + d] * a, pi = c[CB_PI + d] * a;
        h[2 * ((size_t)d * n + j)] = pr * cs + pi * sn;
        h[2 * ((size_t)d * n + j) + 1] = pi * cs - pr * sn;
    }
}

// ------------------------------------------------------------- launchers
hipError_t launch_prep(const DevEvent* d_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                       const double* theta, double* cb, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((P + 255) / 256), dim3(256), 0, s, d_events, ev_of_p, pm, P, theta, cb);
    return hipGetLastError();
}

hipError_t launch_bins(const DevEvent* d_events, const int32_t* ev_of_p, int P, int n_det, int precision,
                       const double* cb, double* mom, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    const dim3 grid((P + BINS_WAVES - 1) / BINS_WAVES), block(64 * BINS_WAVES);
    if (precision == SMCGW_MIXED) {
        switch (n_det) {
        case 1: hipLaunchKernelGGL(bins_mixed_kernel<1>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 2: hipLaunchKernelGGL(bins_mixed_kernel<2>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 3: hipLaunchKernelGGL(bins_mixed_kernel<3>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 4: hipLaunchKernelGGL(bins_mixed_kernel<4>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (n_det) {
        case 1: hipLaunchKernelGGL(bins_fp64_kernel<1>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 2: hipLaunchKernelGGL(bins_fp64_kernel<2>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 3: hipLaunchKernelGGL(bins_fp64_kernel<3>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        case 4: hipLaunchKernelGGL(bins_fp64_kernel<4>, grid, block, 0, s, d_events, ev_of_p, P, cb, mom); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_finish(const DevEvent* d_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                         const double* cb, const double* mom, double* logl, double* grad, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_kernel, dim3((P + 255) / 256), dim3(256), 0, s, d_events, ev_of_p, pm, P, cb, mom, logl,
                       grad);
    return hipGetLastError();
}

hipError_t launch_waveform(const DevEvent* d_events, int event_id, const double* cb, double* h_reim, int n_bins,
                           int n_det, hipStream_t s) {
    hipLaunchKernelGGL(waveform_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, d_events, event_id, cb, h_reim,
                       n_bins, n_det);
    return hipGetLastError();
}

}  // namespace smcgw
