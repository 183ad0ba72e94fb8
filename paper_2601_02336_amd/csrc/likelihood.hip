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
//   prep (eight lanes per particle): coefficient block, FP64 dual numbers with
//        one tangent per lane.
//   bins (one wavefront per particle): lanes stride the frequency bins, the
//        shared per-bin tables are read coalesced and each lane keeps its own
//        partial sums; a wavefront shuffle tree reduces them in FP64 into LDS,
//        and lane 0 forms logL and the gradient from them (FP64).
#include "binloop.h"
#include "coeffs.h"
#include "common.h"
#include "context.h"

namespace smcgw {

constexpr int BINS_WAVES = 4;   // wavefronts (particles) per workgroup

// Eight lanes per particle, as the persistent NUTS kernel splits a leaf's
// prologue: lanes 0-3 carry one intrinsic tangent each (Mc, q, chi1, chi2)
// while lanes 4-7 take the sines and cosines of the four extrinsic angles;
// then lane 4k + d (k = 0, 1) builds detector d with its ra (k = 0) or dec
// (k = 1) tangent, and lane 0 the amplitude.  One particle's chain is a
// quarter of the one-lane prologue's.
constexpr int PREP_LANES = 8;
constexpr int PREP_PER_BLOCK = 256 / PREP_LANES;
static_assert(2 * MAXDET == PREP_LANES && ANG_COUNT == PREP_LANES - 4, "prologue lane split");

__global__ __launch_bounds__(256) void prep_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                   const int32_t* __restrict__ ev_of_p, ParamMap pm, int P,
                                                   const double* __restrict__ theta, double* __restrict__ cb) {
    __shared__ double ang_sh[PREP_PER_BLOCK][ANG_COUNT][2];
    const int g = threadIdx.x / PREP_LANES, j = threadIdx.x % PREP_LANES;
    const int p = blockIdx.x * PREP_PER_BLOCK + g;
    const bool live = p < P;
    double th[NPAR];
    const DevEvent& ev = evs[event_index(ev_of_p, live ? p : 0, n_events)];
    double* c = cb + (size_t)(live ? p : 0) * CB_SIZE;
    if (live) {
        expand_params(pm, theta + (size_t)p * pm.dim, th);
        if (j < 4) {
            prep_intrinsic_n<1>(ev, th, c, j, j == 0);
        } else {
            double sn, cs;
            sincos(extrinsic_angle(ev, th, j - 4), &sn, &cs);
            ang_sh[g][j - 4][0] = sn;
            ang_sh[g][j - 4][1] = cs;
        }
    }
    __syncthreads();
    if (live) {
        ExtAngles ang;
#pragma unroll
        for (int k = 0; k < ANG_COUNT; ++k) { ang.sc[k][0] = ang_sh[g][k][0]; ang.sc[k][1] = ang_sh[g][k][1]; }
        const int k = j / MAXDET, d = j % MAXDET;
        prep_extrinsic_det_n<1>(ev, th, ang, c, d, k, k == 0);
        if (j == 0) prep_extrinsic_common(ev, th, c);
    }
}

// One wavefront per particle over all bins of its event, then the epilogue:
// the wavefront's coefficient block and moments sit in LDS and lane 0 forms
// logL and the gradient over the sampled coordinates.
template <int NDET, int PREC>
__device__ __forceinline__ void bins_and_finish(const DevEvent* __restrict__ evs, int n_events,
                                                const int32_t* __restrict__ ev_of_p, const ParamMap& pm, int P,
                                                const double* __restrict__ cb, double* __restrict__ logl,
                                                double* __restrict__ grad) {
    __shared__ double cb_sh[BINS_WAVES][CB_SIZE];
    __shared__ double mom_sh[BINS_WAVES][MOM_SIZE];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * BINS_WAVES + wave;
    if (p >= P) return;   // the whole wavefront: there is no workgroup barrier below
    const int e = __builtin_amdgcn_readfirstlane(event_index(ev_of_p, p, n_events));
    for (int i = lane; i < CB_SIZE; i += 64) cb_sh[wave][i] = cb[(size_t)p * CB_SIZE + i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const BinCoef k = load_coef(cb_sh[wave]);
    if (PREC == SMCGW_MIXED)
        bins_mixed_wave<NDET>(evs + e, k, 0, 1, mom_sh[wave]);
    else
        bins_fp64_wave<NDET>(evs + e, k, 0, 1, mom_sh[wave]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        double g[NPAR];
        logl[p] = finish_particle(evs[e], cb_sh[wave], mom_sh[wave], g);
        if (grad)
            for (int q = 0; q < pm.dim; ++q) grad[(size_t)p * pm.dim + q] = g[pm.idx[q]];
    }
}

template <int NDET>
__global__ __launch_bounds__(256) void bins_mixed_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                         const int32_t* __restrict__ ev_of_p, ParamMap pm, int P,
                                                         const double* __restrict__ cb, double* __restrict__ logl,
                                                         double* __restrict__ grad) {
    bins_and_finish<NDET, SMCGW_MIXED>(evs, n_events, ev_of_p, pm, P, cb, logl, grad);
}

template <int NDET>
__global__ __launch_bounds__(256) void bins_fp64_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                        const int32_t* __restrict__ ev_of_p, ParamMap pm, int P,
                                                        const double* __restrict__ cb, double* __restrict__ logl,
                                                        double* __restrict__ grad) {
    bins_and_finish<NDET, SMCGW_PLAIN_FP64>(evs, n_events, ev_of_p, pm, P, cb, logl, grad);
}

// Projected strain of one parameter point (FP64), h_reim [n_det][N][2].
__global__ __launch_bounds__(256) void waveform_kernel(const DevEvent* __restrict__ evs, int e,
                                                       const double* __restrict__ c, double* __restrict__ h, int n,
                                                       int n_det) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const DevEvent& ev = evs[e];
    const double f = ev.fwl[(size_t)ROW_F * ev.n_pad + j];
    double B[NBASIS];
    basis_rows(f, ev.fwl[(size_t)ROW_W * ev.n_pad + j], ev.fwl[(size_t)ROW_LN * ev.n_pad + j], B);
    double ph = c[CB_C];
    for (int b = 0; b < NBASIS; ++b) ph = fma(c[CB_C + 1 + b], B[b], ph);
    const double a = pow(f, -7.0 / 6.0) / ev.u_scale * c[CB_AMP];
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

// ------------------------------------------------------------- fixed scratch
// Coefficient blocks of smcgw_loglike_grad_noalloc, for at most
// SMCGW_NOALLOC_MAX_P particles (13 MiB).  Every GPU the library runs on
// holds its own copy until the process ends.  Host code must not pass the
// array's name to a kernel (it is a host-side stand-in there): the device
// address of each GPU's copy is looked up once per device at context set-up
// and kept in noalloc_base.
static __device__ __align__(256) double scratch[(size_t)SMCGW_NOALLOC_MAX_P * CB_SIZE];

constexpr int NOALLOC_DEVICES = 64;
static double* noalloc_base[NOALLOC_DEVICES] = {};

// Resolves this device's scratch address (the device must be current).
int noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_DEVICES) return SMCGW_ERR_INVALID;
    if (noalloc_base[device]) return SMCGW_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SMCGW_ERR_HIP;
    noalloc_base[device] = (double*)ptr;
    return SMCGW_OK;
}

// ------------------------------------------------------------- launchers
hipError_t launch_prep(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                       const double* theta, double* cb, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((P + PREP_PER_BLOCK - 1) / PREP_PER_BLOCK), dim3(256), 0, s, d_events,
                       n_events, ev_of_p, pm, P, theta, cb);
    return hipGetLastError();
}

template <int NDET>
hipError_t launch_bins_ndet(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm,
                            int P, int precision, const double* cb, double* logl, double* grad, hipStream_t s) {
    const dim3 grid((P + BINS_WAVES - 1) / BINS_WAVES), block(64 * BINS_WAVES);
    if (precision == SMCGW_MIXED)
        hipLaunchKernelGGL(bins_mixed_kernel<NDET>, grid, block, 0, s, d_events, n_events, ev_of_p, pm, P, cb, logl, grad);
    else
        hipLaunchKernelGGL(bins_fp64_kernel<NDET>, grid, block, 0, s, d_events, n_events, ev_of_p, pm, P, cb, logl, grad);
    return hipGetLastError();
}

hipError_t launch_bins(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                       int n_det, int precision, const double* cb, double* logl, double* grad, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    switch (n_det) {
    case 1: return launch_bins_ndet<1>(d_events, n_events, ev_of_p, pm, P, precision, cb, logl, grad, s);
    case 2: return launch_bins_ndet<2>(d_events, n_events, ev_of_p, pm, P, precision, cb, logl, grad, s);
    case 3: return launch_bins_ndet<3>(d_events, n_events, ev_of_p, pm, P, precision, cb, logl, grad, s);
    case 4: return launch_bins_ndet<4>(d_events, n_events, ev_of_p, pm, P, precision, cb, logl, grad, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_waveform(const DevEvent* d_events, int event_id, const double* cb, double* h_reim, int n_bins,
                           int n_det, hipStream_t s) {
    hipLaunchKernelGGL(waveform_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, d_events, event_id, cb, h_reim,
                       n_bins, n_det);
    return hipGetLastError();
}

}  // namespace smcgw

using namespace smcgw;

// The batched likelihood of smcgw_loglike_grad with its per-particle coefficient
// blocks in the fixed scratch array: no allocation, no event, no host
// synchronisation.
extern "C" int smcgw_loglike_grad_noalloc(smcgw_ctx* c, int P, const int32_t* event_of_particle, const double* theta,
                                          double* logl, double* grad, int precision) {
    if (!c || P < 0 || (P > 0 && (!theta || !logl))) return SMCGW_ERR_INVALID;
    if (precision != SMCGW_PLAIN_FP64 && precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (P > SMCGW_NOALLOC_MAX_P) return SMCGW_ERR_SHAPE;
    if (c->events.empty()) return SMCGW_ERR_NOT_INIT;
    if (P == 0) return SMCGW_OK;
    if (c->device < 0 || c->device >= NOALLOC_DEVICES || !noalloc_base[c->device]) return SMCGW_ERR_NOT_INIT;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    double* cb = noalloc_base[c->device];
    const int ne = (int)c->events.size();
    if (launch_prep(c->d_events, ne, event_of_particle, c->pmap, P, theta, cb, c->stream) != hipSuccess ||
        launch_bins(c->d_events, ne, event_of_particle, c->pmap, P, c->n_det, precision, cb, logl, grad,
                    c->stream) != hipSuccess)
        return SMCGW_ERR_HIP;
    return SMCGW_OK;
}
