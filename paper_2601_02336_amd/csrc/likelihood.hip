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
#include "binloop.h"
#include "coeffs.h"
#include "common.h"
#include "context.h"

namespace smcgw {

constexpr int BINS_WAVES = 4;   // wavefronts (particles) per workgroup

__global__ __launch_bounds__(256) void prep_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                   const int32_t* __restrict__ ev_of_p, ParamMap pm, int P,
                                                   const double* __restrict__ theta, double* __restrict__ cb) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double th[NPAR];
    expand_params(pm, theta + (size_t)p * pm.dim, th);
    const DevEvent& ev = evs[event_index(ev_of_p, p, n_events)];
    double* c = cb + (size_t)p * CB_SIZE;
    prep_intrinsic(ev, th, c);
    prep_extrinsic(ev, th, c);
}

// One wavefront per particle over all bins of its event.
template <int NDET>
__global__ __launch_bounds__(256) void bins_mixed_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                         const int32_t* __restrict__ ev_of_p, int P,
                                                         const double* __restrict__ cb, double* __restrict__ mom) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p = blockIdx.x * BINS_WAVES + wave;
    if (p >= P) return;
    const int e = __builtin_amdgcn_readfirstlane(event_index(ev_of_p, p, n_events));
    const BinCoef k = load_coef(cb + (size_t)p * CB_SIZE);
    bins_mixed_wave<NDET>(evs + e, k, 0, 1, mom + (size_t)p * MOM_SIZE);
}

template <int NDET>
__global__ __launch_bounds__(256) void bins_fp64_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                        const int32_t* __restrict__ ev_of_p, int P,
                                                        const double* __restrict__ cb, double* __restrict__ mom) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p = blockIdx.x * BINS_WAVES + wave;
    if (p >= P) return;
    const int e = __builtin_amdgcn_readfirstlane(event_index(ev_of_p, p, n_events));
    const BinCoef k = load_coef(cb + (size_t)p * CB_SIZE);
    bins_fp64_wave<NDET>(evs + e, k, 0, 1, mom + (size_t)p * MOM_SIZE);
}

__global__ __launch_bounds__(256) void finish_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                     const int32_t* __restrict__ ev_of_p, ParamMap pm, int P, const double* __restrict__ cb,
                                                     const double* __restrict__ mom, double* __restrict__ logl,
                                                     double* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const DevEvent& ev = evs[event_index(ev_of_p, p, n_events)];
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
// Coefficient and moment blocks of smcgw_loglike_grad_noalloc, for at most
// SMCGW_NOALLOC_MAX_P particles (16 MiB).  Every GPU the library runs on
// holds its own copy until the process ends.  Host code must not pass the
// array's name to a kernel (it is a host-side stand-in there): the device
// address of each GPU's copy is looked up once per device at context set-up
// and kept in noalloc_base.
static __device__ __align__(256) double scratch[(size_t)SMCGW_NOALLOC_MAX_P * (CB_SIZE + MOM_SIZE)];

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
    hipLaunchKernelGGL(prep_kernel, dim3((P + 255) / 256), dim3(256), 0, s, d_events, n_events, ev_of_p, pm, P, theta,
                       cb);
    return hipGetLastError();
}

hipError_t launch_bins(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, int P, int n_det, int precision,
                       const double* cb, double* mom, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    const dim3 grid((P + BINS_WAVES - 1) / BINS_WAVES), block(64 * BINS_WAVES);
    if (precision == SMCGW_MIXED) {
        switch (n_det) {
        case 1: hipLaunchKernelGGL(bins_mixed_kernel<1>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 2: hipLaunchKernelGGL(bins_mixed_kernel<2>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 3: hipLaunchKernelGGL(bins_mixed_kernel<3>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 4: hipLaunchKernelGGL(bins_mixed_kernel<4>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (n_det) {
        case 1: hipLaunchKernelGGL(bins_fp64_kernel<1>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 2: hipLaunchKernelGGL(bins_fp64_kernel<2>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 3: hipLaunchKernelGGL(bins_fp64_kernel<3>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        case 4: hipLaunchKernelGGL(bins_fp64_kernel<4>, grid, block, 0, s, d_events, n_events, ev_of_p, P, cb, mom); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_finish(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                         const double* cb, const double* mom, double* logl, double* grad, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(finish_kernel, dim3((P + 255) / 256), dim3(256), 0, s, d_events, n_events, ev_of_p, pm, P, cb,
                       mom, logl, grad);
    return hipGetLastError();
}

hipError_t launch_waveform(const DevEvent* d_events, int event_id, const double* cb, double* h_reim, int n_bins,
                           int n_det, hipStream_t s) {
    hipLaunchKernelGGL(waveform_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, d_events, event_id, cb, h_reim,
                       n_bins, n_det);
    return hipGetLastError();
}

}  // namespace smcgw

using namespace smcgw;

// The batched likelihood of smcgw_loglike_grad with its per-particle blocks in
// the fixed scratch array: no allocation, no event, no host synchronisation.
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
    double* mom = cb + (size_t)SMCGW_NOALLOC_MAX_P * CB_SIZE;
    const int ne = (int)c->events.size();
    if (launch_prep(c->d_events, ne, event_of_particle, c->pmap, P, theta, cb, c->stream) != hipSuccess ||
        launch_bins(c->d_events, ne, event_of_particle, P, c->n_det, precision, cb, mom, c->stream) != hipSuccess ||
        launch_finish(c->d_events, ne, event_of_particle, c->pmap, P, cb, mom, logl, grad, c->stream) != hipSuccess)
        return SMCGW_ERR_HIP;
    return SMCGW_OK;
}
