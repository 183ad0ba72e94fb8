// The plain form of the likelihood and gradient: the comparison form the
// mixed-precision adjoint path is measured against.
//
// logL = -1/2 <d-h|d-h> (arXiv:2601.02336, Sec. 2, Eq. 2) with every per-bin
// quantity in FP64 and the gradient by forward-mode tangents, the way an
// automatic forward-mode differentiation of the per-bin code computes it (the
// paper differentiates its likelihood automatically, Sec. 5 "JAX
// implementation"): every value carries its derivatives with respect to the
// 11 source parameters, seeded from the prologue's Jacobians, and each bin
// contributes
//   l_dj = Re(u_dj h'_dj) - 1/2 (w a^2)_dj |h'_dj|^2,   h'_dj = P'_d e^{-2 pi i Phi_dj},
// value and 11 tangents, with the per-bin |h|^2 written out (no per-event
// shortcut) and FP64 sin / cos.  No adjoint moments, no FP32.
#include "common.h"
#include "context.h"

namespace smcgw {

constexpr int NT = NPAR;            // tangents: the 11 source parameters
constexpr int TD = NT + 1;          // value + tangents
constexpr int TAN_WAVES = 4;        // particles (wavefronts) per workgroup

// A value with its tangents.
struct TDual {
    double v;
    double d[NT];
};

// Wave-uniform duals of one particle (LDS): phase coefficients in cycles,
// arrival-time terms and the projected amplitudes P'_d.
struct TangentCoef {
    double c[NCOEF][TD];
    double tau[MAXDET][TD];
    double pr[MAXDET][TD], pi[MAXDET][TD];
};

// Entry e of the particle's duals from its coefficient block (entry order:
// c, tau, pr, pi; slot 0 the value, slot 1 + k the tangent of parameter k).
__device__ __forceinline__ double tangent_entry(const double* cb, int e) {
    const int which = e / TD, slot = e % TD, k = slot - 1;
    const double amp = cb[CB_AMP];
    if (which < NCOEF) {   // c_b: intrinsic Jacobian; c_0 also -phi_c / (2 pi)
        const int b = which;
        if (slot == 0) return cb[CB_C + b];
        if (k < 4) return cb[CB_DC + 4 * b + k];
        return (b == 0 && k == P_PHIC) ? -1.0 / TWO_PI : 0.0;
    }
    int r = which - NCOEF;
    if (r < MAXDET) {      // tau_d = t_c + delay_d(ra, dec)
        const int d = r;
        if (slot == 0) return cb[CB_TAU + d];
        return k == P_TC ? 1.0 : k == P_RA ? cb[CB_DTAU + 2 * d] : k == P_DEC ? cb[CB_DTAU + 2 * d + 1] : 0.0;
    }
    r -= MAXDET;
    const bool im = r >= MAXDET;   // P'_d = C_A u_scale P_d
    const int d = im ? r - MAXDET : r;
    const double p = amp * cb[(im ? CB_PI : CB_PR) + d];
    if (slot == 0) return p;
    if (k == P_MC) return cb[CB_DLNCA_MC] * p;
    if (k == P_DL) return cb[CB_DLNCA_DL] * p;
    const int m = k == P_IOTA ? 0 : k == P_PSI ? 1 : k == P_RA ? 2 : k == P_DEC ? 3 : -1;
    return m < 0 ? 0.0 : amp * cb[(im ? CB_DPI : CB_DPR) + 4 * d + m];
}

constexpr int TC_ENTRIES = (NCOEF + 3 * MAXDET) * TD;
static_assert(sizeof(TangentCoef) == TC_ENTRIES * sizeof(double), "entry order of TangentCoef");

// One wavefront per particle; lane l takes bins l, l + 64, ...  The moment
// block of a particle is the bin sum of l_dj, value and tangents, [P][TD].
template <int NDET>
__global__ __launch_bounds__(64 * TAN_WAVES) void bins_tangent_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                                     const int32_t* __restrict__ ev_of_p, int P,
                                                                     const double* __restrict__ cb,
                                                                     const uint8_t* __restrict__ active,
                                                                     double* __restrict__ mom) {
    __shared__ TangentCoef TCs[TAN_WAVES];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * TAN_WAVES + wave;
    if (p >= P || (active && !active[p])) return;
    TangentCoef& K = TCs[wave];
    const double* c = cb + (size_t)p * CB_SIZE;
    double* kk = &K.c[0][0];
    for (int e = lane; e < TC_ENTRIES; e += 64) kk[e] = tangent_entry(c, e);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const DevEvent& ev = evs[event_index(ev_of_p, p, n_events)];
    const int npad = ev.n_pad;
    TDual acc;
    acc.v = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) acc.d[k] = 0.0;
    for (int j = lane; j < ev.n_bins; j += 64) {
        // the particle's duals are read from LDS at every bin (broadcast reads) instead of being held in
        // 216 registers across the loop
        __asm__ volatile("" ::: "memory");
        const double f = ev.fwl[(size_t)ROW_F * npad + j];
        double B[NBASIS];
        basis_rows(f, ev.fwl[(size_t)ROW_W * npad + j], ev.fwl[(size_t)ROW_LN * npad + j], B);
        TDual phi;   // intrinsic phase (cycles), shared by the detectors
        phi.v = K.c[0][0];
#pragma unroll
        for (int k = 0; k < NT; ++k) phi.d[k] = K.c[0][1 + k];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) {
            phi.v = fma(K.c[1 + b][0], B[b], phi.v);
#pragma unroll
            for (int k = 0; k < NT; ++k) phi.d[k] = fma(K.c[1 + b][1 + k], B[b], phi.d[k]);
        }
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            // value: detector phase (cycles), e = e^{-2 pi i Phi} = cs - i sn, h' = P' e, the bin's term
            const double phv = fma(f, K.tau[d][0], phi.v);
            const double x = phv - rint(phv);
            double sn, cs;
            sincospi(2.0 * x, &sn, &cs);
            const double er = cs, ei = -sn;
            const double pr = K.pr[d][0], pim = K.pi[d][0];
            const double hr = pr * er - pim * ei, hi = pr * ei + pim * er;
            const double2 u = ev.u64[(size_t)d * npad + j];
            const double wa = ev.wa2[(size_t)d * npad + j];
            acc.v += u.x * hr - u.y * hi - 0.5 * wa * (hr * hr + hi * hi);
            // tangents, one parameter at a time: dPhi, de = -2 pi (sn + i cs) dPhi, dh' = dP' e + P' de,
            // d(term) = Re(u dh') - (w a^2) Re(conj(h') dh')
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                const double dph = fma(f, K.tau[d][1 + k], phi.d[k]);
                const double der = -TWO_PI * sn * dph, dei = -TWO_PI * cs * dph;
                const double dpr = K.pr[d][1 + k], dpi = K.pi[d][1 + k];
                const double dhr = dpr * er + pr * der - (dpi * ei + pim * dei);
                const double dhi = dpr * ei + pr * dei + (dpi * er + pim * der);
                acc.d[k] += u.x * dhr - u.y * dhi - wa * (hr * dhr + hi * dhi);
            }
        }
    }
    double v[TD];
    int idx[TD];
    v[0] = acc.v;
    idx[0] = 0;
#pragma unroll
    for (int k = 0; k < NT; ++k) { v[1 + k] = acc.d[k]; idx[1 + k] = 1 + k; }
    wave_totals_to<TD>(v, idx, mom + (size_t)p * TD);
}

// logL = -<d|d>/2 + the bin sum; the gradient over the sampled coordinates.
__global__ __launch_bounds__(256) void tangent_finish_kernel(const DevEvent* __restrict__ evs, int n_events,
                                                             const int32_t* __restrict__ ev_of_p, ParamMap pm, int P,
                                                             const uint8_t* __restrict__ active,
                                                             const double* __restrict__ mom, double* __restrict__ logl,
                                                             double* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || (active && !active[p])) return;
    const double* m = mom + (size_t)p * TD;
    logl[p] = -0.5 * evs[event_index(ev_of_p, p, n_events)].dd + m[0];
    if (grad)
        for (int k = 0; k < pm.dim; ++k) grad[(size_t)p * pm.dim + k] = m[1 + pm.idx[k]];
}

// Per-particle scratch of the plain form: coefficient blocks and the tangent
// moment blocks.
int tangent_reserve(smcgw_ctx* c, int P) {
    int rc = ctx_reserve(c, P);
    if (rc) return rc;
    if (P <= c->tan_cap) return SMCGW_OK;
    (void)hipFree(c->d_tan);
    c->d_tan = nullptr;
    c->tan_cap = 0;
    const int cap = std::max(P, c->cap);
    if (hipMalloc(&c->d_tan, (size_t)cap * TD * sizeof(double)) != hipSuccess) return SMCGW_ERR_OOM;
    c->tan_cap = cap;
    return SMCGW_OK;
}

// logL and gradient of the particles with active[p] != 0 (active NULL: all)
// in the plain form, on the context's stream.  Needs tangent_reserve(P).
int queue_loglike_tangent(smcgw_ctx* c, int P, const int32_t* ev_of_p, const double* theta, const uint8_t* active,
                          double* logl, double* grad) {
    const int ne = (int)c->events.size();
    if (launch_prep(c->d_events, ne, ev_of_p, c->pmap, P, theta, c->d_cb, c->stream) != hipSuccess)
        return SMCGW_ERR_HIP;
    const dim3 grid((P + TAN_WAVES - 1) / TAN_WAVES), block(64 * TAN_WAVES);
    {
        TimedLaunch t(c, SMCGW_KERNEL_BINS);
        switch (c->n_det) {
        case 1: hipLaunchKernelGGL(bins_tangent_kernel<1>, grid, block, 0, c->stream, c->d_events, ne, ev_of_p, P, c->d_cb, active, c->d_tan); break;
        case 2: hipLaunchKernelGGL(bins_tangent_kernel<2>, grid, block, 0, c->stream, c->d_events, ne, ev_of_p, P, c->d_cb, active, c->d_tan); break;
        case 3: hipLaunchKernelGGL(bins_tangent_kernel<3>, grid, block, 0, c->stream, c->d_events, ne, ev_of_p, P, c->d_cb, active, c->d_tan); break;
        case 4: hipLaunchKernelGGL(bins_tangent_kernel<4>, grid, block, 0, c->stream, c->d_events, ne, ev_of_p, P, c->d_cb, active, c->d_tan); break;
        default: return SMCGW_ERR_SHAPE;
        }
    }
    hipLaunchKernelGGL(tangent_finish_kernel, dim3((P + 255) / 256), dim3(256), 0, c->stream, c->d_events, ne,
                       ev_of_p, c->pmap, P, active, (const double*)c->d_tan, logl, grad);
    return hipGetLastError() == hipSuccess ? SMCGW_OK : SMCGW_ERR_HIP;
}

// Every event of the context has the per-bin tables of the plain form.
bool tangent_supported(const smcgw_ctx* c) {
    if (c->events.empty()) return false;
    for (const DevEvent& e : c->events)
        if (!e.wa2) return false;
    return true;
}

}  // namespace smcgw

using namespace smcgw;

extern "C" int smcgw_loglike_grad_tangent(smcgw_ctx* c, int P, const int32_t* event_of_particle,
                                          const double* theta, double* logl, double* grad) {
    if (!c || P < 0 || (P > 0 && (!theta || !logl))) return SMCGW_ERR_INVALID;
    if (c->events.empty()) return SMCGW_ERR_NOT_INIT;
    if (!tangent_supported(c)) return SMCGW_ERR_INVALID;
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    int rc = tangent_reserve(c, P);
    if (rc) return rc;
    return queue_loglike_tangent(c, P, event_of_particle, theta, nullptr, logl, grad);
}
