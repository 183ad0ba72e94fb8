// Per-particle prologue of the likelihood: source parameters -> phase-basis
// coefficients, per-detector delay and complex projection, and the Jacobians
// the adjoint needs.  FP64, one particle per lane.
//
// Waveform (not given in the paper, which uses IMRPhenomD): TaylorF2 with
// Newtonian amplitude and 3.5PN stationary-phase phase,
//   Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) sum_k (phi_k + phi_k^l ln v) v^k,
//   v = (pi M f)^{1/3};
// coefficients: Buonanno et al., PRD 80, 084043 (2009), Eq. (3.18) (non-spinning)
// and the aligned-spin terms collected in Khan et al., PRD 93, 044007 (2016), App. B.
// With ln v = (ln(pi M) + ln f)/3 every term is a fixed function of f times a
// per-particle coefficient, so the per-bin phase is a short FP64 dot product
// with the tables' basis rows and needs no per-bin transcendental.
#pragma once

#include "common.h"

namespace smcgw {

// ---------------------------------------------------------------- dual numbers
template <int N>
struct Dv {
    double v;
    double d[N];
};
template <int N> __device__ __forceinline__ Dv<N> dconst(double x) { Dv<N> r; r.v = x;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = 0.0; return r; }
template <int N> __device__ __forceinline__ Dv<N> dvar(double x, int k) { Dv<N> r = dconst<N>(x); r.d[k] = 1.0; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator+(const Dv<N>& a, const Dv<N>& b) { Dv<N> r; r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator-(const Dv<N>& a, const Dv<N>& b) { Dv<N> r; r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator*(const Dv<N>& a, const Dv<N>& b) { Dv<N> r; r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = fma(a.d[i], b.v, a.v * b.d[i]); return r; }
template <int N> __device__ __forceinline__ Dv<N> operator*(double a, const Dv<N>& b) { Dv<N> r; r.v = a * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a * b.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator+(double a, const Dv<N>& b) { Dv<N> r = b; r.v += a; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator-(double a, const Dv<N>& b) { Dv<N> r; r.v = a - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -b.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> recip(const Dv<N>& a) { Dv<N> r; r.v = 1.0 / a.v; const double s = -r.v * r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> operator/(const Dv<N>& a, const Dv<N>& b) { return a * recip(b); }
template <int N> __device__ __forceinline__ Dv<N> scale_chain(const Dv<N>& a, double f, double fp) { Dv<N> r; r.v = f;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = fp * a.d[i]; return r; }
template <int N> __device__ __forceinline__ Dv<N> dlog(const Dv<N>& a) { return scale_chain(a, log(a.v), 1.0 / a.v); }
template <int N> __device__ __forceinline__ Dv<N> dexp(const Dv<N>& a) { const double e = exp(a.v); return scale_chain(a, e, e); }

// ---------------------------------------------------------------- TaylorF2
// Phase coefficients in the (eta, delta = (m1-m2)/M, chi_s, chi_a) form.
template <int N>
__device__ __forceinline__ void tf2_phi(const Dv<N>& eta, const Dv<N>& delta, const Dv<N>& chis, const Dv<N>& chia,
                                        int pn, Dv<N> phi[8], Dv<N>& phi5l, Dv<N>& phi6l) {
    typedef Dv<N> DN;
    const double pi = PI;
    const DN eta2 = eta * eta;
    const DN eta3 = eta2 * eta;
    const DN dchia = delta * chia;
    phi[0] = dconst<N>(1.0);
    phi[1] = dconst<N>(0.0);
    phi[2] = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
    phi[3] = (-16.0 * pi) + (113.0 / 3.0) * dchia + ((113.0 / 3.0) - (76.0 / 3.0) * eta) * chis;
    phi[4] = (15293365.0 / 508032.0) + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * eta2
           + ((-405.0 / 8.0) + 200.0 * eta) * (chia * chia) - (405.0 / 4.0) * (dchia * chis)
           + ((-405.0 / 8.0) + 2.5 * eta) * (chis * chis);
    const DN x5 = (38645.0 * pi / 756.0) - (65.0 * pi / 9.0) * eta
               + ((-732985.0 / 2268.0) - (140.0 / 9.0) * eta) * dchia
               + ((-732985.0 / 2268.0) + (24260.0 / 81.0) * eta + (340.0 / 9.0) * eta2) * chis;
    phi[5] = x5;
    phi5l = 3.0 * x5;
    // 3PN: the constant part carries -6848/21 ln 4 from -6848/63 ln(64 v^3).
    phi[6] = (11583231236531.0 / 4694215680.0 - (6848.0 / 21.0) * 0.57721566490153286061 - (640.0 / 3.0) * pi * pi
              - (6848.0 / 21.0) * 1.38629436111989061883)
           + ((-15737765635.0 / 3048192.0) + (2255.0 / 12.0) * pi * pi) * eta + (76055.0 / 1728.0) * eta2
           - (127825.0 / 1296.0) * eta3 + ((2270.0 / 3.0) * pi) * dchia
           + ((2270.0 / 3.0) * pi - (520.0 * pi) * eta) * chis;
    phi6l = dconst<N>(-6848.0 / 21.0);
    phi[7] = (77096675.0 * pi / 254016.0) + (378515.0 * pi / 1512.0) * eta - (74045.0 * pi / 756.0) * eta2
           + ((-25150083775.0 / 3048192.0) + (26804935.0 / 6048.0) * eta - (1985.0 / 48.0) * eta2) * dchia
           + ((-25150083775.0 / 3048192.0) + (10566655595.0 / 762048.0) * eta - (1042165.0 / 3024.0) * eta2
              + (5345.0 / 36.0) * eta3) * chis;
    for (int k = 0; k < 8; ++k)
        if (k > pn) phi[k] = dconst<N>(0.0);
    if (pn < 5) phi5l = dconst<N>(0.0);
    if (pn < 6) phi6l = dconst<N>(0.0);
}

// Seeds parameter p of (Mc, q, chi1, chi2) as tangent p - k0 when it falls in [k0, k0 + N).
template <int N>
__device__ __forceinline__ Dv<N> seed(double x, int p, int k0) {
    Dv<N> r = dconst<N>(x);
    const int t = p - k0;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (i == t) ? 1.0 : 0.0;
    return r;
}

// Intrinsic part: coefficients c_b (cycles) and their derivatives with respect
// to the N intrinsic parameters k0 .. k0+N-1 of (Mc, q, chi1, chi2); phi_c and
// the -1/8 cycle offset included.  Values are written when write_values.
template <int N>
__device__ __forceinline__ void prep_intrinsic_n(const DevEvent& ev, const double th[NPAR], double* cb, int k0,
                                                 bool write_values) {
    typedef Dv<N> DN;
    const DN mc = seed<N>(th[P_MC], 0, k0);
    const DN q = seed<N>(th[P_Q], 1, k0);
    const DN c1 = seed<N>(th[P_CHI1], 2, k0);
    const DN c2 = seed<N>(th[P_CHI2], 3, k0);
    const DN opq = 1.0 + q;
    const DN iopq = recip(opq);
    const DN eta = q * (iopq * iopq);
    const DN delta = (1.0 - q) * iopq;
    const DN chis = 0.5 * (c1 + c2);
    const DN chia = 0.5 * (c1 - c2);
    const DN lneta = dlog(eta);
    const DN lnmc = dlog(mc);
    // ln(pi M), M = Mc eta^{-3/5} t_sun
    const DN lnpm = lnmc + (-0.6) * lneta + dconst<N>(ev.ln_pi_tsun);
    const DN pm13 = dexp((1.0 / 3.0) * lnpm);
    const DN pmm13 = recip(pm13);
    const DN pm23 = pm13 * pm13;
    const DN pmm23 = pmm13 * pmm13;
    const DN pmm1 = pmm23 * pmm13;
    const DN pmm53 = pmm1 * pmm23;
    DN phi[8], phi5l, phi6l;
    tf2_phi<N>(eta, delta, chis, chia, ev.pn_order, phi, phi5l, phi6l);
    const DN pref = (3.0 / (256.0 * PI)) * recip(eta);   // 3/(128 eta) / (2 pi): cycles
    DN c[NCOEF];
    const DN third5l = (1.0 / 3.0) * phi5l;
    const DN third6l = (1.0 / 3.0) * phi6l;
    c[0] = pref * (phi[5] + third5l * lnpm);
    c[1 + B_M53] = pref * (phi[0] * pmm53);
    c[1 + B_M1] = pref * (phi[2] * pmm1);
    c[1 + B_M23] = pref * (phi[3] * pmm23);
    c[1 + B_M13] = pref * (phi[4] * pmm13);
    c[1 + B_LN] = pref * third5l;
    c[1 + B_P13] = pref * (pm13 * (phi[6] + third6l * lnpm));
    c[1 + B_P13LN] = pref * (pm13 * third6l);
    c[1 + B_P23] = pref * (phi[7] * pm23);
    for (int b = 0; b < NCOEF; ++b) {
        if (write_values) cb[CB_C + b] = (b == 0) ? c[0].v - th[P_PHIC] / TWO_PI - 0.125 : c[b].v;
#pragma unroll
        for (int k = 0; k < N; ++k) cb[CB_DC + 4 * b + k0 + k] = c[b].d[k];
    }
}

__device__ __forceinline__ void prep_intrinsic(const DevEvent& ev, const double th[NPAR], double* cb) {
    prep_intrinsic_n<4>(ev, th, cb, 0, true);
}

// Extrinsic part of detector d: delay, complex projection C_A u_scale P_d and
// their Jacobians (zeros for d >= n_det).
// F+ = A cos 2psi + B sin 2psi, Fx = B cos 2psi - A sin 2psi with
// A = p.Dp - q.Dq, B = 2 p.Dq for the polarisation frame (p, q) at psi = 0.
// The extrinsic transcendentals shared by all detectors: sin / cos of
// ra - gmst, dec, 2 psi and iota.
struct ExtAngles {
    double sc[4][2];   // (sin, cos) of ra - gmst, dec, 2 psi, iota
};
enum { ANG_PHI = 0, ANG_DEC = 1, ANG_PSI2 = 2, ANG_IOTA = 3, ANG_COUNT = 4 };

__device__ __forceinline__ double extrinsic_angle(const DevEvent& ev, const double th[NPAR], int k) {
    return k == ANG_PHI ? th[P_RA] - ev.gmst : k == ANG_DEC ? th[P_DEC] : k == ANG_PSI2 ? 2.0 * th[P_PSI] : th[P_IOTA];
}

__device__ __forceinline__ double extrinsic_amplitude(const DevEvent& ev, const double th[NPAR]) {
    const double camp = 0.45643546458763842789 /* sqrt(5/24) */ * 0.46619407703541166 /* pi^-2/3 */
                      * exp((5.0 / 6.0) * log(th[P_MC] * ev.t_sun)) * ev.c_light / (th[P_DL] * ev.mpc_m);
    return camp * ev.u_scale;
}

__device__ __forceinline__ ExtAngles extrinsic_angles(const DevEvent& ev, const double th[NPAR]) {
    ExtAngles a;
#pragma unroll
    for (int k = 0; k < ANG_COUNT; ++k) sincos(extrinsic_angle(ev, th, k), &a.sc[k][0], &a.sc[k][1]);
    return a;
}

// Detector d's delay, complex projection P_d (without the amplitude, which
// prep_extrinsic_common writes once) and their Jacobians from the shared
// transcendentals (zeros for d >= n_det).  The (ra, dec)
// derivatives are carried as N tangents starting at k0 (N = 2, k0 = 0: both);
// values and the iota / psi derivatives are written when write_values.
template <int N>
__device__ __forceinline__ void prep_extrinsic_det_n(const DevEvent& ev, const double th[NPAR], const ExtAngles& ang,
                                                     double* cb, int d, int k0, bool write_values) {
    if (d >= ev.n_det) {
        if (write_values) {
            cb[CB_TAU + d] = 0.0; cb[CB_PR + d] = 0.0; cb[CB_PI + d] = 0.0;
            for (int k = 0; k < 2; ++k) { cb[CB_DPR + 4 * d + k] = 0.0; cb[CB_DPI + 4 * d + k] = 0.0; }
        }
#pragma unroll
        for (int t = 0; t < N; ++t) {
            cb[CB_DTAU + 2 * d + k0 + t] = 0.0;
            cb[CB_DPR + 4 * d + 2 + k0 + t] = 0.0;
            cb[CB_DPI + 4 * d + 2 + k0 + t] = 0.0;
        }
        return;
    }
    typedef Dv<N> DN;
    const DN phi = seed<N>(th[P_RA] - ev.gmst, 0, k0);
    const DN dec = seed<N>(th[P_DEC], 1, k0);
    const double sp = ang.sc[ANG_PHI][0], cp = ang.sc[ANG_PHI][1];
    const double sd = ang.sc[ANG_DEC][0], cd = ang.sc[ANG_DEC][1];
    const DN sphi = scale_chain(phi, sp, cp), cphi = scale_chain(phi, cp, -sp);
    const DN sdec = scale_chain(dec, sd, cd), cdec = scale_chain(dec, cd, -sd);
    const DN pv[3] = {sphi, dconst<N>(0.0) - cphi, dconst<N>(0.0)};
    const DN qv[3] = {dconst<N>(0.0) - cphi * sdec, dconst<N>(0.0) - sphi * sdec, cdec};
    const DN nv[3] = {cdec * cphi, cdec * sphi, sdec};
    const double s2 = ang.sc[ANG_PSI2][0], c2 = ang.sc[ANG_PSI2][1];
    const double si = ang.sc[ANG_IOTA][0], ci = ang.sc[ANG_IOTA][1];
    const double pp = 0.5 * (1.0 + ci * ci);
    DN Dp[3], Dq[3];
    for (int i = 0; i < 3; ++i) {
        Dp[i] = dconst<N>(0.0);
        Dq[i] = dconst<N>(0.0);
        for (int j = 0; j < 3; ++j) {
            Dp[i] = Dp[i] + ev.resp[d][i][j] * pv[j];
            Dq[i] = Dq[i] + ev.resp[d][i][j] * qv[j];
        }
    }
    DN A = dconst<N>(0.0), B = dconst<N>(0.0), nr = dconst<N>(0.0);
    for (int i = 0; i < 3; ++i) {
        A = A + (pv[i] * Dp[i] - qv[i] * Dq[i]);
        B = B + 2.0 * (pv[i] * Dq[i]);
        nr = nr + ev.pos[d][i] * nv[i];
    }
    const DN fp = c2 * A + s2 * B;
    const DN fx = c2 * B - s2 * A;
    const DN dt = (-1.0 / ev.c_light) * nr;
    if (write_values) {
        cb[CB_TAU + d] = th[P_TC] + dt.v;
        // P = F+ (1 + cos^2 i)/2 - i Fx cos i
        cb[CB_PR + d] = pp * fp.v;
        cb[CB_PI + d] = -ci * fx.v;
        cb[CB_DPR + 4 * d + 0] = -ci * si * fp.v;            // iota
        cb[CB_DPI + 4 * d + 0] = si * fx.v;
        cb[CB_DPR + 4 * d + 1] = pp * 2.0 * fx.v;            // psi: dF+/dpsi = 2 Fx
        cb[CB_DPI + 4 * d + 1] = ci * 2.0 * fp.v;            //      dFx/dpsi = -2 F+
    }
#pragma unroll
    for (int t = 0; t < N; ++t) {                             // ra (k = 0), dec (k = 1)
        cb[CB_DTAU + 2 * d + k0 + t] = dt.d[t];
        cb[CB_DPR + 4 * d + 2 + k0 + t] = pp * fp.d[t];
        cb[CB_DPI + 4 * d + 2 + k0 + t] = -ci * fx.d[t];
    }
}

// Entries shared by all detectors: the amplitude C_A u_scale and the
// derivatives of ln C_A.
__device__ __forceinline__ void prep_extrinsic_common(const DevEvent& ev, const double th[NPAR], double* cb) {
    cb[CB_AMP] = extrinsic_amplitude(ev, th);
    cb[CB_DLNCA_MC] = (5.0 / 6.0) / th[P_MC];
    cb[CB_DLNCA_DL] = -1.0 / th[P_DL];
}

__device__ __forceinline__ void prep_extrinsic(const DevEvent& ev, const double th[NPAR], double* cb) {
    prep_extrinsic_common(ev, th, cb);
    const ExtAngles ang = extrinsic_angles(ev, th);
    for (int d = 0; d < MAXDET; ++d) prep_extrinsic_det_n<2>(ev, th, ang, cb, d, 0, true);
}

__device__ __forceinline__ void expand_params(const ParamMap& pm, const double* x, double th[NPAR]) {
    for (int k = 0; k < NPAR; ++k) th[k] = pm.fixed[k];
    for (int k = 0; k < pm.dim; ++k) th[pm.idx[k]] = x[k];
}

}  // namespace smcgw
