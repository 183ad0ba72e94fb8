// FP64 CPU oracle for the SMC-NUTS gravitational-wave hot path.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file: only the tests, the smoke check and the benchmark's CPU
// baseline leg do.  It shares no code, header, table or constant generator
// with the HIP library.
//
// What it computes (arXiv:2601.02336, "The Sequential Monte Carlo goes NUTS"):
//   * logL = -1/2 <d-h|d-h>, <a|b> = 4 Re int a* b / S_n df        (Sec. 2, Eq. 2)
//     written literally as the residual sum 4 df sum_j |d_j-h_j|^2/S_j;
//   * the gradient of logL by forward-mode dual numbers (11 tangents), an
//     autodiff route independent of the hand-written adjoint      (Sec. 4, last para.)
//   * tempered target p_t ~ L^beta pi                               (Sec. 3, Eq. 3)
//   * reweighting, ESS, adaptive beta, multinomial resampling       (Sec. 3, Eqs. 4-6)
//   * evidence ratios and their product                             (Sec. 3.1, Eqs. 7-8)
//   * Hamiltonian and leapfrog                                      (Sec. 4, Eqs. 9-13)
//   * NUTS (multinomial, generalised U-turn; Hoffman & Gelman 2014,
//     Betancourt 2017 App. A)                                       (Sec. 4)
//   * reflective / periodic boundaries                              (Sec. 5, Eqs. 15-18)
//   * mass matrix from the particle population (covariance reading of the
//     local-geometry metric)                                        (Sec. 5, Eq. 14)
// The waveform is not in the paper (it uses IMRPhenomD); this oracle uses the
// closed-form TaylorF2 stationary-phase waveform with Newtonian amplitude and
// 3.5PN phase:
//   non-spinning coefficients: Buonanno, Iyer, Ochsner, Pan, Sathyaprakash,
//     PRD 80, 084043 (2009), Eq. (3.18) and Table I;
//   aligned-spin spin-orbit / spin-spin terms as collected in Khan et al.,
//     PRD 93, 044007 (2016), Appendix B (from Bohe, Marsat, Blanchet 2013 and
//     Mikoczi, Vasuth, Gergely 2005).  The 3PN and 3.5PN spin-spin terms are
//     omitted.  Every coefficient kept is pinned by an independent derivation:
//     energy balance with the published binding energy and flux (non-spinning
//     and spin-orbit, any mass ratio) and the Kerr test-mass limit (the 2PN
//     self-spin term).
//
// Antenna patterns and arrival-time delays are the textbook long-wavelength
// forms (e.g. Anderson, Brady, Creighton, Flanagan, PRD 63, 042003 (2001),
// App. B): F+ = D:e+, Fx = D:ex with D = (x x^T - y y^T)/2.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
// the run seed, counter = (index, particle, iteration, purpose).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

struct orc_event {
    double f_low, df;
    int32_t n_bins, n_det;
    double gmst;
    double t_sun, mpc_m, c_light;
    int32_t pn_order, reserved;
};

struct orc_detector {
    double lat, lon, az_x, az_y, radius;
};

struct orc_bound {
    double lo, hi;
    int32_t bnd;    // 0 none, 1 reflect, 2 periodic
    int32_t prior;  // 0 flat, 1 uniform, 2 log-uniform, 3 gaussian (lo = mean, hi = sigma)
};

// A sampling target: tempered likelihood times prior over D coordinates.
struct orc_target {
    int32_t kind;   // 0 GW, 1 standard normal, 2 Gaussian x Gaussian, 3 bimodal mixture
    int32_t dim;
    const orc_bound* bounds;        // [dim]
    const double* params;           // kind 2: y[dim], sigma_l[dim]; kind 3: mu1[dim], mu2[dim], sigma
    // GW only:
    const orc_event* ev;
    const orc_detector* dets;
    const double* data_reim;        // [n_det][N][2]
    const double* psd;              // [n_det][N]
    const int32_t* param_index;     // [dim] -> index in the 11 GW parameters
    const double* fixed11;          // values of the 11 GW parameters not sampled
    // Relative binning (GW only; rb_n_edges = 0: the likelihood on every bin).
    int32_t rb_n_edges, rb_reserved;
    const int32_t* rb_edges;        // [rb_n_edges] grid indices of the bin edges
    const double* rb_sum;           // [n_det][rb_n_edges - 1][4]: Re A0, Im A0, Re A1, Im A1 of each bin
    const double* rb_h0;            // [n_det][rb_n_edges][2]: fiducial strain at the edges
};

}  // extern "C"

namespace {

const double PI = 3.14159265358979323846;
const double EULER_GAMMA = 0.57721566490153286061;
const int NP = 11;  // GW parameter count

// ---------------------------------------------------------------- dual numbers
template <int N>
struct Dual {
    double v;
    double d[N];
    Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
    Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N> chain(const Dual<N>& a, double f, double fp) { Dual<N> r; r.v = f; for (int i = 0; i < N; ++i) r.d[i] = fp * a.d[i]; return r; }
template <int N> Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> Dual<N> exp(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> Dual<N> pow(const Dual<N>& a, double p) { double x = std::pow(a.v, p); return chain(a, x, p * std::pow(a.v, p - 1.0)); }

inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }
using std::sin; using std::cos; using std::exp; using std::log; using std::sqrt; using std::pow;

// Plain complex number over any scalar type.
template <class T>
struct Cx {
    T re, im;
};
template <class T> Cx<T> cmul(const Cx<T>& a, const Cx<T>& b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <class T> Cx<T> cadd(const Cx<T>& a, const Cx<T>& b) { return {a.re + b.re, a.im + b.im}; }
template <class T> Cx<T> cscale(const Cx<T>& a, const T& s) { return {a.re * s, a.im * s}; }
template <class T> Cx<T> cexp_i(const T& phase) { return {cos(phase), sin(phase)}; }  // e^{i phase}

// ---------------------------------------------------------------- geometry
struct Vec3 { double x, y, z; };

// Detector position and response tensor from its site descriptor.
void detector_geometry(const orc_detector& det, double pos[3], double resp[3][3]) {
    const double cl = std::cos(det.lat), sl = std::sin(det.lat);
    const double co = std::cos(det.lon), so = std::sin(det.lon);
    pos[0] = det.radius * cl * co;
    pos[1] = det.radius * cl * so;
    pos[2] = det.radius * sl;
    const double east[3] = {-so, co, 0.0};
    const double north[3] = {-sl * co, -sl * so, cl};
    double xa[3], ya[3];
    for (int i = 0; i < 3; ++i) {
        xa[i] = std::cos(det.az_x) * east[i] + std::sin(det.az_x) * north[i];
        ya[i] = std::cos(det.az_y) * east[i] + std::sin(det.az_y) * north[i];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            resp[i][j] = 0.5 * (xa[i] * xa[j] - ya[i] * ya[j]);
}

// Antenna patterns F+, Fx and geocentre-to-detector delay for a source at
// (ra, dec) with polarisation angle psi.
template <class T>
void antenna(const orc_detector& det, const T& ra, const T& dec, const T& psi, double gmst, double c_light,
             T& fplus, T& fcross, T& delay) {
    double pos[3], D[3][3];
    detector_geometry(det, pos, D);
    const T phi = ra - gmst;
    const T cphi = cos(phi), sphi = sin(phi), cd = cos(dec), sd = sin(dec);
    const T cpsi = cos(psi), spsi = sin(psi);
    const T n[3] = {cd * cphi, cd * sphi, sd};
    const T p[3] = {sphi, T(0.0) - cphi, T(0.0)};
    const T qv[3] = {T(0.0) - cphi * sd, T(0.0) - sphi * sd, cd};
    T X[3], Y[3];
    for (int i = 0; i < 3; ++i) {
        X[i] = p[i] * cpsi + qv[i] * spsi;
        Y[i] = qv[i] * cpsi - p[i] * spsi;
    }
    fplus = T(0.0);
    fcross = T(0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            fplus = fplus + D[i][j] * (X[i] * X[j] - Y[i] * Y[j]);
            fcross = fcross + D[i][j] * (X[i] * Y[j] + Y[i] * X[j]);
        }
    delay = T(0.0) - (n[0] * pos[0] + n[1] * pos[1] + n[2] * pos[2]) / c_light;
}

// ---------------------------------------------------------------- TaylorF2
// Coefficients phi_k, phi_k^log of the SPA phase
//   Psi(f) = 2 pi f t_c - phi_c - pi/4 + 3/(128 eta v^5) sum_k (phi_k + phi_k^log ln v) v^k,
// v = (pi M f)^(1/3) with M the total mass in seconds.
template <class T>
void taylorf2_coeffs(const T& eta, const T& delta, const T& chis, const T& chia, int pn_order, T phi[8], T phil[8]) {
    for (int k = 0; k < 8; ++k) { phi[k] = T(0.0); phil[k] = T(0.0); }
    const double pi = PI;
    const T eta2 = eta * eta, eta3 = eta2 * eta;
    phi[0] = T(1.0);
    phi[1] = T(0.0);
    phi[2] = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
    phi[3] = -16.0 * pi + (113.0 / 3.0) * delta * chia + (113.0 / 3.0 - (76.0 / 3.0) * eta) * chis;
    phi[4] = 15293365.0 / 508032.0 + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * eta2
           + (-405.0 / 8.0 + 200.0 * eta) * chia * chia - (405.0 / 4.0) * delta * chia * chis
           + (-405.0 / 8.0 + (5.0 / 2.0) * eta) * chis * chis;
    // 2.5PN: (1 + 3 ln v) times the bracket.
    const T c5 = (38645.0 * pi / 756.0) - (65.0 * pi / 9.0) * eta
               + delta * (-732985.0 / 2268.0 - (140.0 / 9.0) * eta) * chia
               + (-732985.0 / 2268.0 + (24260.0 / 81.0) * eta + (340.0 / 9.0) * eta2) * chis;
    phi[5] = c5;
    phil[5] = 3.0 * c5;
    // 3PN: -6848/63 ln(64 v^3) = -6848/21 ln 4 - 6848/21 ln v.
    phi[6] = 11583231236531.0 / 4694215680.0 - (6848.0 / 21.0) * EULER_GAMMA - (640.0 / 3.0) * pi * pi
           + (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi * pi) * eta
           + (76055.0 / 1728.0) * eta2 - (127825.0 / 1296.0) * eta3
           - (6848.0 / 21.0) * std::log(4.0)
           + (2270.0 / 3.0) * pi * delta * chia + ((2270.0 / 3.0) * pi - 520.0 * pi * eta) * chis;
    phil[6] = T(-6848.0 / 21.0);
    phi[7] = (77096675.0 * pi / 254016.0) + (378515.0 * pi / 1512.0) * eta - (74045.0 * pi / 756.0) * eta2
           + delta * (-25150083775.0 / 3048192.0 + (26804935.0 / 6048.0) * eta - (1985.0 / 48.0) * eta2) * chia
           + (-25150083775.0 / 3048192.0 + (10566655595.0 / 762048.0) * eta - (1042165.0 / 3024.0) * eta2
              + (5345.0 / 36.0) * eta3) * chis;
    for (int k = pn_order + 1; k < 8; ++k) { phi[k] = T(0.0); phil[k] = T(0.0); }
}

// Phase Psi(f) [rad] of the TaylorF2 waveform at one frequency.
template <class T>
T taylorf2_phase(const T& mc, const T& q, const T& chi1, const T& chi2, const T& tc, const T& phic,
                 double f, double t_sun, int pn_order) {
    const T eta = q / ((1.0 + q) * (1.0 + q));
    const T delta = (1.0 - q) / (1.0 + q);
    const T chis = 0.5 * (chi1 + chi2), chia = 0.5 * (chi1 - chi2);
    const T mtot = mc * pow(eta, -0.6) * t_sun;          // total mass [s]
    const T v = pow(PI * mtot * f, 1.0 / 3.0);
    const T lnv = log(v);
    T phi[8], phil[8];
    taylorf2_coeffs(eta, delta, chis, chia, pn_order, phi, phil);
    T sum(0.0);
    T vk(1.0);
    for (int k = 0; k < 8; ++k) {
        sum = sum + (phi[k] + phil[k] * lnv) * vk;
        vk = vk * v;
    }
    const T v5 = pow(v, 5.0);
    return 2.0 * PI * f * tc - phic - PI / 4.0 + 3.0 / (128.0 * eta * v5) * sum;
}

// Projected detector strain h_d(f) of the 11-parameter model at one bin.
template <class T>
Cx<T> detector_strain(const orc_event& ev, const orc_detector& det, const T th[NP], double f) {
    const T& mc = th[0]; const T& q = th[1]; const T& chi1 = th[2]; const T& chi2 = th[3];
    const T& dl = th[4]; const T& iota = th[5]; const T& psi = th[6]; const T& ra = th[7];
    const T& dec = th[8]; const T& tc = th[9]; const T& phic = th[10];
    const T psi_f = taylorf2_phase(mc, q, chi1, chi2, tc, phic, f, ev.t_sun, ev.pn_order);
    // Newtonian amplitude sqrt(5/24) pi^(-2/3) (G Mc/c^3)^(5/6) f^(-7/6) / (d_L / c).
    const T amp = std::sqrt(5.0 / 24.0) * std::pow(PI, -2.0 / 3.0) * pow(mc * ev.t_sun, 5.0 / 6.0)
                * std::pow(f, -7.0 / 6.0) / (dl * (ev.mpc_m / ev.c_light));
    const T ci = cos(iota);
    T fp, fc, dt;
    antenna(det, ra, dec, psi, ev.gmst, ev.c_light, fp, fc, dt);
    // h+ = A (1 + cos^2 i)/2 e^{-i Psi};  hx = -i A cos i e^{-i Psi};  h = F+ h+ + Fx hx.
    const Cx<T> proj = {fp * (1.0 + ci * ci) * 0.5, T(0.0) - fc * ci};
    const T total_phase = T(0.0) - psi_f - 2.0 * PI * f * dt;   // e^{-i Psi} e^{-2 pi i f dt}
    return cmul(cscale(proj, amp), cexp_i(total_phase));
}

template <class T>
T gw_loglike(const orc_event& ev, const orc_detector* dets, const double* data_reim, const double* psd,
             const T th[NP]) {
    T total(0.0);
    const int n = ev.n_bins;
    for (int d = 0; d < ev.n_det; ++d) {
        T acc(0.0);
        for (int j = 0; j < n; ++j) {
            const double f = ev.f_low + ev.df * j;
            const Cx<T> h = detector_strain(ev, dets[d], th, f);
            const double* dd = data_reim + 2 * ((size_t)d * n + j);
            const T rr = dd[0] - h.re, ri = dd[1] - h.im;
            acc = acc + (rr * rr + ri * ri) / psd[(size_t)d * n + j];
        }
        total = total + acc;
    }
    return -0.5 * 4.0 * ev.df * total;
}

// Relative binning (Zackay, Dai & Venumadhav 2018, arXiv:1806.08792; the
// long-segment mitigation named in Secs. 2 and 7).  With a fiducial strain h0
// and the ratio r = h / h0 taken linear in f inside each bin b = [f_b, f_b+1],
//   <d|h> = Re sum_d sum_b [A0_db r_d(f_b) + A1_db (r_d(f_b+1) - r_d(f_b)) / (f_b+1 - f_b)],
//   A0_db = sum_{j in b} 4 df conj(d_dj) h0_dj / S_dj,  A1_db = the same weighted by (f_j - f_b);
// <h|h> and <d|d> are summed over every bin.  Bin b holds the grid points
// [edge_b, edge_b+1) (the last bin also its end point).
template <class T>
T gw_loglike_rb(const orc_target& t, const T th[NP]) {
    const orc_event& ev = *t.ev;
    const int n = ev.n_bins, ne = t.rb_n_edges, nb = ne - 1;
    T dh(0.0), hh(0.0);
    double dd = 0.0;
    for (int d = 0; d < ev.n_det; ++d) {
        std::vector<Cx<T>> r(ne);
        for (int e = 0; e < ne; ++e) {
            const double f = ev.f_low + ev.df * t.rb_edges[e];
            const Cx<T> h = detector_strain(ev, t.dets[d], th, f);
            const double* h0 = t.rb_h0 + 2 * ((size_t)d * ne + e);
            const double m = h0[0] * h0[0] + h0[1] * h0[1];
            r[e] = {(h.re * h0[0] + h.im * h0[1]) / m, (h.im * h0[0] - h.re * h0[1]) / m};   // h conj(h0) / |h0|^2
        }
        for (int b = 0; b < nb; ++b) {
            const double* a = t.rb_sum + 4 * ((size_t)d * nb + b);
            const double wb = ev.df * (t.rb_edges[b + 1] - t.rb_edges[b]);
            const Cx<T> slope = {(r[b + 1].re - r[b].re) / wb, (r[b + 1].im - r[b].im) / wb};
            dh = dh + (a[0] * r[b].re - a[1] * r[b].im) + (a[2] * slope.re - a[3] * slope.im);
        }
        for (int j = 0; j < n; ++j) {
            const Cx<T> h = detector_strain(ev, t.dets[d], th, ev.f_low + ev.df * j);
            const double w = 4.0 * ev.df / t.psd[(size_t)d * n + j];
            hh = hh + w * (h.re * h.re + h.im * h.im);
            const double* x = t.data_reim + 2 * ((size_t)d * n + j);
            dd += w * (x[0] * x[0] + x[1] * x[1]);
        }
    }
    return dh - 0.5 * hh - 0.5 * dd;
}

// --------------------------------------------------------------- targets
typedef Dual<NP> D11;

void expand_gw(const orc_target& t, const double* x, double th[NP]) {
    for (int k = 0; k < NP; ++k) th[k] = t.fixed11 ? t.fixed11[k] : 0.0;
    for (int k = 0; k < t.dim; ++k) th[t.param_index ? t.param_index[k] : k] = x[k];
}

// Log-likelihood (and its gradient over the target's D coordinates).
double target_loglike(const orc_target& t, const double* x, double* grad) {
    const int D = t.dim;
    switch (t.kind) {
    case 0: {
        double th[NP];
        expand_gw(t, x, th);
        if (!grad)
            return t.rb_n_edges > 0 ? gw_loglike_rb<double>(t, th)
                                    : gw_loglike<double>(*t.ev, t.dets, t.data_reim, t.psd, th);
        D11 td[NP];
        for (int k = 0; k < NP; ++k) { td[k] = D11(th[k]); td[k].d[k] = 1.0; }
        const D11 l = t.rb_n_edges > 0 ? gw_loglike_rb<D11>(t, td)
                                       : gw_loglike<D11>(*t.ev, t.dets, t.data_reim, t.psd, td);
        for (int k = 0; k < D; ++k) grad[k] = l.d[t.param_index ? t.param_index[k] : k];
        return l.v;
    }
    case 1: {  // standard normal, logL = -|x|^2/2
        double s = 0.0;
        for (int k = 0; k < D; ++k) { s += x[k] * x[k]; if (grad) grad[k] = -x[k]; }
        return -0.5 * s;
    }
    case 2: {  // normalised Gaussian likelihood N(y; x, diag sigma^2)
        const double* y = t.params; const double* sg = t.params + D;
        double s = 0.0;
        for (int k = 0; k < D; ++k) {
            const double r = (y[k] - x[k]) / sg[k];
            s += -0.5 * r * r - 0.5 * std::log(2.0 * PI * sg[k] * sg[k]);
            if (grad) grad[k] = r / sg[k];
        }
        return s;
    }
    case 3: {  // unweighted sum of two normalised isotropic Gaussians
        const double* m1 = t.params; const double* m2 = t.params + D; const double sg = t.params[2 * D];
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < D; ++k) {
            s1 += (x[k] - m1[k]) * (x[k] - m1[k]);
            s2 += (x[k] - m2[k]) * (x[k] - m2[k]);
        }
        const double c = -0.5 * D * std::log(2.0 * PI * sg * sg);
        const double l1 = c - 0.5 * s1 / (sg * sg), l2 = c - 0.5 * s2 / (sg * sg);
        const double mx = std::max(l1, l2);
        const double w1 = std::exp(l1 - mx), w2 = std::exp(l2 - mx);
        if (grad)
            for (int k = 0; k < D; ++k)
                grad[k] = (w1 * (m1[k] - x[k]) + w2 * (m2[k] - x[k])) / (sg * sg) / (w1 + w2);
        return mx + std::log(w1 + w2);
    }
    }
    return NAN;
}

// Normalised log prior and its gradient.
double target_logprior(const orc_target& t, const double* x, double* grad) {
    double lp = 0.0;
    for (int k = 0; k < t.dim; ++k) {
        const orc_bound& b = t.bounds[k];
        double g = 0.0;
        switch (b.prior) {
        case 0: break;
        case 1:
            if (x[k] < b.lo || x[k] > b.hi) return -INFINITY;
            lp += -std::log(b.hi - b.lo);
            break;
        case 2:
            if (x[k] < b.lo || x[k] > b.hi) return -INFINITY;
            lp += -std::log(x[k]) - std::log(std::log(b.hi / b.lo));
            g = -1.0 / x[k];
            break;
        case 3: {
            const double r = (x[k] - b.lo) / b.hi;
            lp += -0.5 * r * r - 0.5 * std::log(2.0 * PI * b.hi * b.hi);
            g = -r / b.hi;
            break;
        }
        }
        if (grad) grad[k] = g;
    }
    return lp;
}

// ---------------------------------------------------------------- Philox4x32-10
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { PURPOSE_MOMENTUM = 1, PURPOSE_DOUBLING = 2, PURPOSE_LEAF = 3, PURPOSE_RESAMPLE = 4, PURPOSE_RECYCLE = 5 };

// Two uniforms in [0, 1) with 53 random bits each.
void uniforms2(uint64_t seed, uint32_t index, uint32_t particle, uint64_t iteration, uint32_t purpose, double u[2]) {
    const uint32_t ctr[4] = {index, particle, (uint32_t)iteration, purpose};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    philox4x32_10(ctr, key, o);
    const double scale = 1.0 / 9007199254740992.0;  // 2^-53
    u[0] = ((double)(o[0] >> 5) * 67108864.0 + (double)(o[1] >> 6)) * scale;
    u[1] = ((double)(o[2] >> 5) * 67108864.0 + (double)(o[3] >> 6)) * scale;
}

// ---------------------------------------------------------------- linear algebra
// y = M^{-1} r with M^{-1} = L L^T (L lower, row-major D x D).
void inv_mass_apply(int D, const double* L, const double* r, double* y) {
    double t[64];
    for (int j = 0; j < D; ++j) { double s = 0.0; for (int i = j; i < D; ++i) s += L[i * D + j] * r[i]; t[j] = s; }  // L^T r
    for (int i = 0; i < D; ++i) { double s = 0.0; for (int j = 0; j <= i; ++j) s += L[i * D + j] * t[j]; y[i] = s; }
}

// Kinetic energy r^T M^{-1} r / 2.
double kinetic(int D, const double* L, const double* r) {
    double s = 0.0;
    for (int j = 0; j < D; ++j) { double t = 0.0; for (int i = j; i < D; ++i) t += L[i * D + j] * r[i]; s += t * t; }
    return 0.5 * s;
}

// ---------------------------------------------------------------- boundaries
// The drift x += eps M^{-1} r of the leapfrog (Sec. 4, Eq. 12) inside the prior
// box (Sec. 5, Eqs. 15-18).  Reflective walls: the drift runs at velocity
// v = M^{-1} r until the first coordinate k reaches its wall, the momentum is
// reflected there,
//   r -> r - 2 (v_k / (M^{-1})_kk) e_k,
// which reverses v_k and keeps the kinetic energy r^T M^{-1} r / 2, and the
// drift goes on with the new velocity for the rest of the step (a specular
// reflection in the metric; repeated for every wall met).  With a diagonal
// M this is the paper's fold of the coordinate and flip of its momentum
// component; for any M the step stays reversible (drifting back from the
// end point with -r retraces the path) and volume preserving.  Periodic
// coordinates wrap by the box width at the end, the momentum untouched.
void drift(const orc_target& t, const double* L, double eps, double* x, double* r) {
    const int D = t.dim;
    double v[32], minv_kk[32];
    inv_mass_apply(D, L, r, v);
    for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int m = 0; m <= k; ++m) s += L[k * D + m] * L[k * D + m];
        minv_kk[k] = s;   // (L L^T)_kk
    }
    double rem = 1.0;   // fraction of the step left
    for (int it = 0; it < 64; ++it) {
        int first = -1;
        double frac = rem, wall = 0.0;
        for (int k = 0; k < D; ++k) {
            const orc_bound& b = t.bounds[k];
            const double u = eps * v[k];
            if (b.bnd != 1 || u == 0.0) continue;
            const double w = u > 0.0 ? b.hi : b.lo;
            const double f = std::max((w - x[k]) / u, 0.0);
            if (f < frac) { frac = f; first = k; wall = w; }
        }
        if (first < 0) {
            for (int k = 0; k < D; ++k) x[k] += (rem * eps) * v[k];
            break;
        }
        for (int k = 0; k < D; ++k) x[k] += (frac * eps) * v[k];
        x[first] = wall;
        rem -= frac;
        r[first] -= 2.0 * v[first] / minv_kk[first];
        inv_mass_apply(D, L, r, v);
    }
    for (int k = 0; k < D; ++k) {
        const orc_bound& b = t.bounds[k];
        if (b.bnd != 2) continue;
        const double w = b.hi - b.lo;
        for (int it = 0; it < 64 && (x[k] < b.lo || x[k] >= b.hi); ++it) x[k] = (x[k] >= b.hi) ? x[k] - w : x[k] + w;
    }
}

// ---------------------------------------------------------------- one state
struct State {
    double x[32], r[32], g[32];  // position, momentum, gradient of log p_t
    double gl[32];               // gradient of logL
    double logl, logp;           // log-likelihood, tempered log target
};

void eval_state(const orc_target& t, double beta, State& s) {
    double gp[32];
    s.logl = target_loglike(t, s.x, s.gl);
    const double lp = target_logprior(t, s.x, gp);
    s.logp = beta * s.logl + lp;
    for (int k = 0; k < t.dim; ++k) s.g[k] = beta * s.gl[k] + gp[k];
}

// One leapfrog step of size eps (negative eps integrates backwards in time).
void leapfrog(const orc_target& t, double beta, const double* L, double eps, State& s) {
    const int D = t.dim;
    for (int k = 0; k < D; ++k) s.r[k] += 0.5 * eps * s.g[k];     // r - eps/2 dU/dx, U = -log p_t
    drift(t, L, eps, s.x, s.r);
    eval_state(t, beta, s);
    for (int k = 0; k < D; ++k) s.r[k] += 0.5 * eps * s.g[k];
}

double log_add_exp(double a, double b) {
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = std::max(a, b);
    return m + std::log(std::exp(a - m) + std::exp(b - m));
}

// Generalised no-U-turn criterion: continue iff rho.M^{-1}r_a > 0 and rho.M^{-1}r_b > 0.
bool no_uturn(int D, const double* L, const double* rho, const double* ra, const double* rb) {
    double va[32], vb[32];
    inv_mass_apply(D, L, ra, va);
    inv_mass_apply(D, L, rb, vb);
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < D; ++k) { sa += rho[k] * va[k]; sb += rho[k] * vb[k]; }
    return sa > 0.0 && sb > 0.0;
}

struct NutsOut {
    int depth, n_leapfrog, divergent;
    double accept_stat;
};

// One multinomial NUTS transition (iterative doubling).
NutsOut nuts_transition(const orc_target& t, double beta, const double* L, double eps, int max_depth, int uturn,
                        double max_dh, uint64_t seed, uint64_t iteration, uint32_t particle, State& cur) {
    const int D = t.dim;
    NutsOut out = {0, 0, 0, 0.0};
    // Momentum r = L^{-T} z, z ~ N(0, I), so that r ~ N(0, M) with M = (L L^T)^{-1}.
    double z[32];
    for (int p = 0; 2 * p < D; ++p) {
        double u[2];
        uniforms2(seed, (uint32_t)p, particle, iteration, PURPOSE_MOMENTUM, u);
        const double rad = std::sqrt(-2.0 * std::log(1.0 - u[0]));
        z[2 * p] = rad * std::cos(2.0 * PI * u[1]);
        if (2 * p + 1 < D) z[2 * p + 1] = rad * std::sin(2.0 * PI * u[1]);
    }
    for (int i = D - 1; i >= 0; --i) {  // solve L^T r = z
        double s = z[i];
        for (int k = i + 1; k < D; ++k) s -= L[k * D + i] * cur.r[k];
        cur.r[i] = s / L[i * D + i];
    }
    const double h0 = -cur.logp + kinetic(D, L, cur.r);

    State left = cur, right = cur, prop = cur;
    double log_w = 0.0;                 // log sum of exp(-(H - H0)) over the tree
    double rho[32];
    for (int k = 0; k < D; ++k) rho[k] = cur.r[k];
    uint32_t leaf_counter = 0;
    double accept_sum = 0.0;

    for (int j = 0; j < max_depth; ++j) {
        double ud[2];
        uniforms2(seed, (uint32_t)j, particle, iteration, PURPOSE_DOUBLING, ud);
        const int dir = (ud[0] < 0.5) ? -1 : 1;
        State edge = (dir > 0) ? right : left;

        // Build a subtree of 2^j leaves from the edge, in direction dir.
        const int n_leaves = 1 << j;
        double sub_log_w = -INFINITY;
        double sub_rho[32];
        for (int k = 0; k < D; ++k) sub_rho[k] = 0.0;
        State sub_prop = edge;
        bool sub_ok = true;
        // U-turn checkpoints: prefix momentum sum before and momentum at the
        // first leaf of every pending node of height l (l = 1 .. j).
        double ck_rho[16][32], ck_r[16][32];
        for (int n = 0; n < n_leaves; ++n) {
            leapfrog(t, beta, L, dir * eps, edge);
            out.n_leapfrog++;
            const double h = -edge.logp + kinetic(D, L, edge.r);
            const double dh = h - h0;
            accept_sum += (std::isfinite(dh) ? std::min(1.0, std::exp(-dh)) : 0.0);
            if (!std::isfinite(dh) || dh > max_dh) {
                out.divergent = 1;
                sub_ok = false;
                break;
            }
            for (int l = 1; l <= j; ++l)
                if ((n & ((1 << l) - 1)) == 0) {
                    for (int k = 0; k < D; ++k) { ck_rho[l][k] = sub_rho[k]; ck_r[l][k] = edge.r[k]; }
                }
            for (int k = 0; k < D; ++k) sub_rho[k] += edge.r[k];
            // Uniform progressive sampling inside the subtree.
            const double lw = -dh;
            const double new_log_w = log_add_exp(sub_log_w, lw);
            double ul[2];
            uniforms2(seed, leaf_counter++, particle, iteration, PURPOSE_LEAF, ul);
            if (ul[0] < std::exp(lw - new_log_w)) sub_prop = edge;
            sub_log_w = new_log_w;
            // Close every node that this leaf completes and check it for a U-turn.
            if (uturn) {
                for (int l = 1; l <= j; ++l) {
                    if (((n + 1) & ((1 << l) - 1)) == 0) {
                        double node_rho[32];
                        for (int k = 0; k < D; ++k) node_rho[k] = sub_rho[k] - ck_rho[l][k];
                        if (!no_uturn(D, L, node_rho, ck_r[l], edge.r)) { sub_ok = false; break; }
                    }
                }
                if (!sub_ok) break;
            }
        }
        if (!sub_ok) break;  // a rejected subtree contributes nothing
        out.depth = j + 1;
        // Biased progressive sampling at the top level.
        if (ud[1] < std::exp(sub_log_w - log_w)) prop = sub_prop;
        log_w = log_add_exp(log_w, sub_log_w);
        for (int k = 0; k < D; ++k) rho[k] += sub_rho[k];
        if (dir > 0) right = edge; else left = edge;
        if (uturn && !no_uturn(D, L, rho, left.r, right.r)) break;
    }
    out.accept_stat = out.n_leapfrog > 0 ? accept_sum / out.n_leapfrog : 0.0;
    cur = prop;
    return out;
}

double lse(const double* x, int n, double scale) {
    double m = -INFINITY;
    for (int i = 0; i < n; ++i) m = std::max(m, scale * x[i]);
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::exp(scale * x[i] - m);
    return m + std::log(s);
}

// ESS of the incremental weights w_i = L_i^db, from log-sum-exps.
double ess_of(const double* logl, int n, double db) {
    std::vector<double> lw(n);
    for (int i = 0; i < n; ++i) lw[i] = db * logl[i];
    const double a = lse(lw.data(), n, 1.0), b = lse(lw.data(), n, 2.0);
    return std::exp(2.0 * a - b);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

// Threads of the oracle's parallel loops (timing on a chosen number of cores).
int orc_set_num_threads(int n) {
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}

int orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
    return 0;
}

int orc_uniforms2(uint64_t seed, uint32_t index, uint32_t particle, uint64_t iteration, uint32_t purpose, double* u) {
    uniforms2(seed, index, particle, iteration, purpose, u);
    return 0;
}

// Antenna pattern and delay: out = {F+, Fx, delay}.
int orc_antenna(const orc_detector* det, double ra, double dec, double psi, double gmst, double c_light, double* out) {
    double fp, fc, dt;
    antenna<double>(*det, ra, dec, psi, gmst, c_light, fp, fc, dt);
    out[0] = fp; out[1] = fc; out[2] = dt;
    return 0;
}

// Detector position [3] and response tensor [3][3].
int orc_detector_geometry(const orc_detector* det, double* pos, double* resp) {
    double D[3][3];
    detector_geometry(*det, pos, D);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) resp[3 * i + j] = D[i][j];
    return 0;
}

// SPA phase Psi(f) [rad] at n frequencies; theta11 in the 11-parameter order.
int orc_phase(const double* theta11, double t_sun, int pn_order, int n, const double* f, double* psi) {
    for (int i = 0; i < n; ++i)
        psi[i] = taylorf2_phase<double>(theta11[0], theta11[1], theta11[2], theta11[3], theta11[9], theta11[10],
                                        f[i], t_sun, pn_order);
    return 0;
}

// Projected strain of every detector, h_reim [n_det][N][2].
int orc_waveform(const orc_event* ev, const orc_detector* dets, const double* theta11, double* h_reim) {
    for (int d = 0; d < ev->n_det; ++d)
        for (int j = 0; j < ev->n_bins; ++j) {
            const Cx<double> h = detector_strain<double>(*ev, dets[d], theta11, ev->f_low + ev->df * j);
            h_reim[2 * ((size_t)d * ev->n_bins + j)] = h.re;
            h_reim[2 * ((size_t)d * ev->n_bins + j) + 1] = h.im;
        }
    return 0;
}

// logL (and optionally its gradient) for P points of a target.
int orc_loglike_grad(const orc_target* t, int P, const double* x, double* logl, double* grad) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < P; ++i)
        logl[i] = target_loglike(*t, x + (size_t)i * t->dim, grad ? grad + (size_t)i * t->dim : nullptr);
    return 0;
}

int orc_logprior(const orc_target* t, int P, const double* x, double* lp, double* grad) {
    for (int i = 0; i < P; ++i)
        lp[i] = target_logprior(*t, x + (size_t)i * t->dim, grad ? grad + (size_t)i * t->dim : nullptr);
    return 0;
}

// The drift of one leapfrog step, x += eps M^{-1} r inside the box, in place
// for P points (positions x, momenta r) with M^{-1} = chol chol^T (chol
// [D][D], shared by the points).
int orc_drift(const orc_target* t, int P, const double* chol, double eps, double* x, double* r) {
    for (int i = 0; i < P; ++i) drift(*t, chol, eps, x + (size_t)i * t->dim, r + (size_t)i * t->dim);
    return 0;
}

// n_steps leapfrog steps of one point; x, r updated in place; returns H at the end.
int orc_leapfrog(const orc_target* t, double beta, const double* chol, double eps, int n_steps,
                 double* x, double* r, double* energy) {
    State s;
    const int D = t->dim;
    for (int k = 0; k < D; ++k) { s.x[k] = x[k]; s.r[k] = r[k]; }
    eval_state(*t, beta, s);
    energy[0] = -s.logp + kinetic(D, chol, s.r);
    for (int n = 0; n < n_steps; ++n) leapfrog(*t, beta, chol, eps, s);
    for (int k = 0; k < D; ++k) { x[k] = s.x[k]; r[k] = s.r[k]; }
    energy[1] = -s.logp + kinetic(D, chol, s.r);
    return 0;
}

// One NUTS transition for each of P particles.  logl / grad are the
// likelihood and its gradient at x (updated with the selected point).
// chol is one [D][D] factor of M^{-1} shared by all particles, or, with
// chol_per_particle, [P][D][D] (one factor per particle).
int orc_nuts_step(const orc_target* t, int P, double* x, double* logl, double* grad, const double* chol,
                  int chol_per_particle, double step, int max_depth, const int32_t* max_depth_per_particle, int uturn,
                  double max_dh, double beta, uint64_t seed, uint64_t iteration,
                  int32_t* depth, int32_t* n_leapfrog, uint8_t* divergent, double* accept_stat,
                  const int32_t* particle_ids) {
    const int D = t->dim;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < P; ++i) {
        State s;
        for (int k = 0; k < D; ++k) s.x[k] = x[(size_t)i * D + k];
        eval_state(*t, beta, s);
        const int md = max_depth_per_particle ? max_depth_per_particle[i] : max_depth;
        const double* Li = chol_per_particle ? chol + (size_t)i * D * D : chol;
        // random streams of particle particle_ids[i] (i when NULL): a sample of a larger batch replays its own draws
        const uint32_t pid = particle_ids ? (uint32_t)particle_ids[i] : (uint32_t)i;
        const NutsOut o = nuts_transition(*t, beta, Li, step, md, uturn, max_dh, seed, iteration, pid, s);
        logl[i] = s.logl;
        for (int k = 0; k < D; ++k) { x[(size_t)i * D + k] = s.x[k]; if (grad) grad[(size_t)i * D + k] = s.gl[k]; }
        if (depth) depth[i] = o.depth;
        if (n_leapfrog) n_leapfrog[i] = o.n_leapfrog;
        if (divergent) divergent[i] = (uint8_t)o.divergent;
        if (accept_stat) accept_stat[i] = o.accept_stat;
    }
    return 0;
}

// Adaptive temperature: ESS(beta) = alpha P solved by bisection on
// [beta_prev, 1] (lower end returned); evidence increment and normalised
// weights of the new temperature.  Returns -6 on a stalled ladder.
int orc_smc_reweight(int P, const double* logl, double beta_prev, double alpha,
                     double* beta_next, double* dlogz, double* weights) {
    const double target = alpha * P;
    double beta;
    if (ess_of(logl, P, 1.0 - beta_prev) >= target) {
        beta = 1.0;
    } else {
        double lo = beta_prev, hi = 1.0;
        for (int it = 0; it < 100 && hi - lo > 1e-14; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (ess_of(logl, P, mid - beta_prev) >= target) lo = mid; else hi = mid;
        }
        beta = lo;
    }
    std::vector<double> lw(P);
    const double db = beta - beta_prev;
    for (int i = 0; i < P; ++i) lw[i] = db * logl[i];
    const double l = lse(lw.data(), P, 1.0);
    *beta_next = beta;
    *dlogz = l - std::log((double)P);
    for (int i = 0; i < P; ++i) weights[i] = std::exp(lw[i] - l);
    return (beta <= beta_prev) ? -6 : 0;
}

// Multinomial resampling: ancestor_i = first k with cumsum_k > u_i.
int orc_resample(int P, const double* weights, uint64_t seed, uint64_t iteration, int32_t* ancestors) {
    std::vector<double> cum(P);
    double s = 0.0;
    for (int i = 0; i < P; ++i) { s += weights[i]; cum[i] = s; }
    for (int i = 0; i < P; ++i) cum[i] /= s;
    cum[P - 1] = 1.0;
    for (int i = 0; i < P; ++i) {
        double u[2];
        uniforms2(seed, 0u, (uint32_t)i, iteration, PURPOSE_RESAMPLE, u);
        int k = (int)(std::upper_bound(cum.begin(), cum.end(), u[0]) - cum.begin());
        ancestors[i] = std::min(k, P - 1);
    }
    return 0;
}

// Population covariance with diagonal shrinkage, its Cholesky factor.
// Returns 1 when the factorisation failed and a diagonal fallback was used.
int orc_mass_matrix(int P, int D, const double* x, double shrink, double* inv_mass, double* chol) {
    std::vector<double> mu(D, 0.0);
    for (int i = 0; i < P; ++i) for (int k = 0; k < D; ++k) mu[k] += x[(size_t)i * D + k];
    for (int k = 0; k < D; ++k) mu[k] /= P;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int i = 0; i < P; ++i) s += (x[(size_t)i * D + a] - mu[a]) * (x[(size_t)i * D + b] - mu[b]);
            inv_mass[a * D + b] = s / (P - 1);
        }
    for (int k = 0; k < D; ++k) inv_mass[k * D + k] *= (1.0 + shrink);
    int status = 0;
    for (int i = 0; i < D * D; ++i) chol[i] = 0.0;
    for (int j = 0; j < D && status == 0; ++j) {
        double s = inv_mass[j * D + j];
        for (int k = 0; k < j; ++k) s -= chol[j * D + k] * chol[j * D + k];
        if (!(s > 0.0)) { status = 1; break; }
        chol[j * D + j] = std::sqrt(s);
        for (int i = j + 1; i < D; ++i) {
            double t = inv_mass[i * D + j];
            for (int k = 0; k < j; ++k) t -= chol[i * D + k] * chol[j * D + k];
            chol[i * D + j] = t / chol[j * D + j];
        }
    }
    if (status) {
        for (int i = 0; i < D * D; ++i) chol[i] = 0.0;
        for (int k = 0; k < D; ++k) {
            double v = inv_mass[k * D + k];
            if (!(v > 0.0)) v = 1.0;
            for (int b = 0; b < D; ++b) inv_mass[k * D + b] = (b == k) ? v : 0.0;
            chol[k * D + k] = std::sqrt(v);
        }
    }
    return status;
}

// Local-geometry metric of Sec. 5 ("Exploitation of local geometry"): the
// mass matrix of each particle is the Hessian of the tempered posterior's
// negative log density at the particle, read as beta F + diag(prior
// precision), with F the Fisher (Gauss-Newton) matrix of the likelihood,
// F_kl = sum_d 4 df sum_j Re(conj(dh_dj/dtheta_k) dh_dj/dtheta_l) / S_dj,
// from 11-tangent dual numbers of the strain, and the prior precision the
// inverse variance of each coordinate's prior (uniform (hi-lo)^2/12,
// log-uniform its variance, Gaussian sigma^2; 0 for a flat prior).  For the
// analytic test likelihoods F is the exact Hessian of -log L instead (see
// analytic_hessian).  Outputs per particle: fisher [D][D] (may be NULL) and
// chol [D][D], the lower Cholesky factor of M^{-1}.  A particle whose M or M^{-1}
// is not numerically positive definite takes fallback [D][D] (the identity
// when NULL) and status[i] = 1 (status may be NULL).  Returns the number of
// such particles.
// Exact Hessian of -log L of the analytic test likelihoods at x, H [D][D]:
// the standard normal gives the identity, the Gaussian likelihood N(y; x,
// sigma_l^2) gives diag(1 / sigma_l^2), and the unweighted sum of two
// isotropic Gaussians N(m1, s^2) + N(m2, s^2) gives
//   I / s^2 - r1 r2 (m1 - m2)(m1 - m2)^T / s^4
// with r_i = N_i / (N_1 + N_2) the components' shares at x (the Hessian of
// log sum_i N_i is the shares' mean of the components' Hessians plus the
// shares' covariance of their gradients (m_i - x) / s^2).
static void analytic_hessian(const orc_target& t, const double* x, double* H) {
    const int D = t.dim;
    for (int i = 0; i < D * D; ++i) H[i] = 0.0;
    if (t.kind == 1) {
        for (int k = 0; k < D; ++k) H[k * D + k] = 1.0;
    } else if (t.kind == 2) {
        const double* sg = t.params + D;
        for (int k = 0; k < D; ++k) H[k * D + k] = 1.0 / (sg[k] * sg[k]);
    } else {
        const double* m1 = t.params; const double* m2 = t.params + D; const double sg = t.params[2 * D];
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < D; ++k) {
            s1 += (x[k] - m1[k]) * (x[k] - m1[k]);
            s2 += (x[k] - m2[k]) * (x[k] - m2[k]);
        }
        // r1 = 1 / (1 + exp(l2 - l1)), with l_i = -s_i / (2 s^2) (common factors cancel)
        const double r1 = 1.0 / (1.0 + std::exp(-0.5 * (s2 - s1) / (sg * sg))), r2 = 1.0 - r1;
        const double s4 = sg * sg * sg * sg;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                H[a * D + b] = (a == b ? 1.0 / (sg * sg) : 0.0) - r1 * r2 * (m1[a] - m2[a]) * (m1[b] - m2[b]) / s4;
    }
}

int orc_local_metric(const orc_target* t, int P, const double* x, double beta, const double* fallback, double* fisher,
                     double* chol, int32_t* status) {
    if (t->kind < 0 || t->kind > 3) return -1;
    const int D = t->dim;
    std::vector<double> prec(D, 0.0);
    for (int k = 0; k < D; ++k) {
        const orc_bound& b = t->bounds[k];
        if (b.prior == 1) {
            prec[k] = 12.0 / ((b.hi - b.lo) * (b.hi - b.lo));
        } else if (b.prior == 2) {
            const double lr = std::log(b.hi / b.lo);
            const double m1 = (b.hi - b.lo) / lr, m2 = (b.hi * b.hi - b.lo * b.lo) / (2.0 * lr);
            prec[k] = 1.0 / (m2 - m1 * m1);
        } else if (b.prior == 3) {
            prec[k] = 1.0 / (b.hi * b.hi);
        }
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int i = 0; i < P; ++i) {
        std::vector<double> F((size_t)D * D);
        if (t->kind == 0) {
            double th[NP];
            expand_gw(*t, x + (size_t)i * D, th);
            D11 td[NP];
            for (int k = 0; k < NP; ++k) { td[k] = D11(th[k]); td[k].d[k] = 1.0; }
            const orc_event& ev = *t->ev;
            double F11[NP][NP] = {};
            for (int d = 0; d < ev.n_det; ++d)
                for (int j = 0; j < ev.n_bins; ++j) {
                    const double f = ev.f_low + ev.df * j;
                    const Cx<D11> h = detector_strain(ev, t->dets[d], td, f);
                    const double w = 4.0 * ev.df / t->psd[(size_t)d * ev.n_bins + j];
                    for (int a = 0; a < NP; ++a)
                        for (int b = 0; b < NP; ++b)
                            F11[a][b] += w * (h.re.d[a] * h.re.d[b] + h.im.d[a] * h.im.d[b]);
                }
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) {
                    const int ia = t->param_index ? t->param_index[a] : a, ib = t->param_index ? t->param_index[b] : b;
                    F[a * D + b] = F11[ia][ib];
                }
        } else {
            analytic_hessian(*t, x + (size_t)i * D, F.data());
        }
        std::vector<double> M((size_t)D * D), R((size_t)D * D, 0.0), Minv((size_t)D * D), Lo((size_t)D * D, 0.0);
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                if (fisher) fisher[(size_t)i * D * D + a * D + b] = F[a * D + b];
                M[a * D + b] = beta * F[a * D + b] + (a == b ? prec[a] : 0.0);
            }
        // M = R R^T, then M^{-1} column by column (R y = e_j, R^T z = y), then M^{-1} = L L^T.
        bool ok = true;
        for (int j = 0; j < D && ok; ++j) {
            double sjj = M[j * D + j];
            for (int k = 0; k < j; ++k) sjj -= R[j * D + k] * R[j * D + k];
            if (!(sjj > 0.0)) { ok = false; break; }
            R[j * D + j] = std::sqrt(sjj);
            for (int r = j + 1; r < D; ++r) {
                double v = M[r * D + j];
                for (int k = 0; k < j; ++k) v -= R[r * D + k] * R[j * D + k];
                R[r * D + j] = v / R[j * D + j];
            }
        }
        if (ok) {
            for (int c = 0; c < D; ++c) {
                double y[32], z[32];
                for (int r = 0; r < D; ++r) {
                    double v = (r == c) ? 1.0 : 0.0;
                    for (int k = 0; k < r; ++k) v -= R[r * D + k] * y[k];
                    y[r] = v / R[r * D + r];
                }
                for (int r = D - 1; r >= 0; --r) {
                    double v = y[r];
                    for (int k = r + 1; k < D; ++k) v -= R[k * D + r] * z[k];
                    z[r] = v / R[r * D + r];
                }
                for (int r = 0; r < D; ++r) Minv[r * D + c] = z[r];
            }
            for (int j = 0; j < D && ok; ++j) {
                double sjj = Minv[j * D + j];
                for (int k = 0; k < j; ++k) sjj -= Lo[j * D + k] * Lo[j * D + k];
                if (!(sjj > 0.0)) { ok = false; break; }
                Lo[j * D + j] = std::sqrt(sjj);
                for (int r = j + 1; r < D; ++r) {
                    double v = Minv[r * D + j];
                    for (int k = 0; k < j; ++k) v -= Lo[r * D + k] * Lo[j * D + k];
                    Lo[r * D + j] = v / Lo[j * D + j];
                }
            }
        }
        // A particle whose M or M^{-1} is not numerically positive definite
        // takes the fallback factor (the identity when none is given).
        if (!ok) {
            bad += 1;
            for (int k = 0; k < D * D; ++k) Lo[k] = fallback ? fallback[k] : (k % (D + 1) == 0 ? 1.0 : 0.0);
        }
        if (status) status[i] = ok ? 0 : 1;
        for (int k = 0; k < D * D; ++k) chol[(size_t)i * D * D + k] = Lo[k];
    }
    return bad;
}

// Sample recycling (Sec. 5, "Samples recycling"): the populations left by the
// mutations of iterations t = 1..T are pooled and read as draws of the
// mixture (1/T) sum_t p_t, each p_t = L^beta_t pi / Z_t normalised with the
// evidence reached at iteration t.  A pooled point's importance weight for
// the final target p_T = L pi / Z_T against that mixture is
//   w = (L / Z_T) / ((1/T) sum_t L^beta_t / Z_t)
// (the prior cancels); rejection sampling then keeps point i when
// u_i < w_i / max_j w_j, giving i.i.d. draws of p_T.  logl [T][N] (NaN or
// -inf: weight zero), betas [T], logz [T] = log Z_t.  Outputs: logw [T*N],
// accepted [T*N] (the kept pool indices in increasing order, *n_accepted of
// them) and *ess = (sum w)^2 / sum w^2.  u_i is the first uniform of the
// Philox pair (seed; index 0, particle i, iteration 0, purpose RECYCLE).
int orc_recycle(int T, int N, const double* logl, const double* betas, const double* logz, uint64_t seed,
                double* logw, int32_t* accepted, int* n_accepted, double* ess) {
    if (T < 1 || N < 1) return -1;
    const size_t n = (size_t)T * N;
    for (size_t i = 0; i < n; ++i) {
        const double l = logl[i];
        if (!(l > -INFINITY)) { logw[i] = -INFINITY; continue; }   // also NaN
        double m = -INFINITY;
        for (int t = 0; t < T; ++t) m = std::max(m, betas[t] * l - logz[t]);
        double s = 0.0;
        for (int t = 0; t < T; ++t) s += std::exp(betas[t] * l - logz[t] - m);
        const double log_mix = m + std::log(s) - std::log((double)T);
        logw[i] = l - logz[T - 1] - log_mix;
    }
    double wmax = -INFINITY;
    for (size_t i = 0; i < n; ++i) wmax = std::max(wmax, logw[i]);
    double s1 = 0.0, s2 = 0.0;
    int k = 0;
    for (size_t i = 0; i < n; ++i) {
        const double w = std::exp(logw[i] - wmax);
        s1 += w;
        s2 += w * w;
        double u[2];
        uniforms2(seed, 0u, (uint32_t)i, 0u, PURPOSE_RECYCLE, u);
        if (u[0] < w) accepted[k++] = (int32_t)i;
    }
    *n_accepted = k;
    *ess = s2 > 0.0 ? s1 * s1 / s2 : 0.0;
    return 0;
}

// Bin edges of relative binning (criterion of Zackay, Dai & Venumadhav 2018):
// the phase difference between waveforms that the prior allows is bounded by
//   dpsi(f) = 2 pi chi sum_k sgn(g_k) (f / f*_k)^g_k,
//   g_k in {-5/3, -2/3, 1, 5/3, 7/3},  f*_k = f_min (g_k < 0) or f_max (g_k > 0),
// with chi = 1 (each power law moves the phase by at most 2 pi where it is
// largest); dpsi grows monotonically.  The band is cut into
// B = ceil((dpsi(f_max) - dpsi(f_min)) / eps) bins of equal growth: edge k
// (0 < k < B) is the first grid point with dpsi - dpsi(f_min) >= k/B of the
// total; edge 0 is the first grid point, edge B the last.  Repeated edges are
// dropped.  Writes at most cap edges (grid indices); returns their number or
// -1 on bad arguments.
int orc_rb_edges(double f_low, double df, int n, double eps, int32_t* edges, int cap) {
    if (n < 2 || !(df > 0.0) || !(f_low > 0.0) || !(eps > 0.0) || cap < 2) return -1;
    const double g[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    const double fmin = f_low, fmax = f_low + df * (n - 1);
    auto dpsi = [&](double f) {
        double s = 0.0;
        for (int k = 0; k < 5; ++k) s += (g[k] < 0 ? -1.0 : 1.0) * std::pow(f / (g[k] < 0 ? fmin : fmax), g[k]);
        return 2.0 * PI * s;
    };
    const double p0 = dpsi(fmin), total = dpsi(fmax) - p0;
    long nb = (long)std::ceil(total / eps);
    if (nb < 1) nb = 1;
    if (nb > n - 1) nb = n - 1;
    int m = 0;
    edges[m++] = 0;
    int j = 0;
    for (long k = 1; k < nb; ++k) {
        const double target = total * (double)k / (double)nb;
        while (j < n - 1 && dpsi(f_low + df * j) - p0 < target) ++j;
        if (j >= n - 1) break;
        if (j > edges[m - 1]) {
            if (m >= cap - 1) return -1;
            edges[m++] = j;
        }
    }
    edges[m++] = n - 1;
    return m;
}

// Summary data of relative binning for the fiducial parameters theta0 (11):
// sums [n_det][n_edges - 1][4] (A0, A1 of every bin, see gw_loglike_rb) and
// h0 [n_det][n_edges][2] (the fiducial strain at the edges).
int orc_rb_prepare(const orc_event* ev, const orc_detector* dets, const double* data_reim, const double* psd,
                   const double* theta0, int n_edges, const int32_t* edges, double* sums, double* h0) {
    if (n_edges < 2) return -1;
    const int n = ev->n_bins, nb = n_edges - 1;
    for (int d = 0; d < ev->n_det; ++d) {
        for (int e = 0; e < n_edges; ++e) {
            const Cx<double> h = detector_strain<double>(*ev, dets[d], theta0, ev->f_low + ev->df * edges[e]);
            h0[2 * ((size_t)d * n_edges + e)] = h.re;
            h0[2 * ((size_t)d * n_edges + e) + 1] = h.im;
        }
        for (int b = 0; b < nb; ++b) {
            const int j0 = edges[b], j1 = (b == nb - 1) ? edges[b + 1] + 1 : edges[b + 1];
            const double fb = ev->f_low + ev->df * j0;
            double a[4] = {0.0, 0.0, 0.0, 0.0};
            for (int j = j0; j < j1; ++j) {
                const double f = ev->f_low + ev->df * j;
                const Cx<double> hz = detector_strain<double>(*ev, dets[d], theta0, f);
                const double* x = data_reim + 2 * ((size_t)d * n + j);
                const double w = 4.0 * ev->df / psd[(size_t)d * n + j];
                const double re = w * (x[0] * hz.re + x[1] * hz.im);   // 4 df conj(d) h0 / S
                const double im = w * (x[0] * hz.im - x[1] * hz.re);
                a[0] += re;
                a[1] += im;
                a[2] += re * (f - fb);
                a[3] += im * (f - fb);
            }
            for (int k = 0; k < 4; ++k) sums[4 * ((size_t)d * nb + b) + k] = a[k];
        }
    }
    return 0;
}

// Persistent sampling (Karamanis & Seljak 2024, arXiv:2407.20722; the SMC
// variant named as future work in Sec. 7).  Every earlier population stays in
// a pool: iteration s contributed N points drawn from p_s = L^beta_s pi / Z_s
// (s = 0 is the prior sample, beta_0 = 0, Z_0 = 1), and the pool of T
// populations is read as draws of the mixture (1/T) sum_s p_s.  The next
// temperature's unnormalised weights over the pool are
//   w_i(beta) = L_i^beta / ((1/T) sum_s L_i^beta_s / Z_s)
// (the prior cancels).  beta_next solves ESS(beta) = alpha N (N points per
// population; beta_next = 1 when ESS(1) >= alpha N), by the same bisection
// as orc_smc_reweight, and the evidence is the pool mean of the weights,
//   Z(beta_next) = (1 / (T N)) sum_i w_i(beta_next).
// logl [T][N], betas [T], logz [T] (log Z_s).  Outputs: *beta_next,
// *logz_next and weights [T*N] normalised to sum one.  Non-finite log L:
// weight zero.  Returns -6 when beta cannot advance.
int orc_ps_reweight(int T, int N, const double* logl, const double* betas, const double* logz, double beta_prev,
                    double alpha, double* beta_next, double* logz_next, double* weights) {
    if (T < 1 || N < 1) return -1;
    const int n = T * N;
    std::vector<double> lmix(n), lw(n);
    for (int i = 0; i < n; ++i) {
        const double l = logl[i];
        if (!(l > -INFINITY)) { lmix[i] = NAN; continue; }
        std::vector<double> terms(T);
        for (int t = 0; t < T; ++t) terms[t] = betas[t] * l - logz[t];
        lmix[i] = lse(terms.data(), T, 1.0) - std::log((double)T);
    }
    auto logw = [&](double beta, std::vector<double>& out) {
        for (int i = 0; i < n; ++i) out[i] = (logl[i] > -INFINITY) ? beta * logl[i] - lmix[i] : -INFINITY;
    };
    auto ess = [&](double beta) {
        logw(beta, lw);
        const double a = lse(lw.data(), n, 1.0), b = lse(lw.data(), n, 2.0);
        return std::exp(2.0 * a - b);
    };
    const double target = alpha * N;
    double beta;
    if (ess(1.0) >= target) {
        beta = 1.0;
    } else {
        double lo = beta_prev, hi = 1.0;
        for (int it = 0; it < 100 && hi - lo > 1e-14; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (ess(mid) >= target) lo = mid; else hi = mid;
        }
        beta = lo;
    }
    logw(beta, lw);
    const double l = lse(lw.data(), n, 1.0);
    *beta_next = beta;
    *logz_next = l - std::log((double)n);
    for (int i = 0; i < n; ++i) weights[i] = std::exp(lw[i] - l);
    return (beta <= beta_prev && beta_prev < 1.0) ? -6 : 0;
}

// n_draw multinomial draws from n_w weights (orc_resample with the two counts apart).
int orc_resample_n(int n_w, const double* weights, int n_draw, uint64_t seed, uint64_t iteration, int32_t* ancestors) {
    std::vector<double> cum(n_w);
    double s = 0.0;
    for (int i = 0; i < n_w; ++i) { s += weights[i]; cum[i] = s; }
    for (int i = 0; i < n_w; ++i) cum[i] /= s;
    cum[n_w - 1] = 1.0;
    for (int i = 0; i < n_draw; ++i) {
        double u[2];
        uniforms2(seed, 0u, (uint32_t)i, iteration, PURPOSE_RESAMPLE, u);
        int k = (int)(std::upper_bound(cum.begin(), cum.end(), u[0]) - cum.begin());
        ancestors[i] = std::min(k, n_w - 1);
    }
    return 0;
}

// A full SMC run: adaptive tempering, multinomial resampling, covariance mass
// matrix, one NUTS transition per iteration; stops after mutating at beta = 1.
// x [P][D] holds the prior draws on entry and the final population on exit.
int orc_smc_run(const orc_target* t, int P, double* x, double alpha, double step, int max_depth, double shrink,
                uint64_t seed, int max_iter, double* logz, int* n_iter, double* betas, double* dlogzs) {
    const int D = t->dim;
    std::vector<double> logl(P), w(P), xn((size_t)P * D), ll2(P), inv((size_t)D * D), L((size_t)D * D);
    std::vector<int32_t> anc(P);
    orc_loglike_grad(t, P, x, logl.data(), nullptr);
    double beta = 0.0, lz = 0.0;
    int it = 0;
    while (beta < 1.0 && it < max_iter) {
        double bn, dz;
        const int rc = orc_smc_reweight(P, logl.data(), beta, alpha, &bn, &dz, w.data());
        if (rc < 0) return rc;
        lz += dz;
        betas[it] = bn;
        dlogzs[it] = dz;
        orc_resample(P, w.data(), seed, (uint64_t)it, anc.data());
        for (int i = 0; i < P; ++i) {
            for (int k = 0; k < D; ++k) xn[(size_t)i * D + k] = x[(size_t)anc[i] * D + k];
            ll2[i] = logl[anc[i]];
        }
        std::copy(xn.begin(), xn.end(), x);
        orc_mass_matrix(P, D, x, shrink, inv.data(), L.data());
        orc_nuts_step(t, P, x, ll2.data(), nullptr, L.data(), 0, step, max_depth, nullptr, 1, 1000.0, bn, seed,
                      (uint64_t)it, nullptr, nullptr, nullptr, nullptr, nullptr);
        std::copy(ll2.begin(), ll2.end(), logl.begin());
        beta = bn;
        ++it;
    }
    *logz = lz;
    *n_iter = it;
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

}  // extern "C"
