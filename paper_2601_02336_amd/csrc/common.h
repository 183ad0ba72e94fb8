// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smcgw.h"

namespace smcgw {

constexpr int NPAR = 11;            // source parameters
constexpr int MAXDET = SMCGW_MAX_DET;
constexpr int MAXDIM = SMCGW_MAX_DIM;
constexpr int NBASIS = 8;           // per-bin phase basis rows kept in the tables
constexpr int NCOEF = NBASIS + 1;   // + the constant term
constexpr int TABLE_PAD = 512;      // tables are zero-padded to a multiple of this many bins
constexpr double PI = 3.14159265358979323846;
constexpr double TWO_PI = 6.28318530717958647692;

// Source-parameter indices.
enum { P_MC = 0, P_Q, P_CHI1, P_CHI2, P_DL, P_IOTA, P_PSI, P_RA, P_DEC, P_TC, P_PHIC };

// Phase basis: the TaylorF2 phase in cycles is
//   Phi(f) = c_0 + sum_b c_b B_b(f) + f (t_c + dt_det)
// with B = {f^-5/3, f^-1, f^-2/3, f^-1/3, ln f, f^1/3, f^1/3 ln f, f^2/3}.  The
// tables keep three FP64 rows per bin, f, w = f^-1/3 and ln f; every basis
// value is a product of them (basis_rows).
enum { B_M53 = 0, B_M1, B_M23, B_M13, B_LN, B_P13, B_P13LN, B_P23 };
enum { ROW_F = 0, ROW_W = 1, ROW_LN = 2, NROWS = 3 };

__device__ __forceinline__ void basis_rows(double f, double w, double lnf, double B[8]) {
    const double w2 = w * w;
    const double w3 = w2 * w;
    const double u = f * w2;   // f^1/3
    B[B_M53] = w3 * w2;
    B[B_M1] = w3;
    B[B_M23] = w2;
    B[B_M13] = w;
    B[B_LN] = lnf;
    B[B_P13] = u;
    B[B_P13LN] = u * lnf;
    B[B_P23] = u * u;
}

// Cross-lane moves through the VALU's data-parallel-primitive (DPP) lanes:
// no LDS round trip, unlike a shuffle.  A double moves as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront in a fixed order: pairs and quads
// (quad permutations), rows of 16 (row rotations by 4 and 8), then the rows
// through the row-15 and row-31 broadcasts.  The total is valid in lane 63
// only (TOTAL_LANE).
constexpr int TOTAL_LANE = 63;
__device__ __forceinline__ double wave_total(double v) {
    v += dpp_move<0xb1>(v);    // quad_perm [1,0,3,2]
    v += dpp_move<0x4e>(v);    // quad_perm [2,3,0,1]
    v += dpp_move<0x124>(v);   // row_ror:4
    v += dpp_move<0x128>(v);   // row_ror:8
    v += dpp_move<0x142>(v);   // row_bcast:15
    v += dpp_move<0x143>(v);   // row_bcast:31
    return v;
}

// Wavefront totals of K per-lane values, written to out[idx[k]] (any address
// space) by lanes 0..7.  Three halving steps over lane bits 0-2 scatter the
// values: at each step a lane keeps one half of its list (by its lane bit) and
// adds the partner lane's copy of that half, the partner being the lane with the
// opposite bit and the same lower bits (xor 1, xor 2, a rotation by 4 inside
// the row of 16).  A lane then holds ceil(K/8) partial sums, which full sums
// over bits 3-5 (a rotation by 8 inside the row, then xor 16 and xor 32)
// complete.  A list of odd length pads its upper half with a zero.  The order
// of the additions is fixed, so the totals do not depend on anything but the
// inputs.  A halving step costs 7 instructions per kept value (selects of the
// sent and kept halves, two DPP moves, an add), so the reduction takes about
// 7 (K/2 + K/4 + K/8) + 9 K/8 instructions instead of 18 K for K separate
// wavefront sums.
template <int K>
__device__ __forceinline__ void wave_totals_to(const double (&v)[K], const int (&idx)[K], double* out) {
    constexpr int M1 = (K + 1) / 2, M2 = (M1 + 1) / 2, M3 = (M2 + 1) / 2;
    const int lane = threadIdx.x & 63;
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    double c1[M1], c2[M2], c3[M3];
#pragma unroll
    for (int k = 0; k < M1; ++k) {
        const double hi = k + M1 < K ? v[k + M1] : 0.0;
        const double send = b0 ? v[k] : hi;
        c1[k] = (b0 ? hi : v[k]) + dpp_move<0xb1>(send);   // quad_perm [1,0,3,2]
    }
#pragma unroll
    for (int k = 0; k < M2; ++k) {
        const double hi = k + M2 < M1 ? c1[k + M2] : 0.0;
        const double send = b1 ? c1[k] : hi;
        c2[k] = (b1 ? hi : c1[k]) + dpp_move<0x4e>(send);   // quad_perm [2,3,0,1]
    }
#pragma unroll
    for (int k = 0; k < M3; ++k) {
        const double hi = k + M3 < M2 ? c2[k + M3] : 0.0;
        const double send = b2 ? c2[k] : hi;
        c3[k] = (b2 ? hi : c2[k]) + dpp_move<0x124>(send);   // row_ror:4
    }
#pragma unroll
    for (int k = 0; k < M3; ++k) {
        double t = c3[k] + dpp_move<0x128>(c3[k]);   // row_ror:8
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        c3[k] = t;
    }
    if (lane < 8) {
#pragma unroll
        for (int k = 0; k < M3; ++k) {
            const int p2 = b2 ? k + M3 : k;
            const int p1 = b1 ? p2 + M2 : p2;
            const int p0 = b0 ? p1 + M1 : p1;
            if (p2 < M2 && p1 < M1 && p0 < K) out[idx[p0]] = c3[k];
        }
    }
}

__device__ __forceinline__ double wave_max_total(double v) {
    v = fmax(v, dpp_move<0xb1>(v));
    v = fmax(v, dpp_move<0x4e>(v));
    v = fmax(v, dpp_move<0x124>(v));
    v = fmax(v, dpp_move<0x128>(v));
    v = fmax(v, dpp_move<0x142>(v));
    v = fmax(v, dpp_move<0x143>(v));
    return v;
}

// Device view of one event's bin tables (frequency-major, padded to n_pad).
struct DevEvent {
    int n_bins, n_pad, n_det, pn_order;
    double f_low, df;
    const double* fwl;       // [NROWS][n_pad]: f, f^-1/3, ln f
    const float2* u32;       // [n_det][n_pad]  4 df conj(d) f^-7/6 / (S u_scale), FP32
    const double2* u64;      // [n_det][n_pad]  same in FP64
    double hnorm[MAXDET];    // sum_j 4 df f^-7/3 / S / u_scale^2
    double dd;               // sum_d <d|d>_d
    double u_scale;          // power of two keeping the FP32 table near unit magnitude
    double t_sun, mpc_m, c_light, gmst;
    double ln_pi_tsun;       // ln(pi G Msun / c^3)
    double pos[MAXDET][3];   // detector positions [m]
    double resp[MAXDET][3][3];
    const double* wmom;      // [n_det][NGEO][NGEO]: sum_j 4 df f^-7/3 / S / u_scale^2 g_a g_b (local metric)
    const double* wa2;       // [n_det][n_pad]: 4 df f^-7/3 / S / u_scale^2 per bin (plain form; NULL for a
                             // relative-binning event)
};

// Functions of f whose combination is the phase of detector d in cycles:
// g_0 = 1, g_{1+b} = basis row b, g_{NCOEF} = f (the delay term).
constexpr int NGEO = NCOEF + 1;

// Sampled-coordinate map into the 11 source parameters.
struct ParamMap {
    int dim;
    int idx[MAXDIM];
    double fixed[NPAR];
};

// Per-particle coefficient block written by the prologue kernel (FP64).
// The first CB_BINS entries are all the bin loop reads.
enum {
    CB_C = 0,                            // NCOEF phase coefficients (cycles): const, then basis rows
    CB_TAU = CB_C + NCOEF,               // MAXDET: t_c + delay of each detector
    CB_PR = CB_TAU + MAXDET,             // MAXDET: Re P_d (times CB_AMP in use)
    CB_PI = CB_PR + MAXDET,              // MAXDET: Im P_d
    CB_BINS = CB_PI + MAXDET,
    CB_DC = CB_BINS,                     // [NCOEF][4]: d c_b / d(Mc, q, chi1, chi2)
    CB_DTAU = CB_DC + 4 * NCOEF,         // [MAXDET][2]: d tau_d / d(ra, dec)
    CB_DPR = CB_DTAU + 2 * MAXDET,       // [MAXDET][4]: d Re P_d / d(iota, psi, ra, dec)
    CB_DPI = CB_DPR + 4 * MAXDET,        // [MAXDET][4]: d Im P_d / d(iota, psi, ra, dec)
    CB_DLNCA_MC = CB_DPI + 4 * MAXDET,   // d ln C_A / d Mc
    CB_DLNCA_DL = CB_DLNCA_MC + 1,       // d ln C_A / d d_L
    CB_AMP = CB_DLNCA_DL + 1,            // C_A u_scale: the projection P'_d = CB_AMP P_d
    CB_SIZE = 104
};
static_assert(CB_AMP < CB_SIZE, "coefficient block overflow");

// Per-particle bin moments written by the bin loop (FP64).
enum {
    MOM_ZR = 0,                 // MAXDET: Re Z_d = Re sum_j u_dj e^{-2 pi i Phi_dj}
    MOM_ZI = MOM_ZR + MAXDET,   // MAXDET: Im Z_d
    MOM_G = MOM_ZI + MAXDET,    // NCOEF: sum_j psibar_j B_b(f_j) (b = const first)
    MOM_T = MOM_G + NCOEF,      // MAXDET: sum_j q_dj f_j
    MOM_SIZE = 24
};
static_assert(MOM_T + MAXDET <= MOM_SIZE, "moment block overflow");

// Event index of particle p (out-of-range indices are clamped to a valid event).
__device__ __forceinline__ int event_index(const int32_t* ev_of_p, int p, int n_events) {
    if (!ev_of_p) return 0;
    const int e = ev_of_p[p];
    return e < 0 ? 0 : (e >= n_events ? n_events - 1 : e);
}

// ------------------------------------------------------------- host launchers
// (each .hip file exposes host functions; kernels stay in their own unit)
hipError_t launch_metric_moments(const double* d_psd, int n_det, int n_bins, double f_low, double df, double u_scale,
                                 double* wmom, hipStream_t s);
hipError_t launch_rb_tables(const double* fwl_full, const double2* u64_full, int n, int npad_full, int n_det,
                            const double* cb0, const int32_t* edges, int ne, double2* v, double2* a0, double2* a1,
                            int npad, double* fwl, float2* u32, double2* u64, hipStream_t s);
hipError_t launch_build_tables(const double* d_data, const double* d_psd, int n_det, int n_bins, int n_pad,
                               double f_low, double df, double u_scale, double* fwl, float2* u32, double2* u64,
                               double* wa2, double* sums, hipStream_t s);
hipError_t launch_prep(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                       const double* theta, double* cb, hipStream_t s);
// The bin loop and the epilogue of every particle: logl [P] and grad [P][pm.dim] (grad may be NULL).
hipError_t launch_bins(const DevEvent* d_events, int n_events, const int32_t* ev_of_p, const ParamMap& pm, int P,
                       int n_det, int precision, const double* cb, double* logl, double* grad, hipStream_t s);
hipError_t launch_waveform(const DevEvent* d_events, int event_id, const double* cb, double* h_reim, int n_bins,
                           int n_det, hipStream_t s);
int noalloc_init(int device);   // the fixed scratch of smcgw_loglike_grad_noalloc on this device

}  // namespace smcgw
