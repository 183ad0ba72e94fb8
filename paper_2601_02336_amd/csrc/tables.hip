// Event bin tables (built once per event, frequency-major).
//
// For the inner product of arXiv:2601.02336 Sec. 2 (Eq. 2) discretised on
// f_j = f_low + j df, every particle reuses the same per-bin quantities:
//   u_dj = 4 df conj(d_dj) f_j^-7/6 / S_dj            (whitened data x amplitude shape)
//   f_j, f_j^-1/3, ln f_j                           (phase basis generators)
//   H_d  = sum_j 4 df f_j^-7/3 / S_dj,  <d|d>_d = sum_j 4 df |d_dj|^2 / S_dj,
//   w_dj a_j^2 = 4 df f_j^-7/3 / S_dj per bin (the plain form's per-bin <h|h>).
// The tables are zero-padded to a multiple of TABLE_PAD bins; padded bins have
// u = 0 and finite basis values, so they add nothing to any sum.
#include "common.h"

namespace smcgw {

__global__ __launch_bounds__(256) void build_tables_kernel(const double* __restrict__ data, const double* __restrict__ psd,
                                                           int n_det, int n, int npad, double f_low, double df,
                                                           double inv_us, double* __restrict__ fwl,
                                                           float2* __restrict__ u32, double2* __restrict__ u64,
                                                           double* __restrict__ wa2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= npad) return;
    const double f = f_low + df * (double)j;
    fwl[(size_t)ROW_F * npad + j] = f;
    fwl[(size_t)ROW_W * npad + j] = 1.0 / cbrt(f);
    fwl[(size_t)ROW_LN * npad + j] = log(f);
    const double a = pow(f, -7.0 / 6.0);
    for (int d = 0; d < n_det; ++d) {
        double ur = 0.0, ui = 0.0, h = 0.0;
        if (j < n) {
            const double w = 4.0 * df / psd[(size_t)d * n + j];
            const double* dd = data + 2 * ((size_t)d * n + j);
            ur = w * a * dd[0] * inv_us;
            ui = -w * a * dd[1] * inv_us;
            h = w * a * a * inv_us * inv_us;
        }
        u64[(size_t)d * npad + j] = make_double2(ur, ui);
        wa2[(size_t)d * npad + j] = h;
        u32[(size_t)d * npad + j] = make_float2((float)ur, (float)ui);
    }
}

// One workgroup per detector: sums[2d] = H_d, sums[2d+1] = <d|d>_d (fixed-order tree).
__global__ __launch_bounds__(256) void table_sums_kernel(const double* __restrict__ data, const double* __restrict__ psd,
                                                         int n, double f_low, double df, double* __restrict__ sums) {
    __shared__ double sh[2][256];
    const int d = blockIdx.x;
    double h = 0.0, dd = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double f = f_low + df * (double)j;
        const double w = 4.0 * df / psd[(size_t)d * n + j];
        const double a = pow(f, -7.0 / 6.0);
        const double* x = data + 2 * ((size_t)d * n + j);
        h += w * a * a;
        dd += w * (x[0] * x[0] + x[1] * x[1]);
    }
    sh[0][threadIdx.x] = h;
    sh[1][threadIdx.x] = dd;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[2 * d] = sh[0][0];
        sums[2 * d + 1] = sh[1][0];
    }
}

// Basis moments of the local metric, one workgroup per detector:
// W_d[a][b] = sum_j 4 df f_j^-7/3 / S_dj / u_scale^2 g_a(f_j) g_b(f_j) with the
// phase functions g (g_0 = 1, the basis rows, f).  The metric of a particle
// is a quadratic form of these per-event sums (the Fisher matrix of a
// Newtonian-amplitude waveform needs no per-particle bin loop).  Fixed-order
// sums: per-thread partials, then the threads in index order.
constexpr int MOM_THREADS = 256;
constexpr int NGEO_PAIRS = NGEO * (NGEO + 1) / 2;

__global__ __launch_bounds__(MOM_THREADS) void metric_moments_kernel(const double* __restrict__ psd, int n,
                                                                     double f_low, double df, double inv_us2,
                                                                     double* __restrict__ wmom) {
    __shared__ double part[MOM_THREADS];
    const int d = blockIdx.x;
    double acc[NGEO_PAIRS];
#pragma unroll
    for (int e = 0; e < NGEO_PAIRS; ++e) acc[e] = 0.0;
    for (int j = threadIdx.x; j < n; j += MOM_THREADS) {
        const double f = f_low + df * (double)j;
        const double a = pow(f, -7.0 / 6.0);
        const double w = 4.0 * df / psd[(size_t)d * n + j] * a * a * inv_us2;
        double g[NGEO];
        double B[NBASIS];
        basis_rows(f, 1.0 / cbrt(f), log(f), B);
        g[0] = 1.0;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) g[1 + b] = B[b];
        g[NGEO - 1] = f;
        int e = 0;
#pragma unroll
        for (int x = 0; x < NGEO; ++x)
#pragma unroll
            for (int y = 0; y <= x; ++y) acc[e++] += w * g[x] * g[y];
    }
    int e = 0;
#pragma unroll
    for (int x = 0; x < NGEO; ++x)
#pragma unroll
        for (int y = 0; y <= x; ++y) {
            part[threadIdx.x] = acc[e++];   // unrolled: acc stays in registers
            __syncthreads();
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int t = 0; t < MOM_THREADS; ++t) s += part[t];
                wmom[((size_t)d * NGEO + x) * NGEO + y] = s;
                wmom[((size_t)d * NGEO + y) * NGEO + x] = s;
            }
            __syncthreads();
        }
}

hipError_t launch_metric_moments(const double* d_psd, int n_det, int n_bins, double f_low, double df, double u_scale,
                                 double* wmom, hipStream_t s) {
    hipLaunchKernelGGL(metric_moments_kernel, dim3(n_det), dim3(MOM_THREADS), 0, s, d_psd, n_bins, f_low, df,
                       1.0 / (u_scale * u_scale), wmom);
    return hipGetLastError();
}

// ------------------------------------------------------ relative binning
// Relative binning (Zackay, Dai & Venumadhav 2018, arXiv:1806.08792), the
// long-segment mitigation named in arXiv:2601.02336 (Secs. 2 and 7).  With
// the fiducial phase Phi0_d (in cycles) of parameters theta0 and
// rho_d(f) = e^{-2 pi i (Phi_d(f) - Phi0_d(f))} taken linear between the bin
// edges f_e, the data sum of the likelihood becomes
//   Z_d = sum_j u_dj e^{-2 pi i Phi_dj} = sum_j v_dj rho_d(f_j),  v_dj = u_dj e^{-2 pi i Phi0_dj}
//       ~ sum_b [a0_db rho_d(f_b) + a1_db (rho_d(f_b+1) - rho_d(f_b)) / (f_b+1 - f_b)]
//       = sum_e c_de rho_d(f_e) = sum_e u'_de e^{-2 pi i Phi_d(f_e)},
//   a0_db = sum_{j in b} v_dj,  a1_db = sum_{j in b} v_dj (f_j - f_b),
//   c_de = a0_de - a1_de / w_e + a1_d,e-1 / w_e-1,  u'_de = c_de e^{2 pi i Phi0_d(f_e)},
// so the likelihood on the edges is the ordinary bin loop over a table whose
// "bins" are the edges and whose data are u'.  |h|^2 does not depend on the
// phase for this waveform, so H_d and <d|d> keep their values over every bin.

__device__ __forceinline__ double phase_cycles(const double* cb, int d, double f, double w, double l) {
    double B[NBASIS];
    basis_rows(f, w, l, B);
    double ph = cb[CB_C];
    for (int b = 0; b < NBASIS; ++b) ph = fma(cb[CB_C + 1 + b], B[b], ph);
    return fma(f, cb[CB_TAU + d], ph);
}

// v_dj = u_dj e^{-2 pi i Phi0_dj} over the full grid (FP64).
__global__ __launch_bounds__(256) void rb_hetero_kernel(const double* __restrict__ fwl, const double2* __restrict__ u64,
                                                        int n, int npad, int n_det, const double* __restrict__ cb0,
                                                        double2* __restrict__ v) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double f = fwl[(size_t)ROW_F * npad + j];
    const double w = fwl[(size_t)ROW_W * npad + j];
    const double l = fwl[(size_t)ROW_LN * npad + j];
    for (int d = 0; d < n_det; ++d) {
        const double ph = phase_cycles(cb0, d, f, w, l);
        double sn, cs;
        sincospi(2.0 * (ph - rint(ph)), &sn, &cs);
        const double2 u = u64[(size_t)d * npad + j];
        v[(size_t)d * n + j] = make_double2(u.x * cs + u.y * sn, u.y * cs - u.x * sn);
    }
}

// a0, a1 of bin b, detector d: one workgroup, fixed-order sums (per-thread
// strided partials, then a tree).  Bin b holds the grid points
// [edges[b], edges[b+1]), the last bin also its end point.
constexpr int RB_THREADS = 256;
__global__ __launch_bounds__(RB_THREADS) void rb_sums_kernel(const double2* __restrict__ v,
                                                             const double* __restrict__ fwl, int n, int npad,
                                                             const int32_t* __restrict__ edges, int nb,
                                                             double2* __restrict__ a0, double2* __restrict__ a1) {
    __shared__ double sh[4][RB_THREADS];
    const int b = blockIdx.x, d = blockIdx.y;
    const int j0 = edges[b], j1 = (b == nb - 1) ? edges[b + 1] + 1 : edges[b + 1];
    const double fb = fwl[(size_t)ROW_F * npad + j0];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = j0 + threadIdx.x; j < j1; j += RB_THREADS) {
        const double2 x = v[(size_t)d * n + j];
        const double df = fwl[(size_t)ROW_F * npad + j] - fb;
        s[0] += x.x;
        s[1] += x.y;
        s[2] += x.x * df;
        s[3] += x.y * df;
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int h = RB_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a0[(size_t)d * nb + b] = make_double2(sh[0][0], sh[1][0]);
        a1[(size_t)d * nb + b] = make_double2(sh[2][0], sh[3][0]);
    }
}

// Edge table: rows f, f^-1/3, ln f of the edge frequencies and u'_de (FP64
// and FP32); entries past the last edge repeat its frequency with u' = 0.
__global__ __launch_bounds__(256) void rb_edges_kernel(const double* __restrict__ fwl_full, int npad_full,
                                                       const int32_t* __restrict__ edges, int ne, int n_det,
                                                       const double* __restrict__ cb0, const double2* __restrict__ a0,
                                                       const double2* __restrict__ a1, int npad,
                                                       double* __restrict__ fwl, float2* __restrict__ u32,
                                                       double2* __restrict__ u64) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npad) return;
    const int nb = ne - 1;
    const int je = edges[e < ne ? e : ne - 1];
    const double f = fwl_full[(size_t)ROW_F * npad_full + je];
    const double w = fwl_full[(size_t)ROW_W * npad_full + je];
    const double l = fwl_full[(size_t)ROW_LN * npad_full + je];
    fwl[(size_t)ROW_F * npad + e] = f;
    fwl[(size_t)ROW_W * npad + e] = w;
    fwl[(size_t)ROW_LN * npad + e] = l;
    for (int d = 0; d < n_det; ++d) {
        double cr = 0.0, ci = 0.0;
        if (e < ne) {
            if (e < nb) {
                const double wb = fwl_full[(size_t)ROW_F * npad_full + edges[e + 1]] - f;
                const double2 p = a0[(size_t)d * nb + e], q = a1[(size_t)d * nb + e];
                cr += p.x - q.x / wb;
                ci += p.y - q.y / wb;
            }
            if (e > 0) {
                const double wb = f - fwl_full[(size_t)ROW_F * npad_full + edges[e - 1]];
                const double2 q = a1[(size_t)d * nb + e - 1];
                cr += q.x / wb;
                ci += q.y / wb;
            }
        }
        double ur = 0.0, ui = 0.0;
        if (e < ne) {
            const double ph = phase_cycles(cb0, d, f, w, l);
            double sn, cs;
            sincospi(2.0 * (ph - rint(ph)), &sn, &cs);
            ur = cr * cs - ci * sn;   // c e^{+2 pi i Phi0}
            ui = ci * cs + cr * sn;
        }
        u64[(size_t)d * npad + e] = make_double2(ur, ui);
        u32[(size_t)d * npad + e] = make_float2((float)ur, (float)ui);
    }
}

hipError_t launch_rb_tables(const double* fwl_full, const double2* u64_full, int n, int npad_full, int n_det,
                            const double* cb0, const int32_t* edges, int ne, double2* v, double2* a0, double2* a1,
                            int npad, double* fwl, float2* u32, double2* u64, hipStream_t s) {
    hipLaunchKernelGGL(rb_hetero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, fwl_full, u64_full, n, npad_full,
                       n_det, cb0, v);
    hipLaunchKernelGGL(rb_sums_kernel, dim3(ne - 1, n_det), dim3(RB_THREADS), 0, s, v, fwl_full, n, npad_full, edges,
                       ne - 1, a0, a1);
    hipLaunchKernelGGL(rb_edges_kernel, dim3((npad + 255) / 256), dim3(256), 0, s, fwl_full, npad_full, edges, ne,
                       n_det, cb0, a0, a1, npad, fwl, u32, u64);
    return hipGetLastError();
}

hipError_t launch_build_tables(const double* d_data, const double* d_psd, int n_det, int n_bins, int n_pad,
                               double f_low, double df, double u_scale, double* fwl, float2* u32, double2* u64,
                               double* wa2, double* sums, hipStream_t s) {
    hipLaunchKernelGGL(build_tables_kernel, dim3((n_pad + 255) / 256), dim3(256), 0, s, d_data, d_psd, n_det, n_bins,
                       n_pad, f_low, df, 1.0 / u_scale, fwl, u32, u64, wa2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(table_sums_kernel, dim3(n_det), dim3(256), 0, s, d_data, d_psd, n_bins, f_low, df, sums);
    return hipGetLastError();
}

}  // namespace smcgw
