// Event bin tables (built once per event, frequency-major).
//
// For the inner product of arXiv:2601.02336 Sec. 2 (Eq. 2) discretised on
// f_j = f_low + j df, every particle reuses the same per-bin quantities:
//   u_dj = 4 df conj(d_dj) f_j^-7/6 / S_dj            (whitened data x amplitude shape)
//   f_j, f_j^-1/3, ln f_j                           (phase basis generators)
//   H_d  = sum_j 4 df f_j^-7/3 / S_dj,  <d|d>_d = sum_j 4 df |d_dj|^2 / S_dj.
// The tables are zero-padded to a multiple of TABLE_PAD bins; padded bins have
// u = 0 and finite basis values, so they add nothing to any sum.
#include "common.h"

namespace smcgw {

__global__ __launch_bounds__(256) void build_tables_kernel(const double* __restrict__ data, const double* __restrict__ psd,
                                                           int n_det, int n, int npad, double f_low, double df,
                                                           double inv_us, double* __restrict__ fwl,
                                                           float2* __restrict__ u32, double2* __restrict__ u64) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= npad) return;
    const double f = f_low + df * (double)j;
    fwl[(size_t)ROW_F * npad + j] = f;
    fwl[(size_t)ROW_W * npad + j] = 1.0 / cbrt(f);
    fwl[(size_t)ROW_LN * npad + j] = log(f);
    const double a = pow(f, -7.0 / 6.0);
    for (int d = 0; d < n_det; ++d) {
        double ur = 0.0, ui = 0.0;
        if (j < n) {
            const double w = 4.0 * df / psd[(size_t)d * n + j];
            const double* dd = data + 2 * ((size_t)d * n + j);
            ur = w * a * dd[0] * inv_us;
            ui = -w * a * dd[1] * inv_us;
        }
        u64[(size_t)d * npad + j] = make_double2(ur, ui);
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
    for (int x = 0; x < NGEO; ++x)
        for (int y = 0; y <= x; ++y) {
            part[threadIdx.x] = acc[e++];
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

hipError_t launch_build_tables(const double* d_data, const double* d_psd, int n_det, int n_bins, int n_pad,
                               double f_low, double df, double u_scale, double* fwl, float2* u32, double2* u64,
                               double* sums, hipStream_t s) {
    hipLaunchKernelGGL(build_tables_kernel, dim3((n_pad + 255) / 256), dim3(256), 0, s, d_data, d_psd, n_det, n_bins,
                       n_pad, f_low, df, 1.0 / u_scale, fwl, u32, u64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(table_sums_kernel, dim3(n_det), dim3(256), 0, s, d_data, d_psd, n_bins, f_low, df, sums);
    return hipGetLastError();
}

}  // namespace smcgw
