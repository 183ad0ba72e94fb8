// Per-wavefront bin loop of the likelihood and its FP64 epilogue, shared by
// the batched likelihood kernels and the persistent NUTS kernel.
//
// A wavefront walks blocks of TABLE_PAD bins starting at block `blk0` with
// stride `blk_step`.  A block is read in chunks of 128 bins, lane l taking
// bins 2l and 2l + 1 of each chunk (TABLE_PAD/64 bins per lane per block); the
// per-bin tables are read coalesced and shared by every particle.  The
// wavefront's moments (see likelihood.hip), summed in FP64 over the blocks it
// visited, are written to a moment block by lanes 0..7.
#pragma once

#include "common.h"

namespace smcgw {

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


// sin(2 pi x), cos(2 pi x) for 0 <= x < 1 on the hardware transcendental unit
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
        k.pr[d] = uniform_d(cb[CB_PR + d] * cb[CB_AMP]);
        k.pi[d] = uniform_d(cb[CB_PI + d] * cb[CB_AMP]);
    }
    return k;
}

// Per-lane inputs of one bin: f, f^-1/3, ln f and the detectors' whitened data.
template <int NDET, class U>
struct BinIn {
    double f, w, l;
    U u[NDET];
};

// The bin tables as raw buffer resources.  A chunk's loads then take the
// chunk's wave-uniform byte offset in a scalar register and a loop-invariant
// per-lane byte offset, so they cost no vector instructions for addresses.
// Resource word 3 of a raw (stride-0) buffer on this GPU family: 32-bit data
// format, no swizzle.
constexpr int BUF_RSRC_WORD3 = 0x00020000;

struct TableView {
    __amdgpu_buffer_rsrc_t fwl, u;
    int npad;
};

// The pointer and size are made wave-uniform first: a resource must sit in
// scalar registers, and a descriptor read from LDS is not known to be uniform.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, size_t bytes) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)min(bytes, (size_t)0x7fffffff));
    void* q = (void*)(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, n, BUF_RSRC_WORD3);
}

__device__ __forceinline__ double buf_f64(__amdgpu_buffer_rsrc_t r, unsigned lane_bytes, int uniform_bytes) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_bytes, uniform_bytes, 0));
}

// A chunk is 128 consecutive bins; lane l takes bins 2l and 2l + 1, so every
// row of a chunk is read with one 16-byte load per lane.  Wider loads move
// twice the bytes per memory instruction: the bin loop is bound by the memory
// instructions in flight (one wavefront alone) or by the request rate of the
// cache hierarchy (a full device), not by the bytes themselves.
constexpr int CHUNK_BINS = 128;
constexpr int BLK_CHUNKS = TABLE_PAD / CHUNK_BINS;   // chunks per block

template <int NDET, class U>
struct BinPair {
    BinIn<NDET, U> b[2];
};

__device__ __forceinline__ double2 buf_f64x2(__amdgpu_buffer_rsrc_t r, unsigned lane_bytes, int uniform_bytes) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, lane_bytes, uniform_bytes, 0));
}

// One chunk starting at bin `base` (wave-uniform).
template <int NDET>
__device__ __forceinline__ void load_chunk(BinPair<NDET, float2>& x, const TableView& t, int base, unsigned lane) {
    const int np8 = t.npad * 8;
    const double2 f = buf_f64x2(t.fwl, lane * 16u, ROW_F * np8 + base * 8);
    const double2 w = buf_f64x2(t.fwl, lane * 16u, ROW_W * np8 + base * 8);
    const double2 l = buf_f64x2(t.fwl, lane * 16u, ROW_LN * np8 + base * 8);
    x.b[0].f = f.x; x.b[1].f = f.y;
    x.b[0].w = w.x; x.b[1].w = w.y;
    x.b[0].l = l.x; x.b[1].l = l.y;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        const float4 u = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(t.u, lane * 16u,
                                                                                          d * np8 + base * 8, 0));
        x.b[0].u[d] = make_float2(u.x, u.y);
        x.b[1].u[d] = make_float2(u.z, u.w);
    }
}

template <int NDET>
__device__ __forceinline__ void load_chunk(BinPair<NDET, double2>& x, const TableView& t, int base, unsigned lane) {
    const int np8 = t.npad * 8;
    const double2 f = buf_f64x2(t.fwl, lane * 16u, ROW_F * np8 + base * 8);
    const double2 w = buf_f64x2(t.fwl, lane * 16u, ROW_W * np8 + base * 8);
    const double2 l = buf_f64x2(t.fwl, lane * 16u, ROW_LN * np8 + base * 8);
    x.b[0].f = f.x; x.b[1].f = f.y;
    x.b[0].w = w.x; x.b[1].w = w.y;
    x.b[0].l = l.x; x.b[1].l = l.y;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        x.b[0].u[d] = buf_f64x2(t.u, lane * 32u, 2 * (d * np8 + base * 8));
        x.b[1].u[d] = buf_f64x2(t.u, lane * 32u + 16u, 2 * (d * np8 + base * 8));
    }
}

// A wavefront visits the blocks blk0, blk0 + blk_step, ... of the padded
// table; each block is BLK_CHUNKS chunks.  The chunks run through two register
// buffers in turn: while one buffer is computed the other one's table entries
// are in flight.  Every prefetch is unconditional (the one past the last chunk
// re-reads the last chunk), so the buffers need no register copies.  The first
// bin of a block starts the per-lane partial sums and the block ends with
// their flush.  A lane adds its bins in chunk order, each chunk's pair in bin
// order.
template <class In, class Acc>
__device__ __forceinline__ void bin_loop(Acc& A, const BinCoef& k, const TableView& t, int blk0, int blk_step,
                                         int nblk) {
    static_assert(BLK_CHUNKS % 2 == 0, "a block holds a whole number of buffer pairs");
    const unsigned lane = threadIdx.x & 63;
    const int nb = blk0 < nblk ? (nblk - blk0 + blk_step - 1) / blk_step : 0;   // this wave's blocks
    if (nb == 0) return;
    const int last = nb * BLK_CHUNKS - 1;                                      // this wave's last chunk
    auto base_of = [&](int c) {
        return (blk0 + (c / BLK_CHUNKS) * blk_step) * TABLE_PAD + CHUNK_BINS * (c % BLK_CHUNKS);
    };
    In a, b;
    load_chunk(a, t, base_of(0), lane);
    for (int blk = 0; blk < nb; ++blk) {
#pragma unroll
        for (int pr = 0; pr < BLK_CHUNKS / 2; ++pr) {
            const int c = blk * BLK_CHUNKS + 2 * pr;
            load_chunk(b, t, base_of(c + 1), lane);
            A.bin(k, a.b[0], pr == 0);
            A.bin(k, a.b[1], false);
            load_chunk(a, t, base_of(min(c + 2, last)), lane);
            A.bin(k, b.b[0], false);
            A.bin(k, b.b[1], false);
        }
        A.flush();
    }
}

// Moments of NDET detectors from a wavefront's per-lane sums into a moment
// block (MOM_SIZE entries, those of absent detectors zero).
template <int NDET>
__device__ __forceinline__ void store_moments(const double (&Zr)[NDET], const double (&Zi)[NDET],
                                              const double (&T)[NDET], const double (&G)[NCOEF], double* out) {
    constexpr int K = 3 * NDET + NCOEF;
    double v[K];
    int idx[K];
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        v[d] = Zr[d]; idx[d] = MOM_ZR + d;
        v[NDET + d] = Zi[d]; idx[NDET + d] = MOM_ZI + d;
        v[2 * NDET + d] = T[d]; idx[2 * NDET + d] = MOM_T + d;
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) { v[3 * NDET + b] = G[b]; idx[3 * NDET + b] = MOM_G + b; }
    wave_totals_to<K>(v, idx, out);
    const int lane = threadIdx.x & 63;
    constexpr int ABSENT = MAXDET - NDET;
    if (lane >= 8 && lane < 8 + 3 * ABSENT) {
        const int j = lane - 8, d = NDET + j % (ABSENT > 0 ? ABSENT : 1), which = j / (ABSENT > 0 ? ABSENT : 1);
        out[(which == 0 ? MOM_ZR : which == 1 ? MOM_ZI : MOM_T) + d] = 0.0;
    }
}

// MIXED: FP64 phase and argument reduction, FP32 sin/cos, complex products and
// per-lane partial sums (flushed into FP64 once per block), FP64 basis moments.
template <int NDET>
struct MixedAcc {
    float pr[NDET], pim[NDET];
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];
    float zr[NDET], zi[NDET], tq[NDET];

    __device__ __forceinline__ void bin(const BinCoef& k, const BinIn<NDET, float2>& x, bool first) {
        double B[NBASIS];
        basis_rows(x.f, x.w, x.l, B);
        double ph = k.c[0];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) ph = fma(k.c[1 + b], B[b], ph);
        const float ff = (float)x.f;
        float psib;
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            // fractional part of the phase in one FP64 instruction (exact); as a float
            // it is within 2^-25 revolutions of the exact value
            const double phd = fma(x.f, k.tau[d], ph);
            const float xr = (float)__builtin_amdgcn_fract(phd);
            float sn, cs;
            sincos_rev_hw(xr, sn, cs);
            const float sr = fmaf(x.u[d].x, cs, x.u[d].y * sn);    // u e^{-2 pi i x}
            const float si = fmaf(x.u[d].y, cs, -x.u[d].x * sn);
            zr[d] = first ? sr : zr[d] + sr;
            zi[d] = first ? si : zi[d] + si;
            const float q = fmaf(pr[d], si, pim[d] * sr);
            psib = (d == 0) ? q : psib + q;
            tq[d] = first ? q * ff : fmaf(q, ff, tq[d]);
        }
        const double pb = (double)psib;
        G[0] += pb;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(pb, B[b], G[1 + b]);
    }

    // Block end: the block's FP32 partials into the FP64 sums (the next block's
    // first bin restarts them).
    __device__ __forceinline__ void flush() {
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            Zr[d] += zr[d]; Zi[d] += zi[d]; T[d] += tq[d];
        }
    }
};

template <int NDET>
__device__ __forceinline__ void bins_mixed_wave(const DevEvent* __restrict__ ev, const BinCoef& k, int blk0,
                                                int blk_step, double* mom) {
    const int npad = __builtin_amdgcn_readfirstlane(ev->n_pad);
    MixedAcc<NDET> A;
#pragma unroll
    for (int d = 0; d < NDET; ++d) {
        A.pr[d] = (float)k.pr[d]; A.pim[d] = (float)k.pi[d];
        A.Zr[d] = 0.0; A.Zi[d] = 0.0; A.T[d] = 0.0;
    }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) A.G[b] = 0.0;
    const TableView t{raw_rsrc(ev->fwl, (size_t)NROWS * npad * sizeof(double)),
                      raw_rsrc(ev->u32, (size_t)NDET * npad * sizeof(float2)), npad};
    bin_loop<BinPair<NDET, float2>>(A, k, t, blk0, blk_step, npad / TABLE_PAD);
    store_moments<NDET>(A.Zr, A.Zi, A.T, A.G, mom);
}

// PLAIN_FP64: the same algebra in FP64 throughout.
template <int NDET>
struct Fp64Acc {
    double Zr[NDET], Zi[NDET], T[NDET], G[NCOEF];

    __device__ __forceinline__ void bin(const BinCoef& k, const BinIn<NDET, double2>& x, bool) {
        double B[NBASIS];
        basis_rows(x.f, x.w, x.l, B);
        double ph = k.c[0];
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) ph = fma(k.c[1 + b], B[b], ph);
        double psib;
#pragma unroll
        for (int d = 0; d < NDET; ++d) {
            const double phd = fma(x.f, k.tau[d], ph);
            const double xr = phd - rint(phd);
            double sn, cs;
            sincospi(2.0 * xr, &sn, &cs);
            const double sr = fma(x.u[d].x, cs, x.u[d].y * sn);
            const double si = fma(x.u[d].y, cs, -x.u[d].x * sn);
            Zr[d] += sr;
            Zi[d] += si;
            const double q = fma(k.pr[d], si, k.pi[d] * sr);
            psib = (d == 0) ? q : psib + q;
            T[d] = fma(q, x.f, T[d]);
        }
        G[0] += psib;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) G[1 + b] = fma(psib, B[b], G[1 + b]);
    }

    __device__ __forceinline__ void flush() {}
};

template <int NDET>
__device__ __forceinline__ void bins_fp64_wave(const DevEvent* __restrict__ ev, const BinCoef& k, int blk0,
                                               int blk_step, double* mom) {
    const int npad = __builtin_amdgcn_readfirstlane(ev->n_pad);
    Fp64Acc<NDET> A;
#pragma unroll
    for (int d = 0; d < NDET; ++d) { A.Zr[d] = 0.0; A.Zi[d] = 0.0; A.T[d] = 0.0; }
#pragma unroll
    for (int b = 0; b < NCOEF; ++b) A.G[b] = 0.0;
    const TableView t{raw_rsrc(ev->fwl, (size_t)NROWS * npad * sizeof(double)),
                      raw_rsrc(ev->u64, (size_t)NDET * npad * sizeof(double2)), npad};
    bin_loop<BinPair<NDET, double2>>(A, k, t, blk0, blk_step, npad / TABLE_PAD);
    store_moments<NDET>(A.Zr, A.Zi, A.T, A.G, mom);
}

// logL and its gradient with respect to the 11 source parameters from the
// moments and the prologue's Jacobians (FP64, one lane).
__device__ __forceinline__ double finish_particle(const DevEvent& ev, const double* c, const double* m,
                                                  double g[NPAR]) {
    double ll = -0.5 * ev.dd;
    double dlnca = 0.0, sum_t = 0.0;
    const double amp = c[CB_AMP];          // P'_d = amp P_d
    double gp[4] = {0.0, 0.0, 0.0, 0.0};   // iota, psi, ra, dec through P'_d
    for (int k = 0; k < NPAR; ++k) g[k] = 0.0;
    for (int d = 0; d < ev.n_det; ++d) {
        const double pr = c[CB_PR + d] * amp, pi = c[CB_PI + d] * amp;
        const double zr = m[MOM_ZR + d], zi = m[MOM_ZI + d], h = ev.hnorm[d];
        const double re = pr * zr - pi * zi;
        const double p2 = pr * pr + pi * pi;
        ll += re - 0.5 * p2 * h;
        dlnca += re - p2 * h;
        const double ar = zr - h * pr, ai = -zi - h * pi;   // dlogL / d(Re P', Im P')
#pragma unroll
        for (int k = 0; k < 4; ++k) gp[k] += amp * (ar * c[CB_DPR + 4 * d + k] + ai * c[CB_DPI + 4 * d + k]);
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
