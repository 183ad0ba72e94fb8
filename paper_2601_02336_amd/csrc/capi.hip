// Host side of the C ABI declared in smcgw.h: context, event set-up and the
// likelihood entry points.  Sampler entry points live in sampler.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "context.h"

using namespace smcgw;

extern "C" const char* smcgw_status_string(int status) {
    switch (status) {
    case SMCGW_OK: return "ok";
    case SMCGW_WARN_FALLBACK: return "warning: fallback used (diagonal mass matrix)";
    case SMCGW_ERR_INVALID: return "invalid argument";
    case SMCGW_ERR_SHAPE: return "size out of the supported range";
    case SMCGW_ERR_HIP: return "HIP runtime error";
    case SMCGW_ERR_OOM: return "device allocation failed";
    case SMCGW_ERR_NOT_INIT: return "context not initialised (event, prior or target missing)";
    case SMCGW_ERR_STALL: return "tempering ladder cannot advance";
    default: return "unknown status";
    }
}

namespace smcgw {

static hipEvent_t pool_event(smcgw_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

TimedLaunch::TimedLaunch(smcgw_ctx* ctx, int kernel_class) : c(ctx), cls(kernel_class) {
    if (!on()) return;
    a = pool_event(c);
    b = pool_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
}

TimedLaunch::~TimedLaunch() {
    if (!on() || !a || !b) return;
    (void)hipEventRecord(b, c->stream);
    c->ev_pending[cls].push_back({a, b});
}

int ctx_reserve(smcgw_ctx* c, int P) {
    if (P <= c->cap) return SMCGW_OK;
    const int cap = std::max(P, std::max(2 * c->cap, 256));
    (void)hipFree(c->d_cb);
    c->d_cb = nullptr;
    c->cap = 0;
    if (hipMalloc(&c->d_cb, (size_t)cap * CB_SIZE * sizeof(double)) != hipSuccess) return SMCGW_ERR_OOM;
    c->cap = cap;
    return SMCGW_OK;
}

// logL / gradient of P particles on the context's stream (no synchronisation).
int ctx_loglike(smcgw_ctx* c, int P, const int32_t* ev_of_p, const double* theta, double* logl, double* grad,
                int precision) {
    if (c->events.empty()) return SMCGW_ERR_NOT_INIT;
    int rc = ctx_reserve(c, P);
    if (rc) return rc;
    {
        TimedLaunch t(c, SMCGW_KERNEL_PREP);
        if (launch_prep(c->d_events, (int)c->events.size(), ev_of_p, c->pmap, P, theta, c->d_cb, c->stream) != hipSuccess)
            return SMCGW_ERR_HIP;
    }
    {
        TimedLaunch t(c, SMCGW_KERNEL_BINS);
        if (launch_bins(c->d_events, (int)c->events.size(), ev_of_p, c->pmap, P, c->n_det, precision, c->d_cb, logl,
                        grad, c->stream) != hipSuccess)
            return SMCGW_ERR_HIP;
    }
    return SMCGW_OK;
}

}  // namespace smcgw

extern "C" int smcgw_create(smcgw_ctx** out, int device, void* hip_stream) {
    if (!out) return SMCGW_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SMCGW_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess) return SMCGW_ERR_HIP;
    smcgw_ctx* c = new smcgw_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->pmap.dim = NPAR;
    for (int k = 0; k < NPAR; ++k) { c->pmap.idx[k] = k; c->pmap.fixed[k] = 0.0; }
    if (hipMalloc(&c->d_events, SMCGW_MAX_EVENTS * sizeof(DevEvent)) != hipSuccess ||
        hipMalloc(&c->d_small, 4096) != hipSuccess) {
        (void)hipFree(c->d_events);
        delete c;
        return SMCGW_ERR_OOM;
    }
    if (noalloc_init(device) != SMCGW_OK) {   // this device's fixed scratch address, once per device
        (void)hipFree(c->d_events);
        (void)hipFree(c->d_small);
        delete c;
        return SMCGW_ERR_HIP;
    }
    *out = c;
    return SMCGW_OK;
}

extern "C" int smcgw_destroy(smcgw_ctx* c) {
    if (!c) return SMCGW_ERR_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->event_bufs) (void)hipFree(p);
    (void)hipFree(c->d_events);
    (void)hipFree(c->d_small);
    (void)hipFree(c->d_cb);
    (void)hipFree(c->d_tan);
    c->sweep_free();
    c->sampler_free();
    for (auto& v : c->ev_pending)
        for (auto& pr : v) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
    return SMCGW_OK;
}

extern "C" int smcgw_set_option(smcgw_ctx* c, int option, int64_t value) {
    if (!c) return SMCGW_ERR_INVALID;
    switch (option) {
    case SMCGW_OPT_NUTS_WAVES:
        if (value != 0 && value != 2 && value != 4 && value != 6 && value != 8) return SMCGW_ERR_INVALID;
        c->nuts_waves = (int)value;
        return SMCGW_OK;
    case SMCGW_OPT_NUTS_PRIORITY:
        if (value != 0 && value != 1) return SMCGW_ERR_INVALID;
        c->nuts_priority = (int)value;
        return SMCGW_OK;
    case SMCGW_OPT_NUTS_SLOTS_PER_CU:
        if (value < 0 || value > 64) return SMCGW_ERR_INVALID;
        c->nuts_slots_per_cu = (int)value;
        return SMCGW_OK;
    default:
        return SMCGW_ERR_INVALID;
    }
}

extern "C" int smcgw_timing_enable(smcgw_ctx* c, int class_mask) {
    if (!c || class_mask < 0 || class_mask >= (1 << SMCGW_KERNEL_CLASSES)) return SMCGW_ERR_INVALID;
    c->timing_mask = (unsigned)class_mask;
    return SMCGW_OK;
}

extern "C" int smcgw_timing_read(smcgw_ctx* c, int kernel_class, double* total_ms, int64_t* launches) {
    if (!c || kernel_class < 0 || kernel_class >= SMCGW_KERNEL_CLASSES || !total_ms || !launches)
        return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SMCGW_ERR_HIP;
    double tot = 0.0;
    int64_t n = 0;
    for (auto& pr : c->ev_pending[kernel_class]) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            tot += ms;
            ++n;
        }
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_pending[kernel_class].clear();
    *total_ms = tot;
    *launches = n;
    return SMCGW_OK;
}

extern "C" int smcgw_timing_intervals(smcgw_ctx* c, int kernel_class, void* ref_event, double* start_ms,
                                      double* end_ms, int64_t cap, int64_t* launches) {
    if (!c || kernel_class < 0 || kernel_class >= SMCGW_KERNEL_CLASSES || !ref_event || !launches || cap < 0 ||
        (cap > 0 && (!start_ms || !end_ms)))
        return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    const hipEvent_t ref = (hipEvent_t)ref_event;
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipEventSynchronize(ref) != hipSuccess)
        return SMCGW_ERR_HIP;
    int64_t n = 0;
    bool ok = true;
    for (auto& pr : c->ev_pending[kernel_class]) {
        float s = 0.f, e = 0.f;
        if (hipEventElapsedTime(&s, ref, pr.first) == hipSuccess && hipEventElapsedTime(&e, ref, pr.second) == hipSuccess) {
            if (n < cap) {
                start_ms[n] = s;
                end_ms[n] = e;
            }
            ++n;
        } else {
            ok = false;
        }
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_pending[kernel_class].clear();
    *launches = n;
    if (!ok) return SMCGW_ERR_HIP;
    return n > cap ? SMCGW_ERR_SHAPE : SMCGW_OK;
}

extern "C" int smcgw_set_stream(smcgw_ctx* c, void* hip_stream) {
    if (!c) return SMCGW_ERR_INVALID;
    c->stream = (hipStream_t)hip_stream;
    return SMCGW_OK;
}

// Detector position and response tensor D = (x x^T - y y^T)/2 from the site.
static void site_geometry(const smcgw_detector& s, double pos[3], double resp[3][3]) {
    const double cl = std::cos(s.lat), sl = std::sin(s.lat), co = std::cos(s.lon), so = std::sin(s.lon);
    pos[0] = s.radius * cl * co;
    pos[1] = s.radius * cl * so;
    pos[2] = s.radius * sl;
    const double e[3] = {-so, co, 0.0}, nn[3] = {-sl * co, -sl * so, cl};
    double x[3], y[3];
    for (int i = 0; i < 3; ++i) {
        x[i] = std::cos(s.az_x) * e[i] + std::sin(s.az_x) * nn[i];
        y[i] = std::cos(s.az_y) * e[i] + std::sin(s.az_y) * nn[i];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) resp[i][j] = 0.5 * (x[i] * x[j] - y[i] * y[j]);
}

namespace smcgw {
// Buffers of one event's tables.
constexpr int EVENT_BUFS = 5;

// Builds the full-grid tables of one event on the device (synchronises).  On
// success de describes them and bufs holds fwl, u32, u64, wmom and wa2.
static int build_event(smcgw_ctx* c, const smcgw_event_desc* ev, const double* data_reim, const double* psd,
                       const smcgw_detector* dets, DevEvent& de, void* bufs[EVENT_BUFS]) {
    const int n = ev->n_bins, nd = ev->n_det;
    const int npad = ((n + TABLE_PAD - 1) / TABLE_PAD) * TABLE_PAD;
    // Power-of-two scale of the whitened data, so the FP32 table sits near unit magnitude.
    double umax = 0.0;
    for (int d = 0; d < nd; ++d)
        for (int j = 0; j < n; ++j) {
            const double f = ev->f_low + ev->df * j;
            const double* x = data_reim + 2 * ((size_t)d * n + j);
            const double v = 4.0 * ev->df * std::hypot(x[0], x[1]) / psd[(size_t)d * n + j] * std::pow(f, -7.0 / 6.0);
            if (std::isfinite(v)) umax = std::max(umax, v);
        }
    const double us = umax > 0.0 ? std::ldexp(1.0, (int)std::lround(std::log2(umax))) : 1.0;

    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    double *d_data = nullptr, *d_psd = nullptr, *fwl = nullptr, *sums = nullptr, *wmom = nullptr, *wa2 = nullptr;
    float2* u32 = nullptr;
    double2* u64 = nullptr;
    auto fail = [&](int code) {
        (void)hipFree(d_data); (void)hipFree(d_psd); (void)hipFree(fwl); (void)hipFree(u32); (void)hipFree(u64); (void)hipFree(sums); (void)hipFree(wmom);
        (void)hipFree(wa2);
        return code;
    };
    if (hipMalloc(&d_data, sizeof(double) * 2 * nd * (size_t)n) != hipSuccess ||
        hipMalloc(&d_psd, sizeof(double) * nd * (size_t)n) != hipSuccess ||
        hipMalloc(&fwl, sizeof(double) * NROWS * (size_t)npad) != hipSuccess ||
        hipMalloc(&u32, sizeof(float2) * nd * (size_t)npad) != hipSuccess ||
        hipMalloc(&u64, sizeof(double2) * nd * (size_t)npad) != hipSuccess ||
        hipMalloc(&sums, sizeof(double) * 2 * MAXDET) != hipSuccess ||
        hipMalloc(&wmom, sizeof(double) * nd * NGEO * NGEO) != hipSuccess ||
        hipMalloc(&wa2, sizeof(double) * nd * (size_t)npad) != hipSuccess)
        return fail(SMCGW_ERR_OOM);
    if (hipMemcpyAsync(d_data, data_reim, sizeof(double) * 2 * nd * (size_t)n, hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(d_psd, psd, sizeof(double) * nd * (size_t)n, hipMemcpyHostToDevice, c->stream))
        return fail(SMCGW_ERR_HIP);
    if (launch_build_tables(d_data, d_psd, nd, n, npad, ev->f_low, ev->df, us, fwl, u32, u64, wa2, sums, c->stream) ||
        launch_metric_moments(d_psd, nd, n, ev->f_low, ev->df, us, wmom, c->stream))
        return fail(SMCGW_ERR_HIP);
    double hs[2 * MAXDET];
    if (hipMemcpyAsync(hs, sums, sizeof(double) * 2 * nd, hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
        return fail(SMCGW_ERR_HIP);
    (void)hipFree(d_data);
    (void)hipFree(d_psd);
    (void)hipFree(sums);

    std::memset(&de, 0, sizeof(de));
    de.n_bins = n;
    de.n_pad = npad;
    de.n_det = nd;
    de.pn_order = ev->pn_order;
    de.f_low = ev->f_low;
    de.df = ev->df;
    de.fwl = fwl;
    de.u32 = u32;
    de.u64 = u64;
    de.wmom = wmom;
    de.wa2 = wa2;
    de.dd = 0.0;
    for (int d = 0; d < nd; ++d) {
        de.hnorm[d] = hs[2 * d] / (us * us);
        de.dd += hs[2 * d + 1];
        site_geometry(dets[d], de.pos[d], de.resp[d]);
    }
    de.u_scale = us;
    de.t_sun = ev->t_sun;
    de.ln_pi_tsun = std::log(M_PI * ev->t_sun);
    de.mpc_m = ev->mpc_m;
    de.c_light = ev->c_light;
    de.gmst = ev->gmst;
    bufs[0] = fwl;
    bufs[1] = u32;
    bufs[2] = u64;
    bufs[3] = wmom;
    bufs[4] = wa2;
    return SMCGW_OK;
}

static int check_event_desc(smcgw_ctx* c, const smcgw_event_desc* ev) {
    // the bin loop addresses a table row with 32-bit byte offsets
    if (ev->n_bins <= 0 || ev->n_bins > SMCGW_MAX_BINS || ev->n_det <= 0 || ev->n_det > MAXDET || !(ev->df > 0.0) ||
        !(ev->f_low > 0.0) || ev->pn_order < 0 || ev->pn_order > 7)
        return SMCGW_ERR_SHAPE;
    if ((int)c->events.size() >= SMCGW_MAX_EVENTS) return SMCGW_ERR_SHAPE;
    if (!c->events.empty() && ev->n_det != c->n_det) return SMCGW_ERR_SHAPE;
    return SMCGW_OK;
}

static int register_event(smcgw_ctx* c, const DevEvent& de, void* const bufs[EVENT_BUFS], int* event_id) {
    const int id = (int)c->events.size();
    if (hipMemcpyAsync(c->d_events + id, &de, sizeof(de), hipMemcpyHostToDevice, c->stream) ||
        hipStreamSynchronize(c->stream)) {
        for (int k = 0; k < EVENT_BUFS; ++k) (void)hipFree(bufs[k]);
        return SMCGW_ERR_HIP;
    }
    c->events.push_back(de);
    for (int k = 0; k < EVENT_BUFS; ++k)
        if (bufs[k]) c->event_bufs.push_back(bufs[k]);
    c->n_det = de.n_det;
    if (event_id) *event_id = id;
    return SMCGW_OK;
}
}  // namespace smcgw

extern "C" int smcgw_add_event(smcgw_ctx* c, const smcgw_event_desc* ev, const double* data_reim, const double* psd,
                               const smcgw_detector* dets, int* event_id) {
    if (!c || !ev || !data_reim || !psd || !dets) return SMCGW_ERR_INVALID;
    int rc = check_event_desc(c, ev);
    if (rc) return rc;
    DevEvent de;
    void* bufs[EVENT_BUFS];
    rc = build_event(c, ev, data_reim, psd, dets, de, bufs);
    if (rc) return rc;
    return register_event(c, de, bufs, event_id);
}

// Relative-binning edges (host): the phase-difference bound
//   dpsi(f) = 2 pi sum_k sgn(g_k) (f / f*_k)^g_k,  g = -5/3, -2/3, 1, 5/3, 7/3,
// f*_k the band's lower end for negative and its upper end for positive
// exponents, is cut into B = ceil(total growth / eps) steps of equal growth;
// edge k is the first grid point that reaches k of them.
extern "C" int smcgw_rb_edges(double f_low, double df, int n_bins, double eps, int32_t* edges, int cap) {
    if (n_bins < 2 || !(df > 0.0) || !(f_low > 0.0) || !(eps > 0.0) || !edges || cap < 2) return SMCGW_ERR_INVALID;
    static const double expo[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    const double f_hi = f_low + df * (n_bins - 1);
    auto bound = [&](double f) {
        double s = 0.0;
        for (double g : expo) s += g < 0.0 ? -std::pow(f / f_low, g) : std::pow(f / f_hi, g);
        return 2.0 * M_PI * s;
    };
    const double base = bound(f_low), growth = bound(f_hi) - base;
    const long steps = std::min<long>(std::max<long>(1, (long)std::ceil(growth / eps)), n_bins - 1);
    int count = 1;
    edges[0] = 0;
    int j = 0;
    for (long k = 1; k < steps; ++k) {
        const double level = growth * (double)k / (double)steps;
        while (j < n_bins - 1 && bound(f_low + df * j) - base < level) ++j;
        if (j >= n_bins - 1) break;
        if (j == edges[count - 1]) continue;
        if (count >= cap - 1) return SMCGW_ERR_SHAPE;
        edges[count++] = j;
    }
    edges[count++] = n_bins - 1;
    return count;
}

extern "C" int smcgw_add_event_rb(smcgw_ctx* c, const smcgw_event_desc* ev, const double* data_reim,
                                  const double* psd, const smcgw_detector* dets, const double* theta0, double eps,
                                  int* event_id, int* n_edges) {
    if (!c || !ev || !data_reim || !psd || !dets || !theta0 || !(eps > 0.0)) return SMCGW_ERR_INVALID;
    int rc = check_event_desc(c, ev);
    if (rc) return rc;
    if (ev->n_bins < 2) return SMCGW_ERR_SHAPE;
    std::vector<int32_t> ej(ev->n_bins + 1);
    const int ne = smcgw_rb_edges(ev->f_low, ev->df, ev->n_bins, eps, ej.data(), (int)ej.size());
    if (ne < 2) return ne < 0 ? ne : SMCGW_ERR_SHAPE;
    DevEvent full;
    void* fb[EVENT_BUFS];
    rc = build_event(c, ev, data_reim, psd, dets, full, fb);
    if (rc) return rc;
    const int n = ev->n_bins, nd = ev->n_det, id = (int)c->events.size();
    const int npad = ((ne + TABLE_PAD - 1) / TABLE_PAD) * TABLE_PAD;
    double *fwl = nullptr, *cb0 = nullptr, *th0 = nullptr;
    float2* u32 = nullptr;
    double2 *u64 = nullptr, *v = nullptr, *a0 = nullptr, *a1 = nullptr;
    int32_t *d_edges = nullptr, *d_id = nullptr;
    auto release = [&]() {
        (void)hipFree(v); (void)hipFree(a0); (void)hipFree(a1); (void)hipFree(d_edges); (void)hipFree(cb0); (void)hipFree(th0); (void)hipFree(d_id);
        (void)hipFree(fb[0]); (void)hipFree(fb[1]); (void)hipFree(fb[2]); (void)hipFree(fb[4]);
    };
    auto fail = [&](int code) {
        release();
        (void)hipFree(fb[3]); (void)hipFree(fwl); (void)hipFree(u32); (void)hipFree(u64);
        return code;
    };
    if (hipMalloc(&fwl, sizeof(double) * NROWS * (size_t)npad) != hipSuccess ||
        hipMalloc(&u32, sizeof(float2) * nd * (size_t)npad) != hipSuccess ||
        hipMalloc(&u64, sizeof(double2) * nd * (size_t)npad) != hipSuccess ||
        hipMalloc(&v, sizeof(double2) * nd * (size_t)n) != hipSuccess ||
        hipMalloc(&a0, sizeof(double2) * nd * (size_t)(ne - 1)) != hipSuccess ||
        hipMalloc(&a1, sizeof(double2) * nd * (size_t)(ne - 1)) != hipSuccess ||
        hipMalloc(&d_edges, sizeof(int32_t) * ne) != hipSuccess ||
        hipMalloc(&cb0, sizeof(double) * CB_SIZE) != hipSuccess ||
        hipMalloc(&th0, sizeof(double) * NPAR) != hipSuccess || hipMalloc(&d_id, sizeof(int32_t)) != hipSuccess)
        return fail(SMCGW_ERR_OOM);
    // The fiducial coefficient block comes from the likelihood's own prologue,
    // with the full event parked in the slot the new event will take.
    ParamMap pm;
    pm.dim = NPAR;
    for (int k = 0; k < NPAR; ++k) { pm.idx[k] = k; pm.fixed[k] = 0.0; }
    if (hipMemcpyAsync(c->d_events + id, &full, sizeof(full), hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(d_id, &id, sizeof(int32_t), hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(th0, theta0, sizeof(double) * NPAR, hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(d_edges, ej.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice, c->stream))
        return fail(SMCGW_ERR_HIP);
    if (launch_prep(c->d_events, id + 1, d_id, pm, 1, th0, cb0, c->stream) ||
        launch_rb_tables((const double*)fb[0], (const double2*)fb[2], n, full.n_pad, nd, cb0, d_edges, ne, v, a0, a1,
                         npad, fwl, u32, u64, c->stream) ||
        hipStreamSynchronize(c->stream))
        return fail(SMCGW_ERR_HIP);
    release();
    DevEvent de = full;
    de.n_bins = ne;
    de.n_pad = npad;
    de.fwl = fwl;
    de.u32 = u32;
    de.u64 = u64;
    de.wa2 = nullptr;   // the plain form's per-bin <h|h> needs the full grid
    void* bufs[EVENT_BUFS] = {fwl, u32, u64, fb[3], nullptr};
    rc = register_event(c, de, bufs, event_id);
    if (rc == SMCGW_OK && n_edges) *n_edges = ne;
    return rc;
}

extern "C" int smcgw_set_event_map(smcgw_ctx* c, const int32_t* event_of_particle) {
    if (!c) return SMCGW_ERR_INVALID;
    c->ev_of_p = event_of_particle;
    return SMCGW_OK;
}

extern "C" int smcgw_set_param_map(smcgw_ctx* c, int dim, const int32_t* param_index, const double* fixed11) {
    if (!c || dim <= 0 || dim > NPAR || !param_index) return SMCGW_ERR_INVALID;
    ParamMap pm;
    pm.dim = dim;
    for (int k = 0; k < NPAR; ++k) pm.fixed[k] = fixed11 ? fixed11[k] : 0.0;
    for (int k = 0; k < MAXDIM; ++k) pm.idx[k] = 0;
    for (int k = 0; k < dim; ++k) {
        if (param_index[k] < 0 || param_index[k] >= NPAR) return SMCGW_ERR_INVALID;
        pm.idx[k] = param_index[k];
    }
    c->pmap = pm;
    return SMCGW_OK;
}

extern "C" int smcgw_loglike_grad(smcgw_ctx* c, int P, const int32_t* event_of_particle, const double* theta,
                                  double* logl, double* grad, int precision) {
    if (!c || P < 0 || (P > 0 && (!theta || !logl))) return SMCGW_ERR_INVALID;
    if (precision != SMCGW_PLAIN_FP64 && precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (P == 0) return SMCGW_OK;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    return ctx_loglike(c, P, event_of_particle, theta, logl, grad, precision);
}

extern "C" int smcgw_waveform(smcgw_ctx* c, int event_id, const double* theta11, double* h_reim) {
    if (!c || !theta11 || !h_reim) return SMCGW_ERR_INVALID;
    if (event_id < 0 || event_id >= (int)c->events.size()) return SMCGW_ERR_INVALID;
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    int rc = ctx_reserve(c, 1);
    if (rc) return rc;
    // d_small: [0, 88) theta11, [128, 132) event index
    char* small = (char*)c->d_small;
    int32_t eid = event_id;
    if (hipMemcpyAsync(small, theta11, NPAR * sizeof(double), hipMemcpyHostToDevice, c->stream) ||
        hipMemcpyAsync(small + 128, &eid, sizeof(eid), hipMemcpyHostToDevice, c->stream))
        return SMCGW_ERR_HIP;
    ParamMap id;
    id.dim = NPAR;
    for (int k = 0; k < NPAR; ++k) { id.idx[k] = k; id.fixed[k] = 0.0; }
    if (launch_prep(c->d_events, (int)c->events.size(), (const int32_t*)(small + 128), id, 1, (const double*)small,
                    c->d_cb, c->stream))
        return SMCGW_ERR_HIP;
    const DevEvent& e = c->events[event_id];
    if (launch_waveform(c->d_events, event_id, c->d_cb, h_reim, e.n_bins, e.n_det, c->stream)) return SMCGW_ERR_HIP;
    // the small staging buffer is reused by the next call: wait for this one
    if (hipStreamSynchronize(c->stream)) return SMCGW_ERR_HIP;
    return SMCGW_OK;
}
