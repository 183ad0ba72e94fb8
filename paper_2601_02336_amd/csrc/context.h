// The opaque context behind smcgw_ctx (host side only).
#pragma once

#include <unordered_map>
#include <utility>
#include <vector>

#include "common.h"

// Prior / boundary of the sampled coordinates, passed to kernels by value.
namespace smcgw {
struct PriorDesc {
    int dim;
    double lo[MAXDIM], hi[MAXDIM];
    int bnd[MAXDIM], kind[MAXDIM];
};

// Likelihood selector for the sampler kernels, passed by value.
struct TargetDesc {
    int kind;                 // SMCGW_TARGET_*
    int dim;
    const double* params;     // device copy of the analytic target's parameters
};
}  // namespace smcgw

struct smcgw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_det = 0;
    std::vector<smcgw::DevEvent> events;
    std::vector<void*> event_bufs;
    smcgw::DevEvent* d_events = nullptr;
    void* d_small = nullptr;               // 4 KiB staging buffer
    smcgw::ParamMap pmap;
    // likelihood scratch, sized for `cap` particles
    double* d_cb = nullptr;
    int cap = 0;
    double* d_tan = nullptr;               // tangent moment blocks of the plain form, [tan_cap][12]
    int tan_cap = 0;
    // sampler state
    bool prior_set = false;
    smcgw::PriorDesc prior{};
    smcgw::TargetDesc target{SMCGW_TARGET_GW, 0, nullptr};
    double* d_target_params = nullptr;
    // sampler scratch
    void* d_queue = nullptr;               // work-queue counter of the persistent kernels
    int nuts_waves = 0;                    // wavefronts per NUTS slot (0: default)
    int nuts_priority = 1;                 // depth-driven wavefront priority in the NUTS kernel
    int nuts_slots_per_cu = 0;             // cap on resident NUTS workgroups per CU (0: none)
    int32_t* d_order = nullptr;            // NUTS start order built from a work hint
    double* d_mm = nullptr;                // block partials of the population covariance
    size_t mm_bytes = 0;
    int order_cap = 0;
    std::unordered_map<const void*, std::pair<int, int>> resident;   // (CUs, workgroups per CU), per kernel
    const int32_t* ev_of_p = nullptr;      // caller-owned event index per particle (NULL: event 0)
    void* d_sampler = nullptr;
    size_t sampler_bytes = 0;
    double* h_pinned = nullptr;            // small pinned host buffer for scalar read-backs
    // lockstep-sweep transition (the plain comparison form): tree states, next positions, their
    // likelihoods, active flags and count; the captured group of sweeps and the arguments it was captured for
    void* d_sweep = nullptr;
    size_t sweep_bytes = 0;
    hipGraph_t sweep_graph = nullptr;
    hipGraphExec_t sweep_exec = nullptr;
    std::vector<unsigned char> sweep_key;
    // kernel timing (events recorded around launches when enabled)
    unsigned timing_mask = 0;              // bit c: time kernel class c
    std::vector<hipEvent_t> ev_pool;       // free events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[SMCGW_KERNEL_CLASSES];

    void sweep_free() {
        if (sweep_exec) (void)hipGraphExecDestroy(sweep_exec);
        if (sweep_graph) (void)hipGraphDestroy(sweep_graph);
        sweep_exec = nullptr;
        sweep_graph = nullptr;
        sweep_key.clear();
        (void)hipFree(d_sweep);
        d_sweep = nullptr;
        sweep_bytes = 0;
    }

    void sampler_free() {
        (void)hipFree(d_target_params);
        (void)hipFree(d_sampler);
        (void)hipFree(d_queue);
        (void)hipFree(d_order);
        (void)hipFree(d_mm);
        d_mm = nullptr;
        mm_bytes = 0;
        d_queue = nullptr;
        d_order = nullptr;
        order_cap = 0;
        if (h_pinned) (void)hipHostFree(h_pinned);
        d_target_params = nullptr;
        d_sampler = nullptr;
        h_pinned = nullptr;
        sampler_bytes = 0;
    }
};

namespace smcgw {
// Brackets a launch with timing events when the context's timing is on.
struct TimedLaunch {
    smcgw_ctx* c;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(smcgw_ctx* ctx, int kernel_class);
    bool on() const { return (c->timing_mask >> cls) & 1u; }
    ~TimedLaunch();
};
int ctx_reserve(smcgw_ctx* c, int P);
// SMC pieces queued by smcgw_smc_iteration (smc.hip, metric.hip, nuts.hip).
void* sampler_scratch(smcgw_ctx* c, size_t bytes);
double* pinned(smcgw_ctx* c);
size_t reweight_scratch_bytes(int n_runs, int P, int D);
int queue_reweight_resample(smcgw_ctx* c, int n_runs, int P, int D, double beta_prev, double alpha, uint64_t seed,
                            uint64_t iteration, double* theta, double* logl, double* grad, int32_t* carry,
                            int32_t* ancestors, double* st, double* hist, int hist_cap, double** out_dev);
int mm_reserve(smcgw_ctx* c, int n_runs, int P);
int queue_mass_matrix_runs(smcgw_ctx* c, int n_runs, int P, int D, const double* theta, double shrink, double* inv,
                           double* chol, int32_t* status, const double* st);
int queue_local_metric(smcgw_ctx* c, int P, int D, const double* theta, const double* st, int run_size,
                       const double* fallback_runs, double* chol, int32_t* status);
int queue_record(smcgw_ctx* c, int n_runs, int P, const int32_t* nlf, const int32_t* depth, const uint8_t* div,
                 const int32_t* mm_status, const int32_t* metric_status, const double* st, double* hist,
                 int hist_cap);
int nuts_reserve(smcgw_ctx* c, int P, bool hint);
// The plain form of the likelihood (plain.hip).
int tangent_reserve(smcgw_ctx* c, int P);
int queue_loglike_tangent(smcgw_ctx* c, int P, const int32_t* ev_of_p, const double* theta, const uint8_t* active,
                          double* logl, double* grad);
bool tangent_supported(const smcgw_ctx* c);
int ctx_loglike(smcgw_ctx* c, int P, const int32_t* ev_of_p, const double* theta, double* logl, double* grad,
                int precision);
}  // namespace smcgw
