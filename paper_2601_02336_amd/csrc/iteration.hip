// One SMC iteration of several independent runs, queued as a whole, and the
// HIP graph that replays it (arXiv:2601.02336, Sec. 3: tempering, evidence,
// resampling; Sec. 4: the NUTS mutation; Sec. 5: the mass matrix).
//
// Everything the iteration needs from one step to the next lives on the
// device: each run's temperature, running log evidence, iteration index and
// done flag (the run state).  The host only queues the
// work, so the same launch sequence serves every iteration and can be
// captured once.
#include <algorithm>

#include "common.h"
#include "context.h"

using namespace smcgw;

struct smcgw_graph {
    smcgw_ctx* c = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int check_desc(smcgw_ctx* c, const smcgw_smc_iter_desc* d) {
    if (!c || !d) return SMCGW_ERR_INVALID;
    if (d->n_runs < 1 || d->n_runs > SMCGW_MAX_RUNS || d->P < 2 || d->D <= 0 || d->D > MAXDIM) return SMCGW_ERR_SHAPE;
    if ((size_t)d->n_runs * d->P > (size_t)INT32_MAX / 2) return SMCGW_ERR_SHAPE;
    if (!d->theta || !d->logl || !d->grad || !d->ancestors || !d->n_leapfrog || !d->depth || !d->divergent ||
        !d->inv_mass || !d->chol || !d->mm_status || !d->state || (d->chol_pp && !d->metric_status) ||
        (d->history && d->history_cap < 1))
        return SMCGW_ERR_INVALID;
    if (d->nuts_form != SMCGW_NUTS_PERSISTENT && d->nuts_form != SMCGW_NUTS_SWEEPS) return SMCGW_ERR_INVALID;
    if (d->nuts_form == SMCGW_NUTS_SWEEPS && d->precision != SMCGW_PLAIN_FP64) return SMCGW_ERR_INVALID;
    if (d->precision != SMCGW_PLAIN_FP64 && d->precision != SMCGW_MIXED) return SMCGW_ERR_INVALID;
    if (!(d->alpha > 0.0 && d->alpha <= 1.0) || !(d->shrink >= 0.0) || !(d->step > 0.0) || !(d->max_delta_h > 0.0) ||
        d->max_depth < 0 || d->max_depth > SMCGW_MAX_DEPTH)
        return SMCGW_ERR_INVALID;
    if (!c->prior_set || c->prior.dim != d->D) return SMCGW_ERR_NOT_INIT;
    if (c->target.kind == SMCGW_TARGET_GW) {
        if (c->events.empty() || c->pmap.dim != d->D) return SMCGW_ERR_NOT_INIT;
    } else if (c->target.dim != d->D) {
        return SMCGW_ERR_NOT_INIT;
    }
    return SMCGW_OK;
}

// Every device buffer the iteration's kernels use, sized before anything is
// queued (so that a capture records no allocation).
int reserve(smcgw_ctx* c, const smcgw_smc_iter_desc* d) {
    if (hipSetDevice(c->device) != hipSuccess) return SMCGW_ERR_HIP;
    if (!sampler_scratch(c, reweight_scratch_bytes(d->n_runs, d->P, d->D))) return SMCGW_ERR_OOM;
    if (mm_reserve(c, d->n_runs, d->P) != SMCGW_OK) return SMCGW_ERR_OOM;
    if (nuts_reserve(c, d->n_runs * d->P, false) != SMCGW_OK) return SMCGW_ERR_OOM;
    return SMCGW_OK;
}

int queue(smcgw_ctx* c, const smcgw_smc_iter_desc* d) {
    const int R = d->n_runs, P = d->P, D = d->D, n = R * P;
    double* out = nullptr;
    int rc = queue_reweight_resample(c, R, P, D, 0.0, d->alpha, d->seed, 0, d->theta, d->logl, d->grad,
                                     nullptr, d->ancestors, d->state, d->history, d->history_cap, &out);
    if (rc) return rc;
    rc = queue_mass_matrix_runs(c, R, P, D, d->theta, d->shrink, d->inv_mass, d->chol, d->mm_status, d->state);
    if (rc) return rc;
    if (d->chol_pp) {
        rc = queue_local_metric(c, n, D, d->theta, d->state, P, d->chol, d->chol_pp, d->metric_status);
        if (rc) return rc;
    }
    smcgw_nuts_params prm{};
    prm.step = d->step;
    prm.beta = 0.0;
    prm.max_delta_h = d->max_delta_h;
    prm.max_depth = d->max_depth;
    prm.uturn = d->uturn ? 1 : 0;
    prm.seed = d->seed;
    prm.iteration = 0;
    prm.chol_per_particle = d->chol_pp ? 1 : 0;
    prm.state_device = d->state;
    prm.run_size = P;
    if (d->nuts_form == SMCGW_NUTS_SWEEPS) {
        rc = smcgw_nuts_step_sweeps(c, n, D, d->theta, d->logl, d->grad, d->chol_pp ? d->chol_pp : d->chol, &prm,
                                    nullptr, d->depth, d->n_leapfrog, d->divergent, d->accept_stat, 8, nullptr);
    } else {
        // no start-order hint: a particle's leapfrog count hardly depends on its ancestor's, so the launch
        // deals the particles to the XCDs in stripes of neighbours instead
        rc = smcgw_nuts_step(c, n, D, d->theta, d->logl, d->grad, d->chol_pp ? d->chol_pp : d->chol, &prm,
                             nullptr, nullptr, d->precision, d->depth, d->n_leapfrog, d->divergent,
                             d->accept_stat);
    }
    if (rc) return rc;
    if (d->history)
        rc = queue_record(c, R, P, d->n_leapfrog, d->depth, d->divergent, d->mm_status,
                          d->chol_pp ? d->metric_status : nullptr, d->state, d->history, d->history_cap);
    return rc;
}

}  // namespace

extern "C" int smcgw_smc_iteration(smcgw_ctx* c, const smcgw_smc_iter_desc* desc) {
    int rc = check_desc(c, desc);
    if (rc) return rc;
    rc = reserve(c, desc);
    if (rc) return rc;
    return queue(c, desc);
}

extern "C" int smcgw_smc_graph_create(smcgw_ctx* c, const smcgw_smc_iter_desc* desc, smcgw_graph** out) {
    if (!out) return SMCGW_ERR_INVALID;
    *out = nullptr;
    int rc = check_desc(c, desc);
    if (rc) return rc;
    if (desc->nuts_form != SMCGW_NUTS_PERSISTENT) return SMCGW_ERR_INVALID;   // the sweeps wait for the host
    rc = reserve(c, desc);
    if (rc) return rc;
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SMCGW_ERR_HIP;
    const hipStream_t saved = c->stream;
    const unsigned saved_mask = c->timing_mask;
    c->stream = cap;
    c->timing_mask = 0;   // no timing events inside the graph
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        rc = queue(c, desc);
        ok = hipStreamEndCapture(cap, &g) == hipSuccess && rc == SMCGW_OK;
    }
    c->stream = saved;
    c->timing_mask = saved_mask;
    (void)hipStreamDestroy(cap);
    hipGraphExec_t exec = nullptr;
    if (ok) ok = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : SMCGW_ERR_HIP;
    }
    smcgw_graph* h = new smcgw_graph();
    h->c = c;
    h->graph = g;
    h->exec = exec;
    *out = h;
    return SMCGW_OK;
}

extern "C" int smcgw_graph_launch(smcgw_graph* g, int count) {
    if (!g || count < 0) return SMCGW_ERR_INVALID;
    if (hipSetDevice(g->c->device) != hipSuccess) return SMCGW_ERR_HIP;
    for (int k = 0; k < count; ++k)
        if (hipGraphLaunch(g->exec, g->c->stream) != hipSuccess) return SMCGW_ERR_HIP;
    return SMCGW_OK;
}

extern "C" int smcgw_graph_destroy(smcgw_graph* g) {
    if (!g) return SMCGW_ERR_INVALID;
    (void)hipSetDevice(g->c->device);
    (void)hipStreamSynchronize(g->c->stream);
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return SMCGW_OK;
}
