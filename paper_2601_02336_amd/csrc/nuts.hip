// NUTS transition kernels (placeholder until the persistent kernel lands).
#include "common.h"
#include "context.h"

extern "C" int smcgw_nuts_step(smcgw_ctx* c, int P, int D, double* theta, double* logl, double* grad,
                               const double* chol, const smcgw_nuts_params* params,
                               const int32_t* max_depth_per_particle, int precision, int32_t* depth,
                               int32_t* n_leapfrog, uint8_t* divergent, double* accept_stat) {
    (void)c; (void)P; (void)D; (void)theta; (void)logl; (void)grad; (void)chol; (void)params;
    (void)max_depth_per_particle; (void)precision; (void)depth; (void)n_leapfrog; (void)divergent; (void)accept_stat;
    return SMCGW_ERR_NOT_INIT;
}
