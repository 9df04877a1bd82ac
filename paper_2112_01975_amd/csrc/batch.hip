// batch.hip -- batched sweep entry points (persistent kernel; see lbm2p.h).
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/lbm2p.h"

struct lbm_batch {
    std::string err;
};

namespace {
thread_local std::string g_batch_err;
}

extern "C" {
int lbm_batch_create(const lbm_params *, int, lbm_batch **out) {
    if (out) *out = nullptr;
    g_batch_err = "batched path not built in this version";
    return LBM_E_INVAL;
}
int lbm_batch_init_fields(lbm_batch *, int, const double *, const double *) { return LBM_E_INVAL; }
int lbm_batch_step(lbm_batch *, int64_t) { return LBM_E_INVAL; }
int lbm_batch_moments(lbm_batch *, int, double *, double *, double *) { return LBM_E_INVAL; }
void lbm_batch_destroy(lbm_batch *b) { delete b; }
const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_batch_err.c_str(); }
}
