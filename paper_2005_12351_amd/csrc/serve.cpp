// Serving loop (continuous batching) -- placeholder until implemented.
#include "fmm_internal.h"

int serve_destroy(fmm_ctx *) { return FMM_OK; }
extern "C" int fmm_serve_start(fmm_ctx *, int) { set_error("serving not built yet"); return FMM_EINVAL; }
extern "C" int fmm_submit(fmm_ctx *, const fmm_request *, uint64_t *) { set_error("serving not started"); return FMM_ESTATE; }
extern "C" int fmm_poll(fmm_ctx *, uint64_t, int *) { set_error("serving not started"); return FMM_ESTATE; }
extern "C" int fmm_wait(fmm_ctx *, uint64_t, double) { set_error("serving not started"); return FMM_ESTATE; }
extern "C" int fmm_request_times(fmm_ctx *, uint64_t, double *, int64_t *) { set_error("serving not started"); return FMM_ESTATE; }
extern "C" int fmm_serve_stop(fmm_ctx *) { return FMM_OK; }
