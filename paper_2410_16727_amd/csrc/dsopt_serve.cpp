// Serving loop (continuous batching) of the dsopt C ABI.
#include <hip/hip_runtime.h>

#include "dsopt.h"
#include "dsopt_internal.h"

struct Serve {};

void ds_serve_free(ds_plan*) {}

extern "C" {
int ds_serve_start(ds_plan*, int, int, void*) { return DS_ERR_STATE; }
int ds_serve_submit(ds_plan*, const ds_problem*, uint64_t*) { return DS_ERR_STATE; }
int ds_serve_step(ds_plan*) { return DS_ERR_STATE; }
int ds_serve_poll(ds_plan*, uint64_t, ds_result*, float*) { return DS_ERR_STATE; }
int ds_serve_stats(ds_plan*, ds_latency_stats*) { return DS_ERR_STATE; }
int ds_serve_stop(ds_plan*) { return DS_ERR_STATE; }
}
