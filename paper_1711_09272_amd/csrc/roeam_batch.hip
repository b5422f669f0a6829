// roeam_batch.hip -- continuous-batching engine of the C ABI (batch submit,
// run and poll).
#include <hip/hip_runtime.h>

#include "../../include/roeam.h"
#include "roeam_internal.hpp"

extern "C" {

void roeam_batch_release(roeam_ctx *) {}

roeam_status roeam_batch_reserve(roeam_ctx *, size_t) { return ROEAM_EINVAL; }
size_t roeam_batch_footprint(const roeam_grid *) { return 0; }
roeam_status roeam_batch_submit(roeam_ctx *, int, const roeam_solve_desc *, uint64_t *) { return ROEAM_EINVAL; }
roeam_status roeam_batch_run(roeam_ctx *, long, int *) { return ROEAM_EINVAL; }
roeam_status roeam_batch_poll(roeam_ctx *, uint64_t, int *, roeam_step_stats *) { return ROEAM_EINVAL; }

} // extern "C"
