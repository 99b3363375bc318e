// Entry points not implemented yet: they report FEM_ERR_UNSUPPORTED.
#include "fem.h"
#include "fem_internal.hpp"

namespace femq {
int transpose_block_threads(int, int, int, int, int) { return 0; }
hipError_t launch_residual_transpose(int, int, int, int, const ResidualArgs&, const Launch&) {
    return hipErrorInvalidValue;
}
}  // namespace femq

using namespace femq;
extern "C" {
fem_status fem_batch_plan_create(const fem_mesh_desc*, int, int, fem_batch_plan**) {
    set_error("fem_batch_plan_create: not implemented");
    return FEM_ERR_UNSUPPORTED;
}
fem_status fem_batch_run(fem_batch_plan*, void*) { set_error("not implemented"); return FEM_ERR_UNSUPPORTED; }
fem_status fem_batch_capture(fem_batch_plan*, void*) { set_error("not implemented"); return FEM_ERR_UNSUPPORTED; }
fem_status fem_batch_replay(fem_batch_plan*, void*) { set_error("not implemented"); return FEM_ERR_UNSUPPORTED; }
void fem_batch_plan_destroy(fem_batch_plan*) {}
fem_status fem_autotune(int, int, int, int, int64_t, const char*) { set_error("not implemented"); return FEM_ERR_UNSUPPORTED; }
fem_status fem_load_tuning(const char*) { set_error("not implemented"); return FEM_ERR_NO_TUNING; }
}
