#include "common.h"
extern "C" {
int32_t csdyn_ras_workspace_bytes(const csdyn_opctx *, const csdyn_ras_opts *, size_t *) { return CSDYN_EINVAL; }
int32_t csdyn_ras_setup(const csdyn_opctx *, const csdyn_ras_opts *, void *, size_t, void *, csdyn_ras **) { return CSDYN_EINVAL; }
int32_t csdyn_ras_apply(const csdyn_ras *, const double *, double *, void *) { return CSDYN_EINVAL; }
void csdyn_ras_destroy(csdyn_ras *) {}
int32_t csdyn_gmres_workspace_bytes(const csdyn_opctx *, const csdyn_gmres_opts *, size_t *) { return CSDYN_EINVAL; }
int32_t csdyn_gmres_solve(const csdyn_opctx *, const csdyn_ras *, const csdyn_gmres_opts *, const double *, double *, void *, size_t, void *, csdyn_gmres_stats *) { return CSDYN_EINVAL; }
}
