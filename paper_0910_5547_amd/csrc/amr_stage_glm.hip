// amr_stage_glm.hip - the stage kernel's instantiations for GLM-MHD (9 variables), both precisions.
#include "amr_stage.h"

namespace amr {

hipError_t launch_stage_glm9(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  return launch_stage_mhd_t<NVAR_GLM>(mixed, shape, stage, grid, s, a);
}
const void* stage_kernel_ptr_glm9(int mixed, int shape, int stage, bool rec) {
  return stage_kernel_ptr_mhd_t<NVAR_GLM>(mixed, shape, stage, rec);
}

}  // namespace amr
