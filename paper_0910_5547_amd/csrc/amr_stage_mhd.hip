// amr_stage_mhd.hip - the stage kernel's instantiations for ideal MHD (8 variables), both precisions.
#include "amr_stage.h"

namespace amr {

hipError_t launch_stage_mhd8(int mixed, int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  return launch_stage_mhd_t<NVAR_MHD>(mixed, shape, stage, grid, s, a);
}
const void* stage_kernel_ptr_mhd8(int mixed, int shape, int stage, bool rec) {
  return stage_kernel_ptr_mhd_t<NVAR_MHD>(mixed, shape, stage, rec);
}

}  // namespace amr
