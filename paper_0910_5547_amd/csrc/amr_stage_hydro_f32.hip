// amr_stage_hydro_f32.hip - the stage kernel's instantiations for hydro (5 variables), FP32 reconstruction and fluxes (the mixed path).
#include "amr_stage.h"

namespace amr {

hipError_t launch_stage_hydro_f32(int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  return launch_stage_hydro_t<float>(shape, stage, grid, s, a);
}
const void* stage_kernel_ptr_hydro_f32(int shape, int stage, bool rec) {
  return stage_kernel_ptr_hydro_t<float>(shape, stage, rec);
}

}  // namespace amr
