// amr_stage_hydro_f64.hip - the stage kernel's instantiations for hydro (5 variables), FP64 throughout.
#include "amr_stage.h"

namespace amr {

hipError_t launch_stage_hydro_f64(int shape, int stage, int grid, hipStream_t s, const StageArgs& a) {
  return launch_stage_hydro_t<double>(shape, stage, grid, s, a);
}
const void* stage_kernel_ptr_hydro_f64(int shape, int stage, bool rec) {
  return stage_kernel_ptr_hydro_t<double>(shape, stage, rec);
}

}  // namespace amr
