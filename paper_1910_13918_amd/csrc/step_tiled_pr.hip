// Pr != 1 instantiation of the tiled stream + collide kernels (its own
// translation unit so that it compiles in parallel with the others).
#include "step_tiled.hpp"

namespace sllbm {

hipError_t launch_step_tiled_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_tiled_family<true>(fp32, model, c, t, fin, fout, flag, s);
}

}  // namespace sllbm
