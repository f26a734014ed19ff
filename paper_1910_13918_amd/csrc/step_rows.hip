// BGK (Pr = 1) instantiation of the row-segment stream + collide kernels.
#include "step_rows.hpp"

namespace sllbm {

hipError_t launch_step_rows(int fp32, int model, const StepConsts &c, const DevTables &t,
                            const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_rows_family<false>(fp32, model, c, t, fin, fout, flag, s);
}

}  // namespace sllbm
