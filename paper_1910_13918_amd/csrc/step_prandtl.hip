// Pr != 1 instantiations of the direct, records, matrix-core and row-segment
// stream + collide kernels.
#include "step_direct.hpp"
#include "step_mfma.hpp"
#include "step_records.hpp"
#include "step_rows.hpp"

namespace sllbm {

hipError_t launch_step_direct_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                 const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_direct_family<true>(fp32, model, c, t, fin, fout, flag, s);
}

hipError_t launch_step_records_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                  const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_records_family<true>(fp32, model, c, t, fin, fout, flag, s);
}

hipError_t launch_step_mfma_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_mfma_family<true>(fp32, model, c, t, fin, fout, flag, s);
}

hipError_t launch_step_rows_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s) {
  return launch_rows_family<true>(fp32, model, c, t, fin, fout, flag, s);
}

}  // namespace sllbm
