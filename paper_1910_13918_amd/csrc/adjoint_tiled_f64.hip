// double instantiation of the adjoint's tiled transposed gather.
#include "adjoint_tiled.hpp"

namespace sllbm {

template hipError_t launch_adjoint_step_tiled_t<double>(int, const StepConsts &, const DevTables &,
                                                     const void *, const double *, void *,
                                                     hipStream_t);

}  // namespace sllbm
