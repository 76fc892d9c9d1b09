// FP32 instantiations of the fused Chebyshev step (hv_kernels.h).
#include "hv_kernels.h"

namespace polfed {

template void launch_step_batched<float>(hipStream_t, int, const StepArgs<float> &,
                                   const BatchItem<float> *, int, long long, long long,
                                   long long, const BatchTables &, const StepShape &, int);
template long long batched_tile_rows<float>(int, const StepShape &);
template void launch_step<float>(hipStream_t, int, const StepArgs<float> &, const StepShape &,
                                 int);

}  // namespace polfed
