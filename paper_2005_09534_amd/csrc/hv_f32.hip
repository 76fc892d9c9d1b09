// FP32 instantiations of the fused Chebyshev step (hv_kernels.h).
#include "hv_kernels.h"

namespace polfed {

template void launch_step_batched<float>(hipStream_t, int, const StepArgs<float> &,
                                         const BatchItem<float> *, int, long long, long long,
                                         const StepShape &, int);
template void launch_step<float>(hipStream_t, int, const StepArgs<float> &, const StepShape &,
                                 int);

}  // namespace polfed
