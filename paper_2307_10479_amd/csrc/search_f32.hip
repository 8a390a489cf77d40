// Search kernels over FP32 rows.
#include "search_impl.h"

namespace degk {
KernelFn pick_kernel_f32(int metric, int qch, int rreg, int mode) {
    return pick_m<DT_F32>(metric, qch, rreg, mode);
}
}  // namespace degk
