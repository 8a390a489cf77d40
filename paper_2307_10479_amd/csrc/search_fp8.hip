// Search kernels over FP8 E4M3 rows.
#include "search_impl.h"

namespace degk {
KernelFn pick_kernel_fp8(int metric, int qch, int rreg, int mode) {
    return pick_m<DT_FP8>(metric, qch, rreg, mode);
}
}  // namespace degk
