// Search kernels over BF16 rows.
#include "search_impl.h"

namespace degk {
KernelFn pick_kernel_bf16(int metric, int qch, int rreg, int mode) {
    return pick_m<DT_BF16>(metric, qch, rreg, mode);
}
}  // namespace degk
