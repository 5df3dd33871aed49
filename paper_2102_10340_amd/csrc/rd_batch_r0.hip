// Batched forward kernel instances, plain steps (rd_batch_kernel.h).
#include "rd_batch_kernel.h"

namespace rd {

BatchFn batch_fn_r0(int cpl, int depth)
{
    if (cpl == 4) return batch_pick<4, 0>(depth, std::make_integer_sequence<int, kMaxDepthCpl4>{});
    if (cpl == 2) return batch_pick<2, 0>(depth, std::make_integer_sequence<int, kMaxDepthCpl2>{});
    if (cpl == 1) return batch_pick<1, 0>(depth, std::make_integer_sequence<int, kMaxDepthCpl1>{});
    return nullptr;
}

}  // namespace rd
