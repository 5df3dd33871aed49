// Batched forward kernel instances, recording passes (rd_batch_kernel.h).
#include "rd_batch_kernel.h"

namespace rd {

BatchFn batch_fn_rec(int rec, int cpl, int depth)
{
    using S8 = std::make_integer_sequence<int, 8>;
    if (cpl == 2) {
        if (rec == 1) return batch_pick<2, 1>(depth, S8{});
        if (rec == 2) return batch_pick<2, 2>(depth, S8{});
        if (rec == 3) return batch_pick<2, 3>(depth, S8{});
    } else if (cpl == 1) {
        if (rec == 1) return batch_pick<1, 1>(depth, S8{});
        if (rec == 2) return batch_pick<1, 2>(depth, S8{});
        if (rec == 3) return batch_pick<1, 3>(depth, S8{});
    }
    return nullptr;
}

}  // namespace rd
