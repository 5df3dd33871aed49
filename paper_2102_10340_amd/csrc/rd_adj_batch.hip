// Reverse-pass kernel instances over batches: batch_adjoint_kernel and
// batch_adjoint_pair_kernel<CPL, KB, LAMS> (rd_adj_body.h).
#include "rd_adj_body.h"

namespace rd {

namespace {

template <bool LAMS>
BatchAdjFn pick_batch_adj_pair(int cpl, int depth)
{
    if (cpl == 1) {
        if (depth == 2) return &batch_adjoint_pair_kernel<1, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_pair_kernel<1, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_pair_kernel<1, 8, LAMS>;
    } else if (cpl == 2) {
        if (depth == 2) return &batch_adjoint_pair_kernel<2, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_pair_kernel<2, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_pair_kernel<2, 8, LAMS>;
    }
    return nullptr;
}

template <bool LAMS>
BatchAdjFn pick_batch_adj(int cpl, int depth)
{
    if (cpl == 1) {
        if (depth == 2) return &batch_adjoint_kernel<1, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_kernel<1, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_kernel<1, 8, LAMS>;
        if (depth == 1) return &batch_adjoint_kernel<1, 1, LAMS>;
    } else if (cpl == 2) {
        if (depth == 2) return &batch_adjoint_kernel<2, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_kernel<2, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_kernel<2, 8, LAMS>;
        if (depth == 1) return &batch_adjoint_kernel<2, 1, LAMS>;
    }
    return nullptr;
}

}  // namespace

BatchAdjFn batch_adj_fn(bool paired, bool lams, int cpl, int depth)
{
    if (paired) return lams ? pick_batch_adj_pair<true>(cpl, depth) : pick_batch_adj_pair<false>(cpl, depth);
    return lams ? pick_batch_adj<true>(cpl, depth) : pick_batch_adj<false>(cpl, depth);
}

}  // namespace rd
