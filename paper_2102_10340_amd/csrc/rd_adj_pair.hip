// Reverse-pass kernel instances: adjoint_pair_kernel<CPL, KB, LAMS> (rd_adj_body.h).
#include "rd_adj_body.h"

namespace rd {

namespace {

template <bool LAMS>
AdjFn pick_adj_pair(int cpl, int depth)
{
    if (cpl == 1) {
        if (depth == 2) return &adjoint_pair_kernel<1, 2, LAMS>;
        if (depth == 4) return &adjoint_pair_kernel<1, 4, LAMS>;
        if (depth == 6) return &adjoint_pair_kernel<1, 6, LAMS>;
        if (depth == 8) return &adjoint_pair_kernel<1, 8, LAMS>;
    } else if (cpl == 2) {
        if (depth == 2) return &adjoint_pair_kernel<2, 2, LAMS>;
        if (depth == 4) return &adjoint_pair_kernel<2, 4, LAMS>;
        if (depth == 6) return &adjoint_pair_kernel<2, 6, LAMS>;
        if (depth == 8) return &adjoint_pair_kernel<2, 8, LAMS>;
    }
    return nullptr;
}

}  // namespace

AdjFn adj_fn_pair(bool lams, int cpl, int depth)
{
    return lams ? pick_adj_pair<true>(cpl, depth) : pick_adj_pair<false>(cpl, depth);
}

}  // namespace rd
