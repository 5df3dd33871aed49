// Reverse-pass kernel instances: adjoint_kernel<CPL, KB, LAMS> (rd_adj_body.h).
#include "rd_adj_body.h"

namespace rd {

namespace {

template <int CPL, bool LAMS, int... Ks>
constexpr AdjFn pick(int k, std::integer_sequence<int, Ks...>)
{
    AdjFn f = nullptr;
    ((f = (k == Ks + 1) ? &adjoint_kernel<CPL, Ks + 1, LAMS> : f), ...);
    return f;
}

template <bool LAMS>
AdjFn pick_adj(int cpl, int depth)
{
    if (cpl == 4) return pick<4, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl4>{});
    if (cpl == 2) return pick<2, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl2>{});
    if (cpl == 1) return pick<1, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl1>{});
    return nullptr;
}

}  // namespace

AdjFn adj_fn_plain(bool lams, int cpl, int depth)
{
    return lams ? pick_adj<true>(cpl, depth) : pick_adj<false>(cpl, depth);
}

}  // namespace rd
