// rd_fwd_kernel.h -- the single-grid register-streamed forward kernel and the
// tables that map a pass shape onto its template instance.
//
// stream_step_kernel<CPL, K, REC> runs K steps of Eq. (1)-(3) (arXiv
// 2102.10340, Sec. II.A) per pass over HBM for one tile per wavefront; the
// body is rd_fwd_body.h.  The instances are spread over several translation
// units (rd_fwd_r*.hip), one per recording mode and columns-per-lane setting,
// so that they compile in parallel; each defines one table function with
// RD_STREAM_TABLE.
#pragma once

#include <utility>

#include "rd_fwd_body.h"
#include "rd_launch.h"

namespace rd {

template <int CPL, int K, int REC>
__global__ __launch_bounds__(64) void stream_step_kernel(StreamArgs A)
{
    Tile<CPL> t;
    if (!t.init(A.t)) return;
    if (t.fast) {
        if (t.y0 >= K && t.y1 + K + kFetchPast <= A.t.R)
            stream_body<ModelFHN, CPL, K, REC, true, true>(A, t);
        else
            stream_body<ModelFHN, CPL, K, REC, true, false>(A, t);
    } else {
        stream_body<ModelFHN, CPL, K, REC, false, false>(A, t);
    }
}

using StreamFn = void (*)(StreamArgs);

template <int CPL, int REC, int... Ks>
constexpr StreamFn stream_pick(int k, std::integer_sequence<int, Ks...>)
{
    StreamFn f = nullptr;
    ((f = (k == Ks + 1) ? &stream_step_kernel<CPL, Ks + 1, REC> : f), ...);
    return f;
}

// Kernel for `depth` steps (1 .. NK) at recording mode REC and CPL columns per
// lane; null if not instantiated.
#define RD_STREAM_TABLE(NAME, REC, CPL, NK)                                          \
    StreamFn NAME(int depth)                                                         \
    {                                                                                \
        return stream_pick<CPL, REC>(depth, std::make_integer_sequence<int, NK>{});  \
    }

// Recording modes (rd_fwd_body.h): 0 none, 1 every level, 2 / 3 even levels.
StreamFn stream_fn_r0c1(int depth);
StreamFn stream_fn_r0c2(int depth);
StreamFn stream_fn_r0c4(int depth);
StreamFn stream_fn_r1c1(int depth);
StreamFn stream_fn_r1c2(int depth);
StreamFn stream_fn_r1c4(int depth);
StreamFn stream_fn_r2c1(int depth);  // even-level recording: depth <= 8
StreamFn stream_fn_r2c2(int depth);
StreamFn stream_fn_r3c1(int depth);
StreamFn stream_fn_r3c2(int depth);

}  // namespace rd
