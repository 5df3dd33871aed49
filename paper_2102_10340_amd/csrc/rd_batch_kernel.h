// rd_batch_kernel.h -- the batched register-streamed forward kernel: one
// launch advances every instance of a packed batch by K steps of Eq. (1)-(3)
// (arXiv 2102.10340, Sec. II.A), one tile of the flat tile list per wavefront,
// with the single-grid body (rd_fwd_body.h).  Its instances are compiled in
// rd_batch_r0.hip (plain steps) and rd_batch_rec.hip (recording passes).
#pragma once

#include <utility>

#include "rd_fwd_body.h"
#include "rd_launch.h"

namespace rd {

struct BatchArgs {
    const BatchTile *tiles;
    const BatchInst *insts;
    int ntiles;
    const float *in;
    float *out;
    int bc, wout, kpad;
    float *rec;           // packed trajectory, state of level 0 (REC only)
    unsigned rec_stride;  // bytes between packed states
};

// REC: 0 plain steps; 1 record every level; 2 record the even levels (passes
// start at even times); 3 as 2 without level 0 (the input is that state).
template <int CPL, int K, int REC>
__global__ __launch_bounds__(64) void batch_step_kernel(BatchArgs B)
{
    const int id = blockIdx.x;
    if (id >= B.ntiles) return;
    const BatchTile bt = B.tiles[id];
    const BatchInst in = B.insts[bt.inst];
    StreamArgs A;
    A.t.R = in.R;
    A.t.C = in.C;
    A.t.bc = B.bc;
    A.t.wout = B.wout;
    A.t.kpad = B.kpad;
    A.t.h = 0;
    A.t.nsegs = 0;
    A.t.ntiles = 0;
    A.t.per_xcd = 0;
    A.t.vec_ok = (in.C % CPL) == 0;
    A.in = B.in + in.off;
    A.out = B.out + in.off;
    A.g = in.g;
    A.rec = REC ? B.rec + in.off : nullptr;
    A.rec_stride = B.rec_stride;
    Tile<CPL> t;
    t.setup(A.t, id, bt.x0, bt.y0, bt.y1);
    if (t.fast) {
        if (t.y0 >= K && t.y1 + K + kFetchPast <= in.R)
            stream_body<ModelFHN, CPL, K, REC, true, true>(A, t);
        else
            stream_body<ModelFHN, CPL, K, REC, true, false>(A, t);
    } else {
        stream_body<ModelFHN, CPL, K, REC, false, false>(A, t);
    }
}

using BatchFn = void (*)(BatchArgs);

template <int CPL, int REC, int... Ks>
constexpr BatchFn batch_pick(int k, std::integer_sequence<int, Ks...>)
{
    BatchFn f = nullptr;
    ((f = (k == Ks + 1) ? &batch_step_kernel<CPL, Ks + 1, REC> : f), ...);
    return f;
}

// Plain passes: cpl 1, 2 (depth <= 16) or 4 (depth <= 12).
BatchFn batch_fn_r0(int cpl, int depth);
// Recording passes (rec 1, 2 or 3 as above): cpl 1 or 2, depth <= 8.
BatchFn batch_fn_rec(int rec, int cpl, int depth);

}  // namespace rd
