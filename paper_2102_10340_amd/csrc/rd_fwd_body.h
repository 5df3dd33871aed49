// rd_fwd_body.h -- the register-streamed forward pass over one tile, shared by
// the single-grid kernel (rd_forward.hip) and the batched kernel (rd_batch.hip).
//
// K Euler steps of Eq. (1)-(3) (arXiv 2102.10340, Sec. II.A) per pass over HBM.
// One 64-lane wavefront owns a strip of 64*CPL columns and a segment of output
// rows; it walks down the rows once, keeping three rows of (u, v) per time level
// in registers (see the slot scheme below).  East/west neighbours across lanes
// come from DPP wave shifts, north/south ones from the register window.
//
// The body is generic over the cell model M (rd_models.h): the FitzHugh-Nagumo
// kernels are its ModelFHN instance, and further models reuse the same
// streaming, tiling and boundary handling.  Models that read the diagonal
// neighbours get them from DPP shifts of the north and south rows.
#pragma once

#include <type_traits>

#include "rd_models.h"
#include "rd_stream.h"

namespace rd {

// Level-0 rows are fetched this many iterations before their first use
// (at most kFetchPast: the last fetches name rows past the walk).
constexpr int kFwdFetch = 3;
static_assert(kFwdFetch >= 1 && kFwdFetch <= kFetchPast, "level-0 fetch distance");

template <class M>
struct StreamArgsT {
    TileArgs t;
    const float *in;
    float *out;
    typename M::Params g;
    float *rec;           // recording: level j of the pass goes to state j of rec (null: off)
    unsigned rec_stride;  // bytes from one recorded state to the next
};
using StreamArgs = StreamArgsT<ModelFHN>;

// ROWS_IN: every row the tile reads, including the kFetchPast rows fetched
// past the end of its walk, lies inside the grid, so row offsets need no
// boundary mapping (true for all but the first and last segments of a strip).
// REC: 0 no recording; 1 record every level (states q0 .. q0+K-1 of the pass);
// 2 record the even levels only (the pass starts at an even time q0; level j
// goes to recorded state j/2), for the reverse pass that rebuilds odd states;
// 3 as 2 but without level 0, for a pass whose input already is that
// recorded state (the previous pass wrote its output there).
template <class M, int CPL, int K, int REC, bool FAST, bool ROWS_IN>
__device__ __forceinline__ void stream_body(const StreamArgsT<M> &A, const Tile<CPL> &t)
{
    const int C = A.t.C, R = A.t.R, bc = A.t.bc;
    const unsigned pbytes = 4u * (unsigned)R * (unsigned)C;  // one plane
    const unsigned rowb = 4u * (unsigned)C;
    const Buf iu(A.in, pbytes), iv(A.in + (size_t)R * C, pbytes);
    const Buf ou(A.out, pbytes), ov(A.out + (size_t)R * C, pbytes);
    // Recorded states, u plane then v plane each: state j at byte j*rec_stride.
    constexpr int kRecLast = REC >= 2 ? (K - 1) / 2 : K - 1;  // last recorded state of a pass
    const unsigned rstride = A.rec_stride;
    const Buf rb(REC ? A.rec : A.in, REC ? (unsigned)kRecLast * rstride + 2u * pbytes : 0u);
    const typename M::Params g = A.g;
    const int y0 = t.y0, y1 = t.y1;

    const int rbase = y0 - K;            // first row read (level 0)
    const int n_real = y1 - y0 + 2 * K;  // rows walked
    auto roff = [&](int r) -> unsigned {
        return ROWS_IN ? (unsigned)r * rowb : row_off(r, R, C, bc);
    };

    // Row q (counted from rbase) of time level j >= 1 lives in slot q % 3 of
    // level j.  Iteration `it` makes level-(j+1) row it-j-1 from level-j rows
    // it-j-2, it-j-1, it-j; the new row overwrites the slot of level-(j+1) row
    // it-j-4, which nothing needs any more.  Level 0 (the rows read from HBM)
    // has a six-slot ring instead: row q sits in slot q % 6 and is fetched
    // kFwdFetch iterations before it is first used, so the wait for it does not
    // also wait for the stores issued after it (vmcnt retires in issue order
    // and counts stores too).  With the loop unrolled six times every slot
    // index is a compile-time constant, so the windows rotate without
    // register copies.
    float l0u[6][CPL], l0v[6][CPL];
    float bu[K][3][CPL], bv[K][3][CPL];  // levels 1 .. K-1 (index 0 unused)
    // derive(u) of the same rows, in the same slots (kDerived models only)
    constexpr int KD = M::kDerived ? K : 1;
    float l0y[M::kDerived ? 6 : 1][CPL], by[KD][3][CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
#pragma unroll
        for (int q = 0; q < 6; ++q) l0u[q][e] = l0v[q][e] = 0.0f;
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < 3; ++q) bu[j][q][e] = bv[j][q][e] = 0.0f;
        if constexpr (M::kDerived) {
#pragma unroll
            for (int q = 0; q < 6; ++q) l0y[q][e] = 0.0f;
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int q = 0; q < 3; ++q) by[j][q][e] = 0.0f;
        }
    }
#pragma unroll
    for (int q = 0; q < kFwdFetch; ++q) {
        const unsigned ro = roff(rbase + q);
        load_row<CPL, FAST>(iu, ro, t, l0u[q]);
        load_row<CPL, FAST>(iv, ro, t, l0v[q]);
    }

    // Row m is an output row of the tile.  The recording passes test it with
    // one unsigned compare (their scalar unit is the busier one); the plain
    // pass keeps the two signed ones it was tuned with.
    auto inside = [&](const int m) __attribute__((always_inline)) {
        return REC ? (unsigned)(m - y0) < (unsigned)(y1 - y0) : (m >= y0 && m < y1);
    };

    // all: every level is active (it >= 2K); the recording passes run their
    // rounds past the pipeline fill with this set, which drops the per-level
    // activity tests.
    auto iteration = [&](const int it, const int S6, auto all) __attribute__((always_inline)) {
        constexpr bool kAll = decltype(all)::value;
        const int S = S6 % 3;
        // level-0 ring slots of rows it-2 (north), it-1 (centre), it (south)
        const int qN = (S6 + 4) % 6, qC = (S6 + 5) % 6, qS = S6;
        float tu[CPL], tv[CPL];  // row it-K of level K (the pass output)
        if constexpr (M::kDerived) {
#pragma unroll
            for (int e = 0; e < CPL; ++e) l0y[qS][e] = M::derive(l0u[qS][e]);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const Slots sl(S, j);
            float *du = j + 1 < K ? bu[j + 1][sl.cs] : tu;  // level j+1, row it-j-1
            float *dv = j + 1 < K ? bv[j + 1][sl.cs] : tv;
            const float *uN = j == 0 ? l0u[qN] : bu[j][sl.ps];
            const float *uC = j == 0 ? l0u[qC] : bu[j][sl.cs];
            const float *uS = j == 0 ? l0u[qS] : bu[j][sl.ns];
            const float *vN = j == 0 ? l0v[qN] : bv[j][sl.ps];
            const float *vC = j == 0 ? l0v[qC] : bv[j][sl.cs];
            const float *vS = j == 0 ? l0v[qS] : bv[j][sl.ns];
            // the u layer as the update sees it: derive(u) for kDerived models
            const float *yN = uN, *yC = uC, *yS = uS;
            if constexpr (M::kDerived) {
                yN = j == 0 ? l0y[qN] : by[j][sl.ps];
                yC = j == 0 ? l0y[qC] : by[j][sl.cs];
                yS = j == 0 ? l0y[qS] : by[j][sl.ns];
            }
            // Level j+1 has all three input rows from it = 2j+2 on; rows made
            // after it = n_real are beyond the segment's cone.
            if (kAll || (it >= 2 * j + 2 && it < n_real)) {
                // lane-shifted edge columns of the centre row (and, for models
                // reading diagonals, of the north and south rows)
                const float lu = from_left_lane(yC[CPL - 1]);
                const float ru = from_right_lane(yC[0]);
                const float lv = from_left_lane(vC[CPL - 1]);
                const float rv = from_right_lane(vC[0]);
                float luN = 0.0f, ruN = 0.0f, lvN = 0.0f, rvN = 0.0f;
                float luS = 0.0f, ruS = 0.0f, lvS = 0.0f, rvS = 0.0f;
                if (M::kDiag) {
                    luN = from_left_lane(yN[CPL - 1]);
                    ruN = from_right_lane(yN[0]);
                    lvN = from_left_lane(vN[CPL - 1]);
                    rvN = from_right_lane(vN[0]);
                    luS = from_left_lane(yS[CPL - 1]);
                    ruS = from_right_lane(yS[0]);
                    lvS = from_left_lane(vS[CPL - 1]);
                    rvS = from_right_lane(vS[0]);
                }
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    Nbhd n;
                    n.u = uC[e];
                    n.v = vC[e];
                    n.y = yC[e];
                    n.uN = yN[e];
                    n.uS = yS[e];
                    n.vN = vN[e];
                    n.vS = vS[e];
                    n.uW = e == 0 ? lu : yC[e - 1];
                    n.uE = e == CPL - 1 ? ru : yC[e + 1];
                    n.vW = e == 0 ? lv : vC[e - 1];
                    n.vE = e == CPL - 1 ? rv : vC[e + 1];
                    if (M::kDiag) {
                        n.uNW = e == 0 ? luN : yN[e - 1];
                        n.uNE = e == CPL - 1 ? ruN : yN[e + 1];
                        n.vNW = e == 0 ? lvN : vN[e - 1];
                        n.vNE = e == CPL - 1 ? rvN : vN[e + 1];
                        n.uSW = e == 0 ? luS : yS[e - 1];
                        n.uSE = e == CPL - 1 ? ruS : yS[e + 1];
                        n.vSW = e == 0 ? lvS : vS[e - 1];
                        n.vSE = e == CPL - 1 ? rvS : vS[e + 1];
                    }
                    M::update(g, n, du[e], dv[e]);
                    if constexpr (M::kDerived) {
                        if (j + 1 < K) by[j + 1][sl.cs][e] = M::derive(du[e]);
                    }
                }
            }
            // The next level-0 row is loaded before this iteration's stores:
            // vmcnt retires in issue order, so waiting for the load next
            // iteration then does not also wait for the stores.
            if (j == 0) {
                // Fetch level-0 row it+kFwdFetch into the slot of row
                // it+kFwdFetch-6, which no level reads any more.
                const unsigned ro = roff(rbase + it + kFwdFetch);
                load_row<CPL, FAST>(iu, ro, t, l0u[(S6 + kFwdFetch) % 6]);
                load_row<CPL, FAST>(iv, ro, t, l0v[(S6 + kFwdFetch) % 6]);
                if (REC == 1 || REC == 2) {
                    const int m = rbase + it;  // level-0 row it
                    if (inside(m)) {
                        const unsigned o = 4u * (unsigned)m * C;
                        store_row<CPL, FAST>(rb, o, C, t, l0u[qS]);
                        store_row<CPL, FAST>(rb, o + pbytes, C, t, l0v[qS]);
                    }
                }
            }
            if (REC && j + 1 < K && (REC == 1 || (j + 1) % 2 == 0) &&
                (kAll || (it >= 2 * j + 2 && it < n_real))) {
                const int m = rbase + it - j - 1;  // level-(j+1) row just made
                if (inside(m)) {
                    const unsigned o = (unsigned)(REC >= 2 ? (j + 1) / 2 : j + 1) * rstride +
                                       4u * (unsigned)m * C;
                    store_row<CPL, FAST>(rb, o, C, t, bu[j + 1][sl.cs]);
                    store_row<CPL, FAST>(rb, o + pbytes, C, t, bv[j + 1][sl.cs]);
                }
            }
        }
        const int m = rbase + it - K;  // row of level K now in (tu, tv)
        if (inside(m)) {
            const unsigned o = 4u * (unsigned)m * C;
            store_row<CPL, FAST>(ou, o, C, t, tu);
            store_row<CPL, FAST>(ov, o, C, t, tv);
        }
    };

    // Iterations from n_real on would only fetch rows nobody reads: leave the
    // unrolled body as soon as the walk is done (uniform branches).
    const std::integral_constant<bool, false> ramp{};
    if constexpr (REC == 0) {
        for (int it = 0; it < n_real; it += 6) {
            iteration(it, 0, ramp);
            if (it + 1 >= n_real) break;
            iteration(it + 1, 1, ramp);
            if (it + 2 >= n_real) break;
            iteration(it + 2, 2, ramp);
            if (it + 3 >= n_real) break;
            iteration(it + 3, 3, ramp);
            if (it + 4 >= n_real) break;
            iteration(it + 4, 4, ramp);
            if (it + 5 >= n_real) break;
            iteration(it + 5, 5, ramp);
        }
    } else {
        // every level is active from it = 2K on; the rounds from the first
        // multiple of six past that run the copy without the tests
        constexpr int kSteady = (2 * K + 5) / 6 * 6;
        int it = 0;
        for (; it < kSteady && it < n_real; it += 6) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (it + q >= n_real) break;
                iteration(it + q, q, ramp);
            }
        }
        for (; it < n_real; it += 6) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (it + q >= n_real) break;
                iteration(it + q, q, std::integral_constant<bool, true>{});
            }
        }
    }
}

}  // namespace rd
