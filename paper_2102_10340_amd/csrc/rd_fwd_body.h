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

#include "rd_models.h"
#include "rd_stream.h"

namespace rd {

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
// goes to recorded state j/2), for the reverse pass that rebuilds odd states.
template <class M, int CPL, int K, int REC, bool FAST, bool ROWS_IN>
__device__ __forceinline__ void stream_body(const StreamArgsT<M> &A, const Tile<CPL> &t)
{
    const int C = A.t.C, R = A.t.R, bc = A.t.bc;
    const unsigned pbytes = 4u * (unsigned)R * (unsigned)C;  // one plane
    const unsigned rowb = 4u * (unsigned)C;
    const Buf iu(A.in, pbytes), iv(A.in + (size_t)R * C, pbytes);
    const Buf ou(A.out, pbytes), ov(A.out + (size_t)R * C, pbytes);
    // Recorded states, u plane then v plane each: state j at byte j*rec_stride.
    constexpr int kRecLast = REC == 2 ? (K - 1) / 2 : K - 1;  // last recorded state of a pass
    const unsigned rstride = A.rec_stride;
    const Buf rb(REC ? A.rec : A.in, REC ? (unsigned)kRecLast * rstride + 2u * pbytes : 0u);
    const typename M::Params g = A.g;
    const int y0 = t.y0, y1 = t.y1;

    const int rbase = y0 - K;                 // first row read (level 0)
    const int n_real = y1 - y0 + 2 * K;       // rows walked
    const int n_iter = (n_real + 2) / 3 * 3;  // ... padded to a multiple of 3
    auto roff = [&](int r) -> unsigned {
        return ROWS_IN ? (unsigned)r * rowb : row_off(r, R, C, bc);
    };

    // Row q (counted from rbase) of time level j lives in slot q % 3 of level
    // j.  Iteration `it` reads level-0 row it and makes level-(j+1) row it-j-1
    // from level-j rows it-j-2, it-j-1, it-j; the new row overwrites the slot of
    // level-(j+1) row it-j-4, which nothing needs any more.  With the loop
    // unrolled three times every slot index is a compile-time constant, so the
    // window rotates without register copies.
    float bu[K][3][CPL], bv[K][3][CPL];
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int e = 0; e < CPL; ++e) bu[j][q][e] = bv[j][q][e] = 0.0f;
    {
        const unsigned ro = roff(rbase);
        load_row<CPL, FAST>(iu, ro, t, bu[0][0]);
        load_row<CPL, FAST>(iv, ro, t, bv[0][0]);
    }

    auto iteration = [&](const int it, const int S) __attribute__((always_inline)) {
        float tu[CPL], tv[CPL];  // row it-K of level K (the pass output)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const Slots sl(S, j);
            float *du = j + 1 < K ? bu[j + 1][sl.cs] : tu;  // level j+1, row it-j-1
            float *dv = j + 1 < K ? bv[j + 1][sl.cs] : tv;
            // Level j+1 has all three input rows from it = 2j+2 on; rows made
            // after it = n_real are beyond the segment's cone.
            if (it >= 2 * j + 2 && it < n_real) {
                // lane-shifted edge columns of the centre row (and, for models
                // reading diagonals, of the north and south rows)
                const float lu = from_left_lane(bu[j][sl.cs][CPL - 1]);
                const float ru = from_right_lane(bu[j][sl.cs][0]);
                const float lv = from_left_lane(bv[j][sl.cs][CPL - 1]);
                const float rv = from_right_lane(bv[j][sl.cs][0]);
                float luN = 0.0f, ruN = 0.0f, lvN = 0.0f, rvN = 0.0f;
                float luS = 0.0f, ruS = 0.0f, lvS = 0.0f, rvS = 0.0f;
                if (M::kDiag) {
                    luN = from_left_lane(bu[j][sl.ps][CPL - 1]);
                    ruN = from_right_lane(bu[j][sl.ps][0]);
                    lvN = from_left_lane(bv[j][sl.ps][CPL - 1]);
                    rvN = from_right_lane(bv[j][sl.ps][0]);
                    luS = from_left_lane(bu[j][sl.ns][CPL - 1]);
                    ruS = from_right_lane(bu[j][sl.ns][0]);
                    lvS = from_left_lane(bv[j][sl.ns][CPL - 1]);
                    rvS = from_right_lane(bv[j][sl.ns][0]);
                }
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    Nbhd n;
                    n.u = bu[j][sl.cs][e];
                    n.v = bv[j][sl.cs][e];
                    n.uN = bu[j][sl.ps][e];
                    n.uS = bu[j][sl.ns][e];
                    n.vN = bv[j][sl.ps][e];
                    n.vS = bv[j][sl.ns][e];
                    n.uW = e == 0 ? lu : bu[j][sl.cs][e - 1];
                    n.uE = e == CPL - 1 ? ru : bu[j][sl.cs][e + 1];
                    n.vW = e == 0 ? lv : bv[j][sl.cs][e - 1];
                    n.vE = e == CPL - 1 ? rv : bv[j][sl.cs][e + 1];
                    if (M::kDiag) {
                        n.uNW = e == 0 ? luN : bu[j][sl.ps][e - 1];
                        n.uNE = e == CPL - 1 ? ruN : bu[j][sl.ps][e + 1];
                        n.vNW = e == 0 ? lvN : bv[j][sl.ps][e - 1];
                        n.vNE = e == CPL - 1 ? rvN : bv[j][sl.ps][e + 1];
                        n.uSW = e == 0 ? luS : bu[j][sl.ns][e - 1];
                        n.uSE = e == CPL - 1 ? ruS : bu[j][sl.ns][e + 1];
                        n.vSW = e == 0 ? lvS : bv[j][sl.ns][e - 1];
                        n.vSE = e == CPL - 1 ? rvS : bv[j][sl.ns][e + 1];
                    }
                    M::update(g, n, du[e], dv[e]);
                }
            }
            // The next level-0 row is loaded before this iteration's stores:
            // vmcnt retires in issue order, so waiting for the load next
            // iteration then does not also wait for the stores.
            if (j == 0) {
                // Level-0 row it-2 is spent: fetch row it+1 into its slot.
                const unsigned ro = roff(rbase + it + 1);
                load_row<CPL, FAST>(iu, ro, t, bu[0][sl.ps]);
                load_row<CPL, FAST>(iv, ro, t, bv[0][sl.ps]);
                if (REC) {
                    const int m = rbase + it;  // level-0 row it
                    if (m >= y0 && m < y1) {
                        const unsigned o = 4u * (unsigned)m * C;
                        store_row<CPL, FAST>(rb, o, C, t, bu[0][sl.ns]);
                        store_row<CPL, FAST>(rb, o + pbytes, C, t, bv[0][sl.ns]);
                    }
                }
            }
            if (REC && j + 1 < K && (REC == 1 || (j + 1) % 2 == 0) && it >= 2 * j + 2 &&
                it < n_real) {
                const int m = rbase + it - j - 1;  // level-(j+1) row just made
                if (m >= y0 && m < y1) {
                    const unsigned o = (unsigned)(REC == 2 ? (j + 1) / 2 : j + 1) * rstride +
                                       4u * (unsigned)m * C;
                    store_row<CPL, FAST>(rb, o, C, t, bu[j + 1][sl.cs]);
                    store_row<CPL, FAST>(rb, o + pbytes, C, t, bv[j + 1][sl.cs]);
                }
            }
        }
        const int m = rbase + it - K;  // row of level K now in (tu, tv)
        if (m >= y0 && m < y1) {
            const unsigned o = 4u * (unsigned)m * C;
            store_row<CPL, FAST>(ou, o, C, t, tu);
            store_row<CPL, FAST>(ov, o, C, t, tv);
        }
    };

    for (int it = 0; it < n_iter; it += 3) {
        iteration(it, 0);
        iteration(it + 1, 1);
        iteration(it + 2, 2);
    }
}

}  // namespace rd
