// rd_stream.h -- tile geometry and row I/O shared by the register-streamed
// kernels (forward and adjoint).
//
// A pass over an R x C grid is cut into strips of 64*CPL columns (CPL adjacent
// columns per lane of one 64-lane wavefront) and segments of h output rows.  A
// strip overlaps its neighbours by kpad halo columns on each side and a segment
// reads K halo rows above and below, taken from the boundary-extended grid
// (map_index), so a wavefront can run K time levels on its tile without
// talking to any other wavefront.
#pragma once

#include "rd_common.h"

namespace rd {

template <int CPL>
using vecf = float __attribute__((ext_vector_type(CPL)));

struct TileArgs {
    int R, C, bc;
    int wout, kpad, h, nsegs, ntiles, per_xcd;
    int vec_ok;  // C % CPL == 0: rows of a plane keep CPL-float alignment
};

// Where one wavefront's tile sits, and which of its lanes own output columns.
template <int CPL>
struct Tile {
    int tile;            // tile index (strip-major)
    int x0;              // first extended column of the strip
    int y0, y1;          // output rows [y0, y1)
    int cx;              // first column of this lane
    bool fast;           // the whole strip lies inside the grid: vector loads
    bool lane_out;       // this lane's columns are output columns of the tile
    bool lane_vec;       // ... and can be stored with one vector store
    int mc[CPL];         // boundary-mapped column of each of the lane's columns

    __device__ __forceinline__ bool init(const TileArgs &A)
    {
        tile = xcd_tile(blockIdx.x, A.per_xcd);
        if (tile >= A.ntiles) return false;
        const int strip = tile / A.nsegs;
        const int seg = tile - strip * A.nsegs;
        x0 = strip * A.wout - A.kpad;
        y0 = seg * A.h;
        y1 = min(y0 + A.h, A.R);
        cx = x0 + CPL * (int)threadIdx.x;
        fast = A.vec_ok && x0 >= 0 && x0 + 64 * CPL <= A.C;
#pragma unroll
        for (int e = 0; e < CPL; ++e) mc[e] = map_index(cx + e, A.C, A.bc);
        const int oc = cx - x0;
        lane_out = oc >= A.kpad && oc < A.kpad + A.wout && cx < A.C;
        lane_vec = lane_out && A.vec_ok && cx + CPL <= A.C;
        return true;
    }

    // Does element e of this lane hold an output cell?
    __device__ __forceinline__ bool owns(const TileArgs &A, int e) const
    {
        return lane_out && cx + e < A.C;
    }
};

// Load CPL columns of row rr (already mapped into [0, R)) of one plane.
template <int CPL>
__device__ __forceinline__ void load_row(const float *__restrict__ plane, int rr, int C,
                                         const Tile<CPL> &t, float (&x)[CPL])
{
    const float *row = plane + (size_t)rr * C;
    if (t.fast) {
        const vecf<CPL> v = *reinterpret_cast<const vecf<CPL> *>(row + t.cx);
#pragma unroll
        for (int e = 0; e < CPL; ++e) x[e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < CPL; ++e) x[e] = row[t.mc[e]];
    }
}

// Store this lane's output columns of row m (inside [0, R)) of one plane.
template <int CPL>
__device__ __forceinline__ void store_row(float *__restrict__ plane, int m, int C,
                                          const Tile<CPL> &t, const float (&x)[CPL])
{
    float *row = plane + (size_t)m * C;
    if (t.lane_vec) {
        vecf<CPL> v;
#pragma unroll
        for (int e = 0; e < CPL; ++e) v[e] = x[e];
        *reinterpret_cast<vecf<CPL> *>(row + t.cx) = v;
    } else if (t.lane_out) {
#pragma unroll
        for (int e = 0; e < CPL; ++e)
            if (t.cx + e < C) row[t.cx + e] = x[e];
    }
}

// Slots of the three-row window of time level j while row `it` of level 0 is
// read: row it-j (newest), it-j-1 (centre) and it-j-2 (oldest) of level j sit
// in slots (S-j) mod 3, (S-j-1) mod 3 and (S-j-2) mod 3, S = it mod 3.
struct Slots {
    int ns, cs, ps;
    __device__ __forceinline__ constexpr Slots(int S, int j)
        : ns((S - j % 3 + 3) % 3), cs((S - j % 3 + 5) % 3), ps((S - j % 3 + 4) % 3)
    {
    }
};

}  // namespace rd
