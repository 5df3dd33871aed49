// rd_stream.h -- tile geometry and row I/O shared by the register-streamed
// kernels (forward and adjoint).
//
// A pass over an R x C grid is cut into strips of 64*CPL columns (CPL adjacent
// columns per lane of one 64-lane wavefront) and segments of h output rows.  A
// strip overlaps its neighbours by kpad halo columns on each side and a segment
// reads K halo rows above and below, taken from the boundary-extended grid
// (map_index), so a wavefront can run K time levels on its tile without
// talking to any other wavefront.
//
// All row traffic goes through buffer instructions: a plane (or a run of
// consecutive states) is one buffer resource held in scalar registers, the row
// offset is a scalar byte offset and each lane's column offset a loop-invariant
// vector register, so no per-lane address arithmetic runs inside the loops.
// A buffer resource addresses at most 4 GiB, which bounds a plane to fewer
// than 2^30 cells and a run of recorded states to 4 GiB (checked on the host).
#pragma once

#include "rd_common.h"

namespace rd {

template <int CPL>
using vecf = float __attribute__((ext_vector_type(CPL)));  // CPL = 2 or 4

// Third word of a raw (unswizzled, stride 0) buffer resource on gfx9-family
// GPUs: 32-bit data format, no swizzle.
constexpr int kBufferWord3 = 0x00020000;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ Buf(const void *base, unsigned bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kBufferWord3))
    {
    }
};

template <int CPL>
__device__ __forceinline__ void buf_load(const Buf &b, unsigned voff, unsigned soff, float (&x)[CPL]);

template <>
__device__ __forceinline__ void buf_load<1>(const Buf &b, unsigned voff, unsigned soff, float (&x)[1])
{
    x[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, voff, soff, 0));
}

template <>
__device__ __forceinline__ void buf_load<2>(const Buf &b, unsigned voff, unsigned soff, float (&x)[2])
{
    const vecf<2> v = __builtin_bit_cast(vecf<2>, __builtin_amdgcn_raw_buffer_load_b64(b.r, voff, soff, 0));
    x[0] = v[0];
    x[1] = v[1];
}

template <>
__device__ __forceinline__ void buf_load<4>(const Buf &b, unsigned voff, unsigned soff, float (&x)[4])
{
    const vecf<4> v = __builtin_bit_cast(vecf<4>, __builtin_amdgcn_raw_buffer_load_b128(b.r, voff, soff, 0));
    x[0] = v[0];
    x[1] = v[1];
    x[2] = v[2];
    x[3] = v[3];
}

template <int CPL>
__device__ __forceinline__ void buf_store(const Buf &b, unsigned voff, unsigned soff, const float (&x)[CPL]);

template <>
__device__ __forceinline__ void buf_store<1>(const Buf &b, unsigned voff, unsigned soff, const float (&x)[1])
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x[0]), b.r, voff, soff, 0);
}

template <>
__device__ __forceinline__ void buf_store<2>(const Buf &b, unsigned voff, unsigned soff, const float (&x)[2])
{
    vecf<2> v;
    v[0] = x[0];
    v[1] = x[1];
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(unsigned __attribute__((ext_vector_type(2))), v),
                                          b.r, voff, soff, 0);
}

template <>
__device__ __forceinline__ void buf_store<4>(const Buf &b, unsigned voff, unsigned soff, const float (&x)[4])
{
    vecf<4> v;
    v[0] = x[0];
    v[1] = x[1];
    v[2] = x[2];
    v[3] = x[3];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(unsigned __attribute__((ext_vector_type(4))), v),
                                           b.r, voff, soff, 0);
}

__device__ __forceinline__ float buf_load1(const Buf &b, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, voff, soff, 0));
}

__device__ __forceinline__ void buf_store1(const Buf &b, unsigned voff, unsigned soff, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), b.r, voff, soff, 0);
}

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
    bool fast;           // whole strip inside the grid and C % CPL == 0: vector I/O
    bool lane_out;       // this lane's columns are output columns of the tile
    unsigned vo;         // byte offset of the lane's first column (fast tiles)
    unsigned mo[CPL];    // byte offset of each boundary-mapped column (edge tiles)

    // Single grid: tile from the (XCD-renumbered) workgroup index.
    __device__ __forceinline__ bool init(const TileArgs &A)
    {
        const int tl = xcd_tile(blockIdx.x, A.per_xcd);
        if (tl >= A.ntiles) return false;
        const int strip = tl / A.nsegs;
        const int seg = tl - strip * A.nsegs;
        const int sy0 = seg * A.h;
        setup(A, tl, strip * A.wout - A.kpad, sy0, min(sy0 + A.h, A.R));
        return true;
    }

    // A tile given by its first extended column and output rows [ry0, ry1).
    __device__ __forceinline__ void setup(const TileArgs &A, int tl, int sx0, int ry0, int ry1)
    {
        tile = tl;
        x0 = sx0;
        y0 = ry0;
        y1 = ry1;
        cx = x0 + CPL * (int)threadIdx.x;
        fast = A.vec_ok && x0 >= 0 && x0 + 64 * CPL <= A.C;
        vo = 4u * (unsigned)(cx < 0 ? 0 : cx);
#pragma unroll
        for (int e = 0; e < CPL; ++e) mo[e] = 4u * (unsigned)map_index(cx + e, A.C, A.bc);
        const int oc = cx - x0;
        lane_out = oc >= A.kpad && oc < A.kpad + A.wout && cx < A.C;
    }

    // 1 if element e of this lane holds an output cell of the tile, else 0.
    __device__ __forceinline__ float owns(const TileArgs &A, int e) const
    {
        return (lane_out && cx + e < A.C) ? 1.0f : 0.0f;
    }
};

// Load CPL columns of one row; soff is the row's byte offset in the buffer
// (the row already mapped into [0, R)).
template <int CPL, bool FAST>
__device__ __forceinline__ void load_row(const Buf &b, unsigned soff, const Tile<CPL> &t,
                                         float (&x)[CPL])
{
    if (FAST) {
        buf_load<CPL>(b, t.vo, soff, x);
    } else {
#pragma unroll
        for (int e = 0; e < CPL; ++e) x[e] = buf_load1(b, t.mo[e], soff);
    }
}

// Store this lane's output columns of one row (byte offset soff).
template <int CPL, bool FAST>
__device__ __forceinline__ void store_row(const Buf &b, unsigned soff, int C, const Tile<CPL> &t,
                                          const float (&x)[CPL])
{
    if (FAST) {
        if (t.lane_out) buf_store<CPL>(b, t.vo, soff, x);
    } else if (t.lane_out) {
#pragma unroll
        for (int e = 0; e < CPL; ++e)
            if (t.cx + e < C) buf_store1(b, 4u * (unsigned)(t.cx + e), soff, x[e]);
    }
}

// Byte offset of row r (mapped onto the grid) in a plane of C columns.
__device__ __forceinline__ unsigned row_off(int r, int R, int C, int bc)
{
    return 4u * (unsigned)map_index(r, R, bc) * (unsigned)C;
}

// A walk over rows rbase .. rbase+n_real-1 fetches up to this many rows past
// its last one (row prefetches of the last iterations; nothing uses them).  A
// tile takes the unmapped-row (ROWS_IN) path only if those rows are inside the
// grid too: the row offset travels in a buffer instruction's scalar offset, so
// every row it names must lie inside the plane.
constexpr int kFetchPast = 3;

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
