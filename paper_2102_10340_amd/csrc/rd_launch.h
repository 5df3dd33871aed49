// rd_launch.h -- internal launchers of the RD-CNN kernels (not part of the ABI).
#pragma once

#include "rd_common.h"

namespace rd {

// Largest number of time steps one register-streamed pass may take, per
// columns-per-lane setting (bounded by the 256 architected VGPRs a wave has).
constexpr int kMaxDepthCpl2 = 16;
constexpr int kMaxDepthCpl4 = 12;

inline int max_depth(int cpl) { return cpl == 4 ? kMaxDepthCpl4 : cpl == 2 ? kMaxDepthCpl2 : 0; }

// Geometry of one register-streamed pass over an R x C grid.
struct StreamGeom {
    int cpl;     // columns held by one lane (2 or 4)
    int depth;   // time steps done in the pass (K)
    int kpad;    // left/right halo columns of a strip (K rounded up to cpl)
    int wout;    // output columns of a strip (64*cpl - 2*kpad)
    int h;       // output rows of a segment
    int nstrips, nsegs, ntiles, per_xcd;
};

// Fill in the strip/segment decomposition; seg_rows <= 0 picks a default.
// Returns false if the shape cannot be tiled with these settings.
bool stream_geometry(int R, int C, int cpl, int depth, int seg_rows, StreamGeom *g);

// u = v = ka * x over n cells (state holds u then v).
hipError_t launch_init(const float *x, float ka, float *state, long long n, hipStream_t s);

// One step, one thread per cell, neighbours read straight from global memory.
hipError_t launch_naive(const float *in, float *out, int R, int C, int bc, const Gene &g,
                        hipStream_t s);

// `geom.depth` steps in one pass of the register-streamed kernel.
hipError_t launch_stream(const float *in, float *out, int R, int C, int bc, const Gene &g,
                         const StreamGeom &geom, hipStream_t s);

}  // namespace rd
