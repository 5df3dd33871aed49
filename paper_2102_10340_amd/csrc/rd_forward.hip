// rd_forward.hip -- forward kernels of the RD-CNN step (arXiv 2102.10340,
// Sec. II.A, Eq. (1)-(3)) for gfx950.
//
//  * init_kernel        Eq. (1) first line, u = v = k_a x.
//  * naive_step_kernel  one thread per cell, one step per launch; neighbours by
//                       the boundary rule, straight from global memory.  It is
//                       the reference the blocked kernel is compared against.
//  * stream_step_kernel K steps per pass over HBM (temporal blocking).  One
//                       wavefront owns a strip of 64*CPL columns (CPL adjacent
//                       columns per lane) and a segment of H output rows; it
//                       walks down the rows once, keeping for each of the K time
//                       levels a two-row window in registers, so row r of level
//                       j+1 is made as soon as row r+1 of level j exists.  East/
//                       west neighbours across lanes come from DPP wave shifts,
//                       north/south ones from the register window; nothing goes
//                       through LDS.  The strip carries K halo columns on each
//                       side and the segment K halo rows above and below (the
//                       valid region shrinks by one cell per level), read from
//                       the boundary-extended grid (map_index), so the boundary
//                       rule costs nothing inside the loop.  Its template
//                       instances are compiled in rd_fwd_r*.hip.
#include "rd_fwd_kernel.h"

namespace rd {

// ---------------------------------------------------------------- init

__global__ __launch_bounds__(256) void init_kernel(const float *__restrict__ x, float ka,
                                                   float *__restrict__ state, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float u = ka * x[i];
        state[i] = u;
        state[n + i] = u;
    }
}

hipError_t launch_init(const float *x, float ka, float *state, long long n, hipStream_t s)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, ka, state, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finite check

__global__ __launch_bounds__(256) void fill_int_kernel(int *p, int v) { p[threadIdx.x] = v; }

// Adds the number of NaN or infinite values among x[0 .. n) to *count.  The
// count is an integer, so the order of the atomic adds does not matter.
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const float *__restrict__ x,
                                                              long long n, int *count)
{
    int bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad += !__builtin_isfinite(x[i]);
    if (bad) atomicAdd(count, bad);
}

hipError_t launch_count_nonfinite(const float *x, long long n, int *count, hipStream_t s)
{
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, count, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    long long blocks = (n + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- naive

__global__ __launch_bounds__(256) void naive_step_kernel(const float *__restrict__ in,
                                                         float *__restrict__ out, int R, int C,
                                                         int bc, Gene g)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= C) return;
    const size_t plane = (size_t)R * C;
    const bool per = bc == BC_PERIODIC;
    const int jW = j > 0 ? j - 1 : (per ? C - 1 : j);
    const int jE = j < C - 1 ? j + 1 : (per ? 0 : j);
    for (int i = blockIdx.y * 4 + threadIdx.y; i < R; i += gridDim.y * 4) {
        const int iN = i > 0 ? i - 1 : (per ? R - 1 : i);
        const int iS = i < R - 1 ? i + 1 : (per ? 0 : i);
        const size_t k = (size_t)i * C + j;
        const float *u = in, *v = in + plane;
        float uo, vo;
        cell_update(g, u[k], v[k], u[(size_t)iN * C + j], u[(size_t)iS * C + j],
                    u[(size_t)i * C + jW], u[(size_t)i * C + jE], v[(size_t)iN * C + j],
                    v[(size_t)iS * C + j], v[(size_t)i * C + jW], v[(size_t)i * C + jE], uo, vo);
        out[k] = uo;
        out[plane + k] = vo;
    }
}

hipError_t launch_naive(const float *in, float *out, int R, int C, int bc, const Gene &g,
                        hipStream_t s)
{
    const unsigned gx = (unsigned)((C + 63) / 64);
    long long gy = ((long long)R + 3) / 4;
    if (gy > 65535) gy = 65535;
    hipLaunchKernelGGL(naive_step_kernel, dim3(gx, (unsigned)gy), dim3(64, 4), 0, s, in, out, R, C,
                       bc, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------- streamed

bool stream_geometry(int R, int C, int cpl, int depth, int seg_rows, StreamGeom *g)
{
    if (cpl != 1 && cpl != 2 && cpl != 4) return false;
    if (depth < 1 || depth > max_depth(cpl)) return false;
    g->cpl = cpl;
    g->depth = depth;
    g->kpad = (depth + cpl - 1) / cpl * cpl;
    g->wout = 64 * cpl - 2 * g->kpad;
    if (g->wout <= 0) return false;
    g->nstrips = (C + g->wout - 1) / g->wout;
    int h = seg_rows;
    if (h <= 0) {
        // Aim at about two resident wavefronts per SIMD (1024 SIMDs).
        long long want = 2048 / g->nstrips;
        if (want < 1) want = 1;
        h = (int)(((long long)R + want - 1) / want);
        if (h < 4) h = 4;
    }
    if (h > R) h = R;
    g->h = h;
    g->nsegs = (R + h - 1) / h;
    const long long nt = (long long)g->nstrips * g->nsegs;
    if (nt > (1LL << 30)) return false;
    g->ntiles = (int)nt;
    g->per_xcd = (g->ntiles + 7) / 8;
    return true;
}

namespace {

// The instance for a pass: recording mode rec (rd_fwd_body.h), cpl columns per
// lane, depth steps; null if there is none.
StreamFn pick_stream(int rec, int cpl, int depth)
{
    if (rec >= 2) {  // even-state recording: one or two columns per lane, depth <= 8
        if (cpl == 1) return rec == 2 ? stream_fn_r2c1(depth) : stream_fn_r3c1(depth);
        if (cpl == 2) return rec == 2 ? stream_fn_r2c2(depth) : stream_fn_r3c2(depth);
        return nullptr;
    }
    if (cpl == 4) return rec ? stream_fn_r1c4(depth) : stream_fn_r0c4(depth);
    if (cpl == 2) return rec ? stream_fn_r1c2(depth) : stream_fn_r0c2(depth);
    if (cpl == 1) return rec ? stream_fn_r1c1(depth) : stream_fn_r0c1(depth);
    return nullptr;
}

}  // namespace

TileArgs tile_args(int R, int C, int bc, const StreamGeom &geom)
{
    TileArgs t;
    t.R = R;
    t.C = C;
    t.bc = bc;
    t.wout = geom.wout;
    t.kpad = geom.kpad;
    t.h = geom.h;
    t.nsegs = geom.nsegs;
    t.ntiles = geom.ntiles;
    t.per_xcd = geom.per_xcd;
    t.vec_ok = (C % geom.cpl) == 0;
    return t;
}

hipError_t launch_stream(const float *in, float *out, int R, int C, int bc, const Gene &g,
                         const StreamGeom &geom, hipStream_t s, float *rec, long long rec_q0,
                         bool rec_even, bool skip_level0, int rec_every)
{
    if (rec_every < 1) return hipErrorInvalidValue;
    StreamFn f = pick_stream(!rec ? 0 : !rec_even ? 1 : skip_level0 ? 3 : 2, geom.cpl, geom.depth);
    if (!f) return hipErrorInvalidValue;
    StreamArgs a;
    a.t = tile_args(R, C, bc, geom);
    a.in = in;
    a.out = out;
    a.g = g;
    a.rec = rec ? rec + rec_q0 * rec_every * 2LL * R * C : nullptr;
    a.rec_stride = 8u * (unsigned)rec_every * (unsigned)R * (unsigned)C;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
