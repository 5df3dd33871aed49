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
//                       rule costs nothing inside the loop.
#include "rd_launch.h"

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

struct StreamArgs {
    const float *in;
    float *out;
    int R, C, bc;
    Gene g;
    int wout, kpad, h, nsegs, ntiles, per_xcd;
    int vec_ok;  // C % CPL == 0: rows of a plane keep CPL-float alignment
};

template <int CPL>
using vecf = float __attribute__((ext_vector_type(CPL)));

// Load CPL columns of one row: one aligned vector load when the whole strip
// lies inside the grid, else per column through the boundary map.
template <int CPL>
__device__ __forceinline__ void load_row(const float *__restrict__ plane, int rr, int C, bool fast,
                                         int cx, const int (&mc)[CPL], float (&x)[CPL])
{
    const float *row = plane + (size_t)rr * C;
    if (fast) {
        const vecf<CPL> t = *reinterpret_cast<const vecf<CPL> *>(row + cx);
#pragma unroll
        for (int e = 0; e < CPL; ++e) x[e] = t[e];
    } else {
#pragma unroll
        for (int e = 0; e < CPL; ++e) x[e] = row[mc[e]];
    }
}

template <int CPL, int K>
__global__ __launch_bounds__(64) void stream_step_kernel(StreamArgs A)
{
    const int tile = xcd_tile(blockIdx.x, A.per_xcd);
    if (tile >= A.ntiles) return;
    const int lane = threadIdx.x;
    const int strip = tile / A.nsegs;
    const int seg = tile - strip * A.nsegs;
    const int x0 = strip * A.wout - A.kpad;  // first (extended) column of the strip
    const int y0 = seg * A.h;                // first output row of the segment
    const int y1 = min(y0 + A.h, A.R);
    const int cx = x0 + CPL * lane;          // first column of this lane
    const int C = A.C, R = A.R, bc = A.bc;
    const bool fast = A.vec_ok && x0 >= 0 && x0 + 64 * CPL <= C;
    int mc[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) mc[e] = map_index(cx + e, C, bc);
    const int oc = cx - x0;
    const bool lane_out = oc >= A.kpad && oc < A.kpad + A.wout && cx < C;
    const bool lane_vec = lane_out && A.vec_ok && cx + CPL <= C;

    const size_t plane = (size_t)R * C;
    const float *__restrict__ iu = A.in;
    const float *__restrict__ iv = A.in + plane;
    float *__restrict__ ou = A.out;
    float *__restrict__ ov = A.out + plane;
    const Gene g = A.g;

    const int rbase = y0 - K;                         // first row read (level 0)
    const int n_iter = (y1 - y0 + 2 * K + 2) / 3 * 3;  // rows walked, padded to 3

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
        const int rr = map_index(rbase, R, bc);
        load_row<CPL>(iu, rr, C, fast, cx, mc, bu[0][0]);
        load_row<CPL>(iv, rr, C, fast, cx, mc, bv[0][0]);
    }

    auto iteration = [&](const int it, const int S) __attribute__((always_inline)) {
        float tu[CPL], tv[CPL];  // row it-K of level K (the pass output)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int ns = (S - j + 3 * K) % 3;  // slot of level-j row it-j
            const int cs = (ns + 2) % 3;        // row it-j-1
            const int ps = (ns + 1) % 3;        // row it-j-2
            float *du = j + 1 < K ? bu[j + 1][cs] : tu;  // level j+1, row it-j-1
            float *dv = j + 1 < K ? bv[j + 1][cs] : tv;
            if (it >= 2 * j + 2) {  // level j+1 has all three input rows from here on
                const float lu = from_left_lane(bu[j][cs][CPL - 1]);
                const float ru = from_right_lane(bu[j][cs][0]);
                const float lv = from_left_lane(bv[j][cs][CPL - 1]);
                const float rv = from_right_lane(bv[j][cs][0]);
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    const float uW = e == 0 ? lu : bu[j][cs][e - 1];
                    const float uE = e == CPL - 1 ? ru : bu[j][cs][e + 1];
                    const float vW = e == 0 ? lv : bv[j][cs][e - 1];
                    const float vE = e == CPL - 1 ? rv : bv[j][cs][e + 1];
                    cell_update(g, bu[j][cs][e], bv[j][cs][e], bu[j][ps][e], bu[j][ns][e], uW, uE,
                                bv[j][ps][e], bv[j][ns][e], vW, vE, du[e], dv[e]);
                }
            }
            if (j == 0) {
                // Level-0 row it-2 is spent: fetch row it+1 into its slot.
                const int rr = map_index(rbase + it + 1, R, bc);
                load_row<CPL>(iu, rr, C, fast, cx, mc, bu[0][ps]);
                load_row<CPL>(iv, rr, C, fast, cx, mc, bv[0][ps]);
            }
        }
        const int m = rbase + it - K;  // row of level K now in (tu, tv)
        if (m >= y0 && m < y1) {
            float *ru_ = ou + (size_t)m * C;
            float *rv_ = ov + (size_t)m * C;
            if (lane_vec) {
                vecf<CPL> a, b;
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    a[e] = tu[e];
                    b[e] = tv[e];
                }
                *reinterpret_cast<vecf<CPL> *>(ru_ + cx) = a;
                *reinterpret_cast<vecf<CPL> *>(rv_ + cx) = b;
            } else if (lane_out) {
#pragma unroll
                for (int e = 0; e < CPL; ++e)
                    if (cx + e < C) {
                        ru_[cx + e] = tu[e];
                        rv_[cx + e] = tv[e];
                    }
            }
        }
    };

    for (int it = 0; it < n_iter; it += 3) {
        iteration(it, 0);
        iteration(it + 1, 1);
        iteration(it + 2, 2);
    }
}

bool stream_geometry(int R, int C, int cpl, int depth, int seg_rows, StreamGeom *g)
{
    if (cpl != 2 && cpl != 4) return false;
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

using StreamFn = void (*)(StreamArgs);

template <int CPL, int... Ks>
constexpr StreamFn pick(int k, std::integer_sequence<int, Ks...>)
{
    StreamFn f = nullptr;
    ((f = (k == Ks + 1) ? &stream_step_kernel<CPL, Ks + 1> : f), ...);
    return f;
}

}  // namespace

hipError_t launch_stream(const float *in, float *out, int R, int C, int bc, const Gene &g,
                         const StreamGeom &geom, hipStream_t s)
{
    StreamFn f = nullptr;
    if (geom.cpl == 4)
        f = pick<4>(geom.depth, std::make_integer_sequence<int, kMaxDepthCpl4>{});
    else if (geom.cpl == 2)
        f = pick<2>(geom.depth, std::make_integer_sequence<int, kMaxDepthCpl2>{});
    if (!f) return hipErrorInvalidValue;
    StreamArgs a;
    a.in = in;
    a.out = out;
    a.R = R;
    a.C = C;
    a.bc = bc;
    a.g = g;
    a.wout = geom.wout;
    a.kpad = geom.kpad;
    a.h = geom.h;
    a.nsegs = geom.nsegs;
    a.ntiles = geom.ntiles;
    a.per_xcd = geom.per_xcd;
    a.vec_ok = (C % geom.cpl) == 0;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd
