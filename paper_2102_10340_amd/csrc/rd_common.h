// rd_common.h -- device-side building blocks shared by the RD-CNN kernels.
//
// The cell update is Eq. (1)-(3) of arXiv 2102.10340 (Sec. II.A).  Its float32
// rounding order is fixed so that every kernel of this library gives the same
// bits for the same state, whatever its tiling or time blocking:
//   sU = (uN + uS) + (uW + uE);   LU = fma(-4, u, sU)      (same for v)
//   f1 = fma(u, fma(-k3, u*u, c), -v)                       Eq. (2): c u - k3 u^3 - v
//   f2 = fma(eps*b, v, fma(-eps, u, -(eps*a)))              Eq. (3): -eps (u - b v + a)
//   u+ = fma(dt, fma(Du, LU, f1), u);  v+ = fma(dt, fma(Dv, LV, f2), v)
// The sources are built with -ffp-contract=off (no other fusion) and without
// denormal flushing, so v_fma_f32 / v_mul_f32 / v_add_f32 round exactly as
// written.  The (N+S)+(W+E) pairing makes the result invariant under the
// grid's rotations and reflections, which the boundary handling below relies on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

enum { BC_PERIODIC = 0, BC_ZEROFLUX = 1 };

struct Gene {
    float dt, a, b, eps, c, k3, Du, Dv;
};

// One cell of Eq. (1)-(3) in the fixed rounding order above.
__device__ __forceinline__ void cell_update(const Gene &g, float uc, float vc, float uN, float uS,
                                            float uW, float uE, float vN, float vS, float vW,
                                            float vE, float &uo, float &vo)
{
    const float sU = (uN + uS) + (uW + uE);
    const float sV = (vN + vS) + (vW + vE);
    const float LU = __builtin_fmaf(-4.0f, uc, sU);
    const float LV = __builtin_fmaf(-4.0f, vc, sV);
    const float f1 = __builtin_fmaf(uc, __builtin_fmaf(-g.k3, uc * uc, g.c), -vc);
    const float f2 = __builtin_fmaf(g.eps * g.b, vc, __builtin_fmaf(-g.eps, uc, -(g.eps * g.a)));
    uo = __builtin_fmaf(g.dt, __builtin_fmaf(g.Du, LU, f1), uc);
    vo = __builtin_fmaf(g.dt, __builtin_fmaf(g.Dv, LV, f2), vc);
}

// Map an index of the boundary-extended line onto [0, n).
//  periodic : wrap, i mod n.
//  zero-flux: mirror about the half-cell outside each edge (-1 -> 0, n -> n-1,
//             -2 -> 1, ...; period 2n).  One Jacobi step on the extended line
//             keeps this mirror symmetry bit for bit (the pairing above is
//             symmetric), so the ghost value next to an edge cell always equals
//             the edge cell, which is the zero-flux rule, at every depth of a
//             temporally blocked pass.
// Written as fold loops rather than a modulo: an index inside the line costs
// one compare, one within a halo of the edge one fold, and only lines shorter
// than the halo fold more than once (a modulo would be if-converted into an
// always-executed division on the scalar unit).
__device__ __forceinline__ int map_index(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        while (i < 0) i += n;
        while (i >= n) i -= n;
    } else {
        while ((unsigned)i >= (unsigned)n) i = i < 0 ? -1 - i : 2 * n - 1 - i;
    }
    return i;
}

// Lane i receives lane i-1's value (lane 0 receives 0): DPP wave_shr:1.  With
// bound_ctrl set, a lane with no source lane reads 0 directly, so the compiler
// needs no zeroed destination register first and can fold the shift into the
// add that consumes it.
__device__ __forceinline__ float from_left_lane(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                 0x138, 0xF, 0xF, true));
}

// Lane i receives lane i+1's value (lane 63 receives 0): DPP wave_shl:1.
__device__ __forceinline__ float from_right_lane(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                 0x130, 0xF, 0xF, true));
}

// Workgroups are handed to the 8 XCDs round-robin; renumber them so that each
// XCD gets a contiguous run of tiles (neighbouring tiles share halo lines in
// that XCD's L2).
__device__ __forceinline__ int xcd_tile(int block, int per_xcd)
{
    return (block & 7) * per_xcd + (block >> 3);
}

}  // namespace rd
