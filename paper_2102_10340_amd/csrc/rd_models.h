// rd_models.h -- the cell models the streamed kernels are generic over.
//
// The paper's framework is written for the FitzHugh-Nagumo RD-CNN (Sec. II.A)
// and, by its closing remarks (Sec. IV), extends to any finite-difference
// time-domain or cellular model by swapping the cell update.  Here a model is
// a type with
//   Params                 its parameters (kernel argument, scalar registers)
//   kDiag                  whether the update reads the diagonal neighbours
//   kDerived, derive(u)    whether the update sees the u layer only through a
//                          per-cell function derive(u) (plus the raw centre u):
//                          the body then forms derive once per row and time
//                          level and hands it over in the u neighbour fields
//                          of n, with the centre's in n.y
//   update(p, n, uo, vo)   the new (u, v) of one cell from its neighbourhood n
// and the register-streamed body (rd_fwd_body.h) is instantiated per model.
// Every model fixes its float32 rounding order; the CPU oracle writes the same
// order out, so results are bit-identical.
//
// Temporal blocking at a zero-flux edge runs the update on mirrored ghost
// cells; it reproduces the edge-copy rule exactly only if the update gives
// bit-identical results on mirrored neighbourhoods.  FitzHugh-Nagumo and
// Gray-Scott pair (N, S) and (W, E) symmetrically, so they always do; the CNN
// pairs NW/NE, SW/SE, N/S and W/E, so it does when its A template is mirror
// symmetric (checked on the host, which otherwise runs one step per pass).
#pragma once

#include "rd_common.h"

namespace rd {

// Centre and neighbours of both layers (the diagonals only for kDiag models;
// for kDerived models the u neighbour fields hold derive(u), and y the
// centre's derive(u)).
struct Nbhd {
    float u, v, y;
    float uN, uS, uW, uE, vN, vS, vW, vE;
    float uNW, uNE, uSW, uSE, vNW, vNE, vSW, vSE;
};

// FitzHugh-Nagumo, Eq. (1)-(3): the library's main model.
struct ModelFHN {
    using Params = Gene;
    static constexpr bool kDiag = false;
    static constexpr bool kDerived = false;
    __device__ __forceinline__ static void update(const Gene &g, const Nbhd &n, float &uo, float &vo)
    {
        cell_update(g, n.u, n.v, n.uN, n.uS, n.uW, n.uE, n.vN, n.vS, n.vW, n.vE, uo, vo);
    }
};

// Gray-Scott reaction-diffusion:
//   u+ = u + dt (Du Lap u - u v^2 + F (1 - u)),  v+ = v + dt (Dv Lap v + u v^2 - (F + k) v)
// rounding order: sU = (uN+uS)+(uW+uE), LU = fma(-4,u,sU) (same for v),
// uvv = (u*v)*v, ru = fma(Du, LU, fma(F, 1-u, -uvv)),
// rv = fma(Dv, LV, fma(-(F+k), v, uvv)), u+ = fma(dt, ru, u), v+ = fma(dt, rv, v).
struct GrayScottParams {
    float dt, F, k, Du, Dv;
};
struct ModelGrayScott {
    using Params = GrayScottParams;
    static constexpr bool kDiag = false;
    static constexpr bool kDerived = false;
    static constexpr int kMaxCpl = 4;  // widest strip instantiated (columns per lane)
    __device__ __forceinline__ static void update(const Params &p, const Nbhd &n, float &uo, float &vo)
    {
        const float sU = (n.uN + n.uS) + (n.uW + n.uE);
        const float sV = (n.vN + n.vS) + (n.vW + n.vE);
        const float LU = __builtin_fmaf(-4.0f, n.u, sU);
        const float LV = __builtin_fmaf(-4.0f, n.v, sV);
        const float uvv = (n.u * n.v) * n.v;
        const float Fk = p.F + p.k;
        const float ru = __builtin_fmaf(p.Du, LU, __builtin_fmaf(p.F, 1.0f - n.u, -uvv));
        const float rv = __builtin_fmaf(p.Dv, LV, __builtin_fmaf(-Fk, n.v, uvv));
        uo = __builtin_fmaf(p.dt, ru, n.u);
        vo = __builtin_fmaf(p.dt, rv, n.v);
    }
};

// Chua-Yang cellular neural network: state x in the u layer, the constant input
// term w = (B * image) + z in the v layer (formed once by cnn_input_kernel).
//   x+ = x + dt (-x + (A * y) + w),  y = (|x + 1| - |x - 1|) / 2
// A 3x3 template T over values q (index 0..8 = NW, N, NE, W, C, E, SW, S, SE):
//   T*q = (((T0 qNW + T2 qNE) + (T6 qSW + T8 qSE)) + ((T1 qN + T7 qS) + (T3 qW + T5 qE)))
//         + T4 qC          (each product rounded, no fma)
// and x+ = fma(dt, ((A * y) + w) - x, x); w is carried unchanged.
struct CnnParams {
    float dt;
    float A[9];
};

__device__ __forceinline__ float cnn_out(float x)
{
    return 0.5f * (__builtin_fabsf(x + 1.0f) - __builtin_fabsf(x - 1.0f));
}

__device__ __forceinline__ float template3(const float *T, float nw, float n, float ne, float w,
                                           float c, float e, float sw, float s, float se)
{
    return (((T[0] * nw + T[2] * ne) + (T[6] * sw + T[8] * se)) +
            ((T[1] * n + T[7] * s) + (T[3] * w + T[5] * e))) +
           T[4] * c;
}

// The outputs y are formed once per cell and level (kDerived), not once per
// template tap: the same function of the same value, so the same bits.
struct ModelCnn {
    using Params = CnnParams;
    static constexpr bool kDiag = true;
    static constexpr bool kDerived = true;
    static constexpr int kMaxCpl = 2;  // four columns would not fit the 256 VGPRs
    __device__ __forceinline__ static float derive(float x) { return cnn_out(x); }
    __device__ __forceinline__ static void update(const Params &p, const Nbhd &n, float &uo, float &vo)
    {
        const float ay = template3(p.A, n.uNW, n.uN, n.uNE, n.uW, n.y, n.uE, n.uSW, n.uS, n.uSE);
        uo = __builtin_fmaf(p.dt, (ay + n.v) - n.u, n.u);
        vo = n.v;
    }
};

}  // namespace rd
