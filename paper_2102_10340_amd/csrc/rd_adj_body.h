// rd_adj_body.h -- the reverse-pass kernels of the RD-CNN step (templates),
// shared by the translation units that instantiate them (rd_adj_*.hip).
//
// For a loss J of the final state, with lam' = dJ/du_{t+1} and mu' = dJ/dv_{t+1},
// the transpose of the Jacobian of one step of Eq. (1)-(3) (Sec. II.A) is
//   lam_t = lam' + dt [ (c - 3 k3 u_t^2) lam' + Du Lap(lam') - eps mu' ]
//   mu_t  = mu'  + dt [ -lam' + eps b mu' + Dv Lap(mu') ]
// (Lap is symmetric for both boundary rules), and the parameter gradients are
// inner products over cells and steps:
//   dJ/dDu = dt <Lap lam', u>,  dJ/dDv = dt <Lap mu', v>,  dJ/dc = dt <lam', u>,
//   dJ/dk3 = -dt <lam', u^3>,   dJ/deps = -dt <mu', u - b v + a>,
//   dJ/da = -dt eps <mu', 1>,   dJ/db = dt eps <mu', v>,
//   dJ/ddt = <lam', f1> + <mu', f2> + Du <Lap lam', u> + Dv <Lap mu', v>.
// Using <lam', Lap u> = <Lap lam', u> the step needs the state only at the cell
// itself, never its neighbours.
//
// adjoint_kernel<CPL, KB> runs KB reverse steps per pass with the same strip /
// segment / register-window scheme as the forward kernel: (lam, mu) play the role
// of (u, v), the window of level i holds lam_{t_top-i}, and the state row of
// s_{t_top-i-1} is read for the row each level makes (the pass reads the KB
// states s_{t_top-KB} .. s_{t_top-1} through one buffer resource).  Each lane sums eight
// products over the output cells it makes (float32 within one pass); the wave
// reduces them in double and adds them to its tile's slot of a per-tile partial
// buffer, so every launch and every sum has a fixed order (deterministic).
// adjoint_finish_kernel folds the partials into the eight gradients.
#pragma once

#include <type_traits>
#include <utility>

#include "rd_launch.h"
#include "rd_stream.h"

namespace rd {

// The eight sums, in this order.
enum { S_LLU = 0, S_LMV, S_LU, S_LU3, S_LV, S_MU, S_MV, S_M, NSUM };
static_assert(NSUM == kAdjSums, "partial buffer layout");

struct AdjArgs {
    TileArgs t;
    const float *in_l, *in_m;  // lam, mu of level 0, R x C each
    float *out_l, *out_m;      // lam, mu after KB reverse steps
    const float *states;    // the KB states this pass reads, oldest first
    unsigned state_stride;  // bytes from one state to the next ([KB][2][R][C]: 8*R*C)
    Gene g;
    double *partial;      // [>= ntiles][NSUM], accumulated
};

// One reverse step at one cell.  (l, mu) = (lam', mu') there, (Ll, Lm) their
// Laplacians, (u, v) the state the forward step started from; writes the new
// (lam, mu) and, if count, adds the cell's products to the sums with weight we
// (1 for the tile's output cells, 0 for halo cells; FAST tiles weight a lane's
// sums once at the end instead).  LAMS: also the three lam-weighted products
// only dJ/ddt, dJ/dc and dJ/dk3 need (S_LU, S_LU3, S_LV).
// The dt-scaled constants of the reverse step, formed once per wavefront:
//   lam = lam' + (dt c - 3 dt k3 u^2) lam' + dt Du Lap(lam') - dt eps mu'
//   mu  = mu' + dt Dv Lap(mu') + dt eps b mu' - dt lam'
struct AdjConst {
    float dc, d3k, dDu, deps, dDv, depsb, dt;
    __device__ __forceinline__ explicit AdjConst(const Gene &g)
        : dc(g.dt * g.c), d3k(g.dt * (3.0f * g.k3)), dDu(g.dt * g.Du), deps(g.dt * g.eps),
          dDv(g.dt * g.Dv), depsb(g.dt * (g.eps * g.b)), dt(g.dt)
    {
    }
};

template <bool FAST, bool LAMS>
__device__ __forceinline__ void adj_cell(const AdjConst &k, float l, float mu, float Ll, float Lm,
                                         float u, float v, int count, float we, float &lo,
                                         float &mo, float (&acc)[NSUM])
{
    const float u2 = u * u;
    const float gl = __builtin_fmaf(__builtin_fmaf(-k.d3k, u2, k.dc), l, l);
    lo = __builtin_fmaf(k.dDu, Ll, __builtin_fmaf(-k.deps, mu, gl));
    mo = __builtin_fmaf(k.dDv, Lm, __builtin_fmaf(k.depsb, mu, __builtin_fmaf(-k.dt, l, mu)));
    if (count) {  // halo cells enter with weight 0
        const float uw = FAST ? u : we * u, vw = FAST ? v : we * v;
        acc[S_LLU] = __builtin_fmaf(Ll, uw, acc[S_LLU]);
        acc[S_LMV] = __builtin_fmaf(Lm, vw, acc[S_LMV]);
        if (LAMS) {
            acc[S_LU] = __builtin_fmaf(l, uw, acc[S_LU]);
            acc[S_LU3] = __builtin_fmaf(l * uw, u2, acc[S_LU3]);
            acc[S_LV] = __builtin_fmaf(l, vw, acc[S_LV]);
        }
        acc[S_MU] = __builtin_fmaf(mu, uw, acc[S_MU]);
        acc[S_MV] = __builtin_fmaf(mu, vw, acc[S_MV]);
        if (FAST)
            acc[S_M] += mu;
        else
            acc[S_M] = __builtin_fmaf(we, mu, acc[S_M]);
    }
}

// Wave reduction of the sums in double, fixed butterfly order; lane 0 adds them
// to the tile's slot.
template <int CPL, bool FAST>
__device__ __forceinline__ void add_tile_sums(const AdjArgs &A, const Tile<CPL> &t,
                                              const float (&acc)[NSUM])
{
    const float wl = FAST ? t.owns(A.t, 0) : 1.0f;
#pragma unroll
    for (int k = 0; k < NSUM; ++k) {
        double s = (double)(acc[k] * wl);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) A.partial[(size_t)t.tile * NSUM + k] += s;
    }
}

// ROWS_IN: every row the tile reads, including the kFetchPast rows fetched
// past the end of its walk, lies inside the grid, so row offsets need no
// boundary mapping.
template <int CPL, int KB, bool FAST, bool ROWS_IN, bool LAMS>
__device__ __forceinline__ void adjoint_body(const AdjArgs &A, const Tile<CPL> &t)
{
    const int C = A.t.C, R = A.t.R, bc = A.t.bc;
    const unsigned pbytes = 4u * (unsigned)R * (unsigned)C;
    const unsigned rowb = 4u * (unsigned)C;
    const Buf il(A.in_l, pbytes), im(A.in_m, pbytes);
    const Buf ol(A.out_l, pbytes), om(A.out_m, pbytes);
    const unsigned sstride = A.state_stride;
    const Buf sb(A.states, (unsigned)(KB - 1) * sstride + 2u * pbytes);
    const Gene g = A.g;
    const AdjConst kc(g);
    const int y0 = t.y0, y1 = t.y1;
    const int rbase = y0 - KB;
    const int n_real = y1 - y0 + 2 * KB;
    const int n_iter = (n_real + 2) / 3 * 3;
    // Byte offset of row r (rows outside the grid only occur with ROWS_IN false).
    auto roff = [&](int r) -> unsigned {
        return ROWS_IN ? (unsigned)r * rowb : row_off(r, R, C, bc);
    };

    // 1 for this lane's output cells, 0 for halo cells.  In full-width tiles a
    // lane's columns are all output or all halo, so its sums are weighted once
    // at the end; edge tiles weight each product.
    float w[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) w[e] = FAST ? 1.0f : t.owns(A.t, e);

    float bl[KB][3][CPL], bm[KB][3][CPL];  // lam, mu windows per level
    // State rows per level, in the same modulo-3 slots as the window: the row
    // level i uses at iteration it sits in slot (it-i-1) mod 3 and is fetched
    // two iterations ahead.
    float su[KB][3][CPL], sv[KB][3][CPL];
    float acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0.0f;
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
            bl[j][0][e] = bl[j][1][e] = bl[j][2][e] = 0.0f;
            bm[j][0][e] = bm[j][1][e] = bm[j][2][e] = 0.0f;
            su[j][0][e] = su[j][1][e] = su[j][2][e] = 0.0f;
            sv[j][0][e] = sv[j][1][e] = sv[j][2][e] = 0.0f;
        }
    {
        const unsigned ro = roff(rbase);
        load_row<CPL, FAST>(il, ro, t, bl[0][0]);
        load_row<CPL, FAST>(im, ro, t, bm[0][0]);
    }

    auto iteration = [&](const int it, const int S) __attribute__((always_inline)) {
        float tl[CPL], tm[CPL];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const Slots sl(S, i);
            float *dl = i + 1 < KB ? bl[i + 1][sl.cs] : tl;
            float *dm = i + 1 < KB ? bm[i + 1][sl.cs] : tm;
            const int m = rbase + it - i - 1;  // row made by level i+1
            if (it >= 2 * i + 2 && it < n_real) {
                const float ll = from_left_lane(bl[i][sl.cs][CPL - 1]);
                const float rl = from_right_lane(bl[i][sl.cs][0]);
                const float lm = from_left_lane(bm[i][sl.cs][CPL - 1]);
                const float rm = from_right_lane(bm[i][sl.cs][0]);
                // uniform (m, y0, y1 are scalars): a scalar compare and branch
                const int count = m >= y0 && m < y1;
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    const float l = bl[i][sl.cs][e], mu = bm[i][sl.cs][e];
                    const float lW = e == 0 ? ll : bl[i][sl.cs][e - 1];
                    const float lE = e == CPL - 1 ? rl : bl[i][sl.cs][e + 1];
                    const float mW = e == 0 ? lm : bm[i][sl.cs][e - 1];
                    const float mE = e == CPL - 1 ? rm : bm[i][sl.cs][e + 1];
                    // the lane-shifted neighbour first, so its shift folds into
                    // the add (a + b == b + a exactly)
                    const bool sw = CPL > 1 && e == CPL - 1;
                    const float sl_ = sw ? lE + lW : lW + lE;
                    const float sm_ = sw ? mE + mW : mW + mE;
                    const float Ll = __builtin_fmaf(-4.0f, l, (bl[i][sl.ps][e] + bl[i][sl.ns][e]) + sl_);
                    const float Lm = __builtin_fmaf(-4.0f, mu, (bm[i][sl.ps][e] + bm[i][sl.ns][e]) + sm_);
                    adj_cell<FAST, LAMS>(kc, l, mu, Ll, Lm, su[i][sl.cs][e], sv[i][sl.cs][e],
                                         count, w[e], dl[e], dm[e], acc);
                }
            }
            // Loads in the order they are needed (vmcnt retires in issue
            // order): the level-0 row for the next iteration ...
            if (i == 0) {
                const unsigned ro = roff(rbase + it + 1);
                load_row<CPL, FAST>(il, ro, t, bl[0][sl.ps]);
                load_row<CPL, FAST>(im, ro, t, bm[0][sl.ps]);
            }
            // ... then the state row this level needs two iterations on (level
            // i works from it = 2i+2 to n_real-1 and reads state KB-1-i); its
            // slot held the row used one iteration ago.
            if (it + 2 >= 2 * i + 2 && it + 2 < n_real) {
                const unsigned o = (unsigned)(KB - 1 - i) * sstride + roff(m + 2);
                load_row<CPL, FAST>(sb, o, t, su[i][sl.ps]);
                load_row<CPL, FAST>(sb, o + pbytes, t, sv[i][sl.ps]);
            }
        }
        const int m = rbase + it - KB;
        if (m >= y0 && m < y1) {
            const unsigned o = 4u * (unsigned)m * C;
            store_row<CPL, FAST>(ol, o, C, t, tl);
            store_row<CPL, FAST>(om, o, C, t, tm);
        }
    };

    for (int it = 0; it < n_iter; it += 3) {
        iteration(it, 0);
        iteration(it + 1, 1);
        iteration(it + 2, 2);
    }

    add_tile_sums<CPL, FAST>(A, t, acc);
}

template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs A)
{
    Tile<CPL> t;
    if (!t.init(A.t)) return;
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB + kFetchPast <= A.t.R)
            adjoint_body<CPL, KB, true, true, LAMS>(A, t);
        else
            adjoint_body<CPL, KB, true, false, LAMS>(A, t);
    } else {
        adjoint_body<CPL, KB, false, false, LAMS>(A, t);
    }
}

// ---------------------------------------------------------------- paired passes
//
// The same reverse steps from a trajectory that holds the even-time states
// only (half the writes of full recording, half the memory).  A pass of KB
// (even) reverse steps from an even time t_top works in pairs of levels: pair p
// reads the even state E_p = s_{t_top-2p-2} and rebuilds the odd state
// O_p = s_{t_top-2p-1} = F(E_p) one row at a time with the forward cell update
// (the same float32 operations as the forward kernel, so O_p is bit-identical
// to the state the forward pass made).  Level 2p steps lam_{t_top-2p} back with
// O_p, level 2p+1 steps lam_{t_top-2p-1} back with E_p.
//
// Rows: when level 2p makes row m it needs O_p at row m, hence E_p at rows
// m-1, m, m+1, and level 2p+1 needs E_p at row m-1; E_p is read on rows
// rbase+2p .. rbase+n_real-2p-1.  So each pair keeps a six-slot ring of E_p
// rows (three in use, up to three in flight): the row that is newest in the
// window at iteration it sits in slot it mod 6 and is fetched DE iterations
// earlier.  The level-0 (lam, mu) rows get the same ring with fetch distance
// DL.  The loop is unrolled six times so every slot index is a
// compile-time constant.  The rebuilt O_p needs E_p one column beyond the
// columns level 2p makes, which the strip's halo of KB columns already holds.
// Boundary rows and columns are mapped as in the forward kernel, where the
// mirror rule reproduces the zero-flux edge bit for bit.
template <int CPL, int KB, bool FAST, bool ROWS_IN, bool LAMS, int DL, int DE, int NR>
__device__ __forceinline__ void adjoint_pair_body(const AdjArgs &A, const Tile<CPL> &t)
{
    static_assert(KB % 2 == 0 && NR % 3 == 0 && DL >= 1 && DL <= kFetchPast && DL <= NR - 3 &&
                  DE >= 1 && DE <= NR - 3, "pass shape");
    constexpr int P = KB / 2;
    const int C = A.t.C, R = A.t.R, bc = A.t.bc;
    const unsigned pbytes = 4u * (unsigned)R * (unsigned)C;
    const unsigned rowb = 4u * (unsigned)C;
    const Buf il(A.in_l, pbytes), im(A.in_m, pbytes);
    const Buf ol(A.out_l, pbytes), om(A.out_m, pbytes);
    const unsigned sstride = A.state_stride;  // E_p at (P-1-p) * sstride
    const Buf sb(A.states, (unsigned)(P - 1) * sstride + 2u * pbytes);
    const Gene g = A.g;
    const AdjConst kc(g);
    const int y0 = t.y0, y1 = t.y1;
    const int rbase = y0 - KB;
    const int hrows = y1 - y0;  // output rows
    const int n_real = hrows + 2 * KB;
    auto roff = [&](int r) -> unsigned {
        return ROWS_IN ? (unsigned)r * rowb : row_off(r, R, C, bc);
    };

    float w[CPL];
#pragma unroll
    for (int e = 0; e < CPL; ++e) w[e] = FAST ? 1.0f : t.owns(A.t, e);

    float l0[NR][CPL], m0[NR][CPL];        // level 0 ring
    float bl[KB][3][CPL], bm[KB][3][CPL];  // levels 1 .. KB-1 (index 0 unused)
    float eu[P][NR][CPL], ev[P][NR][CPL];  // E_p rings
    float acc[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0.0f;
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            l0[q][e] = m0[q][e] = 0.0f;
#pragma unroll
            for (int p = 0; p < P; ++p) eu[p][q][e] = ev[p][q][e] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < KB; ++j)
#pragma unroll
            for (int q = 0; q < 3; ++q) bl[j][q][e] = bm[j][q][e] = 0.0f;
    }
    // Rows needed before the loop's own fetches reach them.
#pragma unroll
    for (int q = 0; q < DL; ++q) {
        const unsigned ro = roff(rbase + q);
        load_row<CPL, FAST>(il, ro, t, l0[q]);
        load_row<CPL, FAST>(im, ro, t, m0[q]);
    }
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int q = 0; q < DE; ++q)
            if (4 * p - DE + q < 0) {  // fetch iteration before the loop
                // row rbase+2p+q, whose slot the loop's fetch at iteration
                // 4p-DE+q would have filled: (4p + q) mod NR
                const unsigned o = (unsigned)(P - 1 - p) * sstride + roff(rbase + 2 * p + q);
                load_row<CPL, FAST>(sb, o, t, eu[p][(4 * p + q) % NR]);
                load_row<CPL, FAST>(sb, o + pbytes, t, ev[p][(4 * p + q) % NR]);
            }

    // all: a std::integral_constant<bool, ...>; true in rounds where every
    // level is already active (it >= 2 KB), which then skip that test.
    auto iteration = [&](const int it, const int S6, auto all) __attribute__((always_inline)) {
        const int S = S6 % 3;
        // ring slots of rows newest-2 (north), newest-1 (centre), newest (south)
        const int qN = (S6 + NR - 2) % NR, qC = (S6 + NR - 1) % NR, qS = S6;
        float tl[CPL], tm[CPL];
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            const int p = i / 2;
            const Slots sl(S, i);
            float *dl = i + 1 < KB ? bl[i + 1][sl.cs] : tl;
            float *dm = i + 1 < KB ? bm[i + 1][sl.cs] : tm;
            // level i's window: the ring for level 0, modulo-3 slots above
            const float *lN = i == 0 ? l0[qN] : bl[i][sl.ps];
            const float *lC = i == 0 ? l0[qC] : bl[i][sl.cs];
            const float *lS = i == 0 ? l0[qS] : bl[i][sl.ns];
            const float *mN = i == 0 ? m0[qN] : bm[i][sl.ps];
            const float *mC = i == 0 ? m0[qC] : bm[i][sl.cs];
            const float *mS = i == 0 ? m0[qS] : bm[i][sl.ns];
            const int m = rbase + it - i - 1;  // row made by level i+1
            // (every iteration of the walk has it < n_real; the tests below
            // are single unsigned compares to keep the scalar unit, which
            // serves a compute unit's four SIMDs, out of the way)
            if (decltype(all)::value || it >= 2 * i + 2) {
                float u[CPL], v[CPL];  // the state level i steps back with, row m
                if (i % 2 == 0) {
                    // O_p row m from E_p rows m-1, m, m+1
                    const float lu = from_left_lane(eu[p][qC][CPL - 1]);
                    const float ru = from_right_lane(eu[p][qC][0]);
                    const float lv = from_left_lane(ev[p][qC][CPL - 1]);
                    const float rv = from_right_lane(ev[p][qC][0]);
#pragma unroll
                    for (int e = 0; e < CPL; ++e)
                        cell_update(g, eu[p][qC][e], ev[p][qC][e], eu[p][qN][e], eu[p][qS][e],
                                    e == 0 ? lu : eu[p][qC][e - 1],
                                    e == CPL - 1 ? ru : eu[p][qC][e + 1], ev[p][qN][e],
                                    ev[p][qS][e], e == 0 ? lv : ev[p][qC][e - 1],
                                    e == CPL - 1 ? rv : ev[p][qC][e + 1], u[e], v[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < CPL; ++e) {  // E_p row m
                        u[e] = eu[p][qN][e];
                        v[e] = ev[p][qN][e];
                    }
                }
                const float ll = from_left_lane(lC[CPL - 1]);
                const float rl = from_right_lane(lC[0]);
                const float lm = from_left_lane(mC[CPL - 1]);
                const float rm = from_right_lane(mC[0]);
                const int count = (unsigned)(m - y0) < (unsigned)hrows;
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    const float lW = e == 0 ? ll : lC[e - 1];
                    const float lE = e == CPL - 1 ? rl : lC[e + 1];
                    const float mW = e == 0 ? lm : mC[e - 1];
                    const float mE = e == CPL - 1 ? rm : mC[e + 1];
                    const bool sw = CPL > 1 && e == CPL - 1;
                    const float sl_ = sw ? lE + lW : lW + lE;
                    const float sm_ = sw ? mE + mW : mW + mE;
                    const float Ll = __builtin_fmaf(-4.0f, lC[e], (lN[e] + lS[e]) + sl_);
                    const float Lm = __builtin_fmaf(-4.0f, mC[e], (mN[e] + mS[e]) + sm_);
                    adj_cell<FAST, LAMS>(kc, lC[e], mC[e], Ll, Lm, u[e], v[e], count, w[e],
                                         dl[e], dm[e], acc);
                }
            }
            // Fetches, in the order they are needed: the level-0 row DL
            // iterations on, then (after a pair's second level) E_p's row DE
            // iterations on.  A ring slot being refilled held a row no level
            // reads in this iteration.
            if (i == 0) {
                const unsigned ro = roff(rbase + it + DL);
                load_row<CPL, FAST>(il, ro, t, l0[(S6 + DL) % NR]);
                load_row<CPL, FAST>(im, ro, t, m0[(S6 + DL) % NR]);
            }
            // rows of E_p's range: 4p <= it + DE <= n_real - 1
            if (i % 2 == 1 && (unsigned)(it + DE - 4 * p) <= (unsigned)(n_real - 1 - 4 * p)) {
                const unsigned o =
                    (unsigned)(P - 1 - p) * sstride + roff(rbase + it - 2 * p + DE);
                load_row<CPL, FAST>(sb, o, t, eu[p][(S6 + DE) % NR]);
                load_row<CPL, FAST>(sb, o + pbytes, t, ev[p][(S6 + DE) % NR]);
            }
        }
        const int m = rbase + it - KB;
        if ((unsigned)(m - y0) < (unsigned)hrows) {
            const unsigned o = 4u * (unsigned)m * C;
            store_row<CPL, FAST>(ol, o, C, t, tl);
            store_row<CPL, FAST>(om, o, C, t, tm);
        }
    };

    // Iterations from n_real on would only fetch rows nobody reads: leave
    // the unrolled body as soon as the walk is done (uniform branches).
    // Rounds of NR iterations (fully unrolled: every slot index a constant).
    // From the first round boundary at or after 2 KB on, every level is
    // active: those rounds run a copy of the body without the per-level
    // activity tests (one compare and branch per level and iteration saved on
    // the scalar unit).
    constexpr int kSteady = (2 * KB + NR - 1) / NR * NR;
    int it = 0;
    for (; it < kSteady && it < n_real; it += NR) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (it + q >= n_real) break;
            iteration(it + q, q, std::integral_constant<bool, false>{});
        }
    }
    for (; it < n_real; it += NR) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (it + q >= n_real) break;
            iteration(it + q, q, std::integral_constant<bool, true>{});
        }
    }
    add_tile_sums<CPL, FAST>(A, t, acc);
}

// Fetch distances of the paired passes, in iterations.  Three iterations of
// lead let the compiler's wait counts (which assume conditional fetches were
// skipped) stay clear of the newest fetches; a sweep on 1024^2 put (3, 3)
// ahead of (1, 3), (2, 3), (2, 2) and (3, 2).  Nine-slot rings with six
// iterations of lead for the E_p rows (127 VGPRs, still four waves per SIMD)
// measured the same (8.57 against 8.52 ms for 2000 steps on 1024^2).
constexpr int kPairDL = 3;
constexpr int kPairDE = 3;
constexpr int kPairRing = 6;  // ring slots per row stream (a multiple of 3, >= 3 + fetch distance)

template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void adjoint_pair_kernel(AdjArgs A)
{
    Tile<CPL> t;
    if (!t.init(A.t)) return;
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB + kFetchPast <= A.t.R)
            adjoint_pair_body<CPL, KB, true, true, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
        else
            adjoint_pair_body<CPL, KB, true, false, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
    } else {
        adjoint_pair_body<CPL, KB, false, false, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
    }
}

// ---------------------------------------------------------------- batches
//
// The reverse pass over a batch: the same body over a flat tile list covering
// all instances (each tile reads its instance's offset, size and gene).  The
// trajectory holds whole packed batch states, state_stride bytes apart; each
// tile's sums go to its own slot, and batch_adjoint_finish_kernel folds every
// instance's tiles, in a fixed order, into that instance's gradients.
struct BatchAdjArgs {
    const BatchTile *tiles;
    const BatchInst *insts;
    int ntiles;
    const float *in;        // packed (lam, mu) of level 0
    float *out;             // packed (lam, mu) after KB reverse steps
    const float *states;    // packed state q_top-KB+1 of the trajectory
    unsigned state_stride;  // bytes between packed states
    int bc, wout, kpad;
    double *partial;        // [ntiles][NSUM], accumulated
};

// The single-grid arguments of batch tile `id` (its instance's sub-grid).
template <int CPL>
__device__ __forceinline__ void batch_tile_args(const BatchAdjArgs &B, int id, AdjArgs &A,
                                                Tile<CPL> &t)
{
    const BatchTile bt = B.tiles[id];
    const BatchInst in = B.insts[bt.inst];
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
    A.in_l = B.in + in.off;
    A.in_m = A.in_l + (size_t)in.R * in.C;
    A.out_l = B.out + in.off;
    A.out_m = A.out_l + (size_t)in.R * in.C;
    A.states = B.states + in.off;
    A.state_stride = B.state_stride;
    A.g = in.g;
    A.partial = B.partial;
    t.setup(A.t, id, bt.x0, bt.y0, bt.y1);
}

template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void batch_adjoint_kernel(BatchAdjArgs B)
{
    const int id = blockIdx.x;
    if (id >= B.ntiles) return;
    AdjArgs A;
    Tile<CPL> t;
    batch_tile_args<CPL>(B, id, A, t);
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB + kFetchPast <= A.t.R)
            adjoint_body<CPL, KB, true, true, LAMS>(A, t);
        else
            adjoint_body<CPL, KB, true, false, LAMS>(A, t);
    } else {
        adjoint_body<CPL, KB, false, false, LAMS>(A, t);
    }
}

// Paired passes over a batch (even-time trajectory; states points at the
// packed E state of the oldest pair).
template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void batch_adjoint_pair_kernel(BatchAdjArgs B)
{
    const int id = blockIdx.x;
    if (id >= B.ntiles) return;
    AdjArgs A;
    Tile<CPL> t;
    batch_tile_args<CPL>(B, id, A, t);
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB + kFetchPast <= A.t.R)
            adjoint_pair_body<CPL, KB, true, true, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
        else
            adjoint_pair_body<CPL, KB, true, false, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
    } else {
        adjoint_pair_body<CPL, KB, false, false, LAMS, kPairDL, kPairDE, kPairRing>(A, t);
    }
}

using AdjFn = void (*)(AdjArgs);
using BatchAdjFn = void (*)(BatchAdjArgs);

// Kernel tables, one per translation unit (null: no such instance).
//   adj_fn_plain  adjoint_kernel<cpl, depth, lams> (rd_adj_plain.hip)
//   adj_fn_pair   adjoint_pair_kernel, even depth 2..8, cpl 1 or 2 (rd_adj_pair.hip)
//   batch_adj_fn  batch_adjoint_kernel (depth 1, 2, 4, 8) or
//                 batch_adjoint_pair_kernel (2, 4, 8), cpl 1 or 2 (rd_adj_batch.hip)
AdjFn adj_fn_plain(bool lams, int cpl, int depth);
AdjFn adj_fn_pair(bool lams, int cpl, int depth);
BatchAdjFn batch_adj_fn(bool paired, bool lams, int cpl, int depth);

}  // namespace rd
