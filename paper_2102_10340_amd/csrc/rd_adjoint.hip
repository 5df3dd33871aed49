// rd_adjoint.hip -- reverse pass of the RD-CNN step for gfx950.
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
#include "rd_launch.h"
#include "rd_stream.h"

namespace rd {

// The eight sums, in this order.
enum { S_LLU = 0, S_LMV, S_LU, S_LU3, S_LV, S_MU, S_MV, S_M, NSUM };
static_assert(NSUM == kAdjSums, "partial buffer layout");

struct AdjArgs {
    TileArgs t;
    const float *in;      // (lam, mu) of level 0, [2][R][C]
    float *out;           // (lam, mu) after KB reverse steps
    const float *states;    // the KB states this pass reads, oldest first
    unsigned state_stride;  // bytes from one state to the next ([KB][2][R][C]: 8*R*C)
    Gene g;
    double *partial;      // [>= ntiles][NSUM], accumulated
};

// LAMS: also sum the three lam-weighted products only dJ/ddt, dJ/dc and dJ/dk3
// need (S_LU, S_LU3, S_LV).  ROWS_IN: every row the tile reads lies inside the
// grid, so row offsets need no boundary mapping.
template <int CPL, int KB, bool FAST, bool ROWS_IN, bool LAMS>
__device__ __forceinline__ void adjoint_body(const AdjArgs &A, const Tile<CPL> &t)
{
    const int C = A.t.C, R = A.t.R, bc = A.t.bc;
    const unsigned pbytes = 4u * (unsigned)R * (unsigned)C;
    const unsigned rowb = 4u * (unsigned)C;
    const Buf il(A.in, pbytes), im(A.in + (size_t)R * C, pbytes);
    const Buf ol(A.out, pbytes), om(A.out + (size_t)R * C, pbytes);
    const unsigned sstride = A.state_stride;
    const Buf sb(A.states, (unsigned)(KB - 1) * sstride + 2u * pbytes);
    const Gene g = A.g;
    const float c3k = 3.0f * g.k3;
    const float epsb = g.eps * g.b;
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
                // uniform; readfirstlane keeps the branch on the scalar unit
                const int count = __builtin_amdgcn_readfirstlane((int)(m >= y0 && m < y1));
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
                    const float u = su[i][sl.cs][e], v = sv[i][sl.cs][e];
                    const float u2 = u * u;
                    const float gl = __builtin_fmaf(-c3k, u2, g.c) * l;
                    const float rl_ = __builtin_fmaf(-g.eps, mu, __builtin_fmaf(g.Du, Ll, gl));
                    dl[e] = __builtin_fmaf(g.dt, rl_, l);
                    const float rm_ = __builtin_fmaf(g.Dv, Lm, __builtin_fmaf(epsb, mu, -l));
                    dm[e] = __builtin_fmaf(g.dt, rm_, mu);
                    if (count) {  // halo cells enter with weight 0
                        const float uw = FAST ? u : w[e] * u, vw = FAST ? v : w[e] * v;
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
                            acc[S_M] = __builtin_fmaf(w[e], mu, acc[S_M]);
                    }
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

    // Wave reduction in double, fixed butterfly order; lane 0 adds to the tile.
    const float wl = FAST ? t.owns(A.t, 0) : 1.0f;
#pragma unroll
    for (int k = 0; k < NSUM; ++k) {
        double s = (double)(acc[k] * wl);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) A.partial[(size_t)t.tile * NSUM + k] += s;
    }
}

template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs A)
{
    Tile<CPL> t;
    if (!t.init(A.t)) return;
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB <= A.t.R)
            adjoint_body<CPL, KB, true, true, LAMS>(A, t);
        else
            adjoint_body<CPL, KB, true, false, LAMS>(A, t);
    } else {
        adjoint_body<CPL, KB, false, false, LAMS>(A, t);
    }
}

// The eight gradients (order dt, a, b, eps, c, k3, Du, Dv) from the eight
// sums, added to dtheta; gradients outside the mask were not summed and are
// set to NaN.
__device__ void add_grads(const double *S, const Gene &g, unsigned mask, double *dtheta)
{
    const double dt = g.dt, a = g.a, b = g.b, eps = g.eps, c = g.c, k3 = g.k3;
    const double Du = g.Du, Dv = g.Dv;
    const double LLU = S[S_LLU], LMV = S[S_LMV], LU = S[S_LU], LU3 = S[S_LU3], LV = S[S_LV];
    const double MU = S[S_MU], MV = S[S_MV], M = S[S_M];
    const double res = MU - b * MV + a * M;  // <mu', u - b v + a>
    double d[8];
    d[0] = c * LU - k3 * LU3 - LV - eps * res + Du * LLU + Dv * LMV;  // dt
    d[1] = -dt * eps * M;                                             // a
    d[2] = dt * eps * MV;                                             // b
    d[3] = -dt * res;                                                 // eps
    d[4] = dt * LU;                                                   // c
    d[5] = -dt * LU3;                                                 // k3
    d[6] = dt * LLU;                                                  // Du
    d[7] = dt * LMV;                                                  // Dv
    for (int q = 0; q < 8; ++q) dtheta[q] = (mask >> q) & 1u ? dtheta[q] + d[q] : __builtin_nan("");
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

template <int CPL, int KB, bool LAMS>
__global__ __launch_bounds__(64) void batch_adjoint_kernel(BatchAdjArgs B)
{
    const int id = blockIdx.x;
    if (id >= B.ntiles) return;
    const BatchTile bt = B.tiles[id];
    const BatchInst in = B.insts[bt.inst];
    AdjArgs A;
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
    A.in = B.in + in.off;
    A.out = B.out + in.off;
    A.states = B.states + in.off;
    A.state_stride = B.state_stride;
    A.g = in.g;
    A.partial = B.partial;
    Tile<CPL> t;
    t.setup(A.t, id, bt.x0, bt.y0, bt.y1);
    if (t.fast) {
        if (t.y0 >= KB && t.y1 + KB <= in.R)
            adjoint_body<CPL, KB, true, true, LAMS>(A, t);
        else
            adjoint_body<CPL, KB, true, false, LAMS>(A, t);
    } else {
        adjoint_body<CPL, KB, false, false, LAMS>(A, t);
    }
}

// One thread per instance: sum the partials of its tiles (tile ids
// tiles_of[first[i] .. first[i+1]), ascending) and add its gradients to
// dtheta[8 i ..].
__global__ __launch_bounds__(256) void batch_adjoint_finish_kernel(const double *partial,
                                                                   const int *first,
                                                                   const int *tiles_of,
                                                                   const BatchInst *insts, int n,
                                                                   unsigned mask, double *dtheta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double S[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) S[k] = 0.0;
    for (int q = first[i]; q < first[i + 1]; ++q) {
        const double *p = partial + (size_t)tiles_of[q] * NSUM;
#pragma unroll
        for (int k = 0; k < NSUM; ++k) S[k] += p[k];
    }
    add_grads(S, insts[i].g, mask, dtheta + 8 * (size_t)i);
}

__global__ __launch_bounds__(256) void zero_kernel(double *p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// One workgroup: sums the per-tile partials in a fixed order and adds the
// gradients to dtheta.
__global__ __launch_bounds__(256) void adjoint_finish_kernel(const double *partial, int ntiles,
                                                             Gene g, unsigned mask, double *dtheta)
{
    __shared__ double red[NSUM][256];
    double s[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k] = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += 256)
#pragma unroll
        for (int k = 0; k < NSUM; ++k) s[k] += partial[(size_t)i * NSUM + k];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < NSUM; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double S[NSUM];
#pragma unroll
        for (int k = 0; k < NSUM; ++k) S[k] = red[k][0];
        add_grads(S, g, mask, dtheta);
    }
}

// gx = ka (lam + mu): the chain rule through u = v = ka x.
__global__ __launch_bounds__(256) void init_backward_kernel(const float *adj, long long n, float ka,
                                                            float *gx)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        gx[i] = ka * (adj[i] + adj[n + i]);
}

namespace {

using AdjFn = void (*)(AdjArgs);

template <int CPL, bool LAMS, int... Ks>
constexpr AdjFn pick(int k, std::integer_sequence<int, Ks...>)
{
    AdjFn f = nullptr;
    ((f = (k == Ks + 1) ? &adjoint_kernel<CPL, Ks + 1, LAMS> : f), ...);
    return f;
}

template <bool LAMS>
AdjFn pick_adj(int cpl, int depth)
{
    if (cpl == 4) return pick<4, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl4>{});
    if (cpl == 2) return pick<2, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl2>{});
    if (cpl == 1) return pick<1, LAMS>(depth, std::make_integer_sequence<int, kMaxAdjDepthCpl1>{});
    return nullptr;
}

unsigned grid1(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_adjoint(const float *in, float *out, const float *states, long long q_top,
                          int R, int C, int bc, const Gene &g, const StreamGeom &geom,
                          double *partial, bool lam_sums, hipStream_t s)
{
    AdjFn f = lam_sums ? pick_adj<true>(geom.cpl, geom.depth) : pick_adj<false>(geom.cpl, geom.depth);
    if (!f || q_top < geom.depth - 1) return hipErrorInvalidValue;
    AdjArgs a;
    a.t = tile_args(R, C, bc, geom);
    a.in = in;
    a.out = out;
    a.states = states + (q_top - geom.depth + 1) * 2LL * R * C;
    a.state_stride = 8u * (unsigned)R * (unsigned)C;
    a.g = g;
    a.partial = partial;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

namespace {

using BatchAdjFn = void (*)(BatchAdjArgs);

template <bool LAMS>
BatchAdjFn pick_batch_adj(int cpl, int depth)
{
    if (cpl == 1) {
        if (depth == 2) return &batch_adjoint_kernel<1, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_kernel<1, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_kernel<1, 8, LAMS>;
        if (depth == 1) return &batch_adjoint_kernel<1, 1, LAMS>;
    } else if (cpl == 2) {
        if (depth == 2) return &batch_adjoint_kernel<2, 2, LAMS>;
        if (depth == 4) return &batch_adjoint_kernel<2, 4, LAMS>;
        if (depth == 8) return &batch_adjoint_kernel<2, 8, LAMS>;
        if (depth == 1) return &batch_adjoint_kernel<2, 1, LAMS>;
    }
    return nullptr;
}

}  // namespace

hipError_t launch_batch_adjoint(const BatchTile *tiles, const BatchInst *insts, int ntiles,
                                const float *in, float *out, const float *states,
                                unsigned state_stride, int bc, int cpl, int depth, int table_depth,
                                double *partial, bool lam_sums, hipStream_t s)
{
    BatchAdjFn f = lam_sums ? pick_batch_adj<true>(cpl, depth) : pick_batch_adj<false>(cpl, depth);
    if (!f || ntiles < 1) return hipErrorInvalidValue;
    BatchAdjArgs a;
    a.tiles = tiles;
    a.insts = insts;
    a.ntiles = ntiles;
    a.in = in;
    a.out = out;
    a.states = states;
    a.state_stride = state_stride;
    a.bc = bc;
    a.kpad = (table_depth + cpl - 1) / cpl * cpl;  // the tile list's halo (>= depth)
    a.wout = 64 * cpl - 2 * a.kpad;
    a.partial = partial;
    hipLaunchKernelGGL(f, dim3((unsigned)ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_adjoint_finish(const double *partial, const int *first, const int *tiles_of,
                                       const BatchInst *insts, int n, unsigned mask,
                                       double *dtheta, hipStream_t s)
{
    hipLaunchKernelGGL(batch_adjoint_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, partial, first, tiles_of, insts, n, mask, dtheta);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3(grid1(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish(const double *partial, int ntiles, const Gene &g, unsigned mask,
                                 double *dtheta, hipStream_t s)
{
    hipLaunchKernelGGL(adjoint_finish_kernel, dim3(1), dim3(256), 0, s, partial, ntiles, g, mask,
                       dtheta);
    return hipGetLastError();
}

hipError_t launch_init_backward(const float *adj, long long n, float ka, float *gx, hipStream_t s)
{
    hipLaunchKernelGGL(init_backward_kernel, dim3(grid1(n)), dim3(256), 0, s, adj, n, ka, gx);
    return hipGetLastError();
}

}  // namespace rd
