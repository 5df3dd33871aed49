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
//
// The kernel templates are in rd_adj_body.h, instantiated in rd_adj_*.hip; this
// file holds the small folding kernels and the launchers.
#include "rd_adj_body.h"

namespace rd {

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

// Shared parameters: dtheta[q] += sum over instances i = 0 .. n-1, in that
// order, of rows[8 i + q] (one thread per parameter).
__global__ __launch_bounds__(64) void grad_row_sum_kernel(const double *rows, int n, double *dtheta)
{
    const int q = threadIdx.x;
    if (q >= 8) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += rows[8 * (size_t)i + q];
    dtheta[q] += s;
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

unsigned grid1(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_adjoint(const AdjPlanes &io, const float *states, int every, long long q_top,
                          int R, int C, int bc, const Gene &g, const StreamGeom &geom,
                          double *partial, bool lam_sums, hipStream_t s)
{
    AdjFn f = adj_fn_plain(lam_sums, geom.cpl, geom.depth);
    if (!f || q_top < geom.depth - 1 || every < 1) return hipErrorInvalidValue;
    AdjArgs a;
    a.t = tile_args(R, C, bc, geom);
    a.in_l = io.in_l;
    a.in_m = io.in_m;
    a.out_l = io.out_l;
    a.out_m = io.out_m;
    a.states = states + (q_top - geom.depth + 1) * every * 2LL * R * C;
    a.state_stride = 8u * (unsigned)every * (unsigned)R * (unsigned)C;
    a.g = g;
    a.partial = partial;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adjoint_pair(const AdjPlanes &io, const float *even_states, int every,
                               long long t_top, int R, int C, int bc, const Gene &g,
                               const StreamGeom &geom, double *partial, bool lam_sums,
                               hipStream_t s)
{
    AdjFn f = adj_fn_pair(lam_sums, geom.cpl, geom.depth);
    if (!f || (t_top & 1) || t_top < geom.depth || every < 1) return hipErrorInvalidValue;
    AdjArgs a;
    a.t = tile_args(R, C, bc, geom);
    a.in_l = io.in_l;
    a.in_m = io.in_m;
    a.out_l = io.out_l;
    a.out_m = io.out_m;
    a.states = even_states + (t_top - geom.depth) / 2 * every * 2LL * R * C;
    a.state_stride = 8u * (unsigned)every * (unsigned)R * (unsigned)C;
    a.g = g;
    a.partial = partial;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_adjoint(const BatchTile *tiles, const BatchInst *insts, int ntiles,
                                const float *in, float *out, const float *states,
                                unsigned state_stride, int bc, int cpl, int depth, int table_depth,
                                double *partial, bool lam_sums, hipStream_t s, bool paired)
{
    BatchAdjFn f = batch_adj_fn(paired, lam_sums, cpl, depth);
    if (!f || ntiles < 1 || depth > table_depth) return hipErrorInvalidValue;
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

hipError_t launch_grad_row_sum(const double *rows, int n, double *dtheta, hipStream_t s)
{
    hipLaunchKernelGGL(grad_row_sum_kernel, dim3(1), dim3(64), 0, s, rows, n, dtheta);
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
