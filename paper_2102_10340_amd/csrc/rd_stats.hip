// rd_stats.hip -- per-instance statistics of a batch for a parameter atlas.
//
// Sec. III.A of arXiv 2102.10340 scans the diffusion coefficients (Du, Dv) and
// sorts the outcomes by eye into slow growth, dynamic patterns and a
// homogeneous steady state (Fig. 9).  These kernels measure, on every instance
// of a batch, what an automated version of that map needs:
//   0 mean_u   1 var_u   2 mean_v   3 var_v
//   4 frac_far    = #{|u - ref| > theta_far} / N
//   5 frac_moving = #{|u - u_prev| > theta_move} / N
//   6 max_change  = max |u - u_prev|
//   7 rms_change  = sqrt(sum (u - u_prev)^2 / N)
// (5-7 NaN without an earlier state).  Threshold tests and differences are
// taken in float32, the precision of the state, so counts are exact; sums are
// accumulated in double.  The variances are accumulated on values shifted by
// the instance's first cell, so a nearly uniform field (the homogeneous case)
// loses no precision to cancellation.
//
// stats_chunk_kernel: one 256-thread workgroup per chunk of at most kStatChunk
// cells of one instance, reducing in a fixed order into per-chunk partials.
// stats_finish_kernel: one thread per instance folds its chunks in order, so
// every result is deterministic.
#include "rd_launch.h"

namespace rd {

enum { P_SU = 0, P_SU2, P_SV, P_SV2, P_FAR, P_MOV, P_MAX, P_SD2, NPART };
static_assert(NPART == kStats, "partial layout");

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ float wave_max(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return x;
}

template <bool PREV>
__global__ __launch_bounds__(kStatThreads) void stats_chunk_kernel(const BatchInst *insts,
                                                                   const StatChunk *chunks,
                                                                   const float *cur,
                                                                   const float *prev,
                                                                   const float *ref, float theta_far,
                                                                   float theta_move,
                                                                   double *partial)
{
    const StatChunk ch = chunks[blockIdx.x];
    const BatchInst I = insts[ch.inst];
    const long long n = (long long)I.R * I.C;
    const float *u = cur + I.off;
    const float *v = u + n;
    const float *pu = PREV ? prev + I.off : nullptr;
    const float r = ref ? ref[ch.inst] : 0.0f;
    const double su0 = u[0], sv0 = v[0];  // shifts for the variance sums
    double su = 0.0, su2 = 0.0, sv = 0.0, sv2 = 0.0, sd2 = 0.0;
    unsigned far = 0, mov = 0;
    float mx = 0.0f;
    auto cell = [&](float x, float y, float p) __attribute__((always_inline)) {
        const double dx = (double)x - su0, dy = (double)y - sv0;
        su += dx;
        su2 = __builtin_fma(dx, dx, su2);
        sv += dy;
        sv2 = __builtin_fma(dy, dy, sv2);
        far += __builtin_fabsf(x - r) > theta_far ? 1u : 0u;
        if (PREV) {
            const float d = x - p;
            const float ad = __builtin_fabsf(d);
            mov += ad > theta_move ? 1u : 0u;
            mx = fmaxf(mx, ad);
            sd2 = __builtin_fma((double)d, (double)d, sd2);
        }
    };
    // Four cells per load where both planes are 16-byte aligned (instance
    // offsets are; the v plane is when N % 4 == 0; chunk starts are multiples
    // of kStatChunk), the rest one by one.
    int k0 = 0;
    if (n % 4 == 0) {
        const int n4 = ch.count / 4;
        const float4 *u4 = reinterpret_cast<const float4 *>(u + ch.start);
        const float4 *v4 = reinterpret_cast<const float4 *>(v + ch.start);
        const float4 *p4 = PREV ? reinterpret_cast<const float4 *>(pu + ch.start) : nullptr;
        for (int k = (int)threadIdx.x; k < n4; k += kStatThreads) {
            const float4 x = u4[k], y = v4[k];
            const float4 p = PREV ? p4[k] : x;
            cell(x.x, y.x, p.x);
            cell(x.y, y.y, p.y);
            cell(x.z, y.z, p.z);
            cell(x.w, y.w, p.w);
        }
        k0 = 4 * n4;
    }
    for (int k = k0 + (int)threadIdx.x; k < ch.count; k += kStatThreads) {
        const long long i = (long long)ch.start + k;
        cell(u[i], v[i], PREV ? pu[i] : 0.0f);
    }
    // fixed-order reduction: butterfly in each wave, then the waves in order
    __shared__ double red[kStatThreads / 64][NPART];
    const int w = (int)threadIdx.x >> 6;
    const double vals[NPART] = {wave_sum(su),  wave_sum(su2), wave_sum(sv),
                                wave_sum(sv2), (double)wave_sum(far), (double)wave_sum(mov),
                                (double)wave_max(mx), wave_sum(sd2)};
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NPART; ++k) red[w][k] = vals[k];
    __syncthreads();
    if (threadIdx.x < NPART) {
        const int k = (int)threadIdx.x;
        double s = red[0][k];
        for (int q = 1; q < kStatThreads / 64; ++q) s = k == P_MAX ? fmax(s, red[q][k]) : s + red[q][k];
        partial[(size_t)blockIdx.x * NPART + k] = s;
    }
}

// One thread per instance: fold the instance's chunks [first[i], first[i+1])
// in order and form the statistics.
__global__ __launch_bounds__(256) void stats_finish_kernel(const BatchInst *insts, const int *first,
                                                           int n_inst, const double *partial,
                                                           const float *cur, int has_prev,
                                                           double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    double s[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) s[k] = 0.0;
    for (int c = first[i]; c < first[i + 1]; ++c)
#pragma unroll
        for (int k = 0; k < NPART; ++k)
            s[k] = k == P_MAX ? fmax(s[k], partial[(size_t)c * NPART + k])
                              : s[k] + partial[(size_t)c * NPART + k];
    const BatchInst I = insts[i];
    const double n = (double)I.R * (double)I.C;
    const double su0 = cur[I.off], sv0 = cur[I.off + (long long)I.R * I.C];
    const double mu = s[P_SU] / n, mv = s[P_SV] / n;  // means of the shifted values
    const double nan = __builtin_nan("");
    double *o = out + (size_t)i * NPART;
    o[0] = su0 + mu;
    o[1] = fmax(s[P_SU2] / n - mu * mu, 0.0);
    o[2] = sv0 + mv;
    o[3] = fmax(s[P_SV2] / n - mv * mv, 0.0);
    o[4] = s[P_FAR] / n;
    o[5] = has_prev ? s[P_MOV] / n : nan;
    o[6] = has_prev ? s[P_MAX] : nan;
    o[7] = has_prev ? sqrt(s[P_SD2] / n) : nan;
}

hipError_t launch_stats(const BatchInst *insts, const StatChunk *chunks, int nchunks,
                        const int *first, int n_inst, const float *cur, const float *prev,
                        const float *ref, float theta_far, float theta_move, double *partial,
                        double *out, hipStream_t s)
{
    if (prev)
        hipLaunchKernelGGL(stats_chunk_kernel<true>, dim3((unsigned)nchunks), dim3(kStatThreads), 0,
                           s, insts, chunks, cur, prev, ref, theta_far, theta_move, partial);
    else
        hipLaunchKernelGGL(stats_chunk_kernel<false>, dim3((unsigned)nchunks), dim3(kStatThreads),
                           0, s, insts, chunks, cur, prev, ref, theta_far, theta_move, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(stats_finish_kernel, dim3((unsigned)((n_inst + 255) / 256)), dim3(256), 0, s,
                       insts, first, n_inst, partial, cur, prev ? 1 : 0, out);
    return hipGetLastError();
}

}  // namespace rd
