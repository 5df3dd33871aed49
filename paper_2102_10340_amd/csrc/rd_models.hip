// rd_models.hip -- the register-streamed kernel instantiated for the cell
// models beyond FitzHugh-Nagumo (rd_models.h): Gray-Scott reaction-diffusion
// and a Chua-Yang cellular neural network.  Same tiling, boundary handling and
// temporal blocking as the main kernel; only the cell update differs.
#include <string.h>

#include "rd_fwd_body.h"
#include "rd_launch.h"

namespace rd {

template <class M, int CPL, int K>
__global__ __launch_bounds__(64) void model_step_kernel(StreamArgsT<M> A)
{
    Tile<CPL> t;
    if (!t.init(A.t)) return;
    if (t.fast) {
        if (t.y0 >= K && t.y1 + K + kFetchPast <= A.t.R)
            stream_body<M, CPL, K, 0, true, true>(A, t);
        else
            stream_body<M, CPL, K, 0, true, false>(A, t);
    } else {
        stream_body<M, CPL, K, 0, false, false>(A, t);
    }
}

// One thread per cell: w = (B * img) + z with the template sum of rd_models.h.
__global__ __launch_bounds__(256) void cnn_input_kernel(const float *__restrict__ img,
                                                        CnnParams bz, float z, int R, int C,
                                                        int bc, float *__restrict__ w)
{
    const long long n = (long long)R * C;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int i = (int)(k / C), j = (int)(k % C);
        const int iN = map_index(i - 1, R, bc), iS = map_index(i + 1, R, bc);
        const int jW = map_index(j - 1, C, bc), jE = map_index(j + 1, C, bc);
        auto g = [&](int r, int c) { return img[(long long)r * C + c]; };
        w[k] = template3(bz.A, g(iN, jW), g(iN, j), g(iN, jE), g(i, jW), g(i, j), g(i, jE),
                         g(iS, jW), g(iS, j), g(iS, jE)) +
               z;
    }
}

namespace {

template <class M>
using ModelFn = void (*)(StreamArgsT<M>);

template <class M>
ModelFn<M> pick_model(int cpl, int depth)
{
    if (cpl == 1) {
        if (depth == 1) return &model_step_kernel<M, 1, 1>;
        if (depth == 2) return &model_step_kernel<M, 1, 2>;
        if (depth == 4) return &model_step_kernel<M, 1, 4>;
        if (depth == 8) return &model_step_kernel<M, 1, 8>;
    } else if (cpl == 2) {
        if (depth == 1) return &model_step_kernel<M, 2, 1>;
        if (depth == 2) return &model_step_kernel<M, 2, 2>;
        if (depth == 4) return &model_step_kernel<M, 2, 4>;
        if (depth == 8) return &model_step_kernel<M, 2, 8>;
    } else if (cpl == 4) {
        if constexpr (M::kMaxCpl >= 4) {
            if (depth == 1) return &model_step_kernel<M, 4, 1>;
            if (depth == 2) return &model_step_kernel<M, 4, 2>;
            if (depth == 4) return &model_step_kernel<M, 4, 4>;
            if (depth == 8) return &model_step_kernel<M, 4, 8>;
        }
    }
    return nullptr;
}

template <class M>
hipError_t launch_as(const float *in, float *out, int R, int C, int bc,
                     const typename M::Params &p, const StreamGeom &geom, hipStream_t s)
{
    ModelFn<M> f = pick_model<M>(geom.cpl, geom.depth);
    if (!f) return hipErrorInvalidValue;
    StreamArgsT<M> a;
    a.t = tile_args(R, C, bc, geom);
    a.in = in;
    a.out = out;
    a.g = p;
    a.rec = nullptr;
    a.rec_stride = 0;
    hipLaunchKernelGGL(f, dim3((unsigned)(8 * geom.per_xcd)), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int model_max_cpl(int model)
{
    return model == MODEL_GRAY_SCOTT ? ModelGrayScott::kMaxCpl
           : model == MODEL_CNN      ? ModelCnn::kMaxCpl
                                     : 0;
}

bool model_mirror_exact(int model, const float *p)
{
    if (model != MODEL_CNN) return true;
    const float *A = p + 1;  // NW N NE / W C E / SW S SE
    return A[0] == A[2] && A[6] == A[8] && A[0] == A[6] && A[1] == A[7] && A[3] == A[5];
}

hipError_t launch_model(int model, const float *in, float *out, int R, int C, int bc,
                        const float *params, const StreamGeom &geom, hipStream_t s)
{
    if (model == MODEL_GRAY_SCOTT) {
        GrayScottParams p;
        p.dt = params[0];
        p.F = params[1];
        p.k = params[2];
        p.Du = params[3];
        p.Dv = params[4];
        return launch_as<ModelGrayScott>(in, out, R, C, bc, p, geom, s);
    }
    if (model == MODEL_CNN) {
        CnnParams p;
        p.dt = params[0];
        memcpy(p.A, params + 1, sizeof p.A);
        return launch_as<ModelCnn>(in, out, R, C, bc, p, geom, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_cnn_input(const float *img, const float *bz, int R, int C, int bc, float *w,
                            hipStream_t s)
{
    CnnParams b;
    b.dt = 0.0f;
    memcpy(b.A, bz, sizeof b.A);
    long long blocks = ((long long)R * C + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(cnn_input_kernel, dim3((unsigned)blocks), dim3(256), 0, s, img, b, bz[9], R,
                       C, bc, w);
    return hipGetLastError();
}

}  // namespace rd
