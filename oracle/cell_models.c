/*
 * cell_models.c -- plain CPU oracle for two further two-layer cell models on the
 * same grid and boundary rules as the FitzHugh-Nagumo oracle.  The paper closes
 * (Sec. IV) by noting that its framework extends to any finite-difference
 * time-domain or cellular model; these are the two textbook examples the
 * library builds in next to Eq. (1)-(3).
 *
 * TEST INFRASTRUCTURE ONLY (see rdcnn_oracle.c): shares nothing with the GPU
 * library.
 *
 * Gray-Scott reaction-diffusion (two layers u, v), explicit Euler, Jacobi:
 *   u+ = u + dt * ( Du * Lap(u) - u v^2 + F (1 - u) )
 *   v+ = v + dt * ( Dv * Lap(v) + u v^2 - (F + k) v )
 *   parameters p = [dt, F, k, Du, Dv]; rounding order
 *     sU = (uN + uS) + (uW + uE);  LU = fma(-4, u, sU)      (same for v)
 *     uvv = (u * v) * v;  Fk = F + k
 *     ru = fma(Du, LU, fma(F, 1 - u, -uvv))
 *     rv = fma(Dv, LV, fma(-Fk, v, uvv))
 *     u+ = fma(dt, ru, u);  v+ = fma(dt, rv, v)
 *
 * Chua-Yang cellular neural network (state x, input image g):
 *   dx/dt = -x + (A * y) + (B * g) + z,   y = (|x + 1| - |x - 1|) / 2
 *   with 3x3 templates A, B applied as correlations over the neighbourhood
 *   (index 0..8 = NW, N, NE, W, C, E, SW, S, SE), explicit Euler with step dt.
 *   The input term w = (B * g) + z does not change in time; it is formed once
 *   and carried as the second layer.  Rounding order for a template T over
 *   values q:
 *     corners = (T0 qNW + T2 qNE) + (T6 qSW + T8 qSE)
 *     edges   = (T1 qN  + T7 qS ) + (T3 qW  + T5 qE )
 *     T*q     = (corners + edges) + T4 qC          (products rounded, no fma)
 *     y(x)    = 0.5 * (|x + 1| - |x - 1|)
 *     w       = (B * g) + z
 *     x+      = fma(dt, ((A * y) + w) - x, x)
 *   Parameters p = [dt, A0..A8] for the steps and [B0..B8, z] for the input.
 *
 * Boundary rules as in rdcnn_oracle.c: periodic, or zero-flux (a ghost cell
 * copies the edge cell; diagonal ghosts copy the corner by the same rule on
 * each axis).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CM_BC_PERIODIC 0

static long cm_nbr(long i, int d, long n, int bc)
{
    long j = i + d;
    if (j >= 0 && j < n) return j;
    if (bc == CM_BC_PERIODIC) return (j + n) % n;
    return i;
}

/* ---------------------------------------------------------------- Gray-Scott */

#define GS_STEP(NAME, T, FMA)                                                                   \
    static void NAME(long R, long C, int bc, const T p[5], const T *u, const T *v, T *un,      \
                     T *vn)                                                                     \
    {                                                                                           \
        const T dt = p[0], F = p[1], k = p[2], Du = p[3], Dv = p[4];                            \
        const T Fk = F + k;                                                                     \
        long i;                                                                                 \
        _Pragma("omp parallel for schedule(static)") for (i = 0; i < R; ++i)                    \
        {                                                                                       \
            const long iN = cm_nbr(i, -1, R, bc), iS = cm_nbr(i, +1, R, bc);                    \
            for (long j = 0; j < C; ++j) {                                                      \
                const long jW = cm_nbr(j, -1, C, bc), jE = cm_nbr(j, +1, C, bc);                \
                const T uc = u[i * C + j], vc = v[i * C + j];                                   \
                const T sU = (u[iN * C + j] + u[iS * C + j]) + (u[i * C + jW] + u[i * C + jE]); \
                const T sV = (v[iN * C + j] + v[iS * C + j]) + (v[i * C + jW] + v[i * C + jE]); \
                const T LU = FMA((T)-4, uc, sU);                                                \
                const T LV = FMA((T)-4, vc, sV);                                                \
                const T uvv = (uc * vc) * vc;                                                   \
                const T ru = FMA(Du, LU, FMA(F, (T)1 - uc, -uvv));                              \
                const T rv = FMA(Dv, LV, FMA(-Fk, vc, uvv));                                    \
                un[i * C + j] = FMA(dt, ru, uc);                                                \
                vn[i * C + j] = FMA(dt, rv, vc);                                                \
            }                                                                                   \
        }                                                                                       \
    }

GS_STEP(gs_step_f32, float, fmaf)
GS_STEP(gs_step_f64, double, fma)

/* ---------------------------------------------------------------- Chua-Yang CNN */

/* The 3x3 neighbourhood of (i, j) of field q: q9[0..8] = NW, N, NE, W, C, E, SW, S, SE. */
#define GATHER9(T, q, R, C, bc, i, j, q9)                                     \
    do {                                                                      \
        const long iN_ = cm_nbr(i, -1, R, bc), iS_ = cm_nbr(i, +1, R, bc);    \
        const long jW_ = cm_nbr(j, -1, C, bc), jE_ = cm_nbr(j, +1, C, bc);    \
        const long rr_[3] = {iN_, i, iS_}, cc_[3] = {jW_, j, jE_};            \
        for (int a_ = 0; a_ < 3; ++a_)                                        \
            for (int b_ = 0; b_ < 3; ++b_) q9[3 * a_ + b_] = q[rr_[a_] * C + cc_[b_]]; \
    } while (0)

#define TEMPLATE(T, t, q)                                                        \
    ((((t)[0] * (q)[0] + (t)[2] * (q)[2]) + ((t)[6] * (q)[6] + (t)[8] * (q)[8])) + \
      (((t)[1] * (q)[1] + (t)[7] * (q)[7]) + ((t)[3] * (q)[3] + (t)[5] * (q)[5]))) + \
     (t)[4] * (q)[4]

#define CNN_OUT(T, x) ((T)0.5 * (fabs##T##_((x) + (T)1) - fabs##T##_((x) - (T)1)))
static inline float fabsfloat_(float x) { return fabsf(x); }
static inline double fabsdouble_(double x) { return fabs(x); }

#define CNN_INPUT(NAME, T)                                                              \
    static void NAME(long R, long C, int bc, const T bz[10], const T *g, T *w)         \
    {                                                                                   \
        long i;                                                                         \
        _Pragma("omp parallel for schedule(static)") for (i = 0; i < R; ++i)            \
        {                                                                               \
            for (long j = 0; j < C; ++j) {                                              \
                T q9[9];                                                                \
                GATHER9(T, g, R, C, bc, i, j, q9);                                      \
                w[i * C + j] = (TEMPLATE(T, bz, q9)) + bz[9];                           \
            }                                                                           \
        }                                                                               \
    }

#define CNN_STEP(NAME, T, FMA)                                                          \
    static void NAME(long R, long C, int bc, const T p[10], const T *x, const T *w,    \
                     T *xn)                                                             \
    {                                                                                   \
        const T dt = p[0];                                                              \
        const T *A = p + 1;                                                             \
        long i;                                                                         \
        _Pragma("omp parallel for schedule(static)") for (i = 0; i < R; ++i)            \
        {                                                                               \
            for (long j = 0; j < C; ++j) {                                              \
                T q9[9];                                                                \
                GATHER9(T, x, R, C, bc, i, j, q9);                                      \
                for (int k_ = 0; k_ < 9; ++k_) q9[k_] = CNN_OUT(T, q9[k_]);             \
                const T ay = TEMPLATE(T, A, q9);                                        \
                const T xc = x[i * C + j];                                              \
                xn[i * C + j] = FMA(dt, (ay + w[i * C + j]) - xc, xc);                  \
            }                                                                           \
        }                                                                               \
    }

CNN_INPUT(cnn_input_f32, float)
CNN_INPUT(cnn_input_f64, double)
CNN_STEP(cnn_step_f32, float, fmaf)
CNN_STEP(cnn_step_f64, double, fma)

/* ---------------------------------------------------------------- entry points */

/* T Gray-Scott steps in place on (u, v); precision 32 or 64 (pointers to float
 * or double arrays of R*C, p of 5 values of that type). */
int oracle_gs_run(long R, long C, int bc, int prec, const void *p, long T, void *u, void *v)
{
    const size_t es = prec == 64 ? sizeof(double) : sizeof(float);
    void *un = malloc(es * R * C), *vn = malloc(es * R * C);
    if (!un || !vn) {
        free(un);
        free(vn);
        return -1;
    }
    for (long t = 0; t < T; ++t) {
        if (prec == 64)
            gs_step_f64(R, C, bc, (const double *)p, (const double *)u, (const double *)v,
                        (double *)un, (double *)vn);
        else
            gs_step_f32(R, C, bc, (const float *)p, (const float *)u, (const float *)v,
                        (float *)un, (float *)vn);
        memcpy(u, un, es * R * C);
        memcpy(v, vn, es * R * C);
    }
    free(un);
    free(vn);
    return 0;
}

/* w = (B * g) + z; bz = [B0..B8, z]. */
void oracle_cnn_input(long R, long C, int bc, int prec, const void *bz, const void *g, void *w)
{
    if (prec == 64)
        cnn_input_f64(R, C, bc, (const double *)bz, (const double *)g, (double *)w);
    else
        cnn_input_f32(R, C, bc, (const float *)bz, (const float *)g, (float *)w);
}

/* T Chua-Yang steps in place on x with the fixed input layer w; p = [dt, A0..A8]. */
int oracle_cnn_run(long R, long C, int bc, int prec, const void *p, long T, void *x,
                   const void *w)
{
    const size_t es = prec == 64 ? sizeof(double) : sizeof(float);
    void *xn = malloc(es * R * C);
    if (!xn) return -1;
    for (long t = 0; t < T; ++t) {
        if (prec == 64)
            cnn_step_f64(R, C, bc, (const double *)p, (const double *)x, (const double *)w,
                         (double *)xn);
        else
            cnn_step_f32(R, C, bc, (const float *)p, (const float *)x, (const float *)w,
                         (float *)xn);
        memcpy(x, xn, es * R * C);
    }
    free(xn);
    return 0;
}
