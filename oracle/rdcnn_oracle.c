/*
 * rdcnn_oracle.c -- plain CPU oracle for the FitzHugh-Nagumo reaction-diffusion
 * cellular nonlinear network (RD-CNN) of Dogaru & Dogaru, arXiv 2102.10340.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the GPU library, and it includes nothing from it.
 *
 * What it computes (Sec. II.A):
 *   Eq. (1): u = v = k_a * x; then for t = 1..T, for every cell (i,j), a Jacobi
 *            (all cells from the old state) explicit-Euler update
 *              u+ = u + dt * [ f1(u,v) + Du * Lap(u) ]
 *              v+ = v + dt * [ f2(u,v) + Dv * Lap(v) ]
 *            with the unscaled 5-point Laplacian
 *              Lap(u)_ij = u_{i+1,j} + u_{i-1,j} + u_{i,j-1} + u_{i,j+1} - 4 u_ij.
 *   Eq. (2): f1(u,v) = c*u - k3*u^3 - v     (the paper fixes k3 = 1/3; the cubic
 *            coefficient is kept as a parameter because the synthetic workloads
 *            use f1 = u - u^3 - v).
 *   Eq. (3): f2(u,v) = -eps * (u - b*v + a).
 *
 * Parameter vector ("gene", Sec. II.A, in the order of the paper's Pars array
 * plus the cubic coefficient):  p = [dt, a, b, eps, c, k3, Du, Dv].
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *   - Grid layout: 0-based row-major, i = row in [0,R), j = column in [0,C),
 *     flat index i*C + j.  N/S neighbours are rows i-1/i+1, W/E are columns j-1/j+1.
 *   - Boundary: periodic (toroidal, as in all of the paper's kernels) or
 *     zero-flux, read as a ghost cell that copies the edge cell
 *     (u_{-1,j} = u_{0,j}, u_{R,j} = u_{R-1,j}, same for columns).
 *   - Rounding order (the paper does not state one).  In float every cell is
 *     evaluated as
 *       sU  = (uN + uS) + (uW + uE);      LU = fma(-4, u, sU)
 *       sV  = (vN + vS) + (vW + vE);      LV = fma(-4, v, sV)
 *       f1  = fma(u, fma(-k3, u*u, c), -v)             = c u - k3 u^3 - v
 *       f2  = fma(eps*b, v, fma(-eps, u, -(eps*a)))    = -eps (u - b v + a)
 *       u+  = fma(dt, fma(Du, LU, f1), u)
 *       v+  = fma(dt, fma(Dv, LV, f2), v)
 *     (eps*b and eps*a rounded to float once), and in double with the
 *     textbook grouping f1 = fma(-k3, (u*u)*u, fma(c, u, -v)),
 *     f2 = (-eps) * (fma(-b, v, u) + a); fma is the correctly rounded fused
 *     multiply-add of C99.  The build uses -ffp-contract=off so that no other
 *     contraction happens, and no flush-to-zero.
 *
 * Reverse pass (gradient of a loss J(s_T) through the T steps), written from the
 * transpose of the Jacobian of the step above.  With lam' = dJ/du_{t+1},
 * mu' = dJ/dv_{t+1} and Lap symmetric for both boundary rules:
 *   lam_t = lam' + dt * [ (c - 3 k3 u_t^2) lam' + Du Lap(lam') - eps mu' ]
 *   mu_t  = mu'  + dt * [ -lam' + eps b mu' + Dv Lap(mu') ]
 * and, summed over t and cells,
 *   dJ/ddt  += <lam', f1 + Du Lap u_t> + <mu', f2 + Dv Lap v_t>
 *   dJ/da   += -dt eps <mu', 1>          dJ/db  += dt eps <mu', v_t>
 *   dJ/deps += -dt <mu', u_t - b v_t + a>
 *   dJ/dc   += dt <lam', u_t>            dJ/dk3 += -dt <lam', u_t^3>
 *   dJ/dDu  += dt <lam', Lap u_t>        dJ/dDv += dt <mu', Lap v_t>
 * The reverse pass is always evaluated in double precision.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_BC_PERIODIC 0
#define ORACLE_BC_ZEROFLUX 1

/* Neighbour of line index i in direction d (+1 or -1) on a line of n cells. */
static long nbr(long i, int d, long n, int bc)
{
    long j = i + d;
    if (j >= 0 && j < n) return j;
    if (bc == ORACLE_BC_PERIODIC) return (j + n) % n; /* j is -1 or n: wrap */
    return i;                                          /* zero-flux: copy the edge cell */
}

/* ---------------------------------------------------------------- forward */

/* One Jacobi step in float; reads (u,v), writes (un,vn).  The target_clones
 * attribute only lets gcc emit the hardware FMA instruction where the host has
 * one; fmaf is correctly rounded on both paths, so the results are identical. */
__attribute__((target_clones("fma", "default")))
static void step_f32(long R, long C, int bc, const float p[8],
                     const float *u, const float *v, float *un, float *vn)
{
    const float dt = p[0], a = p[1], b = p[2], eps = p[3];
    const float c = p[4], k3 = p[5], Du = p[6], Dv = p[7];
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < R; ++i) {
        const long iN = nbr(i, -1, R, bc), iS = nbr(i, +1, R, bc);
        for (long j = 0; j < C; ++j) {
            const long jW = nbr(j, -1, C, bc), jE = nbr(j, +1, C, bc);
            const float uc = u[i * C + j], vc = v[i * C + j];
            const float sU = (u[iN * C + j] + u[iS * C + j]) + (u[i * C + jW] + u[i * C + jE]);
            const float sV = (v[iN * C + j] + v[iS * C + j]) + (v[i * C + jW] + v[i * C + jE]);
            const float LU = fmaf(-4.0f, uc, sU);
            const float LV = fmaf(-4.0f, vc, sV);
            const float f1 = fmaf(uc, fmaf(-k3, uc * uc, c), -vc);
            const float f2 = fmaf(eps * b, vc, fmaf(-eps, uc, -(eps * a)));
            un[i * C + j] = fmaf(dt, fmaf(Du, LU, f1), uc);
            vn[i * C + j] = fmaf(dt, fmaf(Dv, LV, f2), vc);
        }
    }
}

/* The same step in double. */
__attribute__((target_clones("fma", "default")))
static void step_f64(long R, long C, int bc, const double p[8],
                     const double *u, const double *v, double *un, double *vn)
{
    const double dt = p[0], a = p[1], b = p[2], eps = p[3];
    const double c = p[4], k3 = p[5], Du = p[6], Dv = p[7];
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < R; ++i) {
        const long iN = nbr(i, -1, R, bc), iS = nbr(i, +1, R, bc);
        for (long j = 0; j < C; ++j) {
            const long jW = nbr(j, -1, C, bc), jE = nbr(j, +1, C, bc);
            const double uc = u[i * C + j], vc = v[i * C + j];
            const double sU = (u[iN * C + j] + u[iS * C + j]) + (u[i * C + jW] + u[i * C + jE]);
            const double sV = (v[iN * C + j] + v[iS * C + j]) + (v[i * C + jW] + v[i * C + jE]);
            const double LU = fma(-4.0, uc, sU);
            const double LV = fma(-4.0, vc, sV);
            const double f1 = fma(-k3, (uc * uc) * uc, fma(c, uc, -vc));
            const double f2 = (-eps) * (fma(-b, vc, uc) + a);
            un[i * C + j] = fma(dt, fma(Du, LU, f1), uc);
            vn[i * C + j] = fma(dt, fma(Dv, LV, f2), vc);
        }
    }
}

/*
 * Run T steps in float from (u,v) in place.  p holds float parameters.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_run_f32(long R, long C, int bc, const float *p, long T, float *u, float *v)
{
    if (R < 1 || C < 1 || T < 0 || (bc != 0 && bc != 1) || !p || !u || !v) return -1;
    const long n = R * C;
    float *un = (float *)malloc(sizeof(float) * n), *vn = (float *)malloc(sizeof(float) * n);
    if (!un || !vn) { free(un); free(vn); return -1; }
    for (long t = 0; t < T; ++t) {
        step_f32(R, C, bc, p, u, v, un, vn);
        memcpy(u, un, sizeof(float) * n);
        memcpy(v, vn, sizeof(float) * n);
    }
    free(un); free(vn);
    return 0;
}

/* Run T steps in double from (u,v) in place. */
int oracle_run_f64(long R, long C, int bc, const double *p, long T, double *u, double *v)
{
    if (R < 1 || C < 1 || T < 0 || (bc != 0 && bc != 1) || !p || !u || !v) return -1;
    const long n = R * C;
    double *un = (double *)malloc(sizeof(double) * n), *vn = (double *)malloc(sizeof(double) * n);
    if (!un || !vn) { free(un); free(vn); return -1; }
    for (long t = 0; t < T; ++t) {
        step_f64(R, C, bc, p, u, v, un, vn);
        memcpy(u, un, sizeof(double) * n);
        memcpy(v, vn, sizeof(double) * n);
    }
    free(un); free(vn);
    return 0;
}

/* Apply the 5-point Laplacian of Eq. (1) to one plane (double). */
int oracle_laplacian_f64(long R, long C, int bc, const double *x, double *out)
{
    if (R < 1 || C < 1 || (bc != 0 && bc != 1) || !x || !out) return -1;
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < R; ++i) {
        const long iN = nbr(i, -1, R, bc), iS = nbr(i, +1, R, bc);
        for (long j = 0; j < C; ++j) {
            const long jW = nbr(j, -1, C, bc), jE = nbr(j, +1, C, bc);
            out[i * C + j] = fma(-4.0, x[i * C + j],
                                 (x[iN * C + j] + x[iS * C + j]) + (x[i * C + jW] + x[i * C + jE]));
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- reverse */

/*
 * One reverse step at time t: (lam, mu) holds the adjoint at t+1 on entry and at
 * t on exit; (u, v) is the state s_t the forward step was applied to.  The eight
 * parameter-gradient terms of this step are added to g[] in the order of p.
 * Row partial sums are added up in row order, so the result does not depend on
 * the number of threads.
 */
static int reverse_step(long R, long C, int bc, const double p[8],
                        const double *u, const double *v, double *lam, double *mu,
                        double *Llam, double *Lmu, double *Lu, double *Lv,
                        double *rowsum /* [R][8] */, double g[8])
{
    const double dt = p[0], a = p[1], b = p[2], eps = p[3];
    const double c = p[4], k3 = p[5], Du = p[6], Dv = p[7];
    const long n = R * C;
    oracle_laplacian_f64(R, C, bc, lam, Llam);
    oracle_laplacian_f64(R, C, bc, mu, Lmu);
    oracle_laplacian_f64(R, C, bc, u, Lu);
    oracle_laplacian_f64(R, C, bc, v, Lv);
    long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < R; ++i) {
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (long j = 0; j < C; ++j) {
            const long k = i * C + j;
            const double uc = u[k], vc = v[k], l = lam[k], m = mu[k];
            const double f1 = c * uc - k3 * uc * uc * uc - vc;
            const double f2 = -eps * (uc - b * vc + a);
            s[0] += l * (f1 + Du * Lu[k]) + m * (f2 + Dv * Lv[k]); /* dt  */
            s[1] += -dt * eps * m;                                 /* a   */
            s[2] += dt * eps * m * vc;                             /* b   */
            s[3] += -dt * m * (uc - b * vc + a);                   /* eps */
            s[4] += dt * l * uc;                                   /* c   */
            s[5] += -dt * l * uc * uc * uc;                        /* k3  */
            s[6] += dt * l * Lu[k];                                /* Du  */
            s[7] += dt * m * Lv[k];                                /* Dv  */
        }
        for (int q = 0; q < 8; ++q) rowsum[i * 8 + q] = s[q];
    }
    for (long r = 0; r < R; ++r)
        for (int q = 0; q < 8; ++q) g[q] += rowsum[r * 8 + q];
    /* Adjoint update: both new values from the old (lam', mu'). */
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        const double uc = u[i], l = lam[i], m = mu[i];
        const double nl = l + dt * ((c - 3.0 * k3 * uc * uc) * l + Du * Llam[i] - eps * m);
        const double nm = m + dt * (-l + eps * b * m + Dv * Lmu[i]);
        lam[i] = nl;
        mu[i] = nm;
    }
    return 0;
}

/*
 * Gradient of J(s_T) through T steps from s_0 = (u0, v0), by checkpointing every
 * S steps, recomputing each segment and running the reverse steps over it.
 *   traj_f32 != 0: the trajectory is the float forward (parameters rounded to
 *                  float, states as float values), i.e. the trajectory a float
 *                  implementation follows; the reverse arithmetic stays double.
 *   traj_f32 == 0: the trajectory is the double forward.
 * lam, mu: on entry dJ/du_T, dJ/dv_T; on exit dJ/du_0, dJ/dv_0.
 * g[8]:    on exit dJ/dp in the order [dt, a, b, eps, c, k3, Du, Dv].
 * uT, vT:  if not NULL, receive s_T of the chosen trajectory.
 */
int oracle_grad(long R, long C, int bc, const double *p, int traj_f32,
                const double *u0, const double *v0, long T, long S,
                double *lam, double *mu, double *g, double *uT, double *vT)
{
    if (R < 1 || C < 1 || T < 0 || S < 1 || (bc != 0 && bc != 1) || !p || !u0 || !v0 ||
        !lam || !mu || !g)
        return -1;
    const long n = R * C;
    const long nseg = (T + S - 1) / S;
    float pf[8];
    for (int q = 0; q < 8; ++q) pf[q] = (float)p[q];
    for (int q = 0; q < 8; ++q) g[q] = 0.0;

    double *ck = (double *)malloc(sizeof(double) * 2 * n * (nseg > 0 ? nseg : 1));
    double *seg = (double *)malloc(sizeof(double) * 2 * n * S);
    double *cu = (double *)malloc(sizeof(double) * n), *cv = (double *)malloc(sizeof(double) * n);
    double *du = (double *)malloc(sizeof(double) * n), *dv = (double *)malloc(sizeof(double) * n);
    float *fu = (float *)malloc(sizeof(float) * n), *fv = (float *)malloc(sizeof(float) * n);
    float *fu2 = (float *)malloc(sizeof(float) * n), *fv2 = (float *)malloc(sizeof(float) * n);
    double *w1 = (double *)malloc(sizeof(double) * n), *w2 = (double *)malloc(sizeof(double) * n);
    double *w3 = (double *)malloc(sizeof(double) * n), *w4 = (double *)malloc(sizeof(double) * n);
    double *rs = (double *)malloc(sizeof(double) * 8 * R);
    int rc = -1;
    if (!ck || !seg || !cu || !cv || !du || !dv || !fu || !fv || !fu2 || !fv2 || !w1 || !w2 ||
        !w3 || !w4 || !rs)
        goto done;

    /* One forward step of the chosen trajectory, (cu,cv) -> (cu,cv). */
#define ADVANCE()                                                                   \
    do {                                                                            \
        if (traj_f32) {                                                             \
            for (long z = 0; z < n; ++z) { fu[z] = (float)cu[z]; fv[z] = (float)cv[z]; } \
            step_f32(R, C, bc, pf, fu, fv, fu2, fv2);                               \
            for (long z = 0; z < n; ++z) { cu[z] = fu2[z]; cv[z] = fv2[z]; }       \
        } else {                                                                    \
            step_f64(R, C, bc, p, cu, cv, du, dv);                                  \
            memcpy(cu, du, sizeof(double) * n); memcpy(cv, dv, sizeof(double) * n); \
        }                                                                           \
    } while (0)

    /* Forward sweep, keeping s_{kS}. */
    for (long z = 0; z < n; ++z) {
        cu[z] = traj_f32 ? (double)(float)u0[z] : u0[z];
        cv[z] = traj_f32 ? (double)(float)v0[z] : v0[z];
    }
    for (long t = 0; t < T; ++t) {
        if (t % S == 0) {
            memcpy(ck + 2 * n * (t / S), cu, sizeof(double) * n);
            memcpy(ck + 2 * n * (t / S) + n, cv, sizeof(double) * n);
        }
        ADVANCE();
    }
    if (uT) memcpy(uT, cu, sizeof(double) * n);
    if (vT) memcpy(vT, cv, sizeof(double) * n);

    /* Reverse sweep, one segment at a time, last segment first. */
    for (long k = nseg - 1; k >= 0; --k) {
        const long t0 = k * S, len = (t0 + S <= T) ? S : T - t0;
        memcpy(cu, ck + 2 * n * k, sizeof(double) * n);
        memcpy(cv, ck + 2 * n * k + n, sizeof(double) * n);
        for (long q = 0; q < len; ++q) {
            memcpy(seg + 2 * n * q, cu, sizeof(double) * n);
            memcpy(seg + 2 * n * q + n, cv, sizeof(double) * n);
            if (q + 1 < len) ADVANCE();
        }
        for (long q = len - 1; q >= 0; --q)
            reverse_step(R, C, bc, p, seg + 2 * n * q, seg + 2 * n * q + n, lam, mu, w1, w2, w3,
                         w4, rs, g);
    }
#undef ADVANCE
    rc = 0;
done:
    free(ck); free(seg); free(cu); free(cv); free(du); free(dv);
    free(fu); free(fv); free(fu2); free(fv2); free(w1); free(w2); free(w3); free(w4); free(rs);
    return rc;
}

/* Number of OpenMP threads a parallel region would use (0 when built without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_num_threads(int n) { (void)n; }
#endif
