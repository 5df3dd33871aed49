/*
 * rdcnn.h -- C ABI of the MI355X (gfx950) library for the FitzHugh-Nagumo
 * reaction-diffusion cellular nonlinear network (RD-CNN) of Dogaru & Dogaru,
 * "A Python Framework for Fast Modelling and Simulation of Cellular Nonlinear
 * Networks and other Finite-difference Time-domain Systems" (arXiv 2102.10340).
 *
 * The model (Sec. II.A):
 *   Eq. (1)  u = v = k_a * x, then T Jacobi explicit-Euler steps
 *              u+ = u + dt [ f1(u,v) + Du Lap u ]
 *              v+ = v + dt [ f2(u,v) + Dv Lap v ]
 *            with the unscaled 5-point Laplacian
 *              Lap u_ij = u_{i+1,j} + u_{i-1,j} + u_{i,j-1} + u_{i,j+1} - 4 u_ij.
 *   Eq. (2)  f1 = c u - k3 u^3 - v        (the paper uses k3 = 1/3)
 *   Eq. (3)  f2 = -eps (u - b v + a)
 *
 * Conventions shared by every entry point:
 *   - A grid has `rows` x `cols` cells (both >= 1), row-major, float32.  A
 *     state buffer holds the two layers back to back: u plane then v plane,
 *     i.e. 2 * rows * cols floats, cell (i, j) of u at [i*cols + j] and of v at
 *     [rows*cols + i*cols + j].
 *   - Boundary rule: RDCNN_BC_PERIODIC wraps (toroidal, as in the paper's
 *     kernels); RDCNN_BC_ZEROFLUX lets a missing neighbour copy the edge cell.
 *   - Every pointer named *_dev is device memory owned by the caller; the
 *     library never frees it.  Buffers passed to rdcnn_create must stay valid
 *     until rdcnn_destroy.
 *   - All device work is enqueued on the caller's HIP stream given at creation
 *     (a hipStream_t passed as void*; NULL is the default stream) and is
 *     asynchronous unless stated otherwise.
 *   - Return value: RDCNN_OK (0) or a negative status.  No call throws or
 *     aborts.  rdcnn_last_error() gives a message for the calling thread's most
 *     recent failure.  A handle must not be used from two threads at once.
 *   - Stability is not enforced: explicit Euler with the unscaled Laplacian
 *     needs dt * max(Du, Dv) <= 1/4 to stay bounded; larger values are accepted
 *     and simply diverge, as in the paper's simulator.
 */
#ifndef RDCNN_H
#define RDCNN_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RDCNN_BC_PERIODIC = 0,
    RDCNN_BC_ZEROFLUX = 1
};

enum {
    RDCNN_OK = 0,
    RDCNN_EINVAL = -1,     /* bad argument: null pointer, size < 1, T < 0, non-finite parameter */
    RDCNN_EHIP = -2,       /* a HIP runtime call or kernel launch failed */
    RDCNN_ENONFINITE = -3, /* a checked read found NaN or infinite values in the state */
    RDCNN_ESTATE = -4,     /* call not valid for this handle's state */
    RDCNN_ENOMEM = -5      /* host or device allocation of an internal workspace failed */
};

/* Gene of Sec. II.A (the paper's Pars vector: dt, a, b, eps, c, Du, Dv) plus
 * the cubic coefficient k3 of Eq. (2). */
typedef struct rdcnn_params {
    float dt;  /* Euler step                         */
    float a;   /* Eq. (3) offset                     */
    float b;   /* Eq. (3) v coefficient              */
    float eps; /* Eq. (3) rate, paper sign: f2 = -eps (u - b v + a) */
    float c;   /* Eq. (2) linear coefficient         */
    float k3;  /* Eq. (2) cubic coefficient          */
    float Du;  /* Eq. (1) diffusion of u             */
    float Dv;  /* Eq. (1) diffusion of v             */
} rdcnn_params_t;

typedef struct rdcnn_sim *rdcnn_t;

/*
 * rdcnn_create -- set up one grid and its initial state (Eq. (1), first line:
 * u = v = k_a * x, one float32 multiply per cell).
 *   out       receives the handle (set to NULL on failure)
 *   rows,cols grid size, >= 1 each, rows*cols < 2^30 (a plane below 4 GiB)
 *   bc        RDCNN_BC_PERIODIC or RDCNN_BC_ZEROFLUX
 *   p         parameters (copied); all fields must be finite
 *   x_dev     rows*cols floats, the initial image x (read once, during the call's
 *             stream work; it may be freed after the stream reaches it)
 *   ka        scale k_a (finite)
 *   buf0_dev, buf1_dev
 *             two distinct state buffers of 2*rows*cols floats each, the
 *             ping-pong pair; the initial state is written to buf0_dev
 *   stream    hipStream_t on which all of this handle's work runs
 * Errors: RDCNN_EINVAL for a bad argument, RDCNN_EHIP if the launch fails,
 * RDCNN_ENOMEM if the handle cannot be allocated.
 */
int rdcnn_create(rdcnn_t *out, int rows, int cols, int bc, const rdcnn_params_t *p,
                 const float *x_dev, float ka, float *buf0_dev, float *buf1_dev, void *stream);

/* Built-in cell models for rdcnn_model_create. */
enum {
    RDCNN_MODEL_FITZHUGH_NAGUMO = 0,
    RDCNN_MODEL_GRAY_SCOTT = 1,
    RDCNN_MODEL_CNN = 2
};

/*
 * rdcnn_model_create -- a grid of one of the built-in two-layer cell models,
 * run by the same register-streamed kernel with the model's update swapped in.
 * The paper closes (Sec. IV) by noting that its framework extends to any
 * finite-difference time-domain or cellular model; this is that extension.
 *   RDCNN_MODEL_FITZHUGH_NAGUMO  params (8): dt, a, b, eps, c, k3, Du, Dv
 *       (Eq. (1)-(3)); state starts at (u0, v0).
 *   RDCNN_MODEL_GRAY_SCOTT       params (5): dt, F, k, Du, Dv;
 *       u+ = u + dt (Du Lap u - u v^2 + F (1 - u)),
 *       v+ = v + dt (Dv Lap v + u v^2 - (F + k) v); state starts at (u0, v0).
 *   RDCNN_MODEL_CNN              params (20): dt, A[9], B[9], z (3x3 templates
 *       row-major NW, N, NE, W, C, E, SW, S, SE): a Chua-Yang cellular neural
 *       network x+ = x + dt (-x + (A * y) + w), y = (|x+1| - |x-1|) / 2, with
 *       w = (B * g) + z formed once from the input image g = v0 and kept as the
 *       second layer; the state x starts at u0.
 * Rounding orders are fixed per model (the CPU oracle's cell_models.c writes the
 * same order), so results are bit-identical whatever the pass shape.  A CNN
 * whose A template is not mirror symmetric runs one step per pass at a
 * zero-flux edge (blocked passes would not reproduce the edge-copy rule).
 * rdcnn_step, rdcnn_read, rdcnn_write_state, rdcnn_current, rdcnn_set_kernel
 * (kind 0, 2 or 3) and rdcnn_destroy apply as for rdcnn_create's grids; models
 * other than FitzHugh-Nagumo use passes of 1, 2, 4 or 8 steps and 1 or 2
 * columns per lane (Gray-Scott also 4; a wider setting runs at the model's
 * widest), and have no reverse pass (rdcnn_step_record,
 * rdcnn_adjoint and rdcnn_set_params return RDCNN_EINVAL for them).
 * u0_dev, v0_dev: device, rows*cols floats each; buf0/buf1 as for rdcnn_create.
 * Errors: RDCNN_EINVAL (unknown model, wrong parameter count, non-finite
 * parameter, bad size or buffer), RDCNN_EHIP, RDCNN_ENOMEM.
 */
int rdcnn_model_create(rdcnn_t *out, int model, int rows, int cols, int bc, const float *params,
                       int nparams, const float *u0_dev, const float *v0_dev, float *buf0_dev,
                       float *buf1_dev, void *stream);

/*
 * rdcnn_step -- advance the grid by T time steps of Eq. (1)-(3) ("for t = 1..T").
 * T >= 0; T == 0 does nothing.  Asynchronous.  The current state alternates
 * between the two buffers; rdcnn_current() names the one holding it.
 */
int rdcnn_step(rdcnn_t h, long long T);

/*
 * rdcnn_use_graph -- on != 0: rdcnn_step captures the launch sequence of its T
 * steps into a HIP graph the first time and replays that graph afterwards
 * (one cached graph per starting buffer, rebuilt when T changes; dropped by
 * rdcnn_set_params and rdcnn_set_kernel, whose values the captured launches
 * carry).  This removes the host's per-launch cost for short runs of small
 * grids, where a pass takes a few microseconds.  Results are bit-identical to
 * rdcnn_step without graphs.  The handle's stream must not be the NULL stream.
 * on == 0 drops the graphs.  Errors: RDCNN_EINVAL; capture or instantiation
 * failures later surface from rdcnn_step as RDCNN_EHIP.
 */
int rdcnn_use_graph(rdcnn_t h, int on);

/*
 * rdcnn_read -- copy the current state (the paper's snapshot of A and B,
 * Sec. II.B main loop) into u_dst and v_dst, rows*cols floats each.
 * dst_is_host != 0: host destinations; the call waits for the stream.
 * dst_is_host == 0: device destinations; asynchronous on the stream.
 * With the finite check on (rdcnn_set_check_finite), the call also counts
 * NaN and infinite values of the state on the device, waits for the stream,
 * and returns RDCNN_ENONFINITE if there are any (the copy is made either way):
 * the failure detection for runs that leave the stable range dt*max(Du,Dv) <=
 * 1/4 or are given non-finite inputs.
 * Errors: RDCNN_EINVAL (NULL argument), RDCNN_EHIP, RDCNN_ENONFINITE,
 * RDCNN_ENOMEM (the check's 4-byte device counter, made on first use).
 */
int rdcnn_read(rdcnn_t h, float *u_dst, float *v_dst, int dst_is_host);

/* rdcnn_set_check_finite -- on != 0: later rdcnn_read calls check the state for
 * NaN / Inf (above); 0 (the default): no check.  Errors: RDCNN_EINVAL. */
int rdcnn_set_check_finite(rdcnn_t h, int on);

/*
 * rdcnn_write_state -- replace the current state with (u_dev, v_dev), rows*cols
 * device floats each (checkpoint restore / resume).  Asynchronous.
 */
int rdcnn_write_state(rdcnn_t h, const float *u_dev, const float *v_dev);

/* rdcnn_set_params -- replace the parameters used by later steps. */
int rdcnn_set_params(rdcnn_t h, const rdcnn_params_t *p);

/* rdcnn_current -- device pointer of the buffer holding the current state. */
int rdcnn_current(rdcnn_t h, float **state_dev);

/*
 * rdcnn_set_kernel -- choose how later rdcnn_step calls run (testing and
 * tuning; the default is chosen per grid shape).
 *   kind 0: automatic; 1: one thread per cell, one launch per step (reference
 *   kernel); 2: register-streamed kernel doing up to `depth` steps per HBM pass,
 *   for every call that steps (the recording calls cap it to what they support);
 *   3: as 2 for rdcnn_step and rdcnn_step_checkpoints only, the recording calls
 *   keep their automatic shapes (what an autotuned forward shape wants).
 *   cols_per_lane 1 or 2 (depth 1..16) or 4 (depth 1..12); seg_rows: output rows
 *   per wavefront, 0 = automatic.  Other fields are ignored for kinds 0 and 1.
 *   Every setting gives bit-identical states.  Errors: RDCNN_EINVAL.
 */
int rdcnn_set_kernel(rdcnn_t h, int kind, int depth, int cols_per_lane, int seg_rows);

/*
 * rdcnn_pass_config -- the pass shape later rdcnn_step calls use, with the
 * automatic choices resolved: *kind 1 (one thread per cell) or 2 (streamed),
 * *depth steps per pass, *cols_per_lane, *seg_rows output rows per wavefront
 * (the paper's block/grid choice, Sec. II.B, made explicit).  Host-only, no
 * device work.  Errors: RDCNN_EINVAL (NULL argument).
 */
int rdcnn_pass_config(rdcnn_t h, int *kind, int *depth, int *cols_per_lane, int *seg_rows);

/*
 * rdcnn_step_record -- like rdcnn_step, and also writes the state each of the T
 * steps starts from: s_t, s_{t+1}, ..., s_{t+T-1} (t = the handle's current
 * time) to states_dev[0..T-1], each 2*rows*cols floats (u plane, v plane).
 * These are the states the reverse pass needs.  states_dev: device memory of
 * at least T*2*rows*cols floats.  Asynchronous.
 */
int rdcnn_step_record(rdcnn_t h, long long T, float *states_dev);

/*
 * rdcnn_adjoint -- reverse pass through S steps of Eq. (1)-(3) (the transpose of
 * the Jacobian of the explicit-Euler step; the paper gives the forward model
 * only, Sec. II.A).  For a loss J of the state after the S steps:
 *   states_dev  the S states the steps started from, as written by
 *               rdcnn_step_record (states_dev[q] = s_{t0+q}); read only
 *   adj_dev     [2][rows][cols] floats: on entry (dJ/du, dJ/dv) after the S
 *               steps, on exit (dJ/du, dJ/dv) before them
 *   adj_tmp_dev scratch of the same size (contents overwritten)
 *   dtheta_dev  8 device doubles; dJ/dp of these S steps is ADDED, in the order
 *               dt, a, b, eps, c, k3, Du, Dv (rdcnn_params_t order), for the
 *               parameters of the gradient mask (rdcnn_set_grad_mask; default
 *               all), NaN for the others
 * Uses the handle's current parameters, boundary rule and stream.  S == 0 does
 * nothing.  A call takes a small device workspace for per-tile partial sums
 * (8 doubles per tile) from a process-wide pool, allocating one the first time;
 * rdcnn_destroy returns it to the pool (at most 16 buffers, kept until the
 * process ends), and a later user's stream is ordered after this handle's
 * work on it by an event, so handles can come and go without allocating or
 * synchronizing.  Results
 * are deterministic (fixed reduction order).  Asynchronous.
 * Errors: RDCNN_EINVAL, RDCNN_ENOMEM (workspace), RDCNN_EHIP.
 */
int rdcnn_adjoint(rdcnn_t h, const float *states_dev, long long S, float *adj_dev,
                  float *adj_tmp_dev, double *dtheta_dev);

/*
 * rdcnn_step_record_even -- like rdcnn_step_record, but keeps only the states
 * of even times counted from the handle's current time: s_{t+2i} goes to
 * states_dev[i] for 2i < T, i.e. (T+1)/2 states of 2*rows*cols floats each
 * (half the memory and half the writes).  Passes run 8 steps (or the even
 * depth set with rdcnn_set_kernel; at most 8, one or two columns per lane).
 * The passes also read their input from, and write their output to,
 * states_dev (each recorded state is written once), so states_dev must not
 * overlap the handle's state buffers.  These are the states rdcnn_adjoint_even
 * reads.  Asynchronous.  Errors: RDCNN_EINVAL, RDCNN_EHIP.
 */
int rdcnn_step_record_even(rdcnn_t h, long long T, float *states_dev);

/*
 * rdcnn_adjoint_even -- rdcnn_adjoint from an even-time trajectory: the same
 * reverse pass through S steps of Eq. (1)-(3) (same arguments, results and
 * errors), with states_dev as written by rdcnn_step_record_even
 * (states_dev[i] = s_{t0+2i}, (S+1)/2 states).  Each reverse pass rebuilds
 * the odd-time states it needs from the even ones with the forward cell
 * update, bit-identical to the forward pass, so (dJ/du, dJ/dv) equals
 * rdcnn_adjoint's bit for bit.  Uses rdcnn_set_adjoint_kernel's settings with
 * an even depth of 2..8 and at most two columns per lane.
 */
int rdcnn_adjoint_even(rdcnn_t h, const float *states_dev, long long S, float *adj_dev,
                       float *adj_tmp_dev, double *dtheta_dev);

/*
 * rdcnn_step_checkpoints -- rdcnn_step for T steps that also keeps a checkpoint
 * every S steps: s_{t+jS} goes to ckpt_dev[j] for jS < T (ceil(T/S) states of
 * 2*rows*cols floats; t = the handle's current time, so ckpt_dev[0] is a copy
 * of the current state).  Passes end at every multiple of S, and the pass that
 * ends there writes its output straight into the checkpoint (no extra copy).
 * The forward half of checkpoint-and-recompute; rdcnn_step_bwd is the
 * backward half.  ckpt_dev must not overlap the handle's state buffers.
 * Asynchronous.  Errors: RDCNN_EINVAL (S < 1, T < 0, NULL or overlapping
 * buffer, not a FitzHugh-Nagumo grid), RDCNN_EHIP.
 */
int rdcnn_step_checkpoints(rdcnn_t h, long long T, long long S, float *ckpt_dev);

/*
 * rdcnn_step_record_sparse -- rdcnn_step_record_even writing into a trajectory
 * with one slot per time: s_{t+2i} goes to states_dev[2i] for 2i < T (slots
 * of odd index are not written).  This is the layout rdcnn_step_bwd reads.
 * states_dev: device, at least T+1 states of 2*rows*cols floats; it must not
 * overlap the handle's state buffers (the passes read their input from it).
 * Asynchronous.  Errors: RDCNN_EINVAL, RDCNN_EHIP.
 */
int rdcnn_step_record_sparse(rdcnn_t h, long long T, float *states_dev);

/*
 * rdcnn_step_bwd -- reverse pass through one recorded segment of S steps of
 * Eq. (1)-(3): the transpose of the Jacobian of the explicit-Euler step (the
 * paper gives the forward model only, Sec. II.A), for the gradient of a loss J
 * of the state after the segment.  This is the backward half of
 * checkpoint-and-recompute: restore a checkpoint s_{t0}, record the S steps
 * after it, call rdcnn_step_bwd.
 *   states_dev   [S+1][2][rows][cols] floats, device: states_dev[q] = s_{t0+q},
 *                the state step q of the segment starts from.  Only the slots
 *                of even q < S are read (rdcnn_step_record and
 *                rdcnn_step_record_sparse both fill them); each reverse pass
 *                rebuilds the odd-time states it needs from the even ones with
 *                the forward cell update, bit-identical to the forward pass.
 *                Slot S (the state after the segment, never needed) is
 *                overwritten: it is the reverse passes' workspace.
 *   S            steps (>= 0; 0 does nothing)
 *   lam_dev      rows*cols floats: on entry dJ/du at t0+S, on return dJ/du at t0
 *   mu_dev       rows*cols floats: the same for v (distinct from lam_dev)
 *   dtheta_accum 8 device doubles: dJ/dp of this segment is ADDED, order dt, a,
 *                b, eps, c, k3, Du, Dv, for the parameters of the gradient
 *                mask (rdcnn_set_grad_mask); NaN for the others
 * Uses the handle's parameters, boundary rule, stream and reverse-pass
 * settings (rdcnn_set_adjoint_kernel: an even depth of 2..8, one or two
 * columns per lane).  The per-tile partial sums come from the process-wide
 * pool described at rdcnn_adjoint.  Deterministic.  Asynchronous.
 * Errors: RDCNN_EINVAL (NULL or overlapping buffers, S < 0, not a
 * FitzHugh-Nagumo grid), RDCNN_ENOMEM, RDCNN_EHIP.
 */
int rdcnn_step_bwd(rdcnn_t h, float *states_dev, long long S, float *lam_dev, float *mu_dev,
                   double *dtheta_accum);

/*
 * rdcnn_step_bwd_ckpt -- the whole backward half of checkpoint-and-recompute
 * for T steps whose forward kept a checkpoint every S steps
 * (rdcnn_step_checkpoints): for the segments from last to first, restore the
 * checkpoint, re-run the segment recording the states of its even times
 * (rdcnn_step_record_sparse's layout) and run the reverse passes of
 * rdcnn_step_bwd through it.  The recompute of segment k runs on a second
 * stream while the reverse passes of segment k+1 run on the handle's stream;
 * the two alternate between the two halves of work_dev.  The second stream is
 * the device's: made by the library on first use (default priority), shared by
 * every handle on that device (each orders its own work on it with its own
 * events) and kept until the process ends; rdcnn_destroy waits for the
 * handle's work on it.  The partial
 * sums of all segments go to one buffer, folded once at the end.
 *   ckpt_dev     device, ceil(T/S) states of 2*rows*cols floats: checkpoint j =
 *                s_{t0+jS} (read only)
 *   T, S         steps (T >= 0; 0 does nothing) and checkpoint spacing (S >= 1)
 *   work_dev     device, 2*(min(S,T)+1) states of 2*rows*cols floats (scratch;
 *                overlaps neither ckpt_dev, lam_dev nor mu_dev)
 *   lam_dev      rows*cols floats: on entry dJ/du at t0+T, on return dJ/du at t0
 *   mu_dev       the same for v (distinct from lam_dev)
 *   dtheta_accum 8 device doubles: dJ/dp is ADDED (order dt, a, b, eps, c, k3,
 *                Du, Dv) for the parameters of the gradient mask; NaN for the others
 * Results: (lam, mu) bit-identical to rdcnn_step_bwd run segment by segment
 * on the same recomputed states; dtheta equal up to the order of its final
 * double-precision sum.  Deterministic.  Asynchronous with respect to the host;
 * all work is ordered after the handle's earlier work and before its later
 * work.  Errors: RDCNN_EINVAL (NULL or overlapping buffers, T < 0, S < 1, not a
 * FitzHugh-Nagumo grid, grid too large to record), RDCNN_ENOMEM, RDCNN_EHIP.
 */
int rdcnn_step_bwd_ckpt(rdcnn_t h, const float *ckpt_dev, long long T, long long S,
                        float *work_dev, float *lam_dev, float *mu_dev, double *dtheta_accum);

/*
 * rdcnn_step_bwd_noalloc --rdcnn_step_bwd for callers that cannot allocate
 * device memory: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels, launch order and
 * results (bit for bit) as rdcnn_step_bwd; the per-tile partial sums live in
 * a static device array of the library instead of the pooled buffer, so the
 * call makes no hipMalloc, hipFree or other allocation.  Limit: the reverse
 * passes may use at most 65536 tiles (4 MiB of partial sums; the automatic
 * pass shape uses about 2600 on any grid up to 2^30 cells); more is rejected
 * with RDCNN_EINVAL and a message naming the count.  The array is resolved
 * once per device (at rdcnn_create, or at the first call on a device) and
 * stays allocated until the process ends.  Every call on one device shares
 * that device's array and zeroes it on the stream before use (by a kernel,
 * no memset), so calls that overlap on one device -- on different streams or
 * from different threads -- race; calls ordered on one stream do not.  Its
 * contents after a call are the last call's partial sums.
 * Errors: as rdcnn_step_bwd, plus RDCNN_EINVAL for a tiling over the limit.
 */
int rdcnn_step_bwd_noalloc(rdcnn_t h, float *states_dev, long long S, float *lam_dev,
                           float *mu_dev, double *dtheta_accum);

/*
 * rdcnn_set_adjoint_kernel -- pass settings for rdcnn_adjoint: `depth` reverse
 * steps per HBM pass, cols_per_lane 1 or 2 (depth 1..8) or 4 (depth 1..6), seg_rows
 * output rows per wavefront (0 = automatic).  depth = cols_per_lane = 0 restores
 * the automatic choice.  Errors: RDCNN_EINVAL.
 */
int rdcnn_set_adjoint_kernel(rdcnn_t h, int depth, int cols_per_lane, int seg_rows);

/*
 * rdcnn_set_grad_mask -- which parameter gradients later rdcnn_adjoint calls
 * form: bit q set = parameter q in rdcnn_params_t order (dt = bit 0 ... Dv =
 * bit 7); default 0xFF (all).  Entries outside the mask are set to NaN in
 * dtheta_dev instead of being accumulated.  Leaving dt, c and k3 out skips three
 * of the eight inner products.  mask must be in 1..0xFF.  Errors: RDCNN_EINVAL.
 */
int rdcnn_set_grad_mask(rdcnn_t h, unsigned mask);

/*
 * rdcnn_init_backward -- chain rule through Eq. (1)'s first line (u = v = k_a x):
 * gx[i] = ka * (adj[i] + adj[n + i]) for i < n, with adj laid out as
 * [2][n] (dJ/du then dJ/dv) and gx n floats, both device memory.  Runs on
 * `stream` (a hipStream_t).  Errors: RDCNN_EINVAL, RDCNN_EHIP.
 */
int rdcnn_init_backward(const float *adj_dev, long long n, float ka, float *gx_dev, void *stream);

/* ------------------------------------------------------------ batches
 * Many grids of uneven size and parameters advanced together: the paper's
 * parameter-space exploration (Sec. III), where each simulation was run by hand,
 * one at a time.  Every step of every instance is Eq. (1)-(3) with that
 * instance's parameters, bit-identical to a single-grid run. */
typedef struct rdcnn_batch *rdcnn_batch_t;

/*
 * rdcnn_batch_create -- set up n instances in two packed ping-pong buffers.
 *   rows[i], cols[i]  size of instance i (>= 1, rows*cols < 2^30)
 *   offsets[i]        float offset of instance i in each state buffer, a multiple
 *                     of 64 (256 bytes); the instance occupies 2*rows*cols floats
 *                     there (u plane, v plane); instances must not overlap
 *   params[i]         parameters of instance i (copied; finite)
 *   bc                boundary rule shared by all instances
 *   x_dev, x_offsets  initial image of instance i at x_dev + x_offsets[i]
 *                     (rows*cols floats); u = v = ka*x (Eq. (1), first line)
 *   buf0_dev, buf1_dev, buf_floats
 *                     the two packed state buffers and their length in floats;
 *                     the initial states go to buf0_dev
 *   stream            hipStream_t for all of the batch's work
 * Host arrays are read during the call only.  Allocates two small device
 * tables (instances, tiles), freed by rdcnn_batch_destroy.
 * Errors: RDCNN_EINVAL, RDCNN_ENOMEM, RDCNN_EHIP.
 */
int rdcnn_batch_create(rdcnn_batch_t *out, int n, const int *rows, const int *cols,
                       const long long *offsets, const rdcnn_params_t *params, int bc,
                       const float *x_dev, const long long *x_offsets, float ka, float *buf0_dev,
                       float *buf1_dev, long long buf_floats, void *stream);

/* rdcnn_batch_step -- advance every instance by T steps (asynchronous). */
int rdcnn_batch_step(rdcnn_batch_t b, long long T);

/* rdcnn_batch_current -- the packed buffer holding the current states. */
int rdcnn_batch_current(rdcnn_batch_t b, float **state_dev);

/*
 * rdcnn_batch_read -- copy the current packed state (buf_floats floats, every
 * instance at its offset) to dst_packed_dev (device memory, not overlapping the
 * batch's buffers): the batch's snapshot (Sec. II.B main loop).  Asynchronous
 * on the batch's stream, unless the finite check is on
 * (rdcnn_batch_set_check_finite): then every instance's cells are checked for
 * NaN / Inf on the device, the call waits, and returns RDCNN_ENONFINITE if any
 * are found.  Errors: RDCNN_EINVAL, RDCNN_EHIP, RDCNN_ENONFINITE, RDCNN_ENOMEM.
 */
int rdcnn_batch_read(rdcnn_batch_t b, float *dst_packed_dev);

/* rdcnn_batch_set_check_finite -- on != 0: rdcnn_batch_read checks for NaN /
 * Inf (above).  Errors: RDCNN_EINVAL. */
int rdcnn_batch_set_check_finite(rdcnn_batch_t b, int on);

/*
 * rdcnn_batch_set_kernel -- steps per pass (depth), cols_per_lane (1, 2 or 4) and
 * rows per tile (seg_rows, 0 = default) of later steps; all zero restores the
 * defaults.  Results are bit-identical for every setting.  Errors: RDCNN_EINVAL.
 */
int rdcnn_batch_set_kernel(rdcnn_batch_t b, int depth, int cols_per_lane, int seg_rows);

/*
 * rdcnn_batch_set_class_seg_rows -- rows per tile for every instance of size
 * rows x cols (a size class) in later plain steps (rdcnn_batch_step), in place
 * of the batch-wide seg_rows; 0 returns the class to it.  Steps per pass and
 * columns per lane stay batch-wide: one launch covers every class, so each
 * pass mixes all classes' tiles (longest first) in one grid.  The paper tunes
 * block and grid shapes by hand per run (Sec. II.B); the autotuner picks a
 * height per class with this.  Results are bit-identical for every setting.
 * Errors: RDCNN_EINVAL (seg_rows < 0, or no instance of that size).
 */
int rdcnn_batch_set_class_seg_rows(rdcnn_batch_t b, int rows, int cols, int seg_rows);

/*
 * rdcnn_batch_use_graph -- on != 0: rdcnn_batch_step captures the launches of a
 * T-step run into a HIP graph on first use and replays it afterwards (one graph
 * launch per call).  Needs a non-default stream.  Errors: RDCNN_EINVAL.
 */
int rdcnn_batch_use_graph(rdcnn_batch_t b, int on);

/*
 * rdcnn_batch_use_lds -- on != 0 (the default): instances small enough to sit
 * whole in one workgroup's LDS (at most 16384 cells, (rows+2)*(cols+2) pairs of
 * floats within the device's per-workgroup LDS) run all T steps of a
 * rdcnn_batch_step call in one launch, reading and writing HBM once.  Results
 * are bit-identical either way.  Errors: RDCNN_EINVAL, RDCNN_ENOMEM.
 */
int rdcnn_batch_use_lds(rdcnn_batch_t b, int on);

/* rdcnn_batch_lds_instances -- *count = number of instances that the in-LDS
 * kernel runs under the current setting.  Errors: RDCNN_EINVAL (NULL). */
int rdcnn_batch_lds_instances(rdcnn_batch_t b, int *count);

/*
 * rdcnn_batch_write_state -- replace the current packed state with `packed`
 * (device, buf_floats floats in this batch's layout).  Stream-ordered.
 * Errors: RDCNN_EINVAL (NULL), RDCNN_EHIP.
 */
int rdcnn_batch_write_state(rdcnn_batch_t b, const float *packed);

/*
 * rdcnn_batch_step_record -- rdcnn_batch_step for T steps, also writing the
 * state every step starts from: packed state q (the whole batch before step q,
 * q = 0 .. T-1) goes to traj + q * buf_floats.  traj: device, T * buf_floats
 * floats, caller-owned.  Recording runs every instance on the streamed kernel
 * (no in-LDS path, no graph) with 1 or 2 columns per lane and at most 8 steps
 * per pass, fewer where one instance's span of a pass's states would pass
 * 4 GiB.  Results equal rdcnn_batch_step's bit for bit.  This is the forward
 * half of the batched reverse pass (below).  Errors: RDCNN_EINVAL, RDCNN_ENOMEM,
 * RDCNN_EHIP.
 */
int rdcnn_batch_step_record(rdcnn_batch_t b, long long T, float *traj);

/*
 * rdcnn_batch_set_adjoint_kernel -- pass shape of rdcnn_batch_adjoint: depth
 * (reverse steps per pass: 1, 2, 4 or 8), cols_per_lane (1 or 2), seg_rows
 * (rows per tile); 0 keeps the default (8, 1, 128).  Passes are made shallower
 * where one instance's span of a pass's states would pass 4 GiB.  Errors:
 * RDCNN_EINVAL.
 */
int rdcnn_batch_set_adjoint_kernel(rdcnn_batch_t b, int depth, int cols_per_lane, int seg_rows);

/*
 * rdcnn_batch_adjoint -- the reverse pass of rdcnn_adjoint for every instance
 * of the batch at once (the transpose of the step's Jacobian, Eq. (1)-(3)):
 * traj holds S packed states, state q at traj + q * buf_floats, the states the
 * last S steps started from (as rdcnn_batch_step_record writes them).  adj
 * (device, packed layout, caller-owned): on entry dJ/ds after the S steps, on
 * return dJ/ds before them, per instance (u plane then v plane).  adj_tmp:
 * scratch of buf_floats floats.  dtheta (device, n x 8 doubles,
 * instance-major, order dt, a, b, eps, c, k3, Du, Dv): each instance's
 * parameter gradients are added to its row (or, with rdcnn_batch_set_shared_grad,
 * their sum over instances to dtheta[0 .. 8)); gradients whose bit is clear in
 * mask are not formed and come back NaN.  Sums are folded per instance in a
 * fixed order (deterministic).  The first call allocates the tile list and the
 * per-tile partial buffer (kept until destroy).  Errors: RDCNN_EINVAL (NULL or
 * aliased buffers, S < 0, one instance's state alone above 4 GiB), RDCNN_ENOMEM,
 * RDCNN_EHIP.
 */
int rdcnn_batch_adjoint(rdcnn_batch_t b, const float *traj, long long S, float *adj,
                        float *adj_tmp, unsigned mask, double *dtheta);

/*
 * rdcnn_batch_set_shared_grad -- on != 0: the batch's instances share one
 * parameter vector (the edge-detection fit), and rdcnn_batch_adjoint[_even]
 * add the gradient of that vector to dtheta[0 .. 8): the per-instance
 * gradients summed on the device over instances 0 .. n-1 in index order
 * (deterministic).  0 (the default): one row per instance, dtheta[8 i ..].
 * Errors: RDCNN_EINVAL.
 */
int rdcnn_batch_set_shared_grad(rdcnn_batch_t b, int on);

/*
 * rdcnn_batch_step_record_even -- rdcnn_batch_step_record keeping only the
 * states of even times: packed state 2i goes to traj + i * buf_floats for
 * 2i < T ((T+1)/2 states; half the memory and writes).  Passes take an even
 * depth (at most 8) and read their input from, and write their output to, traj
 * (each recorded state is written once), so traj must not overlap the batch's
 * state buffers.  The trajectory rdcnn_batch_adjoint_even reads.
 * Errors: as rdcnn_batch_step_record.
 */
int rdcnn_batch_step_record_even(rdcnn_batch_t b, long long T, float *traj);

/*
 * rdcnn_batch_adjoint_even -- rdcnn_batch_adjoint from an even-time trajectory
 * (rdcnn_batch_step_record_even; (S+1)/2 packed states).  Each paired reverse
 * pass rebuilds the odd-time states from the even ones with the forward cell
 * update, bit-identical to the forward pass, so dJ/ds equals
 * rdcnn_batch_adjoint's bit for bit.  Same arguments, outputs and errors;
 * also RDCNN_EINVAL when the adjoint depth is 1 (paired passes take 2 or more).
 */
int rdcnn_batch_adjoint_even(rdcnn_batch_t b, const float *traj, long long S, float *adj,
                             float *adj_tmp, unsigned mask, double *dtheta);

/*
 * rdcnn_batch_stats -- per-instance statistics of the current state for a
 * parameter atlas (the automated form of the (Du, Dv) scans of Sec. III.A,
 * Fig. 9).  For instance i with N cells, out[8*i + k] (doubles, device) is
 *   0 mean_u   1 var_u   2 mean_v   3 var_v
 *   4 frac_far    = #{ |u - ref[i]| > theta_far } / N
 *   5 frac_moving = #{ |u - u_prev| > theta_move } / N
 *   6 max_change  = max |u - u_prev|
 *   7 rms_change  = sqrt(sum (u - u_prev)^2 / N)
 * where u_prev comes from `prev` (device, a packed buffer in this batch's
 * layout holding an earlier state, e.g. a copy of rdcnn_batch_current's
 * buffer; 16-byte aligned); with prev NULL entries 5-7 are NaN.  ref: device array of n floats,
 * or NULL for 0.  Threshold tests and differences are taken in float32 (exact
 * counts); sums in double, folded in a fixed order (deterministic).  The first
 * call allocates a chunk table and partial buffer kept until destroy.
 * Stream-ordered on the batch's stream.  Errors: RDCNN_EINVAL (NULL b or out,
 * thresholds negative or not finite, prev misaligned), RDCNN_ENOMEM, RDCNN_EHIP.
 */
int rdcnn_batch_stats(rdcnn_batch_t b, const float *prev, const float *ref, float theta_far,
                      float theta_move, double *out);

/* rdcnn_batch_destroy -- release the batch (not the caller's buffers).  NULL is a no-op. */
int rdcnn_batch_destroy(rdcnn_batch_t b);

/* rdcnn_destroy -- release the handle (not the caller's buffers).  NULL is a no-op. */
int rdcnn_destroy(rdcnn_t h);

/* Message describing the calling thread's most recent failed call ("" if none). */
const char *rdcnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RDCNN_H */
