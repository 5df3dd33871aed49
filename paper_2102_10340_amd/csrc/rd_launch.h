// rd_launch.h -- internal launchers of the RD-CNN kernels (not part of the ABI).
#pragma once

#include "rd_common.h"
#include "rd_stream.h"

namespace rd {

// Record a message for rdcnn_last_error() (thread-local) and return `code`.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Finite check of a state on the host's request: counts the NaN or infinite
// values among x[0 .. n) on the stream, waits for it, and returns
// RDCNN_ENONFINITE (with a message) if there are any, else RDCNN_OK.  *flag
// is a small device counter made on first use (freed by the caller).
int check_finite_state(const float *x, long long n, int **flag, hipStream_t s, const char *who);

// Largest number of time steps one register-streamed pass may take, per
// columns-per-lane setting (bounded by the 256 architected VGPRs a wave has).
constexpr int kMaxDepthCpl1 = 16;
constexpr int kMaxDepthCpl2 = 16;
constexpr int kMaxDepthCpl4 = 12;

inline int max_depth(int cpl)
{
    return cpl == 4 ? kMaxDepthCpl4 : cpl == 2 ? kMaxDepthCpl2 : cpl == 1 ? kMaxDepthCpl1 : 0;
}

// Same bound for the adjoint kernel (it also keeps state rows per level).
constexpr int kMaxAdjDepthCpl1 = 8;
constexpr int kMaxAdjDepthCpl2 = 8;
constexpr int kMaxAdjDepthCpl4 = 6;

inline int max_adj_depth(int cpl)
{
    return cpl == 4 ? kMaxAdjDepthCpl4 : cpl == 2 ? kMaxAdjDepthCpl2 : cpl == 1 ? kMaxAdjDepthCpl1 : 0;
}

// Number of partial sums the adjoint keeps per tile.
constexpr int kAdjSums = 8;

// Geometry of one register-streamed pass over an R x C grid.
struct StreamGeom {
    int cpl;     // columns held by one lane (1, 2 or 4)
    int depth;   // time steps done in the pass (K)
    int kpad;    // left/right halo columns of a strip (K rounded up to cpl)
    int wout;    // output columns of a strip (64*cpl - 2*kpad)
    int h;       // output rows of a segment
    int nstrips, nsegs, ntiles, per_xcd;
};

// Fill in the strip/segment decomposition; seg_rows <= 0 picks a default.
// Returns false if the shape cannot be tiled with these settings.
bool stream_geometry(int R, int C, int cpl, int depth, int seg_rows, StreamGeom *g);

// Kernel arguments describing the tiling of `geom`.
TileArgs tile_args(int R, int C, int bc, const StreamGeom &geom);

// u = v = ka * x over n cells (state holds u then v).
hipError_t launch_init(const float *x, float ka, float *state, long long n, hipStream_t s);

// One step, one thread per cell, neighbours read straight from global memory.
hipError_t launch_naive(const float *in, float *out, int R, int C, int bc, const Gene &g,
                        hipStream_t s);

// `geom.depth` steps in one pass of the register-streamed kernel.  If rec is
// not null, the states the pass steps from (levels 0..depth-1) are also written
// to rec + (rec_q0 + j) * 2*R*C; with rec_even only the even levels, level j to
// rec + (rec_q0 + j/2) * 2*R*C (the pass must start at an even time; cpl 1 or
// 2, depth <= 8), and with skip_level0 too the even levels from 2 on (`in` is
// already recorded state rec_q0).
// rec_every spaces recorded states rec_every states apart (2: even-time states
// into the even slots of a trajectory with a slot per time).
hipError_t launch_stream(const float *in, float *out, int R, int C, int bc, const Gene &g,
                         const StreamGeom &geom, hipStream_t s, float *rec = nullptr,
                         long long rec_q0 = 0, bool rec_even = false, bool skip_level0 = false,
                         int rec_every = 1);

// Cell models other than FitzHugh-Nagumo on the same streamed kernel
// (rd_models.h).  Their passes take depth 1, 2, 4 or 8 and cols_per_lane 1, 2
// or, for models instantiated that wide (model_max_cpl), 4.
enum { MODEL_FHN = 0, MODEL_GRAY_SCOTT = 1, MODEL_CNN = 2 };
constexpr int kModelParams = 20;  // largest parameter vector (CNN: dt, A[9], B[9], z)
inline int model_nparams(int model)
{
    return model == MODEL_FHN ? 8 : model == MODEL_GRAY_SCOTT ? 5 : model == MODEL_CNN ? 20 : -1;
}
// Whether blocked passes are exact at a zero-flux edge for these parameters.
bool model_mirror_exact(int model, const float *params);
// The widest strip a model is instantiated for (columns per lane: 2 or 4).
int model_max_cpl(int model);
hipError_t launch_model(int model, const float *in, float *out, int R, int C, int bc,
                        const float *params, const StreamGeom &geom, hipStream_t s);
// CNN input layer: w = (B * img) + z (bz = B[9], z), with the grid's boundary rule.
hipError_t launch_cnn_input(const float *img, const float *bz, int R, int C, int bc, float *w,
                            hipStream_t s);

// The (lam, mu) planes a reverse pass reads (in) and writes (out), R x C each.
struct AdjPlanes {
    const float *in_l, *in_m;
    float *out_l, *out_m;
};

// `geom.depth` reverse steps: (lam, mu) io.in -> io.out, reading states
// q_top, q_top-1, ... of a trajectory whose state q sits at states + q *
// every * 2*R*C floats; adds each tile's eight sums to partial.
// lam_sums: also form the sums only dJ/ddt, dJ/dc and dJ/dk3 need.
hipError_t launch_adjoint(const AdjPlanes &io, const float *states, int every, long long q_top,
                          int R, int C, int bc, const Gene &g, const StreamGeom &geom,
                          double *partial, bool lam_sums, hipStream_t s);
// A paired pass: `geom.depth` (2, 4, 6 or 8; cpl 1 or 2) reverse steps from the
// even time t_top, reading the even-time states (s_{2i} at even_states + i *
// every * 2*R*C floats: every = 1 for a compact even-time trajectory, 2 for
// the even slots of a trajectory with a slot per time) and rebuilding the odd
// states it needs.
hipError_t launch_adjoint_pair(const AdjPlanes &io, const float *even_states, int every,
                               long long t_top, int R, int C, int bc, const Gene &g,
                               const StreamGeom &geom, double *partial, bool lam_sums,
                               hipStream_t s);

hipError_t launch_zero(double *p, long long n, hipStream_t s);

// *count = number of NaN or infinite values among x[0 .. n) (count is zeroed
// first by a kernel of its own, so the launch sequence can be captured).
hipError_t launch_count_nonfinite(const float *x, long long n, int *count, hipStream_t s);

// Shared parameters of a batch: dtheta[q] += sum of rows[8 i + q] over
// instances i = 0 .. n-1 in index order (deterministic).
hipError_t launch_grad_row_sum(const double *rows, int n, double *dtheta, hipStream_t s);

// Fold ntiles rows of partial sums into the eight gradients, added to dtheta
// for the bits of mask (dt, a, b, eps, c, k3, Du, Dv = bits 0..7); NaN elsewhere.
hipError_t launch_adjoint_finish(const double *partial, int ntiles, const Gene &g, unsigned mask,
                                 double *dtheta, hipStream_t s);

// One instance of a batch: its offset in the packed buffers, size and gene.
struct BatchInst {
    long long off;  // float offset of the instance in a packed buffer
    int R, C;
    Gene g;
};

// One tile of a batch's flat tile list: instance, first extended column and
// output rows [y0, y1).
struct BatchTile {
    int inst, x0, y0, y1;
};

// One launch of the batched kernel: `depth` steps for every tile of the list.
// With rec, the states the pass steps from also go to the packed trajectory:
// level j of instance i to rec + j * rec_stride bytes + its offset (recording
// passes: cpl 1 or 2, depth <= 8); with rec_even only the even levels, level j
// to rec + (j/2) * rec_stride bytes (the pass starts at an even time).
hipError_t launch_batch(const BatchTile *tiles, const BatchInst *insts, int ntiles,
                        const float *in, float *out, int bc, int cpl, int depth, hipStream_t s,
                        float *rec = nullptr, unsigned rec_stride = 0, bool rec_even = false,
                        bool skip_level0 = false);

// Batched reverse pass: `depth` (1, 2, 4 or 8) reverse steps for every tile,
// cpl 1 or 2; states = packed state q_top-depth+1, state_stride bytes apart.
// The tile list was cut for table_depth >= depth (its halo is used as is).
// paired: a paired pass (depth 2, 4 or 8) over an even-time trajectory; states
// = the packed even state s_{t_top-depth}, the oldest the pass reads.
hipError_t launch_batch_adjoint(const BatchTile *tiles, const BatchInst *insts, int ntiles,
                                const float *in, float *out, const float *states,
                                unsigned state_stride, int bc, int cpl, int depth, int table_depth,
                                double *partial, bool lam_sums, hipStream_t s, bool paired = false);
// Per-instance gradients from the per-tile partials (tiles of instance i:
// tiles_of[first[i] .. first[i+1])), added to dtheta[8 i ..].
hipError_t launch_batch_adjoint_finish(const double *partial, const int *first, const int *tiles_of,
                                       const BatchInst *insts, int n, unsigned mask,
                                       double *dtheta, hipStream_t s);

// All T steps of `count` small instances (indices ids), each held in one
// workgroup's LDS (frame_cells = largest (R+2)*(C+2)).
hipError_t launch_batch_lds(const BatchInst *insts, const int *ids, int count, int frame_cells,
                            const float *in, float *out, int bc, long long T, hipStream_t s);

// Per-instance atlas statistics: chunks of at most kStatChunk cells, one
// workgroup each, folded per instance in chunk order (first[i] .. first[i+1]).
constexpr int kStats = 8;
constexpr int kStatThreads = 256;
constexpr int kStatChunk = 16384;
struct StatChunk {
    int inst;   // instance
    int start;  // first cell (within the instance's plane)
    int count;  // cells
};
hipError_t launch_stats(const BatchInst *insts, const StatChunk *chunks, int nchunks,
                        const int *first, int n_inst, const float *cur, const float *prev,
                        const float *ref, float theta_far, float theta_move, double *partial,
                        double *out, hipStream_t s);

// gx = ka (lam + mu) over n cells.
hipError_t launch_init_backward(const float *adj, long long n, float ka, float *gx,
                                hipStream_t s);

}  // namespace rd
