// rd_batch.hip -- many RD-CNN grids of uneven size and parameters advanced
// together (the paper's parameter-space exploration, Sec. III, run as one
// batch instead of one simulation at a time).
//
// All instances live in two packed ping-pong buffers; instance i occupies
// 2*R_i*C_i floats (u plane, v plane) at a 256-byte aligned offset.  One launch
// advances every instance by K steps: its workgroups walk a flat tile list
// that covers all instances (strips x segments of each grid, as in the single
// grid kernel), each tile carrying its instance's offset, size and parameters,
// sorted by decreasing work so the longest tiles start first.  A run of T steps
// is ceil(T/K) such launches, optionally captured once into a HIP graph and
// replayed.  The streamed kernel's template is in rd_batch_kernel.h and its
// instances in rd_batch_r0.hip / rd_batch_rec.hip.
#include <math.h>

#include <algorithm>
#include <new>
#include <vector>

#include "rd_batch_kernel.h"
#include "rdcnn.h"

namespace rd {

// ---------------------------------------------------------------- in-LDS instances
//
// A small instance is held whole in one workgroup's LDS for all T steps: one
// HBM read at the start, one write at the end.  The LDS frame is (R+2) x (C+2)
// (u, v) pairs with a ghost ring; the threads owning edge cells rewrite the
// ghost cells after every step (a copy of the edge cell for zero-flux, of the
// opposite edge for periodic), so the stencil reads fixed offsets.  Thread t
// owns column t mod C and a run of m = ceil(R / s) consecutive rows of it
// (s = 1024 / C runs per column), walking down the run with the north and
// centre values in registers: three LDS reads per cell.  The new values are
// held in registers until every thread has read the old ones.  Same
// cell_update as every other kernel, so results are bit-identical.
constexpr int kLdsThreads = 1024;
constexpr int kLdsRun = 16;  // longest run of rows per thread

// Padded-frame offsets, relative to a cell of the first (left) or last (right)
// column, of the ghost cell that copies it: zero-flux, the ghost beside it;
// periodic, the ghost beyond the opposite edge.  0 for a cell not on that edge
// (a one-column grid is on both).
__device__ __forceinline__ int ghost_left(int c, int C, bool per)
{
    return c == 0 ? (per ? C : -1) : 0;
}
__device__ __forceinline__ int ghost_right(int c, int C, bool per)
{
    return c == C - 1 ? (per ? -C : 1) : 0;
}

__global__ __launch_bounds__(kLdsThreads) void batch_lds_kernel(const BatchInst *insts,
                                                                const int *ids, const float *in,
                                                                float *out, int bc, long long T)
{
    extern __shared__ float2 sm[];
    const BatchInst I = insts[ids[blockIdx.x]];
    const int R = I.R, C = I.C, n = R * C, P = C + 2;
    const bool per = bc == BC_PERIODIC;
    const Gene g = I.g;
    const int runs = kLdsThreads / C;     // host guarantees C <= kLdsThreads
    const int m = (R + runs - 1) / runs;  // host guarantees m <= kLdsRun
    const int t = (int)threadIdx.x;
    const int c = t % C;
    // Every thread walks m cells (a uniform trip count keeps the loop in
    // scalar branches); threads past runs * C walk the first run again, and
    // cells at rows >= R (frame rows up to runs * m, which the host sizes the
    // frame for) are computed from whatever the frame holds but never stored.
    const int r0 = t < runs * C ? (t / C) * m : 0;
    const int len = t < runs * C ? max(0, min(m, R - r0)) : 0;  // cells this thread stores
    const float *iu = in + I.off;
    const float *iv = iu + n;
    float *ou = out + I.off;
    float *ov = ou + n;
    const int base = (r0 + 1) * P + c + 1;  // padded index of the run's first cell
    const int dl = ghost_left(c, C, per), dr = ghost_right(c, C, per);
    // row ghosts: the top row's copy goes to row R (periodic) or -1, the
    // bottom row's to row -1 or R
    const int top_ghost = len > 0 && r0 == 0 ? (per ? base + R * P : base - P) : -1;
    const int bot_ghost = len > 0 && r0 + len == R ? (per ? c + 1 : base + len * P) : -1;
    for (int i = 0; i < len; ++i) {
        const int r = r0 + i;
        const float2 w = make_float2(iu[r * C + c], iv[r * C + c]);
        sm[base + i * P] = w;
        if (dl) sm[base + i * P + dl] = w;
        if (dr) sm[base + i * P + dr] = w;
    }
    if (top_ghost >= 0) sm[top_ghost] = sm[base];
    if (bot_ghost >= 0) sm[bot_ghost] = sm[base + (len - 1) * P];
    __syncthreads();
    for (long long step = 0; step < T; ++step) {
        float2 nw[kLdsRun];
        // Opaque copy of the base: stops the compiler from precomputing all
        // 16 x 4 frame addresses outside the step loop (they would not fit in
        // registers); each cell then costs one address add.
        int pk = base;
        asm volatile("" : "+v"(pk));
        float2 nn = sm[pk - P], ce = sm[pk];
#pragma unroll
        for (int i = 0; i < kLdsRun; ++i) {
            if (i < m) {
                const float2 ss = sm[pk + P], ww = sm[pk - 1], ee = sm[pk + 1];
                pk += P;
                float uo, vo;
                cell_update(g, ce.x, ce.y, nn.x, ss.x, ww.x, ee.x, nn.y, ss.y, ww.y, ee.y, uo,
                            vo);
                nw[i] = make_float2(uo, vo);
                nn = ce;
                ce = ss;
            }
        }
        __syncthreads();
        pk = base;
        asm volatile("" : "+v"(pk));
#pragma unroll
        for (int i = 0; i < kLdsRun; ++i)
            if (i < len) {
                sm[pk] = nw[i];
                if (dl) sm[pk + dl] = nw[i];
                if (dr) sm[pk + dr] = nw[i];
                pk += P;
            }
        // the thread's own writes above are visible to its own reads
        if (top_ghost >= 0) sm[top_ghost] = sm[base];
        if (bot_ghost >= 0) sm[bot_ghost] = sm[base + (len - 1) * P];
        __syncthreads();
    }
    for (int i = 0; i < len; ++i) {
        const int r = r0 + i;
        const float2 w = sm[base + i * P];
        ou[r * C + c] = w.x;
        ov[r * C + c] = w.y;
    }
}

hipError_t launch_batch_lds(const BatchInst *insts, const int *ids, int count, int frame_cells,
                            const float *in, float *out, int bc, long long T, hipStream_t s)
{
    const size_t bytes = sizeof(float2) * (size_t)frame_cells;
    hipError_t e = hipFuncSetAttribute((const void *)batch_lds_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_lds_kernel, dim3((unsigned)count), dim3(kLdsThreads), bytes, s, insts,
                       ids, in, out, bc, T);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchTile *tiles, const BatchInst *insts, int ntiles,
                        const float *in, float *out, int bc, int cpl, int depth, hipStream_t s,
                        float *rec, unsigned rec_stride, bool rec_even, bool skip_level0)
{
    BatchFn f = !rec ? batch_fn_r0(cpl, depth)
                     : batch_fn_rec(rec_even ? (skip_level0 ? 3 : 2) : 1, cpl, depth);
    if (!f || ntiles < 1) return hipErrorInvalidValue;
    BatchArgs a;
    a.tiles = tiles;
    a.insts = insts;
    a.ntiles = ntiles;
    a.in = in;
    a.out = out;
    a.bc = bc;
    a.kpad = (depth + cpl - 1) / cpl * cpl;
    a.wout = 64 * cpl - 2 * a.kpad;
    a.rec = rec;
    a.rec_stride = rec_stride;
    hipLaunchKernelGGL(f, dim3((unsigned)ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace rd

// ---------------------------------------------------------------- C ABI

struct TileTable {
    int depth = 0;
    int ntiles = 0;
    rd::BatchTile *dev = nullptr;
};

struct rdcnn_batch {
    int n, bc;
    int use_lds;                // hold small instances in LDS for a whole run
    int lds_limit;              // frame cells one workgroup's LDS can hold
    std::vector<char> in_lds;   // instance i runs in the in-LDS kernel
    int *lds_ids_dev;           // their indices
    int lds_count, lds_frame;   // how many, largest frame
    std::vector<int> R, C;
    std::vector<int> seg_of;    // per-instance rows per tile of plain passes (0: the batch's)
    std::vector<long long> off;
    std::vector<rd::Gene> g;
    float *buf[2];
    int cur;
    hipStream_t stream;
    int cpl, depth, seg_rows;  // forced settings, 0 = automatic
    rd::BatchInst *insts_dev;
    std::vector<TileTable> tables;
    int use_graph;
    hipGraphExec_t graph;
    long long graph_T;
    int graph_cur, graph_cpl, graph_depth, graph_seg;
    // atlas statistics: chunk list, per-instance chunk ranges, partials (made
    // on the first rdcnn_batch_stats call)
    rd::StatChunk *stat_chunks;
    int *stat_first;
    double *stat_partial;
    int stat_nchunks;
    long long total;                 // floats in one packed state buffer
    std::vector<TileTable> rec_tables;  // recording passes (every instance streamed)
    int rec_cpl;
    // reverse pass: one tile list (cut for adj_depth), per-instance tile lists
    TileTable adj_table;
    int adj_cpl, adj_depth, adj_seg;
    int *adj_first, *adj_tiles_of;
    double *adj_partial;
    int shared_grad;     // dtheta is one gradient of parameters shared by all instances
    double *grad_rows;   // per-instance rows summed into it (made on first use)
    int check_finite;    // rdcnn_batch_read checks the state for NaN / Inf
    int *finite_flag;    // device counter of that check (made on first use)
};

#define bfail(...) rd::set_error(__VA_ARGS__)

namespace {

void free_tables(rdcnn_batch *b)
{
    for (TileTable &t : b->tables)
        if (t.dev) (void)hipFree(t.dev);
    b->tables.clear();
    for (TileTable &t : b->rec_tables)
        if (t.dev) (void)hipFree(t.dev);
    b->rec_tables.clear();
}

void drop_graph(rdcnn_batch *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->graph_T = -1;
}

// Defaults from a sweep of the 1024-instance parameter-sweep workload on MI355X
// (two columns per lane, twelve steps per pass and 128-row tiles led).
void free_stats(rdcnn_batch *b)
{
    if (b->stat_chunks) (void)hipFree(b->stat_chunks);
    if (b->stat_first) (void)hipFree(b->stat_first);
    if (b->stat_partial) (void)hipFree(b->stat_partial);
    b->stat_chunks = nullptr;
    b->stat_first = nullptr;
    b->stat_partial = nullptr;
    b->stat_nchunks = 0;
}

int setup_stats(rdcnn_batch *b)
{
    std::vector<rd::StatChunk> ch;
    std::vector<int> first(b->n + 1);
    for (int i = 0; i < b->n; ++i) {
        first[i] = (int)ch.size();
        const long long cells = (long long)b->R[i] * b->C[i];
        for (long long s = 0; s < cells; s += rd::kStatChunk) {
            rd::StatChunk c;
            c.inst = i;
            c.start = (int)s;
            c.count = (int)(cells - s < rd::kStatChunk ? cells - s : rd::kStatChunk);
            ch.push_back(c);
        }
    }
    first[b->n] = (int)ch.size();
    if (ch.size() >= (1u << 31)) return bfail(RDCNN_EINVAL, "rdcnn_batch_stats: too many chunks");
    hipError_t e = hipMalloc((void **)&b->stat_chunks, sizeof(rd::StatChunk) * ch.size());
    if (e == hipSuccess) e = hipMalloc((void **)&b->stat_first, sizeof(int) * first.size());
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->stat_partial, sizeof(double) * rd::kStats * ch.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->stat_chunks, ch.data(), sizeof(rd::StatChunk) * ch.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->stat_first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_stats(b);
        return bfail(RDCNN_ENOMEM, "rdcnn_batch_stats: %s", hipGetErrorString(e));
    }
    b->stat_nchunks = (int)ch.size();
    return RDCNN_OK;
}

void free_lds(rdcnn_batch *b)
{
    if (b->lds_ids_dev) (void)hipFree(b->lds_ids_dev);
    b->lds_ids_dev = nullptr;
    b->lds_count = b->lds_frame = 0;
    b->in_lds.assign(b->n, 0);
}

// Decide which instances the in-LDS kernel takes and upload their indices.
int setup_lds(rdcnn_batch *b)
{
    free_lds(b);
    if (!b->use_lds) return RDCNN_OK;
    std::vector<int> ids;
    int frame = 0;
    for (int i = 0; i < b->n; ++i) {
        const int R = b->R[i], C = b->C[i];
        if (C > rd::kLdsThreads) continue;
        const int runs = rd::kLdsThreads / C;
        const int m = (R + runs - 1) / runs;
        const long long fr = (long long)(runs * m + 2) * (C + 2);  // frame incl. unstored rows
        if (m <= rd::kLdsRun && fr <= b->lds_limit) {
            b->in_lds[i] = 1;
            ids.push_back(i);
            if (fr > frame) frame = (int)fr;
        }
    }
    if (ids.empty()) return RDCNN_OK;
    hipError_t e = hipMalloc((void **)&b->lds_ids_dev, sizeof(int) * ids.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->lds_ids_dev, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_lds(b);
        return bfail(RDCNN_ENOMEM, "batch: in-LDS table: %s", hipGetErrorString(e));
    }
    b->lds_count = (int)ids.size();
    b->lds_frame = frame;
    return RDCNN_OK;
}

void batch_config(const rdcnn_batch *b, int *cpl, int *depth, int *seg)
{
    *cpl = b->cpl ? b->cpl : 2;
    *depth = b->depth ? b->depth : 12;
    *seg = b->seg_rows ? b->seg_rows : 128;
}

// Tile list for one pass depth: every instance (but those run in LDS, if
// skip_lds) cut into strips of wout output columns and segments of `seg` rows
// (with class_seg, an instance's own rows per tile where one was set for its
// size class), longest tiles first.
int build_tiles(const rdcnn_batch *b, int cpl, int depth, int seg, bool skip_lds,
                std::vector<rd::BatchTile> &tiles, bool class_seg = false)
{
    const int kpad = (depth + cpl - 1) / cpl * cpl;
    const int wout = 64 * cpl - 2 * kpad;
    if (wout <= 0) return bfail(RDCNN_EINVAL, "batch: depth %d too large for cpl %d", depth, cpl);
    tiles.clear();
    for (int i = 0; i < b->n; ++i) {
        if (skip_lds && b->in_lds[i]) continue;
        const int R = b->R[i], C = b->C[i];
        const int si = class_seg && b->seg_of[i] > 0 ? b->seg_of[i] : seg;
        const int h = si < R ? si : R;
        for (int sx = 0; sx * wout < C; ++sx)
            for (int y0 = 0; y0 < R; y0 += h) {
                rd::BatchTile t;
                t.inst = i;
                t.x0 = sx * wout - kpad;
                t.y0 = y0;
                t.y1 = y0 + h < R ? y0 + h : R;
                tiles.push_back(t);
            }
    }
    if (tiles.size() >= (1u << 31)) return bfail(RDCNN_EINVAL, "batch: too many tiles");
    std::stable_sort(tiles.begin(), tiles.end(), [](const rd::BatchTile &a, const rd::BatchTile &c) {
        return (a.y1 - a.y0) > (c.y1 - c.y0);
    });
    return RDCNN_OK;
}

// Upload a tile list into t (t.dev stays null for an empty list).
int upload_tiles(const std::vector<rd::BatchTile> &tiles, int depth, TileTable &t)
{
    t.depth = depth;
    t.ntiles = (int)tiles.size();
    t.dev = nullptr;
    if (tiles.empty()) return RDCNN_OK;
    hipError_t e = hipMalloc((void **)&t.dev, sizeof(rd::BatchTile) * tiles.size());
    if (e != hipSuccess) return bfail(RDCNN_ENOMEM, "batch: tile table: %s", hipGetErrorString(e));
    e = hipMemcpy(t.dev, tiles.data(), sizeof(rd::BatchTile) * tiles.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t.dev);
        t.dev = nullptr;
        return bfail(RDCNN_EHIP, "batch: tile table upload: %s", hipGetErrorString(e));
    }
    return RDCNN_OK;
}

// The table of `depth` in a set (built on first use).
int table_in(rdcnn_batch *b, std::vector<TileTable> &set, int cpl, int depth, int seg,
             bool skip_lds, const TileTable **out, bool class_seg = false)
{
    for (const TileTable &t : set)
        if (t.depth == depth) {
            *out = &t;
            return RDCNN_OK;
        }
    std::vector<rd::BatchTile> tiles;
    int rc = build_tiles(b, cpl, depth, seg, skip_lds, tiles, class_seg);
    if (rc != RDCNN_OK) return rc;
    TileTable t;
    rc = upload_tiles(tiles, depth, t);
    if (rc != RDCNN_OK) return rc;
    set.push_back(t);
    *out = &set.back();
    return RDCNN_OK;
}

int table_for(rdcnn_batch *b, int cpl, int depth, int seg, const TileTable **out)
{
    return table_in(b, b->tables, cpl, depth, seg, true, out, true);
}

void free_adj(rdcnn_batch *b)
{
    if (b->adj_table.dev) (void)hipFree(b->adj_table.dev);
    if (b->adj_first) (void)hipFree(b->adj_first);
    if (b->adj_tiles_of) (void)hipFree(b->adj_tiles_of);
    if (b->adj_partial) (void)hipFree(b->adj_partial);
    b->adj_table = TileTable();
    b->adj_first = b->adj_tiles_of = nullptr;
    b->adj_partial = nullptr;
    if (b->grad_rows) (void)hipFree(b->grad_rows);
    b->grad_rows = nullptr;
}

// Fold the per-tile partials into the gradients: one row of 8 per instance
// added to dtheta, or with shared parameters the rows summed over instances
// in index order and added to dtheta[0 .. 8).
hipError_t finish_grads(rdcnn_batch *b, unsigned mask, double *dtheta)
{
    if (!b->shared_grad)
        return rd::launch_batch_adjoint_finish(b->adj_partial, b->adj_first, b->adj_tiles_of,
                                               b->insts_dev, b->n, mask, dtheta, b->stream);
    if (!b->grad_rows) {
        hipError_t e = hipMalloc((void **)&b->grad_rows, sizeof(double) * 8 * (size_t)b->n);
        if (e != hipSuccess) {
            b->grad_rows = nullptr;
            return e;
        }
    }
    hipError_t e = rd::launch_zero(b->grad_rows, 8LL * b->n, b->stream);
    if (e == hipSuccess)
        e = rd::launch_batch_adjoint_finish(b->adj_partial, b->adj_first, b->adj_tiles_of,
                                            b->insts_dev, b->n, mask, b->grad_rows, b->stream);
    if (e == hipSuccess) e = rd::launch_grad_row_sum(b->grad_rows, b->n, dtheta, b->stream);
    return e;
}

// The reverse pass's tile list (every instance, cut for adj_depth), its
// per-instance tile lists and the per-tile partial buffer.
int setup_adj(rdcnn_batch *b)
{
    free_adj(b);
    std::vector<rd::BatchTile> tiles;
    int rc = build_tiles(b, b->adj_cpl, b->adj_depth, b->adj_seg, false, tiles);
    if (rc != RDCNN_OK) return rc;
    std::vector<int> first(b->n + 1, 0), tiles_of(tiles.size());
    for (const rd::BatchTile &t : tiles) ++first[t.inst + 1];
    for (int i = 0; i < b->n; ++i) first[i + 1] += first[i];
    {
        std::vector<int> pos(first.begin(), first.end() - 1);
        for (int k = 0; k < (int)tiles.size(); ++k) tiles_of[pos[tiles[k].inst]++] = k;
    }
    rc = upload_tiles(tiles, b->adj_depth, b->adj_table);
    if (rc != RDCNN_OK) return rc;
    hipError_t e = hipMalloc((void **)&b->adj_first, sizeof(int) * first.size());
    if (e == hipSuccess) e = hipMalloc((void **)&b->adj_tiles_of, sizeof(int) * (tiles_of.size() + 1));
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->adj_partial, sizeof(double) * rd::kAdjSums * (tiles.size() + 1));
    if (e == hipSuccess)
        e = hipMemcpy(b->adj_first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tiles_of.empty())
        e = hipMemcpy(b->adj_tiles_of, tiles_of.data(), sizeof(int) * tiles_of.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_adj(b);
        return bfail(RDCNN_ENOMEM, "rdcnn_batch_adjoint: %s", hipGetErrorString(e));
    }
    return RDCNN_OK;
}

// Largest depth <= want whose passes keep one instance's span of recorded
// states (depth-1 packed strides plus its own state) within a 4 GiB buffer
// resource.
int state_depth_cap(const rdcnn_batch *b, int want)
{
    long long maxrc = 0;
    for (int i = 0; i < b->n; ++i)
        if ((long long)b->R[i] * b->C[i] > maxrc) maxrc = (long long)b->R[i] * b->C[i];
    int k = want;
    while (k > 1 && (long long)(k - 1) * b->total * 4 + 8 * maxrc > 0xFFFFFFFFLL) --k;
    if ((long long)8 * maxrc > 0xFFFFFFFFLL || b->total * 4 > 0xFFFFFFFFLL) return 0;
    return k;
}

// Enqueue the launches of T steps; cur flips once per streamed launch.  The
// in-LDS instances go first, in one launch, and write their final state to the
// buffer that will be current after the T steps.
int enqueue_steps(rdcnn_batch *b, long long T, int cpl, int depth)
{
    if (b->lds_count > 0 && T > 0) {
        const long long passes = (T + depth - 1) / depth;
        const int after = (passes % 2) ? 1 - b->cur : b->cur;
        hipError_t e = rd::launch_batch_lds(b->insts_dev, b->lds_ids_dev, b->lds_count,
                                            b->lds_frame, b->buf[b->cur], b->buf[after], b->bc,
                                            T, b->stream);
        if (e != hipSuccess) return bfail(RDCNN_EHIP, "batch: in-LDS launch: %s", hipGetErrorString(e));
    }
    while (T > 0) {
        const int k = (int)(T < depth ? T : depth);
        const TileTable *t = nullptr;
        for (const TileTable &x : b->tables)
            if (x.depth == k) t = &x;
        if (!t) return bfail(RDCNN_ESTATE, "batch: missing tile table for depth %d", k);
        if (t->ntiles > 0) {
            hipError_t e = rd::launch_batch(t->dev, b->insts_dev, t->ntiles, b->buf[b->cur],
                                            b->buf[1 - b->cur], b->bc, cpl, k, b->stream);
            if (e != hipSuccess) return bfail(RDCNN_EHIP, "batch: launch: %s", hipGetErrorString(e));
        }
        b->cur = 1 - b->cur;
        T -= k;
    }
    return RDCNN_OK;
}

bool finite_gene(const rdcnn_params_t &p)
{
    const float v[8] = {p.dt, p.a, p.b, p.eps, p.c, p.k3, p.Du, p.Dv};
    for (float x : v)
        if (!isfinite(x)) return false;
    return true;
}

}  // namespace

extern "C" {

int rdcnn_batch_create(rdcnn_batch_t *out, int n, const int *rows, const int *cols,
                       const long long *offsets, const rdcnn_params_t *params, int bc,
                       const float *x_dev, const long long *x_offsets, float ka, float *buf0_dev,
                       float *buf1_dev, long long buf_floats, void *stream)
{
    if (!out) return bfail(RDCNN_EINVAL, "rdcnn_batch_create: out is NULL");
    *out = nullptr;
    if (n < 1 || !rows || !cols || !offsets || !params || !x_dev || !x_offsets || !buf0_dev ||
        !buf1_dev)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_create: NULL argument or n < 1");
    if (bc != RDCNN_BC_PERIODIC && bc != RDCNN_BC_ZEROFLUX)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_create: unknown boundary rule %d", bc);
    if (buf0_dev == buf1_dev) return bfail(RDCNN_EINVAL, "rdcnn_batch_create: buffers alias");
    if (!isfinite(ka)) return bfail(RDCNN_EINVAL, "rdcnn_batch_create: non-finite ka");
    // Instances must be aligned, inside the buffers and pairwise disjoint.
    std::vector<std::pair<long long, long long>> span(n);
    for (int i = 0; i < n; ++i) {
        if (rows[i] < 1 || cols[i] < 1 || (long long)rows[i] * cols[i] >= (1LL << 30))
            return bfail(RDCNN_EINVAL, "rdcnn_batch_create: instance %d has size %dx%d", i, rows[i],
                         cols[i]);
        if (offsets[i] < 0 || offsets[i] % 64 != 0)
            return bfail(RDCNN_EINVAL, "rdcnn_batch_create: offset of instance %d not a multiple "
                         "of 64 floats", i);
        const long long len = 2LL * rows[i] * cols[i];
        if (offsets[i] + len > buf_floats)
            return bfail(RDCNN_EINVAL, "rdcnn_batch_create: instance %d runs past the buffer", i);
        if (x_offsets[i] < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_create: bad x offset %d", i);
        if (!finite_gene(params[i]))
            return bfail(RDCNN_EINVAL, "rdcnn_batch_create: non-finite parameter (instance %d)", i);
        span[i] = {offsets[i], offsets[i] + len};
    }
    std::sort(span.begin(), span.end());
    for (int i = 1; i < n; ++i)
        if (span[i].first < span[i - 1].second)
            return bfail(RDCNN_EINVAL, "rdcnn_batch_create: instances overlap");
    rdcnn_batch *b = new (std::nothrow) rdcnn_batch;
    if (!b) return bfail(RDCNN_ENOMEM, "rdcnn_batch_create: out of host memory");
    b->n = n;
    b->bc = bc;
    b->R.assign(rows, rows + n);
    b->C.assign(cols, cols + n);
    b->seg_of.assign(n, 0);
    b->off.assign(offsets, offsets + n);
    b->g.resize(n);
    std::vector<rd::BatchInst> inst(n);
    for (int i = 0; i < n; ++i) {
        const rdcnn_params_t &p = params[i];
        rd::Gene g{p.dt, p.a, p.b, p.eps, p.c, p.k3, p.Du, p.Dv};
        b->g[i] = g;
        inst[i].off = offsets[i];
        inst[i].R = rows[i];
        inst[i].C = cols[i];
        inst[i].g = g;
    }
    b->buf[0] = buf0_dev;
    b->buf[1] = buf1_dev;
    b->cur = 0;
    b->stream = (hipStream_t)stream;
    b->cpl = b->depth = b->seg_rows = 0;
    b->insts_dev = nullptr;
    b->use_graph = 0;
    b->graph = nullptr;
    b->graph_T = -1;
    b->graph_cur = b->graph_cpl = b->graph_depth = b->graph_seg = 0;
    b->stat_chunks = nullptr;
    b->stat_first = nullptr;
    b->stat_partial = nullptr;
    b->stat_nchunks = 0;
    b->total = buf_floats;
    b->rec_cpl = 2;
    b->adj_table = TileTable();
    // reverse-pass defaults from a sweep of 64 x 1024^2 on MI355X
    b->adj_cpl = 1;
    b->adj_depth = 8;
    b->adj_seg = 128;
    b->adj_first = b->adj_tiles_of = nullptr;
    b->adj_partial = nullptr;
    b->shared_grad = 0;
    b->grad_rows = nullptr;
    b->check_finite = 0;
    b->finite_flag = nullptr;
    b->use_lds = 1;
    b->lds_ids_dev = nullptr;
    b->lds_count = b->lds_frame = 0;
    b->in_lds.assign(n, 0);
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            b->lds_limit = lds / (int)sizeof(float2);
        else
            b->lds_limit = 0;
    }
    hipError_t e = hipMalloc((void **)&b->insts_dev, sizeof(rd::BatchInst) * n);
    if (e != hipSuccess) {
        delete b;
        return bfail(RDCNN_ENOMEM, "rdcnn_batch_create: instance table: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(b->insts_dev, inst.data(), sizeof(rd::BatchInst) * n, hipMemcpyHostToDevice);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = rd::launch_init(x_dev + x_offsets[i], ka, buf0_dev + offsets[i],
                            (long long)rows[i] * cols[i], b->stream);
    if (e != hipSuccess) {
        (void)hipFree(b->insts_dev);
        delete b;
        return bfail(RDCNN_EHIP, "rdcnn_batch_create: %s", hipGetErrorString(e));
    }
    int rc = setup_lds(b);
    if (rc != RDCNN_OK) {
        (void)hipFree(b->insts_dev);
        delete b;
        return rc;
    }
    *out = b;
    return RDCNN_OK;
}

int rdcnn_batch_write_state(rdcnn_batch_t b, const float *packed)
{
    if (!b || !packed) return bfail(RDCNN_EINVAL, "rdcnn_batch_write_state: NULL argument");
    hipError_t e = hipMemcpyAsync(b->buf[b->cur], packed, sizeof(float) * b->total,
                                  hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess)
        return bfail(RDCNN_EHIP, "rdcnn_batch_write_state: %s", hipGetErrorString(e));
    return RDCNN_OK;
}

namespace {

// Recording passes of T steps; with even, only the states of even times
// (s_{2i} to traj[i]).
int batch_record(rdcnn_batch *b, long long T, float *traj, bool even, const char *who)
{
    if (!b) return bfail(RDCNN_EINVAL, "%s: NULL handle", who);
    if (T < 0) return bfail(RDCNN_EINVAL, "%s: T = %lld < 0", who, T);
    if (T == 0) return RDCNN_OK;
    if (!traj) return bfail(RDCNN_EINVAL, "%s: NULL trajectory", who);
    {
        // the recorded states (and, for even recording, the passes' inputs)
        // must not overlap the batch's state buffers
        const long long n = even ? (T + 1) / 2 : T;
        const char *t0 = (const char *)traj, *t1 = t0 + sizeof(float) * b->total * n;
        for (float *p : b->buf) {
            const char *b0 = (const char *)p, *b1 = b0 + sizeof(float) * b->total;
            if (t0 < b1 && b0 < t1)
                return bfail(RDCNN_EINVAL, "%s: trajectory overlaps a state buffer of the batch",
                             who);
        }
    }
    int cpl, depth, seg;
    batch_config(b, &cpl, &depth, &seg);
    if (cpl > 2) cpl = 2;  // recording passes exist for 1 or 2 columns per lane
    if (depth > 8) depth = 8;
    // Recording waits on its stores more than on arithmetic: shorter tiles
    // led sweeps on 64 x 1024^2 (full: 64 rows; even-time: 32 rows, 0.57
    // Tcell-steps/s against 0.50 at 64).
    if (!b->seg_rows) seg = even ? 32 : 64;
    if (even) {
        // a pass spans depth/2 recorded states; every pass but the last starts
        // at an even time, so the depth is even
        const int cap = state_depth_cap(b, 4);
        if (depth > 2 * cap) depth = 2 * cap;
        if (depth > 1) depth &= ~1;
    } else {
        depth = state_depth_cap(b, depth);
    }
    if (depth < 1) return bfail(RDCNN_EINVAL, "%s: packed state too large to record", who);
    if (cpl != b->rec_cpl) {
        for (TileTable &t : b->rec_tables)
            if (t.dev) (void)hipFree(t.dev);
        b->rec_tables.clear();
        b->rec_cpl = cpl;
    }
    long long q = 0;
    if (even && depth >= 2) {
        // As for a single grid: every pass but the last writes its output into
        // the trajectory slot of the even time it ends at, and the next pass
        // reads it there and records from level 2 on (each recorded state is
        // written once); the last pass writes the batch's other buffer.
        const float *in = b->buf[b->cur];
        while (T > 0) {
            const int k = (int)(T < depth ? T : depth);
            const TileTable *t = nullptr;
            int rc = table_in(b, b->rec_tables, cpl, k, seg, false, &t);
            if (rc != RDCNN_OK) return rc;
            float *out = T == k ? b->buf[1 - b->cur] : traj + (q + k) / 2 * b->total;
            hipError_t e = rd::launch_batch(t->dev, b->insts_dev, t->ntiles, in, out, b->bc, cpl,
                                            k, b->stream, traj + q / 2 * b->total,
                                            (unsigned)(4 * b->total), true, q > 0);
            if (e != hipSuccess) return bfail(RDCNN_EHIP, "%s: %s", who, hipGetErrorString(e));
            in = out;
            q += k;
            T -= k;
        }
        b->cur = 1 - b->cur;
        return RDCNN_OK;
    }
    while (T > 0) {
        const int k = (int)(T < depth ? T : depth);
        const TileTable *t = nullptr;
        int rc = table_in(b, b->rec_tables, cpl, k, seg, false, &t);
        if (rc != RDCNN_OK) return rc;
        hipError_t e;
        if (even && q % 2 == 1)  // depth-1 passes: odd times are not kept
            e = rd::launch_batch(t->dev, b->insts_dev, t->ntiles, b->buf[b->cur],
                                 b->buf[1 - b->cur], b->bc, cpl, k, b->stream);
        else
            e = rd::launch_batch(t->dev, b->insts_dev, t->ntiles, b->buf[b->cur],
                                 b->buf[1 - b->cur], b->bc, cpl, k, b->stream,
                                 traj + (even ? q / 2 : q) * b->total, (unsigned)(4 * b->total),
                                 even);
        if (e != hipSuccess) return bfail(RDCNN_EHIP, "%s: %s", who, hipGetErrorString(e));
        b->cur = 1 - b->cur;
        q += k;
        T -= k;
    }
    return RDCNN_OK;
}

}  // namespace

int rdcnn_batch_step_record(rdcnn_batch_t b, long long T, float *traj)
{
    return batch_record(b, T, traj, false, "rdcnn_batch_step_record");
}

int rdcnn_batch_step_record_even(rdcnn_batch_t b, long long T, float *traj)
{
    return batch_record(b, T, traj, true, "rdcnn_batch_step_record_even");
}

int rdcnn_batch_set_adjoint_kernel(rdcnn_batch_t b, int depth, int cols_per_lane, int seg_rows)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_adjoint_kernel: NULL handle");
    if (depth == 0) depth = 8;
    if (cols_per_lane == 0) cols_per_lane = 1;
    if (seg_rows == 0) seg_rows = 128;
    if (depth != 1 && depth != 2 && depth != 4 && depth != 8)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_set_adjoint_kernel: depth %d not in {1,2,4,8}", depth);
    if (cols_per_lane != 1 && cols_per_lane != 2)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_set_adjoint_kernel: cols_per_lane %d not in {1,2}",
                     cols_per_lane);
    if (seg_rows < 1) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_adjoint_kernel: seg_rows < 1");
    free_adj(b);
    b->adj_depth = depth;
    b->adj_cpl = cols_per_lane;
    b->adj_seg = seg_rows;
    return RDCNN_OK;
}

int rdcnn_batch_adjoint(rdcnn_batch_t b, const float *traj, long long S, float *adj,
                        float *adj_tmp, unsigned mask, double *dtheta)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint: NULL handle");
    if (S < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint: S = %lld < 0", S);
    if (!adj || !adj_tmp || !dtheta || (S > 0 && !traj))
        return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint: NULL buffer");
    if (adj == adj_tmp) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint: adj and adj_tmp alias");
    // deepest pass whose states fit one buffer resource (the tile list is cut
    // for adj_depth; shallower passes reuse it)
    int kmax = b->adj_depth;
    const int cap = state_depth_cap(b, kmax);
    if (cap < 1) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint: packed state too large");
    while (kmax > cap) kmax >>= 1;
    if (!b->adj_partial) {
        const int rc = setup_adj(b);
        if (rc != RDCNN_OK) return rc;
    }
    const int ntiles = b->adj_table.ntiles;
    hipError_t e = rd::launch_zero(b->adj_partial, (long long)rd::kAdjSums * (ntiles + 1), b->stream);
    const bool lam_sums = (mask & ((1u << 0) | (1u << 4) | (1u << 5))) != 0;
    float *src = adj, *dst = adj_tmp;
    long long top = S - 1;  // state the next reverse step steps back over
    while (e == hipSuccess && top >= 0 && ntiles > 0) {
        int k = kmax;
        while (k > 1 && k > top + 1) k >>= 1;
        e = rd::launch_batch_adjoint(b->adj_table.dev, b->insts_dev, ntiles, src, dst,
                                     traj + (top - k + 1) * b->total, (unsigned)(4 * b->total),
                                     b->bc, b->adj_cpl, k, b->adj_depth, b->adj_partial, lam_sums,
                                     b->stream);
        float *x = src;
        src = dst;
        dst = x;
        top -= k;
    }
    if (e == hipSuccess && src != adj)
        e = hipMemcpyAsync(adj, src, sizeof(float) * b->total, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = finish_grads(b, mask, dtheta);
    if (e != hipSuccess) return bfail(RDCNN_EHIP, "rdcnn_batch_adjoint: %s", hipGetErrorString(e));
    return RDCNN_OK;
}

int rdcnn_batch_adjoint_even(rdcnn_batch_t b, const float *traj, long long S, float *adj,
                             float *adj_tmp, unsigned mask, double *dtheta)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: NULL handle");
    if (S < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: S = %lld < 0", S);
    if (!adj || !adj_tmp || !dtheta || (S > 0 && !traj))
        return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: NULL buffer");
    if (adj == adj_tmp)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: adj and adj_tmp alias");
    if (b->adj_depth < 2)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: paired passes need an adjoint "
                     "depth of 2, 4 or 8 (rdcnn_batch_set_adjoint_kernel)");
    // deepest paired pass whose depth/2 even states fit one buffer resource
    int kmax = b->adj_depth;
    const int cap = state_depth_cap(b, kmax / 2);
    if (cap < 1) return bfail(RDCNN_EINVAL, "rdcnn_batch_adjoint_even: packed state too large");
    while (kmax > 2 && kmax / 2 > cap) kmax >>= 1;
    if (!b->adj_partial) {
        const int rc = setup_adj(b);
        if (rc != RDCNN_OK) return rc;
    }
    const int ntiles = b->adj_table.ntiles;
    hipError_t e = rd::launch_zero(b->adj_partial, (long long)rd::kAdjSums * (ntiles + 1), b->stream);
    const bool lam_sums = (mask & ((1u << 0) | (1u << 4) | (1u << 5))) != 0;
    float *src = adj, *dst = adj_tmp;
    auto flip = [&]() {
        float *x = src;
        src = dst;
        dst = x;
    };
    if (e == hipSuccess && (S & 1) && ntiles > 0) {  // the top step alone: s_{S-1} is even
        e = rd::launch_batch_adjoint(b->adj_table.dev, b->insts_dev, ntiles, src, dst,
                                     traj + (S - 1) / 2 * b->total, (unsigned)(4 * b->total),
                                     b->bc, b->adj_cpl, 1, b->adj_depth, b->adj_partial, lam_sums,
                                     b->stream);
        flip();
    }
    long long top = S & ~1LL;  // even time the next paired pass starts from
    while (e == hipSuccess && top > 0 && ntiles > 0) {
        int k = kmax;
        while (k > 2 && k > top) k >>= 1;
        e = rd::launch_batch_adjoint(b->adj_table.dev, b->insts_dev, ntiles, src, dst,
                                     traj + (top - k) / 2 * b->total, (unsigned)(4 * b->total),
                                     b->bc, b->adj_cpl, k, b->adj_depth, b->adj_partial, lam_sums,
                                     b->stream, true);
        flip();
        top -= k;
    }
    if (e == hipSuccess && src != adj)
        e = hipMemcpyAsync(adj, src, sizeof(float) * b->total, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = finish_grads(b, mask, dtheta);
    if (e != hipSuccess)
        return bfail(RDCNN_EHIP, "rdcnn_batch_adjoint_even: %s", hipGetErrorString(e));
    return RDCNN_OK;
}

int rdcnn_batch_stats(rdcnn_batch_t b, const float *prev, const float *ref, float theta_far,
                      float theta_move, double *out)
{
    if (!b || !out) return bfail(RDCNN_EINVAL, "rdcnn_batch_stats: NULL argument");
    if (!(theta_far >= 0.0f) || !(theta_move >= 0.0f) || !isfinite(theta_far) ||
        !isfinite(theta_move))
        return bfail(RDCNN_EINVAL, "rdcnn_batch_stats: thresholds must be finite and >= 0");
    if ((uintptr_t)prev % 16 != 0)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_stats: prev must be 16-byte aligned");
    if (!b->stat_chunks) {
        const int rc = setup_stats(b);
        if (rc != RDCNN_OK) return rc;
    }
    hipError_t e = rd::launch_stats(b->insts_dev, b->stat_chunks, b->stat_nchunks, b->stat_first,
                                    b->n, b->buf[b->cur], prev, ref, theta_far, theta_move,
                                    b->stat_partial, out, b->stream);
    if (e != hipSuccess) return bfail(RDCNN_EHIP, "rdcnn_batch_stats: %s", hipGetErrorString(e));
    return RDCNN_OK;
}

int rdcnn_batch_lds_instances(rdcnn_batch_t b, int *count)
{
    if (!b || !count) return bfail(RDCNN_EINVAL, "rdcnn_batch_lds_instances: NULL argument");
    *count = b->lds_count;
    return RDCNN_OK;
}

int rdcnn_batch_use_lds(rdcnn_batch_t b, int on)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_use_lds: NULL handle");
    b->use_lds = on ? 1 : 0;
    free_tables(b);
    drop_graph(b);
    return setup_lds(b);
}

int rdcnn_batch_set_kernel(rdcnn_batch_t b, int depth, int cols_per_lane, int seg_rows)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_kernel: NULL handle");
    if (depth == 0 && cols_per_lane == 0 && seg_rows == 0) {
        b->cpl = b->depth = b->seg_rows = 0;
    } else {
        if (cols_per_lane != 1 && cols_per_lane != 2 && cols_per_lane != 4)
            return bfail(RDCNN_EINVAL, "rdcnn_batch_set_kernel: cols_per_lane %d", cols_per_lane);
        if (depth < 1 || depth > rd::max_depth(cols_per_lane))
            return bfail(RDCNN_EINVAL, "rdcnn_batch_set_kernel: depth %d", depth);
        if (seg_rows < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_kernel: seg_rows < 0");
        b->cpl = cols_per_lane;
        b->depth = depth;
        b->seg_rows = seg_rows;
    }
    free_tables(b);
    drop_graph(b);
    return RDCNN_OK;
}

int rdcnn_batch_set_class_seg_rows(rdcnn_batch_t b, int rows, int cols, int seg_rows)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_class_seg_rows: NULL handle");
    if (seg_rows < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_class_seg_rows: seg_rows < 0");
    int hits = 0;
    for (int i = 0; i < b->n; ++i)
        if (b->R[i] == rows && b->C[i] == cols) {
            b->seg_of[i] = seg_rows;
            ++hits;
        }
    if (!hits)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_set_class_seg_rows: no instance of size %dx%d",
                     rows, cols);
    free_tables(b);
    drop_graph(b);
    return RDCNN_OK;
}

int rdcnn_batch_use_graph(rdcnn_batch_t b, int on)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_use_graph: NULL handle");
    b->use_graph = on ? 1 : 0;
    if (!on) drop_graph(b);
    return RDCNN_OK;
}

int rdcnn_batch_step(rdcnn_batch_t b, long long T)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_step: NULL handle");
    if (T < 0) return bfail(RDCNN_EINVAL, "rdcnn_batch_step: T < 0");
    if (T == 0) return RDCNN_OK;
    int cpl, depth, seg;
    batch_config(b, &cpl, &depth, &seg);
    const TileTable *t;
    int rc = table_for(b, cpl, depth, seg, &t);
    if (rc == RDCNN_OK && T % depth) rc = table_for(b, cpl, (int)(T % depth), seg, &t);
    if (rc != RDCNN_OK) return rc;
    const long long passes = (T + depth - 1) / depth;
    if (!b->use_graph) return enqueue_steps(b, T, cpl, depth);
    if (!b->stream) return bfail(RDCNN_EINVAL, "batch: graph capture needs a non-default stream");
    if (!(b->graph && b->graph_T == T && b->graph_cur == b->cur && b->graph_cpl == cpl &&
          b->graph_depth == depth && b->graph_seg == seg)) {
        drop_graph(b);
        const int cur0 = b->cur;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return bfail(RDCNN_EHIP, "batch: begin capture: %s", hipGetErrorString(e));
        rc = enqueue_steps(b, T, cpl, depth);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->stream, &g);
        b->cur = cur0;
        if (rc != RDCNN_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return bfail(RDCNN_EHIP, "batch: end capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->graph = nullptr;
            return bfail(RDCNN_EHIP, "batch: instantiate: %s", hipGetErrorString(e));
        }
        b->graph_T = T;
        b->graph_cur = cur0;
        b->graph_cpl = cpl;
        b->graph_depth = depth;
        b->graph_seg = seg;
    }
    hipError_t e = hipGraphLaunch(b->graph, b->stream);
    if (e != hipSuccess) return bfail(RDCNN_EHIP, "batch: graph launch: %s", hipGetErrorString(e));
    if (passes % 2) b->cur = 1 - b->cur;
    return RDCNN_OK;
}

int rdcnn_batch_current(rdcnn_batch_t b, float **state_dev)
{
    if (!b || !state_dev) return bfail(RDCNN_EINVAL, "rdcnn_batch_current: NULL argument");
    *state_dev = b->buf[b->cur];
    return RDCNN_OK;
}

int rdcnn_batch_read(rdcnn_batch_t b, float *dst_packed_dev)
{
    if (!b || !dst_packed_dev) return bfail(RDCNN_EINVAL, "rdcnn_batch_read: NULL argument");
    const float *src = b->buf[b->cur];
    const char *d0 = (const char *)dst_packed_dev, *s0 = (const char *)src;
    const size_t bytes = sizeof(float) * (size_t)b->total;
    if (d0 < s0 + bytes && s0 < d0 + bytes)
        return bfail(RDCNN_EINVAL, "rdcnn_batch_read: destination overlaps the current state");
    hipError_t e = hipMemcpyAsync(dst_packed_dev, src, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bfail(RDCNN_EHIP, "rdcnn_batch_read: %s", hipGetErrorString(e));
    if (b->check_finite) {
        // only the instances' cells: padding between them is not state
        for (int i = 0; i < b->n; ++i) {
            const int rc = rd::check_finite_state(src + b->off[i], 2LL * b->R[i] * b->C[i],
                                                  &b->finite_flag, b->stream, "rdcnn_batch_read");
            if (rc != RDCNN_OK) return rc;
        }
    }
    return RDCNN_OK;
}

int rdcnn_batch_set_check_finite(rdcnn_batch_t b, int on)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_check_finite: NULL handle");
    b->check_finite = on != 0;
    return RDCNN_OK;
}

int rdcnn_batch_set_shared_grad(rdcnn_batch_t b, int on)
{
    if (!b) return bfail(RDCNN_EINVAL, "rdcnn_batch_set_shared_grad: NULL handle");
    b->shared_grad = on != 0;
    return RDCNN_OK;
}

int rdcnn_batch_destroy(rdcnn_batch_t b)
{
    if (!b) return RDCNN_OK;
    drop_graph(b);
    free_tables(b);
    free_lds(b);
    free_stats(b);
    free_adj(b);
    if (b->finite_flag) (void)hipFree(b->finite_flag);
    if (b->insts_dev) (void)hipFree(b->insts_dev);
    delete b;
    return RDCNN_OK;
}

}  // extern "C"
