// rd_api.hip -- C ABI of the RD-CNN library (declared in include/rdcnn.h).
//
// Host-side bookkeeping only: argument checks, the ping-pong state buffers, the
// choice of kernel and pass depth, the adjoint's partial-sum workspace, and error
// reporting.  All arithmetic of the method runs in the kernels of rd_forward.hip
// and rd_adjoint.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "rd_launch.h"
#include "rdcnn.h"

struct rdcnn_sim {
    int R, C, bc;
    rd::Gene g;
    float *buf[2];
    int cur;  // index of the buffer holding the current state
    hipStream_t stream;
    int kind;  // 0 automatic, 1 naive, 2 streamed
    int depth, cpl, seg_rows;
    int adj_depth, adj_cpl, adj_seg_rows;  // 0: automatic
    unsigned grad_mask;                    // gradients rdcnn_adjoint forms (bit q: param q)
    double *partial;                       // adjoint per-tile partial sums (pooled)
    long long partial_cap;                 // tiles it can hold
    int partial_device;                    // device it lives on
    int model;                             // rd::MODEL_*; g holds the FHN gene
    float mparams[rd::kModelParams];       // parameters of the other models
    int check_finite;                      // rdcnn_read checks the state for NaN / Inf
    int *finite_flag;                      // device counter of that check (made on first use)
    hipStream_t side;                      // rdcnn_step_bwd_ckpt's recompute stream (the device's, see side_stream)
    hipEvent_t ev[5];                      // its events: ready[2], done[2], start
    int use_graph;                         // rdcnn_step replays captured launch sequences
    struct StepGraph {
        hipGraphExec_t exec;  // null: empty entry
        long long T;          // steps it runs
        int cur0, cur1;       // buffer holding the state before / after
    } graph[2];               // one per starting buffer
};

namespace {
thread_local char g_err[512];
}

int rd::set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define fail(...) rd::set_error(__VA_ARGS__)

namespace {

int hip_fail(hipError_t e, const char *what)
{
    return fail(RDCNN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// The adjoint's per-tile partial sums (a few hundred KB) come from a
// process-wide pool: a handle returns its buffer on destroy instead of freeing
// it, so short-lived handles (one per autograd call) allocate nothing after the
// first and never call hipFree, which would wait for the whole device.  A
// returned buffer carries an event recorded on its last user's stream; the
// next user's stream waits for it, so work still queued on the old stream
// finishes with the buffer first.  Pooled buffers stay allocated until the
// process ends.
struct PooledPartial {
    int device;
    long long cap;      // tiles
    double *p;
    hipEvent_t ready;   // the last user's work on it is done (null: nothing queued)
};
std::mutex g_pool_mu;
std::vector<PooledPartial> g_pool;
constexpr size_t kPoolMax = 16;

void release_entry(PooledPartial &x)
{
    (void)hipFree(x.p);  // waits for the device, so also for x.ready
    if (x.ready) (void)hipEventDestroy(x.ready);
}

void pool_put(int device, long long cap, double *p, hipStream_t last_user)
{
    if (!p) return;
    PooledPartial x{device, cap, p, nullptr};
    if (hipEventCreateWithFlags(&x.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(x.ready, last_user) != hipSuccess) {
        if (x.ready) (void)hipEventDestroy(x.ready);
        x.ready = nullptr;
        (void)hipStreamSynchronize(last_user);
    }
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (g_pool.size() >= kPoolMax) {  // keep the larger buffers
        size_t k = 0;
        for (size_t i = 1; i < g_pool.size(); ++i)
            if (g_pool[i].cap < g_pool[k].cap) k = i;
        if (g_pool[k].cap >= cap) {
            release_entry(x);
            return;
        }
        release_entry(g_pool[k]);
        g_pool.erase(g_pool.begin() + (long)k);
    }
    g_pool.push_back(x);
}

// Make h->partial hold at least `need` tiles on the current device.
int ensure_partial(rdcnn_sim *h, long long need, const char *who)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (h->partial && h->partial_cap >= need && h->partial_device == dev) return RDCNN_OK;
    pool_put(h->partial_device, h->partial_cap, h->partial, h->stream);
    h->partial = nullptr;
    h->partial_cap = 0;
    hipEvent_t ready = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_pool_mu);
        long long best = -1;
        for (size_t i = 0; i < g_pool.size(); ++i)
            if (g_pool[i].device == dev && g_pool[i].cap >= need &&
                (best < 0 || g_pool[i].cap < g_pool[(size_t)best].cap))
                best = (long long)i;
        if (best >= 0) {
            h->partial = g_pool[(size_t)best].p;
            h->partial_cap = g_pool[(size_t)best].cap;
            ready = g_pool[(size_t)best].ready;
            g_pool.erase(g_pool.begin() + best);
        }
    }
    if (ready) {  // queued after the previous user's work on the buffer
        e = hipStreamWaitEvent(h->stream, ready, 0);
        (void)hipEventDestroy(ready);
        if (e != hipSuccess) return hip_fail(e, who);
    }
    if (!h->partial) {
        e = hipMalloc((void **)&h->partial, sizeof(double) * rd::kAdjSums * need);
        if (e != hipSuccess) {
            h->partial = nullptr;
            return fail(RDCNN_ENOMEM, "%s: partial buffer: %s", who, hipGetErrorString(e));
        }
        h->partial_cap = need;
    }
    h->partial_device = dev;
    return RDCNN_OK;
}

}  // namespace

// Partial-sum workspace of rdcnn_step_bwd_noalloc: a fixed device array in
// place of the pooled buffer, for callers that cannot allocate (HIP graph
// capture, serving loops).  kNoAllocTiles tiles of kAdjSums doubles (4 MiB);
// each device the library runs on holds its own copy until the process ends.
// Host code never names the array itself (on the host its name is only a
// stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, resolved once per device below.
constexpr long long kNoAllocTiles = 65536;
static __device__ __align__(256) double scratch[rd::kAdjSums * kNoAllocTiles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices];  // scratch's address on each device (null: not resolved yet)

// The address of `scratch` on the current device, resolved on the first call
// for that device (rdcnn_create makes that call, so a handle's device is
// resolved before any of its work can be captured).
int scratch_address(double **out, const char *who)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RDCNN_EINVAL, "%s: device %d beyond the %d the workspace table holds", who, dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RDCNN_EHIP, "%s: address of the static workspace: %s", who,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return RDCNN_OK;
}

// The recompute stream of rdcnn_step_bwd_ckpt: one per device, made on first
// use and kept until the process ends.  Making a stream takes ~70 us of host
// time, which a handle per autograd call would otherwise pay in every
// backward.  Handles on a device share it; each orders its own recomputes with
// its own events, so one handle's recomputes only queue behind another's.
std::mutex g_side_mu;
hipStream_t g_side[kMaxDevices];

int side_stream(hipStream_t *out, const char *who)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RDCNN_EINVAL, "%s: device %d beyond the %d the stream table holds", who, dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_side_mu);
    if (!g_side[dev]) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, who);
        g_side[dev] = s;
    }
    *out = g_side[dev];
    return RDCNN_OK;
}

}  // namespace

int rd::check_finite_state(const float *x, long long n, int **flag, hipStream_t s, const char *who)
{
    if (!*flag) {
        hipError_t e = hipMalloc((void **)flag, 256);
        if (e != hipSuccess) {
            *flag = nullptr;
            return fail(RDCNN_ENOMEM, "%s: finite-check counter: %s", who, hipGetErrorString(e));
        }
    }
    int bad = 0;
    hipError_t e = rd::launch_count_nonfinite(x, n, *flag, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, *flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, who);
    if (bad) return fail(RDCNN_ENONFINITE, "%s: %d non-finite values in the state", who, bad);
    return RDCNN_OK;
}

namespace {

bool finite_params(const rdcnn_params_t *p)
{
    const float v[8] = {p->dt, p->a, p->b, p->eps, p->c, p->k3, p->Du, p->Dv};
    for (float x : v)
        if (!isfinite(x)) return false;
    return true;
}

rd::Gene to_gene(const rdcnn_params_t *p)
{
    rd::Gene g;
    g.dt = p->dt;
    g.a = p->a;
    g.b = p->b;
    g.eps = p->eps;
    g.c = p->c;
    g.k3 = p->k3;
    g.Du = p->Du;
    g.Dv = p->Dv;
    return g;
}

// The (lam, mu) planes of a chain of reverse passes: each pass reads one pair
// and writes the other; copy_back leaves the result in the first pair.
struct Pingpong {
    float *p[2][2];  // [pair][lam, mu]
    int cur = 0;
    Pingpong(float *l0, float *m0, float *l1, float *m1) : p{{l0, m0}, {l1, m1}} {}
    rd::AdjPlanes io() const { return {p[cur][0], p[cur][1], p[1 - cur][0], p[1 - cur][1]}; }
    void flip() { cur = 1 - cur; }
    hipError_t copy_back(size_t n, hipStream_t s)
    {
        if (cur == 0) return hipSuccess;
        hipError_t e = hipMemcpyAsync(p[0][0], p[1][0], sizeof(float) * n,
                                      hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p[0][1], p[1][1], sizeof(float) * n, hipMemcpyDeviceToDevice, s);
        cur = 0;
        return e;
    }
};

// Default pass settings for a grid when the caller has not forced any (from
// sweeps on MI355X: wide strips and deep passes pay off only on large grids;
// smaller grids are latency bound and want more, narrower wavefronts).
void auto_config(const rdcnn_sim *h, int *cpl, int *depth, int *seg_rows, bool record,
                 bool record_even = false)
{
    *seg_rows = 0;
    if (record && record_even) {
        // Even-state recording writes half as much; one column per lane and
        // segments for ~2816 wavefronts led a sweep on 1024^2 (10 % over the
        // full recording's shape).
        *cpl = 1;
        *depth = 8;
        const long long nstrips = (h->C + 47) / 48;
        long long want = 2816 / nstrips;
        if (want < 1) want = 1;
        long long seg = (h->R + want - 1) / want;
        *seg_rows = (int)(seg < 4 ? 4 : seg);
    } else if (record) {
        // Recording is bound by its stores; two columns per lane and segments
        // for ~2560 wavefronts led a sweep on 1024^2 (7 % over one column).
        *cpl = 2;
        *depth = 8;
        const long long nstrips = (h->C + 111) / 112;
        long long want = 2560 / nstrips;
        if (want < 1) want = 1;
        long long seg = (h->R + want - 1) / want;
        *seg_rows = (int)(seg < 4 ? 4 : seg);
    } else if (h->R >= 3072 && h->C >= 3072) {
        *cpl = 4;
        *depth = 8;
    } else if (h->R >= 2048 && h->C >= 2048) {
        // four columns per lane leave too few wavefronts below ~3072^2:
        // 992 against 802 Gcell-updates/s at 2048^2, 1150 against 1063 at 2560^2
        *cpl = 2;
        *depth = 8;
    } else {
        *cpl = 1;
        *depth = 8;
    }
}

// Steps of a model other than FitzHugh-Nagumo: passes of 8, 4, 2 or 1 steps
// (the instantiated depths), one step per pass at a zero-flux edge when the
// update is not mirror-exact for these parameters.
// Pass shape of a grid of another cell model: the forced settings, else 8
// steps per pass with 4 columns per lane from 3072^2 (models instantiated
// that wide), 2 from 2048^2, 1 below; widths beyond the model's widest are
// narrowed to it.
void model_shape(const rdcnn_sim *h, int *cpl, int *depth, int *seg)
{
    const int wmax = rd::model_max_cpl(h->model);
    *cpl = h->cpl;
    *depth = h->depth;
    *seg = h->seg_rows;
    if (h->kind == 0) {
        *cpl = h->R >= 3072 && h->C >= 3072 ? 4 : h->R >= 2048 && h->C >= 2048 ? 2 : 1;
        *depth = 8;
        *seg = 0;
    }
    if (*cpl > wmax) *cpl = wmax;
}

int run_model_steps(rdcnn_sim *h, long long n)
{
    if (h->kind == 1) return fail(RDCNN_EINVAL, "rdcnn_step: the one-thread-per-cell kernel "
                                                "exists for FitzHugh-Nagumo only");
    int cpl, depth, seg;
    model_shape(h, &cpl, &depth, &seg);
    if (h->bc == RDCNN_BC_ZEROFLUX && !rd::model_mirror_exact(h->model, h->mparams)) depth = 1;
    while (n > 0) {
        int k = 8;
        while (k > 1 && (k > depth || k > n)) k >>= 1;
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, cpl, k, seg, &geom))
            return fail(RDCNN_EINVAL, "rdcnn_step: cannot tile %dx%d with cpl=%d depth=%d", h->R,
                        h->C, cpl, k);
        hipError_t e = rd::launch_model(h->model, h->buf[h->cur], h->buf[1 - h->cur], h->R, h->C,
                                        h->bc, h->mparams, geom, h->stream);
        if (e != hipSuccess) return hip_fail(e, "rdcnn_step: model kernel launch");
        h->cur = 1 - h->cur;
        n -= k;
    }
    return RDCNN_OK;
}

// Even-time recording of n steps from the state at `in` on stream s: passes
// of `depth` (even) steps; every pass but the last writes its output straight
// into the trajectory slot of the (even) time it ends at (s_{2i} at rec + 2i *
// every / 2 states, i.e. rec + i * every states), and the next pass reads its
// input from there and records from level 2 on, so each recorded state is
// written once.  No pass reads a slot it writes.  The last pass writes
// last_out.  The first pass records its input as s_0.
int record_even_chain(const rdcnn_sim *h, const float *in, long long n, float *rec, int every,
                      float *last_out, int cpl, int depth, int seg, hipStream_t s, const char *who)
{
    const size_t state = 2 * (size_t)h->R * h->C;
    long long q = 0;
    while (n > 0) {
        const int k = (int)(n < depth ? n : depth);
        float *out = n == k ? last_out : rec + (size_t)((q + k) / 2) * every * state;
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, cpl, k, seg, &geom))
            return fail(RDCNN_EINVAL, "%s: cannot tile %dx%d with cpl=%d depth=%d", who, h->R, h->C,
                        cpl, k);
        hipError_t e = rd::launch_stream(in, out, h->R, h->C, h->bc, h->g, geom, s, rec, q / 2, true,
                                         q > 0, every);
        if (e != hipSuccess) return hip_fail(e, who);
        in = out;
        n -= k;
        q += k;
    }
    return RDCNN_OK;
}

// Pass shape of an even-time recording run: the handle's forced streamed
// settings, else the automatic ones, made even (<= 8) with one or two columns
// per lane and cut so a pass's recorded states (`every` slots apart) fit one
// buffer resource.  Returns false if the grid is too large to record.
bool even_record_shape(const rdcnn_sim *h, int every, int *cpl, int *depth, int *seg)
{
    *cpl = h->cpl;
    *depth = h->depth;
    *seg = h->seg_rows;
    if (h->kind != 2) auto_config(h, cpl, depth, seg, true, true);
    const long long cap = ((1LL << 32) - 1) / (8LL * h->R * h->C);
    if (cap < 1) return false;
    if (*cpl > 2) *cpl = 2;
    if (*depth > 8) *depth = 8;
    const long long dmax = 2 * ((cap - 1) / every + 1);
    if (*depth > dmax) *depth = (int)dmax;
    if (*depth > 1) *depth &= ~1;
    return *depth >= 2;
}

// Run n steps from buf[cur]; flips cur once per pass.  If rec is not null the
// state each step starts from is also written to rec[0..n-1] (2*R*C floats
// each); with rec_even only the states of even times, s_{2i} to rec[i * every]
// (every = 1: a compact even-time trajectory; 2: the even slots of a
// trajectory with a slot per time).
int run_steps(rdcnn_sim *h, long long n, float *rec, bool rec_even = false, int every = 1)
{
    if (h->model != rd::MODEL_FHN) {
        if (rec) return fail(RDCNN_EINVAL, "rdcnn_step_record: FitzHugh-Nagumo grids only");
        return run_model_steps(h, n);
    }
    long long q = 0;
    int kind = h->kind, cpl = h->cpl, depth = h->depth, seg = h->seg_rows;
    if (kind == 3) kind = rec ? 0 : 2;  // forced shape for plain steps only
    if (kind == 0) {
        kind = 2;
        auto_config(h, &cpl, &depth, &seg, rec != nullptr, rec_even);
    }
    if (rec && kind == 2) {
        // A pass's recorded states are addressed through one 4 GiB buffer resource.
        const long long cap = ((1LL << 32) - 1) / (8LL * h->R * h->C);
        if (cap < 1)
            return fail(RDCNN_EINVAL, "rdcnn_step_record: grid too large to record");
        if (rec_even) {
            // Even-state recording: every pass but the last starts at an even
            // time, so passes of an even depth (<= 8; one or two columns per lane).
            // A pass spans its (depth-1)/2 further recorded states, `every`
            // slots apart, past the first.
            if (cpl > 2) cpl = 2;
            if (depth > 8) depth = 8;
            const long long dmax = 2 * ((cap - 1) / every + 1);
            if (depth > dmax) depth = (int)dmax;
            if (depth > 1) depth &= ~1;
        } else if (depth > cap) {
            depth = (int)cap;
        }
    }
    if (rec && rec_even && kind == 2 && depth >= 2 && n > 0) {
        const int rc = record_even_chain(h, h->buf[h->cur], n, rec, every, h->buf[1 - h->cur], cpl,
                                         depth, seg, h->stream, "rdcnn_step");
        if (rc != RDCNN_OK) return rc;
        h->cur = 1 - h->cur;
        return RDCNN_OK;
    }
    while (n > 0) {
        hipError_t e;
        const float *in = h->buf[h->cur];
        float *out = h->buf[1 - h->cur];
        long long done;
        if (kind == 1) {
            e = hipSuccess;
            if (rec && (!rec_even || q % 2 == 0))
                e = hipMemcpyAsync(rec + (rec_even ? q / 2 * every : q) * 2LL * h->R * h->C, in,
                                   sizeof(float) * 2 * h->R * h->C, hipMemcpyDeviceToDevice,
                                   h->stream);
            if (e == hipSuccess) e = rd::launch_naive(in, out, h->R, h->C, h->bc, h->g, h->stream);
            done = 1;
        } else {
            const int k = (int)(n < depth ? n : depth);
            rd::StreamGeom geom;
            if (!rd::stream_geometry(h->R, h->C, cpl, k, seg, &geom))
                return fail(RDCNN_EINVAL, "rdcnn_step: cannot tile %dx%d with cpl=%d depth=%d",
                            h->R, h->C, cpl, k);
            if (rec && rec_even && q % 2 == 1)  // depth-1 passes: odd times are not kept
                e = rd::launch_stream(in, out, h->R, h->C, h->bc, h->g, geom, h->stream);
            else
                e = rd::launch_stream(in, out, h->R, h->C, h->bc, h->g, geom, h->stream, rec,
                                      rec_even ? q / 2 : q, rec_even, false, every);
            done = k;
        }
        if (e != hipSuccess) return hip_fail(e, "rdcnn_step: kernel launch");
        h->cur = 1 - h->cur;
        n -= done;
        q += done;
    }
    return RDCNN_OK;
}

// Captured step sequences bake in the parameters and pass settings: drop them
// when either changes.
void drop_graphs(rdcnn_sim *h)
{
    for (auto &gr : h->graph) {
        if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
        gr.exec = nullptr;
    }
}

// rdcnn_step with graphs on: the launch sequence of T steps from buf[cur] is
// captured once (run_steps only launches kernels) and replayed after that.
int step_graph(rdcnn_sim *h, long long T)
{
    auto &gr = h->graph[h->cur];
    if (!(gr.exec && gr.T == T && gr.cur0 == h->cur)) {
        if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
        gr.exec = nullptr;
        const int cur0 = h->cur;
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(e, "rdcnn_step: begin capture");
        const int rc = run_steps(h, T, nullptr);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->stream, &g);
        const int cur1 = h->cur;
        h->cur = cur0;
        if (rc != RDCNN_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "rdcnn_step: end capture");
        e = hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            gr.exec = nullptr;
            return hip_fail(e, "rdcnn_step: graph instantiate");
        }
        gr.T = T;
        gr.cur0 = cur0;
        gr.cur1 = cur1;
    }
    hipError_t e = hipGraphLaunch(gr.exec, h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_step: graph launch");
    h->cur = gr.cur1;
    return RDCNN_OK;
}

// Gradients that need the lam-weighted sums: dt (bit 0), c (bit 4), k3 (bit 5).
constexpr unsigned kLamSumGrads = (1u << 0) | (1u << 4) | (1u << 5);

// Adjoint pass shape: one column per lane, four reverse steps, and segments
// short enough for about 4608 wavefronts (4.5 per SIMD).  The adjoint waits on
// memory more than the forward, so it gains from more resident wavefronts
// despite the extra halo rows (a sweep on 1024^2: 8 % over two columns per lane
// and ~2048 wavefronts).
void adj_auto_config(const rdcnn_sim *h, int *cpl, int *depth, int *seg_rows)
{
    *cpl = 1;
    *depth = 4;
    const long long nstrips = (h->C + (64 - 2 * 4) - 1) / (64 - 2 * 4);
    long long want = 4608 / nstrips;
    if (want < 1) want = 1;
    long long seg = (h->R + want - 1) / want;
    if (seg < 4) seg = 4;  // as the forward's automatic segments
    *seg_rows = (int)seg;
}

// Default shape of the paired reverse passes: three pairs per pass, one column
// per lane, and segments for ~2560 wavefronts led an interleaved sweep on
// 1024^2 (4 % over the plain reverse pass's shape of 4 steps and ~4608).
void adj_even_auto_config(const rdcnn_sim *h, int *cpl, int *depth, int *seg_rows)
{
    *cpl = 1;
    *depth = 6;
    const long long nstrips = (h->C + (64 - 2 * 6) - 1) / (64 - 2 * 6);
    long long want = 2560 / nstrips;
    if (want < 1) want = 1;
    long long seg = (h->R + want - 1) / want;
    if (seg < 4) seg = 4;
    *seg_rows = (int)seg;
}

int check_grid(const char *who, int rows, int cols, int bc, const float *buf0, const float *buf1)
{
    if (rows < 1 || cols < 1) return fail(RDCNN_EINVAL, "%s: grid %dx%d", who, rows, cols);
    if ((long long)rows * cols >= (1LL << 30))
        return fail(RDCNN_EINVAL, "%s: grid of %lld cells; at most 2^30-1 (one plane must stay "
                    "below 4 GiB)", who, (long long)rows * cols);
    if (bc != RDCNN_BC_PERIODIC && bc != RDCNN_BC_ZEROFLUX)
        return fail(RDCNN_EINVAL, "%s: unknown boundary rule %d", who, bc);
    if (!buf0 || !buf1) return fail(RDCNN_EINVAL, "%s: NULL device buffer", who);
    if (buf0 == buf1) return fail(RDCNN_EINVAL, "%s: the two state buffers alias", who);
    return RDCNN_OK;
}

rdcnn_sim *new_sim(int rows, int cols, int bc, float *buf0, float *buf1, void *stream)
{
    rdcnn_sim *h = new (std::nothrow) rdcnn_sim;
    if (!h) return nullptr;
    h->R = rows;
    h->C = cols;
    h->bc = bc;
    h->g = rd::Gene{};
    h->buf[0] = buf0;
    h->buf[1] = buf1;
    h->cur = 0;
    h->stream = (hipStream_t)stream;
    h->kind = 0;
    h->depth = 0;
    h->cpl = 0;
    h->seg_rows = 0;
    h->adj_depth = 0;
    h->adj_cpl = 0;
    h->adj_seg_rows = 0;
    h->grad_mask = 0xFFu;
    h->partial = nullptr;
    h->partial_cap = 0;
    h->partial_device = 0;
    h->model = rd::MODEL_FHN;
    for (float &x : h->mparams) x = 0.0f;
    h->check_finite = 0;
    h->finite_flag = nullptr;
    h->side = nullptr;
    for (hipEvent_t &e : h->ev) e = nullptr;
    h->use_graph = 0;
    for (auto &gr : h->graph) gr.exec = nullptr;
    return h;
}

}  // namespace

extern "C" {

const char *rdcnn_last_error(void) { return g_err; }

int rdcnn_create(rdcnn_t *out, int rows, int cols, int bc, const rdcnn_params_t *p,
                 const float *x_dev, float ka, float *buf0_dev, float *buf1_dev, void *stream)
{
    if (!out) return fail(RDCNN_EINVAL, "rdcnn_create: out is NULL");
    *out = nullptr;
    const int rc = check_grid("rdcnn_create", rows, cols, bc, buf0_dev, buf1_dev);
    if (rc != RDCNN_OK) return rc;
    if (!p || !finite_params(p)) return fail(RDCNN_EINVAL, "rdcnn_create: missing or non-finite parameters");
    if (!isfinite(ka)) return fail(RDCNN_EINVAL, "rdcnn_create: non-finite ka");
    if (!x_dev) return fail(RDCNN_EINVAL, "rdcnn_create: NULL device buffer");
    double *ws = nullptr;  // set-up of rdcnn_step_bwd_noalloc's workspace on this device
    const int rs = scratch_address(&ws, "rdcnn_create");
    if (rs != RDCNN_OK) return rs;
    rdcnn_sim *h = new_sim(rows, cols, bc, buf0_dev, buf1_dev, stream);
    if (!h) return fail(RDCNN_ENOMEM, "rdcnn_create: out of host memory");
    h->g = to_gene(p);
    hipError_t e = rd::launch_init(x_dev, ka, buf0_dev, (long long)rows * cols, h->stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "rdcnn_create: init launch");
    }
    *out = h;
    return RDCNN_OK;
}

int rdcnn_model_create(rdcnn_t *out, int model, int rows, int cols, int bc, const float *params,
                       int nparams, const float *u0_dev, const float *v0_dev, float *buf0_dev,
                       float *buf1_dev, void *stream)
{
    if (!out) return fail(RDCNN_EINVAL, "rdcnn_model_create: out is NULL");
    *out = nullptr;
    const int rc = check_grid("rdcnn_model_create", rows, cols, bc, buf0_dev, buf1_dev);
    if (rc != RDCNN_OK) return rc;
    const int want = rd::model_nparams(model);
    if (want < 0) return fail(RDCNN_EINVAL, "rdcnn_model_create: unknown model %d", model);
    if (nparams != want || !params)
        return fail(RDCNN_EINVAL, "rdcnn_model_create: model %d takes %d parameters, got %d",
                    model, want, nparams);
    for (int i = 0; i < nparams; ++i)
        if (!isfinite(params[i]))
            return fail(RDCNN_EINVAL, "rdcnn_model_create: parameter %d is not finite", i);
    if (!u0_dev || !v0_dev) return fail(RDCNN_EINVAL, "rdcnn_model_create: NULL initial state");
    rdcnn_sim *h = new_sim(rows, cols, bc, buf0_dev, buf1_dev, stream);
    if (!h) return fail(RDCNN_ENOMEM, "rdcnn_model_create: out of host memory");
    h->model = model;
    for (int i = 0; i < nparams; ++i) h->mparams[i] = params[i];
    if (model == rd::MODEL_FHN) {
        const rdcnn_params_t p{params[0], params[1], params[2], params[3],
                               params[4], params[5], params[6], params[7]};
        h->g = to_gene(&p);
    }
    const size_t n = (size_t)rows * cols;
    hipError_t e = hipMemcpyAsync(buf0_dev, u0_dev, sizeof(float) * n, hipMemcpyDeviceToDevice,
                                  h->stream);
    if (e == hipSuccess) {
        if (model == rd::MODEL_CNN)  // second layer: w = (B * image) + z
            e = rd::launch_cnn_input(v0_dev, params + 10, rows, cols, bc, buf0_dev + n, h->stream);
        else
            e = hipMemcpyAsync(buf0_dev + n, v0_dev, sizeof(float) * n, hipMemcpyDeviceToDevice,
                               h->stream);
    }
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "rdcnn_model_create: initial state");
    }
    *out = h;
    return RDCNN_OK;
}

int rdcnn_step(rdcnn_t h, long long T)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_step: NULL handle");
    if (T < 0) return fail(RDCNN_EINVAL, "rdcnn_step: T = %lld < 0", T);
    if (h->use_graph && T > 0) return step_graph(h, T);
    return run_steps(h, T, nullptr);
}

int rdcnn_use_graph(rdcnn_t h, int on)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_use_graph: NULL handle");
    if (on && !h->stream)
        return fail(RDCNN_EINVAL, "rdcnn_use_graph: graph capture needs a non-NULL stream");
    h->use_graph = on ? 1 : 0;
    if (!on) drop_graphs(h);
    return RDCNN_OK;
}

int rdcnn_step_record(rdcnn_t h, long long T, float *states_dev)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_step_record: NULL handle");
    if (T < 0) return fail(RDCNN_EINVAL, "rdcnn_step_record: T = %lld < 0", T);
    if (T > 0 && !states_dev) return fail(RDCNN_EINVAL, "rdcnn_step_record: NULL states buffer");
    return run_steps(h, T, states_dev);
}

int rdcnn_step_record_even(rdcnn_t h, long long T, float *states_dev)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_step_record_even: NULL handle");
    if (T < 0) return fail(RDCNN_EINVAL, "rdcnn_step_record_even: T = %lld < 0", T);
    if (T > 0 && !states_dev)
        return fail(RDCNN_EINVAL, "rdcnn_step_record_even: NULL states buffer");
    if (T > 0) {
        // the passes read their input from the trajectory: it must not overlap
        // the handle's state buffers
        const size_t state = 2 * (size_t)h->R * h->C;
        const char *t0 = (const char *)states_dev;
        const char *t1 = t0 + sizeof(float) * state * (size_t)((T + 1) / 2);
        for (float *b : h->buf) {
            const char *b0 = (const char *)b, *b1 = b0 + sizeof(float) * state;
            if (t0 < b1 && b0 < t1)
                return fail(RDCNN_EINVAL, "rdcnn_step_record_even: states buffer overlaps a "
                                          "state buffer of the handle");
        }
    }
    return run_steps(h, T, states_dev, true);
}

int rdcnn_set_adjoint_kernel(rdcnn_t h, int depth, int cols_per_lane, int seg_rows)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_set_adjoint_kernel: NULL handle");
    if (depth == 0 && cols_per_lane == 0) {
        h->adj_depth = h->adj_cpl = h->adj_seg_rows = 0;
        return RDCNN_OK;
    }
    if (cols_per_lane != 1 && cols_per_lane != 2 && cols_per_lane != 4)
        return fail(RDCNN_EINVAL, "rdcnn_set_adjoint_kernel: cols_per_lane %d not in {1,2,4}",
                    cols_per_lane);
    if (depth < 1 || depth > rd::max_adj_depth(cols_per_lane))
        return fail(RDCNN_EINVAL, "rdcnn_set_adjoint_kernel: depth %d out of range", depth);
    if (seg_rows < 0) return fail(RDCNN_EINVAL, "rdcnn_set_adjoint_kernel: seg_rows < 0");
    h->adj_depth = depth;
    h->adj_cpl = cols_per_lane;
    h->adj_seg_rows = seg_rows;
    return RDCNN_OK;
}

int rdcnn_adjoint(rdcnn_t h, const float *states_dev, long long S, float *adj_dev,
                  float *adj_tmp_dev, double *dtheta_dev)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_adjoint: NULL handle");
    if (h->model != rd::MODEL_FHN)
        return fail(RDCNN_EINVAL, "rdcnn_adjoint: FitzHugh-Nagumo grids only");
    if (S < 0) return fail(RDCNN_EINVAL, "rdcnn_adjoint: S = %lld < 0", S);
    if (!adj_dev || !adj_tmp_dev || !dtheta_dev || (S > 0 && !states_dev))
        return fail(RDCNN_EINVAL, "rdcnn_adjoint: NULL argument");
    if (adj_dev == adj_tmp_dev) return fail(RDCNN_EINVAL, "rdcnn_adjoint: adj buffers alias");
    if (S == 0) return RDCNN_OK;
    int cpl = h->adj_cpl, depth = h->adj_depth, seg = h->adj_seg_rows;
    if (depth == 0) adj_auto_config(h, &cpl, &depth, &seg);
    {
        // A pass reads its states through one 4 GiB buffer resource.
        const long long cap = ((1LL << 32) - 1) / (8LL * h->R * h->C);
        if (cap < 1) return fail(RDCNN_EINVAL, "rdcnn_adjoint: grid too large");
        if (depth > cap) depth = (int)cap;
    }
    // Every pass has `depth` steps except possibly the last; size the partial
    // buffer for the larger tiling of the two.
    rd::StreamGeom gfull, glast;
    const int klast = (int)(S % depth == 0 ? depth : S % depth);
    if (!rd::stream_geometry(h->R, h->C, cpl, (int)(S < depth ? S : depth), seg, &gfull) ||
        !rd::stream_geometry(h->R, h->C, cpl, klast, seg, &glast))
        return fail(RDCNN_EINVAL, "rdcnn_adjoint: cannot tile %dx%d", h->R, h->C);
    const long long need = gfull.ntiles > glast.ntiles ? gfull.ntiles : glast.ntiles;
    {
        const int rc = ensure_partial(h, need, "rdcnn_adjoint");
        if (rc != RDCNN_OK) return rc;
    }
    hipError_t e = rd::launch_zero(h->partial, rd::kAdjSums * need, h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_adjoint: zero");
    const size_t n = (size_t)h->R * h->C;
    Pingpong pp(adj_dev, adj_dev + n, adj_tmp_dev, adj_tmp_dev + n);
    long long q_top = S - 1, left = S;
    while (left > 0) {
        const int k = (int)(left < depth ? left : depth);
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, cpl, k, seg, &geom))
            return fail(RDCNN_EINVAL, "rdcnn_adjoint: cannot tile %dx%d", h->R, h->C);
        e = rd::launch_adjoint(pp.io(), states_dev, 1, q_top, h->R, h->C, h->bc, h->g, geom,
                               h->partial, (h->grad_mask & kLamSumGrads) != 0, h->stream);
        if (e != hipSuccess) return hip_fail(e, "rdcnn_adjoint: kernel launch");
        pp.flip();
        q_top -= k;
        left -= k;
    }
    e = pp.copy_back(n, h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_adjoint: copy back");
    e = rd::launch_adjoint_finish(h->partial, (int)need, h->g, h->grad_mask, dtheta_dev, h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_adjoint: finish");
    return RDCNN_OK;
}

namespace {

// Pass shape and partial-sum tiles of the paired reverse passes through S
// steps, reading even states `every` slots apart.
struct PairPlan {
    int cpl, depth, seg;
    long long need;  // tiles of the widest tiling
};

int plan_pairs(const rdcnn_sim *h, long long S, int every, const char *who, PairPlan *pl)
{
    int cpl = h->adj_cpl, depth = h->adj_depth, seg = h->adj_seg_rows;
    if (depth == 0) adj_even_auto_config(h, &cpl, &depth, &seg);
    // Paired passes: an even depth of 2..8, one or two columns per lane.
    if (cpl > 2) cpl = 2;
    if (depth > 8) depth = 8;
    if (depth < 2) depth = 2;
    depth &= ~1;
    {
        // A pass reads its depth/2 even states, `every` slots apart, through
        // one 4 GiB buffer resource.
        const long long cap = ((1LL << 32) - 1) / (8LL * h->R * h->C);
        if (cap < 1) return fail(RDCNN_EINVAL, "%s: grid too large", who);
        const long long dmax = 2 * ((cap - 1) / every + 1);
        if (depth > dmax) depth = (int)dmax;
    }
    // An odd S starts with one plain reverse step (state s_{S-1} is even);
    // then paired passes of `depth` steps and one shorter even remainder.
    const long long even = S & ~1LL;
    const int klast = even == 0 ? 0 : (int)(even % depth == 0 ? depth : even % depth);
    long long need = 0;
    for (int k : {(S & 1) ? 1 : 0, (int)(even < depth ? even : depth), klast}) {
        if (k == 0) continue;
        rd::StreamGeom gk;
        if (!rd::stream_geometry(h->R, h->C, cpl, k, seg, &gk))
            return fail(RDCNN_EINVAL, "%s: cannot tile %dx%d", who, h->R, h->C);
        if (gk.ntiles > need) need = gk.ntiles;
    }
    pl->cpl = cpl;
    pl->depth = depth;
    pl->seg = seg;
    pl->need = need;
    return RDCNN_OK;
}

// The paired reverse passes through S steps from an even-time trajectory
// (state s_{t0+2i} at states + i * every states), ping-ponging (lam, mu)
// between pp's two pairs of planes; the per-tile sums go to `partial` (need
// tiles, zeroed here) and are folded into dtheta.
// zero / fold: clear the partials first / fold them into dtheta at the end
// (a chain of segments clears once and folds once).
int run_pairs(rdcnn_sim *h, const float *states, int every, long long S, Pingpong &pp,
              const PairPlan &pl, double *partial, double *dtheta, const char *who,
              bool zero = true, bool fold = true)
{
    hipError_t e = hipSuccess;
    if (zero) e = rd::launch_zero(partial, rd::kAdjSums * pl.need, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    const bool lam_sums = (h->grad_mask & kLamSumGrads) != 0;
    const long long even = S & ~1LL;
    if (S & 1) {
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, pl.cpl, 1, pl.seg, &geom))
            return fail(RDCNN_EINVAL, "%s: cannot tile %dx%d", who, h->R, h->C);
        e = rd::launch_adjoint(pp.io(), states, every, (S - 1) / 2, h->R, h->C, h->bc, h->g, geom,
                               partial, lam_sums, h->stream);
        if (e != hipSuccess) return hip_fail(e, who);
        pp.flip();
    }
    for (long long t_top = even; t_top > 0;) {
        const int k = (int)(t_top < pl.depth ? t_top : pl.depth);
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, pl.cpl, k, pl.seg, &geom))
            return fail(RDCNN_EINVAL, "%s: cannot tile %dx%d", who, h->R, h->C);
        e = rd::launch_adjoint_pair(pp.io(), states, every, t_top, h->R, h->C, h->bc, h->g, geom,
                                    partial, lam_sums, h->stream);
        if (e != hipSuccess) return hip_fail(e, who);
        pp.flip();
        t_top -= k;
    }
    e = pp.copy_back((size_t)h->R * h->C, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    if (fold) e = rd::launch_adjoint_finish(partial, (int)pl.need, h->g, h->grad_mask, dtheta, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    return RDCNN_OK;
}

// Checks shared by the reverse-pass entry points; fills *done when S == 0.
int check_bwd(const rdcnn_sim *h, long long S, const void *states, const void *a, const void *b,
              const void *dtheta, const char *who)
{
    if (!h) return fail(RDCNN_EINVAL, "%s: NULL handle", who);
    if (h->model != rd::MODEL_FHN) return fail(RDCNN_EINVAL, "%s: FitzHugh-Nagumo grids only", who);
    if (S < 0) return fail(RDCNN_EINVAL, "%s: S = %lld < 0", who, S);
    if (!a || !b || !dtheta || (S > 0 && !states)) return fail(RDCNN_EINVAL, "%s: NULL argument", who);
    if (a == b) return fail(RDCNN_EINVAL, "%s: buffers alias", who);
    return RDCNN_OK;
}

// rdcnn_step_bwd's buffers: lam and mu are distinct planes, and the workspace
// slot S of the trajectory overlaps neither.
int check_step_bwd(const rdcnn_sim *h, const float *states, long long S, const float *lam,
                   const float *mu, const char *who)
{
    const size_t n = (size_t)h->R * h->C;
    const char *l0 = (const char *)lam, *m0 = (const char *)mu;
    const char *w0 = (const char *)(states + (size_t)S * 2 * n);
    const size_t pb = sizeof(float) * n;
    auto overlap = [](const char *x, size_t nx, const char *y, size_t ny) {
        return x < y + ny && y < x + nx;
    };
    if (overlap(l0, pb, m0, pb)) return fail(RDCNN_EINVAL, "%s: lam and mu overlap", who);
    if (overlap(w0, 2 * pb, l0, pb) || overlap(w0, 2 * pb, m0, pb))
        return fail(RDCNN_EINVAL, "%s: lam or mu overlaps the trajectory's workspace slot S", who);
    return RDCNN_OK;
}

}  // namespace

int rdcnn_adjoint_even(rdcnn_t h, const float *states_dev, long long S, float *adj_dev,
                       float *adj_tmp_dev, double *dtheta_dev)
{
    const char *who = "rdcnn_adjoint_even";
    int rc = check_bwd(h, S, states_dev, adj_dev, adj_tmp_dev, dtheta_dev, who);
    if (rc != RDCNN_OK || S == 0) return rc;
    PairPlan pl;
    if ((rc = plan_pairs(h, S, 1, who, &pl)) != RDCNN_OK) return rc;
    if ((rc = ensure_partial(h, pl.need, who)) != RDCNN_OK) return rc;
    const size_t n = (size_t)h->R * h->C;
    Pingpong pp(adj_dev, adj_dev + n, adj_tmp_dev, adj_tmp_dev + n);
    return run_pairs(h, states_dev, 1, S, pp, pl, h->partial, dtheta_dev, who);
}

int rdcnn_step_record_sparse(rdcnn_t h, long long T, float *states_dev)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_step_record_sparse: NULL handle");
    if (T < 0) return fail(RDCNN_EINVAL, "rdcnn_step_record_sparse: T = %lld < 0", T);
    if (T > 0 && !states_dev)
        return fail(RDCNN_EINVAL, "rdcnn_step_record_sparse: NULL states buffer");
    if (T > 0) {
        // the passes read their input from the trajectory's even slots: they
        // must not overlap the handle's state buffers
        const size_t state = 2 * (size_t)h->R * h->C;
        const char *t0 = (const char *)states_dev;
        const char *t1 = t0 + sizeof(float) * state * (size_t)(T + 1);
        for (float *b : h->buf) {
            const char *b0 = (const char *)b, *b1 = b0 + sizeof(float) * state;
            if (t0 < b1 && b0 < t1)
                return fail(RDCNN_EINVAL, "rdcnn_step_record_sparse: states buffer overlaps a "
                                          "state buffer of the handle");
        }
    }
    return run_steps(h, T, states_dev, true, 2);
}

int rdcnn_step_checkpoints(rdcnn_t h, long long T, long long S, float *ckpt_dev)
{
    const char *who = "rdcnn_step_checkpoints";
    if (!h) return fail(RDCNN_EINVAL, "%s: NULL handle", who);
    if (T < 0 || S < 1) return fail(RDCNN_EINVAL, "%s: T = %lld, S = %lld", who, T, S);
    if (T == 0) return RDCNN_OK;
    if (!ckpt_dev) return fail(RDCNN_EINVAL, "%s: NULL checkpoint buffer", who);
    if (h->model != rd::MODEL_FHN) return fail(RDCNN_EINVAL, "%s: FitzHugh-Nagumo grids only", who);
    const size_t state = 2 * (size_t)h->R * h->C;
    const long long nseg = (T + S - 1) / S;
    {
        const char *c0 = (const char *)ckpt_dev, *c1 = c0 + sizeof(float) * state * (size_t)nseg;
        for (float *b : h->buf) {
            const char *b0 = (const char *)b, *b1 = b0 + sizeof(float) * state;
            if (c0 < b1 && b0 < c1)
                return fail(RDCNN_EINVAL, "%s: checkpoint buffer overlaps a state buffer", who);
        }
    }
    int kind = h->kind == 3 ? 2 : h->kind, cpl = h->cpl, depth = h->depth, seg = h->seg_rows;
    if (kind == 0) {
        kind = 2;
        auto_config(h, &cpl, &depth, &seg, false);
    }
    hipError_t e = hipMemcpyAsync(ckpt_dev, h->buf[h->cur], sizeof(float) * state,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    // Passes stop at every multiple of S; the pass that ends at jS < T writes
    // its output straight into checkpoint j and the next pass reads it there.
    const float *in = h->buf[h->cur];
    for (long long q = 0; q < T;) {
        const long long bound = (q / S + 1) * S;
        long long k = kind == 1 ? 1 : depth;
        if (k > T - q) k = T - q;
        if (k > bound - q) k = bound - q;
        const long long end = q + k;
        float *out = end % S == 0 && end < T ? ckpt_dev + (size_t)(end / S) * state
                     : in == h->buf[0]      ? h->buf[1]
                                            : h->buf[0];
        if (kind == 1) {
            e = rd::launch_naive(in, out, h->R, h->C, h->bc, h->g, h->stream);
        } else {
            rd::StreamGeom geom;
            if (!rd::stream_geometry(h->R, h->C, cpl, (int)k, seg, &geom))
                return fail(RDCNN_EINVAL, "%s: cannot tile %dx%d with cpl=%d depth=%lld", who, h->R,
                            h->C, cpl, k);
            e = rd::launch_stream(in, out, h->R, h->C, h->bc, h->g, geom, h->stream);
        }
        if (e != hipSuccess) return hip_fail(e, who);
        in = out;
        q = end;
    }
    h->cur = in == h->buf[0] ? 0 : 1;
    return RDCNN_OK;
}

int rdcnn_step_bwd(rdcnn_t h, float *states_dev, long long S, float *lam_dev, float *mu_dev,
                   double *dtheta_accum)
{
    const char *who = "rdcnn_step_bwd";
    int rc = check_bwd(h, S, states_dev, lam_dev, mu_dev, dtheta_accum, who);
    if (rc != RDCNN_OK || S == 0) return rc;
    if ((rc = check_step_bwd(h, states_dev, S, lam_dev, mu_dev, who)) != RDCNN_OK) return rc;
    PairPlan pl;
    if ((rc = plan_pairs(h, S, 2, who, &pl)) != RDCNN_OK) return rc;
    if ((rc = ensure_partial(h, pl.need, who)) != RDCNN_OK) return rc;
    const size_t n = (size_t)h->R * h->C;
    float *work = states_dev + (size_t)S * 2 * n;  // slot S: never read as a state
    Pingpong pp(lam_dev, mu_dev, work, work + n);
    return run_pairs(h, states_dev, 2, S, pp, pl, h->partial, dtheta_accum, who);
}

int rdcnn_step_bwd_noalloc(rdcnn_t h, float *states_dev, long long S, float *lam_dev,
                           float *mu_dev, double *dtheta_accum)
{
    const char *who = "rdcnn_step_bwd_noalloc";
    int rc = check_bwd(h, S, states_dev, lam_dev, mu_dev, dtheta_accum, who);
    if (rc != RDCNN_OK || S == 0) return rc;
    if ((rc = check_step_bwd(h, states_dev, S, lam_dev, mu_dev, who)) != RDCNN_OK) return rc;
    PairPlan pl;
    if ((rc = plan_pairs(h, S, 2, who, &pl)) != RDCNN_OK) return rc;
    if (pl.need > kNoAllocTiles)
        return fail(RDCNN_EINVAL, "%s: the reverse passes of this %dx%d grid use %lld tiles; the "
                    "static workspace holds %lld (use rdcnn_step_bwd, or fewer, taller segments "
                    "via rdcnn_set_adjoint_kernel)", who, h->R, h->C, pl.need, kNoAllocTiles);
    double *ws = nullptr;
    if ((rc = scratch_address(&ws, who)) != RDCNN_OK) return rc;
    const size_t n = (size_t)h->R * h->C;
    float *work = states_dev + (size_t)S * 2 * n;  // slot S: never read as a state
    Pingpong pp(lam_dev, mu_dev, work, work + n);
    return run_pairs(h, states_dev, 2, S, pp, pl, ws, dtheta_accum, who);
}

int rdcnn_step_bwd_ckpt(rdcnn_t h, const float *ckpt_dev, long long T, long long S,
                        float *work_dev, float *lam_dev, float *mu_dev, double *dtheta_accum)
{
    const char *who = "rdcnn_step_bwd_ckpt";
    if (!h) return fail(RDCNN_EINVAL, "%s: NULL handle", who);
    if (h->model != rd::MODEL_FHN) return fail(RDCNN_EINVAL, "%s: FitzHugh-Nagumo grids only", who);
    if (T < 0 || S < 1) return fail(RDCNN_EINVAL, "%s: T = %lld, S = %lld", who, T, S);
    if (T == 0) return RDCNN_OK;
    if (!ckpt_dev || !work_dev || !lam_dev || !mu_dev || !dtheta_accum)
        return fail(RDCNN_EINVAL, "%s: NULL argument", who);
    const size_t n = (size_t)h->R * h->C, state = 2 * n;
    const long long nseg = (T + S - 1) / S;
    const long long Smax = S < T ? S : T;
    {
        auto overlap = [](const void *x, size_t nx, const void *y, size_t ny) {
            const char *a = (const char *)x, *b = (const char *)y;
            return a < b + ny && b < a + nx;
        };
        const size_t pb = sizeof(float) * n;
        const size_t wb = sizeof(float) * state * 2 * (size_t)(Smax + 1);
        const size_t cb = sizeof(float) * state * (size_t)nseg;
        if (overlap(lam_dev, pb, mu_dev, pb)) return fail(RDCNN_EINVAL, "%s: lam and mu overlap", who);
        if (overlap(work_dev, wb, lam_dev, pb) || overlap(work_dev, wb, mu_dev, pb) ||
            overlap(work_dev, wb, ckpt_dev, cb))
            return fail(RDCNN_EINVAL, "%s: the workspace overlaps lam, mu or the checkpoints", who);
    }
    int cpl, depth, seg;
    if (!even_record_shape(h, 2, &cpl, &depth, &seg))
        return fail(RDCNN_EINVAL, "%s: grid too large to record", who);
    // The recompute shares the GPU with the reverse passes of the next
    // segment, so it aims at ~940 wavefronts, a third of what a recording run
    // alone aims at (taller segments, less halo work; never shorter ones than
    // alone), in passes of 6 steps.  On 1024^2, T = 2000 (22 strips: 24-row
    // segments) the backward took 9.96 ms against 10.06 at 8 steps, 10.3 at
    // 16 rows and 10.6 at 8 rows, in sweeps over 8 to 32 rows.
    if (h->kind != 2) {
        rd::StreamGeom sg;
        if (rd::stream_geometry(h->R, h->C, cpl, depth, seg, &sg)) {
            const long long per_strip = (940 + sg.nstrips - 1) / sg.nstrips;
            const long long rows = (h->R + per_strip - 1) / per_strip;
            if (rows > seg) seg = (int)rows;
        }
        if (depth > 6) depth = 6;
    }
    // One partial buffer for every segment: cleared once, folded once.
    const long long Llast = T - (nseg - 1) * S;
    PairPlan pl, plast;
    int rc = plan_pairs(h, Smax, 2, who, &pl);
    if (rc == RDCNN_OK) rc = plan_pairs(h, Llast, 2, who, &plast);
    if (rc != RDCNN_OK) return rc;
    const long long need = pl.need > plast.need ? pl.need : plast.need;
    if ((rc = ensure_partial(h, need, who)) != RDCNN_OK) return rc;
    hipError_t e = hipSuccess;
    if (!h->side && (rc = side_stream(&h->side, who)) != RDCNN_OK) return rc;
    for (hipEvent_t &ev : h->ev) {
        if (ev) continue;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            ev = nullptr;
            return hip_fail(e, who);
        }
    }
    hipEvent_t *ready = h->ev, *done = h->ev + 2, start = h->ev[4];
    e = rd::launch_zero(h->partial, rd::kAdjSums * need, h->stream);
    if (e == hipSuccess) e = hipEventRecord(start, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->side, start, 0);  // the caller's earlier work
    if (e != hipSuccess) return hip_fail(e, who);
    float *segbuf[2] = {work_dev, work_dev + (size_t)(Smax + 1) * state};
    for (long long idx = 0; idx < nseg; ++idx) {
        const long long k = nseg - 1 - idx;
        const long long L = k == nseg - 1 ? Llast : S;
        const int b = (int)(idx & 1);
        float *traj = segbuf[b];
        // Recompute segment k on the side stream once the reverse pass that
        // read this buffer two segments ago is done; its final state goes to
        // slot L, the reverse passes' workspace (never read as a state).
        if (idx >= 2 && (e = hipStreamWaitEvent(h->side, done[b], 0)) != hipSuccess)
            return hip_fail(e, who);
        rc = record_even_chain(h, ckpt_dev + (size_t)k * state, L, traj, 2, traj + (size_t)L * state,
                               cpl, depth, seg, h->side, who);
        if (rc != RDCNN_OK) return rc;
        if ((e = hipEventRecord(ready[b], h->side)) != hipSuccess ||
            (e = hipStreamWaitEvent(h->stream, ready[b], 0)) != hipSuccess)
            return hip_fail(e, who);
        // Reverse passes of segment k on the handle's stream, overlapping the
        // recompute of segment k-1.
        PairPlan plk;
        if ((rc = plan_pairs(h, L, 2, who, &plk)) != RDCNN_OK) return rc;
        float *ws = traj + (size_t)L * state;
        Pingpong pp(lam_dev, mu_dev, ws, ws + n);
        rc = run_pairs(h, traj, 2, L, pp, plk, h->partial, dtheta_accum, who, false, false);
        if (rc != RDCNN_OK) return rc;
        if ((e = hipEventRecord(done[b], h->stream)) != hipSuccess) return hip_fail(e, who);
    }
    e = rd::launch_adjoint_finish(h->partial, (int)need, h->g, h->grad_mask, dtheta_accum, h->stream);
    if (e != hipSuccess) return hip_fail(e, who);
    return RDCNN_OK;
}

int rdcnn_set_grad_mask(rdcnn_t h, unsigned mask)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_set_grad_mask: NULL handle");
    if (mask == 0 || mask > 0xFFu) return fail(RDCNN_EINVAL, "rdcnn_set_grad_mask: mask 0x%x", mask);
    h->grad_mask = mask;
    return RDCNN_OK;
}

int rdcnn_init_backward(const float *adj_dev, long long n, float ka, float *gx_dev, void *stream)
{
    if (!adj_dev || !gx_dev || n < 0) return fail(RDCNN_EINVAL, "rdcnn_init_backward: bad argument");
    if (!isfinite(ka)) return fail(RDCNN_EINVAL, "rdcnn_init_backward: non-finite ka");
    if (n == 0) return RDCNN_OK;
    hipError_t e = rd::launch_init_backward(adj_dev, n, ka, gx_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_init_backward");
    return RDCNN_OK;
}

int rdcnn_read(rdcnn_t h, float *u_dst, float *v_dst, int dst_is_host)
{
    if (!h || !u_dst || !v_dst) return fail(RDCNN_EINVAL, "rdcnn_read: NULL argument");
    const size_t bytes = sizeof(float) * (size_t)h->R * h->C;
    const float *s = h->buf[h->cur];
    const hipMemcpyKind kind = dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(u_dst, s, bytes, kind, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(v_dst, s + (size_t)h->R * h->C, bytes, kind, h->stream);
    if (e == hipSuccess && dst_is_host && !h->check_finite) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_read");
    if (h->check_finite)
        return rd::check_finite_state(s, 2LL * h->R * h->C, &h->finite_flag, h->stream, "rdcnn_read");
    return RDCNN_OK;
}

int rdcnn_set_check_finite(rdcnn_t h, int on)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_set_check_finite: NULL handle");
    h->check_finite = on != 0;
    return RDCNN_OK;
}

int rdcnn_write_state(rdcnn_t h, const float *u_dev, const float *v_dev)
{
    if (!h || !u_dev || !v_dev) return fail(RDCNN_EINVAL, "rdcnn_write_state: NULL argument");
    const size_t n = (size_t)h->R * h->C;
    float *d = h->buf[h->cur];
    hipError_t e = hipMemcpyAsync(d, u_dev, sizeof(float) * n, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + n, v_dev, sizeof(float) * n, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(e, "rdcnn_write_state");
    return RDCNN_OK;
}

int rdcnn_set_params(rdcnn_t h, const rdcnn_params_t *p)
{
    if (!h || !p) return fail(RDCNN_EINVAL, "rdcnn_set_params: NULL argument");
    if (!finite_params(p)) return fail(RDCNN_EINVAL, "rdcnn_set_params: non-finite parameter");
    if (h->model != rd::MODEL_FHN)
        return fail(RDCNN_EINVAL, "rdcnn_set_params: FitzHugh-Nagumo grids only");
    h->g = to_gene(p);
    drop_graphs(h);
    return RDCNN_OK;
}

int rdcnn_current(rdcnn_t h, float **state_dev)
{
    if (!h || !state_dev) return fail(RDCNN_EINVAL, "rdcnn_current: NULL argument");
    *state_dev = h->buf[h->cur];
    return RDCNN_OK;
}

int rdcnn_set_kernel(rdcnn_t h, int kind, int depth, int cols_per_lane, int seg_rows)
{
    if (!h) return fail(RDCNN_EINVAL, "rdcnn_set_kernel: NULL handle");
    drop_graphs(h);
    if (kind == 0 || kind == 1) {
        h->kind = kind;
        return RDCNN_OK;
    }
    if (kind != 2 && kind != 3) return fail(RDCNN_EINVAL, "rdcnn_set_kernel: unknown kind %d", kind);
    if (cols_per_lane != 1 && cols_per_lane != 2 && cols_per_lane != 4)
        return fail(RDCNN_EINVAL, "rdcnn_set_kernel: cols_per_lane %d not in {1,2,4}", cols_per_lane);
    if (depth < 1 || depth > rd::max_depth(cols_per_lane))
        return fail(RDCNN_EINVAL, "rdcnn_set_kernel: depth %d out of range for cols_per_lane %d",
                    depth, cols_per_lane);
    if (seg_rows < 0) return fail(RDCNN_EINVAL, "rdcnn_set_kernel: seg_rows < 0");
    h->kind = kind;
    h->depth = depth;
    h->cpl = cols_per_lane;
    h->seg_rows = seg_rows;
    return RDCNN_OK;
}

int rdcnn_pass_config(rdcnn_t h, int *kind, int *depth, int *cols_per_lane, int *seg_rows)
{
    if (!h || !kind || !depth || !cols_per_lane || !seg_rows)
        return fail(RDCNN_EINVAL, "rdcnn_pass_config: NULL argument");
    int k = h->kind == 3 ? 2 : h->kind, cpl = h->cpl, d = h->depth, seg = h->seg_rows;
    if (h->model != rd::MODEL_FHN) {
        if (k == 0) k = 2;
        model_shape(h, &cpl, &d, &seg);
    } else if (k == 0) {
        k = 2;
        auto_config(h, &cpl, &d, &seg, false);
    }
    if (k == 1) {
        cpl = d = 1;
        seg = 1;
    } else {
        rd::StreamGeom geom;
        if (!rd::stream_geometry(h->R, h->C, cpl, d, seg, &geom))
            return fail(RDCNN_EINVAL, "rdcnn_pass_config: cannot tile %dx%d", h->R, h->C);
        seg = geom.h;
    }
    *kind = k;
    *depth = d;
    *cols_per_lane = cpl;
    *seg_rows = seg;
    return RDCNN_OK;
}

int rdcnn_destroy(rdcnn_t h)
{
    if (!h) return RDCNN_OK;
    pool_put(h->partial_device, h->partial_cap, h->partial, h->stream);
    if (h->finite_flag) (void)hipFree(h->finite_flag);
    // The recompute stream is the device's and stays; wait for this handle's
    // recomputes on it (each ends with one of its events) before the caller
    // may free the buffers they use.
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventSynchronize(e);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    drop_graphs(h);
    delete h;
    return RDCNN_OK;
}

}  // extern "C"
