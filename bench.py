"""Benchmark of the RD-CNN forward path on one MI355X (arXiv 2102.10340).

Workload (slow growth at scale): one 4096x4096 float32 grid, zero-flux,
f1 = u - u^3 - v, f2 = 0.1 (u - v), Du = 0.05, Dv = 1, dt = 0.1; x is zero
except a 16x16 random U[-1,1] centre patch (seed 0); u = v = x.  The job runs
T = 100000 steps and snapshots (u, v) every 10000 steps into device memory.
One benchmark step = 10000 time steps + one snapshot, so the default
``--steps 10`` is the whole job.  Inputs are resident in HBM before timing.

Prints one JSON line: Gcell-updates/s (cells x time steps / s), the roofline of
the dominant kernel (effective HBM GB/s at 16 B per cell-update, the naive
traffic of one explicit step), and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

R = C = 4096
T_CHUNK = 10000
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 16  # read u, v and write u, v once per explicit step
# Algorithmic flops of one cell-update of Eq. (1)-(3): two 5-point Laplacians
# (3 adds + 1 fma each), u^3 and f1, f2 and the two Euler updates: 28 flops
# (an fma counts 2).  The kernels' rounding order issues 17 VALU instructions.
FLOPS_PER_CELL_UPDATE = 28
VALU_OPS_PER_CELL_UPDATE = 17
# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz.  The published FP32 vector
# peak, 157.3 TFLOP/s, counts packed (two-wide) FMAs; without packed FP32 the
# ceiling is one FMA per lane per clock, 78.6 TFLOP/s, and the issue rate is
# 39.3 T lane-instructions/s.
ALU_PEAK_TFLOPS = 157.3
ALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--chunk", type=int, default=T_CHUNK,
                    help="time steps per benchmark step (profiler runs use fewer)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="first run a plain device copy of this size (scales HBM counters)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the differentiation and parameter-sweep workloads")
    ap.add_argument("--only-extra", choices=["fwd_bwd", "batched", "small_batch", "atlas", "models",
                                                   "plain", "edge", "table1"],
                    help="run just this extra workload after the forward steps (profiling)")
    return ap.parse_args()


def measured_traffic(kernel_prefix: str):
    """HBM bytes per launch of the kernel from the committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.json"))):
        with open(path) as f:
            rec = json.load(f)
        if rec.get("kernel") != kernel_prefix:
            continue
        h = hashlib.sha256()
        for rel in rec["sources"]:
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec["traffic_bytes_per_launch"]
    return None


def _timed(fn, stream):
    """Seconds for fn() between HIP events on `stream`, synchronized on both sides."""
    import torch
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / 1e3


def bench_fwd_bwd(stream):
    """Differentiation workload: 1024x1024, T = 2000, plain gene, x ~ U[-1,1]
    (seed 0), loss = MSE(u_T, three-sinusoid stripe target); gradients with
    respect to x, Du, Dv and eps (and, separately, all eight parameters).
    Schedules: checkpoint every ceil(sqrt(T)) steps (rounded up to the pass
    depth: 48) and recompute each segment in the backward, overlapped with
    the reverse pass of the segment after it (the workload's schedule), and
    the whole trajectory recorded in the forward."""
    import torch
    from paper_2102_10340_amd import Simulation, simulate
    from paper_2102_10340_amd import autograd as AG
    N, T = 1024, 2000
    g = W.PLAIN_GENE
    keys = ("dt", "a", "b", "eps", "c", "k3", "Du", "Dv")
    x = torch.from_numpy(W.uniform_x(N, N, 0)).cuda()
    target = torch.from_numpy(W.stripe_target(N, N, 0)).cuda()

    def fwd():
        sim = Simulation(x, g, "zeroflux")
        sim.step(T)
        sim.read()
        sim.close()

    def fwd_bwd(grads, S):
        def run():
            xt = x.clone().requires_grad_(True)
            theta = torch.tensor([g[k] for k in keys], dtype=torch.float64, requires_grad=True)
            u, _ = simulate(xt, theta, T, "zeroflux", S=S, grads=grads)
            ((u - target) ** 2).mean().backward()
        return run

    def best(fn, n=3):
        fn()
        return min(_timed(fn, stream) for _ in range(n))

    sub = ("Du", "Dv", "eps")
    tf = best(fwd)
    S = AG.default_segment(T)
    t_sq = best(fwd_bwd(sub, 0))
    t_sq8 = best(fwd_bwd(None, 0))
    t_wh = best(fwd_bwd(sub, -1))
    cells = N * N * T
    return {"workload": "1024x1024 zero-flux, T=2000, MSE to stripe target, grads wrt x, Du, Dv "
                        "and eps",
            "fwd_ms": tf * 1e3, "fwd_gcells": cells / tf / 1e9,
            "sqrt_t": {"schedule": f"checkpoint every {S} steps (ceil(sqrt(T)) rounded up to the "
                                   "pass depth), segments recomputed on a second stream "
                                   "overlapping the reverse pass of the next segment",
                       "segment_steps": S, "fwd_bwd_ms": t_sq * 1e3,
                       "fwd_bwd_gcells": cells / t_sq / 1e9, "ratio_fwd_bwd_to_fwd": t_sq / tf,
                       "all8_ms": t_sq8 * 1e3, "ratio_all8_to_fwd": t_sq8 / tf},
            "whole_trajectory": {"schedule": "states of even times of all T steps recorded in HBM",
                                 "fwd_bwd_ms": t_wh * 1e3, "fwd_bwd_gcells": cells / t_wh / 1e9,
                                 "ratio_fwd_bwd_to_fwd": t_wh / tf},
            "ratio_fwd_bwd_to_fwd": t_sq / tf}


def bench_batched(stream, per_class=8):
    """Parameter sweep: 1024 instances, side uniform over {128,256,512,1024},
    Du ~ U[0.01,0.2], Dv ~ U[0.2,1], epsilon ~ U[0.02,0.2], zero-flux, x ~ U[-1,1]
    per instance, T = 5000, one graph launch.  Baseline: the same instances run
    one at a time (rdcnn_step(T) on one stream, each size with the autotuner's
    cached single-grid shape), timed on `per_class` instances of each size and
    scaled by the class counts.  Both
    sides are timed on steps T..2T (after an untimed first T steps, which also
    captures the batch's graph), and the sampled instances are compared bit for
    bit between the two."""
    import torch
    from paper_2102_10340_amd import Batch, Simulation
    T = 5000
    inst = W.sweep_instances(1024, 0)
    xs = [torch.from_numpy(W.uniform_x(d["rows"], d["cols"], d["seed"])).cuda() for d in inst]
    b = Batch(xs, [d["gene"] for d in inst], "zeroflux")
    batch_from = b.tuned_from or "library default"
    b.use_graph(True)
    b.step(T)  # captures the T-step graph and runs it once (untimed)
    tb = _timed(lambda: b.step(T), stream)  # graph replay: steps T..2T
    cells = sum(d["rows"] * d["cols"] for d in inst)
    # per-instance baseline on a sample of each size class
    t_single, same, single_from = 0.0, True, {}
    for side in (128, 256, 512, 1024):
        idx = [i for i, d in enumerate(inst) if d["rows"] == side]
        ts = []
        for i in idx[:per_class]:
            sim = Simulation(xs[i], inst[i]["gene"], "zeroflux")
            single_from[side] = sim.tuned_from or "library default"
            sim.step(T)
            ts.append(_timed(lambda: sim.step(T), stream))
            same &= bool(torch.equal(sim.state(), b.state(i)))
            sim.close()
        t_single += sum(ts) / len(ts) * len(idx)
    b.close()
    return {"workload": "1024 instances, sides {128,256,512,1024}, per-instance Du/Dv/eps, "
                        "zero-flux, T=5000, one graph launch",
            "batched_gcells": cells * T / tb / 1e9, "batched_s": tb,
            "per_instance_gcells": cells * T / t_single / 1e9, "per_instance_s_est": t_single,
            "speedup_vs_per_instance": t_single / tb, "sampled_instances_bitwise_equal": same,
            "baseline_sample": f"{per_class} instances per size class, scaled by class counts",
            "pass_shape_from": {"batch": batch_from, "per_instance": single_from}}


def bench_small_batch(stream, per_instance_sample=8):
    """Many small grids: 1024 instances of 128x128 (the paper's smallest Table I
    side), per-instance Du ~ U[0.01,0.2], Dv ~ U[0.2,1], epsilon ~ U[0.02,0.2],
    zero-flux, x ~ U[-1,1] per instance, T = 10^4.  Three ways: the in-LDS
    kernel (each instance whole in one workgroup's LDS for all steps), the
    streamed batch kernel replayed from a graph, and one instance at a time
    (sampled, scaled by the count).  The LDS and streamed results are compared
    bit for bit."""
    import torch
    from paper_2102_10340_amd import Batch, Simulation
    T = 10000
    inst = W.sweep_instances(1024, 7, sides=(128,))
    xs = [torch.from_numpy(W.uniform_x(d["rows"], d["cols"], d["seed"])).cuda() for d in inst]
    genes = [d["gene"] for d in inst]
    cells = sum(d["rows"] * d["cols"] for d in inst)
    lds = Batch(xs, genes, "zeroflux")
    n_lds = lds.lds_instances()
    t_lds = _timed(lambda: lds.step(T), stream)
    st = Batch(xs, genes, "zeroflux")
    st.use_lds(False)
    st.use_graph(True)
    t_st = _timed(lambda: st.step(T), stream)  # includes the one-off graph capture
    same = all(bool(torch.equal(lds.state(i), st.state(i))) for i in range(len(inst)))
    st.step(T)  # steps T..2T from the captured graph
    t_st = min(t_st, _timed(lambda: st.step(T), stream))
    lds.close()
    st.close()
    ts = []
    for i in range(per_instance_sample):
        sim = Simulation(xs[i], genes[i], "zeroflux")
        sim.step(100)
        ts.append(_timed(lambda: sim.step(T), stream))
        sim.close()
    t_one = sum(ts) / len(ts) * len(inst)
    return {"workload": "1024 instances 128x128, per-instance Du/Dv/eps, zero-flux, T=10000",
            "in_lds_instances": n_lds, "in_lds_gcells": cells * T / t_lds / 1e9,
            "in_lds_s": t_lds, "streamed_graph_gcells": cells * T / t_st / 1e9,
            "streamed_s": t_st, "per_instance_gcells": cells * T / t_one / 1e9,
            "per_instance_s_est": t_one, "lds_vs_streamed": t_st / t_lds,
            "lds_vs_per_instance": t_one / t_lds, "lds_equals_streamed_bitwise": same,
            "baseline_sample": f"{per_instance_sample} instances run alone, scaled by 1024"}


def bench_atlas(stream):
    """Parameter atlas after Sec. III.A: (Du, Dv) on a 32 x 32 grid (Du = 0.025 ..
    0.8, Dv = 0.05 .. 1.6), the paper's default gene, periodic, 256x256 with the
    random 11x11 centre patch, T = 10^4 steps in one batch; per-instance
    statistics at T - 10^3 and T on the GPU, one class per point on the host.
    Reports the whole scan's rate and the statistics kernels' HBM rate (12 B per
    cell read with the earlier state, 8 B without)."""
    import numpy as np
    import torch
    from paper_2102_10340_amd import Batch, atlas
    T, dT, N = 10000, 1000, 256
    du = 0.025 * np.arange(1, 33)
    dv = 0.05 * np.arange(1, 33)
    g = W.gene(W.PAPER_DEFAULT_GENE)
    genes = [dict(g, Du=float(a), Dv=float(b)) for a in du for b in dv]
    x = torch.from_numpy(W.centre_patch_x(N, N, 11, 0)).cuda()
    b = Batch([x] * len(genes), genes, "periodic")
    ref = torch.tensor([atlas.rest_state(q)[0] for q in genes], dtype=torch.float32, device="cuda")
    out = {}

    def run():
        b.step(T - dT)
        out["prev"] = b.snapshot()
        out["s0"] = b.stats(None, ref, 0.05, 1e-3)
        b.step(dT)
        out["s1"] = b.stats(out["prev"], ref, 0.05, 1e-3)

    t_scan = _timed(run, stream)
    cells = len(genes) * N * N
    t_stats = _timed(lambda: [b.stats(out["prev"], ref, 0.05, 1e-3) for _ in range(10)], stream) / 10
    cls = atlas.classify(out["s0"].cpu().numpy(), out["s1"].cpu().numpy()).reshape(32, 32)
    b.close()
    named = {}
    for (a, c) in ((0.3, 1.0), (0.5, 0.8), (0.7, 0.8)):
        named[f"{a},{c}"] = atlas.CLASSES[cls[int(round(a / 0.025)) - 1, int(round(c / 0.05)) - 1]]
    return {"workload": "32x32 (Du,Dv) scan, 256x256 periodic, paper gene, 11x11 patch, T=10000, "
                        "stats at T-1000 and T",
            "scan_gcells": cells * T / t_scan / 1e9, "scan_s": t_scan,
            "stats_ms": t_stats * 1e3, "stats_gbs": 12 * cells / t_stats / 1e9,
            "classes": {atlas.CLASSES[k]: int((cls == k).sum()) for k in range(4)},
            "paper_points": named}


def bench_models(stream):
    """The further cell models on the streamed kernel at the headline grid size:
    Gray-Scott (dt=0.5, F=0.037, k=0.06, Du=0.2, Dv=0.1, periodic, u = 1 and
    v = 0 with a seeded 512x512 square of (0.5, 0.25) plus U[0,0.05] noise) and
    the Chua-Yang edge template (A = 2 at the centre, B = 8 / -1, z = -1,
    dt = 0.1, zero-flux) on a 4096x4096 two-level rectangle image; T = 2000
    each, default pass settings."""
    import numpy as np
    import torch
    from paper_2102_10340_amd import Simulation
    N, T = 4096, 2000
    rng = np.random.default_rng(0)
    u = np.ones((N, N), np.float32)
    v = rng.uniform(0, 0.05, (N, N)).astype(np.float32)
    u[1792:2304, 1792:2304] = 0.5
    v[1792:2304, 1792:2304] += 0.25
    out = {}
    gs = Simulation.gray_scott(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(), 0.5, 0.037,
                               0.06, 0.2, 0.1, "periodic")
    gs.step(16)
    t = _timed(lambda: gs.step(T), stream)
    gs.close()
    out["gray_scott_gcells"] = N * N * T / t / 1e9
    _, clean = W.rect_image(N, N, 1)
    img = torch.from_numpy(np.where(clean > 0, 1.0, -1.0).astype(np.float32)).cuda()
    cnn = Simulation.cnn(torch.zeros_like(img), img, [[0, 0, 0], [0, 2, 0], [0, 0, 0]],
                         [[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]], -1.0, 0.1, "zeroflux")
    cnn.step(16)
    t = _timed(lambda: cnn.step(T), stream)
    cnn.close()
    out["cnn_edge_gcells"] = N * N * T / t / 1e9
    out["workload"] = "4096x4096, T=2000: Gray-Scott (periodic) and Chua-Yang edge CNN (zero-flux)"
    return out


def bench_plain(stream):
    """Plain method: 256x256, T=1000, zero-flux, x ~ U[-1,1] (seed 0)."""
    import torch
    from paper_2102_10340_amd import Simulation
    N, T = 256, 1000
    x = torch.from_numpy(W.uniform_x(N, N, 0)).cuda()
    sim = Simulation(x, W.PLAIN_GENE, "zeroflux")
    sim.step(T)
    state = sim.read_host()  # s_T, compared with the oracle in the CPU leg
    t = min(_timed(lambda: sim.step(T), stream) for _ in range(3))
    sim.close()
    # the same run replayed from a captured HIP graph (rdcnn_use_graph)
    sim = Simulation(x, W.PLAIN_GENE, "zeroflux").use_graph(True)
    sim.step(T)  # captures the graph from buffer 0 (an odd pass count flips the buffer)
    same = bool(np.array_equal(sim.read_host()[0], state[0]))
    sim.step(T)  # ... and from buffer 1
    tg = min(_timed(lambda: sim.step(T), stream) for _ in range(4))
    sim.close()
    return {"workload": "256x256 zero-flux, T=1000, x~U[-1,1]", "gcells": N * N * T / t / 1e9,
            "ms": t * 1e3, "graph_gcells": N * N * T / tg / 1e9, "graph_ms": tg * 1e3,
            "graph_first_T_bitwise_equal": same}, state


def bench_edge_fit(stream, n_img=64, iters=4):
    """Edge detection fitted by gradient: 64 synthetic 1024x1024 images (20..60
    random rectangles of levels U[-1,1] plus N(0, 0.05^2) noise), x = image,
    T = 50, zero-flux; Du, Dv and epsilon (shared by all images) fitted by Adam
    to the normalized Sobel magnitude of the clean images.  Each iteration is
    one batched forward+backward over all 64 images (simulate_batch: even-time
    recording batch kernel, batched paired reverse passes).  Reports the loss curve, the fwd+bwd
    rate, and for comparison one iteration run image by image over four
    streams with the single-grid path."""
    import torch
    from paper_2102_10340_amd import simulate, simulate_batch
    N, T = 1024, 50
    imgs, targets = [], []
    for i in range(n_img):
        noisy, clean = W.rect_image(N, N, 500 + i)
        imgs.append(torch.from_numpy(noisy).cuda())
        targets.append(torch.from_numpy(W.sobel_target(clean)).cuda())
    g = W.PLAIN_GENE
    p = torch.tensor([g["Du"], g["Dv"], -g["eps"]], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.02)
    grads = ("Du", "Dv", "eps")

    def theta_of(q):
        return torch.stack([torch.tensor(g["dt"], dtype=torch.float64),
                            torch.tensor(g["a"], dtype=torch.float64),
                            torch.tensor(g["b"], dtype=torch.float64), -q[2],
                            torch.tensor(g["c"], dtype=torch.float64),
                            torch.tensor(g["k3"], dtype=torch.float64), q[0], q[1]])

    def batched(theta):
        outs = simulate_batch(imgs, theta, T, "zeroflux", grads=grads)
        total = torch.stack([((u - tg) ** 2).mean() for (u, _), tg in zip(outs, targets)]).sum()
        total = total / n_img
        total.backward()
        return float(total.detach())

    streams = [torch.cuda.Stream() for _ in range(4)]

    def per_image(theta):
        losses = []
        for i, (x, tg) in enumerate(zip(imgs, targets)):
            s = streams[i % len(streams)]
            s.wait_stream(stream)
            with torch.cuda.stream(s):
                u, _ = simulate(x, theta, T, "zeroflux", grads=grads)
                losses.append(((u - tg) ** 2).mean() / n_img)
        for s in streams:
            stream.wait_stream(s)
        total = torch.stack(losses).sum()
        total.backward()
        return float(total)

    losses, times = [], []
    for _ in range(iters):
        opt.zero_grad()
        t0 = time.perf_counter()
        losses.append(batched(theta_of(p)))
        stream.synchronize()
        times.append(time.perf_counter() - t0)
        opt.step()
        with torch.no_grad():
            p[0].clamp_(0.0, 2.4)
            p[1].clamp_(0.0, 2.4)
            p[2].clamp_(1e-3, 1.0)
    t = min(times)
    q = p.detach().clone().requires_grad_(True)
    per_image(theta_of(q))  # warm
    q.grad = None
    stream.synchronize()
    t0 = time.perf_counter()
    per_image(theta_of(q))
    stream.synchronize()
    t_img = time.perf_counter() - t0
    return {"workload": f"{n_img} images 1024x1024, T=50, fit Du, Dv, eps by Adam to Sobel targets",
            "loss_curve": losses, "params_final": {"Du": float(p[0]), "Dv": float(p[1]),
                                                   "epsilon": float(p[2])},
            "fwd_bwd_gcells": n_img * N * N * T / t / 1e9, "iter_s": t,
            "per_image_streams_gcells": n_img * N * N * T / t_img / 1e9,
            "batched_vs_per_image": t_img / t}


# Table I of the paper: PyCUDA on a Tesla P100-PCIE, 10^4 iterations of the
# default gene, Mcells/s per grid side.
PAPER_TABLE1_PYCUDA = {128: 470, 256: 1941, 512: 7581, 1024: 13059, 2048: 14198, 4096: 14545}


def bench_paper_table1(stream, nsnp=5):
    """The paper's Table I workload: the default gene (a=-0.3, b=1.3, eps=-0.1,
    c=1, k3=1/3, Du=0.06, Dv=1, dt=0.1), periodic boundary, random 11x11 centre
    patch, 10^4 iterations, N = 128 ... 4096, with the paper's main-loop
    snapshots: nsnp = 5 snapshots, one every test_mod = 10^4 / 5 iterations,
    kept in device memory (Sec. II.B main loop; the paper copies them to the
    host).  Mcells/s (snapshots included) next to the paper's PyCUDA figures
    (P100)."""
    import torch
    from paper_2102_10340_amd import Simulation
    T = 10000
    test_mod = T // nsnp
    out = {"snapshots": nsnp, "test_mod": test_mod}
    for N, ref in PAPER_TABLE1_PYCUDA.items():
        x = torch.from_numpy(W.centre_patch_x(N, N, 11, 0)).cuda()
        sim = Simulation(x, W.gene(W.PAPER_DEFAULT_GENE), "periodic")
        snaps = torch.empty((nsnp + 1, 2, N, N), dtype=torch.float32, device="cuda")

        def job():
            sim.read_into(snaps[0, 0], snaps[0, 1])
            for k in range(nsnp):
                sim.step(test_mod)
                sim.read_into(snaps[k + 1, 0], snaps[k + 1, 1])

        sim.step(200)
        t = _timed(job, stream)
        sim.close()
        rate = N * N * T / t / 1e6
        out[str(N)] = {"mcells_s": rate, "s": t, "paper_pycuda_p100_mcells_s": ref,
                       "ratio": rate / ref}
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(fn, cells_per_step, budget_s, max_steps=2000):
    """Cell-updates/s of fn(n) (n oracle steps), n sized to about budget_s."""
    t0 = time.perf_counter()
    fn(2)
    per = (time.perf_counter() - t0) / 2
    n = int(max(2, min(max_steps, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    fn(n)
    dt = time.perf_counter() - t0
    return cells_per_step * n / dt, n


def cpu_baseline(budget_s: float):
    """The oracle (plain C loops, float32, OpenMP over rows) on a bounded sample
    of the same workload: the 4096x4096 slow-growth grid and initial state, for
    as many steps as fit the budget, on all the host's OpenMP threads and on
    one thread."""
    import oracle
    x = W.centre_patch_x(R, C, 16, 0)
    u, v = oracle.init_state(x, 1.0)
    nthr = oracle.num_threads()

    def run(n):
        oracle.run(u, v, W.PLAIN_GENE, "zeroflux", n, "f32")

    rate, n = _oracle_rate(run, R * C, budget_s * 0.7)
    oracle.set_num_threads(1)
    try:
        rate1, n1 = _oracle_rate(run, R * C, budget_s * 0.3)
    finally:
        oracle.set_num_threads(nthr)
    return {"value": rate / 1e9, "unit": "Gcell-updates/s", "cores": nthr, "kind": "oracle",
            "sample": f"4096x4096 slow-growth grid from the job's initial state, {n} steps "
                      f"(float32 oracle, {nthr} OpenMP threads)",
            "one_thread": {"value": rate1 / 1e9, "steps": n1}, "cpu_model": _cpu_model()}


def oracle_workloads(gpu_plain_state=None):
    """The oracle timed on the other workloads (all OpenMP threads): the plain
    method at full T (float32, plus the float64 run that states the float32
    drift), a 32-instance subset of the parameter sweep (200 steps each), and
    the differentiation workload's forward plus its float64 reverse pass."""
    import oracle
    out = {"cores": oracle.num_threads(), "cpu_model": _cpu_model()}
    # plain method, 256^2, T = 1000
    x = W.uniform_x(256, 256, 0)
    u0, v0 = oracle.init_state(x, 1.0)
    t0 = time.perf_counter()
    u32 = oracle.run(u0, v0, W.PLAIN_GENE, "zeroflux", 1000, "f32")
    t32 = time.perf_counter() - t0
    u64 = oracle.run(u0, v0, W.PLAIN_GENE, "zeroflux", 1000, "f64")
    drift = max(float(np.abs(u32[0] - u64[0]).max()), float(np.abs(u32[1] - u64[1]).max()))
    plain = {"gcells": 256 * 256 * 1000 / t32 / 1e9, "s": t32,
             "float32_vs_float64_drift_T1000": drift}
    if gpu_plain_state is not None:
        plain["gpu_equals_float32_oracle_bitwise"] = bool(
            np.array_equal(gpu_plain_state[0], u32[0]) and np.array_equal(gpu_plain_state[1], u32[1]))
    out["plain_256_T1000"] = plain
    # parameter sweep: the first 32 instances, 200 steps each
    inst = W.sweep_instances(1024, 0)[:32]
    T = 200
    t0 = time.perf_counter()
    cells = 0
    for d in inst:
        xi = W.uniform_x(d["rows"], d["cols"], d["seed"])
        oracle.run(*oracle.init_state(xi, 1.0), d["gene"], "zeroflux", T, "f32")
        cells += d["rows"] * d["cols"] * T
    ts = time.perf_counter() - t0
    out["sweep_32_instances_T200"] = {"gcells": cells / ts / 1e9, "s": ts}
    # differentiation workload: forward (float32) + float64 reverse pass
    N, T = 1024, 2000
    x = W.uniform_x(N, N, 0)
    tgt = W.stripe_target(N, N, 0)
    t0 = time.perf_counter()
    uT = oracle.run(*oracle.init_state(x, 1.0), W.PLAIN_GENE, "zeroflux", T, "f32")[0]
    tf = time.perf_counter() - t0
    lam = 2.0 * (uT.astype(np.float64) - tgt) / (N * N)
    t0 = time.perf_counter()
    oracle.grad(x, x, W.PLAIN_GENE, "zeroflux", T, lam, np.zeros_like(lam), traj="f32")
    tb = time.perf_counter() - t0
    out["differentiation_1024_T2000"] = {"fwd_s": tf, "fwd_gcells": N * N * T / tf / 1e9,
                                         "float64_reverse_pass_s": tb,
                                         "fwd_bwd_gcells": N * N * T / (tf + tb) / 1e9}
    return out


def copy_ceiling(dev) -> float:
    """Attainable HBM rate on this GPU: a plain 512 MiB device copy (torch's
    copy kernel), best of five, counting the bytes read and written."""
    import torch
    n = (512 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * n * 4 / (best / 1e3) / 1e9


def main():
    args = parse()
    plain_state = None
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the simulator runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2102_10340_amd import Simulation

    from paper_2102_10340_amd._lib import check, lib

    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    x = torch.from_numpy(W.centre_patch_x(R, C, 16, 0)).to(dev)
    chunk = args.chunk
    snaps = torch.empty((args.steps + 1, 2, R, C), dtype=torch.float32, device=dev)

    warm = Simulation(x, W.PLAIN_GENE, "zeroflux", 1.0)
    for _ in range(args.warmup):
        warm.step(chunk)
    torch.cuda.synchronize()
    warm.close()

    # The timed job starts from the initial state; snapshot 0 is s_0.
    sim = Simulation(x, W.PLAIN_GENE, "zeroflux", 1.0)
    shape = sim.pass_config()  # the autotuner's cached shape for 4096^2, else the library's
    depth, cpl = shape["depth"], shape["cols_per_lane"]
    check(lib.rdcnn_read(sim._h, snaps[0, 0].data_ptr(), snaps[0, 1].data_ptr(), 0))
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_host = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        sim.step(chunk)
        check(lib.rdcnn_read(sim._h, snaps[k + 1, 0].data_ptr(), snaps[k + 1, 1].data_ptr(), 0))
    ev1.record()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = ev0.elapsed_time(ev1)
    steps_total = args.steps * chunk
    rate = R * C * steps_total / (ms / 1e3)  # cell-updates / s
    launches = args.steps * (-(-chunk // depth))
    launch_s = ms / 1e3 / launches  # upper bound: includes the snapshot copies
    cells_per_launch = R * C * depth
    tflops = FLOPS_PER_CELL_UPDATE * cells_per_launch / launch_s / 1e12
    eff_gbs = BYTES_PER_CELL_UPDATE * cells_per_launch / launch_s / 1e9
    alive = float(snaps[-1, 0].abs().max())
    traffic = measured_traffic(f"void rd::stream_step_kernel<{cpl}, {depth}, 0>")
    pass_min = 16 * R * C  # one read and one write of the state per pass

    out = {
        "metric": "Gcell-updates/s FP32 forward (slow-growth 4096^2) + % of HBM roofline",
        "value": rate / 1e9,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slow-growth 4096x4096 zero-flux, 16x16 random centre patch, "
                               "dt=0.1 Du=0.05 Dv=1 f1=u-u^3-v f2=0.1(u-v), T=10000 per step + "
                               "device snapshot", "time_steps_per_step": chunk,
                   "grid": [R, C], "kernel": f"stream_step_kernel<{cpl},{depth},0>",
                   "pass_shape": shape,
                   "pass_shape_from": sim.tuned_from or "library default",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": ALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / ALU_PEAK_TFLOPS, "traffic": traffic,
                     "basis": f"{FLOPS_PER_CELL_UPDATE} algorithmic flops per cell-update x "
                              f"R*C*{depth} cell-updates per launch / mean launch time (HIP events "
                              "over the timed region, snapshot copies included)",
                     "peak_nonpacked": ALU_NONPACKED_TFLOPS,
                     "frac_nonpacked": tflops / ALU_NONPACKED_TFLOPS,
                     "issue": {"valu_instructions_per_cell_update": VALU_OPS_PER_CELL_UPDATE,
                               "achieved_tops": VALU_OPS_PER_CELL_UPDATE * cells_per_launch
                               / launch_s / 1e12,
                               "peak_tops": VALU_PEAK_TOPS,
                               "frac": VALU_OPS_PER_CELL_UPDATE * cells_per_launch / launch_s
                               / 1e12 / VALU_PEAK_TOPS},
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated); null if the kernel changed since",
                     "measured_hbm": None if traffic is None else {
                         "gbs": traffic / launch_s / 1e9,
                         "frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS,
                         "traffic_over_pass_minimum": traffic / pass_min,
                         "pass_minimum_bytes": pass_min},
                     "effective_hbm": {"basis": "16 B per cell-update (the naive step's traffic)",
                                       "gbs": eff_gbs, "frac": eff_gbs / HBM_PEAK_GBS}},
        "host_wall_s": t_host,
        "final_max_abs_u": alive,
    }
    sim.close()
    # (not in counter runs: their calibration copies must stay the largest)
    if args.copy_calibration == 0:
        copy_gbs = copy_ceiling(dev)
        out["roofline"]["copy_ceiling"] = {
            "basis": "best of 5 device-to-device copies of 512 MiB (read + write bytes / time)",
            "gbs": copy_gbs, "frac_of_peak": copy_gbs / HBM_PEAK_GBS}
        if out["roofline"]["measured_hbm"] is not None:
            out["roofline"]["measured_hbm"]["frac_of_copy"] = (
                out["roofline"]["measured_hbm"]["gbs"] / copy_gbs)
    if not args.no_extra:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            if args.only_extra in (None, "fwd_bwd"):
                out["fwd_bwd"] = bench_fwd_bwd(stream)
            if args.only_extra in (None, "batched"):
                out["batched"] = bench_batched(stream)
            if args.only_extra in (None, "small_batch"):
                out["small_batch"] = bench_small_batch(stream)
            if args.only_extra in (None, "atlas"):
                out["atlas"] = bench_atlas(stream)
            if args.only_extra in (None, "models"):
                out["models"] = bench_models(stream)
            if args.only_extra in (None, "plain"):
                out["plain"], plain_state = bench_plain(stream)
            if args.only_extra in (None, "edge"):
                out["edge_fit"] = bench_edge_fit(stream)
            if args.only_extra in (None, "table1"):
                out["paper_table1"] = bench_paper_table1(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        if not args.no_extra and args.only_extra is None:
            out["cpu_baseline"]["workloads"] = oracle_workloads(plain_state)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
