"""Autotuner for the pass shape of the streamed kernels.

For a grid shape and a mode -- "forward" (rdcnn_step), "record"
(rdcnn_step_record), "record_even" (rdcnn_step_record_even), "adjoint"
(rdcnn_adjoint), "adjoint_even" (rdcnn_adjoint_even, the paired passes) or
"batch" (rdcnn_batch_step over a given mix of instance sizes) -- it times
candidate settings

    depth          time steps per HBM pass
    cols_per_lane  1, 2 or 4 adjacent columns per lane (strip = 64 * cols)
    seg_rows       output rows per wavefront (0 = the library's choice)

with HIP events on the current stream and keeps the fastest.  For a batch it
then times, one size class at a time (largest total cells first), the rows
per tile of that class with the others fixed (rdcnn_batch_set_class_seg_rows):
steps per pass and columns per lane are per launch, and one launch covers
every class.  Every setting gives bit-identical states (the forward) or the
same adjoint up to float32 summation order, so tuning only changes speed.
Results are cached in a JSON file keyed by GPU architecture, mode, size and
boundary rule; ``apply`` sets a cached choice on a Simulation (for plain runs,
or for the even recording and paired adjoint that gradients use) or a Batch.
Simulation and Batch apply the cached forward / batch entry themselves when
constructed (``tuned=True``).

The package ships ``tuned.json`` with results measured on an MI355X for the
benchmark shapes; ``RDCNN_TUNE_CACHE`` names another file.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from .sim import Simulation

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
MAX_DEPTH = {1: 16, 2: 16, 4: 12}
MAX_ADJ_DEPTH = {1: 8, 2: 8, 4: 6}
EVEN_DEPTHS = (2, 4, 6, 8)  # even-time recording and paired passes: even depths, <= 2 columns
# A stable, non-trivial parameter set for timing (speed does not depend on it).
TUNE_GENE = dict(dt=0.1, a=0.0, b=1.0, eps=-0.1, c=1.0, k3=1.0, Du=0.05, Dv=1.0)


def cache_path() -> str:
    return os.environ.get("RDCNN_TUNE_CACHE", SHIPPED)


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key(mode: str, rows: int, cols: int, bc: str) -> str:
    return f"{_arch()}/{mode}/{rows}x{cols}/{bc}"


def batch_key(shapes, bc: str) -> str:
    hist = {}
    for r, c in shapes:
        hist[f"{r}x{c}"] = hist.get(f"{r}x{c}", 0) + 1
    desc = ",".join(f"{k}*{v}" for k, v in sorted(hist.items()))
    return f"{_arch()}/batch/{desc}/{bc}"


def load(path: str = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(entries: dict, path: str = None) -> None:
    path = path or cache_path()
    data = load(path)
    data.update(entries)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates(mode: str, rows: int, cols: int):
    out = []
    if mode in ("forward", "record", "batch"):
        for cpl in (1, 2, 4):
            if cpl > 1 and 64 * cpl > 2 * cols:
                continue  # strips much wider than the grid only add halo work
            for depth in (2, 4, 6, 8, 12, 16):
                if depth > MAX_DEPTH[cpl]:
                    continue
                for seg in ((0, 64, 128) if mode == "batch" else (0, 4, 8, 16, 32)):
                    out.append((depth, cpl, seg))
    elif mode == "adjoint":
        for cpl in (1, 2, 4):
            for depth in (2, 3, 4, 6, 8):
                if depth > MAX_ADJ_DEPTH[cpl]:
                    continue
                for seg in (0, 8):
                    out.append((depth, cpl, seg))
    elif mode in ("record_even", "adjoint_even"):
        segs = (0, 4, 6, 8, 16, 32) if mode == "record_even" else (0, 4, 5, 6, 8)
        for cpl in (1, 2):
            if cpl > 1 and 64 * cpl > 2 * cols:
                continue
            for depth in EVEN_DEPTHS:
                for seg in segs:
                    out.append((depth, cpl, seg))
    else:
        raise ValueError(mode)
    return out


def _timer(stream):
    def run(fn, reps=2):
        fn()
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3
    return run


def _steps_for(cells: int) -> int:
    # about 2e9 cell-updates per timed call, at least 16 steps
    return int(max(16, min(2000, 2e9 // max(cells, 1))))


def tune(mode: str, rows: int, cols: int, bc: str = "zeroflux", gene=None, budget_s: float = 60.0,
         write: bool = True, verbose: bool = False):
    """Time the candidates for one grid shape on a random U[-1,1] grid; returns
    (best, {setting: Gcell/s})."""
    gene = gene or TUNE_GENE
    stream = torch.cuda.current_stream()
    run = _timer(stream)
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand((rows, cols), generator=gen, device="cuda", dtype=torch.float32) * 2 - 1
    sim = Simulation(x, gene, bc, tuned=False)
    T = _steps_for(rows * cols)
    results = {}
    t_end = time.time() + budget_s
    S = min(T, 64)
    even = mode in ("record_even", "adjoint_even")
    if mode in ("record", "record_even", "adjoint", "adjoint_even"):
        states = torch.empty(((S + 1) // 2 if even else S, 2, rows, cols), dtype=torch.float32,
                             device="cuda")
    if mode in ("adjoint", "adjoint_even"):
        (sim.step_record_even if even else sim.step_record)(S, states)
        adj = torch.randn((2, rows, cols), device="cuda")
        tmp = torch.empty_like(adj)
        dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    for cand in candidates(mode, rows, cols):
        if time.time() > t_end:
            break
        depth, cpl, seg = cand
        if mode == "forward":
            sim.set_kernel(2, depth, cpl, seg)
            t = run(lambda: sim.step(T))
            rate = rows * cols * T / t / 1e9
        elif mode in ("record", "record_even"):
            sim.set_kernel(2, depth, cpl, seg)
            rec = sim.step_record_even if even else sim.step_record
            t = run(lambda: rec(S, states))
            rate = rows * cols * S / t / 1e9
        else:
            sim.set_adjoint_kernel(depth, cpl, seg)
            adjf = sim.adjoint_even if even else sim.adjoint
            t = run(lambda: adjf(states, S, adj, tmp, dth))
            rate = rows * cols * S / t / 1e9
        results[cand] = rate
        if verbose:
            print(mode, rows, cols, cand, f"{rate:.1f} Gcell/s", flush=True)
    sim.close()
    best = max(results, key=results.get)
    if write:
        save({key(mode, rows, cols, bc): {"depth": best[0], "cols_per_lane": best[1],
                                          "seg_rows": best[2], "gcells": results[best]}})
    return best, results


def tune_batch(xs, genes, bc: str = "zeroflux", steps: int = 240, budget_s: float = 120.0,
               write: bool = True, verbose: bool = False):
    """Time candidate batch settings for a mix of instances (tensors xs)."""
    from .batch import Batch
    stream = torch.cuda.current_stream()
    run = _timer(stream)
    b = Batch(xs, genes, bc, tuned=False)
    cells = sum(int(x.numel()) for x in xs)
    shapes = [tuple(int(v) for v in x.shape) for x in xs]
    side = int(np.sqrt(max(r * c for r, c in shapes)))
    results = {}
    t_end = time.time() + budget_s
    for cand in candidates("batch", side, side):
        if time.time() > t_end:
            break
        b.set_kernel(*cand)
        t = run(lambda: b.step(steps))
        results[cand] = cells * steps / t / 1e9
        if verbose:
            print("batch", cand, f"{results[cand]:.1f} Gcell/s", flush=True)
    best = max(results, key=results.get)
    b.set_kernel(*best)
    # rows per tile per size class, largest classes first, the others held
    counts = {}
    for r, c in shapes:
        counts[(r, c)] = counts.get((r, c), 0) + 1
    rate = results[best]
    class_seg = {}
    for (r, c) in sorted(counts, key=lambda k: -counts[k] * k[0] * k[1]):
        keep = 0
        for h in (16, 32, 64, 128, 256, 512):
            if h > r or h == best[2]:
                continue
            b.set_class_seg_rows(r, c, h)
            g = cells * steps / run(lambda: b.step(steps)) / 1e9
            if verbose:
                print("batch class", (r, c), "rows", h, f"{g:.1f} Gcell/s", flush=True)
            if g > rate * 1.01:  # keep a class height only for a clear gain
                keep, rate = h, g
        b.set_class_seg_rows(r, c, keep)
        if keep:
            class_seg[f"{r}x{c}"] = keep
    b.close()
    if write:
        save({batch_key(shapes, bc): {"depth": best[0], "cols_per_lane": best[1],
                                      "seg_rows": best[2], "class_seg_rows": class_seg,
                                      "gcells": rate}})
    return best, dict(results, class_seg_rows=class_seg, gcells=rate)


def lookup(k: str, path: str = None):
    e = load(path).get(k)
    return None if e is None else (e["depth"], e["cols_per_lane"], e["seg_rows"])


def apply(obj, path: str = None, grad: bool = False, modes=None):
    """Set the cached settings (if any) on a Simulation or a Batch; returns the
    cache key(s) applied ("+"-joined), or None.  For a Simulation, grad=False
    takes the "forward" and "adjoint" entries, grad=True the "record_even" and
    "adjoint_even" ones (what a gradient run uses); `modes` restricts that to
    the named ones.  A Batch takes its size mix's entry, with the rows per tile
    of each size class the tuner kept."""
    from .batch import Batch
    if _arch() == "unknown":
        return None
    if isinstance(obj, Batch):
        k = batch_key(obj.shapes, obj.bc)
        e = load(path).get(k)
        if e is None:
            return None
        obj.set_kernel(e["depth"], e["cols_per_lane"], e["seg_rows"])
        present = set(obj.shapes)
        for cls, h in e.get("class_seg_rows", {}).items():
            r, c = (int(v) for v in cls.split("x"))
            if (r, c) in present:
                obj.set_class_seg_rows(r, c, int(h))
        return k
    done = []
    for mode in (("record_even", "adjoint_even") if grad else ("forward", "adjoint")):
        if modes is not None and mode not in modes:
            continue
        k = key(mode, obj.rows, obj.cols, obj.bc)
        cfg = lookup(k, path)
        if not cfg:
            continue
        if mode == "forward":  # plain steps only: recording keeps its own shapes
            obj.set_kernel(3, *cfg)
        elif mode == "record_even":
            obj.set_kernel(2, *cfg)
        else:
            obj.set_adjoint_kernel(*cfg)
        done.append(k)
    return "+".join(done) if done else None


if __name__ == "__main__":
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="tune pass shapes and update the cache")
    ap.add_argument("--mode", default="forward",
                    choices=["forward", "record", "record_even", "adjoint", "adjoint_even",
                             "batch-sweep", "bench"])
    ap.add_argument("--size", type=int, nargs="+", default=[4096, 1024, 256])
    ap.add_argument("--bc", default="zeroflux")
    ap.add_argument("--budget", type=float, default=60.0)
    ap.add_argument("--cache", default=None)
    a = ap.parse_args()
    if a.cache:
        os.environ["RDCNN_TUNE_CACHE"] = a.cache
    if a.mode == "bench":
        # the shapes the benchmark runs: the forward of every grid side it times
        # one at a time (headline, differentiation, per-instance baselines) and
        # the 1024-instance parameter-sweep mix
        for n in (4096, 1024, 512, 256, 128):
            best, res = tune("forward", n, n, a.bc, budget_s=a.budget)
            print("forward", n, "best", best, f"{res[best]:.1f} Gcell/s", flush=True)
        # and the paper's Table I sweep (periodic grids, N = 128 ... 4096)
        for n in (4096, 2048, 1024, 512, 256, 128):
            best, res = tune("forward", n, n, "periodic", budget_s=a.budget)
            print("forward periodic", n, "best", best, f"{res[best]:.1f} Gcell/s", flush=True)
        a.mode = "batch-sweep"
    if a.mode == "batch-sweep":
        # the 1024-instance parameter-sweep workload (seeded synthetic inputs)
        import workloads as W
        inst = W.sweep_instances(1024, 0)
        xs = [torch.from_numpy(W.uniform_x(d["rows"], d["cols"], d["seed"])).cuda() for d in inst]
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            best, res = tune_batch(xs, [d["gene"] for d in inst], a.bc, budget_s=a.budget)
        print("batch-sweep best", best, "class rows", res["class_seg_rows"],
              f"{res['gcells']:.1f} Gcell/s", flush=True)
    else:
        for n in a.size:
            best, res = tune(a.mode, n, n, a.bc, budget_s=a.budget)
            print(a.mode, n, "best", best, f"{res[best]:.1f} Gcell/s", flush=True)
