"""Autotuner: cache keys, candidate lists and the JSON round trip (CPU), and a
small tuning run whose chosen settings keep the results bit-exact (GPU)."""
import json

import numpy as np
import pytest


def test_candidates_respect_depth_limits():
    from paper_2102_10340_amd import tune
    for mode in ("forward", "record", "adjoint", "batch", "record_even", "adjoint_even"):
        c = tune.candidates(mode, 1024, 1024)
        assert c and len(set(c)) == len(c)
        lim = tune.MAX_ADJ_DEPTH if mode == "adjoint" else tune.MAX_DEPTH
        assert all(1 <= d <= lim[cpl] and cpl in (1, 2, 4) and s >= 0 for d, cpl, s in c)
        if mode.endswith("_even"):  # paired passes and even recording: even depths <= 8, <= 2 columns
            assert all(d % 2 == 0 and d <= 8 and cpl <= 2 for d, cpl, _ in c)
    # narrow grids do not try strips much wider than themselves
    assert all(cpl == 1 for _, cpl, _ in tune.candidates("forward", 64, 16))


def test_cache_round_trip(tmp_path, monkeypatch):
    from paper_2102_10340_amd import tune
    path = tmp_path / "t.json"
    monkeypatch.setenv("RDCNN_TUNE_CACHE", str(path))
    tune.save({"a/forward/8x8/zeroflux": {"depth": 4, "cols_per_lane": 2, "seg_rows": 0, "gcells": 1.0}})
    tune.save({"a/adjoint/8x8/zeroflux": {"depth": 2, "cols_per_lane": 1, "seg_rows": 8, "gcells": 2.0}})
    data = json.load(open(path))
    assert set(data) == {"a/forward/8x8/zeroflux", "a/adjoint/8x8/zeroflux"}
    assert tune.lookup("a/adjoint/8x8/zeroflux") == (2, 1, 8)
    assert tune.lookup("missing") is None
    assert tune.batch_key([(2, 3), (4, 5), (2, 3)], "periodic").endswith("/batch/2x3*2,4x5*1/periodic")


def test_shipped_cache_is_valid():
    from paper_2102_10340_amd import tune
    for k, e in tune.load(tune.SHIPPED).items():
        mode = k.split("/")[1]
        lim = tune.MAX_ADJ_DEPTH if mode == "adjoint" else tune.MAX_DEPTH
        assert e["cols_per_lane"] in (1, 2, 4) and 1 <= e["depth"] <= lim[e["cols_per_lane"]], k
        for cls, h in e.get("class_seg_rows", {}).items():  # per size class rows per tile
            r, c = (int(v) for v in cls.split("x"))
            assert mode == "batch" and f"{r}x{c}*" in k and h > 0, (k, cls)


@pytest.mark.gpu
def test_tuned_settings_stay_bitwise(tmp_path, monkeypatch):
    import torch
    import oracle
    import workloads as W
    from paper_2102_10340_amd import Simulation, tune
    monkeypatch.setenv("RDCNN_TUNE_CACHE", str(tmp_path / "t.json"))
    best, res = tune.tune("forward", 96, 200, "zeroflux", budget_s=5.0)
    assert best in res and all(v > 0 for v in res.values())
    x = W.uniform_x(96, 200, 2)
    sim = Simulation(torch.from_numpy(x).cuda(), W.PLAIN_GENE, "zeroflux")
    assert sim.tuned_from == tune.key("forward", 96, 200, "zeroflux")  # applied on construction
    assert tune.apply(sim)
    sim.step(30)
    u, v = sim.read_host()
    sim.close()
    ou, ov = oracle.run(*oracle.init_state(x, 1.0), W.PLAIN_GENE, "zeroflux", 30, "f32")
    assert np.array_equal(u, ou) and np.array_equal(v, ov)


@pytest.mark.gpu
def test_tuned_gradient_settings_keep_the_adjoint(tmp_path, monkeypatch):
    """Tuning the even recording and the paired adjoint, then applying them with
    grad=True, leaves dJ/ds bit-identical to the default settings (the per-cell
    arithmetic does not depend on the pass shape)."""
    import torch
    import workloads as W
    from paper_2102_10340_amd import Simulation, tune
    monkeypatch.setenv("RDCNN_TUNE_CACHE", str(tmp_path / "t.json"))
    R, C, T = 96, 200, 21
    for mode in ("record_even", "adjoint_even"):
        best, res = tune.tune(mode, R, C, "zeroflux", budget_s=3.0)
        assert best in res and all(v > 0 for v in res.values())
    x = torch.from_numpy(W.uniform_x(R, C, 5)).cuda()
    w = torch.from_numpy(np.random.default_rng(5).standard_normal((2, R, C)).astype(np.float32)).cuda()
    out = []
    for tuned in (False, True):
        sim = Simulation(x, W.PLAIN_GENE, "zeroflux")
        if tuned:
            assert tune.apply(sim, grad=True)
        st = torch.empty(((T + 1) // 2, 2, R, C), device="cuda")
        sim.step_record_even(T, st)
        adj = w.clone()
        sim.adjoint_even(st, T, adj, torch.empty_like(adj), torch.zeros(8, dtype=torch.float64, device="cuda"))
        out.append((st.clone(), adj))
        sim.close()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


@pytest.mark.gpu
def test_batch_class_tuning_stays_bitwise(tmp_path, monkeypatch):
    """Tuning a mix of sizes picks a batch-wide shape and rows per tile per size
    class; a Batch of that mix takes them on construction, and its states equal
    an untuned batch's and the float32 oracle's bit for bit."""
    import torch
    import oracle
    import workloads as W
    from paper_2102_10340_amd import Batch, tune
    monkeypatch.setenv("RDCNN_TUNE_CACHE", str(tmp_path / "t.json"))
    shapes = [(300, 260), (300, 260), (160, 410), (520, 200), (300, 260)]
    xs_np = [W.uniform_x(r, c, 11 + i) for i, (r, c) in enumerate(shapes)]
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    genes = [W.gene(Du=0.05 + 0.01 * i, Dv=0.5) for i in range(len(shapes))]
    best, res = tune.tune_batch(xs, genes, "zeroflux", steps=24, budget_s=8.0)
    e = tune.load()[tune.batch_key(shapes, "zeroflux")]
    assert (e["depth"], e["cols_per_lane"], e["seg_rows"]) == best
    assert set(e["class_seg_rows"]) <= {"300x260", "160x410", "520x200"}
    tuned = Batch(xs, genes, "zeroflux")
    assert tuned.tuned_from == tune.batch_key(shapes, "zeroflux")
    plain = Batch(xs, genes, "zeroflux", tuned=False)
    assert plain.tuned_from is None
    T = 27
    tuned.step(T)
    plain.step(T)
    for i, x in enumerate(xs_np):
        assert torch.equal(tuned.state(i), plain.state(i)), i
        ou, ov = oracle.run(*oracle.init_state(x, 1.0), genes[i], "zeroflux", T, "f32")
        st = tuned.state(i).cpu().numpy()
        assert np.array_equal(st[0], ou) and np.array_equal(st[1], ov), i
    tuned.close()
    plain.close()
