"""GPU parity of the forward path (Eq. (1)-(3), Sec. II.A) against the CPU oracle.

The GPU kernels and the float32 oracle follow the same rounding order, so the
bar is bit-for-bit equality (the stated tolerances of 1e-5 after 100 steps and
1e-3 after 1000 steps are checked as well).  The float64 oracle states the
float32 drift, the one anchor of the float32 trajectory that does not share
its rounding order; each workload's drift carries a bar about 2.5x above the
measured value:
  plain workload (256^2, seeds 0-2, both rules): <= 4.2e-5 after 100 steps
    (bar 1e-4, the "non-chaotic" reading: float32 within 1e-4 of float64),
    <= 9e-7 after 1000 (bar 3e-6);
  slow growth (4096^2): 1.4e-6 after 100 steps (bar 5e-6), 3.9e-4 after 1000
    (bar 1e-3: the growth front moves cells through the steep part of the
    cubic, where rounding shifts it measurably).
All inputs come from the seeded generators in ``workloads``.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

BCS = ("periodic", "zeroflux")
# max |float32 - float64| after T steps, per workload (T: bar)
PLAIN_DRIFT_BAR = {100: 1e-4, 1000: 3e-6}
SLOW_GROWTH_DRIFT_BAR = {100: 5e-6, 1000: 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401  (fails loudly if the library is missing)


def gpu_run(x, gene, bc, T, kernel=None, ka=1.0, chunks=None):
    from paper_2102_10340_amd import Simulation
    xt = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    sim = Simulation(xt, gene, bc, ka)
    if kernel is not None:
        sim.set_kernel(*kernel)
    for t in (chunks or [T]):
        sim.step(t)
    u, v = sim.read_host()
    sim.close()
    return u, v


def oracle_run(x, gene, bc, T, ka=1.0, precision="f32"):
    u0, v0 = oracle.init_state(x, ka)
    return oracle.run(u0, v0, gene, bc, T, precision)


def assert_bitwise(got, want, what=""):
    gu, gv = got
    wu, wv = want
    if not (np.array_equal(gu, wu) and np.array_equal(gv, wv)):
        du = np.abs(gu.astype(np.float64) - wu).max()
        dv = np.abs(gv.astype(np.float64) - wv).max()
        bad = np.argwhere(gu != wu)[:5]
        raise AssertionError(f"{what}: not bitwise; max|du|={du:.3g} max|dv|={dv:.3g} first={bad.tolist()}")


KERNELS = [
    (1, 0, 0, 0),   # one thread per cell
    (2, 8, 4, 0),   # streamed, 4 columns per lane, 8 steps per pass
    (2, 16, 2, 0),  # 2 columns per lane, 16 steps per pass
    (2, 3, 4, 5),   # short segments
    (2, 1, 2, 1),   # one row per segment, one step per pass
    (2, 12, 4, 7),
    (2, 5, 2, 3),
    (2, 4, 1, 0),   # one column per lane
    (2, 16, 1, 2),
]
# The last three have C % 4 == 0 and C >= 488, so with four columns per lane
# some strips lie wholly inside the grid and take the vector-load body (the
# body of the 4096^2 launch); the others reach it only partly or not at all.
SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (17, 33), (64, 64), (37, 257), (130, 515), (256, 256),
          (130, 516), (77, 1000), (300, 1024)]


def test_init_state_bitwise():
    x = W.uniform_x(37, 45, 3)
    u, v = gpu_run(x, W.PLAIN_GENE, "zeroflux", 0, ka=0.7)
    ou, ov = oracle.init_state(x, 0.7)
    assert_bitwise((u, v), (ou, ov), "init")


@pytest.mark.parametrize("kernel", KERNELS, ids=lambda k: "k%d_d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_small_grids_bitwise(shape, bc, kernel):
    R, C = shape
    x = W.uniform_x(R, C, R * 1000 + C)
    g = W.gene(W.PAPER_DEFAULT_GENE) if bc == "periodic" else W.PLAIN_GENE
    T = 23
    print(f"case shape={shape} bc={bc} kernel={kernel} T={T}", flush=True)
    assert_bitwise(gpu_run(x, g, bc, T, kernel), oracle_run(x, g, bc, T), f"{shape} {bc} {kernel}")


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_workload_parity(bc, seed):
    """256x256, T=100 and T=1000, dt=0.1, Du=0.05, Dv=1, f1=u-u^3-v,
    f2=0.1(u-v), x ~ U[-1,1]: bitwise against the float32 oracle, hence within
    the 1e-5 (T=100) and 1e-3 (T=1000) bars; the float64 drift is printed."""
    x = W.uniform_x(256, 256, seed)
    g = W.PLAIN_GENE
    for T in (100, 1000):
        got = gpu_run(x, g, bc, T)
        want = oracle_run(x, g, bc, T)
        assert_bitwise(got, want, f"plain T={T}")
        tol = 1e-5 if T == 100 else 1e-3
        assert np.abs(got[0] - want[0]).max() <= tol and np.abs(got[1] - want[1]).max() <= tol
        r64 = oracle_run(x, g, bc, T, precision="f64")
        drift = max(np.abs(got[0] - r64[0]).max(), np.abs(got[1] - r64[1]).max())
        print(f"plain bc={bc} seed={seed} T={T}: float32 vs float64 drift {drift:.3g}")
        assert drift <= PLAIN_DRIFT_BAR[T], (T, drift)


def test_step_chunks_compose_bitwise():
    x = W.uniform_x(100, 300, 5)
    g = W.PLAIN_GENE
    ref = gpu_run(x, g, "zeroflux", 61)
    assert_bitwise(gpu_run(x, g, "zeroflux", 61, chunks=[0, 7, 1, 20, 33]), ref, "chunks")
    assert_bitwise(ref, oracle_run(x, g, "zeroflux", 61), "oracle")


def test_denormals_are_kept():
    """IEEE denormals survive on the GPU exactly as on the host (no flush)."""
    x = np.full((8, 70), 3e-39, dtype=np.float32)
    x[3, 5] = 7e-40
    x[0, 0] = -1e-45
    g = W.gene(c=0.5, k3=1.0, eps=-0.01, Du=0.05, Dv=0.1)
    for bc in BCS:
        got = gpu_run(x, g, bc, 3)
        assert_bitwise(got, oracle_run(x, g, bc, 3), "denormal")
        assert np.any((got[0] != 0) & (np.abs(got[0]) < np.finfo(np.float32).tiny))


def test_write_state_and_set_params():
    from paper_2102_10340_amd import Simulation
    x = W.uniform_x(90, 130, 8)
    g1, g2 = W.PLAIN_GENE, W.gene(Du=0.12, Dv=0.6, eps=-0.05)
    sim = Simulation(torch.from_numpy(x).cuda(), g1, "periodic")
    sim.step(10)
    sim.set_params(g2)
    sim.step(15)
    got = sim.read_host()
    want = oracle.run(*oracle_run(x, g1, "periodic", 10), g2, "periodic", 15, "f32")
    assert_bitwise(got, want, "set_params")
    u0 = torch.from_numpy(W.uniform_x(90, 130, 9)).cuda()
    v0 = torch.from_numpy(W.uniform_x(90, 130, 10)).cuda()
    sim.write_state(u0, v0)
    sim.step(9)
    got = sim.read_host()
    want = oracle.run(u0.cpu().numpy(), v0.cpu().numpy(), g2, "periodic", 9, "f32")
    assert_bitwise(got, want, "write_state")
    st = sim.state()
    assert torch.equal(st[0].cpu(), torch.from_numpy(got[0]))
    sim.close()


def test_full_size_blocked_equals_reference_kernel():
    """4096x4096 (the slow-growth grid), random x: the default blocked pass
    configuration and the one-thread-per-cell kernel agree bit for bit."""
    x = W.uniform_x(4096, 4096, 1)
    g = W.PLAIN_GENE
    a = gpu_run(x, g, "zeroflux", 24)
    b = gpu_run(x, g, "zeroflux", 24, kernel=(1, 0, 0, 0))
    assert_bitwise(a, b, "4096 blocked vs reference")


def _window_oracle(x0u, x0v, gene, bc, T, cells):
    """Oracle value of selected cells after T steps, each from the smallest
    window that contains its dependence cone (T cells in every direction),
    clipped at the true grid edges where the boundary rule applies."""
    R, C = x0u.shape
    out = []
    for (i, j) in cells:
        r0, r1 = max(0, i - T - 1), min(R, i + T + 2)
        c0, c1 = max(0, j - T - 1), min(C, j + T + 2)
        u, v = oracle.run(x0u[r0:r1, c0:c1], x0v[r0:r1, c0:c1], gene, bc, T, "f32")
        out.append((u[i - r0, j - c0], v[i - r0, j - c0]))
    return out


def test_slow_growth_full_size_sampled():
    """Slow-growth workload at full size (4096x4096, zero-flux, 16x16 random
    centre patch), in the launch configuration the benchmark times: sampled
    cells after 300 steps equal the oracle's, computed cell by cell."""
    R = C = 4096
    x = W.centre_patch_x(R, C, 16, 0)
    g = W.PLAIN_GENE
    T = 300
    u, v = gpu_run(x, g, "zeroflux", T)
    lo, hi = W.patch_bounds(R, 16)
    cells = [(lo, lo), (lo + 7, hi - 1), (2048, 2048), (lo - 40, lo + 3), (hi + 60, hi + 60),
             (0, 0), (R - 1, 17), (1000, C - 1)]
    u0, v0 = oracle.init_state(x, 1.0)
    for (i, j), (ou, ov) in zip(cells, _window_oracle(u0, v0, g, "zeroflux", T, cells)):
        assert u[i, j] == ou and v[i, j] == ov, ((i, j), u[i, j], ou, v[i, j], ov)
    assert np.abs(u).max() > 0.1  # the patch is alive


def test_periodic_wraparound_sampled():
    """Periodic rule at a ragged size: cells near the wrap seams against the
    oracle run on the whole grid."""
    x = W.uniform_x(301, 517, 12)
    g = W.gene(W.PAPER_DEFAULT_GENE)
    assert_bitwise(gpu_run(x, g, "periodic", 40), oracle_run(x, g, "periodic", 40), "periodic ragged")


def _assert_full_grid(got, want, what, tol=None):
    assert_bitwise(got, want, what)
    if tol is not None:
        assert np.abs(got[0] - want[0]).max() <= tol and np.abs(got[1] - want[1]).max() <= tol


def _headline_kernels():
    """The pass shapes to check at 4096^2: the one the benchmark's Simulation
    takes (the autotuner's cached shape, else the library's automatic one) and
    the library's automatic one, four columns per lane and eight steps per
    pass (the shape whose strips inside the grid take the 16-byte vector loads
    and unmapped row offsets), once if they are the same."""
    from paper_2102_10340_amd import Simulation
    out = []
    for tuned in (True, False):
        sim = Simulation(torch.zeros((4096, 4096), device="cuda"), W.PLAIN_GENE, "zeroflux",
                         tuned=tuned)
        cfg = sim.pass_config()
        sim.close()
        if not tuned:
            assert (cfg["cols_per_lane"], cfg["depth"]) == (4, 8), cfg
        k = (2, cfg["depth"], cfg["cols_per_lane"], cfg["seg_rows"])
        if k not in out:
            out.append(k)
    return out


def test_slow_growth_headline_launch_whole_grid():
    """The slow-growth workload (4096x4096, zero-flux, 16x16 random centre
    patch) in the launch the benchmark times: every cell after 100 and after
    1000 steps equals the float32 oracle's bit for bit (so within 1e-5 and
    1e-3), and the float64 oracle states the drift, asserted below its bar."""
    from paper_2102_10340_amd import Simulation
    kernels = _headline_kernels()
    R = C = 4096
    g = W.PLAIN_GENE
    x = W.centre_patch_x(R, C, 16, 0)
    sims = [Simulation(torch.from_numpy(x).cuda(), g, "zeroflux", 1.0, tuned=False)
            for _ in kernels]
    for sim, k in zip(sims, kernels):
        sim.set_kernel(*k)
    u32, v32 = oracle.init_state(x, 1.0)
    u64, v64 = oracle.init_state(x, 1.0, np.float64)
    done = 0
    for T, tol in ((100, 1e-5), (1000, 1e-3)):
        u32, v32 = oracle.run(u32, v32, g, "zeroflux", T - done, "f32")
        u64, v64 = oracle.run(u64, v64, g, "zeroflux", T - done, "f64")
        for sim, k in zip(sims, kernels):
            print(f"case slow-growth 4096^2 T={T} kernel {k}", flush=True)
            sim.step(T - done)
            got = sim.read_host()
            _assert_full_grid(got, (u32, v32), f"slow growth T={T} {k}", tol)
            drift = max(np.abs(got[0] - u64).max(), np.abs(got[1] - v64).max())
            print(f"slow growth T={T}: float32 vs float64 drift {drift:.3g}", flush=True)
            assert drift <= SLOW_GROWTH_DRIFT_BAR[T], (T, drift)
        done = T
    assert np.abs(got[0]).max() > 0.1  # the patch is alive
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("bc", BCS)
def test_random_grid_headline_launch_whole_grid(bc):
    """4096x4096 with x ~ U[-1,1] over the whole grid, so every tile of the
    default launch (vector body, mapped edge strips and segments, both rules)
    carries live values: bitwise against the float32 oracle after 100 steps.
    Periodic uses the paper's gene (the Table I launch with a random image),
    zero-flux the plain gene."""
    x = W.uniform_x(4096, 4096, 11)
    g = W.gene(W.PAPER_DEFAULT_GENE) if bc == "periodic" else W.PLAIN_GENE
    want = oracle_run(x, g, bc, 100)
    for k in _headline_kernels():
        print(f"case random 4096^2 {bc} T=100 kernel {k}", flush=True)
        _assert_full_grid(gpu_run(x, g, bc, 100, k), want, f"random 4096 {bc} {k}", 1e-5)


def test_table1_launch_whole_grid():
    """The paper's Table I workload at its largest size (4096x4096, default
    gene, periodic, random 11x11 centre patch): the whole grid after 300
    steps equals the float32 oracle bit for bit."""
    x = W.centre_patch_x(4096, 4096, 11, 0)
    g = W.gene(W.PAPER_DEFAULT_GENE)
    print("case table1 4096^2 periodic T=300", flush=True)
    got = gpu_run(x, g, "periodic", 300)
    _assert_full_grid(got, oracle_run(x, g, "periodic", 300), "table1 4096")


def test_plain_only_kernel_setting():
    """rdcnn_set_kernel kind 3 sets the shape of plain steps (reported by
    rdcnn_pass_config as a streamed shape) and leaves results bit-identical,
    also for a recording call in between (which keeps its automatic shape)."""
    from paper_2102_10340_amd import Simulation
    R, C = 70, 300
    x = W.uniform_x(R, C, 12)
    sim = Simulation(torch.from_numpy(x).cuda(), W.PLAIN_GENE, "zeroflux", tuned=False)
    sim.set_kernel(3, 4, 2, 8)
    cfg = sim.pass_config()
    assert (cfg["kind"], cfg["depth"], cfg["cols_per_lane"], cfg["seg_rows"]) == (2, 4, 2, 8), cfg
    sim.step(9)
    st = torch.empty((6, 2, R, C), device="cuda")
    sim.step_record_even(11, st)
    sim.step(5)
    got = sim.read_host()
    sim.close()
    want = oracle_run(x, W.PLAIN_GENE, "zeroflux", 25)
    assert_bitwise(got, want, "kind 3")
