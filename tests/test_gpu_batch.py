"""GPU parity of the batched path: every instance of a batch (uneven sizes,
per-instance parameters) is bit-identical to the same grid run alone and to the
float32 oracle; graph replay equals eager launches on every replay."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _single(x, g, bc, T):
    from paper_2102_10340_amd import Simulation
    sim = Simulation(torch.from_numpy(x).cuda(), g, bc)
    sim.step(T)
    out = sim.read_host()
    sim.close()
    return out


def _mixed(seed, n=11):
    rng = np.random.default_rng(seed)
    shapes = [(1, 1), (3, 7), (130, 17), (64, 64), (257, 300), (128, 128), (37, 513), (2, 600),
              (300, 5), (511, 129), (96, 256)][:n]
    xs, genes = [], []
    for i, (R, C) in enumerate(shapes):
        xs.append(W.uniform_x(R, C, 1000 + i))
        genes.append(W.gene(Du=rng.uniform(0.01, 0.2), Dv=rng.uniform(0.2, 1.0),
                            eps=-rng.uniform(0.02, 0.2)))
    return xs, genes


@pytest.mark.parametrize("kernel", [None, (8, 4, 0), (4, 2, 16), (3, 4, 5), (16, 2, 200),
                                    (6, 1, 32)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_batch_instances_bitwise(bc, kernel):
    from paper_2102_10340_amd import Batch
    xs, genes = _mixed(3)
    b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
    if kernel is not None:
        b.set_kernel(*kernel)
    T = 29
    b.step(11).step(18)
    torch.cuda.synchronize()
    for i, (x, g) in enumerate(zip(xs, genes)):
        st = b.state(i).cpu().numpy()
        ou, ov = oracle.run(*oracle.init_state(x, 1.0), g, bc, T, "f32")
        assert np.array_equal(st[0], ou) and np.array_equal(st[1], ov), (i, x.shape)
    b.close()


def test_batch_graph_replays_match_eager():
    """Graph capture of a 20-step run, replayed four times with eager work and
    synchronizations in between; every replay equals the eager result."""
    from paper_2102_10340_amd import Batch
    xs, genes = _mixed(5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = Batch([torch.from_numpy(x).cuda() for x in xs], genes, "zeroflux")
        graph = Batch([torch.from_numpy(x).cuda() for x in xs], genes, "zeroflux")
        graph.use_graph(True)
        for rep in range(4):
            eager.step(20)
            graph.step(20)
            junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work
            s.synchronize()
            for i in range(len(xs)):
                assert torch.equal(eager.state(i), graph.state(i)), (rep, i)
            del junk
        eager.close()
        graph.close()


def test_batch_rejects_bad_layouts():
    import ctypes
    from paper_2102_10340_amd import _lib
    L = _lib.lib
    h = ctypes.c_void_p()
    rows = (ctypes.c_int * 2)(4, 4)
    cols = (ctypes.c_int * 2)(4, 4)
    pars = (_lib.Params * 2)(_lib.Params.from_mapping(W.PLAIN_GENE), _lib.Params.from_mapping(W.PLAIN_GENE))
    xo = (ctypes.c_longlong * 2)(0, 16)
    buf = torch.empty(256, device="cuda")
    buf2 = torch.empty(256, device="cuda")
    x = torch.zeros(32, device="cuda")
    for offs, total in [((0, 16), 256), ((0, 32), 256), ((0, 64), 64), ((-64, 64), 256)]:
        o = (ctypes.c_longlong * 2)(*offs)
        rc = L.rdcnn_batch_create(ctypes.byref(h), 2, rows, cols, o, pars, 1, x.data_ptr(), xo, 1.0,
                                  buf.data_ptr(), buf2.data_ptr(), total, None)
        assert rc == _lib.EINVAL, offs


def test_parameter_sweep_workload_sampled():
    """The sweep workload at full size: 1024 instances, sides uniform over
    {128, 256, 512, 1024}, Du ~ U[0.01,0.2], Dv ~ U[0.2,1], epsilon ~ U[0.02,0.2],
    zero-flux, x ~ U[-1,1] per instance, T = 5000, in one batch.  Sixteen
    instances are re-run alone on the GPU (bitwise), six small and medium ones
    are checked against the float32 oracle at full T."""
    from paper_2102_10340_amd import Batch
    inst = W.sweep_instances(1024, 0)
    xs = [torch.from_numpy(W.uniform_x(d["rows"], d["cols"], d["seed"])).cuda() for d in inst]
    b = Batch(xs, [d["gene"] for d in inst], "zeroflux")
    T = 5000
    b.step(T)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    for i in rng.choice(len(inst), 16, replace=False):
        d = inst[i]
        got = b.state(int(i)).cpu().numpy()
        ref = _single(xs[i].cpu().numpy(), d["gene"], "zeroflux", T)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), i
    picked = []
    for side in (128, 256, 512):
        picked += [i for i, d in enumerate(inst) if d["rows"] == side][:2]
    for i in picked:
        d = inst[i]
        got = b.state(i).cpu().numpy()
        ou, ov = oracle.run(*oracle.init_state(xs[i].cpu().numpy(), 1.0), d["gene"], "zeroflux", T, "f32")
        assert np.array_equal(got[0], ou) and np.array_equal(got[1], ov), i
    b.close()


# Shapes around the in-LDS limits: one row or column, C up to 1024 threads,
# up to 16 rows per thread, 128x128 (the largest square), and two just past
# the limits (129x129: 19 rows per thread; 40x600: 40 rows per thread).
LDS_SHAPES = [(1, 1), (1, 2), (2, 1), (1, 7), (7, 1), (3, 5), (17, 33), (64, 64), (100, 100),
              (128, 128), (2, 1000), (1, 1024), (200, 40), (129, 129), (40, 600)]


def _lds_frame_bytes(R, C):
    """Frame the in-LDS kernel needs, or None if the shape is not taken."""
    if C > 1024:
        return None
    runs = 1024 // C
    m = -(-R // runs)
    return None if m > 16 else (runs * m + 2) * (C + 2) * 8


@pytest.mark.parametrize("T,depth", [(1, 8), (23, 8), (24, 8), (37, 5)], ids=lambda v: str(v))
@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_in_lds_instances_bitwise(bc, T, depth):
    """Small instances held whole in LDS for all T steps: bit-identical to the
    float32 oracle and to the streamed kernel (use_lds off), with odd and even
    numbers of streamed passes (the in-LDS result goes to the buffer that is
    current afterwards)."""
    from paper_2102_10340_amd import Batch
    rng = np.random.default_rng(T)
    xs, genes = [], []
    for i, (R, C) in enumerate(LDS_SHAPES):
        xs.append(W.uniform_x(R, C, 77 + i))
        genes.append(W.gene(W.PAPER_DEFAULT_GENE, Du=rng.uniform(0.01, 0.2))
                     if bc == "periodic" else
                     W.gene(Du=rng.uniform(0.01, 0.2), Dv=rng.uniform(0.2, 1.0),
                            eps=-rng.uniform(0.02, 0.2)))
    dev = [torch.from_numpy(x).cuda() for x in xs]
    a = Batch(dev, genes, bc)
    a.set_kernel(depth, 2, 0)
    n_lds = a.lds_instances()
    small = sum(1 for s in LDS_SHAPES if (_lds_frame_bytes(*s) or 1 << 30) <= 64 * 1024)
    takeable = sum(1 for s in LDS_SHAPES if _lds_frame_bytes(*s) is not None)
    print(f"in-LDS instances {n_lds} of {len(LDS_SHAPES)} (at least {small}, at most {takeable})",
          flush=True)
    assert small <= n_lds <= takeable
    b = Batch(dev, genes, bc)
    b.set_kernel(depth, 2, 0)
    b.use_lds(False)
    assert b.lds_instances() == 0
    a.step(T)
    b.step(T)
    torch.cuda.synchronize()
    for i, (x, g) in enumerate(zip(xs, genes)):
        sa, sb = a.state(i).cpu().numpy(), b.state(i).cpu().numpy()
        ou, ov = oracle.run(*oracle.init_state(x, 1.0), g, bc, T, "f32")
        assert np.array_equal(sa[0], ou) and np.array_equal(sa[1], ov), ("lds", i, x.shape)
        assert np.array_equal(sb[0], ou) and np.array_equal(sb[1], ov), ("streamed", i, x.shape)
    a.close()
    b.close()


def test_in_lds_only_batch_and_graph():
    """A batch whose instances all run in LDS (no streamed tiles at all), in
    chunks of steps, eager and replayed from a graph four times."""
    from paper_2102_10340_amd import Batch
    shapes = [(64, 64), (128, 128), (32, 96), (5, 1000), (128, 8)]
    xs = [W.uniform_x(R, C, 5 + i) for i, (R, C) in enumerate(shapes)]
    g = [W.PLAIN_GENE] * len(xs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = Batch([torch.from_numpy(x).cuda() for x in xs], g, "zeroflux")
        graph = Batch([torch.from_numpy(x).cuda() for x in xs], g, "zeroflux")
        graph.use_graph(True)
        if eager.lds_instances() != len(xs):
            pytest.skip(f"device LDS holds {eager.lds_instances()} of these instances")
        done = 0
        for rep in range(4):
            eager.step(13)
            graph.step(13)
            done += 13
            s.synchronize()
            for i, x in enumerate(xs):
                assert torch.equal(eager.state(i), graph.state(i)), (rep, i)
        for i, x in enumerate(xs):
            ou, ov = oracle.run(*oracle.init_state(x, 1.0), W.PLAIN_GENE, "zeroflux", done, "f32")
            st = eager.state(i).cpu().numpy()
            assert np.array_equal(st[0], ou) and np.array_equal(st[1], ov), i
        eager.close()
        graph.close()
