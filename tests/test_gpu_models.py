"""GPU parity of the further cell models on the streamed kernel
(rdcnn_model_create): Gray-Scott and the Chua-Yang CNN bit for bit against the
oracle's cell_models.c, and FitzHugh-Nagumo through the model entry point bit
for bit against the main kernels."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

BCS = ("periodic", "zeroflux")
GS = dict(dt=0.5, F=0.037, k=0.06, Du=0.2, Dv=0.1)
SHAPES = [(1, 1), (3, 5), (17, 33), (64, 64), (130, 515), (256, 256)]
KERNELS = [None, (2, 1, 1, 0), (2, 2, 2, 0), (2, 3, 1, 5), (2, 5, 2, 7), (2, 8, 1, 0), (2, 8, 2, 16)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _gs_init(R, C, seed):
    rng = np.random.default_rng(seed)
    u = np.ones((R, C), np.float32)
    v = np.zeros((R, C), np.float32)
    u += rng.uniform(-0.05, 0.05, (R, C)).astype(np.float32)
    r0, c0 = R // 3, C // 3
    u[r0:r0 + max(1, R // 4), c0:c0 + max(1, C // 4)] = 0.5
    v[r0:r0 + max(1, R // 4), c0:c0 + max(1, C // 4)] = 0.25
    v += rng.uniform(0, 0.05, (R, C)).astype(np.float32)
    return u, v


def _run(sim, T, kernel, chunks=None):
    if kernel is not None:
        sim.set_kernel(*kernel)
    for t in (chunks or [T]):
        sim.step(t)
    out = sim.read_host()
    sim.close()
    return out


# Gray-Scott is also instantiated four columns per lane wide; (40, 1024) has
# whole-width vector strips at that width.
GS_KERNELS = KERNELS + [(2, 8, 4, 0), (2, 3, 4, 5), (2, 4, 4, 0)]
GS_SHAPES = SHAPES + [(40, 1024)]


@pytest.mark.parametrize("kernel", GS_KERNELS, ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k[1:])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", GS_SHAPES, ids=lambda s: "%dx%d" % s)
def test_gray_scott_bitwise(shape, bc, kernel):
    from paper_2102_10340_amd import Simulation
    R, C = shape
    u0, v0 = _gs_init(R, C, R * 7 + C)
    T = 27
    print(f"case gray-scott shape={shape} bc={bc} kernel={kernel}", flush=True)
    got = _run(Simulation.gray_scott(_t(u0), _t(v0), bc=bc, **GS), T, kernel)
    want = oracle.gs_run(u0, v0, GS, bc, T)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (shape, bc, kernel)


SYM_A = [[0.1, 0.3, 0.1], [0.3, 1.5, 0.3], [0.1, 0.3, 0.1]]
ASYM_A = [[0.0, 0.4, -0.2], [0.7, 1.2, 0.1], [0.3, -0.5, 0.25]]
B = [[-0.3, 0.6, -0.1], [0.2, 2.0, -0.7], [0.5, 0.1, -0.4]]


@pytest.mark.parametrize("kernel", KERNELS, ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k[1:])
@pytest.mark.parametrize("A", [SYM_A, ASYM_A], ids=["symmetric", "asymmetric"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_cnn_bitwise(shape, bc, A, kernel):
    """Blocked passes under both rules for the symmetric template; the
    asymmetric one runs one step per pass at zero-flux edges."""
    from paper_2102_10340_amd import Simulation
    R, C = shape
    rng = np.random.default_rng(R * 13 + C)
    x0 = rng.uniform(-1.5, 1.5, (R, C)).astype(np.float32)
    img = rng.uniform(-1, 1, (R, C)).astype(np.float32)
    T, dt, z = 19, 0.1, -0.3
    print(f"case cnn shape={shape} bc={bc} kernel={kernel}", flush=True)
    got = _run(Simulation.cnn(_t(x0), _t(img), A, B, z, dt, bc), T, kernel)
    w = oracle.cnn_input(img, B, z, bc)
    want = oracle.cnn_run(x0, w, dt, A, bc, T)
    assert np.array_equal(got[1], w), "input layer"
    assert np.array_equal(got[0], want), (shape, bc, kernel)


def test_fhn_through_model_entry_point_bitwise():
    """FitzHugh-Nagumo via rdcnn_model_create equals the main kernels and the
    oracle bit for bit."""
    from paper_2102_10340_amd import Simulation
    u0 = W.uniform_x(90, 130, 1)
    v0 = W.uniform_x(90, 130, 2)
    g = W.PLAIN_GENE
    params = [g[k] for k in ("dt", "a", "b", "eps", "c", "k3", "Du", "Dv")]
    for bc in BCS:
        a = _run(Simulation.model("fitzhugh_nagumo", _t(u0), _t(v0), params, bc), 41, None)
        b = Simulation.from_state(_t(u0), _t(v0), g, bc)
        b.step(41)
        b = b.read_host()
        want = oracle.run(u0, v0, g, bc, 41, "f32")
        for x, y in ((a, b), (a, want)):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]), bc


def test_cnn_edge_extraction_textbook_result():
    """The Chua-Yang edge template on a 256x256 two-level image settles to the
    edge map (+1 where a +1 pixel has a -1 neighbour), bit for bit as the
    oracle."""
    from paper_2102_10340_amd import Simulation
    noisy, clean = W.rect_image(256, 256, 3)
    img = np.where(clean > 0, 1.0, -1.0).astype(np.float32)
    A = [[0, 0, 0], [0, 2, 0], [0, 0, 0]]
    Bt = [[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]
    T = 300
    got = _run(Simulation.cnn(_t(np.zeros_like(img)), _t(img), A, Bt, -1.0, 0.1, "zeroflux"), T, None)
    want = oracle.cnn_run(np.zeros_like(img), oracle.cnn_input(img, Bt, -1.0, "zeroflux"), 0.1, A,
                          "zeroflux", T)
    assert np.array_equal(got[0], want)
    pad = np.pad(img, 1, mode="edge")
    nbmin = np.min([pad[i:i + 256, j:j + 256] for i in range(3) for j in range(3)], axis=0)
    edge = (img > 0) & (nbmin < 0)
    y = np.clip(got[0], -1, 1)
    assert np.array_equal(y > 0.99, edge) and np.all(np.abs(y) > 0.99)


def test_gray_scott_full_size():
    """1024x1024 Gray-Scott, 200 steps, default pass settings: whole grid bit
    for bit against the oracle."""
    from paper_2102_10340_amd import Simulation
    u0, v0 = _gs_init(1024, 1024, 5)
    got = _run(Simulation.gray_scott(_t(u0), _t(v0), bc="periodic", **GS), 200, None)
    want = oracle.gs_run(u0, v0, GS, "periodic", 200)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_gray_scott_wide_strips_full_size():
    """3072x3072 Gray-Scott, 64 steps, default pass settings (four columns per
    lane from 3072^2 on): whole grid bit for bit against the oracle; the CNN
    asked for four columns runs two (its widest) and stays bitwise too."""
    from paper_2102_10340_amd import Simulation
    u0, v0 = _gs_init(3072, 3072, 9)
    sim = Simulation.gray_scott(_t(u0), _t(v0), bc="zeroflux", **GS)
    assert sim.pass_config()["cols_per_lane"] == 4
    got = _run(sim, 64, None)
    want = oracle.gs_run(u0, v0, GS, "zeroflux", 64)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    img = W.uniform_x(64, 300, 4)
    cnn = Simulation.cnn(_t(np.zeros_like(img)), _t(img), SYM_A, B, -0.5, 0.1, "zeroflux")
    cnn.set_kernel(2, 8, 4, 0)
    assert cnn.pass_config()["cols_per_lane"] == 2
    got = _run(cnn, 19, None)
    want = oracle.cnn_run(np.zeros_like(img), oracle.cnn_input(img, B, -0.5, "zeroflux"), 0.1, SYM_A,
                          "zeroflux", 19)
    assert np.array_equal(got[0], want)


def test_model_grids_reject_fhn_only_calls():
    from paper_2102_10340_amd import RDCNNError, Simulation
    u0, v0 = _gs_init(32, 32, 1)
    sim = Simulation.gray_scott(_t(u0), _t(v0), **GS)
    states = torch.empty((4, 2, 32, 32), device="cuda")
    with pytest.raises(RDCNNError):
        sim.step_record(4, states)
    with pytest.raises(RDCNNError):
        sim.set_params(W.PLAIN_GENE)
    with pytest.raises(RDCNNError):
        sim.set_kernel(1)
        sim.step(1)
    sim.close()
