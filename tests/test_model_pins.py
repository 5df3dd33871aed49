"""Pins of the oracle's two further cell models (oracle/cell_models.c): closed
forms, conservation laws, symmetries, a library routine and the textbook
steady state of the Chua-Yang edge-detection template."""
import numpy as np
import pytest
from scipy import ndimage

import oracle

BCS = ("periodic", "zeroflux")
MODE = {"periodic": "wrap", "zeroflux": "nearest"}
GS = dict(dt=0.5, F=0.037, k=0.06, Du=0.2, Dv=0.1)


def _rand(shape, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


# ---------------------------------------------------------------- Gray-Scott

@pytest.mark.parametrize("bc", BCS)
def test_gs_trivial_state_is_fixed(bc):
    u = np.ones((7, 9), np.float32)
    v = np.zeros((7, 9), np.float32)
    uu, vv = oracle.gs_run(u, v, GS, bc, 25)
    assert np.array_equal(uu, u) and np.array_equal(vv, v)


@pytest.mark.parametrize("bc", BCS)
def test_gs_without_feed_conserves_total(bc):
    """With F = k = 0 the reaction terms -u v^2 and +u v^2 cancel and the
    Laplacian sums to zero, so sum(u + v) is conserved; a sign slip in either
    reaction term breaks it."""
    u, v = _rand((12, 10), 1), _rand((12, 10), 2)
    p = dict(GS, F=0.0, k=0.0)
    uu, vv = oracle.gs_run(u, v, p, bc, 40, "f64")
    assert abs((uu + vv).sum() - (u + v).sum()) < 1e-11
    assert np.abs(uu - u).max() > 1e-3  # the state did move


@pytest.mark.parametrize("layer", ["u", "v"])
def test_gs_pure_diffusion_mode_closed_form(layer):
    """v = 0, F = 0 (or u = 0, F = k = 0): the other layer diffuses, and a
    periodic Fourier mode decays by exactly (1 + dt D lambda)^T."""
    R, C, p, q, T = 16, 12, 3, 2, 30
    i = np.arange(R)[:, None]
    j = np.arange(C)[None, :]
    mode = np.cos(2 * np.pi * (p * i / R + q * j / C)) + 0.0 * j
    lam = -4 + 2 * np.cos(2 * np.pi * p / R) + 2 * np.cos(2 * np.pi * q / C)
    prm = dict(GS, F=0.0, k=0.0)
    if layer == "u":
        uu, vv = oracle.gs_run(mode, np.zeros_like(mode), prm, "periodic", T, "f64")
        got, D = uu, prm["Du"]
        assert np.all(vv == 0)
    else:
        uu, vv = oracle.gs_run(np.zeros_like(mode), mode, prm, "periodic", T, "f64")
        got, D = vv, prm["Dv"]
        assert np.all(uu == 0)
    want = (1 + prm["dt"] * D * lam) ** T * mode
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_gs_zeroflux_mode_closed_form():
    """Zero-flux (ghost copies the edge): the DCT-II mode cos(pi p (i+1/2)/R)
    decays by (1 + dt Du (2 cos(pi p/R) - 2))^T."""
    R, C, p, T = 13, 5, 4, 25
    i = np.arange(R)[:, None] + 0.0 * np.arange(C)[None, :]
    mode = np.cos(np.pi * p * (i + 0.5) / R)
    lam = 2 * np.cos(np.pi * p / R) - 2
    prm = dict(GS, F=0.0, k=0.0)
    uu, _ = oracle.gs_run(mode, np.zeros_like(mode), prm, "zeroflux", T, "f64")
    assert np.allclose(uu, (1 + prm["dt"] * prm["Du"] * lam) ** T * mode, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_gs_d4_and_translation_bitwise(bc):
    u, v = _rand((9, 9), 3).astype(np.float32), _rand((9, 9), 4).astype(np.float32)
    ref = oracle.gs_run(u, v, GS, bc, 12)
    for f in (np.transpose, np.fliplr, np.flipud, np.rot90):
        got = oracle.gs_run(f(u), f(v), GS, bc, 12)
        assert np.array_equal(got[0], f(ref[0])) and np.array_equal(got[1], f(ref[1]))
    if bc == "periodic":
        got = oracle.gs_run(np.roll(u, (2, -3), (0, 1)), np.roll(v, (2, -3), (0, 1)), GS, bc, 12)
        assert np.array_equal(got[0], np.roll(ref[0], (2, -3), (0, 1)))


def test_gs_f32_tracks_f64():
    u, v = _rand((20, 20), 5), _rand((20, 20), 6) * 0.3
    a = oracle.gs_run(u, v, GS, "periodic", 200, "f32")
    b = oracle.gs_run(u, v, GS, "periodic", 200, "f64")
    assert np.abs(a[0] - b[0]).max() < 1e-4 and np.abs(a[1] - b[1]).max() < 1e-4


# ---------------------------------------------------------------- Chua-Yang CNN

def _sat(x):
    return np.clip(x, -1.0, 1.0)


@pytest.mark.parametrize("bc", BCS)
def test_cnn_input_layer_is_a_correlation(bc):
    """w = (B * g) + z against scipy's correlation with the same boundary rule."""
    g = _rand((11, 14), 7, -1, 1)
    B = _rand((3, 3), 8, -1, 1)
    w = oracle.cnn_input(g, B, -0.25, bc, "f64")
    assert np.allclose(w, ndimage.correlate(g, B, mode=MODE[bc]) - 0.25, atol=1e-13)


@pytest.mark.parametrize("bc", BCS)
def test_cnn_step_is_a_correlation_of_the_output(bc):
    """One step: x + dt (-x + A * y(x) + w), A * y against scipy, y = clip."""
    x = _rand((10, 13), 9, -2, 2)
    w = _rand((10, 13), 10, -1, 1)
    A = _rand((3, 3), 11, -1, 1)
    got = oracle.cnn_run(x, w, 0.2, A, bc, 1, "f64")
    want = x + 0.2 * (-x + ndimage.correlate(_sat(x), A, mode=MODE[bc]) + w)
    assert np.allclose(got, want, atol=1e-13)


def test_cnn_saturated_relaxation_closed_form():
    """All cells saturated at +1 stay saturated: x_t = x* + (x_0 - x*)(1-dt)^t
    with x* = sum(A) + w."""
    x0 = 1.5 + _rand((6, 7), 12)
    A = np.full((3, 3), 0.25)
    A[1, 1] = 2.0
    w = np.full((6, 7), 0.5)
    dt, T = 0.1, 40
    got = oracle.cnn_run(x0, w, dt, A, "periodic", T, "f64")
    xs = A.sum() + 0.5
    assert np.allclose(got, xs + (x0 - xs) * (1 - dt) ** T, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_cnn_symmetric_template_reflections_bitwise(bc):
    """A mirror-symmetric template commutes with reflecting the grid across
    either axis bit for bit (the summation pairs NW with NE and SW with SE, N
    with S and W with E); transposes agree up to rounding only (the corner
    pairing is not transpose-symmetric)."""
    A = np.array([[0.1, 0.3, 0.1], [0.3, 1.5, 0.3], [0.1, 0.3, 0.1]], np.float32)
    x = _rand((9, 11), 13, -1.5, 1.5).astype(np.float32)
    w = _rand((9, 11), 14, -1, 1).astype(np.float32)
    ref = oracle.cnn_run(x, w, 0.1, A, bc, 15)
    for f in (np.fliplr, np.flipud, lambda a: np.flipud(np.fliplr(a))):
        assert np.array_equal(oracle.cnn_run(f(x), f(w), 0.1, A, bc, 15), f(ref))
    for f in (np.transpose, np.rot90):
        assert np.allclose(oracle.cnn_run(f(x), f(w), 0.1, A, bc, 15), f(ref), atol=1e-5)


def test_cnn_edge_template_textbook_result():
    """Chua-Yang edge extraction (A = 2 at the centre, B = 8 at the centre and -1
    around, z = -1) on a +-1 image from x = 0: the settled output is +1 exactly
    where a +1 pixel has a -1 pixel among its 8 neighbours (zero-flux: pixels
    outside copy the edge)."""
    rng = np.random.default_rng(15)
    img = -np.ones((24, 20))
    for _ in range(6):
        r0, c0 = rng.integers(0, 20, 2)
        img[r0:r0 + rng.integers(3, 9), c0:c0 + rng.integers(3, 9)] = 1.0
    A = np.zeros((3, 3))
    A[1, 1] = 2.0
    B = -np.ones((3, 3))
    B[1, 1] = 8.0
    w = oracle.cnn_input(img, B, -1.0, "zeroflux", "f64")
    x = oracle.cnn_run(np.zeros_like(img), w, 0.1, A, "zeroflux", 400, "f64")
    y = _sat(x)
    pad = np.pad(img, 1, mode="edge")
    edge = np.zeros_like(img, dtype=bool)
    for i in range(img.shape[0]):
        for j in range(img.shape[1]):
            nb = pad[i:i + 3, j:j + 3]
            edge[i, j] = img[i, j] > 0 and (nb < 0).any()
    assert np.array_equal(y > 0.99, edge) and np.all((y > 0.99) | (y < -0.99))
