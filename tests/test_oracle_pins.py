"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle (Sec. II.A, Eq. (1)-(3)) against something other
than itself: hand-worked steps, closed forms, library routines, invariants,
brute force on tiny grids, and finite differences for the reverse pass.  The
cases are chosen so that a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
import workloads as W

BCS = ("periodic", "zeroflux")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_steps.txt")


def _read_golden():
    cases, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], bc=tok[2], R=int(tok[3]), C=int(tok[4]),
                       gene=dict(zip(oracle.PARAM_ORDER, map(float, tok[5:13]))))
            cases.append(cur)
        else:
            cur[tok[0]] = np.array(list(map(float, tok[1:]))).reshape(cur["R"], cur["C"])
    return cases


@pytest.mark.parametrize("case", _read_golden(), ids=lambda c: c["name"])
def test_hand_worked_steps(case):
    """One step against values worked out by hand from Eq. (1)-(3)."""
    u, v = oracle.run(case["u0"], case["v0"], case["gene"], case["bc"], 1, "f64")
    np.testing.assert_allclose(u, case["u1"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(v, case["v1"], rtol=0, atol=1e-15)
    u, v = oracle.run(case["u0"], case["v0"], case["gene"], case["bc"], 1, "f32")
    np.testing.assert_allclose(u, case["u1"], rtol=0, atol=2e-7)
    np.testing.assert_allclose(v, case["v1"], rtol=0, atol=2e-7)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (2, 2), (7, 13), (16, 16)])
def test_laplacian_of_constant_is_zero(bc, shape):
    """Eq. (1)'s Laplacian annihilates constants, exactly, for both rules."""
    for val in (0.0, 1.0, -0.731, 3.5e-39):
        x = np.full(shape, val)
        assert np.all(oracle.laplacian(x, bc) == 0.0)


@pytest.mark.parametrize("shape", [(8, 8), (8, 5), (3, 1), (2, 7)])
@pytest.mark.parametrize("bc", BCS)
def test_laplacian_matches_scipy_convolve(bc, shape):
    """Library pin: the 5-point stencil [[0,1,0],[1,-4,1],[0,1,0]] with scipy's
    'wrap' (periodic) and 'nearest' (edge copy = zero-flux ghost) modes."""
    x = np.random.default_rng(1).standard_normal(shape)
    k = np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]], dtype=np.float64)
    ref = ndimage.convolve(x, k, mode="wrap" if bc == "periodic" else "nearest")
    np.testing.assert_allclose(oracle.laplacian(x, bc), ref, rtol=0, atol=1e-13)


def _dense_laplacian(R, C, bc):
    """Brute force: assemble the Laplacian as an (RC x RC) matrix, one row per
    cell, from the neighbour definition (4 neighbours, periodic wrap or ghost
    copy of the edge cell), minus 4 on the diagonal."""
    n = R * C
    L = np.zeros((n, n))
    for i in range(R):
        for j in range(C):
            k = i * C + j
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if bc == "periodic":
                    ii, jj = ii % R, jj % C
                else:
                    ii = i if not (0 <= ii < R) else ii
                    jj = j if not (0 <= jj < C) else jj
                L[k, ii * C + jj] += 1.0
            L[k, k] -= 4.0
    return L


@pytest.mark.parametrize("shape", [(8, 8), (8, 5), (1, 6), (2, 3)])
@pytest.mark.parametrize("bc", BCS)
def test_brute_force_linear_dynamics(bc, shape):
    """Brute force on tiny grids: with k3 = 0 the step is affine,
    [u;v]+ = M [u;v] + d, with M assembled from the dense Laplacian.  T = 40
    oracle steps must equal 40 applications of that matrix."""
    R, C = shape
    n = R * C
    g = W.gene(k3=0.0, a=0.23, b=1.3, eps=-0.17, c=0.6, Du=0.11, Dv=0.37, dt=0.07)
    L = _dense_laplacian(R, C, bc)
    np.testing.assert_allclose(L, L.T)  # both boundary rules give a symmetric operator
    I = np.eye(n)
    M = np.block([[I + g["dt"] * (g["c"] * I + g["Du"] * L), -g["dt"] * I],
                  [-g["dt"] * g["eps"] * I, I + g["dt"] * (g["eps"] * g["b"] * I + g["Dv"] * L)]])
    d = np.concatenate([np.zeros(n), np.full(n, -g["dt"] * g["eps"] * g["a"])])
    rng = np.random.default_rng(5)
    u0, v0 = rng.uniform(-1, 1, shape), rng.uniform(-1, 1, shape)
    s = np.concatenate([u0.ravel(), v0.ravel()])
    for _ in range(40):
        s = M @ s + d
    u, v = oracle.run(u0, v0, g, bc, 40, "f64")
    np.testing.assert_allclose(u.ravel(), s[:n], rtol=0, atol=1e-12)
    np.testing.assert_allclose(v.ravel(), s[n:], rtol=0, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_linear_mode_closed_form(bc):
    """Closed form: with k3 = 0 and a = 0 a Fourier mode (periodic) or a DCT-II
    mode (zero-flux) stays a pure mode whose amplitudes evolve by the 2x2 matrix
    [[1 + dt (c + Du lam), -dt], [-dt eps, 1 + dt (eps b + Dv lam)]], lam the
    mode's Laplacian eigenvalue."""
    R, C, p, q, T = 24, 20, 3, 2, 60
    g = W.gene(k3=0.0, a=0.0, b=1.3, eps=-0.1, c=0.3, Du=0.05, Dv=0.4, dt=0.1)
    i = np.arange(R)[:, None]
    j = np.arange(C)[None, :]
    if bc == "periodic":
        mode = np.cos(2 * np.pi * (p * i / R + q * j / C))
        lam = -4 + 2 * np.cos(2 * np.pi * p / R) + 2 * np.cos(2 * np.pi * q / C)
    else:
        mode = np.cos(np.pi * p * (i + 0.5) / R) * np.cos(np.pi * q * (j + 0.5) / C)
        lam = -4 + 2 * np.cos(np.pi * p / R) + 2 * np.cos(np.pi * q / C)
    np.testing.assert_allclose(oracle.laplacian(mode, bc), lam * mode, atol=1e-13)
    M = np.array([[1 + g["dt"] * (g["c"] + g["Du"] * lam), -g["dt"]],
                  [-g["dt"] * g["eps"], 1 + g["dt"] * (g["eps"] * g["b"] + g["Dv"] * lam)]])
    amp = np.linalg.matrix_power(M, T) @ np.array([0.8, -0.3])
    u, v = oracle.run(0.8 * mode, -0.3 * mode, g, bc, T, "f64")
    np.testing.assert_allclose(u, amp[0] * mode, rtol=0, atol=1e-12 * max(1, abs(amp[0])))
    np.testing.assert_allclose(v, amp[1] * mode, rtol=0, atol=1e-12 * max(1, abs(amp[1])))


@pytest.mark.parametrize("bc", BCS)
def test_laplacian_sums_to_zero(bc):
    """Invariant: the Laplacian conserves the total for both rules, so the
    diffusion terms cannot change the grid sum of one step."""
    x = np.random.default_rng(2).standard_normal((13, 9))
    assert abs(oracle.laplacian(x, bc).sum()) < 1e-12
    rng = np.random.default_rng(3)
    u0, v0 = rng.uniform(-1, 1, (13, 9)), rng.uniform(-1, 1, (13, 9))
    g = W.gene(W.PAPER_DEFAULT_GENE)
    u1, v1 = oracle.run(u0, v0, g, bc, 1, "f64")
    u2, v2 = oracle.run(u0, v0, dict(g, Du=0.0, Dv=0.0), bc, 1, "f64")
    assert abs(u1.sum() - u2.sum()) < 1e-12
    assert abs(v1.sum() - v2.sum()) < 1e-12


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("bc", BCS)
def test_uniform_grid_stays_uniform(bc, prec):
    """A uniform grid stays bitwise uniform, and with zero diffusion every cell
    follows its own map, so a cell's trajectory does not depend on the grid it
    sits in (a 1x1 grid gives the same bits)."""
    g = W.gene(W.PAPER_DEFAULT_GENE)
    u, v = oracle.run(np.full((6, 9), 0.37), np.full((6, 9), -0.21), g, bc, 50, prec)
    assert np.all(u == u.flat[0]) and np.all(v == v.flat[0])
    u1, v1 = oracle.run(np.full((1, 1), 0.37), np.full((1, 1), -0.21), g, bc, 50, prec)
    assert u1[0, 0] == u.flat[0] and v1[0, 0] == v.flat[0]
    x = W.uniform_x(5, 7, 11)
    gz = dict(g, Du=0.0, Dv=0.0)
    uz, vz = oracle.run(x, x, gz, bc, 30, prec)
    for (r, c) in [(0, 0), (4, 6), (2, 3)]:
        us, vs = oracle.run(x[r:r + 1, c:c + 1], x[r:r + 1, c:c + 1], gz, bc, 30, prec)
        assert us[0, 0] == uz[r, c] and vs[0, 0] == vz[r, c]


def test_zero_state_is_fixed_point():
    g = W.gene()  # a = 0
    for bc in BCS:
        u, v = oracle.run(np.zeros((9, 4)), np.zeros((9, 4)), g, bc, 25, "f32")
        assert not u.any() and not v.any()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("bc", BCS)
def test_d4_equivariance_bitwise(bc, prec):
    """Rotations, reflections and transposition of the grid commute with the
    step, bit for bit (Eq. (1) treats the four neighbours alike)."""
    x = W.uniform_x(7, 13, 4)
    g = W.PLAIN_GENE
    u, v = oracle.run(x, x, g, bc, 20, prec)
    for f in (np.rot90, np.transpose, np.flipud, np.fliplr, lambda a: np.rot90(a, 3)):
        xf = np.ascontiguousarray(f(x))
        uf, vf = oracle.run(xf, xf, g, bc, 20, prec)
        assert np.array_equal(uf, f(u)) and np.array_equal(vf, f(v))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_translation_equivariance_periodic(prec):
    x = W.uniform_x(11, 6, 9)
    g = W.PLAIN_GENE
    u, v = oracle.run(x, x, g, "periodic", 15, prec)
    for sh in [(1, 0), (0, 1), (5, 4), (-3, 2)]:
        xs = np.roll(x, sh, axis=(0, 1))
        us, vs = oracle.run(xs, xs, g, "periodic", 15, prec)
        assert np.array_equal(us, np.roll(u, sh, axis=(0, 1)))
        assert np.array_equal(vs, np.roll(v, sh, axis=(0, 1)))


def test_zero_steps_is_identity_and_steps_compose():
    x = W.uniform_x(9, 10, 1)
    for bc in BCS:
        u, v = oracle.run(x, x, W.PLAIN_GENE, bc, 0, "f32")
        assert np.array_equal(u, x) and np.array_equal(v, x)
        ua, va = oracle.run(x, x, W.PLAIN_GENE, bc, 37, "f32")
        ub, vb = oracle.run(*oracle.run(x, x, W.PLAIN_GENE, bc, 20, "f32"), W.PLAIN_GENE, bc, 17, "f32")
        assert np.array_equal(ua, ub) and np.array_equal(va, vb)


def test_f32_tracks_f64_on_nonchaotic_case():
    """The float32 trajectory stays within float32 rounding of the float64 one
    over 1000 steps of the plain workload (stated drift, not a bitwise claim)."""
    x = W.uniform_x(48, 40, 0)
    u32, v32 = oracle.run(x, x, W.PLAIN_GENE, "zeroflux", 1000, "f32")
    u64, v64 = oracle.run(x, x, W.PLAIN_GENE, "zeroflux", 1000, "f64")
    assert np.abs(u32 - u64).max() < 1e-4 and np.abs(v32 - v64).max() < 1e-4


def test_init_state_scales_both_layers():
    x = W.uniform_x(4, 5, 2)
    u, v = oracle.init_state(x, 0.5)
    assert np.array_equal(u, np.float32(0.5) * x) and np.array_equal(v, u)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.run(np.zeros((2, 2)), np.zeros((2, 3)), W.PLAIN_GENE, "zeroflux", 1)
    with pytest.raises(ValueError):
        oracle.run(np.zeros((2, 2)), np.zeros((2, 2)), W.PLAIN_GENE, "zeroflux", -1)


# ------------------------------------------------------------ reverse pass

def _loss_and_seed(R, C, seed):
    """J(s_T) = <wu, u_T> + <wv, v_T>; its adjoint seed is (wu, wv)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((R, C)), rng.standard_normal((R, C))


def _J(u0, v0, g, bc, T, wu, wv):
    u, v = oracle.run(u0, v0, g, bc, T, "f64")
    return float((wu * u).sum() + (wv * v).sum())


@pytest.mark.parametrize("bc", BCS)
def test_reverse_pass_parameter_gradients_match_finite_differences(bc):
    """Every dJ/dp from the reverse pass against central differences of the
    (pinned) float64 forward, h = 1e-6 relative."""
    R, C, T = 10, 7, 30
    g = W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6)
    rng = np.random.default_rng(7)
    u0, v0 = rng.uniform(-1, 1, (R, C)), rng.uniform(-1, 1, (R, C))
    wu, wv = _loss_and_seed(R, C, 8)
    lam0, mu0, dp, uT, vT = oracle.grad(u0, v0, g, bc, T, wu, wv, traj="f64", S=7)
    uref, vref = oracle.run(u0, v0, g, bc, T, "f64")
    assert np.array_equal(uT, uref) and np.array_equal(vT, vref)
    for k in oracle.PARAM_ORDER:
        h = 1e-6 * max(1.0, abs(g[k]))
        jp = _J(u0, v0, dict(g, **{k: g[k] + h}), bc, T, wu, wv)
        jm = _J(u0, v0, dict(g, **{k: g[k] - h}), bc, T, wu, wv)
        fd = (jp - jm) / (2 * h)
        assert abs(dp[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, dp[k], fd)


@pytest.mark.parametrize("bc", BCS)
def test_reverse_pass_state_gradient_dot_product(bc):
    """<lam0, du0> + <mu0, dv0> equals the directional derivative of J along a
    random (du0, dv0), by central differences."""
    R, C, T = 9, 12, 25
    g = W.gene(Du=0.1, Dv=0.5)
    rng = np.random.default_rng(9)
    u0, v0 = rng.uniform(-1, 1, (R, C)), rng.uniform(-1, 1, (R, C))
    du, dv = rng.standard_normal((R, C)), rng.standard_normal((R, C))
    wu, wv = _loss_and_seed(R, C, 10)
    lam0, mu0, _, _, _ = oracle.grad(u0, v0, g, bc, T, wu, wv, traj="f64")
    h = 1e-6
    fd = (_J(u0 + h * du, v0 + h * dv, g, bc, T, wu, wv) -
          _J(u0 - h * du, v0 - h * dv, g, bc, T, wu, wv)) / (2 * h)
    an = float((lam0 * du).sum() + (mu0 * dv).sum())
    assert abs(an - fd) <= 1e-7 * max(1.0, abs(fd))


def test_reverse_pass_independent_of_checkpoint_spacing():
    R, C, T = 8, 8, 23
    g = W.gene(Du=0.12, Dv=0.7)
    x = W.uniform_x(R, C, 3).astype(np.float64)
    wu, wv = _loss_and_seed(R, C, 4)
    ref = oracle.grad(x, x, g, "zeroflux", T, wu, wv, traj="f32", S=1)
    for S in (2, 5, 23, 40):
        got = oracle.grad(x, x, g, "zeroflux", T, wu, wv, traj="f32", S=S)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert got[2] == ref[2]


def test_reverse_pass_zero_steps():
    wu, wv = _loss_and_seed(3, 4, 1)
    lam, mu, dp, _, _ = oracle.grad(np.zeros((3, 4)), np.zeros((3, 4)), W.PLAIN_GENE,
                                    "periodic", 0, wu, wv)
    assert np.array_equal(lam, wu) and np.array_equal(mu, wv)
    assert all(val == 0.0 for val in dp.values())


@pytest.mark.parametrize("R", [64, 128])
def test_adjoint_stationary_scale_invariance(R):
    """Closed-form identities of the reverse pass at a stationary state.  With
    a = 0, b = 1 the Euler fixed point solves f1 + Du Lap u = 0 and
    -eps (u - v) + Dv Lap v = 0 (Eq. (1)-(3)): it depends on (eps, Dv) only
    through Dv / eps and not on dt.  Once the plain workload has settled
    (T = 2000), a loss of the final state therefore has
    eps dL/deps + Dv dL/dDv = 0 and dL/ddt = 0.  A wrong sign or a dropped term
    in any of these three gradients, or in the mu recursion, breaks them."""
    x = W.uniform_x(R, R, 0)
    tgt = W.stripe_target(R, R, 0)
    g = W.PLAIN_GENE
    T = 2000
    u, _ = oracle.run(x, x, g, "zeroflux", T, "f64")
    u_prev, _ = oracle.run(x, x, g, "zeroflux", T - 100, "f64")
    assert np.array_equal(u, u_prev), "the state has settled"
    lam = 2.0 * (u - tgt) / u.size
    _, _, dp, _, _ = oracle.grad(x, x, g, "zeroflux", T, lam, np.zeros_like(lam), traj="f64")
    se, sd = g["eps"] * dp["eps"], g["Dv"] * dp["Dv"]
    assert abs(se) > 1e-3
    assert abs(se + sd) <= 1e-10 * abs(se)
    assert abs(g["dt"] * dp["dt"]) <= 1e-10 * abs(se)


def _complex_run(u, v, g, bc, T):
    """T Euler steps of Eq. (1)-(3) in complex128 (test-side, for complex-step
    derivatives); its real part is checked against the oracle's float64 run."""
    def nb(q):
        if bc == "periodic":
            return np.roll(q, 1, 0), np.roll(q, -1, 0), np.roll(q, 1, 1), np.roll(q, -1, 1)
        p = np.pad(q, 1, mode="edge")
        return p[:-2, 1:-1], p[2:, 1:-1], p[1:-1, :-2], p[1:-1, 2:]
    for _ in range(T):
        uN, uS, uW, uE = nb(u)
        vN, vS, vW, vE = nb(v)
        lu = uN + uS + uW + uE - 4 * u
        lv = vN + vS + vW + vE - 4 * v
        f1 = g["c"] * u - g["k3"] * u ** 3 - v
        f2 = -g["eps"] * (u - g["b"] * v + g["a"])
        u, v = u + g["dt"] * (f1 + g["Du"] * lu), v + g["dt"] * (f2 + g["Dv"] * lv)
    return u, v


@pytest.mark.parametrize("bc", BCS)
def test_reverse_pass_matches_complex_step(bc):
    """Every dJ/dp and a directional dJ/ds_0 from the reverse pass against
    complex-step derivatives (the step is a polynomial, so Im J(p + i h) / h with
    h = 1e-30 is exact to rounding, with no cancellation), to 1e-10."""
    R, C, T = 12, 9, 40
    g = W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6)
    rng = np.random.default_rng(11)
    u0, v0 = rng.uniform(-1, 1, (R, C)), rng.uniform(-1, 1, (R, C))
    wu, wv = _loss_and_seed(R, C, 12)
    lam0, mu0, dp, _, _ = oracle.grad(u0, v0, g, bc, T, wu, wv, traj="f64")
    ur, vr = _complex_run(u0.astype(complex), v0.astype(complex), g, bc, T)
    uo, vo = oracle.run(u0, v0, g, bc, T, "f64")
    assert np.abs(ur.real - uo).max() < 1e-13 and np.abs(vr.real - vo).max() < 1e-13
    h = 1e-30

    def J(u, v):
        return (wu * u).sum() + (wv * v).sum()

    for k in oracle.PARAM_ORDER:
        gk = {q: complex(val) for q, val in g.items()}
        gk[k] += 1j * h
        cs = J(*_complex_run(u0.astype(complex), v0.astype(complex), gk, bc, T)).imag / h
        assert abs(dp[k] - cs) <= 1e-10 * max(1.0, abs(cs)), (k, dp[k], cs)
    du, dv = rng.standard_normal((R, C)), rng.standard_normal((R, C))
    cs = J(*_complex_run(u0 + 1j * h * du, v0 + 1j * h * dv, g, bc, T)).imag / h
    an = float((lam0 * du).sum() + (mu0 * dv).sum())
    assert abs(an - cs) <= 1e-10 * max(1.0, abs(cs))
