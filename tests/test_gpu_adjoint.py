"""GPU parity of the reverse pass (state recording, adjoint kernel, autograd)
against the CPU oracle's float64 reverse pass on the same float32 trajectory.

Tolerance: the adjoint runs in float32 on the GPU and float64 in the oracle,
over the identical float32 trajectory (the recorded states are bit-exact).  The
adjoint recursion is linear, so its float32 rounding error grows like the
number of steps times the float32 unit roundoff relative to the adjoint's own
size: 1e-4 relative (max-norm) leaves an order of magnitude of margin at
T <= 200 steps, and 1e-3 on the scalar parameter gradients (which also carry
the float32 per-pass partial sums).  At the full 1024x1024, T = 2000 size the
bars are relative 1e-3 on scalars and max |error| <= 1e-3 max |dJ/dx| element
by element on dJ/dx.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

BCS = ("periodic", "zeroflux")
KEYS = oracle.PARAM_ORDER


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def _grad_scale(dp):
    return max(abs(v) for v in dp.values())


def gpu_record(x, gene, bc, T, kernel=None):
    from paper_2102_10340_amd import Simulation
    R, C = x.shape
    sim = Simulation(torch.from_numpy(x).cuda(), gene, bc, 1.0)
    if kernel is not None:
        sim.set_kernel(*kernel)
    states = torch.empty((T, 2, R, C), dtype=torch.float32, device="cuda")
    sim.step_record(T, states)
    return sim, states


@pytest.mark.parametrize("kernel", [(1, 0, 0, 0), (2, 8, 4, 0), (2, 5, 2, 3), (2, 16, 2, 0),
                                    (2, 6, 1, 0)],
                         ids=lambda k: "k%d_d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (5, 9), (40, 300), (129, 257)], ids=lambda s: "%dx%d" % s)
def test_recorded_states_bitwise(shape, bc, kernel):
    R, C = shape
    x = W.uniform_x(R, C, 31 * R + C)
    g = W.PLAIN_GENE
    T = 19
    sim, states = gpu_record(x, g, bc, T, kernel)
    st = states.cpu().numpy()
    u, v = oracle.init_state(x, 1.0)
    for q in range(T):
        assert np.array_equal(st[q, 0], u) and np.array_equal(st[q, 1], v), q
        u, v = oracle.run(u, v, g, bc, 1, "f32")
    uT, vT = sim.read_host()
    assert np.array_equal(uT, u) and np.array_equal(vT, v)
    sim.close()


def _adjoint_case(R, C, bc, gene, T, kernel, seed=0):
    x = W.uniform_x(R, C, seed)
    sim, states = gpu_record(x, gene, bc, T)
    if kernel is not None:
        sim.set_adjoint_kernel(*kernel)
    rng = np.random.default_rng(seed + 1)
    lam = rng.standard_normal((R, C)).astype(np.float32)
    mu = rng.standard_normal((R, C)).astype(np.float32)
    adj = torch.from_numpy(np.stack([lam, mu])).cuda().contiguous()
    tmp = torch.empty_like(adj)
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    sim.adjoint(states, T, adj, tmp, dth)
    got = adj.cpu().numpy()
    sim.close()
    l0, m0, dp, _, _ = oracle.grad(x, x, gene, bc, T, lam, mu, traj="f32")
    return got, dth.cpu().numpy(), l0, m0, dp


@pytest.mark.parametrize("kernel", [None, (4, 4, 0), (8, 2, 0), (3, 4, 5), (1, 2, 1), (6, 4, 7),
                                    (4, 1, 0), (8, 1, 3)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (3, 70), (33, 17), (64, 64), (131, 300)],
                         ids=lambda s: "%dx%d" % s)
def test_adjoint_matches_oracle(shape, bc, kernel):
    R, C = shape
    g = W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6) if bc == "periodic" else \
        W.gene(Du=0.1, Dv=0.5)
    T = 37
    print(f"case shape={shape} bc={bc} adj_kernel={kernel} T={T}", flush=True)
    got, dth, l0, m0, dp = _adjoint_case(R, C, bc, g, T, kernel)
    assert _rel(got[0], l0) < 1e-4 and _rel(got[1], m0) < 1e-4, (_rel(got[0], l0), _rel(got[1], m0))
    scale = _grad_scale(dp)
    for i, k in enumerate(KEYS):
        assert abs(dth[i] - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (k, dth[i], dp[k])


def test_adjoint_deterministic_and_zero_steps():
    R, C = 70, 190
    g = W.PLAIN_GENE
    a = _adjoint_case(R, C, "zeroflux", g, 25, None)
    b = _adjoint_case(R, C, "zeroflux", g, 25, None)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    from paper_2102_10340_amd import Simulation
    sim = Simulation(torch.zeros((4, 5), device="cuda"), g, "zeroflux")
    adj = torch.ones((2, 4, 5), device="cuda")
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    sim.adjoint(torch.empty(0), 0, adj, torch.empty_like(adj), dth)
    assert torch.all(adj == 1) and torch.all(dth == 0)
    sim.close()


@pytest.mark.parametrize("bc", BCS)
def test_autograd_function_matches_oracle(bc):
    """simulate(x, theta) with checkpoint-and-recompute: J = <w, u_T> + <z, v_T>."""
    from paper_2102_10340_amd import simulate
    R, C, T = 96, 80, 150
    g = W.gene(Du=0.07, Dv=0.8, eps=-0.12)
    x = W.uniform_x(R, C, 4)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((R, C)).astype(np.float32)
    z = rng.standard_normal((R, C)).astype(np.float32)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    for S in (0, -1, 1, 7, 150):
        xt.grad = None
        theta.grad = None
        u, v = simulate(xt, theta, T, bc, 1.0, S)
        J = (u * torch.from_numpy(w).cuda()).sum() + (v * torch.from_numpy(z).cuda()).sum()
        J.backward()
        l0, m0, dp, uT, vT = oracle.grad(x, x, g, bc, T, w, z, traj="f32")
        assert np.array_equal(u.detach().cpu().numpy(), uT.astype(np.float32))
        gx = xt.grad.cpu().numpy()
        assert _rel(gx, l0 + m0) < 1e-4
        scale = _grad_scale(dp)
        for i, k in enumerate(KEYS):
            assert abs(theta.grad[i].item() - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (S, k)


@pytest.fixture(scope="module")
def diff_workload_reference():
    """The oracle's reverse pass for the differentiation workload (1024x1024,
    T = 2000, MSE to the seeded stripe target) on the float32 trajectory; the
    loss gradient at u_T uses the GPU's u_T, which must equal the oracle's."""
    R = C = 1024
    T = 2000
    g = W.PLAIN_GENE
    x = W.uniform_x(R, C, 0)
    target = W.stripe_target(R, C, 0)
    uT = oracle.run(*oracle.init_state(x, 1.0), g, "zeroflux", T, "f32")[0]
    lamT = 2.0 * (uT.astype(np.float64) - target) / (R * C)
    l0, m0, dp, uo, _ = oracle.grad(x, x, g, "zeroflux", T, lamT, np.zeros_like(lamT), traj="f32")
    return dict(x=x, target=target, uT=uo.astype(np.float32), ref=l0 + m0, dp=dp, T=T, g=g)


@pytest.mark.parametrize("S", [0, -1], ids=["sqrtT_checkpoints", "whole_trajectory"])
def test_differentiation_workload_full_size(S, diff_workload_reference):
    """1024x1024, T = 2000, loss = MSE(u_T, seeded sinusoid-stripe target),
    through autograd with sqrt(T) checkpoint-and-recompute (the workload's
    schedule) and with the whole trajectory recorded: dJ/dx element by
    element (max |g - ref| <= 1e-3 max |ref|) and dJ/dDu, dJ/dDv, dJ/deps
    (1e-3 relative) against the oracle's reverse pass."""
    from paper_2102_10340_amd import simulate
    ref = diff_workload_reference
    g, T = ref["g"], ref["T"]
    print(f"case differentiation 1024^2 T={T} S={S}", flush=True)
    xt = torch.from_numpy(ref["x"]).cuda().requires_grad_(True)
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    u, v = simulate(xt, theta, T, "zeroflux", S=S)
    loss = ((u - torch.from_numpy(ref["target"]).cuda()) ** 2).mean()
    loss.backward()
    assert np.array_equal(u.detach().cpu().numpy(), ref["uT"])
    gx = xt.grad.cpu().numpy().astype(np.float64)
    err = float(np.abs(gx - ref["ref"]).max() / np.abs(ref["ref"]).max())
    print(f"dJ/dx max-abs error / max|ref| = {err:.3e}; grads gpu {theta.grad.tolist()} "
          f"oracle {[ref['dp'][k] for k in KEYS]}", flush=True)
    assert err <= 1e-3
    for i, k in enumerate(KEYS):
        if k in ("Du", "Dv", "eps"):
            assert abs(theta.grad[i].item() - ref["dp"][k]) <= 1e-3 * abs(ref["dp"][k]), \
                (k, theta.grad[i].item(), ref["dp"][k])


def test_schedules_give_identical_gradients():
    """Checkpoint spacings, the whole trajectory and the overlapped or serial
    recompute run the same reverse passes on the same states: identical bits."""
    from paper_2102_10340_amd import autograd as AG
    from paper_2102_10340_amd import Simulation
    R, C, T = 80, 150, 70
    g = W.gene(Du=0.08, Dv=0.6)
    x = torch.from_numpy(W.uniform_x(R, C, 6)).cuda()
    w = torch.from_numpy(np.random.default_rng(2).standard_normal((R, C)).astype(np.float32)).cuda()
    outs = []
    for S, overlap in ((-1, True), (16, True), (16, False), (10, True), (8, True), (70, True)):
        sim = Simulation(x, g, "zeroflux")
        u, v, ck, nseg = AG._forward(sim, T, S, x.device)
        lam, mu, dth = AG._backward(sim, ck, nseg, T, S, w, None, x.device, overlap=overlap)
        sim.close()
        outs.append((u.cpu(), lam.cpu(), mu.cpu(), dth.cpu(), (S, overlap)))
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]), o[4]
        assert torch.equal(o[1], outs[0][1]) and torch.equal(o[2], outs[0][2]), o[4]
        # the float32 per-pass partial sums depend on how passes are cut
        assert float((o[3] - outs[0][3]).abs().max()) <= 1e-4 * float(outs[0][3].abs().max()), o[4]


def test_no_grad_forward_and_single_backward():
    """Under no_grad nothing is recorded and the result is the plain run's;
    a second backward through one run raises a clear error."""
    from paper_2102_10340_amd import Simulation, simulate
    R, C, T = 40, 60, 30
    g = W.PLAIN_GENE
    x = torch.from_numpy(W.uniform_x(R, C, 8)).cuda()
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    with torch.no_grad():
        u, v = simulate(x, theta, T)
    sim = Simulation(x, g, "zeroflux")
    sim.step(T)
    st = sim.state()
    assert torch.equal(u, st[0]) and torch.equal(v, st[1])
    sim.close()
    u, v = simulate(x, theta, T)
    J = u.sum()
    J.backward(retain_graph=True)
    with pytest.raises(RuntimeError, match="released by its first backward"):
        J.backward()


def test_gradient_mask_subset_equal_and_rest_nan():
    """Forming only dJ/dDu, dJ/dDv, dJ/deps (no lam-weighted sums) gives the same
    values as forming all eight; the rest come back NaN; dJ/dx is unchanged."""
    from paper_2102_10340_amd import simulate
    R, C, T = 70, 300, 60
    g = W.gene(Du=0.09, Dv=0.7)
    x = W.uniform_x(R, C, 21)
    w = torch.from_numpy(np.random.default_rng(3).standard_normal((R, C)).astype(np.float32)).cuda()
    out = []
    for grads in (None, ("Du", "Dv", "eps")):
        xt = torch.from_numpy(x).cuda().requires_grad_(True)
        theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
        u, v = simulate(xt, theta, T, "zeroflux", grads=grads)
        (u * w).sum().backward()
        out.append((xt.grad.cpu().numpy(), theta.grad.numpy()))
    assert np.array_equal(out[0][0], out[1][0])
    for i, k in enumerate(KEYS):
        if k in ("Du", "Dv", "eps"):
            assert abs(out[0][1][i] - out[1][1][i]) <= 1e-9 * max(1.0, abs(out[0][1][i])), k
        else:
            assert np.isnan(out[1][1][i]) and np.isfinite(out[0][1][i]), k


def test_shared_parameters_over_many_images():
    """Gradients of a loss summed over several images that share the parameters
    (the edge-detection fit) equal the sum of the oracle's per-image gradients."""
    from paper_2102_10340_amd import simulate
    R, C, T = 48, 70, 30
    g = W.gene(Du=0.1, Dv=0.5)
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    ref = {k: 0.0 for k in KEYS}
    for i in range(3):
        noisy, clean = W.rect_image(R, C, 40 + i)
        tgt = W.sobel_target(clean)
        xt = torch.from_numpy(noisy).cuda()
        u, _ = simulate(xt, theta, T, "zeroflux")
        loss = ((u - torch.from_numpy(tgt).cuda()) ** 2).mean()
        loss.backward()
        uT = u.detach().cpu().numpy().astype(np.float64)
        lam = 2.0 * (uT - tgt) / (R * C)
        _, _, dp, _, _ = oracle.grad(noisy, noisy, g, "zeroflux", T, lam, np.zeros_like(lam), traj="f32")
        for k in KEYS:
            ref[k] += dp[k]
    scale = max(abs(v) for v in ref.values())
    for i, k in enumerate(KEYS):
        assert abs(theta.grad[i].item() - ref[k]) <= 1e-3 * max(abs(ref[k]), 1e-3 * scale), k


def test_full_size_stationary_identities():
    """The differentiation workload at full size (1024^2, T = 2000, MSE to the
    stripe target, autograd through the even-time trajectory and the paired
    passes).  The plain workload settles, and at a stationary state the fixed
    point depends on (eps, Dv) only through Dv / eps and not on dt, so
    eps dL/deps + Dv dL/dDv = 0 and dL/ddt = 0 (the CPU oracle meets both to
    1e-10 on a float64 trajectory).  The GPU sums in float32 per pass; measured,
    both hold to ~2e-7 of eps dL/deps, and the bar is 1e-5."""
    from paper_2102_10340_amd import simulate
    N, T = 1024, 2000
    g = W.PLAIN_GENE
    x = torch.from_numpy(W.uniform_x(N, N, 0)).cuda()
    target = torch.from_numpy(W.stripe_target(N, N, 0)).cuda()
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    u, _ = simulate(x.clone().requires_grad_(True), theta, T, "zeroflux")
    ((u - target) ** 2).mean().backward()
    d = dict(zip(KEYS, theta.grad.tolist()))
    se, sd, st = g["eps"] * d["eps"], g["Dv"] * d["Dv"], g["dt"] * d["dt"]
    print(f"eps*dL/deps {se:.6e}  Dv*dL/dDv {sd:.6e}  dt*dL/ddt {st:.3e}", flush=True)
    assert abs(se) > 1e-3
    assert abs(se + sd) <= 1e-5 * abs(se), (se, sd)
    assert abs(st) <= 1e-5 * abs(se), st
