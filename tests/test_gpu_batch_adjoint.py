"""GPU parity of the batched reverse pass (rdcnn_batch_step_record,
rdcnn_batch_adjoint, simulate_batch): the recorded packed trajectory equals the
single-grid recording bit for bit, dJ/dx equals the single-grid adjoint bit for
bit (the per-cell arithmetic is the same whatever the tiling), and the
parameter gradients match the oracle's float64 reverse pass within the
single-grid bars (relative 1e-4 on dJ/dx, 1e-3 on scalars)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

KEYS = oracle.PARAM_ORDER
SHAPES = [(1, 1), (5, 9), (64, 64), (40, 300), (129, 257), (200, 130)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _genes(n, seed):
    rng = np.random.default_rng(seed)
    return [W.gene(Du=rng.uniform(0.02, 0.2), Dv=rng.uniform(0.2, 1.0), eps=-rng.uniform(0.02, 0.2))
            for _ in range(n)]


@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_batch_recording_bitwise(bc):
    from paper_2102_10340_amd import Batch, Simulation
    xs = [W.uniform_x(R, C, 10 + i) for i, (R, C) in enumerate(SHAPES)]
    genes = _genes(len(xs), 1)
    b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
    T = 13
    traj = torch.empty((T, b.total), device="cuda")
    b.step_record(T, traj)
    for i, (x, g) in enumerate(zip(xs, genes)):
        R, C = x.shape
        sim = Simulation(torch.from_numpy(x).cuda(), g, bc)
        st = torch.empty((T, 2, R, C), device="cuda")
        sim.step_record(T, st)
        for q in range(T):
            assert torch.equal(b.view(traj[q], i), st[q]), (i, q)
        assert torch.equal(b.state(i), sim.state()), i
        sim.close()
    b.close()


@pytest.mark.parametrize("kernel", [None, (1, 1, 16), (2, 2, 5), (8, 1, 64), (4, 2, 3)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_batch_adjoint_matches_single_and_oracle(bc, kernel):
    """J = sum_i <w_i, u_T,i> + <z_i, v_T,i> over a ragged batch: dJ/ds_0 bit for
    bit as the single-grid adjoint, dJ/dtheta per instance against the oracle."""
    from paper_2102_10340_amd import Batch, Simulation
    xs = [W.uniform_x(R, C, 30 + i) for i, (R, C) in enumerate(SHAPES)]
    genes = _genes(len(xs), 2)
    T = 21
    b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
    if kernel is not None:
        b.set_adjoint_kernel(*kernel)
    traj = torch.empty((T, b.total), device="cuda")
    b.step_record(T, traj)
    rng = np.random.default_rng(3)
    ws = [rng.standard_normal((2,) + x.shape).astype(np.float32) for x in xs]
    adj = torch.zeros(b.total, device="cuda")
    for i, w in enumerate(ws):
        b.view(adj, i).copy_(torch.from_numpy(w))
    tmp = torch.empty_like(adj)
    dth = torch.zeros((len(xs), 8), dtype=torch.float64, device="cuda")
    b.adjoint(traj, T, adj, tmp, 0xFF, dth)
    dth = dth.cpu().numpy()
    for i, (x, g, w) in enumerate(zip(xs, genes, ws)):
        R, C = x.shape
        sim = Simulation(torch.from_numpy(x).cuda(), g, bc)
        st = torch.empty((T, 2, R, C), device="cuda")
        sim.step_record(T, st)
        a1 = torch.from_numpy(w).cuda().contiguous()
        t1 = torch.empty_like(a1)
        d1 = torch.zeros(8, dtype=torch.float64, device="cuda")
        sim.adjoint(st, T, a1, t1, d1)
        assert torch.equal(b.view(adj, i), a1), ("adjoint state", i)
        l0, m0, dp, _, _ = oracle.grad(x, x, g, bc, T, w[0], w[1], traj="f32")
        got = b.view(adj, i).cpu().numpy()
        ref = np.stack([l0, m0])
        assert np.abs(got - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-30), i
        scale = max(abs(v) for v in dp.values())
        for q, k in enumerate(KEYS):
            assert abs(dth[i, q] - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (i, k, dth[i, q], dp[k])
        sim.close()
    b.close()


@pytest.mark.parametrize("S", [0, -1, 1, 6])
def test_simulate_batch_shared_theta(S):
    """The edge-detection setting: images sharing (Du, Dv, eps), loss summed over
    the images; gradients equal the single-grid autograd's (x: bit for bit,
    theta: to float rounding) and the oracle's."""
    from paper_2102_10340_amd import simulate, simulate_batch
    shapes = [(48, 70), (33, 64), (64, 33), (1, 5)]
    g = W.gene(Du=0.1, Dv=0.5, eps=-0.08)
    T = 17
    imgs, tgts = [], []
    for i, (R, C) in enumerate(shapes):
        noisy, clean = W.rect_image(R, C, 60 + i)
        imgs.append(noisy)
        tgts.append(W.sobel_target(clean))
    theta = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    xs = [torch.from_numpy(x).cuda().requires_grad_(True) for x in imgs]
    outs = simulate_batch(xs, theta, T, "zeroflux", 1.0, S)
    loss = sum(((u - torch.from_numpy(t).cuda()) ** 2).mean() for (u, _), t in zip(outs, tgts))
    loss.backward()
    theta1 = torch.tensor([g[k] for k in KEYS], dtype=torch.float64, requires_grad=True)
    for i, (x, t) in enumerate(zip(imgs, tgts)):
        x1 = torch.from_numpy(x).cuda().requires_grad_(True)
        u1, _ = simulate(x1, theta1, T, "zeroflux")
        assert torch.equal(u1, outs[i][0]), i
        ((u1 - torch.from_numpy(t).cuda()) ** 2).mean().backward()
        assert torch.equal(x1.grad, xs[i].grad), ("dJ/dx", i)
    # the tilings differ, so do the float32 per-lane partial sums
    g0, g1 = theta.grad.numpy(), theta1.grad.numpy()
    scale = np.abs(g1).max()
    assert np.all(np.abs(g0 - g1) <= 1e-4 * scale), (g0, g1)


def test_simulate_batch_per_instance_theta():
    from paper_2102_10340_amd import simulate_batch
    shapes = [(30, 40), (25, 25), (40, 30)]
    genes = _genes(len(shapes), 9)
    T = 12
    xs_np = [W.uniform_x(R, C, 70 + i) for i, (R, C) in enumerate(shapes)]
    theta = torch.tensor([[g[k] for k in KEYS] for g in genes], dtype=torch.float64,
                         requires_grad=True)
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    outs = simulate_batch(xs, theta, T, "periodic")
    rng = np.random.default_rng(1)
    ws = [rng.standard_normal(x.shape).astype(np.float32) for x in xs_np]
    J = sum((u * torch.from_numpy(w).cuda()).sum() for (u, _), w in zip(outs, ws))
    J.backward()
    for i, (x, g, w) in enumerate(zip(xs_np, genes, ws)):
        _, _, dp, _, _ = oracle.grad(x, x, g, "periodic", T, w, np.zeros_like(w), traj="f32")
        scale = max(abs(v) for v in dp.values())
        for q, k in enumerate(KEYS):
            assert abs(theta.grad[i, q].item() - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (i, k)


def test_batch_adjoint_rejects_bad_buffers():
    from paper_2102_10340_amd import Batch, RDCNNError
    b = Batch([torch.zeros((8, 8), device="cuda")], [W.PLAIN_GENE])
    adj = torch.zeros(b.total, device="cuda")
    dth = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    traj = torch.zeros((2, b.total), device="cuda")
    with pytest.raises(RDCNNError):
        b.adjoint(traj, 2, adj, adj, 0xFF, dth)  # aliased
    with pytest.raises(RDCNNError):
        b.set_adjoint_kernel(3, 2, 8)
    b.close()
