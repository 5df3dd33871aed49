"""GPU parity of the even-time trajectory and the paired reverse pass
(rdcnn_step_record_even, rdcnn_adjoint_even).

The even recording must equal every other state of the full recording bit for
bit, and the paired passes rebuild the odd states with the forward cell update,
so dJ/ds equals the full-trajectory adjoint bit for bit.  The parameter sums
are bit-identical too when both reverse passes cut S into the same passes (S
even, same even depth); otherwise the float32 per-pass sums are regrouped and
are held to 1e-4 of the largest gradient.  One case per rule is also checked
against the oracle's float64 reverse pass at the bars of the full-trajectory
adjoint (relative 1e-4 on dJ/ds, 1e-3 on scalars)."""
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


def _sim(x, g, bc, kernel=None):
    from paper_2102_10340_amd import Simulation
    sim = Simulation(torch.from_numpy(x).cuda(), g, bc, 1.0)
    if kernel is not None:
        sim.set_kernel(*kernel)
    return sim


@pytest.mark.parametrize("kernel", [None, (1, 0, 0, 0), (2, 8, 2, 0), (2, 5, 4, 3), (2, 1, 1, 0),
                                    (2, 6, 1, 7)],
                         ids=lambda k: "auto" if k is None else "k%d_d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (5, 9), (40, 300), (129, 257)], ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("T", [1, 9, 17, 18, 23])
def test_even_recording_bitwise(shape, bc, kernel, T):
    R, C = shape
    x = W.uniform_x(R, C, 7 * R + C)
    g = W.PLAIN_GENE
    print(f"case shape={shape} bc={bc} kernel={kernel} T={T}", flush=True)
    a = _sim(x, g, bc, kernel)
    full = torch.empty((T, 2, R, C), device="cuda")
    a.step_record(T, full)
    b = _sim(x, g, bc, kernel)
    n = (T + 1) // 2
    even = torch.full((n + 1, 2, R, C), 7.0, device="cuda")  # one spare state stays untouched
    b.step_record_even(T, even)
    assert torch.equal(even[:n], full[0::2]), "even states"
    assert torch.all(even[n] == 7.0), "wrote past (T+1)/2 states"
    assert torch.equal(a.state(), b.state()), "final state"
    a.close()
    b.close()


def _both(x, g, bc, S, adj_kernel, seed):
    R, C = x.shape
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((2, R, C)).astype(np.float32)
    out = []
    for even in (False, True):
        sim = _sim(x, g, bc)
        if adj_kernel is not None:
            sim.set_adjoint_kernel(*adj_kernel)
        n = (S + 1) // 2 if even else S
        st = torch.empty((max(n, 1), 2, R, C), device="cuda")
        (sim.step_record_even if even else sim.step_record)(S, st)
        adj = torch.from_numpy(w).cuda().contiguous()
        tmp = torch.empty_like(adj)
        dth = torch.zeros(8, dtype=torch.float64, device="cuda")
        (sim.adjoint_even if even else sim.adjoint)(st, S, adj, tmp, dth)
        out.append((adj.cpu().numpy(), dth.cpu().numpy()))
        sim.close()
    return out, w


@pytest.mark.parametrize("adj_kernel", [None, (2, 1, 16), (8, 1, 64), (4, 2, 5), (6, 2, 0), (8, 2, 3),
                                        (3, 1, 0), (1, 1, 0), (4, 4, 0)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (5, 9), (64, 64), (40, 300), (129, 257), (200, 130)],
                         ids=lambda s: "%dx%d" % s)
@pytest.mark.parametrize("S", [1, 2, 20, 27])
def test_adjoint_even_matches_full(shape, bc, adj_kernel, S):
    R, C = shape
    g = W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6) if bc == "periodic" else \
        W.gene(Du=0.1, Dv=0.5)
    print(f"case shape={shape} bc={bc} adj_kernel={adj_kernel} S={S}", flush=True)
    x = W.uniform_x(R, C, R + 3 * C)
    ((a_full, d_full), (a_even, d_even)), _ = _both(x, g, bc, S, adj_kernel, S)
    assert np.array_equal(a_even, a_full), "dJ/ds"
    # same pass cut: a forced shape (the automatic ones differ: the paired
    # passes default to 6 steps, the plain ones to 4), even S and an even depth
    if adj_kernel is not None and S % 2 == 0 and adj_kernel[0] % 2 == 0 and adj_kernel[1] <= 2:
        assert np.array_equal(d_even, d_full), (d_even, d_full)
    else:
        # regrouped float32 per-pass sums: the bar two tilings of the batched
        # reverse pass are held to (1e-4 of the largest gradient)
        scale = np.abs(d_full).max()
        assert np.all(np.abs(d_even - d_full) <= 1e-4 * scale), (d_even, d_full)


@pytest.mark.parametrize("bc", BCS)
def test_adjoint_even_matches_oracle(bc):
    R, C, S = 70, 133, 41
    g = W.gene(Du=0.07, Dv=0.8, eps=-0.12)
    x = W.uniform_x(R, C, 12)
    (_, (got, dth)), w = _both(x, g, bc, S, None, 5)
    l0, m0, dp, _, _ = oracle.grad(x, x, g, bc, S, w[0], w[1], traj="f32")
    for a, b in ((got[0], l0), (got[1], m0)):
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max()
    scale = max(abs(v) for v in dp.values())
    for i, k in enumerate(KEYS):
        assert abs(dth[i] - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (k, dth[i], dp[k])


def test_even_entry_points_reject_bad_buffers():
    from paper_2102_10340_amd import RDCNNError, Simulation, _lib
    sim = Simulation(torch.zeros((8, 8), device="cuda"), W.PLAIN_GENE, "zeroflux")
    st = torch.zeros((4, 2, 8, 8), device="cuda")
    with pytest.raises(ValueError):
        sim.step_record_even(9, st)  # needs 5 states
    with pytest.raises(RDCNNError):  # the trajectory may not overlap the state buffers
        _lib.check(_lib.lib.rdcnn_step_record_even(sim._h, 2, sim.buf[1].data_ptr()))
    adj = torch.zeros((2, 8, 8), device="cuda")
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(RDCNNError):
        from paper_2102_10340_amd import _lib
        _lib.check(_lib.lib.rdcnn_adjoint_even(sim._h, st.data_ptr(), 4, adj.data_ptr(),
                                               adj.data_ptr(), dth.data_ptr()))
    sim.close()


# ---------------------------------------------------------------- batches

BATCH_SHAPES = [(1, 1), (5, 9), (64, 64), (40, 300), (129, 257), (200, 130)]


def _genes(n, seed):
    rng = np.random.default_rng(seed)
    return [W.gene(Du=rng.uniform(0.02, 0.2), Dv=rng.uniform(0.2, 1.0), eps=-rng.uniform(0.02, 0.2))
            for _ in range(n)]


@pytest.mark.parametrize("kernel", [None, (1, 1, 0), (5, 2, 7)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("T", [1, 9, 16, 17, 21])
def test_batch_even_recording_bitwise(bc, kernel, T):
    from paper_2102_10340_amd import Batch
    xs = [W.uniform_x(R, C, 40 + i) for i, (R, C) in enumerate(BATCH_SHAPES)]
    genes = _genes(len(xs), 3)
    runs = []
    for even in (False, True):
        b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
        if kernel is not None:
            b.set_kernel(*kernel)
        n = (T + 1) // 2 if even else T
        traj = torch.full((n + 1, b.total), 7.0, device="cuda")
        (b.step_record_even if even else b.step_record)(T, traj)
        runs.append((traj, [b.state(i).clone() for i in range(len(xs))]))
        b.close()
    (full, s0), (even, s1) = runs
    n = (T + 1) // 2
    # the gaps between instances hold 7.0 in both trajectories
    assert torch.equal(even[:n], full[0:T:2]), "even states"
    assert torch.all(even[n] == 7.0), "wrote past (T+1)/2 states"
    for i in range(len(xs)):
        assert torch.equal(s0[i], s1[i]), ("final state", i)


@pytest.mark.parametrize("kernel", [None, (2, 1, 16), (4, 2, 5), (8, 2, 64)],
                         ids=lambda k: "auto" if k is None else "d%d_c%d_h%d" % k)
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("S", [1, 2, 20, 23])
def test_batch_adjoint_even_matches_full(bc, kernel, S):
    from paper_2102_10340_amd import Batch
    xs = [W.uniform_x(R, C, 60 + i) for i, (R, C) in enumerate(BATCH_SHAPES)]
    genes = _genes(len(xs), 4)
    rng = np.random.default_rng(S)
    ws = [rng.standard_normal((2,) + x.shape).astype(np.float32) for x in xs]
    print(f"case bc={bc} adj_kernel={kernel} S={S}", flush=True)
    res = []
    for even in (False, True):
        b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
        if kernel is not None:
            b.set_adjoint_kernel(*kernel)
        n = (S + 1) // 2 if even else S
        traj = torch.empty((max(n, 1), b.total), device="cuda")
        (b.step_record_even if even else b.step_record)(S, traj)
        adj = torch.zeros(b.total, device="cuda")
        for i, w in enumerate(ws):
            b.view(adj, i).copy_(torch.from_numpy(w))
        tmp = torch.empty_like(adj)
        dth = torch.zeros((len(xs), 8), dtype=torch.float64, device="cuda")
        (b.adjoint_even if even else b.adjoint)(traj, S, adj, tmp, 0xFF, dth)
        res.append((adj.cpu().numpy(), dth.cpu().numpy()))
        b.close()
    (a0, d0), (a1, d1) = res
    assert np.array_equal(a0, a1), "dJ/ds"
    if S % 2 == 0:  # both cut S into the same passes
        assert np.array_equal(d0, d1)
    else:
        scale = np.abs(d0).max(axis=1, keepdims=True)
        assert np.all(np.abs(d1 - d0) <= 1e-4 * scale), (d0, d1)


def test_batch_adjoint_even_rejects_depth_one():
    from paper_2102_10340_amd import Batch, RDCNNError
    b = Batch([torch.zeros((8, 8), device="cuda")], [W.PLAIN_GENE])
    b.set_adjoint_kernel(1, 1, 8)
    traj = torch.zeros((2, b.total), device="cuda")
    adj = torch.zeros(b.total, device="cuda")
    dth = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(RDCNNError):
        b.adjoint_even(traj, 4, adj, torch.empty_like(adj), 0xFF, dth)
    from paper_2102_10340_amd import _lib
    with pytest.raises(RDCNNError):  # the trajectory may not overlap the state buffers
        _lib.check(_lib.lib.rdcnn_batch_step_record_even(b._h, 2, b.buf[0].data_ptr()))
    b.close()
