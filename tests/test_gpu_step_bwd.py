"""GPU tests of the checkpoint-and-recompute entry points: rdcnn_step_checkpoints
(forward with a checkpoint every S steps), rdcnn_step_record_sparse (even-time
states in their own slots), rdcnn_step_bwd (the reverse pass through one
segment) and rdcnn_step_bwd_ckpt (the whole recompute-and-reverse schedule),
called through the C ABI, against the CPU oracle's float64 reverse
pass on the same float32 trajectory (bars as in test_gpu_adjoint: 1e-4
relative max-norm on dJ/ds, 1e-3 on dJ/dp), plus the finite check on reads,
the batch's packed read and its shared-parameter gradient sum."""
import ctypes

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


def _sim(x, g, bc):
    from paper_2102_10340_amd import Simulation
    return Simulation(torch.from_numpy(x).cuda(), g, bc, 1.0)


def _gene(bc):
    return W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6) if bc == "periodic" else \
        W.gene(Du=0.1, Dv=0.5)


@pytest.mark.parametrize("layout", ["full", "sparse"])
@pytest.mark.parametrize("S", [1, 2, 7, 20, 37])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(1, 1), (33, 17), (64, 64), (131, 300)], ids=lambda s: "%dx%d" % s)
def test_step_bwd_through_cabi_matches_oracle(shape, bc, S, layout):
    """rdcnn_step_bwd called with raw device pointers (ctypes): (lam, mu) and
    dJ/dp against the oracle's float64 reverse pass; the states come from a
    full recording (every slot) or the sparse one (even slots only)."""
    from paper_2102_10340_amd._lib import check, lib
    R, C = shape
    g = _gene(bc)
    x = W.uniform_x(R, C, 7 * R + C)
    sim = _sim(x, g, bc)
    states = torch.full((S + 1, 2, R, C), float("nan"), device="cuda")
    if layout == "full":
        sim.step_record(S, states)
    else:
        sim.step_record_sparse(S, states)
    rng = np.random.default_rng(S)
    lam0 = rng.standard_normal((R, C)).astype(np.float32)
    mu0 = rng.standard_normal((R, C)).astype(np.float32)
    lam = torch.from_numpy(lam0).cuda()
    mu = torch.from_numpy(mu0).cuda()
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    print(f"case step_bwd {shape} {bc} S={S} {layout}", flush=True)
    check(lib.rdcnn_step_bwd(sim._h, states.data_ptr(), S, lam.data_ptr(), mu.data_ptr(),
                             dth.data_ptr()))
    got_l, got_m, got_p = lam.cpu().numpy(), mu.cpu().numpy(), dth.cpu().numpy()
    sim.close()
    l0, m0, dp, _, _ = oracle.grad(x, x, g, bc, S, lam0, mu0, traj="f32")
    assert _rel(got_l, l0) < 1e-4 and _rel(got_m, m0) < 1e-4, (_rel(got_l, l0), _rel(got_m, m0))
    scale = max(abs(v) for v in dp.values())
    for i, k in enumerate(KEYS):
        assert abs(got_p[i] - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (k, got_p[i], dp[k])


@pytest.mark.parametrize("bc", BCS)
def test_step_bwd_equals_compact_even_adjoint_bitwise(bc):
    """rdcnn_step_bwd on a sparse trajectory and rdcnn_adjoint_even on the
    compact even-time trajectory of the same run give the same bits (same
    passes, states read at a different spacing)."""
    R, C, S = 90, 260, 45
    g = _gene(bc)
    x = W.uniform_x(R, C, 3)
    a = _sim(x, g, bc)
    sparse = torch.empty((S + 1, 2, R, C), device="cuda")
    a.step_record_sparse(S, sparse)
    b = _sim(x, g, bc)
    compact = torch.empty(((S + 1) // 2, 2, R, C), device="cuda")
    b.step_record_even(S, compact)
    assert torch.equal(a.state(), b.state())
    for q in range(0, S, 2):
        assert torch.equal(sparse[q], compact[q // 2]), q
    rng = np.random.default_rng(0)
    adj = torch.from_numpy(rng.standard_normal((2, R, C)).astype(np.float32)).cuda()
    lam, mu = adj[0].clone(), adj[1].clone()
    d1 = torch.zeros(8, dtype=torch.float64, device="cuda")
    d2 = torch.zeros_like(d1)
    a.step_bwd(sparse, S, lam, mu, d1)
    adj2 = adj.clone()
    b.adjoint_even(compact, S, adj2, torch.empty_like(adj2), d2)
    assert torch.equal(lam, adj2[0]) and torch.equal(mu, adj2[1])
    assert torch.equal(d1, d2)
    a.close()
    b.close()


@pytest.mark.parametrize("T,S", [(0, 5), (1, 1), (40, 8), (45, 45), (45, 7), (100, 16), (23, 50)])
@pytest.mark.parametrize("bc", BCS)
def test_step_checkpoints_bitwise(bc, T, S):
    """Checkpoint j equals the oracle's state after jS steps and the final
    state equals a plain run, bit for bit; passes are cut at multiples of S."""
    R, C = 70, 130
    g = _gene(bc)
    x = W.uniform_x(R, C, 11)
    sim = _sim(x, g, bc)
    nseg = -(-T // S)
    ckpt = torch.full((max(nseg, 1), 2, R, C), float("nan"), device="cuda")
    sim.step_checkpoints(T, S, ckpt)
    u, v = oracle.init_state(x, 1.0)
    for j in range(nseg):
        assert np.array_equal(ckpt[j, 0].cpu().numpy(), u) and \
            np.array_equal(ckpt[j, 1].cpu().numpy(), v), j
        u, v = oracle.run(u, v, g, bc, min(S, T - j * S), "f32")
    got = sim.read_host()
    assert np.array_equal(got[0], u) and np.array_equal(got[1], v)
    sim.close()


@pytest.mark.parametrize("T,S", [(1, 1), (23, 50), (40, 8), (45, 7), (45, 45), (100, 16), (61, 12)])
@pytest.mark.parametrize("bc", BCS)
def test_step_bwd_ckpt_through_cabi(bc, T, S):
    """rdcnn_step_bwd_ckpt (the library's checkpoint-and-recompute backward,
    recompute on a second stream) called with raw device pointers: (lam, mu)
    bit for bit equal to rdcnn_step_bwd run segment by segment on a serially
    recomputed trajectory, dJ/dp equal up to the order of the final double
    sum, and both against the oracle's float64 reverse pass (1e-4 / 1e-3)."""
    from paper_2102_10340_amd._lib import check, lib
    R, C = 70, 130
    g = _gene(bc)
    x = W.uniform_x(R, C, T + 3 * S)
    nseg = -(-T // S)
    rng = np.random.default_rng(T * S)
    lam0 = rng.standard_normal((R, C)).astype(np.float32)
    mu0 = rng.standard_normal((R, C)).astype(np.float32)
    sim = _sim(x, g, bc)
    ckpt = torch.empty((nseg, 2, R, C), device="cuda")
    sim.step_checkpoints(T, S, ckpt)
    lam = torch.from_numpy(lam0).cuda()
    mu = torch.from_numpy(mu0).cuda()
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    work = torch.full((2 * (min(S, T) + 1), 2, R, C), float("nan"), device="cuda")
    print(f"case step_bwd_ckpt {bc} T={T} S={S}", flush=True)
    check(lib.rdcnn_step_bwd_ckpt(sim._h, ckpt.data_ptr(), T, S, work.data_ptr(), lam.data_ptr(),
                                  mu.data_ptr(), dth.data_ptr()))
    got_l, got_m, got_p = lam.cpu().numpy(), mu.cpu().numpy(), dth.cpu().numpy()
    # serial reference: the same passes, segment by segment, one stream
    lam2 = torch.from_numpy(lam0).cuda()
    mu2 = torch.from_numpy(mu0).cuda()
    dth2 = torch.zeros(8, dtype=torch.float64, device="cuda")
    seg = torch.empty((min(S, T) + 1, 2, R, C), device="cuda")
    for k in range(nseg - 1, -1, -1):
        L = min(S, T - k * S)
        sim.write_state_packed(ckpt[k])
        sim.step_record_sparse(L, seg)
        sim.step_bwd(seg, L, lam2, mu2, dth2)
    assert np.array_equal(got_l, lam2.cpu().numpy()) and np.array_equal(got_m, mu2.cpu().numpy())
    ref_p = dth2.cpu().numpy()
    assert np.abs(got_p - ref_p).max() <= 1e-12 * np.abs(ref_p).max()
    sim.close()
    l0, m0, dp, _, _ = oracle.grad(x, x, g, bc, T, lam0, mu0, traj="f32")
    assert _rel(got_l, l0) < 1e-4 and _rel(got_m, m0) < 1e-4, (_rel(got_l, l0), _rel(got_m, m0))
    scale = max(abs(v) for v in dp.values())
    for i, k in enumerate(KEYS):
        assert abs(got_p[i] - dp[k]) <= 1e-3 * max(abs(dp[k]), 1e-3 * scale), (k, got_p[i], dp[k])


def test_step_bwd_ckpt_two_handles_share_the_recompute_stream():
    """Two handles on two streams of one device run rdcnn_step_bwd_ckpt back to
    back with no synchronisation between the calls.  The recompute stream is
    the device's and both queue their recomputes on it; each result is bit for
    bit what the same handle gives when it runs alone."""
    from paper_2102_10340_amd._lib import check, lib
    cases = [(70, 130, "zeroflux", 41, 9), (96, 64, "periodic", 60, 16)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rng = np.random.default_rng(7)
    setups = []
    for (R, C, bc, T, S), s in zip(cases, streams):
        with torch.cuda.stream(s):
            g = _gene(bc)
            x = W.uniform_x(R, C, T + S)
            sim = _sim(x, g, bc)
            nseg = -(-T // S)
            ckpt = torch.empty((nseg, 2, R, C), device="cuda")
            sim.step_checkpoints(T, S, ckpt)
            lam0 = torch.from_numpy(rng.standard_normal((R, C)).astype(np.float32)).cuda()
            mu0 = torch.from_numpy(rng.standard_normal((R, C)).astype(np.float32)).cuda()
            work = torch.empty((2 * (min(S, T) + 1), 2, R, C), device="cuda")
            setups.append((sim, s, ckpt, T, S, work, lam0, mu0))
    torch.cuda.synchronize()

    def run(sim, s, ckpt, T, S, work, lam0, mu0):
        with torch.cuda.stream(s):
            lam, mu = lam0.clone(), mu0.clone()
            dth = torch.zeros(8, dtype=torch.float64, device="cuda")
            check(lib.rdcnn_step_bwd_ckpt(sim._h, ckpt.data_ptr(), T, S, work.data_ptr(),
                                          lam.data_ptr(), mu.data_ptr(), dth.data_ptr()))
        return lam, mu, dth

    alone = []
    for st in setups:
        alone.append(run(*st))
        torch.cuda.synchronize()
    for rep in range(3):
        print(f"case two handles, shared recompute stream, rep {rep}", flush=True)
        together = [run(*st) for st in setups]  # queued back to back, no sync
        torch.cuda.synchronize()
        for a, b in zip(alone, together):
            for u, v in zip(a, b):
                assert torch.equal(u, v)
    for st in setups:
        st[0].close()


def test_step_bwd_ckpt_rejects_bad_arguments():
    from paper_2102_10340_amd._lib import EINVAL, lib
    R, C, T, S = 16, 20, 12, 4
    sim = _sim(W.uniform_x(R, C, 1), W.PLAIN_GENE, "zeroflux")
    ckpt = torch.zeros((3, 2, R, C), device="cuda")
    work = torch.zeros((2 * (S + 1), 2, R, C), device="cuda")
    lam = torch.zeros((R, C), device="cuda")
    mu = torch.zeros((R, C), device="cuda")
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    f = lib.rdcnn_step_bwd_ckpt
    assert f(sim._h, ckpt.data_ptr(), T, 0, work.data_ptr(), lam.data_ptr(), mu.data_ptr(),
             dth.data_ptr()) == EINVAL                                  # S < 1
    assert f(sim._h, ckpt.data_ptr(), -1, S, work.data_ptr(), lam.data_ptr(), mu.data_ptr(),
             dth.data_ptr()) == EINVAL                                  # T < 0
    assert f(sim._h, ckpt.data_ptr(), T, S, work.data_ptr(), lam.data_ptr(), lam.data_ptr(),
             dth.data_ptr()) == EINVAL                                  # lam == mu
    assert f(sim._h, ckpt.data_ptr(), T, S, work.data_ptr(), work[3, 0].data_ptr(),
             mu.data_ptr(), dth.data_ptr()) == EINVAL                   # lam inside the workspace
    assert f(sim._h, ckpt.data_ptr(), T, S, ckpt.data_ptr(), lam.data_ptr(), mu.data_ptr(),
             dth.data_ptr()) == EINVAL                                  # workspace over checkpoints
    assert f(sim._h, ckpt.data_ptr(), 0, S, None, None, None, None) == 0  # T = 0: nothing to do
    sim.close()


def test_sparse_recording_leaves_odd_slots():
    """rdcnn_step_record_sparse writes the even slots only."""
    R, C, T = 40, 70, 17
    x = W.uniform_x(R, C, 5)
    sim = _sim(x, W.PLAIN_GENE, "zeroflux")
    st = torch.full((T + 1, 2, R, C), 7.25, device="cuda")
    sim.step_record_sparse(T, st)
    u, v = oracle.init_state(x, 1.0)
    for q in range(T + 1):
        if q % 2 == 0 and q < T:
            assert np.array_equal(st[q, 0].cpu().numpy(), u), q
        else:
            assert bool(torch.all(st[q] == 7.25)), q
        u, v = oracle.run(u, v, W.PLAIN_GENE, "zeroflux", 1, "f32")
    sim.close()


def test_step_bwd_rejects_overlapping_buffers():
    from paper_2102_10340_amd._lib import EINVAL, lib
    R, C, S = 16, 20, 4
    sim = _sim(W.uniform_x(R, C, 1), W.PLAIN_GENE, "zeroflux")
    st = torch.zeros((S + 1, 2, R, C), device="cuda")
    lam = torch.zeros((R, C), device="cuda")
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = st[S, 0]
    assert lib.rdcnn_step_bwd(sim._h, st.data_ptr(), S, ws.data_ptr(), lam.data_ptr(),
                              dth.data_ptr()) == EINVAL
    assert lib.rdcnn_step_bwd(sim._h, st.data_ptr(), S, lam.data_ptr(), lam.data_ptr(),
                              dth.data_ptr()) == EINVAL
    assert lib.rdcnn_step_bwd(sim._h, st.data_ptr(), -1, lam.data_ptr(), ws.data_ptr(),
                              dth.data_ptr()) == EINVAL
    sim.close()


def test_finite_check_on_read():
    """A state holding NaN or Inf: reads with the check on return
    RDCNN_ENONFINITE (the copy is still made); with it off they succeed."""
    from paper_2102_10340_amd._lib import ENONFINITE, RDCNNError
    R, C = 50, 80
    sim = _sim(W.uniform_x(R, C, 2), W.PLAIN_GENE, "zeroflux")
    sim.set_check_finite(True)
    sim.step(3)
    sim.read()  # finite: no error
    u = torch.from_numpy(W.uniform_x(R, C, 3)).cuda()
    v = u.clone()
    v[7, 9] = float("inf")
    u[0, 0] = float("nan")
    sim.write_state(u, v)
    with pytest.raises(RDCNNError) as e:
        sim.read_host()
    assert e.value.code == ENONFINITE and "2 non-finite" in str(e.value)
    sim.set_check_finite(False)
    uu, vv = sim.read_host()
    assert np.isnan(uu[0, 0]) and np.isinf(vv[7, 9])
    sim.close()


def test_batch_read_and_finite_check():
    from paper_2102_10340_amd import Batch
    from paper_2102_10340_amd._lib import ENONFINITE, RDCNNError
    xs = [torch.from_numpy(W.uniform_x(r, c, r + c)).cuda() for r, c in ((30, 40), (17, 5), (64, 64))]
    b = Batch(xs, [W.PLAIN_GENE] * 3, "zeroflux")
    b.step(9)
    out = torch.full((b.total,), -3.0, device="cuda")
    b.read_into(out)
    assert torch.equal(out, b.current())
    b.set_check_finite(True)
    b.read_into(out)
    bad = b.current().clone()
    bad[b.offsets[2] + 5] = float("nan")
    b.write_state(bad)
    with pytest.raises(RDCNNError) as e:
        b.read_into(out)
    assert e.value.code == ENONFINITE
    b.close()


def test_batch_shared_gradient_is_instance_sum():
    """Shared parameters: the device sum over instances equals the per-instance
    rows summed in instance order on the host (the same float64 additions)."""
    from paper_2102_10340_amd import Batch
    shapes = [(40, 70), (64, 64), (17, 130), (90, 33)]
    xs = [torch.from_numpy(W.uniform_x(r, c, 9 + r)).cuda() for r, c in shapes]
    g = W.gene(Du=0.09, Dv=0.7)
    T = 12
    rows = None
    for shared in (False, True):
        b = Batch(xs, [g] * len(xs), "zeroflux")
        traj = torch.empty(((T + 1) // 2, b.total), device="cuda")
        b.step_record_even(T, traj)
        adj = torch.from_numpy(np.random.default_rng(4).standard_normal(b.total).astype(np.float32)).cuda()
        b.set_shared_grad(shared)
        dth = torch.zeros((8,) if shared else (len(xs), 8), dtype=torch.float64, device="cuda")
        b.adjoint_even(traj, T, adj, torch.empty_like(adj), 0xFF, dth)
        if not shared:
            rows = dth.cpu().numpy()
        else:
            want = np.zeros(8)
            for i in range(len(xs)):
                want = want + rows[i]
            assert np.array_equal(dth.cpu().numpy(), want)
        b.close()
