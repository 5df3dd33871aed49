"""GPU parity of the per-instance atlas statistics (rdcnn_batch_stats, after
Sec. III.A) against the oracle's definitions: counts and the largest change
exactly, the moments within a tolerance derived from double summation."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import atlas as oracle_atlas

pytestmark = pytest.mark.gpu

# Double sums of N float32 values of size O(1): the two summation orders differ
# by at most ~N * 2^-53 relative; with N <= 2^20 that is below 1e-10.
RTOL, ATOL = 1e-9, 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _check(got, u, v, prev, ref, tf, tm, what):
    want = oracle_atlas.instance_stats(u, v, prev, ref, tf, tm)
    assert np.array_equal(np.isnan(got), np.isnan(want)), (what, got, want)
    for k in (4, 5, 6):  # exact: float32 decisions and the float32 maximum
        if not np.isnan(want[k]):
            assert got[k] == want[k], (what, k, got[k], want[k])
    for k in (0, 1, 2, 3, 7):
        if not np.isnan(want[k]):
            assert abs(got[k] - want[k]) <= ATOL + RTOL * abs(want[k]), (what, k, got[k], want[k])


# ragged sizes: N % 4 != 0 (scalar path), N % 4 == 0 (vector path), chunk tails
SHAPES = [(1, 1), (3, 7), (300, 257), (64, 64), (128, 128), (600, 200), (2, 1000), (257, 300),
          (129, 127), (130, 126)]


@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_stats_match_oracle(bc):
    from paper_2102_10340_amd import Batch
    rng = np.random.default_rng(7)
    xs = [W.uniform_x(R, C, 40 + i) for i, (R, C) in enumerate(SHAPES)]
    genes = [W.gene(Du=rng.uniform(0.01, 0.2), Dv=rng.uniform(0.2, 1.0), eps=-rng.uniform(0.02, 0.2))
             for _ in SHAPES]
    b = Batch([torch.from_numpy(x).cuda() for x in xs], genes, bc)
    ref = rng.uniform(-0.5, 0.5, len(SHAPES)).astype(np.float32)
    s0 = b.stats(None, torch.from_numpy(ref).cuda(), 0.3, 0.0).cpu().numpy()
    for i, x in enumerate(xs):
        _check(s0[i], x, x, None, ref[i], 0.3, 0.0, ("init", i))
    b.step(17)
    prev = b.snapshot()
    prev_states = [b.state(i).cpu().numpy() for i in range(len(xs))]
    b.step(9)
    s1 = b.stats(prev, torch.from_numpy(ref).cuda(), 0.5, 1e-3).cpu().numpy()
    s2 = b.stats(prev, torch.from_numpy(ref).cuda(), 0.5, 1e-3).cpu().numpy()
    assert np.array_equal(s1.view(np.int64), s2.view(np.int64))  # deterministic
    for i in range(len(xs)):
        st = b.state(i).cpu().numpy()
        _check(s1[i], st[0], st[1], prev_states[i][0], ref[i], 0.5, 1e-3, ("step", i))
    # default reference 0 and zero thresholds
    s3 = b.stats(prev).cpu().numpy()
    for i in range(len(xs)):
        st = b.state(i).cpu().numpy()
        _check(s3[i], st[0], st[1], prev_states[i][0], 0.0, 0.0, 0.0, ("ref0", i))
    b.close()


def test_stats_uniform_field_variance_is_exact():
    """A uniform instance (the homogeneous class) has variance 0 exactly: the
    sums are taken on values shifted by the first cell."""
    from paper_2102_10340_amd import Batch
    x = np.full((300, 300), np.float32(1.1399983), dtype=np.float32)
    b = Batch([torch.from_numpy(x).cuda()], [W.PLAIN_GENE], "periodic")
    s = b.stats(None, None, 0.0, 0.0).cpu().numpy()[0]
    assert s[1] == 0.0 and s[3] == 0.0 and s[0] == float(np.float32(1.1399983))
    b.close()


def test_stats_reject_bad_thresholds():
    from paper_2102_10340_amd import Batch, RDCNNError
    b = Batch([torch.zeros((4, 4), device="cuda")], [W.PLAIN_GENE])
    for tf, tm in [(-1.0, 0.0), (0.0, float("nan")), (float("inf"), 0.0)]:
        with pytest.raises(RDCNNError):
            b.stats(None, None, tf, tm)
    b.close()


def test_stats_on_sweep_workload_sampled():
    """The 1024-instance sweep at full size (sides 128..1024), stats of every
    instance in one call after 240 steps: twelve instances, including the largest
    (64 chunks each), checked against the oracle."""
    from paper_2102_10340_amd import Batch
    inst = W.sweep_instances(1024, 0)
    xs = [torch.from_numpy(W.uniform_x(d["rows"], d["cols"], d["seed"])).cuda() for d in inst]
    b = Batch(xs, [d["gene"] for d in inst], "zeroflux")
    b.step(200)
    prev = b.snapshot()
    picks = [i for i, d in enumerate(inst) if d["rows"] == 1024][:3]
    picks += list(np.random.default_rng(3).choice(len(inst), 9, replace=False))
    before = {i: b.state(int(i))[0].cpu().numpy() for i in picks}
    b.step(40)
    s = b.stats(prev, None, 0.5, 1e-4).cpu().numpy()
    assert s.shape == (1024, 8) and np.isfinite(s).all()
    for i in picks:
        st = b.state(int(i)).cpu().numpy()
        _check(s[i], st[0], st[1], before[i], 0.0, 0.5, 1e-4, ("sweep", int(i)))
    b.close()
