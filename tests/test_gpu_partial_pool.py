"""The adjoint's per-tile partial-sum buffers come from a process-wide pool:
rdcnn_destroy returns a handle's buffer with an event on the handle's stream,
and the next handle to take it, possibly on another stream, waits for that
event.  Handles created and destroyed back to back on two streams, each
returning its buffer while its own work may still be queued, must give the
same bits as the same runs one at a time on one stream."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(96, 80), (64, 64), (130, 40), (33, 257)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _case(k, T=26):
    from paper_2102_10340_amd import Simulation
    R, C = SHAPES[k % len(SHAPES)]
    x = torch.from_numpy(W.uniform_x(R, C, 200 + k)).cuda()
    w = torch.from_numpy(np.random.default_rng(k).standard_normal((2, R, C)).astype(np.float32)).cuda()
    sim = Simulation(x, W.gene(Du=0.05 + 0.01 * k, Dv=0.6), "zeroflux")
    even = torch.empty(((T + 1) // 2, 2, R, C), device="cuda")
    sim.step_record_even(T, even)
    adj = w.clone()
    tmp = torch.empty_like(adj)
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    sim.adjoint_even(even, T, adj, tmp, dth)
    sim.close()  # the buffer goes back to the pool; the work may still be queued
    return adj, dth


def test_pooled_partials_across_streams():
    n = 12
    refs = []
    for k in range(n):
        refs.append(_case(k))
        torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = []
    for k in range(n):
        with torch.cuda.stream(streams[k % 2]):
            got.append(_case(k))
    torch.cuda.synchronize()
    for k in range(n):
        assert torch.equal(got[k][0], refs[k][0]), ("dJ/ds", k)
        assert torch.equal(got[k][1], refs[k][1]), ("dJ/dtheta", k)
