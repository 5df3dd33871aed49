"""GPU tests of rdcnn_use_graph: a single grid's rdcnn_step replayed from a
captured HIP graph gives the same bits as eager launches on every replay, with
the program's own eager work between replays, for both starting buffers (odd
pass counts flip the buffer), after a parameter or pass-shape change (which
drops the graph), and against the float32 oracle."""
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


@pytest.mark.parametrize("T", [16, 20, 3])
@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_graph_replays_match_eager(bc, T):
    from paper_2102_10340_amd import Simulation
    R, C = 96, 200
    g = W.PLAIN_GENE if bc == "zeroflux" else W.PAPER_DEFAULT_GENE
    x = W.uniform_x(R, C, T)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xt = torch.from_numpy(x).cuda()
        eager = Simulation(xt, g, bc)
        graph = Simulation(xt, g, bc).use_graph(True)
        ou, ov = oracle.init_state(x, 1.0)
        for rep in range(5):
            print(f"case graph {bc} T={T} replay {rep}", flush=True)
            eager.step(T)
            graph.step(T)
            (eager.state() * 2.0).sum()  # eager work between replays
            s.synchronize()
            assert torch.equal(eager.state(), graph.state()), rep
            ou, ov = oracle.run(ou, ov, g, bc, T, "f32")
            gu, gv = graph.read_host()
            assert np.array_equal(gu, ou) and np.array_equal(gv, ov), rep
        eager.close()
        graph.close()


def test_graph_dropped_on_parameter_and_kernel_change():
    from paper_2102_10340_amd import Simulation
    R, C, T = 64, 130, 12
    x = W.uniform_x(R, C, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xt = torch.from_numpy(x).cuda()
        eager = Simulation(xt, W.PLAIN_GENE, "zeroflux")
        graph = Simulation(xt, W.PLAIN_GENE, "zeroflux").use_graph(True)
        g2 = W.gene(Du=0.11, Dv=0.4)
        for step, change in enumerate((None, "params", "kernel", None, "off")):
            if change == "params":
                eager.set_params(g2)
                graph.set_params(g2)
            elif change == "kernel":
                eager.set_kernel(2, 4, 2, 8)
                graph.set_kernel(2, 4, 2, 8)
            elif change == "off":
                graph.use_graph(False)
            eager.step(T)
            graph.step(T)
            s.synchronize()
            assert torch.equal(eager.state(), graph.state()), (step, change)
        eager.close()
        graph.close()


def test_graph_for_other_cell_model():
    from paper_2102_10340_amd import Simulation
    R, C, T = 80, 120, 9
    rng = np.random.default_rng(3)
    u = torch.from_numpy(np.ones((R, C), np.float32)).cuda()
    v = torch.from_numpy(rng.uniform(0, 0.3, (R, C)).astype(np.float32)).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        eager = Simulation.gray_scott(u, v, 0.5, 0.037, 0.06, 0.2, 0.1, "periodic")
        graph = Simulation.gray_scott(u, v, 0.5, 0.037, 0.06, 0.2, 0.1, "periodic").use_graph(True)
        for rep in range(3):
            eager.step(T)
            graph.step(T)
            s.synchronize()
            assert torch.equal(eager.state(), graph.state()), rep
        eager.close()
        graph.close()


def test_graph_needs_a_stream():
    from paper_2102_10340_amd import Simulation
    from paper_2102_10340_amd._lib import RDCNNError
    x = torch.from_numpy(W.uniform_x(8, 8, 0)).cuda()
    sim = Simulation(x, W.PLAIN_GENE, "zeroflux")  # torch's default (NULL) stream
    with pytest.raises(RDCNNError):
        sim.use_graph(True)
    sim.close()
