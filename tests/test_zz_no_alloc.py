"""GPU test of rdcnn_step_bwd_noalloc, the reverse pass that allocates nothing
(its partial sums live in a static device array): called through the C ABI, it
must give the same bits as rdcnn_step_bwd on the same inputs, on two calls in a
row of which the second is smaller (the array keeps the first call's sums and
must be cleared), and it must reject a tiling larger than the array."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2102_10340_amd  # noqa: F401


def _case(R, C, S, bc, seed):
    """(lam, mu, dtheta) from rdcnn_step_bwd and from rdcnn_step_bwd_noalloc on
    one recorded segment of S steps of an R x C grid."""
    from paper_2102_10340_amd import Simulation
    from paper_2102_10340_amd._lib import check, lib
    g = W.gene(Du=0.1, Dv=0.5) if bc == "zeroflux" else \
        W.gene(W.PAPER_DEFAULT_GENE, k3=0.45, Du=0.08, Dv=0.6)
    x = W.uniform_x(R, C, seed)
    sim = Simulation(torch.from_numpy(x).cuda(), g, bc, 1.0)
    states = torch.empty((S + 1, 2, R, C), device="cuda")
    sim.step_record_sparse(S, states)
    rng = np.random.default_rng(seed)
    lam0 = torch.from_numpy(rng.standard_normal((R, C)).astype(np.float32)).cuda()
    mu0 = torch.from_numpy(rng.standard_normal((R, C)).astype(np.float32)).cuda()
    out = {}
    for name in ("rdcnn_step_bwd", "rdcnn_step_bwd_noalloc"):
        st = states.clone()  # slot S is each call's workspace
        lam, mu = lam0.clone(), mu0.clone()
        dth = torch.full((8,), 0.25, dtype=torch.float64, device="cuda")  # accumulated into
        print(f"case {name} {R}x{C} S={S} {bc}", flush=True)
        check(getattr(lib, name)(sim._h, st.data_ptr(), S, lam.data_ptr(), mu.data_ptr(),
                                 dth.data_ptr()))
        torch.cuda.synchronize()
        out[name] = (lam.cpu(), mu.cpu(), dth.cpu())
    sim.close()
    return out["rdcnn_step_bwd"], out["rdcnn_step_bwd_noalloc"]


def _same(ref, got):
    for a, b, what in zip(ref, got, ("lam", "mu", "dtheta")):
        assert torch.equal(a, b), what


@pytest.mark.parametrize("bc", ["zeroflux", "periodic"])
def test_noalloc_equals_step_bwd_on_two_calls(bc):
    """A large call then a smaller one (fewer tiles, fewer steps): both give
    rdcnn_step_bwd's bits."""
    ref, got = _case(1024, 1024, 30, bc, 1)
    _same(ref, got)
    ref, got = _case(77, 130, 9, bc, 2)
    _same(ref, got)


def test_noalloc_rejects_tiling_beyond_workspace():
    """Two-step passes on 4-row segments of a 4096^2 grid need 70656 tiles,
    more than the static array's 65536: EINVAL with a message, no launch."""
    from paper_2102_10340_amd import Simulation
    from paper_2102_10340_amd._lib import EINVAL, last_error, lib
    R = C = 4096
    sim = Simulation(torch.zeros((R, C), device="cuda"), W.gene(), "zeroflux", 1.0)
    sim.set_adjoint_kernel(2, 1, 4)
    states = torch.zeros((3, 2, R, C), device="cuda")
    lam = torch.zeros((R, C), device="cuda")
    mu = torch.zeros((R, C), device="cuda")
    dth = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = lib.rdcnn_step_bwd_noalloc(sim._h, states.data_ptr(), 2, lam.data_ptr(), mu.data_ptr(),
                                    dth.data_ptr())
    msg = last_error()
    assert rc == EINVAL and "70656 tiles" in msg and "65536" in msg, (rc, msg)
    # the same request through the pooled entry point still runs
    rc = lib.rdcnn_step_bwd(sim._h, states.data_ptr(), 2, lam.data_ptr(), mu.data_ptr(),
                            dth.data_ptr())
    torch.cuda.synchronize()
    assert rc == 0, last_error()
    sim.close()
