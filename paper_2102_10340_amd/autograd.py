"""Differentiable RD-CNN runs: torch.autograd.Function wrappers around the
library's forward, checkpointing, recording and reverse-pass calls.

The reverse pass is rdcnn_step_bwd: it reads the states of even times of a
recorded segment and rebuilds each odd state from the even one before it with
the forward cell update, bit-identical to the forward pass, so the gradients
equal those of a fully recorded trajectory.  The schedule is chosen by S:
* S = 0 (default) or S > 0, checkpoint-and-recompute (the differentiation
  workload's schedule): the forward keeps one checkpoint every S steps
  (rdcnn_step_checkpoints; each is written by the pass that ends there); the
  backward (rdcnn_step_bwd_ckpt) walks the segments from last to first,
  re-runs each from its checkpoint recording its even states and runs the
  reverse passes of rdcnn_step_bwd through them.  The recompute of segment k
  needs only checkpoint k, so the library runs it on a second stream while
  the reverse pass of segment k+1 runs on the caller's stream (two segment
  buffers in turn).
  S = 0 picks S = ceil(sqrt(T)) rounded up to the forward's pass depth of 8,
  so checkpoints fall on pass boundaries: O(sqrt(T)) states of memory.
* S = -1, whole trajectory: the forward records the even states of all T
  steps and the backward runs rdcnn_step_bwd straight through them (memory
  O(T) states; an MI355X's 288 GB holds 1024x1024 x 2000 steps many times).
With no input needing a gradient the forward records nothing.

Parameters travel as a tensor theta of 8 values in the order
(dt, a, b, eps, c, k3, Du, Dv), the paper's gene (Sec. II.A) plus the cubic
coefficient; its gradient is float64 from the library, cast to theta's dtype.
"""
from __future__ import annotations

import math

import torch

from ._lib import PARAM_FIELDS
from .sim import Simulation, init_backward

PASS_DEPTH = 8  # steps per pass of the library's forward kernels


def default_segment(T: int) -> int:
    """ceil(sqrt(T)) rounded up to a multiple of the forward pass depth."""
    s = max(1, math.ceil(math.sqrt(max(T, 1))))
    s = -(-s // PASS_DEPTH) * PASS_DEPTH
    return max(1, min(s, T if T > 0 else 1))


def choose_schedule(T: int, rows: int, cols: int, S: int, device=None) -> int:
    """-1 (record the whole trajectory) or a checkpoint spacing > 0."""
    if S < 0:
        return -1
    if S > 0:
        return S
    return default_segment(T)


def grad_mask(grads) -> int:
    """Bit mask for the parameters named in `grads` (None or "all": all eight)."""
    if grads is None or grads == "all":
        return 0xFF
    m = 0
    for name in grads:
        m |= 1 << PARAM_FIELDS.index(name)
    return m


def _gene(theta: torch.Tensor):
    vals = theta.detach().to("cpu", torch.float64).tolist()
    if len(vals) != 8:
        raise ValueError("theta must hold 8 values (dt, a, b, eps, c, k3, Du, Dv)")
    return dict(zip(PARAM_FIELDS, vals))


def _forward(sim: Simulation, T: int, S: int, dev, record: bool = True):
    """Run T steps; returns (u_T, v_T, saved states, number of segments)."""
    R, C = sim.rows, sim.cols
    if not record:
        sim.step(T)
        u, v = sim.read()
        return u, v, None, 0
    if S < 0:  # whole trajectory: even-time states in their own slots, slot T = workspace
        states = torch.empty((T + 1, 2, R, C), dtype=torch.float32, device=dev)
        sim.step_record_sparse(T, states)
        u, v = sim.read()
        return u, v, states, 0
    nseg = -(-T // S) if T > 0 else 0
    ckpt = torch.empty((max(nseg, 1), 2, R, C), dtype=torch.float32, device=dev)
    sim.step_checkpoints(T, S, ckpt)
    u, v = sim.read()
    return u, v, ckpt, nseg


def _backward(sim: Simulation, ckpt, nseg: int, T: int, S: int, gu, gv, dev, kernel=None,
              mask: int = 0xFF, overlap: bool = True):
    R, C = sim.rows, sim.cols
    lam = gu.detach().contiguous().clone() if gu is not None else \
        torch.zeros((R, C), dtype=torch.float32, device=dev)
    mu = gv.detach().contiguous().clone() if gv is not None else \
        torch.zeros((R, C), dtype=torch.float32, device=dev)
    dtheta = torch.zeros(8, dtype=torch.float64, device=dev)
    if kernel is not None:
        sim.set_adjoint_kernel(*kernel)
    sim.set_grad_mask(mask)
    if S < 0:  # ckpt holds the whole trajectory's even-time states
        sim.step_bwd(ckpt, T, lam, mu, dtheta)
        return lam, mu, dtheta
    Smax = min(S, max(T, 1))
    if not overlap or nseg < 2:
        seg = torch.empty((Smax + 1, 2, R, C), dtype=torch.float32, device=dev)
        for k in range(nseg - 1, -1, -1):
            L = min(S, T - k * S)
            sim.write_state_packed(ckpt[k])
            sim.step_record_sparse(L, seg)
            sim.step_bwd(seg, L, lam, mu, dtheta)
        return lam, mu, dtheta
    # The library runs the whole schedule: segment k recomputed on its second
    # stream while the reverse pass of segment k+1 runs on this one, two
    # segment buffers in turn, the partial sums folded once at the end.
    work = torch.empty((2 * (Smax + 1), 2, R, C), dtype=torch.float32, device=dev)
    sim.step_bwd_ckpt(ckpt, T, S, work, lam, mu, dtheta)
    return lam, mu, dtheta


def _release(ctx):
    if ctx.sim is not None:
        ctx.sim.close()
    ctx.sim = None
    ctx.ckpt = None


def _check_once(ctx):
    if ctx.sim is None:
        raise RuntimeError("the saved trajectory of this RD-CNN run was released by its first "
                           "backward; run the forward again to differentiate it again")


class RDCNNFunction(torch.autograd.Function):
    """(x, theta) -> (u_T, v_T) with u_0 = v_0 = ka x (Eq. (1)) and T steps."""

    @staticmethod
    def forward(ctx, x, theta, T: int, bc: str = "zeroflux", ka: float = 1.0, S: int = 0,
                adj_kernel=None, mask: int = 0xFF):
        x = x.detach().contiguous()
        T = int(T)
        S = choose_schedule(T, x.shape[0], x.shape[1], int(S), x.device)
        record = bool(ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
        sim = Simulation(x, _gene(theta), bc, ka, tuned=True)
        u, v, ckpt, nseg = _forward(sim, T, S, x.device, record)
        if not record:
            sim.close()
            sim = None
        ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, ctx.ka = sim, ckpt, nseg, T, S, ka
        ctx.adj_kernel, ctx.mask = adj_kernel, mask
        ctx.theta_meta = (theta.dtype, theta.device)
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        _check_once(ctx)
        dev = ctx.ckpt.device
        lam, mu, dtheta = _backward(ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, gu, gv, dev,
                                    ctx.adj_kernel, ctx.mask)
        gx = init_backward(torch.stack((lam, mu)), ctx.ka)
        _release(ctx)
        dt, dd = ctx.theta_meta
        return gx, dtheta.to(device=dd, dtype=dt), None, None, None, None, None, None


class RDCNNStateFunction(torch.autograd.Function):
    """(u0, v0, theta) -> (u_T, v_T): T steps from an explicit state."""

    @staticmethod
    def forward(ctx, u0, v0, theta, T: int, bc: str = "zeroflux", S: int = 0, adj_kernel=None,
                mask: int = 0xFF):
        u0 = u0.detach().contiguous()
        v0 = v0.detach().contiguous()
        T = int(T)
        S = choose_schedule(T, u0.shape[0], u0.shape[1], int(S), u0.device)
        record = bool(any(ctx.needs_input_grad[:3]))
        sim = Simulation.from_state(u0, v0, _gene(theta), bc, tuned=True)
        u, v, ckpt, nseg = _forward(sim, T, S, u0.device, record)
        if not record:
            sim.close()
            sim = None
        ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S = sim, ckpt, nseg, T, S
        ctx.adj_kernel, ctx.mask = adj_kernel, mask
        ctx.theta_meta = (theta.dtype, theta.device)
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        _check_once(ctx)
        dev = ctx.ckpt.device
        lam, mu, dtheta = _backward(ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, gu, gv, dev,
                                    ctx.adj_kernel, ctx.mask)
        _release(ctx)
        dt, dd = ctx.theta_meta
        return lam, mu, dtheta.to(device=dd, dtype=dt), None, None, None, None, None


def simulate(x, theta, T, bc="zeroflux", ka=1.0, S=0, grads=None):
    """Differentiable T-step run from u = v = ka x; returns (u_T, v_T).
    S: 0 checkpoint every ceil(sqrt(T)) steps (rounded up to 8), > 0 every S
    steps, -1 record the whole trajectory.  grads: parameter names whose
    gradients are formed (default all); the others come back NaN in theta.grad."""
    return RDCNNFunction.apply(x, theta, T, bc, ka, S, None, grad_mask(grads))


def simulate_state(u0, v0, theta, T, bc="zeroflux", S=0, grads=None):
    """Differentiable T-step run from (u0, v0); returns (u_T, v_T)."""
    return RDCNNStateFunction.apply(u0, v0, theta, T, bc, S, None, grad_mask(grads))


# ---------------------------------------------------------------- batches

class RDCNNBatchFunction(torch.autograd.Function):
    """(theta, x_1 .. x_n) -> (u_T,1, v_T,1, ..., u_T,n, v_T,n) of a batch,
    u_0 = v_0 = ka x_i.  theta is [8] (shared by every instance) or [n, 8] (one
    gene per instance).  The forward records the packed states of even times
    when they fit a quarter of the free memory (else a checkpoint every S
    steps); the backward runs the batched paired reverse passes.  Separate outputs per instance
    keep autograd from forming a full-size gradient per instance."""

    @staticmethod
    def forward(ctx, theta, T: int, bc: str, ka: float, S: int, mask: int, *xs):
        from .batch import Batch
        xs = [x.detach().contiguous() for x in xs]
        n = len(xs)
        th = theta.detach().to("cpu", torch.float64)
        if th.dim() == 1:
            genes = [dict(zip(PARAM_FIELDS, th.tolist()))] * n
        elif tuple(th.shape) == (n, 8):
            genes = [dict(zip(PARAM_FIELDS, th[i].tolist())) for i in range(n)]
        else:
            raise ValueError("theta must be [8] or [n, 8]")
        b = Batch(xs, genes, bc, ka, tuned=False)
        dev = xs[0].device
        T = int(T)
        if S == 0:
            free, _ = torch.cuda.mem_get_info(dev)
            S = -1 if 4 * b.total * max((T + 1) // 2, 1) <= free // 4 else \
                max(1, math.ceil(math.sqrt(T)))
        if S < 0:
            store = torch.empty((max((T + 1) // 2, 1), b.total), dtype=torch.float32, device=dev)
            b.step_record_even(T, store)
            nseg = 0
        else:
            nseg = -(-T // S) if T > 0 else 0
            store = torch.empty((max(nseg, 1), b.total), dtype=torch.float32, device=dev)
            for k in range(nseg):
                b.read_into(store[k])
                b.step(min(S, T - k * S))
        outs = []
        for i in range(n):
            st = b.state(i)
            outs += [st[0].clone(), st[1].clone()]
        b.set_shared_grad(th.dim() == 1)
        ctx.b, ctx.store, ctx.nseg, ctx.T, ctx.S, ctx.ka, ctx.mask = b, store, nseg, T, S, ka, mask
        ctx.theta_meta = (theta.dtype, theta.device, theta.dim())
        return tuple(outs)

    @staticmethod
    def backward(ctx, *gouts):
        if ctx.b is None:
            raise RuntimeError("the saved trajectory of this batch run was released by its "
                               "first backward; run the forward again to differentiate it again")
        b, T, S = ctx.b, ctx.T, ctx.S
        adj = torch.zeros(b.total, dtype=torch.float32, device=b.device)
        for i in range(len(b)):
            a = b.view(adj, i)
            for layer in range(2):
                gg = gouts[2 * i + layer]
                if gg is not None:
                    a[layer].copy_(gg)
        tmp = torch.empty_like(adj)
        dt, dd, dim = ctx.theta_meta
        # shared parameters: the library sums the instances' gradients on the
        # device in a fixed order (rdcnn_batch_set_shared_grad)
        dtheta = torch.zeros((8,) if dim == 1 else (len(b), 8), dtype=torch.float64,
                             device=adj.device)
        if S < 0:
            b.adjoint_even(ctx.store, T, adj, tmp, ctx.mask, dtheta)
        else:
            seg = torch.empty(((min(S, max(T, 1)) + 1) // 2, b.total), dtype=torch.float32,
                              device=adj.device)
            for k in range(ctx.nseg - 1, -1, -1):
                L = min(S, T - k * S)
                b.write_state(ctx.store[k])
                b.step_record_even(L, seg)
                b.adjoint_even(seg, L, adj, tmp, ctx.mask, dtheta)
        gxs = [init_backward(b.view(adj, i), ctx.ka) for i in range(len(b))]
        b.close()
        ctx.b = None
        ctx.store = None
        return (dtheta.to(device=dd, dtype=dt), None, None, None, None, None, *gxs)


def simulate_batch(xs, theta, T, bc="zeroflux", ka=1.0, S=0, grads=None):
    """Differentiable T-step run of a batch of grids (any sizes) in one go;
    returns [(u_T, v_T) for each x].  theta: [8] shared or [n, 8] per instance;
    grads: parameter names whose gradients are formed (default all)."""
    out = RDCNNBatchFunction.apply(theta, int(T), bc, float(ka), int(S), grad_mask(grads), *xs)
    return [(out[2 * i], out[2 * i + 1]) for i in range(len(xs))]
