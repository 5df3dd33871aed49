"""Differentiable RD-CNN runs: torch.autograd.Function wrappers around the
library's forward, state-recording and adjoint kernels.

Both schedules keep only the states of even times (rdcnn_step_record_even,
4 bytes per cell and step); the paired reverse passes (rdcnn_adjoint_even)
rebuild each odd state from the even one before it with the forward cell
update, bit-identical to the forward pass, so the gradients equal those of a
fully recorded trajectory.  The schedule is chosen by S:
* S = -1, whole trajectory: the forward records the even states and the
  backward runs the adjoint straight through them.  An MI355X has 288 GB of
  HBM, so this is the default whenever the trajectory fits a quarter of the
  free device memory (8 GiB for 1024x1024 x 2000 steps).
* S > 0, checkpoint-and-recompute: the forward keeps one checkpoint every S
  steps; the backward walks the segments from last to first, restores a
  checkpoint, re-runs the segment while recording its even states and runs the
  adjoint through them.  With S near sqrt(T) memory is O(sqrt(T)) states; the
  default S is ceil(sqrt(T)) capped so that one segment's states stay within
  half of the 256 MB last-level cache, where the adjoint reads them right after
  they are written.
S = 0 picks the whole trajectory if it fits, else the checkpointed schedule.

Parameters travel as a tensor theta of 8 values in the order
(dt, a, b, eps, c, k3, Du, Dv), the paper's gene (Sec. II.A) plus the cubic
coefficient; its gradient is float64 from the library, cast to theta's dtype.
"""
from __future__ import annotations

import math

import torch

from ._lib import PARAM_FIELDS
from .sim import Simulation, init_backward

LLC_BYTES = 256 << 20


def default_segment(T: int, rows: int, cols: int) -> int:
    """ceil(sqrt(T)), capped so that a segment's even states fit half the last-level cache."""
    s = max(1, math.ceil(math.sqrt(max(T, 1))))
    cap = max(1, 2 * ((LLC_BYTES // 2) // (8 * rows * cols)))
    return max(1, min(s, cap, T if T > 0 else 1))


def choose_schedule(T: int, rows: int, cols: int, S: int, device) -> int:
    """-1 (record the whole trajectory) or a checkpoint spacing > 0."""
    if S != 0:
        return S
    need = 8 * rows * cols * max((T + 1) // 2, 1)
    free, _ = torch.cuda.mem_get_info(device)
    if need <= free // 4:
        return -1
    return default_segment(T, rows, cols)


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


def _forward(sim: Simulation, T: int, S: int, dev):
    if S < 0:  # whole trajectory, even times
        states = torch.empty((max((T + 1) // 2, 1), 2, sim.rows, sim.cols), dtype=torch.float32,
                             device=dev)
        sim.step_record_even(T, states)
        u, v = sim.read()
        return u, v, states, 0
    nseg = -(-T // S) if T > 0 else 0
    ckpt = torch.empty((max(nseg, 1), 2, sim.rows, sim.cols), dtype=torch.float32, device=dev)
    for k in range(nseg):
        sim.read_into(ckpt[k, 0], ckpt[k, 1])
        sim.step(min(S, T - k * S))
    u, v = sim.read()
    return u, v, ckpt, nseg


def _backward(sim: Simulation, ckpt, nseg: int, T: int, S: int, gu, gv, dev, kernel=None,
              mask: int = 0xFF):
    R, C = sim.rows, sim.cols
    adj = torch.empty((2, R, C), dtype=torch.float32, device=dev)
    for k, gk in enumerate((gu, gv)):
        if gk is None:
            adj[k].zero_()
        else:
            adj[k].copy_(gk)
    tmp = torch.empty_like(adj)
    dtheta = torch.zeros(8, dtype=torch.float64, device=dev)
    if kernel is not None:
        sim.set_adjoint_kernel(*kernel)
    sim.set_grad_mask(mask)
    if S < 0:  # ckpt holds the whole even-time trajectory
        sim.adjoint_even(ckpt, T, adj, tmp, dtheta)
        return adj, dtheta
    seg = torch.empty(((min(S, max(T, 1)) + 1) // 2, 2, R, C), dtype=torch.float32, device=dev)
    for k in range(nseg - 1, -1, -1):
        L = min(S, T - k * S)
        sim.write_state_packed(ckpt[k])
        sim.step_record_even(L, seg)
        sim.adjoint_even(seg, L, adj, tmp, dtheta)
    return adj, dtheta


class RDCNNFunction(torch.autograd.Function):
    """(x, theta) -> (u_T, v_T) with u_0 = v_0 = ka x (Eq. (1)) and T steps."""

    @staticmethod
    def forward(ctx, x, theta, T: int, bc: str = "zeroflux", ka: float = 1.0, S: int = 0,
                adj_kernel=None, mask: int = 0xFF):
        x = x.detach().contiguous()
        T = int(T)
        S = choose_schedule(T, x.shape[0], x.shape[1], int(S), x.device)
        sim = Simulation(x, _gene(theta), bc, ka)
        u, v, ckpt, nseg = _forward(sim, T, S, x.device)
        ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, ctx.ka = sim, ckpt, nseg, T, S, ka
        ctx.adj_kernel, ctx.mask = adj_kernel, mask
        ctx.theta_meta = (theta.dtype, theta.device)
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        dev = ctx.ckpt.device
        adj, dtheta = _backward(ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, gu, gv, dev,
                                ctx.adj_kernel, ctx.mask)
        gx = init_backward(adj, ctx.ka)
        ctx.sim.close()
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
        sim = Simulation.from_state(u0, v0, _gene(theta), bc)
        u, v, ckpt, nseg = _forward(sim, T, S, u0.device)
        ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S = sim, ckpt, nseg, T, S
        ctx.adj_kernel, ctx.mask = adj_kernel, mask
        ctx.theta_meta = (theta.dtype, theta.device)
        return u, v

    @staticmethod
    def backward(ctx, gu, gv):
        dev = ctx.ckpt.device
        adj, dtheta = _backward(ctx.sim, ctx.ckpt, ctx.nseg, ctx.T, ctx.S, gu, gv, dev,
                                ctx.adj_kernel, ctx.mask)
        ctx.sim.close()
        dt, dd = ctx.theta_meta
        return (adj[0].clone(), adj[1].clone(), dtheta.to(device=dd, dtype=dt), None, None, None,
                None, None)


def simulate(x, theta, T, bc="zeroflux", ka=1.0, S=0, grads=None):
    """Differentiable T-step run from u = v = ka x; returns (u_T, v_T).
    grads: parameter names whose gradients are formed (default all); the
    others come back NaN in theta.grad."""
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
        b = Batch(xs, genes, bc, ka)
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
                store[k].copy_(b.current())
                b.step(min(S, T - k * S))
        outs = []
        for i in range(n):
            st = b.state(i)
            outs += [st[0].clone(), st[1].clone()]
        ctx.b, ctx.store, ctx.nseg, ctx.T, ctx.S, ctx.ka, ctx.mask = b, store, nseg, T, S, ka, mask
        ctx.theta_meta = (theta.dtype, theta.device, theta.dim())
        return tuple(outs)

    @staticmethod
    def backward(ctx, *gouts):
        b, T, S = ctx.b, ctx.T, ctx.S
        adj = torch.zeros(b.total, dtype=torch.float32, device=b.device)
        for i in range(len(b)):
            a = b.view(adj, i)
            for layer in range(2):
                gg = gouts[2 * i + layer]
                if gg is not None:
                    a[layer].copy_(gg)
        tmp = torch.empty_like(adj)
        dtheta = torch.zeros((len(b), 8), dtype=torch.float64, device=adj.device)
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
        dt, dd, dim = ctx.theta_meta
        g = dtheta.cpu()
        if dim == 1:  # shared parameters: sum over instances in a fixed order
            g = g.sum(0)
        return (g.to(device=dd, dtype=dt), None, None, None, None, None, *gxs)


def simulate_batch(xs, theta, T, bc="zeroflux", ka=1.0, S=0, grads=None):
    """Differentiable T-step run of a batch of grids (any sizes) in one go;
    returns [(u_T, v_T) for each x].  theta: [8] shared or [n, 8] per instance;
    grads: parameter names whose gradients are formed (default all)."""
    out = RDCNNBatchFunction.apply(theta, int(T), bc, float(ka), int(S), grad_mask(grads), *xs)
    return [(out[2 * i], out[2 * i + 1]) for i in range(len(xs))]
