"""Python face of one RD-CNN grid on the GPU (arXiv 2102.10340, Sec. II).

PyTorch only provides the device memory and the stream; the library's kernels
do every step of Eq. (1)-(3).  Mirrors the paper's workflow: an initial state
built from an image x and the gene (get_init_state), T iterations of the cell
kernel, and snapshots of the A (u) and B (v) arrays.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import BC, PARAM_FIELDS, Params, check, lib


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Simulation:
    """One rows x cols grid.  ``x`` is a float32 CUDA tensor (the initial image),
    ``gene`` a mapping with keys dt, a, b, eps, c, k3, Du, Dv, ``bc`` one of
    "periodic" / "zeroflux".  The state lives in two caller-owned [2, R, C]
    buffers (u plane, v plane) that ping-pong between steps."""

    def __init__(self, x: torch.Tensor, gene, bc: str = "zeroflux", ka: float = 1.0,
                 tuned: bool = True):
        """tuned: take the forward pass shape the autotuner cached for this grid
        size and boundary rule (tune.py, tuned.json), if there is one; else the
        library's automatic one.  The recording calls keep their own automatic
        shapes (rdcnn_set_kernel kind 3)."""
        if x.dim() != 2 or x.dtype != torch.float32 or not x.is_cuda:
            raise ValueError("x must be a 2-D float32 CUDA tensor")
        self.device = x.device
        self.rows, self.cols = int(x.shape[0]), int(x.shape[1])
        self.bc = bc
        self._x = x.contiguous()
        self.buf = [torch.empty((2, self.rows, self.cols), dtype=torch.float32, device=self.device)
                    for _ in range(2)]
        self._h = ctypes.c_void_p()
        self._params = Params.from_mapping(gene)
        self._kernel = (0, 0, 0, 0)
        with torch.cuda.device(self.device):
            check(lib.rdcnn_create(ctypes.byref(self._h), self.rows, self.cols, BC[bc],
                                   ctypes.byref(self._params), self._x.data_ptr(), float(ka),
                                   self.buf[0].data_ptr(), self.buf[1].data_ptr(),
                                   _stream_handle(self.device)))
        self.tuned_from = None  # tuned.json key of the applied pass shape, if any
        if tuned:
            from . import tune
            self.tuned_from = tune.apply(self, modes=("forward",))

    MODELS = {"fitzhugh_nagumo": 0, "gray_scott": 1, "cnn": 2}

    @classmethod
    def model(cls, name: str, u0: torch.Tensor, v0: torch.Tensor, params, bc: str = "zeroflux"):
        """A grid of a built-in cell model (rdcnn_model_create): name is one of
        MODELS, params the model's float vector, (u0, v0) its two starting
        layers (for "cnn": the state x0 and the input image)."""
        if u0.dim() != 2 or u0.shape != v0.shape or u0.dtype != torch.float32 or not u0.is_cuda:
            raise ValueError("u0, v0 must be 2-D float32 CUDA tensors of one shape")
        sim = cls.__new__(cls)
        sim.device = u0.device
        sim.rows, sim.cols = int(u0.shape[0]), int(u0.shape[1])
        sim.bc = bc
        sim._x = (u0.contiguous(), v0.contiguous())
        sim.buf = [torch.empty((2, sim.rows, sim.cols), dtype=torch.float32, device=sim.device)
                   for _ in range(2)]
        sim._h = ctypes.c_void_p()
        sim._kernel = (0, 0, 0, 0)
        p = (ctypes.c_float * len(params))(*[float(x) for x in params])
        with torch.cuda.device(sim.device):
            check(lib.rdcnn_model_create(ctypes.byref(sim._h), cls.MODELS[name], sim.rows, sim.cols,
                                         BC[bc], p, len(params), sim._x[0].data_ptr(),
                                         sim._x[1].data_ptr(), sim.buf[0].data_ptr(),
                                         sim.buf[1].data_ptr(), _stream_handle(sim.device)))
        return sim

    @classmethod
    def gray_scott(cls, u0, v0, dt, F, k, Du, Dv, bc: str = "periodic"):
        """Gray-Scott reaction-diffusion on the streamed kernel."""
        return cls.model("gray_scott", u0, v0, [dt, F, k, Du, Dv], bc)

    @classmethod
    def cnn(cls, x0, image, A, B, z, dt, bc: str = "zeroflux"):
        """Chua-Yang cellular neural network with 3x3 templates A, B and bias z."""
        a = [float(v) for v in torch.as_tensor(A, dtype=torch.float64).reshape(9)]
        b = [float(v) for v in torch.as_tensor(B, dtype=torch.float64).reshape(9)]
        return cls.model("cnn", x0, image, [dt] + a + b + [float(z)], bc)

    @classmethod
    def from_state(cls, u0: torch.Tensor, v0: torch.Tensor, gene, bc: str = "zeroflux",
                   tuned: bool = True):
        """A grid whose state starts at (u0, v0) instead of k_a x."""
        sim = cls(u0, gene, bc, 1.0, tuned)
        sim.write_state(u0, v0)
        return sim

    # -- control ---------------------------------------------------------
    def step(self, T: int) -> "Simulation":
        """Advance by T steps (asynchronous on the current stream)."""
        check(lib.rdcnn_step(self._h, int(T)))
        return self

    def use_graph(self, on: bool = True) -> "Simulation":
        """rdcnn_use_graph: step() replays a captured HIP graph of its launches
        (per T and starting buffer).  Needs a non-default current stream."""
        check(lib.rdcnn_use_graph(self._h, 1 if on else 0))
        return self

    def step_record(self, T: int, states: torch.Tensor) -> "Simulation":
        """Advance by T steps and write the state each step starts from into
        states[0..T-1] (a float32 CUDA tensor of shape [>= T, 2, R, C])."""
        if T > 0:
            self._check_states(states, T)
        check(lib.rdcnn_step_record(self._h, int(T), states.data_ptr() if T > 0 else None))
        return self

    def step_record_even(self, T: int, states: torch.Tensor) -> "Simulation":
        """Advance by T steps keeping only the even-time states: s_{2i} goes to
        states[i] for 2i < T (shape [>= (T+1)//2, 2, R, C]); the trajectory
        adjoint_even reads."""
        if T > 0:
            self._check_states(states, (T + 1) // 2)
        check(lib.rdcnn_step_record_even(self._h, int(T), states.data_ptr() if T > 0 else None))
        return self

    def step_record_sparse(self, T: int, states: torch.Tensor) -> "Simulation":
        """Advance by T steps writing the even-time states into their own slots
        of a trajectory with one slot per time: s_{2i} to states[2i] (shape
        [>= T+1, 2, R, C]); the layout step_bwd reads."""
        if T > 0:
            self._check_states(states, T + 1)
        check(lib.rdcnn_step_record_sparse(self._h, int(T), states.data_ptr() if T > 0 else None))
        return self

    def step_checkpoints(self, T: int, S: int, ckpt: torch.Tensor) -> "Simulation":
        """Advance by T steps keeping s_{jS} in ckpt[j] for jS < T (shape
        [>= ceil(T/S), 2, R, C]); each checkpoint is written by the pass that
        ends there."""
        if T > 0:
            self._check_states(ckpt, -(-int(T) // int(S)))
        check(lib.rdcnn_step_checkpoints(self._h, int(T), int(S), ckpt.data_ptr() if T > 0 else None))
        return self

    def step_bwd(self, states: torch.Tensor, S: int, lam: torch.Tensor, mu: torch.Tensor,
                 dtheta: torch.Tensor) -> None:
        """rdcnn_step_bwd: reverse pass through the S steps whose start states
        sit in states[q] (the even q are read; states[S] is workspace).  lam, mu
        ([R, C] each) go from dJ/d(u, v) after the steps to before them; dJ/dp
        (float64 [8]) is added to dtheta."""
        if S > 0:
            self._check_states(states, S + 1)
        for t in (lam, mu):
            if t.shape != (self.rows, self.cols) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("lam and mu must be contiguous float32 [R, C]")
        if dtheta.dtype != torch.float64 or dtheta.numel() != 8 or not dtheta.is_cuda:
            raise ValueError("dtheta must be a CUDA float64 tensor of 8 elements")
        check(lib.rdcnn_step_bwd(self._h, states.data_ptr() if S > 0 else None, int(S),
                                 lam.data_ptr(), mu.data_ptr(), dtheta.data_ptr()))

    def step_bwd_ckpt(self, ckpt: torch.Tensor, T: int, S: int, work: torch.Tensor,
                      lam: torch.Tensor, mu: torch.Tensor, dtheta: torch.Tensor) -> None:
        """rdcnn_step_bwd_ckpt: the backward of checkpoint-and-recompute through
        T steps whose checkpoints (one every S steps) sit in ckpt; each segment
        is recomputed on the library's second stream while the reverse pass of
        the next runs.  work: [>= 2 (min(S, T) + 1), 2, R, C] scratch.  lam, mu
        ([R, C]) go from dJ/d(u, v) after the T steps to before them; dJ/dp
        (float64 [8]) is added to dtheta."""
        if T > 0:
            self._check_states(ckpt, -(-int(T) // int(S)))
            self._check_states(work, 2 * (min(int(S), int(T)) + 1))
        for t in (lam, mu):
            if t.shape != (self.rows, self.cols) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("lam and mu must be contiguous float32 [R, C]")
        if dtheta.dtype != torch.float64 or dtheta.numel() != 8 or not dtheta.is_cuda:
            raise ValueError("dtheta must be a CUDA float64 tensor of 8 elements")
        check(lib.rdcnn_step_bwd_ckpt(self._h, ckpt.data_ptr() if T > 0 else None, int(T), int(S),
                                      work.data_ptr() if T > 0 else None, lam.data_ptr(),
                                      mu.data_ptr(), dtheta.data_ptr()))

    def set_check_finite(self, on: bool = True) -> None:
        """Reads check the state for NaN / Inf and raise (RDCNN_ENONFINITE)."""
        check(lib.rdcnn_set_check_finite(self._h, 1 if on else 0))

    def adjoint(self, states: torch.Tensor, S: int, adj: torch.Tensor, adj_tmp: torch.Tensor,
                dtheta: torch.Tensor) -> None:
        """Reverse pass through S steps recorded in states[0..S-1]: adj [2, R, C]
        goes from dJ/ds after the steps to dJ/ds before them; dJ/dp (float64 [8],
        order dt, a, b, eps, c, k3, Du, Dv) is added to dtheta."""
        if S > 0:
            self._check_states(states, S)
        self._check_adjoint(adj, adj_tmp, dtheta)
        check(lib.rdcnn_adjoint(self._h, states.data_ptr() if S > 0 else None, int(S),
                                adj.data_ptr(), adj_tmp.data_ptr(), dtheta.data_ptr()))

    def adjoint_even(self, states: torch.Tensor, S: int, adj: torch.Tensor, adj_tmp: torch.Tensor,
                     dtheta: torch.Tensor) -> None:
        """adjoint() from an even-time trajectory (step_record_even): the odd
        states are rebuilt inside the reverse passes; same results."""
        if S > 0:
            self._check_states(states, (S + 1) // 2)
        self._check_adjoint(adj, adj_tmp, dtheta)
        check(lib.rdcnn_adjoint_even(self._h, states.data_ptr() if S > 0 else None, int(S),
                                     adj.data_ptr(), adj_tmp.data_ptr(), dtheta.data_ptr()))

    def _check_adjoint(self, adj, adj_tmp, dtheta):
        for t in (adj, adj_tmp):
            if t.shape != (2, self.rows, self.cols) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("adjoint buffers must be contiguous float32 [2, R, C]")
        if dtheta.dtype != torch.float64 or dtheta.numel() != 8 or not dtheta.is_cuda:
            raise ValueError("dtheta must be a CUDA float64 tensor of 8 elements")

    def set_grad_mask(self, mask: int) -> None:
        """Parameter gradients the adjoint forms (bit q = parameter q in the order
        dt, a, b, eps, c, k3, Du, Dv); the others come back NaN."""
        check(lib.rdcnn_set_grad_mask(self._h, int(mask)))

    def set_adjoint_kernel(self, depth: int = 0, cols_per_lane: int = 0, seg_rows: int = 0) -> None:
        check(lib.rdcnn_set_adjoint_kernel(self._h, int(depth), int(cols_per_lane), int(seg_rows)))

    def _check_states(self, states, n):
        if (states.dtype != torch.float32 or not states.is_contiguous() or states.dim() != 4
                or states.shape[0] < n or tuple(states.shape[1:]) != (2, self.rows, self.cols)):
            raise ValueError("states must be contiguous float32 [>= n, 2, R, C]")

    @property
    def gene(self) -> dict:
        """The current parameters (dt, a, b, eps, c, k3, Du, Dv) as floats."""
        return {k: float(getattr(self._params, k)) for k in PARAM_FIELDS}

    def kernel_setting(self):
        """The arguments of the last set_kernel call ((0, 0, 0, 0): automatic)."""
        return self._kernel

    def set_params(self, gene) -> None:
        self._params = Params.from_mapping(gene)
        check(lib.rdcnn_set_params(self._h, ctypes.byref(self._params)))

    def set_kernel(self, kind: int = 0, depth: int = 0, cols_per_lane: int = 0,
                   seg_rows: int = 0) -> None:
        """0 automatic, 1 one-thread-per-cell reference kernel, 2 streamed kernel
        with `depth` steps per pass, 3 the same for plain steps only (the
        recording calls keep their automatic shapes); bit-identical results
        for every choice."""
        check(lib.rdcnn_set_kernel(self._h, int(kind), int(depth), int(cols_per_lane),
                                   int(seg_rows)))
        self._kernel = (int(kind), int(depth), int(cols_per_lane), int(seg_rows))

    def pass_config(self) -> dict:
        """The pass shape rdcnn_step uses now (automatic choices resolved)."""
        v = [ctypes.c_int() for _ in range(4)]
        check(lib.rdcnn_pass_config(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("kind", "depth", "cols_per_lane", "seg_rows"), [x.value for x in v]))

    # -- state -----------------------------------------------------------
    def state(self) -> torch.Tensor:
        """View [2, R, C] of the buffer holding the current state (no copy)."""
        p = ctypes.c_void_p()
        check(lib.rdcnn_current(self._h, ctypes.byref(p)))
        for b in self.buf:
            if b.data_ptr() == p.value:
                return b
        raise RuntimeError("current state buffer not found")

    def read(self):
        """Device copies (u, v) of the current state (the paper's snapshot)."""
        u = torch.empty((self.rows, self.cols), dtype=torch.float32, device=self.device)
        v = torch.empty_like(u)
        check(lib.rdcnn_read(self._h, u.data_ptr(), v.data_ptr(), 0))
        return u, v

    def read_into(self, u_dst: torch.Tensor, v_dst: torch.Tensor) -> None:
        """Copy the current state into caller-owned device tensors (asynchronous)."""
        for t in (u_dst, v_dst):
            if t.shape != (self.rows, self.cols) or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError("destination must be contiguous float32 [R, C]")
        check(lib.rdcnn_read(self._h, u_dst.data_ptr(), v_dst.data_ptr(), 0))

    def read_host(self):
        """Host numpy copies (u, v); waits for the stream."""
        u = torch.empty((self.rows, self.cols), dtype=torch.float32, pin_memory=True)
        v = torch.empty_like(u, pin_memory=True)
        check(lib.rdcnn_read(self._h, u.data_ptr(), v.data_ptr(), 1))
        return u.numpy().copy(), v.numpy().copy()

    def write_state(self, u: torch.Tensor, v: torch.Tensor) -> None:
        u = u.contiguous()
        v = v.contiguous()
        if u.shape != (self.rows, self.cols) or v.shape != u.shape:
            raise ValueError("state shape mismatch")
        self._keep = (u, v)
        check(lib.rdcnn_write_state(self._h, u.data_ptr(), v.data_ptr()))

    def write_state_packed(self, s: torch.Tensor) -> None:
        """Replace the current state with s, a [2, R, C] tensor (u, v)."""
        self.write_state(s[0], s[1])

    def close(self) -> None:
        if self._h:
            lib.rdcnn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_backward(adj: torch.Tensor, ka: float, out: torch.Tensor = None) -> torch.Tensor:
    """Chain rule through u = v = ka x: returns ka (adj[0] + adj[1])."""
    adj = adj.contiguous()
    if out is None:
        out = torch.empty(adj.shape[1:], dtype=torch.float32, device=adj.device)
    check(lib.rdcnn_init_backward(adj.data_ptr(), adj[0].numel(), float(ka), out.data_ptr(),
                                  _stream_handle(adj.device)))
    return out
