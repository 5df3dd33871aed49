"""Python face of a batch of RD-CNN grids (many sizes and parameter sets
advanced together; the paper's parameter-space exploration, Sec. III).

Argument marshalling only: the library packs nothing on the host side beyond
computing aligned offsets; every step runs in the batched HIP kernel.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import BC, Params, check, lib

ALIGN = 64  # floats (256 bytes)


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def packed_layout(shapes):
    """Float offsets of each instance's [2, R, C] state in a packed buffer
    (256-byte aligned) and the buffer's length."""
    offs, pos = [], 0
    for (R, C) in shapes:
        offs.append(pos)
        pos += -(-2 * R * C // ALIGN) * ALIGN
    return offs, pos


class Batch:
    """Instances given by initial images ``xs`` (2-D float32 CUDA tensors, any
    sizes) and one gene per instance; shared boundary rule and k_a.  The states
    live in two packed [total] float32 buffers; ``state(i)`` views instance i."""

    def __init__(self, xs, genes, bc: str = "zeroflux", ka: float = 1.0, tuned: bool = True):
        """tuned: take the pass shape the autotuner cached for this exact mix of
        sizes (tune.py, tuned.json), if there is one; else the library's."""
        if len(xs) != len(genes) or not xs:
            raise ValueError("need one gene per instance and at least one instance")
        self.device = xs[0].device
        self.bc = bc
        self.shapes = [(int(x.shape[0]), int(x.shape[1])) for x in xs]
        n = len(xs)
        offs, pos = packed_layout(self.shapes)
        xoffs, xpos = [], 0
        for (R, C) in self.shapes:
            xoffs.append(xpos)
            xpos += R * C
        self.offsets = offs
        self.total = pos
        self._x = torch.cat([x.contiguous().reshape(-1) for x in xs]).to(torch.float32)
        self.buf = [torch.empty(self.total, dtype=torch.float32, device=self.device) for _ in range(2)]
        rows = (ctypes.c_int * n)(*[s[0] for s in self.shapes])
        cols = (ctypes.c_int * n)(*[s[1] for s in self.shapes])
        coff = (ctypes.c_longlong * n)(*offs)
        cxoff = (ctypes.c_longlong * n)(*xoffs)
        pars = (Params * n)(*[Params.from_mapping(g) for g in genes])
        self._h = ctypes.c_void_p()
        self._shared = False
        with torch.cuda.device(self.device):
            check(lib.rdcnn_batch_create(ctypes.byref(self._h), n, rows, cols, coff, pars, BC[bc],
                                         self._x.data_ptr(), cxoff, float(ka),
                                         self.buf[0].data_ptr(), self.buf[1].data_ptr(),
                                         self.total, _stream_handle(self.device)))
        self.tuned_from = None  # tuned.json key of the applied pass shape, if any
        if tuned:
            from . import tune
            self.tuned_from = tune.apply(self)

    def __len__(self):
        return len(self.shapes)

    def step(self, T: int) -> "Batch":
        check(lib.rdcnn_batch_step(self._h, int(T)))
        return self

    def set_kernel(self, depth: int = 0, cols_per_lane: int = 0, seg_rows: int = 0) -> None:
        check(lib.rdcnn_batch_set_kernel(self._h, int(depth), int(cols_per_lane), int(seg_rows)))

    def set_class_seg_rows(self, rows: int, cols: int, seg_rows: int) -> None:
        """Rows per tile for every instance of size rows x cols (0: the batch-wide value)."""
        check(lib.rdcnn_batch_set_class_seg_rows(self._h, int(rows), int(cols), int(seg_rows)))

    def use_lds(self, on: bool = True) -> None:
        """Run instances that fit one workgroup's LDS whole, all steps in one launch."""
        check(lib.rdcnn_batch_use_lds(self._h, 1 if on else 0))

    def lds_instances(self) -> int:
        """How many instances the in-LDS kernel runs."""
        n = ctypes.c_int()
        check(lib.rdcnn_batch_lds_instances(self._h, ctypes.byref(n)))
        return n.value

    def use_graph(self, on: bool = True) -> None:
        check(lib.rdcnn_batch_use_graph(self._h, 1 if on else 0))

    def current(self) -> torch.Tensor:
        p = ctypes.c_void_p()
        check(lib.rdcnn_batch_current(self._h, ctypes.byref(p)))
        for b in self.buf:
            if b.data_ptr() == p.value:
                return b
        raise RuntimeError("current buffer not found")

    def write_state(self, packed: torch.Tensor) -> None:
        """Replace the current packed state (float32 [total] on the device)."""
        if packed.dtype != torch.float32 or packed.numel() < self.total or not packed.is_contiguous():
            raise ValueError("packed state must be contiguous float32 of the batch's size")
        self._keep = packed
        check(lib.rdcnn_batch_write_state(self._h, packed.data_ptr()))

    def _check_traj(self, traj, n):
        if (traj.dtype != torch.float32 or not traj.is_contiguous() or traj.dim() != 2
                or traj.shape[0] < n or traj.shape[1] != self.total):
            raise ValueError("traj must be contiguous float32 [>= %d, total]" % n)

    def step_record(self, T: int, traj: torch.Tensor) -> "Batch":
        """Advance T steps, writing the packed state each step starts from into
        traj[q] (float32 [>= T, total], contiguous)."""
        if T > 0:
            self._check_traj(traj, T)
        check(lib.rdcnn_batch_step_record(self._h, int(T), traj.data_ptr() if T > 0 else None))
        return self

    def step_record_even(self, T: int, traj: torch.Tensor) -> "Batch":
        """Advance T steps keeping the packed states of even times: state 2i in
        traj[i] (float32 [>= (T+1)//2, total]); what adjoint_even reads."""
        if T > 0:
            self._check_traj(traj, (T + 1) // 2)
        check(lib.rdcnn_batch_step_record_even(self._h, int(T), traj.data_ptr() if T > 0 else None))
        return self

    def set_adjoint_kernel(self, depth: int = 0, cols_per_lane: int = 0, seg_rows: int = 0) -> None:
        check(lib.rdcnn_batch_set_adjoint_kernel(self._h, int(depth), int(cols_per_lane),
                                                 int(seg_rows)))

    def adjoint(self, traj: torch.Tensor, S: int, adj: torch.Tensor, adj_tmp: torch.Tensor,
                mask: int, dtheta: torch.Tensor) -> None:
        """Reverse pass through the S steps recorded in traj[0..S-1] for every
        instance: adj (packed) goes from dJ/ds after to dJ/ds before; per-instance
        parameter gradients are added to dtheta (float64 [n, 8])."""
        self._check_adjoint(adj, adj_tmp, dtheta)
        if S > 0:
            self._check_traj(traj, S)
        check(lib.rdcnn_batch_adjoint(self._h, traj.data_ptr() if S > 0 else None, int(S),
                                      adj.data_ptr(), adj_tmp.data_ptr(), int(mask) & 0xFF,
                                      dtheta.data_ptr()))

    def adjoint_even(self, traj: torch.Tensor, S: int, adj: torch.Tensor, adj_tmp: torch.Tensor,
                     mask: int, dtheta: torch.Tensor) -> None:
        """adjoint() from an even-time trajectory (step_record_even); the odd
        states are rebuilt inside the reverse passes, with the same results."""
        self._check_adjoint(adj, adj_tmp, dtheta)
        if S > 0:
            self._check_traj(traj, (S + 1) // 2)
        check(lib.rdcnn_batch_adjoint_even(self._h, traj.data_ptr() if S > 0 else None, int(S),
                                           adj.data_ptr(), adj_tmp.data_ptr(), int(mask) & 0xFF,
                                           dtheta.data_ptr()))

    def _check_adjoint(self, adj, adj_tmp, dtheta):
        for t in (adj, adj_tmp):
            if t.dtype != torch.float32 or t.numel() < self.total or not t.is_contiguous():
                raise ValueError("adj buffers must be contiguous float32 of the batch's size")
        want = (8,) if self._shared else (len(self), 8)
        if dtheta.dtype != torch.float64 or tuple(dtheta.shape) != want or not dtheta.is_contiguous():
            raise ValueError(f"dtheta must be contiguous float64 {list(want)}")

    def set_shared_grad(self, on: bool = True) -> None:
        """The instances share one parameter vector: adjoint() then adds the
        gradient summed over instances (on the device, in instance order) to a
        float64 [8] dtheta instead of one row per instance."""
        check(lib.rdcnn_batch_set_shared_grad(self._h, 1 if on else 0))
        self._shared = bool(on)

    def set_check_finite(self, on: bool = True) -> None:
        """read_into() checks every instance for NaN / Inf (RDCNN_ENONFINITE)."""
        check(lib.rdcnn_batch_set_check_finite(self._h, 1 if on else 0))

    def read_into(self, dst: torch.Tensor) -> None:
        """Copy the current packed state into dst (float32 [>= total] on the
        device; rdcnn_batch_read)."""
        if dst.dtype != torch.float32 or dst.numel() < self.total or not dst.is_contiguous() \
                or dst.device != self.device:
            raise ValueError("dst must be contiguous float32 of the batch's size on its device")
        check(lib.rdcnn_batch_read(self._h, dst.data_ptr()))

    def view(self, packed: torch.Tensor, i: int) -> torch.Tensor:
        """View [2, R, C] of instance i in a packed tensor of this batch's layout."""
        R, C = self.shapes[i]
        o = self.offsets[i]
        return packed[o:o + 2 * R * C].view(2, R, C)

    def snapshot(self) -> torch.Tensor:
        """A copy of the current packed state (for the change statistics)."""
        out = torch.empty(self.total, dtype=torch.float32, device=self.device)
        self.read_into(out)
        return out

    STAT_NAMES = ("mean_u", "var_u", "mean_v", "var_v", "frac_far", "frac_moving",
                  "max_change", "rms_change")

    def stats(self, prev: torch.Tensor = None, ref=None, theta_far: float = 0.0,
              theta_move: float = 0.0) -> torch.Tensor:
        """Per-instance statistics of the current state, [n, 8] float64 on the
        device (columns STAT_NAMES; rdcnn_batch_stats).  prev: an earlier
        snapshot(); ref: per-instance reference value of u (sequence or tensor)."""
        out = torch.empty((len(self), 8), dtype=torch.float64, device=self.device)
        if prev is not None and (prev.dtype != torch.float32 or prev.numel() < self.total
                                 or prev.device != self.device):
            raise ValueError("prev must be a float32 snapshot() of this batch")
        r = None
        if ref is not None:
            r = torch.as_tensor(ref, dtype=torch.float32, device=self.device).reshape(-1).contiguous()
            if r.numel() != len(self):
                raise ValueError("ref needs one value per instance")
        check(lib.rdcnn_batch_stats(self._h, None if prev is None else prev.data_ptr(),
                                    None if r is None else r.data_ptr(), float(theta_far),
                                    float(theta_move), out.data_ptr()))
        return out

    def state(self, i: int) -> torch.Tensor:
        """View [2, R, C] (u, v) of instance i in the current buffer."""
        R, C = self.shapes[i]
        o = self.offsets[i]
        return self.current()[o:o + 2 * R * C].view(2, R, C)

    def close(self) -> None:
        if self._h:
            lib.rdcnn_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
