"""Automated parameter atlas (the (Du, Dv) scans of Sec. III.A, Fig. 9).

The paper runs the simulator over a grid of diffusion coefficients and sorts
the outcomes by eye into slow growth, dynamic patterns and a homogeneous steady
state.  Here every grid point is one instance of a Batch; after T steps the
library's per-instance statistics (rdcnn_batch_stats) are taken at two times,
T - dT and T, and each instance is given one class:

  homogeneous  spatial variance of u below var_tol (a uniform steady state)
  growing      the share of cells away from the rest state grew between the
               two times and is still below full (a front spreading from the
               initial patch: slow growth)
  dynamic      more than move_tol of the cells still change by more than
               theta_move over dT (patterns that keep moving)
  stationary   a pattern that no longer changes

The thresholds are this module's reading (the paper names the classes but gives
no numbers for them); the statistics are computed on the GPU, the classes on
the host.
"""
from __future__ import annotations

import numpy as np
import torch

from .batch import Batch

CLASSES = ("homogeneous", "growing", "dynamic", "stationary")


def rest_state(gene) -> tuple:
    """The uniform rest state (u*, v*) of Eq. (2)-(3): f1 = f2 = 0 with no
    diffusion, so v = (u + a) / b and c u - k3 u^3 - (u + a) / b = 0; of the
    cubic's real roots, the one closest to 0."""
    a, b, c, k3 = gene["a"], gene["b"], gene["c"], gene["k3"]
    if b == 0:
        raise ValueError("rest state needs b != 0")
    roots = np.roots([-k3, 0.0, c - 1.0 / b, -a / b])
    real = sorted((r.real for r in roots if abs(r.imag) < 1e-9), key=abs)
    u = float(real[0])
    return u, (u + a) / b


def classify(s_prev: np.ndarray, s_now: np.ndarray, var_tol: float = 1e-6,
             move_tol: float = 1e-3, full: float = 0.99) -> np.ndarray:
    """Class index per instance (CLASSES) from the statistics at T - dT (s_prev)
    and at T with the change since T - dT (s_now), both [n, 8] arrays."""
    var_u = s_now[:, 1]
    far_prev, far_now = s_prev[:, 4], s_now[:, 4]
    moving = s_now[:, 5]
    out = np.full(len(s_now), 3, dtype=np.int64)  # stationary
    dyn = moving > move_tol
    grow = (far_now > far_prev) & (far_now < full) & dyn
    out[dyn] = 2
    out[grow] = 1
    out[var_u < var_tol] = 0
    return out


def scan(du, dv, gene, x, T: int, dT: int, bc: str = "periodic", theta_far: float = 0.05,
         theta_move: float = 1e-3, stream=None):
    """Run the (Du, Dv) grid du x dv from the initial image x (2-D CUDA tensor)
    for T steps and classify every point.  Returns (classes [len(du), len(dv)],
    stats at T [len(du), len(dv), 8] as numpy)."""
    genes = [dict(gene, Du=float(a), Dv=float(b)) for a in du for b in dv]
    b = Batch([x] * len(genes), genes, bc)
    ref = torch.tensor([rest_state(g)[0] for g in genes], dtype=torch.float32, device=x.device)
    b.step(T - dT)
    prev = b.snapshot()
    s_prev = b.stats(None, ref, theta_far, theta_move)
    b.step(dT)
    s_now = b.stats(prev, ref, theta_far, theta_move)
    s_prev, s_now = s_prev.cpu().numpy(), s_now.cpu().numpy()
    b.close()
    cls = classify(s_prev, s_now)
    return cls.reshape(len(du), len(dv)), s_now.reshape(len(du), len(dv), 8)
