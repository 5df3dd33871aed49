"""Oracle for the per-instance statistics of a parameter atlas (Sec. III.A).

TEST INFRASTRUCTURE ONLY (see the package docstring): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.

Sec. III.A scans the diffusion coefficients (Du, Dv) and sorts the outcomes by
eye into slow growth, dynamic patterns and a homogeneous steady state (Fig. 9).
The statistics below are what an automated version of that map measures on
each instance's state.  They are plain definitions, written out in numpy.  Sums
are taken in float64 over the float32 state.  Each threshold test is decided in
float32, the precision of the state, so the counts are exact.

For an instance with N cells, state (u, v), an earlier state u_prev (or None),
a reference value ref and thresholds theta_far and theta_move:

  0  mean_u      = sum(u) / N
  1  var_u       = sum((u - mean_u)^2) / N
  2  mean_v      = sum(v) / N
  3  var_v       = sum((v - mean_v)^2) / N
  4  frac_far    = #{ |u - ref| > theta_far } / N          (float32 test)
  5  frac_moving = #{ |u - u_prev| > theta_move } / N      (float32 test)
  6  max_change  = max |u - u_prev|                        (float32 difference)
  7  rms_change  = sqrt( sum((u - u_prev)^2) / N )          (float32 difference)

Entries 5-7 are NaN when u_prev is None.
"""
from __future__ import annotations

import numpy as np

NSTATS = 8
STAT_NAMES = ("mean_u", "var_u", "mean_v", "var_v", "frac_far", "frac_moving",
              "max_change", "rms_change")


def instance_stats(u, v, u_prev=None, ref=0.0, theta_far=0.0, theta_move=0.0) -> np.ndarray:
    u = np.asarray(u, dtype=np.float32)
    v = np.asarray(v, dtype=np.float32)
    n = u.size
    u64 = u.astype(np.float64)
    v64 = v.astype(np.float64)
    out = np.full(NSTATS, np.nan)
    out[0] = u64.sum() / n
    out[1] = ((u64 - out[0]) ** 2).sum() / n
    out[2] = v64.sum() / n
    out[3] = ((v64 - out[2]) ** 2).sum() / n
    far = np.abs(u - np.float32(ref)) > np.float32(theta_far)
    out[4] = np.count_nonzero(far) / n
    if u_prev is not None:
        d = u - np.asarray(u_prev, dtype=np.float32)  # float32 difference
        ad = np.abs(d)
        out[5] = np.count_nonzero(ad > np.float32(theta_move)) / n
        out[6] = float(ad.max())
        out[7] = np.sqrt((d.astype(np.float64) ** 2).sum() / n)
    return out
