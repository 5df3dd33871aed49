"""CPU oracle for the FitzHugh-Nagumo RD-CNN step (arXiv 2102.10340, Sec. II.A).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, plain reference that the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does, and this module imports nothing from it.

The arithmetic lives in ``rdcnn_oracle.c`` (plain C loops, built by :func:`build`
with gcc); this module only marshals numpy arrays.  What is computed:

* :func:`init_state` -- Eq. (1), first line: ``u = v = k_a * x``.
* :func:`run` -- Eq. (1)-(3) iterated T times (Jacobi explicit Euler), in float32
  (the canonical rounding order that the GPU path reproduces) or float64.
* :func:`laplacian` -- the unscaled 5-point Laplacian of Eq. (1).
* :func:`grad` -- reverse pass of Eq. (1)-(3): dJ/ds_0 and dJ/dp for a loss
  J(s_T), by checkpoint-and-recompute.

Two further cell models on the same grid and boundary rules (``cell_models.c``,
after the extension to other finite-difference and cellular models that Sec. IV
names): :func:`gs_run` (Gray-Scott reaction-diffusion) and :func:`cnn_input` /
:func:`cnn_run` (a Chua-Yang cellular neural network with 3x3 templates).

The per-instance statistics of a parameter atlas (Sec. III.A) are plain
definitions written out in numpy in :mod:`oracle.atlas`.

Parameters are given as a mapping with keys ``dt, a, b, eps, c, k3, Du, Dv``
(the paper's gene, Sec. II.A, plus the cubic coefficient k3 of Eq. (2), which
the paper fixes at 1/3).  Boundary rule: ``"periodic"`` (toroidal, as in the
paper's kernels) or ``"zeroflux"`` (ghost cell copies the edge cell).

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
and ``tests/test_atlas_pins.py``
(closed forms, invariants, brute force, library routines, hand-worked golden
values and finite differences); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rdcnn_oracle.c")
_SRC_MODELS = os.path.join(_HERE, "cell_models.c")
_LIB = os.path.join(_HERE, "liboracle_rdcnn.so")

PARAM_ORDER = ("dt", "a", "b", "eps", "c", "k3", "Du", "Dv")
_BC = {"periodic": 0, "zeroflux": 1}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction, OpenMP rows)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, _SRC_MODELS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                os.path.getmtime(_SRC_MODELS)):
        build()
    lib = ctypes.CDLL(_LIB)
    L, I, P = ctypes.c_long, ctypes.c_int, ctypes.c_void_p
    lib.oracle_run_f32.argtypes = [L, L, I, P, L, P, P]
    lib.oracle_run_f64.argtypes = [L, L, I, P, L, P, P]
    lib.oracle_laplacian_f64.argtypes = [L, L, I, P, P]
    lib.oracle_grad.argtypes = [L, L, I, P, I, P, P, L, L, P, P, P, P, P]
    for f in (lib.oracle_run_f32, lib.oracle_run_f64, lib.oracle_laplacian_f64, lib.oracle_grad):
        f.restype = ctypes.c_int
    lib.oracle_gs_run.argtypes = [L, L, I, I, P, L, P, P]
    lib.oracle_gs_run.restype = ctypes.c_int
    lib.oracle_cnn_input.argtypes = [L, L, I, I, P, P, P]
    lib.oracle_cnn_input.restype = None
    lib.oracle_cnn_run.argtypes = [L, L, I, I, P, L, P, P]
    lib.oracle_cnn_run.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pvec(params, dtype):
    return np.array([float(params[k]) for k in PARAM_ORDER], dtype=dtype)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def init_state(x: np.ndarray, ka: float, dtype=np.float32):
    """Eq. (1), first line: both layers start at k_a * x (one rounding in dtype)."""
    x = np.asarray(x, dtype=dtype)
    u = (dtype(ka) * x).astype(dtype)
    return u, u.copy()


def run(u0: np.ndarray, v0: np.ndarray, params, bc: str, T: int, precision: str = "f32"):
    """Advance (u0, v0) by T steps of Eq. (1)-(3); returns new arrays (u_T, v_T).

    precision "f32": float32 arithmetic with float32-rounded parameters.
    precision "f64": float64 arithmetic with the parameters as given.
    """
    lib = _load()
    if precision == "f32":
        u = np.array(u0, dtype=np.float32, copy=True, order="C")
        v = np.array(v0, dtype=np.float32, copy=True, order="C")
        p = _pvec(params, np.float32)
        fn = lib.oracle_run_f32
    elif precision == "f64":
        u = np.array(u0, dtype=np.float64, copy=True, order="C")
        v = np.array(v0, dtype=np.float64, copy=True, order="C")
        p = _pvec(params, np.float64)
        fn = lib.oracle_run_f64
    else:
        raise ValueError(precision)
    if u.ndim != 2 or u.shape != v.shape:
        raise ValueError("u0 and v0 must be 2-D arrays of equal shape")
    R, C = u.shape
    rc = fn(R, C, _BC[bc], _ptr(p), int(T), _ptr(u), _ptr(v))
    if rc != 0:
        raise ValueError("oracle run rejected its arguments")
    return u, v


def run_snapshots(u0, v0, params, bc, T, every, precision="f32"):
    """Snapshots s_0, s_every, s_2*every, ... up to s_T (the paper's A_show/B_show)."""
    snaps = [(np.array(u0), np.array(v0))]
    u, v = u0, v0
    done = 0
    while done < T:
        n = min(every, T - done)
        u, v = run(u, v, params, bc, n, precision)
        done += n
        snaps.append((u, v))
    return snaps


def laplacian(x: np.ndarray, bc: str) -> np.ndarray:
    """Unscaled 5-point Laplacian of Eq. (1) in float64."""
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    out = np.empty_like(x)
    R, C = x.shape
    if _load().oracle_laplacian_f64(R, C, _BC[bc], _ptr(x), _ptr(out)) != 0:
        raise ValueError("bad laplacian arguments")
    return out


def grad(u0, v0, params, bc, T, lamT, muT, traj="f32", S=None):
    """Reverse pass: returns (lam0, mu0, dtheta dict, uT, vT).

    lamT, muT: dJ/du_T, dJ/dv_T.  traj: "f32" follows the float32 trajectory
    (what a float32 implementation computes), "f64" the float64 one; the reverse
    arithmetic is float64 either way.  S: checkpoint spacing (default ceil(sqrt T)).
    """
    lib = _load()
    u0 = np.array(u0, dtype=np.float64, copy=True, order="C")
    v0 = np.array(v0, dtype=np.float64, copy=True, order="C")
    R, C = u0.shape
    lam = np.array(lamT, dtype=np.float64, copy=True, order="C").reshape(R, C)
    mu = np.array(muT, dtype=np.float64, copy=True, order="C").reshape(R, C)
    if S is None:
        S = max(1, int(np.ceil(np.sqrt(max(T, 1)))))
    g = np.zeros(8, dtype=np.float64)
    uT = np.empty_like(u0)
    vT = np.empty_like(v0)
    p = _pvec(params, np.float64)
    rc = lib.oracle_grad(R, C, _BC[bc], _ptr(p), 1 if traj == "f32" else 0, _ptr(u0), _ptr(v0),
                         int(T), int(S), _ptr(lam), _ptr(mu), _ptr(g), _ptr(uT), _ptr(vT))
    if rc != 0:
        raise ValueError("oracle grad rejected its arguments")
    return lam, mu, dict(zip(PARAM_ORDER, g.tolist())), uT, vT


GS_ORDER = ("dt", "F", "k", "Du", "Dv")


def _prec(precision):
    return (64, np.float64) if precision == "f64" else (32, np.float32)


def gs_run(u0, v0, params, bc: str, T: int, precision: str = "f32"):
    """T Gray-Scott steps (cell_models.c): params maps dt, F, k, Du, Dv."""
    bits, dt = _prec(precision)
    u = np.array(u0, dtype=dt, copy=True, order="C")
    v = np.array(v0, dtype=dt, copy=True, order="C")
    p = np.array([float(params[k]) for k in GS_ORDER], dtype=dt)
    R, C = u.shape
    if _load().oracle_gs_run(R, C, _BC[bc], bits, _ptr(p), int(T), _ptr(u), _ptr(v)) != 0:
        raise MemoryError("oracle_gs_run")
    return u, v


def cnn_input(img, B, z: float, bc: str, precision: str = "f32"):
    """The Chua-Yang input layer w = (B * img) + z (cell_models.c); B is 3x3."""
    bits, dt = _prec(precision)
    g = np.array(img, dtype=dt, copy=True, order="C")
    bz = np.array(list(np.asarray(B, dtype=np.float64).reshape(9)) + [float(z)], dtype=dt)
    w = np.empty_like(g)
    R, C = g.shape
    _load().oracle_cnn_input(R, C, _BC[bc], bits, _ptr(bz), _ptr(g), _ptr(w))
    return w


def cnn_run(x0, w, dt_step: float, A, bc: str, T: int, precision: str = "f32"):
    """T Chua-Yang steps of the state x with the fixed input layer w (cell_models.c)."""
    bits, dt = _prec(precision)
    x = np.array(x0, dtype=dt, copy=True, order="C")
    ww = np.ascontiguousarray(w, dtype=dt)
    p = np.array([float(dt_step)] + list(np.asarray(A, dtype=np.float64).reshape(9)), dtype=dt)
    R, C = x.shape
    if _load().oracle_cnn_run(R, C, _BC[bc], bits, _ptr(p), int(T), _ptr(x), _ptr(ww)) != 0:
        raise MemoryError("oracle_cnn_run")
    return x
