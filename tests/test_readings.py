"""Evidence for the reading of the cubic term (Sec. II.A, Eq. (2)).

Eq. (2) and the NumPy/CuPy listings give f1 = c u - u^3/3 - v; the PyCUDA and
Numba kernels as printed compute u (c - eps u) - v, a quadratic term that
reuses eps.  The library follows Eq. (2) with the cubic coefficient as a
parameter.  These tests show what the printed quadratic term would do from
the paper's own default state: with the default gene (a = -0.3, b = 1.3,
eps = -0.1, c = 1, Du = 0.06, Dv = 1, dt = 0.1) and a random 11x11 centre
patch it blows up within a few dozen steps, at the default (Du, Dv) and at the
three points Sec. III.A names, so it cannot be the model behind the paper's
figures; Eq. (2)'s cubic stays bounded.  The quadratic update is written out
here in float64 numpy (it is not part of the library or the oracle); the
cubic run is the oracle's.
"""
import numpy as np
import pytest

import oracle
import workloads as W

N, T = 64, 300


def _lap_periodic(q):
    return np.roll(q, 1, 0) + np.roll(q, -1, 0) + np.roll(q, 1, 1) + np.roll(q, -1, 1) - 4.0 * q


def _listing_quadratic_run(g, x, T):
    """Eq. (1) with the printed kernels' f1 = u (c - eps u) - v, periodic."""
    u = x.astype(np.float64).copy()
    v = u.copy()
    with np.errstate(over="ignore", invalid="ignore"):
        for t in range(T):
            f1 = u * (g["c"] - g["eps"] * u) - v
            f2 = -g["eps"] * (u - g["b"] * v + g["a"])
            u, v = u + g["dt"] * (f1 + g["Du"] * _lap_periodic(u)), \
                v + g["dt"] * (f2 + g["Dv"] * _lap_periodic(v))
            if not (np.isfinite(u).all() and np.isfinite(v).all()):
                return t + 1, None
    return None, (u, v)


@pytest.mark.parametrize("du,dv", [(0.06, 1.0), (0.3, 1.0), (0.5, 0.8), (0.7, 0.8)])
def test_printed_quadratic_term_diverges_from_the_default_state(du, dv):
    g = dict(W.PAPER_DEFAULT_GENE, Du=du, Dv=dv)
    x = W.centre_patch_x(N, N, 11, 0)
    blew_up_at, _ = _listing_quadratic_run(g, x, T)
    assert blew_up_at is not None and blew_up_at < 150, blew_up_at


@pytest.mark.parametrize("du,dv", [(0.06, 1.0), (0.3, 1.0), (0.5, 0.8), (0.7, 0.8)])
def test_cubic_term_stays_bounded_from_the_default_state(du, dv):
    g = dict(W.PAPER_DEFAULT_GENE, Du=du, Dv=dv)
    u0, v0 = oracle.init_state(W.centre_patch_x(N, N, 11, 0), 1.0, np.float64)
    u, v = oracle.run(u0, v0, g, "periodic", T, "f64")
    assert np.isfinite(u).all() and np.isfinite(v).all()
    assert np.abs(u).max() < 3.0 and np.abs(v).max() < 3.0
