"""Seeded synthetic inputs for the RD-CNN workloads (arXiv 2102.10340).

This module is shared by the tests, the benchmark and the oracle checks.  It
holds only input generation (initial images, parameter draws, target patterns);
none of the method's arithmetic lives here, and it imports neither the oracle
nor the GPU package.

Parameter sets use the paper's sign convention (Sec. II.A, Eq. (3)):
``f2 = -eps * (u - b*v + a)``.  A workload quoted with a positive rate
``epsilon`` in ``f2 = epsilon * (u - v)`` therefore has ``eps = -epsilon``,
``a = 0`` and ``b = 1``; one quoted with ``f1 = u - u^3 - v`` has ``c = 1`` and a
cubic coefficient ``k3 = 1`` (the paper's Eq. (2) uses ``k3 = 1/3``).
"""
from __future__ import annotations

import numpy as np

PARAM_KEYS = ("dt", "a", "b", "eps", "c", "k3", "Du", "Dv")

#: The paper's default gene (Sec. II.A, defaults of get_init_state): a=-0.3,
#: b=1.3, eps=-0.1, c=1, Du=0.06, Dv=1, dt=0.1, with Eq. (2)'s cubic 1/3.
PAPER_DEFAULT_GENE = dict(dt=0.1, a=-0.3, b=1.3, eps=-0.1, c=1.0, k3=1.0 / 3.0, Du=0.06, Dv=1.0)

#: Plain-method workload: f1 = u - u^3 - v, f2 = 0.1 (u - v), Du=0.05, Dv=1,
#: dt=0.1 (also used by the slow-growth and differentiation workloads).
PLAIN_GENE = dict(dt=0.1, a=0.0, b=1.0, eps=-0.1, c=1.0, k3=1.0, Du=0.05, Dv=1.0)


def gene(base=None, **overrides):
    """A parameter dict: ``base`` (default PLAIN_GENE) with keyword overrides."""
    g = dict(PLAIN_GENE if base is None else base)
    for k, v in overrides.items():
        if k not in PARAM_KEYS:
            raise KeyError(k)
        g[k] = float(v)
    return g


def uniform_x(rows: int, cols: int, seed: int) -> np.ndarray:
    """Fully random initial image (the paper's typ=2): x ~ U[-1, 1], float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(rows, cols)).astype(np.float32)


def patch_bounds(n: int, s: int):
    """Start/stop of a centred patch of side s on a line of n cells."""
    s = min(s, n)
    lo = (n - s) // 2
    return lo, lo + s


def centre_patch_x(rows: int, cols: int, side: int, seed: int) -> np.ndarray:
    """Zero image with a random U[-1,1] square of the given side in the middle
    (the paper's typ=1 uses an 11x11 patch; the slow-growth workload a 16x16 one)."""
    x = np.zeros((rows, cols), dtype=np.float32)
    r0, r1 = patch_bounds(rows, side)
    c0, c1 = patch_bounds(cols, side)
    rng = np.random.default_rng(seed)
    x[r0:r1, c0:c1] = rng.uniform(-1.0, 1.0, size=(r1 - r0, c1 - c0)).astype(np.float32)
    return x


def sweep_instances(n: int = 1024, seed: int = 0, sides=(128, 256, 512, 1024)):
    """Parameter-sweep instances: side uniform over ``sides``, Du ~ U[0.01,0.2],
    Dv ~ U[0.2,1.0], epsilon ~ U[0.02,0.2] (eps = -epsilon), other values as
    PLAIN_GENE.  Each instance also carries the seed of its initial image."""
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides), size=n)
    du = rng.uniform(0.01, 0.2, size=n)
    dv = rng.uniform(0.2, 1.0, size=n)
    ep = rng.uniform(0.02, 0.2, size=n)
    out = []
    for i in range(n):
        out.append(dict(rows=int(side[i]), cols=int(side[i]),
                        gene=gene(Du=float(du[i]), Dv=float(dv[i]), eps=-float(ep[i])),
                        seed=int(seed) * 100003 + i))
    return out


def stripe_target(rows: int, cols: int, seed: int, waves: int = 3) -> np.ndarray:
    """Target pattern of random sinusoid stripes: the mean of ``waves`` plane
    waves sin(k (cos(th) i + sin(th) j) + phi), k ~ U[0.05, 0.3] rad/cell,
    th ~ U[0, pi), phi ~ U[0, 2 pi).  float32."""
    rng = np.random.default_rng(seed)
    i = np.arange(rows, dtype=np.float64)[:, None]
    j = np.arange(cols, dtype=np.float64)[None, :]
    acc = np.zeros((rows, cols))
    for _ in range(waves):
        k = rng.uniform(0.05, 0.3)
        th = rng.uniform(0.0, np.pi)
        ph = rng.uniform(0.0, 2 * np.pi)
        acc += np.sin(k * (np.cos(th) * i + np.sin(th) * j) + ph)
    return (acc / waves).astype(np.float32)


def rect_image(rows: int, cols: int, seed: int, noise: float = 0.05):
    """Synthetic image: 20..60 random axis-aligned rectangles with levels
    U[-1,1] painted in order on a zero background, plus N(0, noise^2) noise.
    Returns (noisy image, clean image), float32 / float64."""
    rng = np.random.default_rng(seed)
    img = np.zeros((rows, cols))
    for _ in range(int(rng.integers(20, 61))):
        r = np.sort(rng.integers(0, rows + 1, size=2))
        c = np.sort(rng.integers(0, cols + 1, size=2))
        img[r[0]:r[1], c[0]:c[1]] = rng.uniform(-1.0, 1.0)
    noisy = img + rng.normal(0.0, noise, size=img.shape)
    return noisy.astype(np.float32), img


def sobel_target(clean: np.ndarray) -> np.ndarray:
    """Edge target: Sobel gradient magnitude of the clean image (edge-copy
    boundary), divided by its maximum.  float32."""
    from scipy import ndimage
    gx = ndimage.sobel(clean, axis=1, mode="nearest")
    gy = ndimage.sobel(clean, axis=0, mode="nearest")
    mag = np.hypot(gx, gy)
    m = mag.max()
    return (mag / m if m > 0 else mag).astype(np.float32)
