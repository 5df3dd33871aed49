"""Pins of the atlas-statistics oracle (Sec. III.A) against hand-worked values,
library routines and invariants."""
import os

import numpy as np
import pytest

from oracle import atlas

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "atlas_stats.txt")


def _cases():
    cases, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], R=int(tok[2]), C=int(tok[3]), ref=float(tok[5]),
                       far=float(tok[7]), move=float(tok[9]), prev=None)
            cases.append(cur)
        elif tok[0] == "want":
            cur["want"] = np.array([float(x) for x in tok[1:]])
        else:
            cur[tok[0]] = np.array([float(x) for x in tok[1:]], dtype=np.float32).reshape(cur["R"], cur["C"])
    return cases


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_worked_stats(case):
    got = atlas.instance_stats(case["u"], case["v"], case["prev"], case["ref"], case["far"],
                               case["move"])
    want = case["want"]
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.allclose(got[ok], want[ok], rtol=1e-15, atol=1e-15), (got, want)


def test_threshold_decided_in_float32():
    """0.1 rounded to float32 sits exactly at a float32 threshold of 0.1: not
    counted, although in float64 it exceeds 0.1."""
    u = np.full((2, 2), np.float32(0.1))
    assert float(u[0, 0]) > 0.1  # the float64 test would count it
    s = atlas.instance_stats(u, u, u * 0, 0.0, 0.1, 0.1)
    assert s[4] == 0.0 and s[5] == 0.0
    s = atlas.instance_stats(u, u, u * 0, 0.0, 0.0999, 0.0999)
    assert s[4] == 1.0 and s[5] == 1.0


def test_against_numpy_moments_and_invariants():
    rng = np.random.default_rng(4)
    u = rng.uniform(-1, 1, (37, 53)).astype(np.float32)
    v = rng.normal(0.3, 2.0, (37, 53)).astype(np.float32)
    p = (u + rng.normal(0, 0.01, u.shape)).astype(np.float32)
    s = atlas.instance_stats(u, v, p, 0.2, 0.5, 0.01)
    assert np.isclose(s[0], np.mean(u, dtype=np.float64), rtol=1e-13)
    assert np.isclose(s[1], np.var(u, dtype=np.float64), rtol=1e-12)
    assert np.isclose(s[2], np.mean(v, dtype=np.float64), rtol=1e-13)
    assert np.isclose(s[3], np.var(v, dtype=np.float64), rtol=1e-12)
    d = (u - p).astype(np.float64)
    assert np.isclose(s[7], np.sqrt(np.mean(d * d)), rtol=1e-13)
    assert s[6] == np.max(np.abs(u - p))
    # shifting v by a constant moves its mean by it and keeps its variance
    t = atlas.instance_stats(u, v + np.float32(4.0), p, 0.2, 0.5, 0.01)
    assert np.isclose(t[2], s[2] + 4.0, rtol=1e-12)
    assert np.isclose(t[3], s[3], rtol=1e-6)
    # permuting cells changes nothing but rounding
    perm = rng.permutation(u.size)
    q = atlas.instance_stats(u.ravel()[perm], v.ravel()[perm], p.ravel()[perm], 0.2, 0.5, 0.01)
    assert np.allclose(q, s, rtol=1e-12) and q[4] == s[4] and q[5] == s[5] and q[6] == s[6]
    # the far fraction is the fraction of cells outside [ref - theta, ref + theta]
    assert s[4] == np.count_nonzero((u < np.float32(0.2 - 0.5)) | (u > np.float32(0.2 + 0.5))) / u.size
