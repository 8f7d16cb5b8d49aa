"""Pins of the oracle's counter-based generator and direction sampler.

Philox4x64-10 is checked against the published known-answer vectors and the
independent numpy implementation; the direction sampler against isotropy
statistics (Sec. 2: emission directions follow the source's angular PDF,
isotropic for every workload here)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLD, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert [int(v) for v in O.philox(ctr, key)] == out


def _numpy_block(ctr, key):
    """Block at counter `ctr` from numpy's Philox (it increments before use)."""
    v = (sum(int(c) << (64 * i) for i, c in enumerate(ctr)) - 1) % (1 << 256)
    c = np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=c, key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


def test_philox_matches_numpy():
    rng = np.random.default_rng(11)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 1 << 63, 4)]
        key = [int(x) for x in rng.integers(0, 1 << 63, 2)]
        assert [int(v) for v in O.philox(ctr, key)] == _numpy_block(ctr, key)
    # carries across counter words
    M = (1 << 64) - 1
    for ctr in ([M, 0, 0, 0], [M, M, 0, 7], [0, 1, 2, 3]):
        assert [int(v) for v in O.philox(ctr, [5, 9])] == _numpy_block(ctr, [5, 9])


def test_direction_is_first_accepted_block():
    """Components come from the top 21 bits of the first accepted block."""
    for g in range(300):
        c, att = O.direction(3, 2, g, 17)
        blk = _numpy_block([g, 17, att - 1, 0], [3, 2])
        v = np.array([(b >> 43) - (1 << 20) for b in blk[:3]])
        assert np.array_equal(c, v)
        q = int((v.astype(np.int64) ** 2).sum())
        assert (1 << 36) <= q <= (1 << 40)
        for a in range(att - 1):            # every earlier attempt was rejected
            b = _numpy_block([g, 17, a, 0], [3, 2])
            u = np.array([(x >> 43) - (1 << 20) for x in b[:3]], dtype=np.int64)
            qq = int((u ** 2).sum())
            assert not ((1 << 36) <= qq <= (1 << 40))


def _dirs(n, seed=1, octant=False, step=0):
    return np.array([O.direction(seed, 0, g, step, octant)[0] for g in range(n)], dtype=np.float64)


def test_direction_isotropy():
    d = _dirs(60000)
    u = d / np.linalg.norm(d, axis=1)[:, None]
    n = len(u)
    # mean vector ~ 0 (each component has variance 1/3)
    assert np.all(np.abs(u.mean(0)) < 4.0 * np.sqrt(1.0 / 3.0 / n))
    # second moments 1/3 each, cross moments 0
    m2 = (u[:, :, None] * u[:, None, :]).mean(0)
    sd = np.sqrt((1.0 / 5.0 - 1.0 / 9.0) / n)     # var of u_a^2 = 1/5 - 1/9
    assert np.all(np.abs(np.diag(m2) - 1.0 / 3.0) < 5 * sd)
    assert np.all(np.abs(m2[~np.eye(3, dtype=bool)]) < 5 * np.sqrt(1.0 / 15.0 / n))
    # cos(theta) uniform on [-1, 1], azimuth uniform on [0, 2 pi)
    assert stats.kstest(u[:, 2], "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    phi = np.arctan2(u[:, 1], u[:, 0]) + np.pi
    assert stats.kstest(phi, "uniform", args=(0.0, 2 * np.pi)).pvalue > 1e-3


def test_direction_octant_and_streams():
    d = _dirs(5000, octant=True)
    assert np.all(d >= 0)
    u = d / np.linalg.norm(d, axis=1)[:, None]
    assert stats.kstest(u[:, 0], "uniform", args=(0.0, 1.0)).pvalue > 1e-3
    # different sub-step indices and seeds give different streams
    a, b, c = _dirs(64), _dirs(64, step=1), _dirs(64, seed=2)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    # acceptance: about (4/3 pi)(1 - 1/64) / 8 of the cube
    atts = [O.direction(9, 0, g, 0)[1] for g in range(20000)]
    acc = 20000 / np.sum(atts)
    assert abs(acc - (4.0 / 3.0 * np.pi * (1 - 1 / 64) / 8.0)) < 0.01
