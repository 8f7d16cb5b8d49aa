"""Pins of the oracle's cell traversal (Sec. 2: the path length of a packet in
every crossed cell) against brute-force exact-rational slab intersection and
against Cauchy's mean-chord law."""
from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import oracle as O


def brute_force(n, o, c):
    """Cells of positive-length intersection with the ray o + t c (t > 0) and
    the ray parameter where each is left, from all grid-plane crossings."""
    ts = {Fraction(0)}
    for a in range(3):
        if c[a] == 0:
            continue
        for m in range(n[a] + 1):
            t = Fraction(2 * m - o[a], c[a])
            if t > 0:
                ts.add(t)
    ts = sorted(ts)
    cells, s_exit = [], []
    for i in range(len(ts) - 1):
        tm = (ts[i] + ts[i + 1]) / 2
        k = [math.floor((o[a] + tm * c[a]) / 2) for a in range(3)]
        if any(k[a] < 0 or k[a] >= n[a] for a in range(3)):
            break
        cells.append(k[0] + n[0] * (k[1] + n[1] * k[2]))
        s_exit.append(ts[i + 1])
    face = 0
    if s_exit:
        t = s_exit[-1]
        for a in range(3):
            p = o[a] + t * c[a]
            if c[a] > 0 and p == 2 * n[a]:
                face |= (1 << a) | (8 << a)
            if c[a] < 0 and p == 0:
                face |= 1 << a
    return cells, s_exit, face


def check(n, o, c):
    cells, s, face, cnt = O.trace_ray(n, o, c)
    bc, bs, bface = brute_force(n, o, c)
    assert cnt == len(bc), (n, o, c)
    assert list(cells) == bc, (n, o, c)
    # exit parameters: correctly rounded quotients of exact rationals
    assert list(s) == [float(t) for t in bs], (n, o, c)
    assert face == bface, (n, o, c)


DEGENERATE = [
    ((1 << 19), 0, 0), (0, -(1 << 19), 0), (0, 0, 5),          # axis aligned
    (3, 3, 0), (-7, 7, 0), (0, 2, -2),                        # face diagonals
    (1, 1, 1), (-4, 4, -4), (5, -5, 5),                       # body diagonals
    (2, 1, 0), (1, 2, 2), (-3, 1, 2), (6, -2, 3), (1, 0, -1),
]


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 3, 1), (4, 4, 4), (5, 2, 7)])
def test_degenerate_rays_match_brute_force(n):
    origins = []
    for i in range(n[0]):
        for j in range(n[1]):
            for k in range(n[2]):
                origins.append((2 * i + 1, 2 * j + 1, 2 * k + 1))   # cell centres
    origins += [(0, 0, 0), (2 * n[0], 0, 0), (0, 2 * n[1], 2 * n[2])]  # grid corners
    for o in origins:
        for c in DEGENERATE:
            for sgn in ((1, 1, 1), (-1, 1, 1), (1, -1, -1)):
                cc = tuple(c[a] * sgn[a] for a in range(3))
                # corner origins only with directions pointing into the grid
                if any((o[a] == 0 and cc[a] < 0) or (o[a] == 2 * n[a] and cc[a] > 0)
                       for a in range(3)):
                    continue
                if any(o[a] in (0, 2 * n[a]) and cc[a] == 0 for a in range(3)):
                    continue
                check(n, o, cc)


def test_random_rays_match_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(400):
        n = tuple(int(v) for v in rng.integers(1, 9, 3))
        o = tuple(int(rng.integers(1, 2 * n[a])) for a in range(3))   # interior, may sit on planes
        if rng.random() < 0.5:
            c = tuple(int(v) for v in rng.integers(-3, 4, 3))          # many exact ties
        else:
            c = tuple(int(v) for v in rng.integers(-(1 << 20), 1 << 20, 3))
        if c == (0, 0, 0):
            continue
        check(n, o, c)


def test_sampled_directions_match_brute_force():
    n = (16, 16, 16)
    for g in range(150):
        c, _ = O.direction(1, 0, g, 0)
        check(n, (15, 17, 9), tuple(int(v) for v in c))


def test_cauchy_mean_chord():
    """For isotropic lines the mean chord through a unit cube is 4V/S = 2/3;
    equivalently a ray of length L enters 1.5 L cells on average."""
    n = (64, 64, 64)
    rng = np.random.default_rng(3)
    # start points sit on the half-cell lattice, so count face crossings in a
    # window [a, a + lam] away from the start where their phase is uniform
    a0, lam = 3.0, 20.0
    entered = 0
    rays = 6000
    for g in range(rays):
        c, _ = O.direction(7, 0, g, 0)
        o = tuple(int(v) for v in rng.integers(56, 72, 3))
        cells, s, face, cnt = O.trace_ray(n, o, c)
        dist = s * np.linalg.norm(c.astype(np.float64)) / 2.0       # cells
        entered += int(np.sum((dist[:-1] >= a0) & (dist[:-1] < a0 + lam)))
        # crossing count identity: 1 + sum |dk| without ties
        k0 = np.array([cells[0] % 64, (cells[0] // 64) % 64, cells[0] // 4096])
        k1 = np.array([cells[-1] % 64, (cells[-1] // 64) % 64, cells[-1] // 4096])
        assert cnt <= 1 + int(np.abs(k1 - k0).sum())
    mean_chord = rays * lam / entered
    # per-ray count variance is small (about 0.2 L); 4 sigma band
    sd = (2.0 / 3.0) * math.sqrt(0.3 * lam / rays) / (1.5 * lam) * 1.5
    assert abs(mean_chord - 2.0 / 3.0) < 4 * sd + 2e-3, mean_chord
