"""The oracle on the two validation set-ups of Sec. 4.2 (Test 2: H II region
with the temperature followed; Test 3: H+He H II region of the CLOUDY94
comparison), at 16^3 over their whole runs.

No reference profiles are available, so these are sanity bands and
invariants (parity unpinned for the thermal and helium physics beyond them):
photo-heated gas at 1-3e4 K, hard photons pre-heating the gas ahead of the
front, helium mostly singly ionised by a 6e4 K source, the H+He front at its
equilibrium (Stroemgren) radius for the recombination coefficient at the
temperature reached, fractions summing to one."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W


def radius_cells(w, o):
    """Ionised-volume radius r = (6V/pi)^(1/3) of a corner source (Test 0's
    definition), in cells."""
    return (6.0 * o.x[1].sum() / math.pi) ** (1.0 / 3.0)


def corner_distance(n):
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return np.sqrt((i + 0.5) ** 2 + (j + 0.5) ** 2 + (k + 0.5) ** 2).transpose(2, 1, 0).reshape(-1)


@pytest.fixture(scope="module")
def test3_run():
    w = W.hhe_test3(n=16, packets=40000, steps=6, n_sub=20)
    o = O.OracleSolve(w)
    radii = []
    for _ in range(w.steps):
        st = o.step()
        res = abs(st["emitted"] - (st["absorbed"] + st["escaped"] + st["truncated"])) / st["emitted"]
        assert res <= 1e-12
        radii.append(radius_cells(w, o))
    return w, o, radii


def test_test3_helium_region_sanity_bands(test3_run):
    w, o, radii = test3_run
    r = corner_distance(w.n[0])
    inner = r < 0.6 * radii[-1]
    assert inner.sum() >= 10
    T = o.T[inner]
    assert 1.0e4 < np.median(T) < 3.0e4
    assert np.median(o.x[0][inner]) < 1e-2                     # hydrogen ionised
    assert np.median(o.x[3][inner]) > 0.9                      # helium mostly HeII
    assert np.median(o.x[4][inner]) < 0.1                      # little HeIII from a 6e4 K source
    outer = r > 1.5 * radii[-1]
    assert np.all(o.x[0][outer] > 0.99) and np.all(o.T[outer] < 200.0)
    for a in (o.x[0] + o.x[1], o.x[2] + o.x[3] + o.x[4]):
        assert np.max(np.abs(a - 1.0)) < 1e-12


def test_test3_front_at_equilibrium_stroemgren_radius(test3_run):
    w, o, radii = test3_run
    # equilibrium: the front stops moving (the run is five recombination times)
    assert abs(radii[-1] / radii[-2] - 1.0) < 0.03
    # Stroemgren radius of the corner octant: N/8 = (1/8)(4 pi/3) r^3 alpha_B(T) n_e n_H,
    # n_e from hydrogen and singly ionised helium, alpha at the ionised gas's temperature
    r = corner_distance(w.n[0])
    inner = r < 0.6 * radii[-1]
    T = float(np.median(o.T[inner]))
    ne = 0.9 * (1.0 + (1.0 / 9.0) * (np.median(o.x[3][inner]) + 2.0 * np.median(o.x[4][inner])))
    alpha = O.rates_at(T).a_hii
    rs = (3.0 * w.src_ndot[0] / (4.0 * math.pi * alpha * ne * 0.9)) ** (1.0 / 3.0) / w.cell_cm
    assert abs(radii[-1] / rs - 1.0) < 0.15, (radii[-1], rs)


def test_test2_heating_and_preheating():
    w = W.thermal_test2(n=16, packets=40000, steps=5, n_sub=20)
    o = O.OracleSolve(w)
    r = corner_distance(w.n[0])
    radii, t_out = [], []
    for _ in range(w.steps):
        st = o.step()
        res = abs(st["emitted"] - (st["absorbed"] + st["escaped"] + st["truncated"])) / st["emitted"]
        assert res <= 1e-12
        radii.append(radius_cells(w, o))
        t_out.append(float(np.median(o.T[r > 1.5 * radii[-1]])))
    inner = r < 0.6 * radii[-1]
    assert 1.0e4 < np.median(o.T[inner]) < 3.0e4
    assert np.median(o.x[0][inner]) < 1e-2
    # the front still grows at 50 Myr (t_rec = 122 Myr at n_H = 1e-3)
    assert all(b > a for a, b in zip(radii, radii[1:]))
    # hard photons run ahead of the front and heat the neutral gas above 100 K, more with time
    assert t_out[0] > 100.0 and all(b > a for a, b in zip(t_out, t_out[1:]))
