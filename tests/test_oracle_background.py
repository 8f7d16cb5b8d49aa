"""Pins of the oracle's background field (Sec. 2: packets from diffuse fields
such as the UV background), taken as an isotropic intensity entering the box
through its faces: packets start at boundary cell faces chosen uniformly over
the boundary area, with isotropic inward directions weighted by 2 cos(theta)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W


def bg_box(n, nh, *, packets=20000, ndot=1.0e50, periodic=False, path_cells=0, seed=5):
    ncell = n[0] * n[1] * n[2]
    x = np.zeros((5, ncell))
    x[W.X_HI] = 1.0
    x[W.X_HEI] = 1.0
    bins = W.monochromatic_table(13.6)
    return W.Workload(
        name="background_test", n=tuple(n), cell_cm=3.0e20, y_he=0.0, bins=bins, redshift=-1.0,
        n_h=np.asarray(nh, np.float64).reshape(-1), x=x, temp=np.full(ncell, 1.0e4),
        src_ijk=np.zeros((0, 3), np.int32), src_ndot=np.zeros(0), src_sed=np.zeros((0, 1)),
        dt_s=1.0e12, packets=0, n_sub=1, flags=W.ISOTHERMAL | W.FP64_MARCH, seed=seed,
        periodic=periodic, path_cells=path_cells,
        background=W.Background(ndot, np.ones(1), packets))


def test_mean_chord_is_cauchys():
    """Thin uniform gas: absorbed / emitted = n sigma <l>, and for an isotropic
    field the flux-weighted mean chord of a convex body is 4V/S (Cauchy); the
    box is not a cube, so the split of packets over the faces matters."""
    n = (4, 8, 16)
    nh = np.full(n[0] * n[1] * n[2], 1.0e-7)
    w = bg_box(n, nh, packets=40000)
    led = O.OracleSolve(w).step()
    sig = float(w.bins.sigma[0, 0])
    V = n[0] * n[1] * n[2]
    S = 2 * (n[0] * n[1] + n[1] * n[2] + n[0] * n[2])
    tau_per_cell = 1.0e-7 * sig * w.cell_cm
    want = tau_per_cell * 4.0 * V / S
    assert led["emitted"] == pytest.approx(w.background.ndot * w.dt_s, rel=0.02, abs=0)
    assert led["absorbed"] / led["emitted"] == pytest.approx(want, rel=0.02, abs=0)
    assert led["escaped"] + led["absorbed"] == pytest.approx(led["emitted"], rel=1e-13, abs=0)
    assert led["packets"] == 40000 and led["n_escaped"] == 40000


def test_thin_gas_is_lit_uniformly():
    """An isotropic field in optically thin gas gives every cell the same
    photo-ionisation: absorbed per cell = 4 Ndot n sigma V dt / A."""
    n = (10, 10, 10)
    nh = np.full(1000, 1.0e-7)
    w = bg_box(n, nh, packets=200000)
    s = O.OracleSolve(w)
    s.step()
    sig = float(w.bins.sigma[0, 0])
    A = 2.0 * 3 * 100 * w.cell_cm ** 2
    V = w.cell_cm ** 3
    want = 4.0 * w.background.ndot * 1.0e-7 * sig * V * w.dt_s / A
    d = s.acc[0].reshape(10, 10, 10)
    assert d.mean() == pytest.approx(want, rel=0.01, abs=0)
    assert d[3:7, 3:7, 3:7].mean() == pytest.approx(want, rel=0.03, abs=0)       # centre
    assert d[[0, -1]][:, [0, -1]][:, :, [0, -1]].mean() == pytest.approx(want, rel=0.1, abs=0)  # corners


def test_directions_point_inward_and_weights_average_one():
    """Opaque boundary cells: every background photon is absorbed in the first
    boundary layer (inward directions), so the box interior gets nothing."""
    n = (6, 6, 6)
    nh = np.full(216, 10.0)
    w = bg_box(n, nh, packets=3000)
    s = O.OracleSolve(w)
    led = s.step()
    d = s.acc[0].reshape(6, 6, 6)
    assert led["escaped"] < 1e-10 * led["emitted"]
    assert d[1:-1, 1:-1, 1:-1].sum() < 1e-10 * d.sum()
    assert led["emitted"] == pytest.approx(w.background.ndot * w.dt_s, rel=0.05, abs=0)


def test_periodic_background_absorbs_more_and_closes():
    n = (6, 6, 6)
    nh = np.full(216, 1.0e-4)
    lp = O.OracleSolve(bg_box(n, nh, packets=3000, periodic=True, path_cells=40)).step()
    lo = O.OracleSolve(bg_box(n, nh, packets=3000)).step()
    for led in (lp, lo):
        assert abs(led["emitted"] - led["absorbed"] - led["escaped"] - led["truncated"]) <= 1e-13 * led["emitted"]
    assert lp["absorbed"] > 2.0 * lo["absorbed"]


SCAN_C = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int orc_direction_ex(uint64_t, uint64_t, uint64_t, uint64_t, int, uint64_t, int32_t *);
int main(int argc, char **argv) {
    const uint64_t seed = strtoull(argv[1], 0, 10), n = strtoull(argv[2], 0, 10);
    int32_t c[3];
    for (uint64_t b = 0; b < n; ++b) {
        orc_direction_ex(seed, 0, b, 0, 0, 3, c);
        for (int a = 0; a < 3; ++a)
            if (c[a] == 0) printf("%llu %d\n", (unsigned long long)b, a);
    }
    return 0;
}
"""


def test_zero_normal_component_is_taken_as_one(tmp_path):
    """Reading of the face entry: a background packet whose isotropic
    direction has no component along its face's normal (probability ~2^-21
    per packet) would run along the face; it is sent inward with normal
    component 1 and weighted 2 |c_n| / |c| as any other.  Packets with a zero
    component are found by scanning the direction stream (a C loop over the
    oracle's sampler)."""
    import subprocess
    src = tmp_path / "scan.c"
    src.write_text(SCAN_C)
    exe = tmp_path / "scan"
    lib = O.build()
    subprocess.check_call(["gcc", "-O2", "-o", str(exe), str(src), lib, f"-Wl,-rpath,{os.path.dirname(lib)}"])
    seed = 7
    hits = subprocess.check_output([str(exe), str(seed), str(1 << 24)], text=True).split("\n")
    hits = [tuple(int(v) for v in h.split()) for h in hits if h.strip()]
    assert len(hits) >= 5
    g = O.Grid()
    g.n[0], g.n[1], g.n[2] = 3, 4, 5
    g.cell_cm = 1.0
    g.n_bins = 1
    ndot, dt, P = 1.0e50, 2.0, 1 << 24
    checked = 0
    for b, a in hits:
        raw, _ = O.direction_ex(seed, 0, b, 0, False, 3)
        o, c, w = O.background_packet(g, ndot, [1.0], dt, P, seed, 0, 0, b)
        axis = [k for k in range(3) if o[k] in (0, 2 * g.n[k])]
        assert len(axis) == 1
        axis = axis[0]
        assert all(c[k] == raw[k] for k in range(3) if k != axis)
        inward = 1 if o[axis] == 0 else -1
        if raw[axis] == 0:
            assert c[axis] == inward
            checked += 1
        else:
            assert c[axis] == inward * abs(raw[axis])
        q = float(c[0]) ** 2 + float(c[1]) ** 2 + float(c[2]) ** 2
        assert w == pytest.approx(ndot * dt / P * 2.0 * abs(c[axis]) / math.sqrt(q), rel=1e-14, abs=0)
    assert checked >= 1
