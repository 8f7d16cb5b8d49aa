"""Pins of the oracle's periodic boundaries (Sec. 2: a packet follows the grid
until it is extinguished or, without periodic boundaries, leaves the box;
with them it re-enters through the opposite face).  A periodic packet also
ends once it has crossed more than path_cells cell faces along one axis, its
photons then counted as escaped."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W


def box(n, nh, *, tau_kill=30.0, path_cells=0, periodic=True, src=((0, 0, 0),), packets=1, e_ev=13.6,
        cell_cm=3.0e20):
    ncell = n[0] * n[1] * n[2]
    x = np.zeros((5, ncell))
    x[W.X_HI] = 1.0
    x[W.X_HEI] = 1.0
    bins = W.monochromatic_table(e_ev)
    return W.Workload(
        name="periodic_test", n=tuple(n), cell_cm=cell_cm, y_he=0.0, bins=bins, redshift=-1.0,
        n_h=np.asarray(nh, np.float64).reshape(-1), x=x, temp=np.full(ncell, 1.0e4),
        src_ijk=np.array(src, np.int32), src_ndot=np.full(len(src), 1.0e48),
        src_sed=np.ones((len(src), 1)), dt_s=1.0e13, packets=packets, n_sub=1, tau_kill=tau_kill,
        flags=W.ISOTHERMAL | W.FP64_MARCH, seed=3, periodic=periodic, path_cells=path_cells)


@pytest.mark.parametrize("n,L,g", [((4, 4, 4), 10, 0), ((5, 3, 7), 23, 1), ((6, 6, 6), 1, 2), ((3, 8, 5), 40, 5)])
def test_path_limit_escape_is_the_closed_form(n, L, g):
    """One packet in a uniform, nearly transparent periodic box: it ends at the
    (L+1)-th face crossing along some axis, t_end = min_a (1 + 2L)/|c_a| (half-cell
    units from the cell centre), so escaped = w exp(-n sigma |c| t_end dx / 2)."""
    nh = np.full(n[0] * n[1] * n[2], 1.0e-6)
    w = box(n, nh, tau_kill=1.0e6, path_cells=L, src=((1, 2, 0),), packets=1)
    s = O.OracleSolve(w)
    led = s.step(seed=w.seed + g, trace_n=1, trace_len=4096)
    c, _ = O.direction(w.seed + g, 0, 0, 0)
    t_end = min(Fraction(1 + 2 * L, abs(int(ca))) for ca in c if ca != 0)
    length = float(t_end) * math.sqrt(float(sum(int(v) * int(v) for v in c))) * 0.5 * w.cell_cm
    sigma = float(w.bins.sigma[0, 0])
    wgt = 1.0e48 * w.dt_s
    assert led["n_escaped"] == 1 and led["n_truncated"] == 0
    assert led["escaped"] == pytest.approx(wgt * math.exp(-1.0e-6 * sigma * length), rel=1e-12, abs=0)
    assert s.trace[0][1] == O.FATE_PATH
    assert led["emitted"] == pytest.approx(led["absorbed"] + led["escaped"], rel=1e-14, abs=0)


def test_equals_the_unfolded_box():
    """A periodic grid is the unit cell of an infinite periodic medium: the same
    packets in a 5x5x5 tiling of the grid (non-periodic, sources in the middle
    copy) deposit, folded back onto the unit cell, what the periodic run
    deposits, as long as they are extinguished inside the tiling."""
    n = (5, 6, 7)
    rng = np.random.default_rng(4)
    nh = np.exp(rng.normal(0.0, 0.5, size=n[::-1])).ravel() * 2.0e-3      # natural order (x fastest)
    src = ((1, 2, 3), (4, 0, 6))
    P = 400
    per = box(n, nh, tau_kill=8.0, path_cells=2046, src=src, packets=P)
    big_n = tuple(5 * v for v in n)
    big_nh = np.tile(nh.reshape(n[::-1]), (5, 5, 5)).ravel()
    big_src = tuple((a + 2 * n[0], b + 2 * n[1], c + 2 * n[2]) for a, b, c in src)
    big = box(big_n, big_nh, tau_kill=8.0, periodic=False, src=big_src, packets=P)
    sp, sb = O.OracleSolve(per), O.OracleSolve(big)
    lp = sp.step()
    lb = sb.step()
    assert lb["n_escaped"] == 0 and lp["n_escaped"] == 0          # all extinguished inside the tiling
    assert lp["crossings"] == lb["crossings"] and lp["n_truncated"] == lb["n_truncated"] == P
    assert lp["absorbed"] == pytest.approx(lb["absorbed"], rel=1e-13, abs=0)
    folded = sb.acc[0].reshape(big_n[::-1]).reshape(5, n[2], 5, n[1], 5, n[0]).sum(axis=(0, 2, 4)).ravel()
    assert np.allclose(sp.acc[0], folded, rtol=1e-12, atol=0.0)
    assert np.count_nonzero(folded) > 0.5 * folded.size


def test_ledger_closes_and_wraps_absorb_more():
    n = (6, 6, 6)
    nh = np.full(216, 1.0e-4)
    kw = dict(tau_kill=30.0, src=((2, 3, 1),), packets=300)
    lp = O.OracleSolve(box(n, nh, path_cells=30, **kw)).step()
    lo = O.OracleSolve(box(n, nh, periodic=False, **kw)).step()
    for led in (lp, lo):
        assert abs(led["emitted"] - led["absorbed"] - led["escaped"] - led["truncated"]) <= 1e-13 * led["emitted"]
    # tau ~ 0.19 per cell: a packet leaves the plain box after a few cells, but in
    # the periodic one it travels > 30 cells, so almost nothing escapes
    assert lo["escaped"] > 0.3 * lo["emitted"]
    assert lp["escaped"] < 0.02 * lp["emitted"]
    assert lp["crossings"] > 5 * lo["crossings"]
