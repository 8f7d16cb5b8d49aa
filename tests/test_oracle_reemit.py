"""Pins of the oracle's recombination re-emission (Sec. 2: the network records
the recombinations N_rec of each cell; once N_rec >= f_rec N_a the cell emits
a packet of recombination photons with a Milne spectrum and its counter
restarts; Sec. 3: pCRASH2 emits when a packet crosses such a cell).

Each pin rests on something other than the oracle's own formulas: textbook
recombination coefficients, quadrature of the exact rate-equation solution,
number conservation, a closed-form spectrum, brute-force selection, and the
on-the-spot approximation of a Stroemgren sphere."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.linalg import expm
from scipy.special import exp1

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W


def one_cell(y_he=0.0, n_chem=8, cell_cm=3.0e20):
    g = O.Grid()
    g.n[0] = g.n[1] = g.n[2] = 1
    g.cell_cm = cell_cm
    g.y_he = y_he
    g.n_bins = 1
    g.redshift = -1.0
    g.tau_kill = 30.0
    g.n_chem = n_chem
    g.flags = 1
    return g


# --------------------------------------------------------------------------
# rates
# --------------------------------------------------------------------------
def test_case_a_hydrogen_matches_textbook():
    """Osterbrock & Ferland (2006), Table 2.1 at 1e4 K: alpha_A = 4.18e-13,
    alpha_B = 2.59e-13 cm^3/s, so 38 % of recombinations reach n = 1."""
    a = O.rates_case_a(1.0e4).a_hii
    b = O.rates_at(1.0e4).a_hii
    assert a == pytest.approx(4.18e-13, rel=0.03, abs=0)
    assert b == pytest.approx(2.59e-13, rel=0.01, abs=0)
    assert O.ground_fraction(1.0e4)[0] == pytest.approx((4.18 - 2.59) / 4.18, rel=0.05, abs=0)


def test_hydrogenic_scaling_of_heiii():
    """A hydrogenic ion of charge Z has alpha_Z(T) = Z alpha_1(T / Z^2) (up to
    the ratio of the ionisation temperatures used by the fits); the share of
    ground-state recombinations is therefore the same at scaled temperatures."""
    ratio = 631515.0 / 157807.0
    for t in (3.0e3, 1.0e4, 4.0e4):
        assert O.rates_case_a(t * ratio).a_heiii == pytest.approx(2.0 * O.rates_case_a(t).a_hii, rel=1e-12, abs=0)
        assert O.rates_at(t * ratio).a_heiii == pytest.approx(2.0 * O.rates_at(t).a_hii, rel=1e-12, abs=0)
        p_h, _, p_he = O.ground_fraction(t), None, O.ground_fraction(t * ratio)
        assert p_he[2] == pytest.approx(p_h[0], rel=1e-12, abs=0)


def test_ground_fractions_in_range():
    for t in np.geomspace(10.0, 1.0e9, 33):
        p = O.ground_fraction(t)
        assert np.all(p >= 0.0) and np.all(p < 1.0)
        assert p[0] > 0.0 and p[2] > 0.0 and (t < 100.0 or p[1] > 0.0)
        # case A exceeds case B by the ground-state term (the HeII power-law
        # fits cross below ~70 K, outside their range)
        assert O.rates_case_a(t).a_hii > O.rates_at(t).a_hii
        assert t < 100.0 or O.rates_case_a(t).a_heii > O.rates_at(t).a_heii


# --------------------------------------------------------------------------
# recombination counting
# --------------------------------------------------------------------------
@pytest.mark.parametrize("I,R,h,x0", [(1e-13, 4e-16, 1e13, 0.3), (0.0, 2e-15, 5e14, 0.9),
                                      (3e-12, 1e-15, 1e12, 0.0), (1e-17, 1e-17, 1e10, 0.5)])
def test_hii_time_is_the_integral_of_the_solution(I, R, h, x0):
    """Integral over h of x_HII(t) = eq + (x0 - eq) exp(-(I+R) t), by quadrature."""
    lam = I + R
    eq = I / lam
    xt = lambda t: eq + (x0 - eq) * math.exp(-lam * t)
    want = quad(xt, 0.0, h, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    got = O.hii_time(x0, xt(h), I, R, h)
    assert got == pytest.approx(want, rel=1e-9, abs=1e-12 * h)


@pytest.mark.parametrize("rates,h", [((1e-13, 3e-15, 2e-14, 5e-15), 1e13), ((0.0, 2e-15, 0.0, 4e-15), 3e14),
                                     ((5e-12, 1e-16, 1e-12, 3e-16), 1e12), ((1e-14, 1e-14, 1e-14, 1e-14), 2e13)])
def test_he_ion_time_is_the_integral_of_the_chain(rates, h):
    """Integrals of x_HeII(t), x_HeIII(t) along exp(M t) x0 (scipy's matrix
    exponential), by Gauss-Legendre quadrature."""
    I1, R2, I2, R3 = rates
    M = np.array([[-I1, R2, 0.0], [I1, -(R2 + I2), R3], [0.0, I2, -R3]])
    x0 = np.array([0.5, 0.3, 0.2])
    xh = expm(M * h) @ x0
    nodes, wts = np.polynomial.legendre.leggauss(64)
    ts = 0.5 * h * (nodes + 1.0)
    vals = np.array([expm(M * t) @ x0 for t in ts])
    want = 0.5 * h * (wts[:, None] * vals).sum(axis=0)
    got = O.he_ion_time(x0, xh, I1, R2, I2, R3, h)
    assert got[0] == pytest.approx(want[1], rel=1e-9, abs=0)
    assert got[1] == pytest.approx(want[2], rel=1e-9, abs=0)


def test_pure_recombination_counts_the_ions_lost():
    """No photons and no collisional ionisation (3000 K): every recombination
    removes an ion, so the counters equal the ion fractions lost (H) and the
    HeI gained / HeIII lost (He)."""
    g = one_cell(y_he=0.1, n_chem=16)
    x0 = [0.2, 0.8, 0.1, 0.5, 0.4]
    x, t, rc = O.update_cell_rx(g, 3.0e14, 1.0e-2, x0, 3000.0, [0, 0, 0, 0], [0, 0, 0])
    assert x[1] < 0.8 * 0.9                             # a good part recombined
    assert rc[0] == pytest.approx(x0[1] - x[1], rel=1e-10, abs=0)
    assert rc[1] == pytest.approx(x[2] - x0[2], rel=1e-10, abs=0)
    assert rc[2] == pytest.approx(x0[4] - x[4], rel=1e-10, abs=0)


def test_counting_update_recombines_at_the_case_a_rate():
    """Pure H, no photons, 3000 K (no collisional ionisation): with
    recombinations counted the update follows dx/dt = -alpha_A n_H x^2, whose
    solution is x0 / (1 + alpha_A n_H x0 t), and the counter is x0 - x."""
    g = one_cell(y_he=0.0, n_chem=64)
    a = O.rates_case_a(3000.0).a_hii
    nh, t, x0 = 1.0e-2, 3.0e13, 0.9
    x, _, rc = O.update_cell_rx(g, t, nh, [1 - x0, x0, 1, 0, 0], 3000.0, [0, 0, 0, 0], [0, 0, 0])
    assert x[1] < 0.8 * x0
    assert x[1] == pytest.approx(x0 / (1.0 + a * nh * x0 * t), rel=2e-3, abs=0)
    assert rc[0] == pytest.approx(x0 - x[1], rel=1e-9, abs=0)


def test_counters_add_to_their_start_values():
    g = one_cell(y_he=0.1)
    args = (g, 1.0e13, 1.0e-2, [0.2, 0.8, 0.1, 0.5, 0.4], 3000.0, [0, 0, 0, 0])
    _, _, a = O.update_cell_rx(*args, [0, 0, 0])
    _, _, b = O.update_cell_rx(*args, [0.25, 0.5, 1.0])
    assert np.allclose(b - np.array([0.25, 0.5, 1.0]), a, rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# Milne spectrum table (an input both implementations receive)
# --------------------------------------------------------------------------
def test_milne_rows_and_low_temperature_limit():
    b = W.blackbody_table(1.0e5)
    m = W.milne_table(b)
    assert np.allclose(m.sum(axis=2), 1.0, atol=1e-14)
    assert np.all(m >= 0.0)
    # at 10 K every photon sits within meV of its threshold: the bin holding it
    # (the first edge, 13.6 eV, sits just above the HI threshold)
    hold = [max(0, int(np.searchsorted(b.edges_ev, e, side="right") - 1)) for e in W.E_TH_EV]
    for a in range(3):
        assert m[a, 0, hold[a]] == pytest.approx(1.0, abs=1e-12)
    # nothing below an ion's own threshold
    assert np.all(m[1, :, :3] == 0.0) and np.all(m[2, :, :5] == 0.0)


def test_milne_quadrature_against_closed_form(monkeypatch):
    """With a power-law cross-section sigma ~ E^-3 the photon spectrum is
    exp(-(E-E0)/kT)/E, whose bin integrals are exponential integrals."""
    e0s = W.E_TH_EV
    monkeypatch.setattr(W, "verner_sigma", lambda a, e: (np.asarray(e) / e0s[a]) ** -3.0)
    b = W.blackbody_table(1.0e5)
    t0, per = 5.0, 4
    m = W.milne_table(b, log10_t0=t0, log10_t1=7.0, per_decade=per)
    edges = b.edges_ev
    for a in range(3):
        for k in range(m.shape[1]):
            kt = W.K_B * 10.0 ** (t0 + k / per) / W.EV_ERG
            part = []
            for j in range(len(edges) - 1):
                lo, hi = max(edges[j], e0s[a]), edges[j + 1]
                part.append(math.exp(e0s[a] / kt) * (exp1(lo / kt) - exp1(hi / kt)) if hi > lo else 0.0)
            part = np.array(part) / sum(part)
            part[part < 1e-12] = 0.0
            assert np.allclose(m[a, k], part / part.sum(), rtol=1e-8, atol=1e-13)


def test_spectrum_interpolation():
    """Linear in log10 T between the table's nodes: a node's row at a node
    temperature, the mean of two rows halfway (in log T) between them, the end
    rows beyond the table."""
    w = W.with_recombination(W.small_mixed(n=8, n_src=1, packets=10), 0.1)
    r, nb = w.recomb, w.bins.n_bins
    for ion in range(3):
        for k in (0, 17, 48, 100, r.n_t - 1):
            t = 10.0 ** (r.log10_t0 + k * r.dlog10_t)
            assert np.allclose(O.milne_at(r, nb, ion, t), r.milne[ion, k], rtol=1e-12, atol=1e-15)
        for k in (3, 47, 64):
            t = 10.0 ** (r.log10_t0 + (k + 0.5) * r.dlog10_t)
            want = 0.5 * (r.milne[ion, k] + r.milne[ion, k + 1])
            assert np.allclose(O.milne_at(r, nb, ion, t), want, rtol=1e-9, atol=1e-15)
        assert np.array_equal(O.milne_at(r, nb, ion, 1.0), r.milne[ion, 0])
        assert np.array_equal(O.milne_at(r, nb, ion, 1.0e12), r.milne[ion, -1])


def test_diffuse_direction_stream():
    """Diffuse packets draw from stream word 1 keyed by the cell index."""
    c1, _ = O.direction_ex(5, 0, 17, 3, False, 1)
    c1b, _ = O.direction_ex(5, 0, 17, 3, False, 1)
    c0, _ = O.direction_ex(5, 0, 17, 3, False, 0)
    assert np.array_equal(c1, c1b) and not np.array_equal(c1, c0)
    assert np.array_equal(c0, O.direction(5, 0, 17, 3)[0])
    u = np.array([O.direction_ex(9, 0, g, 0, False, 1)[0] for g in range(4000)], np.float64)
    u /= np.linalg.norm(u, axis=1)[:, None]
    assert np.all(np.abs(u.mean(axis=0)) < 4.0 / math.sqrt(4000))


# --------------------------------------------------------------------------
# emission: selection, ledger, physics
# --------------------------------------------------------------------------
def small_reemit(f_rec=0.05, y_he=0.0, iso=True):
    w = W.small_mixed(n=12, n_src=3, packets=3000, seed=11, fp64=True, isothermal=iso,
                      y_he=y_he, ionised_fraction=0.6)
    # long enough steps for a few per cent of the atoms to recombine
    return W.with_recombination(w.with_(dt_s=30.0 * W.MYR_S), f_rec)


@pytest.mark.parametrize("y_he", [0.0, 0.08])
def test_emitters_are_crossed_cells_over_threshold(y_he):
    """Brute force: march the source packets alone, take every cell they
    deposited in whose counter is positive and >= f_rec; the step's diffuse
    packets and photons must be exactly those."""
    w = small_reemit(f_rec=0.05, y_he=y_he)
    rng = np.random.default_rng(3)
    rc0 = np.zeros((3, w.ncell))
    ions = 3 if y_he > 0 else 1
    rc0[:ions] = rng.random((ions, w.ncell)) * 0.1
    rc0[:ions, ::7] = 0.05                                # exactly at the threshold
    s = O.OracleSolve(w)
    s.rc[:] = rc0
    ref = O.OracleSolve(w)
    acc, _, _ = ref.march(0, w.packets, dt=w.dt_s, packets=w.packets, seed=w.seed, step_index=0)
    crossed = (acc[0] > 0) | (acc[1] > 0) | (acc[2] > 0)
    assert 0 < crossed.sum() < w.ncell
    led = s.step()
    V = w.cell_cm ** 3
    atoms = np.array([w.n_h * V, y_he * w.n_h * V, y_he * w.n_h * V])
    want_n, want_ph = 0, 0.0
    for c in np.nonzero(crossed)[0]:
        p = O.ground_fraction(w.temp[c])
        hit = [(rc0[a, c] > 0 and rc0[a, c] >= 0.05) for a in range(ions)]
        if any(hit):
            want_n += 1
            want_ph += sum(rc0[a, c] * atoms[a][c] * p[a] for a in range(ions) if hit[a])
    assert want_n > 0
    assert led["diffuse_packets"] == want_n
    assert led["diffuse_emitted"] == pytest.approx(want_ph, rel=1e-12, abs=0)
    # counters after the step: emitting ions restart from zero, the others keep
    # theirs; both then add the cell update's recombinations (one sub-step, so
    # the update saw the initial state and the step's final deposits)
    g = O.make_grid(w)
    for c in range(0, w.ncell, 5):
        _, _, inc = O.update_cell_rx(g, w.dt_s, w.n_h[c], w.x[:, c], w.temp[c], s.acc[:, c], [0, 0, 0])
        hit = crossed[c] and np.any((rc0[:ions, c] > 0) & (rc0[:ions, c] >= 0.05))
        for a in range(ions):
            reset = hit and rc0[a, c] > 0 and rc0[a, c] >= 0.05
            want = inc[a] + (0.0 if reset else rc0[a, c])
            assert s.rc[a, c] == pytest.approx(want, rel=1e-12, abs=1e-300), (c, a)


def test_ledger_closes_with_diffuse_photons():
    w = small_reemit(f_rec=0.02, y_he=0.08, iso=False).with_(n_sub=3)
    s = O.OracleSolve(w)
    total = 0
    for i in range(3):
        led = s.step()
        total += led["diffuse_packets"]
        res = led["emitted"] - led["absorbed"] - led["escaped"] - led["truncated"]
        assert abs(res) <= 1e-12 * led["emitted"]
        assert led["packets"] == w.packets + led["diffuse_packets"]
    assert total > 0
    assert np.all(s.rc >= 0.0)


def test_unreachable_threshold_emits_nothing():
    w = small_reemit(f_rec=1.0e9)
    s = O.OracleSolve(w)
    led = s.step()
    assert led["diffuse_packets"] == 0 and led["diffuse_emitted"] == 0.0
    assert s.rc[0].max() > 0.0


@pytest.mark.slow
def test_reemission_recovers_the_on_the_spot_volume():
    """Case-A recombination alone shrinks an isothermal H II region well below
    the case-B (on-the-spot) one; following the ground-state recombination
    photons as packets brings it back to the case-B volume (Test 0's set-up with
    recombination radiation at a 10 % threshold, 500 Myr)."""
    vols = {}
    base = W.stromgren_reemit(packets=60000, f_rec=None)
    for name, w in [("B", base), ("A", W.with_recombination(base, 1.0e9)),
                    ("reemit", W.with_recombination(base, 0.1))]:
        s = O.OracleSolve(w)
        for _ in range(w.steps):
            s.step()
        vols[name] = float(s.x[1].sum())
    assert vols["A"] < 0.85 * vols["B"]
    assert vols["reemit"] == pytest.approx(vols["B"], rel=0.1, abs=0)
