"""Seeded synthetic inputs for the Monte-Carlo radiative-transfer hot path.

This module builds *inputs only*: grids, gas fields, source lists, per-bin
spectral tables and run parameters.  It holds none of the method's own
arithmetic (no emission, traversal, attenuation, deposition or cell update);
both the HIP library and the CPU oracle consume what it returns.

Shapes follow the paper's workloads (Partl et al. 2011):

* a pure-hydrogen isothermal Stroemgren sphere, the convergence test of
  Sec. 4.1 (Test 0, itself the first test of the Iliev et al. 2006 comparison);
* multiple black-body sources in a z~9 cosmological field with H+He and
  photo-heating (Sec. 4.2.4, Test 4; Sec. 4.5, the thousand-source 512^3 run).

The cosmological density snapshots the paper uses are not available, so the
gas is a seeded lognormal field with a power-law spectrum and the sources sit
in its densest cells (stand-ins with the same grid sizes, mean density,
clustering and source counts).

All floating-point state values are rounded to float32-representable numbers
so that the float32-state form of the GPU path and the float64 oracle start
from bit-identical fields.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# ----------------------------------------------------------------------------
# Physical constants (cgs).  1 eV and k_B are the exact SI-derived values.
# ----------------------------------------------------------------------------
EV_ERG = 1.602176634e-12
K_B = 1.380649e-16
KPC_CM = 3.0856775814913673e21
MPC_CM = 1.0e3 * KPC_CM
YR_S = 3.15576e7
MYR_S = 1.0e6 * YR_S
HUBBLE_H = 0.7            # the paper assumes h = 0.7 throughout (Sec. 1)
# Ionisation thresholds of HI, HeI, HeII (eV).
E_TH_EV = (13.598434, 24.587387, 54.417760)

MAX_BINS = 16

# Field-array order of the ionisation fractions (five per cell).
X_HI, X_HII, X_HEI, X_HEII, X_HEIII = range(5)


# ----------------------------------------------------------------------------
# Photo-ionisation cross-sections: analytic fits of Verner et al. (1996).
# The paper only states that the cell optical depth sums the HI, HeI and HeII
# contributions (Sec. 2); it gives no cross-sections, so this published fit is
# used to build the per-bin tables handed to both implementations.
# ----------------------------------------------------------------------------
# (E0 [eV], sigma0 [Mb], ya, P, yw, y0, y1)
_VERNER = {
    0: (0.4298, 5.475e4, 32.88, 2.963, 0.0, 0.0, 0.0),        # HI
    1: (13.61, 9.492e2, 1.469, 3.188, 2.039, 0.4434, 2.136),  # HeI
    2: (1.720, 1.369e4, 32.88, 2.963, 0.0, 0.0, 0.0),         # HeII
}


def verner_sigma(species: int, e_ev):
    """Photo-ionisation cross-section [cm^2] of species 0=HI, 1=HeI, 2=HeII."""
    e0, s0, ya, p, yw, y0, y1 = _VERNER[species]
    e = np.asarray(e_ev, dtype=np.float64)
    x = e / e0 - y0
    y = np.sqrt(x * x + y1 * y1)
    f = ((x - 1.0) ** 2 + yw * yw) * y ** (0.5 * p - 5.5) * (1.0 + np.sqrt(y / ya)) ** (-p)
    sig = s0 * f * 1.0e-18
    return np.where(e >= E_TH_EV[species], sig, 0.0)


@dataclasses.dataclass
class BinTable:
    """Per-frequency-bin inputs: photon energy, cross-sections and SED."""
    e_ev: np.ndarray          # (nb,) representative photon energy of each bin
    sigma: np.ndarray         # (3, nb) HI, HeI, HeII cross-section [cm^2]
    sed: np.ndarray           # (nb,) fraction of emitted photons in each bin
    edges_ev: Optional[np.ndarray] = None

    @property
    def n_bins(self) -> int:
        return int(self.e_ev.shape[0])


def monochromatic_table(e_ev: float = 13.6) -> BinTable:
    """One bin at energy e_ev (cross-sections taken at that energy)."""
    sig = np.array([[float(verner_sigma(s, e_ev))] for s in range(3)])
    return BinTable(np.array([e_ev]), sig, np.array([1.0]))


def blackbody_edges(lo=13.6, hi=200.0):
    """Nine bin edges over [lo, hi] eV: 3 log-spaced bins below the HeI
    threshold, 2 between the HeI and HeII thresholds, 3 above."""
    e1, e2 = E_TH_EV[1], E_TH_EV[2]
    a = np.geomspace(lo, e1, 4)
    b = np.geomspace(e1, e2, 3)
    c = np.geomspace(e2, hi, 4)
    return np.concatenate([a[:-1], b[:-1], c])


def blackbody_table(t_bb: float = 1.0e5, edges_ev=None) -> BinTable:
    """Photon-number weighted bin table for a black body of temperature t_bb.

    Photon spectrum dN/dE ~ E^2 / (exp(E/kT) - 1).  SED_j is the photon
    fraction in bin j renormalised over the covered range, E_j the
    photon-weighted mean energy and sigma_{s,j} the photon-weighted mean
    cross-section (adaptive quadrature, float64).
    """
    from scipy.integrate import quad

    if edges_ev is None:
        edges_ev = blackbody_edges()
    edges_ev = np.asarray(edges_ev, dtype=np.float64)
    kt = K_B * t_bb / EV_ERG

    def nph(e):
        return e * e / math.expm1(e / kt)

    nb = len(edges_ev) - 1
    n = np.zeros(nb)
    en = np.zeros(nb)
    sg = np.zeros((3, nb))
    for j in range(nb):
        lo, hi = float(edges_ev[j]), float(edges_ev[j + 1])
        kw = dict(epsabs=0.0, epsrel=1e-12, limit=200)
        n[j] = quad(nph, lo, hi, **kw)[0]
        en[j] = quad(lambda e: e * nph(e), lo, hi, **kw)[0]
        for s in range(3):
            # split at the threshold so the quadrature never straddles the edge
            pts = [E_TH_EV[s]] if lo < E_TH_EV[s] < hi else None
            sg[s, j] = quad(lambda e: float(verner_sigma(s, e)) * nph(e), lo, hi,
                            points=pts, **kw)[0]
    sed = n / n.sum()
    return BinTable(en / n, sg / n, sed, edges_ev)


# ----------------------------------------------------------------------------
# Gas fields
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class RecombEmission:
    """Inputs of recombination re-emission: the threshold and the per-bin
    spectra of the ground-state recombination photons of HII, HeII and HeIII
    on a grid of temperatures (node m at log10 T = log10_t0 + m dlog10_t)."""
    f_rec: float
    log10_t0: float
    dlog10_t: float
    milne: np.ndarray         # (3, n_t, nb) photon fraction per bin; rows sum to 1

    @property
    def n_t(self) -> int:
        return int(self.milne.shape[1])


def milne_table(bins: BinTable, log10_t0: float = 1.0, log10_t1: float = 9.0,
                per_decade: int = 16) -> np.ndarray:
    """Photon fractions per bin of the recombination continuum to the ground
    state of HI, HeI and HeII (from HII, HeII, HeIII) at each temperature node.

    Milne relation (detailed balance with photo-ionisation): the photon-number
    spectrum above the threshold E0 is dN/dE ~ E^2 sigma(E) exp(-(E - E0)/kT),
    sigma the Verner fit of the recombined species.  Fractions are taken over
    the bins' covered range [E0, last edge] (adaptive quadrature in
    x = (E - E0)/kT, float64); fractions below 1e-12 are set to zero and the
    rest renormalised.  A table without edges (one bin) sends every photon to
    that bin."""
    from scipy.integrate import quad

    nt = int(round((log10_t1 - log10_t0) * per_decade)) + 1
    nb = bins.n_bins
    out = np.zeros((3, nt, nb))
    if bins.edges_ev is None:
        if nb != 1:
            raise ValueError("a multi-bin table needs bin edges")
        out[:] = 1.0
        return out
    edges = np.asarray(bins.edges_ev, np.float64)
    top = float(edges[-1])
    for a in range(3):
        e0 = E_TH_EV[a]
        for m in range(nt):
            kt = K_B * 10.0 ** (log10_t0 + m / per_decade) / EV_ERG

            def f(x):
                e = e0 + kt * x
                return e * e * float(verner_sigma(a, e)) * math.exp(-x)

            part = np.zeros(nb)
            for j in range(nb):
                lo, hi = max(float(edges[j]), e0), min(float(edges[j + 1]), top)
                if hi <= lo:
                    continue
                xlo, xhi = (lo - e0) / kt, min((hi - e0) / kt, 800.0)
                if xhi <= xlo:
                    continue
                part[j] = quad(f, xlo, xhi, epsabs=0.0, epsrel=1e-12, limit=400)[0]
            tot = part.sum()
            if tot > 0.0:
                part = part / tot
                part[part < 1e-12] = 0.0          # photons that cannot matter: no bin kept alive for them
                out[a, m] = part / part.sum()
    return out


def with_recombination(w: "Workload", f_rec: float = 0.1) -> "Workload":
    """The same workload with recombination photons re-emitted as packets."""
    t0, per = 1.0, 16
    return w.with_(recomb=RecombEmission(float(f_rec), t0, 1.0 / per, milne_table(w.bins, t0, 9.0, per)))


def lognormal_field(n: int, sigma_ln: float, mean: float, seed: int) -> np.ndarray:
    """Seeded lognormal density, natural order (i fastest), float64 values
    that are exactly float32-representable.

    White noise -> FFT -> amplitude * k^-1 (power spectrum ~ k^-2), zero mean
    mode -> inverse FFT -> unit variance g -> mean * exp(sigma g)/<exp(sigma g)>.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    k0 = np.fft.fftfreq(n) * n
    k2 = np.fft.rfftfreq(n) * n
    kk = np.sqrt(k0[:, None, None] ** 2 + k0[None, :, None] ** 2 + k2[None, None, :] ** 2)
    kk[0, 0, 0] = 1.0
    fk /= kk
    fk[0, 0, 0] = 0.0
    g = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    rho = np.exp(sigma_ln * g)
    rho *= mean / rho.mean()
    return rho.astype(np.float32).astype(np.float64).reshape(-1)


def powerlaw_luminosities(count: int, lmin: float, lmax: float, rng) -> np.ndarray:
    """Luminosities with dN/dL ~ L^-2 on [lmin, lmax] by inverse CDF."""
    u = rng.random(count)
    return 1.0 / (1.0 / lmin - u * (1.0 / lmin - 1.0 / lmax))


def cells_to_ijk(cells, n: Sequence[int]) -> np.ndarray:
    cells = np.asarray(cells, dtype=np.int64)
    i = cells % n[0]
    j = (cells // n[0]) % n[1]
    k = cells // (n[0] * n[1])
    return np.stack([i, j, k], axis=1).astype(np.int32)


# ----------------------------------------------------------------------------
# Workload description consumed by both implementations
# ----------------------------------------------------------------------------
ISOTHERMAL = 0x1
FP64_MARCH = 0x2
SRC_CORNER_OCTANT = 0x1


@dataclasses.dataclass
class Background:
    """An isotropic background field entering the box through its faces:
    photons per second through the whole boundary, their spectrum over the
    bins, and packets per step."""
    ndot: float
    sed: np.ndarray
    packets: int


def background_rate(j_photons: float, n: Sequence[int], cell_cm: float) -> float:
    """Photons per second entering a box through all six faces from an
    isotropic intensity j_photons [photons s^-1 cm^-2 sr^-1]: the inward flux
    through a surface is pi j, times the boundary area."""
    area = 2.0 * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1]) * cell_cm * cell_cm
    return math.pi * j_photons * area


@dataclasses.dataclass
class Workload:
    name: str
    n: tuple                    # cells per axis
    cell_cm: float              # proper cell size
    y_he: float                 # n_He / n_H (0 -> pure hydrogen)
    bins: BinTable
    redshift: float             # < 0 disables Compton coupling
    n_h: np.ndarray             # (ncell,) hydrogen number density, natural order
    x: np.ndarray               # (5, ncell) x_HI, x_HII, x_HeI, x_HeII, x_HeIII
    temp: np.ndarray            # (ncell,) temperature [K]
    src_ijk: np.ndarray         # (S, 3) int32 cell of each source
    src_ndot: np.ndarray        # (S,) photons / s
    src_sed: np.ndarray         # (S, nb) photon fraction per bin (rows sum to 1)
    src_flags: int = 0          # SRC_CORNER_OCTANT for a corner source
    dt_s: float = MYR_S         # duration of one step
    packets: int = 100000       # packets per step
    steps: int = 1
    n_sub: int = 1              # frozen sub-steps per step
    n_chem: int = 8             # fixed chemistry sub-steps per frozen sub-step
    tau_kill: float = 30.0
    flags: int = 0
    seed: int = 1
    solve_id: int = 0
    recomb: Optional[RecombEmission] = None   # recombination re-emission (None: off)
    periodic: bool = False      # periodic boundaries (packets re-enter through the opposite face)
    path_cells: int = 0         # periodic: faces a packet may cross along one axis (0: the longest side)
    background: Optional[Background] = None   # background field through the faces (None: none)

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _neutral_state(ncell: int, t0: float):
    x = np.zeros((5, ncell))
    x[X_HI] = 1.0
    x[X_HEI] = 1.0
    return x, np.full(ncell, float(np.float32(t0)))


def stromgren_c1(n: int = 32, packets: int = 100000, steps: int = 10, n_sub: int = 100,
                 fp64: bool = True) -> Workload:
    """Plain method: 32^3, box 6.6 kpc, uniform pure H n_H=1e-3, T=1e4 K
    (isothermal), x_HI=1, one monochromatic 13.6 eV source of 5e48 ph/s at the
    grid corner, 1e5 packets per 1 Myr step, 10 steps."""
    box = 6.6 * KPC_CM
    ncell = n ** 3
    x, t = _neutral_state(ncell, 1.0e4)
    bins = monochromatic_table(13.6)
    return Workload(
        name=f"stromgren_{n}^3", n=(n, n, n), cell_cm=box / n, y_he=0.0, bins=bins,
        redshift=-1.0, n_h=np.full(ncell, 1.0e-3), x=x, temp=t,
        src_ijk=np.zeros((1, 3), np.int32), src_ndot=np.array([5.0e48]),
        src_sed=np.ones((1, 1)), src_flags=SRC_CORNER_OCTANT,
        dt_s=MYR_S, packets=packets, steps=steps, n_sub=n_sub, n_chem=8,
        flags=ISOTHERMAL | (FP64_MARCH if fp64 else 0), seed=1)


def thermal_test2(n: int = 32, packets: int = 100000, steps: int = 5, n_sub: int = 50,
                  fp64: bool = False, box_kpc: float = 15.0) -> Workload:
    """The thermal H II region of Sec. 4.2 (Test 2): Test 0's set-up (uniform
    pure H, n_H = 1e-3, one corner source of 5e48 ph/s) with a 1e5 K black body
    in 8 bins, the gas initially neutral at 100 K and its temperature followed;
    box 15 kpc (the comparison project's box; the paper only says larger),
    10 Myr steps."""
    box = box_kpc * KPC_CM
    ncell = n ** 3
    x, t = _neutral_state(ncell, 100.0)
    bins = blackbody_table(1.0e5)
    return Workload(
        name=f"thermal_test2_{n}^3", n=(n, n, n), cell_cm=box / n, y_he=0.0, bins=bins,
        redshift=-1.0, n_h=np.full(ncell, float(np.float32(1.0e-3))), x=x, temp=t,
        src_ijk=np.zeros((1, 3), np.int32), src_ndot=np.array([5.0e48]),
        src_sed=bins.sed[None, :].copy(), src_flags=SRC_CORNER_OCTANT,
        dt_s=10.0 * MYR_S, packets=packets, steps=steps, n_sub=n_sub, n_chem=8,
        flags=(FP64_MARCH if fp64 else 0), seed=1)


def stromgren_reemit(n: int = 32, packets: int = 100000, steps: int = 10, n_sub: int = 10,
                     f_rec: Optional[float] = 0.1, fp64: bool = True, box_kpc: float = 17.3) -> Workload:
    """Test 0's gas (uniform pure H, n_H = 1e-3, isothermal 1e4 K, initially
    neutral) around one 5e48 ph/s source with a 1e5 K black-body spectrum in 8
    bins, with recombination photons re-emitted at threshold f_rec (Sec. 4.1
    uses 10 %).  The source sits at the centre cell of the box (not a corner),
    so diffuse photons are not lost through symmetry planes; the box (17.3 kpc
    on 32 cells) puts the case-B Stroemgren radius near 10 cells.  50 Myr steps,
    10 steps = 500 Myr (Test 0's simulated time, about four recombination
    times).  f_rec None: case-B rates and no re-emission."""
    box = box_kpc * KPC_CM
    ncell = n ** 3
    x, t = _neutral_state(ncell, 1.0e4)
    bins = blackbody_table(1.0e5)
    w = Workload(
        name=f"stromgren_reemit_{n}^3", n=(n, n, n), cell_cm=box / n, y_he=0.0, bins=bins,
        redshift=-1.0, n_h=np.full(ncell, 1.0e-3), x=x, temp=t,
        src_ijk=np.full((1, 3), n // 2, np.int32), src_ndot=np.array([5.0e48]),
        src_sed=bins.sed[None, :].copy(), src_flags=0,
        dt_s=50.0 * MYR_S, packets=packets, steps=steps, n_sub=n_sub, n_chem=8,
        flags=ISOTHERMAL | (FP64_MARCH if fp64 else 0), seed=1)
    return w if f_rec is None else with_recombination(w, f_rec)


def hii_region_reemit(n: int = 256, packets: int = 10_000_000, f_rec: float = 0.1, seed: int = 21,
                      fp64: bool = False):
    """An established H II region with recombination radiation, for measuring
    re-emission at scale: Test 0's gas (uniform pure H, n_H = 1e-3, isothermal
    1e4 K) around one central 5e48 ph/s source with a 1e5 K black body in 8
    bins; the box (18 kpc) puts the case-B Stroemgren radius at 0.3 n cells.
    Cells inside that radius start ionised (x_HI = 1e-3) with recombination
    counters drawn uniformly in [0, 2 f_rec) (seeded), so about half of them
    emit in the first sub-step; outside, the gas is neutral with zero counters.
    Returns (workload, counters [1][ncell])."""
    box = 18.0 * KPC_CM
    ncell = n ** 3
    x, t = _neutral_state(ncell, 1.0e4)
    c = (np.arange(n) + 0.5 - n / 2.0)
    r2 = (c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2).transpose(2, 1, 0).ravel()
    inside = r2 < (0.3 * n) ** 2
    x[X_HI, inside] = float(np.float32(1.0e-3))
    x[X_HII, inside] = float(np.float32(1.0 - 1.0e-3))
    rng = np.random.default_rng(seed)
    counters = np.zeros((1, ncell))
    counters[0, inside] = rng.random(int(inside.sum())) * (2.0 * f_rec)
    bins = blackbody_table(1.0e5)
    w = Workload(
        name=f"hii_region_reemit_{n}^3", n=(n, n, n), cell_cm=box / n, y_he=0.0, bins=bins,
        redshift=-1.0, n_h=np.full(ncell, float(np.float32(1.0e-3))), x=x, temp=t,
        src_ijk=np.full((1, 3), n // 2, np.int32), src_ndot=np.array([5.0e48]),
        src_sed=bins.sed[None, :].copy(), src_flags=0, dt_s=MYR_S, packets=packets, steps=2, n_sub=1,
        n_chem=8, flags=ISOTHERMAL | (FP64_MARCH if fp64 else 0), seed=1)
    return with_recombination(w, f_rec), counters


def blackbody_photon_rate(luminosity_erg_s: float, t_bb: float, lo_ev: float = 13.6,
                          hi_ev: float = 200.0) -> float:
    """Photons/s in [lo_ev, hi_ev] of a black body of total luminosity L."""
    from scipy.integrate import quad
    kt = K_B * t_bb / EV_ERG
    energy = quad(lambda e: e ** 3 / math.expm1(e / kt), 1e-8 * kt, 60.0 * kt, epsabs=0.0, epsrel=1e-12,
                  limit=400)[0]
    photons = quad(lambda e: e * e / math.expm1(e / kt), lo_ev, hi_ev, epsabs=0.0, epsrel=1e-12,
                   limit=400)[0]
    return luminosity_erg_s / EV_ERG * photons / energy


def hhe_test3(n: int = 32, packets: int = 200000, steps: int = 6, n_sub: int = 50,
              fp64: bool = False) -> Workload:
    """The H+He H II region of Sec. 4.2 (Test 3, the CLOUDY94 comparison): a
    6e4 K black body of 1e38 erg/s (its photons in 13.6-200 eV, 8 bins) in a
    uniform medium of 1 particle/cm^3, 90 % hydrogen by number (n_H = 0.9,
    y = 1/9), initially neutral at 100 K, temperature followed; box 128 pc with
    the source at its corner (the paper does not place it); 6e5 yr in steps of
    1e5 yr."""
    box = 128.0e-3 * KPC_CM
    ncell = n ** 3
    x, t = _neutral_state(ncell, 100.0)
    bins = blackbody_table(6.0e4)
    ndot = blackbody_photon_rate(1.0e38, 6.0e4)
    return Workload(
        name=f"hhe_test3_{n}^3", n=(n, n, n), cell_cm=box / n, y_he=1.0 / 9.0, bins=bins,
        redshift=-1.0, n_h=np.full(ncell, float(np.float32(0.9))), x=x, temp=t,
        src_ijk=np.zeros((1, 3), np.int32), src_ndot=np.array([ndot]),
        src_sed=bins.sed[None, :].copy(), src_flags=SRC_CORNER_OCTANT,
        dt_s=1.0e5 * YR_S, packets=packets, steps=steps, n_sub=n_sub, n_chem=8,
        flags=(FP64_MARCH if fp64 else 0), seed=1)


def cosmo_cell_cm(n: int, box_mpc_h: float = 10.0, z: float = 9.0) -> float:
    """Proper cell size of an n^3 grid on a comoving box of box_mpc_h Mpc/h."""
    return box_mpc_h / HUBBLE_H * MPC_CM / (1.0 + z) / n


def cosmological(n: int, n_src: int, packets: int, *, sigma_ln: float = 1.0,
                 mean_nh: float = 2.0e-4, field_seed: int = 2, src_seed: int = 3,
                 top_fraction: Optional[float] = None, steps: int = 1,
                 dt_s: float = 1.0e4 * YR_S, fp64: bool = False,
                 name: Optional[str] = None) -> Workload:
    """Lognormal H+He gas (X=0.76, Y=0.24) at z=9 on a 10 Mpc/h box, T0=100 K,
    fully neutral, n_src 1e5 K black-body sources with L ~ L^-2 on
    [1e50, 1e53] ph/s, 8 frequency bins.  Sources sit at cell centres drawn
    uniformly without replacement, either over the whole grid or over the
    densest `top_fraction` of cells."""
    z = 9.0
    ncell = n ** 3
    nh = lognormal_field(n, sigma_ln, mean_nh, field_seed)
    rng = np.random.default_rng(src_seed)
    if top_fraction is None:
        cells = rng.choice(ncell, size=n_src, replace=False)
    else:
        ntop = max(n_src, int(round(top_fraction * ncell)))
        top = np.argpartition(nh, ncell - ntop)[ncell - ntop:]
        top.sort()
        cells = rng.choice(top, size=n_src, replace=False)
    lum = powerlaw_luminosities(n_src, 1.0e50, 1.0e53, rng)
    bins = blackbody_table(1.0e5)
    x, t = _neutral_state(ncell, 100.0)
    return Workload(
        name=name or f"lognormal_{n}^3_{n_src}src", n=(n, n, n),
        cell_cm=cosmo_cell_cm(n), y_he=0.24 / (4.0 * 0.76), bins=bins, redshift=z,
        n_h=nh, x=x, temp=t, src_ijk=cells_to_ijk(cells, (n, n, n)), src_ndot=lum,
        src_sed=np.tile(bins.sed, (n_src, 1)), dt_s=dt_s, packets=packets,
        steps=steps, n_sub=1, n_chem=8, flags=(FP64_MARCH if fp64 else 0), seed=1)


def lognormal_128(fp64: bool = False, packets: int = 10_000_000) -> Workload:
    """128^3, 100 sources anywhere, 1e7 packets per step."""
    return cosmological(128, 100, packets, steps=10, fp64=fp64, name="lognormal_128^3_100src")


def lognormal_256(fp64: bool = False, packets: int = 100_000_000) -> Workload:
    """256^3, 1e4 sources in the densest 1 % of cells, 1e8 packets per step."""
    return cosmological(256, 10_000, packets, top_fraction=0.01, steps=20, fp64=fp64,
                        name="lognormal_256^3_1e4src")


def lognormal_512(fp64: bool = False, packets: int = 500_000_000) -> Workload:
    """512^3, sigma_ln=1.5, 1e5 sources in the densest 1 % of cells."""
    return cosmological(512, 100_000, packets, sigma_ln=1.5, field_seed=5, src_seed=6,
                        top_fraction=0.01, steps=2, fp64=fp64,
                        name="lognormal_512^3_1e5src")


def small_mixed(n: int = 24, n_src: int = 5, packets: int = 20000, seed: int = 7,
                fp64: bool = True, isothermal: bool = False, y_he: Optional[float] = None,
                ionised_fraction: float = 0.0) -> Workload:
    """A small H+He lognormal case with black-body sources for parity tests
    (not a multiple of the brick size, several sources, 8 bins)."""
    w = cosmological(n, n_src, packets, sigma_ln=1.0, field_seed=seed,
                     src_seed=seed + 1, fp64=fp64, name=f"small_{n}^3")
    w = w.with_(cell_cm=w.cell_cm * 128.0 / n)   # keep optical depths per cell moderate
    if y_he is not None:
        w = w.with_(y_he=y_he)
    if isothermal:
        w = w.with_(flags=w.flags | ISOTHERMAL)
    if ionised_fraction > 0.0:
        rng = np.random.default_rng(seed + 2)
        xi = (rng.random(w.ncell) * ionised_fraction).astype(np.float32).astype(np.float64)
        x = w.x.copy()
        x[X_HII] = xi
        x[X_HI] = (1.0 - xi).astype(np.float32).astype(np.float64)
        x[X_HEII] = (0.5 * xi).astype(np.float32).astype(np.float64)
        x[X_HEIII] = (0.1 * xi).astype(np.float32).astype(np.float64)
        x[X_HEI] = (1.0 - x[X_HEII] - x[X_HEIII]).astype(np.float32).astype(np.float64)
        t = (100.0 + 2.0e4 * xi).astype(np.float32).astype(np.float64)
        w = w.with_(x=x, temp=t)
    return w


# ----------------------------------------------------------------------------
# Serving stream: independent small solves arriving as a Poisson process
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    work: Workload


def serving_stream(count: int = 512, rate_per_s: float = 200.0, seed: int = 4,
                   steps: int = 5, n_sub: int = 10, sides=(16, 24, 32, 48, 64),
                   log_packets=(4.0, 6.0), max_sources: int = 16) -> List[Request]:
    """Independent pure-H isothermal solves with uneven sizes: side from
    {16,24,32,48,64}, uniform or lognormal gas (50/50), 1-16 monochromatic
    13.6 eV sources of 5e48 ph/s at cell centres, 1e4-1e6 packets per step
    (log-uniform), 5 steps of 1 Myr; cell size as in the Stroemgren case.
    Arrivals are a Poisson process of the given mean rate."""
    rng = np.random.default_rng(seed)
    sides = tuple(sides)
    bins = monochromatic_table(13.6)
    dl = 6.6 * KPC_CM / 32
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(rng.choice(sides))
        ncell = n ** 3
        if rng.random() < 0.5:
            nh = np.full(ncell, 1.0e-3)
        else:
            nh = lognormal_field(n, 1.0, 1.0e-3, int(rng.integers(1 << 31)))
        n_src = int(rng.integers(1, max_sources + 1))
        cells = rng.choice(ncell, size=n_src, replace=False)
        packets = int(round(10.0 ** rng.uniform(*log_packets)))
        packets = max(packets - packets % n_sub, n_sub * n_src)
        x, temp = _neutral_state(ncell, 1.0e4)
        w = Workload(
            name=f"req{rid}_{n}^3", n=(n, n, n), cell_cm=dl, y_he=0.0, bins=bins,
            redshift=-1.0, n_h=nh, x=x, temp=temp, src_ijk=cells_to_ijk(cells, (n, n, n)),
            src_ndot=np.full(n_src, 5.0e48), src_sed=np.ones((n_src, 1)),
            dt_s=MYR_S, packets=packets, steps=steps, n_sub=n_sub, n_chem=8,
            flags=ISOTHERMAL, seed=1, solve_id=rid)
        out.append(Request(rid, t, w))
    return out
