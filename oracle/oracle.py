"""Python binding of the float64 CPU oracle (oracle/rt_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product library never imports this
module.  The C source is compiled on first use (gcc, -O2, contraction off).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

MAX_BINS = 16
FATE_TRUNC, FATE_ESCAPE, FATE_PATH = 1, 2, 3
PERIODIC = 0x2
TRACE_HDR = 8

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle shared library next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("cell_cm", C.c_double), ("y_he", C.c_double),
                ("n_bins", C.c_int32), ("e_ev", C.c_double * MAX_BINS),
                ("sigma", (C.c_double * MAX_BINS) * 3), ("redshift", C.c_double),
                ("tau_kill", C.c_double), ("n_chem", C.c_int32), ("flags", C.c_uint32),
                ("path_cells", C.c_int32)]


class Reemit(C.Structure):
    _fields_ = [("f_rec", C.c_double), ("n_t", C.c_int32), ("log10_t0", C.c_double),
                ("dlog10_t", C.c_double), ("milne", C.POINTER(C.c_double))]


class Background(C.Structure):
    _fields_ = [("ndot", C.c_double), ("sed", C.POINTER(C.c_double)), ("packets", C.c_int64)]


class Rates(C.Structure):
    _fields_ = [("a_hii", C.c_double), ("a_heii", C.c_double), ("a_heiii", C.c_double),
                ("b_hi", C.c_double), ("b_hei", C.c_double), ("b_heii", C.c_double)]


_P = C.POINTER


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            dp, ip, i64p, u64p = _P(C.c_double), _P(C.c_int32), _P(C.c_int64), _P(C.c_uint64)
            gp = _P(Grid)
            L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
            L.orc_direction.argtypes = [C.c_uint64] * 4 + [C.c_int, ip]
            L.orc_direction.restype = C.c_int
            L.orc_trace_ray.argtypes = [ip, ip, ip, C.c_int64, i64p, dp, ip]
            L.orc_trace_ray.restype = C.c_int64
            L.orc_march.argtypes = [gp, dp, C.c_int32, ip, dp, dp, C.c_uint32, C.c_double,
                                    C.c_int64, C.c_uint64, C.c_uint64, C.c_uint64,
                                    C.c_int64, C.c_int64, dp, dp, C.c_int32, C.c_int32, C.c_int32, ip]
            L.orc_rates_at.argtypes = [C.c_double, _P(Rates)]
            L.orc_cooling.argtypes = [C.c_double] * 7
            L.orc_cooling.restype = C.c_double
            L.orc_cooling_terms.argtypes = [C.c_double] * 7 + [dp]
            L.orc_compton_coeff.argtypes = [C.c_double]
            L.orc_compton_coeff.restype = C.c_double
            L.orc_update_cell_ex.argtypes = [gp, C.c_double, C.c_double, dp, dp, dp,
                                             _P(Rates), C.c_int]
            L.orc_update_cells.argtypes = [gp, C.c_double, dp, dp, dp, dp, C.c_int64, i64p]
            L.orc_absorbers.argtypes = [gp, dp, dp, dp]
            L.orc_step.argtypes = [gp, dp, dp, dp, C.c_int32, ip, dp, dp, C.c_uint32,
                                   C.c_double, C.c_int64, C.c_int32, C.c_uint64, C.c_uint64,
                                   u64p, dp, dp, dp, C.c_int32, C.c_int32, C.c_int32, ip]
            L.orc_step.restype = C.c_int
            L.orc_step_rx.argtypes = L.orc_step.argtypes + [_P(Reemit), dp, _P(Background)]
            L.orc_step_rx.restype = C.c_int
            L.orc_rates_case_a.argtypes = [C.c_double, _P(Rates)]
            L.orc_ground_fraction.argtypes = [C.c_double, dp]
            L.orc_update_cell_rx.argtypes = [gp, C.c_double, C.c_double, dp, dp, dp,
                                             _P(Rates), C.c_int, C.c_int, dp]
            L.orc_milne_at.argtypes = [_P(Reemit), C.c_int, C.c_int, C.c_double, dp]
            L.orc_hii_time.argtypes = [C.c_double] * 5
            L.orc_hii_time.restype = C.c_double
            L.orc_he_ion_time.argtypes = [dp, dp] + [C.c_double] * 5 + [dp]
            L.orc_background_packet.argtypes = [gp, _P(Background), C.c_double, C.c_int64, C.c_uint64,
                                                C.c_uint64, C.c_uint64, C.c_uint64, ip, ip]
            L.orc_background_packet.restype = C.c_double
            L.orc_direction_ex.argtypes = [C.c_uint64] * 4 + [C.c_int, C.c_uint64, ip]
            L.orc_direction_ex.restype = C.c_int
            _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray], ct):
    if a is None:
        return None
    return a.ctypes.data_as(_P(ct))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def direction(seed: int, solve_id: int, g: int, step_index: int, octant: bool = False):
    c = np.zeros(3, np.int32)
    att = lib().orc_direction(seed, solve_id, g, step_index, int(octant), _ptr(c, C.c_int32))
    return c, att


def trace_ray(n, o, c, max_len: int = 4096):
    n = np.ascontiguousarray(n, np.int32)
    o = np.ascontiguousarray(o, np.int32)
    c = np.ascontiguousarray(c, np.int32)
    cells = np.zeros(max_len, np.int64)
    s = np.zeros(max_len, np.float64)
    face = np.zeros(1, np.int32)
    cnt = lib().orc_trace_ray(_ptr(n, C.c_int32), _ptr(o, C.c_int32), _ptr(c, C.c_int32),
                              max_len, _ptr(cells, C.c_int64), _ptr(s, C.c_double),
                              _ptr(face, C.c_int32))
    m = min(cnt, max_len)
    return cells[:m].copy(), s[:m].copy(), int(face[0]), int(cnt)


def make_grid(work, flags: Optional[int] = None, n_chem: Optional[int] = None) -> Grid:
    g = Grid()
    for a in range(3):
        g.n[a] = int(work.n[a])
    g.cell_cm = float(work.cell_cm)
    g.y_he = float(work.y_he)
    nb = work.bins.n_bins
    g.n_bins = nb
    for j in range(nb):
        g.e_ev[j] = float(work.bins.e_ev[j])
        for s in range(3):
            g.sigma[s][j] = float(work.bins.sigma[s, j])
    g.redshift = float(work.redshift)
    g.tau_kill = float(work.tau_kill)
    g.n_chem = int(work.n_chem if n_chem is None else n_chem)
    g.flags = (int(work.flags if flags is None else flags) & 1) | (PERIODIC if work.periodic else 0)
    g.path_cells = int(work.path_cells or max(work.n))
    return g


def rates_at(T: float) -> Rates:
    r = Rates()
    lib().orc_rates_at(float(T), C.byref(r))
    return r


def rates_case_a(T: float) -> Rates:
    r = Rates()
    lib().orc_rates_case_a(float(T), C.byref(r))
    return r


def ground_fraction(T: float) -> np.ndarray:
    """Share of HII, HeII, HeIII recombinations that reach the ground state."""
    p = np.zeros(3)
    lib().orc_ground_fraction(float(T), _ptr(p, C.c_double))
    return p


def milne_at(recomb, nb: int, ion: int, T: float) -> np.ndarray:
    """The spectrum the oracle gives recombination photons of ion at T."""
    tab = _c64(recomb.milne).copy()
    e = Reemit(float(recomb.f_rec), int(recomb.n_t), float(recomb.log10_t0), float(recomb.dlog10_t),
               _ptr(tab, C.c_double))
    out = np.zeros(nb)
    lib().orc_milne_at(C.byref(e), int(nb), int(ion), float(T), _ptr(out, C.c_double))
    return out


def hii_time(x0: float, xh: float, I: float, R: float, h: float) -> float:
    return lib().orc_hii_time(float(x0), float(xh), float(I), float(R), float(h))


def he_ion_time(x0, xh, I1, R2, I2, R3, h) -> np.ndarray:
    a, b, out = _c64(x0), _c64(xh), np.zeros(2)
    lib().orc_he_ion_time(_ptr(a, C.c_double), _ptr(b, C.c_double), float(I1), float(R2), float(I2),
                          float(R3), float(h), _ptr(out, C.c_double))
    return out


def direction_ex(seed: int, solve_id: int, g: int, step_index: int, octant: bool, stream: int):
    c = np.zeros(3, np.int32)
    att = lib().orc_direction_ex(seed, solve_id, g, step_index, int(octant), stream, _ptr(c, C.c_int32))
    return c, att


def background_packet(grid: Grid, ndot: float, sed, dt: float, packets: int, seed: int, solve_id: int,
                      step_index: int, b: int):
    """Background packet b of a sub-step: (start point o, direction c, weight)."""
    row = _c64(sed).copy()
    bg = Background(float(ndot), _ptr(row, C.c_double), int(packets))
    o = np.zeros(3, np.int32)
    c = np.zeros(3, np.int32)
    w = lib().orc_background_packet(C.byref(grid), C.byref(bg), float(dt), int(packets), int(seed),
                                    int(solve_id), int(step_index), int(b), _ptr(o, C.c_int32),
                                    _ptr(c, C.c_int32))
    return o, c, float(w)


def update_cell_rx(grid: Grid, dt: float, nh: float, x, T: float, acc, rc,
                   fixed: Optional[Rates] = None, case_a: bool = True):
    """Advance one cell with recombination counting; returns (x[5], T, rc[3])."""
    xv = _c64(np.array(x, dtype=np.float64).copy())
    tv = np.array([T], np.float64)
    av = _c64(acc)
    rv = _c64(np.array(rc, dtype=np.float64).copy())
    lib().orc_update_cell_rx(C.byref(grid), float(dt), float(nh), _ptr(xv, C.c_double),
                             _ptr(tv, C.c_double), _ptr(av, C.c_double),
                             C.byref(fixed) if fixed is not None else None, 0, int(case_a),
                             _ptr(rv, C.c_double))
    return xv, float(tv[0]), rv


def cooling(T, ne, n_hi, n_hii, n_hei, n_heii, n_heiii) -> float:
    return lib().orc_cooling(*(float(v) for v in (T, ne, n_hi, n_hii, n_hei, n_heii, n_heiii)))


COOLING_TERMS = ("exc_hi", "exc_heii", "ci_hi", "ci_hei", "ci_heii", "rec_hii", "rec_heii", "rec_heiii",
                 "diel_heii", "brems")


def cooling_terms(T, ne, n_hi, n_hii, n_hei, n_heii, n_heiii) -> dict:
    """The cooling function's processes one by one (erg cm^-3 s^-1)."""
    out = np.zeros(10)
    lib().orc_cooling_terms(*(float(v) for v in (T, ne, n_hi, n_hii, n_hei, n_heii, n_heiii)),
                            _ptr(out, C.c_double))
    return dict(zip(COOLING_TERMS, out.tolist()))


def compton_coeff(z: float) -> float:
    return lib().orc_compton_coeff(float(z))


def update_cell(grid: Grid, dt: float, nh: float, x, T: float, acc,
                fixed: Optional[Rates] = None, no_cool: bool = False):
    """Advance one cell; returns (x[5], T)."""
    xv = _c64(np.array(x, dtype=np.float64).copy())
    tv = np.array([T], np.float64)
    av = _c64(acc)
    lib().orc_update_cell_ex(C.byref(grid), float(dt), float(nh), _ptr(xv, C.c_double),
                             _ptr(tv, C.c_double), _ptr(av, C.c_double),
                             C.byref(fixed) if fixed is not None else None, int(no_cool))
    return xv, float(tv[0])


LEDGER_KEYS = ("emitted", "absorbed", "escaped", "truncated")


def ledger_dict(led: np.ndarray) -> dict:
    d = {k: float(led[2 * i] + led[2 * i + 1]) for i, k in enumerate(LEDGER_KEYS)}
    d.update(crossings=int(led[8]), n_escaped=int(led[9]), n_truncated=int(led[10]),
             packets=int(led[11]), diffuse_emitted=float(led[12] + led[13]),
             diffuse_packets=int(led[14]))
    return d


class OracleSolve:
    """Float64 state of one solve in natural cell order, advanced by the oracle."""

    def __init__(self, work, seed: Optional[int] = None):
        self.work = work
        self.grid = make_grid(work)
        nc = work.ncell
        self.nh = _c64(work.n_h).copy()
        self.x = _c64(work.x).reshape(5, nc).copy()
        self.T = _c64(work.temp).copy()
        self.src_ijk = np.ascontiguousarray(work.src_ijk, np.int32).reshape(-1, 3)
        self.src_ndot = _c64(work.src_ndot)
        self.src_sed = _c64(work.src_sed).reshape(len(self.src_ndot), work.bins.n_bins)
        self.src_flags = int(work.src_flags)
        self.acc = np.zeros((4, nc))
        self.kappa = np.zeros((3, nc))
        self.step_index = np.zeros(1, np.uint64)
        self.seed = work.seed if seed is None else seed
        self.trace = None
        # recombination counters (per atom, HII, HeII, HeIII) and the emission inputs
        self.rc = np.zeros((3, nc))
        self._reemit = None
        if work.recomb is not None:
            r = work.recomb
            self._milne = _c64(r.milne).copy()
            self._reemit = Reemit(float(r.f_rec), int(r.n_t), float(r.log10_t0), float(r.dlog10_t),
                                  _ptr(self._milne, C.c_double))
        self._bg = None
        if getattr(work, "background", None) is not None:
            b = work.background
            self._bg_sed = _c64(b.sed).copy()
            self._bg = Background(float(b.ndot), _ptr(self._bg_sed, C.c_double), int(b.packets))

    def step(self, dt: Optional[float] = None, packets: Optional[int] = None,
             seed: Optional[int] = None, trace_n: int = 0, trace_len: int = 0,
             trace_stride: int = 1) -> dict:
        w = self.work
        dt = w.dt_s if dt is None else dt
        packets = w.packets if packets is None else packets
        seed = self.seed if seed is None else seed
        led = np.zeros(16)
        tr = np.zeros((max(trace_n, 0), TRACE_HDR + trace_len), np.int32) if trace_n else None
        rc = lib().orc_step_rx(C.byref(self.grid), _ptr(self.nh, C.c_double), _ptr(self.x, C.c_double),
                               _ptr(self.T, C.c_double), len(self.src_ndot),
                               _ptr(self.src_ijk, C.c_int32), _ptr(self.src_ndot, C.c_double),
                               _ptr(self.src_sed, C.c_double), self.src_flags, float(dt),
                               int(packets), int(w.n_sub), int(seed), int(w.solve_id),
                               _ptr(self.step_index, C.c_uint64), _ptr(self.acc, C.c_double),
                               _ptr(self.kappa, C.c_double), _ptr(led, C.c_double),
                               int(trace_n), int(trace_len), int(trace_stride), _ptr(tr, C.c_int32),
                               C.byref(self._reemit) if self._reemit is not None else None,
                               _ptr(self.rc, C.c_double),
                               C.byref(self._bg) if self._bg is not None else None)
        if rc != 0:
            raise ValueError("oracle step rejected: fewer packets than sources in a sub-step")
        self.trace = tr
        return ledger_dict(led)

    def absorbers(self) -> np.ndarray:
        lib().orc_absorbers(C.byref(self.grid), _ptr(self.nh, C.c_double),
                            _ptr(self.x, C.c_double), _ptr(self.kappa, C.c_double))
        return self.kappa

    def march(self, g_begin: int, g_end: int, *, dt: float, packets: int, seed: int,
              step_index: int, trace_n: int = 0, trace_len: int = 0, trace_stride: int = 1,
              acc=None, absorbers: bool = True):
        """March packet ids [g_begin, g_end) of one sub-step over the current
        frozen state (absorbers recomputed unless absorbers=False); returns
        (acc, ledger, trace)."""
        if absorbers:
            self.absorbers()
        acc = np.zeros((4, self.work.ncell)) if acc is None else acc
        led = np.zeros(16)
        tr = np.zeros((max(trace_n, 0), TRACE_HDR + trace_len), np.int32) if trace_n else None
        lib().orc_march(C.byref(self.grid), _ptr(self.kappa, C.c_double), len(self.src_ndot),
                        _ptr(self.src_ijk, C.c_int32), _ptr(self.src_ndot, C.c_double),
                        _ptr(self.src_sed, C.c_double), self.src_flags, float(dt), int(packets),
                        int(seed), int(self.work.solve_id), int(step_index), int(g_begin),
                        int(g_end), _ptr(acc, C.c_double), _ptr(led, C.c_double),
                        int(trace_n), int(trace_len), int(trace_stride), _ptr(tr, C.c_int32))
        return acc, ledger_dict(led), tr

    def update_cells(self, dt: float, acc: np.ndarray, idx: Optional[np.ndarray] = None):
        """Apply the cell update to the cells in idx (all when None) in place."""
        acc = _c64(acc)
        if idx is None:
            lib().orc_update_cells(C.byref(self.grid), float(dt), _ptr(self.nh, C.c_double),
                                   _ptr(self.x, C.c_double), _ptr(self.T, C.c_double),
                                   _ptr(acc, C.c_double), self.work.ncell, None)
        else:
            ix = np.ascontiguousarray(idx, np.int64)
            lib().orc_update_cells(C.byref(self.grid), float(dt), _ptr(self.nh, C.c_double),
                                   _ptr(self.x, C.c_double), _ptr(self.T, C.c_double),
                                   _ptr(acc, C.c_double), len(ix), _ptr(ix, C.c_int64))
