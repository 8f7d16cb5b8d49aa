"""Helpers shared by the GPU parity tests: run one workload through the HIP
library and through the oracle on identical seeded inputs and compare."""
import math

import numpy as np

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W

# error measures (deposits relative to max(|ref|, 1e-12 * mean); fractions
# relative to max(ref, 1e-8); temperature relative)
def deposit_err(g, o, allow=0.0):
    """|g - o| relative to max(|o|, 1e-12 * mean |o|), after subtracting an
    absolute allowance (photons the compared form may legitimately move, e.g.
    the e^-30 remainders the float32 form drops)."""
    mean = float(np.mean(np.abs(o)))
    floor = 1e-12 * mean if mean > 0 else 1e-300
    return np.maximum(np.abs(g - o) - allow, 0.0) / np.maximum(np.abs(o), floor)


def frac_err(g, o, floor=1e-8):
    return np.abs(g - o) / np.maximum(o, floor)


def temp_err(g, o):
    return np.abs(g - o) / o


def run_both(work, *, fp64, steps=1, trace_n=0, trace_len=0, stride=1, seeds=None, **tiles):
    from paper_1101_4127_amd import rt
    s = rt.Solve(work, fp64=fp64, trace_packets=trace_n, trace_len=trace_len, trace_stride=stride,
                 **tiles)
    o = O.OracleSolve(work)
    stats = []
    for k in range(steps):
        seed = work.seed if seeds is None else seeds[k]
        gst = s.step(seed=seed)
        ost = o.step(seed=seed, trace_n=trace_n, trace_len=trace_len, trace_stride=stride)
        stats.append((gst, ost))
    fields = s.fetch()
    trace = s.trace() if trace_n else None
    s.release()
    return o, stats, fields, trace


def compare_state(o, fields, work, *, frac_tol, temp_tol, dep_tol, frac_floor=1e-8, dep_allow=0.0,
                  heat_allow=0.0):
    """Per-field maximum errors; asserts them against the tolerances.
    dep_allow / heat_allow: absolute allowances on the deposits (photons) and
    the heat (erg)."""
    rep = {}
    iso = bool(work.flags & W.ISOTHERMAL)
    for f in range(5):
        rep[f"x{f}"] = float(np.max(frac_err(fields[1 + f], o.x[f], frac_floor)))
    rep["T"] = float(np.max(temp_err(fields[6], o.T)))
    for f in range(3):
        rep[f"D{f}"] = float(np.max(deposit_err(fields[7 + f], o.acc[f], dep_allow)))
    rep["Q"] = 0.0 if iso else float(np.max(deposit_err(fields[10], o.acc[3], heat_allow)))
    assert np.array_equal(fields[0], o.nh)
    for k, v in rep.items():
        tol = frac_tol if k.startswith("x") else (temp_tol if k == "T" else dep_tol)
        assert v <= tol, (k, v, rep)
    return rep


def ledger_close(g, o, tol):
    e = o["emitted"]
    assert abs(g["emitted"] - e) <= 1e-13 * e
    for k in ("absorbed", "escaped", "truncated"):
        assert abs(g[k] - o[k]) <= tol * e, (k, g[k], o[k])
    resid = g["emitted"] - (g["absorbed"] + g["escaped"] + g["truncated"])
    return abs(resid) / e


def trace_cells(rec):
    n = min(int(rec[0]), len(rec) - 8)
    return rec[8:8 + n]


def traces_equal(a, b):
    """Records equal in their defined part (slots past the count are unspecified)."""
    if a.shape != b.shape:
        return False
    return all(np.array_equal(x[:8], y[:8]) and np.array_equal(trace_cells(x), trace_cells(y))
               for x, y in zip(a, b))


def source_origin(work, src):
    ijk = np.asarray(work.src_ijk[src], dtype=np.int64)
    return 2 * ijk if work.src_flags & W.SRC_CORNER_OCTANT else 2 * ijk + 1


def tmin_profile(work, kappa, rec):
    """Oracle-precision min_j (accumulated tau_j) after each crossed cell."""
    src = int(rec[7])
    c = rec[4:7].astype(np.int64)
    cells, s, face, cnt = O.trace_ray(work.n, source_origin(work, src), c, max_len=1 << 14)
    L = math.sqrt(float((c * c).sum())) * (0.5 * work.cell_cm)
    l = np.diff(np.concatenate([[0.0], s])) * L
    sed = np.asarray(work.src_sed[src])
    sig = work.bins.sigma
    k = kappa[:, cells]                       # (3, ncross)
    K = (k[0][:, None] * sig[0][None, :] + k[1][:, None] * sig[1][None, :]) + k[2][:, None] * sig[2][None, :]
    T = np.cumsum(l[:, None] * K, axis=0)
    T[:, sed <= 0] = np.inf
    return T.min(axis=1)


def compare_traces(work, kappa, g_tr, o_tr, exact, guard=1e-4):
    """exact: every record identical.  Otherwise cell sequences, directions and
    sources identical; a fate or length may differ only where the oracle's
    minimum accumulated optical depth is within guard * tau_kill of tau_kill."""
    mismatched = 0
    for gr, orr in zip(g_tr, o_tr):
        if exact:
            assert np.array_equal(gr[:8], orr[:8]), (gr[:8], orr[:8])
            assert np.array_equal(trace_cells(gr), trace_cells(orr))
            continue
        assert np.array_equal(gr[4:8], orr[4:8])
        gc, oc = trace_cells(gr), trace_cells(orr)
        m = min(len(gc), len(oc))
        assert np.array_equal(gc[:m], oc[:m])
        if np.array_equal(gr[:4], orr[:4]):
            continue
        mismatched += 1
        assert O.FATE_TRUNC in (int(gr[1]), int(orr[1])), (gr[:8], orr[:8])
        at = min(int(gr[0]), int(orr[0])) - 1
        tm = tmin_profile(work, kappa, orr)
        assert abs(tm[at] - work.tau_kill) <= guard * work.tau_kill, (tm[at], gr[:8], orr[:8])
    return mismatched


# The float32 form ends a bin once its optical depth reaches max(tau_kill, 30)
# and books its remainder (at most e^-30 of the bin's photons) as truncated,
# where the oracle carries it on.  Every cell's deposit can
# therefore differ by at most the photons so dropped, all packets together:
# e^-30 of the emitted photons, and their heat at most that times the largest
# photon energy above a threshold.
DROP_FRACTION = math.exp(-30.0)


def drop_allowance(work, emitted):
    """(deposit, heat) allowances of the float32 form's bin dropping."""
    de = float(np.max(np.asarray(work.bins.e_ev) - W.E_TH_EV[0])) * W.EV_ERG
    return DROP_FRACTION * emitted, DROP_FRACTION * emitted * de
