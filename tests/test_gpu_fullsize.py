"""Parity at full size: the 256^3 lognormal H+He workload (1e4 sources, 8
bins, 1e8 packets per step) in the launch configuration bench.py times (tiled
march, every packet of the step in flight, default runs and grid), both
forms, and the 512^3 one (sigma_ln 1.5, 1e5 sources, 5e8 packets per step)
in the float32 form, checked on outputs the oracle can compute one by one:

* packet histories of a sample of packet ids (every 50 000th), each marched
  alone by the oracle over the same frozen state: cell sequences, directions
  and sources identical; fates identical (float64 form) or identical outside
  the extinction guard band (float32 form);
* the cell update of a sample of cells, driven by the deposits the GPU
  accumulated, against the oracle's update of the same cells;
* properties that hold at any size: photon conservation, every packet ending
  once, fractions in [0, 1] summing to one, finite non-negative deposits."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W

import parity as PT

pytestmark = pytest.mark.gpu

STRIDE = 50_000
TRACE_LEN = 1024            # > 3 * 256 cells, the longest path through the grid
STRIDE_512 = 1_000_000
TRACE_LEN_512 = 1600        # > 3 * 512


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()
    return torch


@pytest.fixture(scope="module")
def work():
    return W.lognormal_256()


@pytest.fixture(scope="module")
def oracle_state(work):
    o = O.OracleSolve(work)
    o.absorbers()
    return o


def oracle_traces(o, work, ids, trace_len=TRACE_LEN):
    """Histories of the sampled packets, one oracle march per packet (the
    record of packet g is written at index g / stride = 1 with stride g)."""
    acc = np.zeros((4, work.ncell))
    out = []
    for g in ids:
        g = int(g)
        stride = g if g > 0 else 1
        _, _, tr = o.march(g, g + 1, dt=work.dt_s / work.n_sub, packets=work.packets, seed=1,
                           step_index=0, trace_n=2, trace_len=trace_len, trace_stride=stride, acc=acc,
                           absorbers=False)
        out.append(tr[1 if g > 0 else 0])
    return np.array(out)


def run_gpu(work, fp64, stride=STRIDE, trace_len=TRACE_LEN):
    from paper_1101_4127_amd import rt
    n = work.packets // stride
    s = rt.Solve(work, fp64=fp64, inflight=work.packets, trace_packets=n, trace_len=trace_len,
                 trace_stride=stride)
    st = s.step(seed=1)
    fields = s.fetch()
    tr = s.trace()
    s.release()
    return st, fields, tr


def check_properties(st, fields, work, resid_tol, sum_tol):
    assert st["errors"] == 0 and st["nonfinite"] == 0
    assert st["packets"] == work.packets
    assert st["n_escaped"] + st["n_truncated"] == work.packets
    resid = abs(st["emitted"] - (st["absorbed"] + st["escaped"] + st["truncated"])) / st["emitted"]
    assert resid <= resid_tol, resid
    x = fields[1:6]
    assert np.all(x >= 0.0) and np.all(x <= 1.0 + 1e-6)
    assert np.max(np.abs(x[0] + x[1] - 1.0)) < 1e-5
    assert np.max(np.abs(x[2] + x[3] + x[4] - 1.0)) < 1e-5
    dep = fields[7:11]
    assert np.all(np.isfinite(dep)) and np.all(dep >= 0.0)
    # every photon absorbed in a cell is in the accumulators: their sum is
    # the ledger's absorbed count (the species split sums to the absorbed
    # photons up to the march precision's rounding)
    assert abs(dep[0:3].sum() - st["absorbed"]) <= sum_tol * st["absorbed"]


def check_sampled_updates(work, fields, tol, o=None):
    """Cell updates of a sample of cells driven by the GPU's deposits, against
    the oracle's update of the same cells; returns the per-field maxima."""
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(work.ncell, 2000, replace=False))
    # include the cells with the largest deposits (the ionised and heated ones)
    idx = np.unique(np.concatenate([idx, np.argpartition(fields[7], -500)[-500:]]))
    o = O.OracleSolve(work) if o is None else o
    acc = np.zeros((4, work.ncell))
    acc[:, idx] = fields[7:11][:, idx]
    o.update_cells(work.dt_s / work.n_sub, acc, idx)
    rep = {name: float(np.max(PT.frac_err(fields[1 + f][idx], o.x[f][idx])))
           for f, name in enumerate(("x_HI", "x_HII", "x_HeI", "x_HeII", "x_HeIII"))}
    rep["T"] = float(np.max(PT.temp_err(fields[6][idx], o.T[idx])))
    print("sampled cell updates, max error per field:", rep)
    assert max(rep.values()) <= tol, rep
    return rep


def test_fullsize_fp32_bench_configuration(gpu, work, oracle_state):
    st, fields, tr = run_gpu(work, fp64=False)
    check_properties(st, fields, work, resid_tol=1e-6, sum_tol=1e-6)
    ids = np.arange(0, work.packets, STRIDE)
    otr = oracle_traces(oracle_state, work, ids)
    assert np.all(otr[:, 0] > 0) and {1, 2} <= set(np.unique(otr[:, 1]).tolist())
    mism = PT.compare_traces(work, oracle_state.kappa, tr, otr, exact=False)
    assert mism <= len(ids) // 100, mism
    check_sampled_updates(work, fields, 1e-5)


def test_fullsize_fp64_plain(gpu, work, oracle_state):
    st, fields, tr = run_gpu(work, fp64=True)
    check_properties(st, fields, work, resid_tol=1e-12, sum_tol=1e-12)
    ids = np.arange(0, work.packets, STRIDE)
    otr = oracle_traces(oracle_state, work, ids)
    assert np.all(otr[:, 0] > 0) and {1, 2} <= set(np.unique(otr[:, 1]).tolist())
    PT.compare_traces(work, oracle_state.kappa, tr, otr, exact=True)
    check_sampled_updates(work, fields, 1e-9)


def test_fullsize_512_fp32():
    """512^3, 5e8 packets in flight (about 80 GB of records and lists)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()
    torch.cuda.empty_cache()
    work = W.lognormal_512()
    st, fields, tr = run_gpu(work, fp64=False, stride=STRIDE_512, trace_len=TRACE_LEN_512)
    check_properties(st, fields, work, resid_tol=1e-6, sum_tol=1e-6)
    o = O.OracleSolve(work)
    o.absorbers()
    ids = np.arange(0, work.packets, STRIDE_512)
    otr = oracle_traces(o, work, ids, TRACE_LEN_512)
    assert np.all(otr[:, 0] > 0)
    mism = PT.compare_traces(work, o.kappa, tr, otr, exact=False)
    print(f"512^3: {len(ids)} sampled packet histories, {mism} fates in the extinction guard band")
    assert mism <= len(ids) // 100, mism
    del o
    check_sampled_updates(work, fields, 1e-5)



def test_fullsize_reemission_256(gpu):
    """The re-emission measurement case (256^3 H II region, 1e7 source packets,
    about half of the ionised cells over the threshold), float32 march, as
    bench.py runs it: every ionised cell is crossed by the source's packets, so
    the recombination packets are exactly the cells whose input counter is
    >= f_rec; conservation; and for a sample of cells the update (fractions and
    counters: reset for emitting cells), driven by the GPU's deposits, against
    the oracle's update of the same cell."""
    from paper_1101_4127_amd import rt
    w, rc0 = W.hii_region_reemit()
    s = rt.Solve(w, counters=rc0)
    st = s.step(seed=7)
    f = s.fetch()
    s.release()
    want = int(np.count_nonzero((rc0[0] > 0) & (rc0[0] >= w.recomb.f_rec)))
    assert st["diffuse_packets"] == want > 100000
    assert abs(st["emitted"] - st["absorbed"] - st["escaped"] - st["truncated"]) <= 1e-6 * st["emitted"]
    assert np.all(f[11] >= 0.0) and np.all(np.isfinite(f[11]))
    g = O.make_grid(w)
    rng = np.random.default_rng(1)
    inside = np.nonzero(rc0[0] > 0)[0]
    cells = np.concatenate([rng.choice(inside, 1500, replace=False), rng.choice(w.ncell, 500, replace=False)])
    worst_x = worst_r = 0.0
    for c in cells:
        acc = np.array([f[7, c], f[8, c], f[9, c], f[10, c]])
        x, _, inc = O.update_cell_rx(g, w.dt_s, w.n_h[c], w.x[:, c], w.temp[c], acc, [0, 0, 0])
        emitted = acc[0] > 0 and rc0[0, c] > 0 and rc0[0, c] >= w.recomb.f_rec
        r_want = inc[0] + (0.0 if emitted else rc0[0, c])
        worst_x = max(worst_x, abs(f[2, c] - x[1]) / max(x[1], 1e-8))
        # counters relative to max(|b|, 1e-6 f_rec): in neutral cells the
        # increment is h x_eq - (x_h - x_0)/lambda with lambda h ~ 1e-10, so its
        # few digits differ between two libm's exp; no threshold sees them
        worst_r = max(worst_r, abs(f[11, c] - r_want) / max(abs(r_want), 1e-6 * w.recomb.f_rec))
    assert worst_x <= 1e-6, worst_x            # float32 storage of a float64 update
    assert worst_r <= 1e-9, worst_r


def test_fullsize_periodic_background_fp64(gpu, work):
    """The benchmark workload with periodic boundaries (256 faces) and a
    background field (2.5e7 packets, a quarter of the sources' rate), as
    bench.py's periodic leg runs it, in the float64 form: sampled source packet
    histories bit-exact against the oracle marching each alone (paths up to 256
    cells per axis, wrapping), conservation, every packet ending once, sampled
    cell updates driven by the GPU's deposits (source and background) at 1e-9."""
    bg = W.Background(0.25 * float(np.sum(work.src_ndot)), work.bins.sed.copy(), work.packets // 4)
    w = work.with_(periodic=True, path_cells=256, background=bg)
    st, fields, tr = run_gpu(w, fp64=True)
    assert st["errors"] == 0 and st["nonfinite"] == 0
    assert st["packets"] == w.packets + bg.packets
    assert st["n_escaped"] + st["n_truncated"] == st["packets"]
    assert abs(st["emitted"] - st["absorbed"] - st["escaped"] - st["truncated"]) <= 1e-12 * st["emitted"]
    o = O.OracleSolve(w)
    o.absorbers()
    ids = np.arange(0, w.packets, STRIDE)
    otr = oracle_traces(o, w, ids)
    assert {1, 3} <= set(np.unique(otr[:, 1]).tolist())          # extinguished and path-limited
    PT.compare_traces(w, o.kappa, tr, otr, exact=True)
    check_sampled_updates(w, fields, 1e-9, o=O.OracleSolve(w))
