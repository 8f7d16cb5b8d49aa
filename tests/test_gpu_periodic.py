"""GPU parity of periodic boundaries (Sec. 2: packets re-enter through the
opposite face; they end when extinguished or past path_cells faces along an
axis) against the oracle, through the C ABI."""
import numpy as np
import pytest

import parity as PT
from paper_1101_4127_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()
    return torch


def periodic_case(*, n=20, fp64=True, path_cells=0, tau_kill=30.0, packets=4000, ionised=0.9, y_he=None,
                  n_src=4, seed=13, thin=1.0):
    """thin scales the cell size (and so every cell's optical depth) down."""
    w = W.small_mixed(n=n, n_src=n_src, packets=packets, seed=seed, fp64=fp64, ionised_fraction=ionised,
                      y_he=y_he)
    return w.with_(periodic=True, path_cells=path_cells, tau_kill=tau_kill, cell_cm=w.cell_cm * thin)


@pytest.mark.parametrize("n,path_cells,tau_kill,thin", [(20, 0, 30.0, 0.1), (20, 7, 30.0, 0.1), (12, 50, 6.0, 0.02),
                                                        (6, 13, 30.0, 0.02), (9, 30, 30.0, 0.02), (6, 1, 30.0, 0.02)])
def test_fp64_bitexact_traces_deposits_state(n, path_cells, tau_kill, thin):
    """Ragged grids (20, 9: partial tiles; 12: two tiles per axis; 6: one tile,
    so wraps stay in the tile), short and long path limits, packets ending both
    ways."""
    w = periodic_case(n=n, path_cells=path_cells, tau_kill=tau_kill, thin=thin)
    print(f"periodic fp64 n={n} L={path_cells} tau_kill={tau_kill}", flush=True)
    o, stats, fields, tr = PT.run_both(w, fp64=True, trace_n=w.packets // 4, trace_len=256, stride=4)
    g, r = stats[0]
    assert g["crossings"] == r["crossings"]
    assert g["n_escaped"] == r["n_escaped"] and g["n_truncated"] == r["n_truncated"]
    assert g["n_escaped"] + g["n_truncated"] == w.packets
    PT.compare_traces(w, o.kappa, tr, o.trace, exact=True)
    if r["n_escaped"] > 50:
        assert np.any(tr[:, 1] == 3)                      # traced packets that end at the path limit
    assert PT.ledger_close(g, r, 1e-12) <= 1e-12
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)


def test_longest_path():
    """path_cells at its maximum (2046) in a nearly transparent 6^3 box: packets
    wrap ~340 times along an axis (up to ~5700 crossings) before the limit;
    their recorded first 256 cells, fates and the deposits match the oracle."""
    from paper_1101_4127_amd import rt
    w = periodic_case(n=6, path_cells=rt.RT_MAX_PATH_CELLS, tau_kill=1.0e4, thin=0.0005, packets=400)
    o, stats, fields, tr = PT.run_both(w, fp64=True, trace_n=100, trace_len=256, stride=4)
    g, r = stats[0]
    assert g["crossings"] == r["crossings"] > 1000000
    assert g["n_escaped"] == r["n_escaped"] == w.packets
    PT.compare_traces(w, o.kappa, tr, o.trace, exact=True)
    assert np.all(tr[:, 1] == 3) and tr[:, 0].max() > 5000
    assert PT.ledger_close(g, r, 1e-12) <= 1e-12
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)


def test_fp32_within_stated_tolerance():
    """tau_kill = 1000: the packets end at the path limit (an integer decision),
    so no fate falls in the float32 guard band."""
    w = periodic_case(n=20, fp64=False, packets=8000, ionised=0.6, tau_kill=1000.0)
    o, stats, fields, tr = PT.run_both(w, fp64=False, steps=2, seeds=[5, 6], trace_n=2000, trace_len=256,
                                       stride=4)
    for g, r in stats:
        assert PT.ledger_close(g, r, 1e-5) <= 1e-6
        assert abs(g["crossings"] - r["crossings"]) <= 1e-4 * r["crossings"]
    PT.compare_traces(w, o.kappa, tr, o.trace, exact=False)
    PT.compare_state(o, fields, w, frac_tol=1e-4, temp_tol=1e-4, dep_tol=1e-5)


def test_schedules_do_not_change_results():
    w = periodic_case(n=20, packets=3000, path_cells=40)
    from paper_1101_4127_amd import rt
    ref = None
    for tiles in (dict(), dict(run_len=64, refill_min=4), dict(inflight=700, park_lanes=8), dict(finish_pass=1),
                  dict(finish_pass=4, run_len=64)):
        s = rt.Solve(w, fp64=True, **tiles)
        st = s.step(seed=9)
        f = s.fetch()
        s.release()
        if ref is None:
            ref = (st, f)
            continue
        assert st["crossings"] == ref[0]["crossings"] and st["n_escaped"] == ref[0]["n_escaped"]
        assert np.max(PT.deposit_err(f[7:11], ref[1][7:11])) <= 1e-12


def test_with_reemission_fp64():
    """Periodic boundaries and recombination re-emission together."""
    w = W.with_recombination(periodic_case(n=12, packets=3000, ionised=0.6).with_(dt_s=30.0 * W.MYR_S,
                                                                                  n_sub=2), 0.02)
    from oracle import oracle as O
    from paper_1101_4127_amd import rt
    s = rt.Solve(w, fp64=True)
    o = O.OracleSolve(w)
    total = 0
    for k in range(2):
        g, r = s.step(seed=20 + k), o.step(seed=20 + k)
        assert g["diffuse_packets"] == r["diffuse_packets"] and g["crossings"] == r["crossings"]
        assert PT.ledger_close(g, r, 1e-12) <= 1e-12
        total += g["diffuse_packets"]
    f = s.fetch()
    s.release()
    assert total > 0
    PT.compare_state(o, f, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)


def test_rejected_with_the_per_packet_march():
    from paper_1101_4127_amd import rt
    w = periodic_case(n=8)
    d = rt.desc_from_workload(w, direct=True)
    with pytest.raises(rt.RTError) as ex:
        rt.rt_workspace_bytes(d, 4)
    assert ex.value.status == rt.RT_EINVAL
