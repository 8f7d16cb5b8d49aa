"""GPU parity of recombination re-emission (Sec. 2: a cell whose recombinations
reach f_rec N_a emits a packet of recombination photons with a Milne spectrum;
Sec. 3: pCRASH2 emits when a packet crosses such a cell) against the oracle,
through the C ABI."""
import ctypes as C

import numpy as np
import pytest

import parity as PT
from oracle import oracle as O
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


def reemit_case(*, fp64=True, n=20, y_he=0.08, iso=False, f_rec=0.02, packets=6000, n_sub=2,
                ionised=0.6, seed=11):
    w = W.small_mixed(n=n, n_src=4, packets=packets, seed=seed, fp64=fp64, isothermal=iso, y_he=y_he,
                      ionised_fraction=ionised)
    return W.with_recombination(w.with_(dt_s=30.0 * W.MYR_S, n_sub=n_sub), f_rec)


def run_both(w, *, fp64, steps, counters=None, **tiles):
    from paper_1101_4127_amd import rt
    s = rt.Solve(w, fp64=fp64, counters=counters, **tiles)
    o = O.OracleSolve(w)
    if counters is not None:
        o.rc[:len(counters)] = counters
    stats = []
    for k in range(steps):
        stats.append((s.step(seed=w.seed + k), o.step(seed=w.seed + k)))
    fields = s.fetch()
    s.release()
    return o, stats, fields


def counter_err(g, o):
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1e-12)))


def check_counters(o, fields, ions, tol):
    for q in range(ions):
        e = counter_err(fields[11 + q], o.rc[q])
        assert e <= tol, (q, e)
    for q in range(ions, 3):
        assert np.all(fields[11 + q] == 0.0)


@pytest.mark.parametrize("y_he,iso", [(0.08, False), (0.0, True), (0.0, False)])
def test_fp64_matches_oracle(y_he, iso):
    w = reemit_case(y_he=y_he, iso=iso)
    print(f"reemit fp64 y_he={y_he} iso={iso} n={w.n}", flush=True)
    o, stats, fields = run_both(w, fp64=True, steps=2)
    total = 0
    for g, r in stats:
        assert g["diffuse_packets"] == r["diffuse_packets"]
        assert g["packets"] == r["packets"] and g["crossings"] == r["crossings"]
        assert g["diffuse_emitted"] == pytest.approx(r["diffuse_emitted"], rel=1e-12, abs=0.0)
        assert PT.ledger_close(g, r, 1e-12) <= 1e-12
        total += g["diffuse_packets"]
    assert total > 0
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)
    check_counters(o, fields, 3 if y_he > 0 else 1, 1e-9)


def test_fp64_many_emitters_every_substep():
    """f_rec = 0: every crossed cell with any recombination emits each sub-step
    (more recombination packets than source packets)."""
    w = reemit_case(f_rec=0.0, packets=2000, n_sub=3)
    o, stats, fields = run_both(w, fp64=True, steps=1)
    g, r = stats[0]
    assert g["diffuse_packets"] == r["diffuse_packets"] > w.packets
    assert g["crossings"] == r["crossings"]
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)
    check_counters(o, fields, 3, 1e-9)


@pytest.mark.parametrize("tau_kill", [30.0, 60.0])
def test_fp32_given_counters_one_substep(tau_kill):
    """One sub-step whose emitters follow from the input counters: the
    recombination packets are the oracle's exactly; the state within the float32
    march's tolerance.  The float32 form drops a bin once its depth passes
    max(tau_kill, 30) (its remainder, at most e^-30 of the bin, goes to the
    truncated ledger) where the oracle carries it on; recombination packets are
    light and reach cells nothing else reaches, where that remainder is all
    there is.  So deposits are held to 1e-5 relative plus the photons that
    dropping can move (e^-30 of the emitted photons); at tau_kill = 60 dropping
    and extinction coincide and the allowance is not needed."""
    w = reemit_case(fp64=False, n_sub=1, ionised=0.95, f_rec=0.05).with_(tau_kill=tau_kill)
    rng = np.random.default_rng(7)
    rc = rng.random((3, w.ncell)) * 0.1
    o, stats, fields = run_both(w, fp64=False, steps=1, counters=rc)
    g, r = stats[0]
    assert r["diffuse_packets"] > 100
    assert g["diffuse_packets"] == r["diffuse_packets"]
    assert g["diffuse_emitted"] == pytest.approx(r["diffuse_emitted"], rel=1e-6, abs=0)
    # the float32 form carries each packet's spectrum in float32: the emitted
    # photons are those it carries
    e = r["emitted"]
    assert g["emitted"] == pytest.approx(e, rel=1e-7, abs=0)
    for k in ("absorbed", "escaped", "truncated"):
        assert abs(g[k] - r[k]) <= 1e-5 * e, k
    assert abs(g["emitted"] - (g["absorbed"] + g["escaped"] + g["truncated"])) <= 1e-6 * g["emitted"]
    da, ha = PT.drop_allowance(w, e) if tau_kill < 60.0 else (0.0, 0.0)
    PT.compare_state(o, fields, w, frac_tol=1e-4, temp_tol=1e-4, dep_tol=1e-5, dep_allow=da, heat_allow=ha)
    check_counters(o, fields, 3, 1e-4)


def test_fp32_multistep_ledger_and_counters():
    w = reemit_case(fp64=False, packets=8000, n_sub=3)
    from paper_1101_4127_amd import rt
    s = rt.Solve(w)
    total = 0
    for k in range(3):
        st = s.step(seed=40 + k)
        total += st["diffuse_packets"]
        resid = st["emitted"] - (st["absorbed"] + st["escaped"] + st["truncated"])
        assert abs(resid) <= 1e-6 * st["emitted"]
        assert st["packets"] == w.packets + st["diffuse_packets"]
        assert st["nonfinite"] == 0 and st["errors"] == 0
    f = s.fetch()
    s.release()
    assert total > 0
    assert np.all(np.isfinite(f[11:])) and np.all(f[11:] >= 0.0)


def test_schedules_do_not_change_results():
    w = reemit_case(packets=4000)
    ref = None
    for tiles in (dict(), dict(run_len=64, refill_min=4), dict(inflight=1500, park_lanes=8)):
        from paper_1101_4127_amd import rt
        s = rt.Solve(w, fp64=True, **tiles)
        st = [s.step(seed=3 + k) for k in range(2)]
        f = s.fetch()
        s.release()
        if ref is None:
            ref = (st, f)
            continue
        for a, b in zip(st, ref[0]):
            assert a["diffuse_packets"] == b["diffuse_packets"] and a["crossings"] == b["crossings"]
        dep = PT.deposit_err(f[7:11], ref[1][7:11])
        assert np.max(dep) <= 1e-12
        assert np.max(np.abs(f[1:7] - ref[1][1:7]) / np.maximum(np.abs(ref[1][1:7]), 1e-8)) <= 1e-12
        assert counter_err(f[11:], ref[1][11:]) <= 1e-12


def test_rejections():
    import torch
    from paper_1101_4127_amd import rt
    w = reemit_case(packets=1000)
    d = rt.desc_from_workload(w, fp64=True)
    d.flags |= rt.RT_DIRECT_MARCH
    with pytest.raises(rt.RTError) as ex:
        rt.rt_workspace_bytes(d, 4)
    assert ex.value.status == rt.RT_EINVAL
    # stepping before the inputs are set
    d = rt.desc_from_workload(w, fp64=True, inflight=1000)
    ws = torch.empty(rt.rt_workspace_bytes(d, 4), dtype=torch.uint8, device="cuda")
    dt = torch.float64
    nh = torch.as_tensor(w.n_h, dtype=dt, device="cuda")
    x = torch.as_tensor(w.x.reshape(5, -1), dtype=dt, device="cuda").contiguous()
    t = torch.as_tensor(w.temp, dtype=dt, device="cuda")
    h = rt.rt_init_grid(d, ws, 4, nh, x, t)
    rt.rt_add_sources(h, w.src_ijk, w.src_ndot, w.src_sed)
    with pytest.raises(rt.RTError) as ex:
        rt.rt_step(h, w.dt_s, w.packets, 1)
    assert ex.value.status == rt.RT_ESTATE
    r = w.recomb
    bad = r.milne.copy()
    bad[0, 3] *= 0.5                                  # a row that does not sum to 1
    for args in ((-0.1, r.log10_t0, r.dlog10_t, r.milne), (0.1, r.log10_t0, 0.0, r.milne),
                 (0.1, r.log10_t0, r.dlog10_t, bad), (0.1, r.log10_t0, r.dlog10_t, r.milne[:, :1])):
        with pytest.raises(rt.RTError) as ex:
            rt.rt_set_recombination(h, *args)
        assert ex.value.status == rt.RT_EINVAL
    rt.rt_set_recombination(h, r.f_rec, r.log10_t0, r.dlog10_t, r.milne)
    st = rt.rt_step(h, w.dt_s, w.packets, 1)
    assert st["packets"] >= w.packets
    rt.rt_release(h)
    # the fused steps of many solves do not take re-emission (a pure-H one-bin
    # solve, which they would take without it)
    wh = W.with_recombination(W.stromgren_c1(n=8, packets=1000, n_sub=1), 0.1)
    sh = rt.Solve(wh)
    b = rt.Batch(2, wh, fp64=bool(wh.flags & W.FP64_MARCH), max_round_packets=wh.packets,
                 max_tiles=2 * rt.tiles_of(wh.n), graph=False)
    with pytest.raises(rt.RTError) as ex:
        b.step([sh])
    assert ex.value.status == rt.RT_EINVAL
    b.release()
    sh.release()
    # a solve without re-emission refuses the inputs
    w0 = W.small_mixed(n=12, n_src=2, packets=500)
    s0 = rt.Solve(w0)
    with pytest.raises(rt.RTError) as ex:
        rt.rt_set_recombination(s0.h, r.f_rec, r.log10_t0, r.dlog10_t, r.milne)
    assert ex.value.status == rt.RT_ESTATE
    s0.release()


@pytest.mark.parametrize("periodic", [False, True])
def test_one_bin_pure_hydrogen_fp64(periodic):
    """The one-bin instances (13.6 eV, every recombination photon in that bin):
    Test 0's corner source on 16^3 with re-emission, also with periodic
    boundaries."""
    w = W.stromgren_c1(n=16, packets=20000, steps=2, n_sub=4, fp64=True)
    w = W.with_recombination(w.with_(periodic=periodic, path_cells=24 if periodic else 0), 0.002)
    o, stats, fields = run_both(w, fp64=True, steps=2)
    total = 0
    for g, r in stats:
        assert g["diffuse_packets"] == r["diffuse_packets"] and g["crossings"] == r["crossings"]
        assert PT.ledger_close(g, r, 1e-12) <= 1e-12
        total += g["diffuse_packets"]
    assert total > 0
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)
    check_counters(o, fields, 1, 1e-9)
