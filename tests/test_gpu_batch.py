"""Fused steps of many solves (rt_step_many) and the continuous-batching
server, on the serving workload's kind of solves (pure hydrogen, one 13.6 eV
bin, isothermal, uneven grid sides, uniform or lognormal gas).

* every solve's result in a fused batch is the one rt_step gives alone, up to
  the order of float64 deposit additions: packets and crossings equal,
  deposits and fractions (relative to max(x, 1e-6)) within 1e-9 (float64) /
  fractions within 1e-4 and deposits within 1e-5 (float32 march), the stated
  bars of the two forms;
* a captured graph, replayed several times with eager work and
  synchronisations between the replays and with a different set of solves,
  gives what the eager launches give;
* against the float64 oracle, solve by solve;
* served requests (admission by free slots, joins between fused calls) end
  where the same requests end alone."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1101_4127_amd import workloads as W

import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()
    return torch


def stream(count=8, seed=41, steps=2, n_sub=4, sides=(16, 24, 32), log_packets=(3.5, 4.3), rate=2000.0):
    return W.serving_stream(count=count, rate_per_s=rate, seed=seed, steps=steps, n_sub=n_sub, sides=sides,
                            log_packets=log_packets, max_sources=6)


# Fused solves keep their fields in bricks of 8^3 cells, as the fused march
# reads them: every tiled solve does, and so does a per-packet-march solve
# asked for that brick size.
TILED = dict()
BRICK = dict(direct=True, brick_log2=3)


def batch_for(works, fp64, graph=True, max_solves=None, **tiles):
    """A batch sized for these solves: their tiles and one sub-step of
    packets of them all."""
    from paper_1101_4127_amd import rt
    works = list(works)
    pk = sum(-(-int(w.packets) // int(w.n_sub)) for w in works)
    nt = sum(rt.tiles_of(w.n) for w in works)
    return rt.Batch(max_solves or len(works), works[0], fp64=fp64, max_round_packets=max(pk, 1),
                    max_tiles=nt, graph=graph, **tiles)


def alone(reqs, fp64):
    from paper_1101_4127_amd import rt
    out = []
    for r in reqs:
        s = rt.Solve(r.work, fp64=fp64, **TILED)
        led = [s.step() for _ in range(r.work.steps)]
        out.append((s.fetch(), led))
        s.release()
    return out


def batched(reqs, fp64, graph):
    from paper_1101_4127_amd import rt
    b = batch_for([r.work for r in reqs], fp64, graph)
    solves = [rt.Solve(r.work, fp64=fp64, stream=b.stream, **TILED) for r in reqs]
    leds = [[] for _ in reqs]
    for _ in range(reqs[0].work.steps):
        for i, st in enumerate(b.step(solves, stats=True)):
            leds[i].append(st)
    out = [(s.fetch(), led) for s, led in zip(solves, leds)]
    for s in solves:
        s.release()
    b.release()
    return out


def assert_same(a, m, fp64, work):
    fa, la = a
    fm, lm = m
    for x, y in zip(la, lm):
        assert x["packets"] == y["packets"]
        assert x["substeps"] == y["substeps"] == work.n_sub
        assert abs(x["crossings"] - y["crossings"]) <= 1e-6 * x["crossings"]
        assert abs(x["emitted"] - y["emitted"]) <= 1e-12 * x["emitted"]
        for k in ("absorbed", "escaped", "truncated"):
            assert abs(x[k] - y[k]) <= 1e-9 * x["emitted"], k
        assert y["nonfinite"] == 0 and y["errors"] == 0
    # float64: the two runs differ only in the order of float64 deposit
    # additions, i.e. by rounding; fractions are compared relative to
    # max(x, 1e-6) (a rounding-level absolute difference of 1e-16 on a
    # fraction of 1e-10 is not a 1e-6 relative error)
    ft, dt, floor = (1e-9, 1e-9, 1e-6) if fp64 else (1e-4, 1e-5, 1e-8)
    assert np.array_equal(fa[0], fm[0])
    for f in (1, 2):
        assert np.max(PT.frac_err(fm[f], fa[f], floor)) <= ft, f
    assert np.max(PT.deposit_err(fm[7], fa[7])) <= dt
    assert np.array_equal(fa[6], fm[6])          # isothermal


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_fused_step_equals_alone(fp64, graph):
    reqs = stream()
    a = alone(reqs, fp64)
    m = batched(reqs, fp64, graph)
    for r, x, y in zip(reqs, a, m):
        assert_same(x, y, fp64, r.work)


def test_graph_replays_match_eager_launches():
    """Three fused calls of the same solves through a captured graph and
    through eager launches, the fields fetched (eager copies, synchronising)
    after every call; then the graph again with another set of solves."""
    from paper_1101_4127_amd import rt
    reqs = stream(count=6, seed=43, steps=3)
    be, bg = batch_for([r.work for r in reqs], True, False), batch_for([r.work for r in reqs], True, True)
    se = [rt.Solve(r.work, fp64=True, stream=be.stream, **TILED) for r in reqs]
    sg = [rt.Solve(r.work, fp64=True, stream=bg.stream, **TILED) for r in reqs]
    for _ in range(3):
        le = be.step(se, stats=True)
        lg = bg.step(sg, stats=True)
        for x, y in zip(le, lg):
            assert x["packets"] == y["packets"] and x["crossings"] == y["crossings"]
        for a, b in zip(se, sg):
            fa, fb = a.fetch(), b.fetch()
            assert np.max(PT.frac_err(fb[1], fa[1], 1e-6)) <= 1e-9
            assert np.max(PT.deposit_err(fb[7], fa[7])) <= 1e-9
    # the same graph shape with three of the solves, in another order
    sub_e, sub_g = [se[4], se[1], se[2]], [sg[4], sg[1], sg[2]]
    be.step(sub_e, stats=True)
    bg.step(sub_g, stats=True)
    for a, b in zip(sub_e, sub_g):
        fa, fb = a.fetch(), b.fetch()
        assert np.max(PT.frac_err(fb[1], fa[1], 1e-6)) <= 1e-9
    for s in se + sg:
        s.release()
    be.release()
    bg.release()


def test_fused_step_against_oracle():
    """Float64 fused steps of three small solves (per-packet-march solves in
    bricks of 8^3) against the oracle run on each alone (multi-step float64
    bar: 1e-6 on fractions and deposits)."""
    from paper_1101_4127_amd import rt
    reqs = stream(count=3, seed=44, steps=2, n_sub=3, sides=(16,), log_packets=(3.3, 3.6))
    b = batch_for([r.work for r in reqs], True)
    solves = [rt.Solve(r.work, fp64=True, stream=b.stream, **BRICK) for r in reqs]
    oracles = [O.OracleSolve(r.work) for r in reqs]
    for _ in range(2):
        led = b.step(solves, stats=True)
        for o, g in zip(oracles, led):
            ost = o.step()
            assert g["packets"] == ost["packets"]
            assert abs(g["crossings"] - ost["crossings"]) <= 1e-6 * ost["crossings"]
            assert abs(g["emitted"] - ost["emitted"]) <= 1e-12 * ost["emitted"]
            res = abs(g["emitted"] - (g["absorbed"] + g["escaped"] + g["truncated"])) / g["emitted"]
            assert res <= 1e-12
    for r, s, o in zip(reqs, solves, oracles):
        PT.compare_state(o, s.fetch(), r.work, frac_tol=1e-6, temp_tol=1e-12, dep_tol=1e-6)
        s.release()
    b.release()


def test_fused_step_rejects_what_it_cannot_fuse():
    from paper_1101_4127_amd import rt
    reqs = stream(count=2, seed=45)
    b = batch_for([r.work for r in reqs] * 2, True, False, max_solves=2)
    s64 = rt.Solve(reqs[0].work, fp64=True, stream=b.stream, **BRICK)
    s32 = rt.Solve(reqs[1].work, fp64=False, stream=b.stream, **BRICK)
    hhe = rt.Solve(W.small_mixed(n=8, n_src=2, packets=2000), fp64=True, stream=b.stream, **BRICK)
    per = rt.Solve(reqs[0].work.with_(periodic=True), fp64=True, stream=b.stream)
    b1 = rt.Solve(reqs[1].work, fp64=True, direct=True, brick_log2=1, stream=b.stream)
    traced = rt.Solve(reqs[1].work, fp64=True, stream=b.stream, trace_packets=10, trace_len=8, **BRICK)
    for bad in ([s64, s32], [s64, s64], [hhe], [s64, s64, s64], [per], [s64, per], [b1], [traced]):
        with pytest.raises(rt.RTError) as e:
            b.step(bad)
        assert e.value.status == rt.RT_EINVAL
    # more packets in one round than the batch holds
    with pytest.raises(rt.RTError) as e:
        b.step([s64], packets=[100 * (reqs[0].work.packets + reqs[1].work.packets)])
    assert e.value.status == rt.RT_ENOMEM
    # nothing was enqueued: the solves still step alone
    assert s64.step()["packets"] == reqs[0].work.packets
    for s in (s64, s32, hhe, per, b1, traced):
        s.release()
    b.release()


def test_served_results_equal_results_alone():
    """Twelve requests arriving faster than they are served, at most five
    admitted at once: each served result equals the request run alone."""
    from paper_1101_4127_amd import serve
    reqs = stream(count=12, seed=46, steps=3, rate=400.0)
    srv = serve.Server(max_slots=5, fp64=False, graph=True)
    got = srv.run(reqs)
    srv.release()
    assert [g.rid for g in got] == [r.rid for r in reqs]
    assert max(srv.call_solves) <= 5 and srv.calls >= 3 * 12 / 5
    ref, _ = serve.run_alone(reqs, fp64=False, direct=False)
    for g, a, r in zip(got, ref, reqs):
        assert g.steps == r.work.steps and g.packets == a.packets
        assert g.latency_s > 0 and g.admit_s >= 0
        assert abs(g.crossings - a.crossings) <= 1e-6 * a.crossings
        assert np.max(PT.frac_err(g.fields[1], a.fields[1])) <= 1e-4
        assert np.max(PT.deposit_err(g.fields[7], a.fields[7])) <= 1e-5
        assert g.residual <= 1e-6


def test_autotuned_parameters_leave_results_unchanged():
    """The tuner on a small H+He case (both march kinds, one sweep), then the
    chosen parameters against the defaults: same ledger, same deposits."""
    from paper_1101_4127_amd import autotune, rt
    w = W.small_mixed(n=24, n_src=4, packets=20000, fp64=True)
    r = autotune.tune(w, fp64=True, steps=1, sweeps=1)
    assert len(r["trials"]) >= 10 and r["march_ms"] > 0
    cfg = dict(r["config"])
    a = rt.Solve(w, fp64=True)
    sa = a.step()
    fa = a.fetch()
    a.release()
    b = rt.Solve(w, fp64=True, **cfg)
    sb = b.step()
    fb = b.fetch()
    b.release()
    assert sa["crossings"] == sb["crossings"] and sa["packets"] == sb["packets"]
    assert sa["n_escaped"] == sb["n_escaped"] and sa["n_truncated"] == sb["n_truncated"]
    for f in range(7, 11):
        assert np.max(PT.deposit_err(fb[f], fa[f])) <= 1e-9


def test_fused_step_single_solve_and_solve_without_sources():
    """A batch of one, and a batch holding a solve without sources (its cell
    update still runs, with no packets), each against the same solves alone."""
    from paper_1101_4127_amd import rt
    reqs = stream(count=2, seed=47)
    empty = reqs[1].work.with_(src_ijk=np.zeros((0, 3), np.int32), src_ndot=np.zeros(0), src_sed=np.zeros((0, 1)))
    works = [reqs[0].work, empty]
    for batch in ([0], [0, 1]):
        b = batch_for(works, True, True)
        fused = [rt.Solve(works[i], fp64=True, stream=b.stream, **BRICK) for i in batch]
        alone = [rt.Solve(works[i], fp64=True, **BRICK) for i in batch]
        for _ in range(2):
            led = b.step(fused, stats=True)
            ref = [s.step() for s in alone]
            for x, y in zip(ref, led):
                assert x["packets"] == y["packets"] and x["substeps"] == y["substeps"]
        for a, f in zip(alone, fused):
            fa, fm = a.fetch(), f.fetch()
            assert np.max(PT.frac_err(fm[1], fa[1], 1e-6)) <= 1e-9
            assert np.max(PT.deposit_err(fm[7], fa[7])) <= 1e-9
            a.release()
            f.release()
        b.release()



@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_fused_hhe_eight_bins_against_alone_and_oracle(fp64):
    """H+He solves of 8 black-body bins (thermal) fuse too: each fused solve
    against the same solve alone (float64: 1e-9; float32: its bars) and, in
    float64, one sub-step against the oracle (1e-9)."""
    from paper_1101_4127_amd import rt
    works = [W.small_mixed(n=n, n_src=k, packets=p, fp64=fp64, seed=sd)
             for n, k, p, sd in ((12, 2, 3000, 31), (20, 4, 6000, 33), (9, 1, 2000, 35))]
    works = [w.with_(n_sub=1) for w in works]
    print(f"fused H+He 8 bins, fp64={fp64}", flush=True)
    b = batch_for(works, fp64)
    fused = [rt.Solve(w, fp64=fp64, stream=b.stream, **TILED) for w in works]
    alone = [rt.Solve(w, fp64=fp64, **TILED) for w in works]
    led = b.step(fused, stats=True)
    ref = [s.step() for s in alone]
    for x, y in zip(ref, led):
        assert x["packets"] == y["packets"] and x["crossings"] == y["crossings"]
        for k in ("absorbed", "escaped", "truncated"):
            assert abs(x[k] - y[k]) <= 1e-9 * x["emitted"], k
    ft, dt = (1e-9, 1e-9) if fp64 else (1e-4, 1e-5)
    for w, a, f in zip(works, alone, fused):
        fa, fm = a.fetch(), f.fetch()
        for k in range(1, 7):
            assert np.max(PT.frac_err(fm[k], fa[k], 1e-6)) <= ft, k
        for k in range(7, 11):
            assert np.max(PT.deposit_err(fm[k], fa[k])) <= dt, k
        if fp64:
            o = O.OracleSolve(w)
            o.step()
            PT.compare_state(o, fm, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9, frac_floor=1e-7)
        a.release()
        f.release()
    b.release()


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_fused_finishing_pass(fp64):
    """Fused steps whose rounds end with a finishing pass after 2 tile passes
    (serving-shaped solves of sides 16-48, up to 6 tile passes) against the
    same solves alone without one: same counters, deposits and fractions
    within the float64 (1e-9) or float32 bars."""
    from paper_1101_4127_amd import rt
    reqs = stream(count=5, seed=48, steps=2, n_sub=3, sides=(16, 32, 48))
    print(f"fused finishing pass, fp64={fp64}", flush=True)
    a = alone(reqs, fp64)
    b = batch_for([r.work for r in reqs], fp64, True, finish_pass=2)
    solves = [rt.Solve(r.work, fp64=fp64, stream=b.stream, **TILED) for r in reqs]
    leds = [[] for _ in reqs]
    for _ in range(2):
        for i, st in enumerate(b.step(solves, stats=True)):
            leds[i].append(st)
    m = [(s.fetch(), led) for s, led in zip(solves, leds)]
    for s in solves:
        s.release()
    b.release()
    for r, x, y in zip(reqs, a, m):
        assert_same(x, y, fp64, r.work)


def test_launch_then_wait_and_ordering_of_the_solves_streams():
    """A fused call that returns at once: the solves' fields fetched before
    the wait (their own streams, opened on another stream than the batch's,
    are ordered after the call when next used) and the ledgers from
    rt_batch_wait equal those of the same call made synchronously; a wait
    for another solve count is refused."""
    import torch
    from paper_1101_4127_amd import rt
    reqs = stream(count=4, seed=49, steps=2, n_sub=3)
    side = torch.cuda.Stream()
    ref_b = batch_for([r.work for r in reqs], True, True)
    ref = [rt.Solve(r.work, fp64=True, stream=ref_b.stream, **TILED) for r in reqs]
    b = batch_for([r.work for r in reqs], True, True)
    sv = [rt.Solve(r.work, fp64=True, stream=side, **TILED) for r in reqs]
    for _ in range(2):
        lr = ref_b.step(ref, stats=True)
        b.launch(sv)
        fields = [s.fetch() for s in sv]           # before the wait
        with pytest.raises(rt.RTError) as e:
            rt.rt_batch_wait(b.b, len(sv) - 1)
        assert e.value.status == rt.RT_EINVAL
        lw = b.wait()
        for x, y in zip(lr, lw):
            assert x["packets"] == y["packets"] and x["crossings"] == y["crossings"]
            assert x["substeps"] == y["substeps"]
            for k in ("emitted", "absorbed", "escaped", "truncated"):
                assert abs(x[k] - y[k]) <= 1e-12 * x["emitted"], k
        for s, f in zip(ref, fields):
            fr = s.fetch()
            assert np.max(PT.frac_err(f[1], fr[1], 1e-6)) <= 1e-9
            assert np.max(PT.deposit_err(f[7], fr[7])) <= 1e-9
    for s in ref + sv:
        s.release()
    ref_b.release()
    b.release()


@pytest.mark.gpu
def test_two_batches_stepping_the_same_solves_in_turn():
    """Solves stepped by one batch and, before that call has ended, by
    another: the second batch's call waits for the first's, so both ledgers
    and the final state equal those of one batch stepping them every time."""
    import torch
    from paper_1101_4127_amd import rt
    reqs = stream(count=3, seed=53, steps=4, n_sub=2)
    side = torch.cuda.Stream()
    ref_b = batch_for([r.work for r in reqs], True, True)
    ref = [rt.Solve(r.work, fp64=True, stream=side, **TILED) for r in reqs]
    b1 = batch_for([r.work for r in reqs], True, True)
    b2 = batch_for([r.work for r in reqs], True, False)
    sv = [rt.Solve(r.work, fp64=True, stream=side, **TILED) for r in reqs]
    for _ in range(2):
        lr = [ref_b.step(ref, stats=True), ref_b.step(ref, stats=True)]
        b1.launch(sv)
        b2.launch(sv)                                # while the first call may still run
        lw = [b1.wait(), b2.wait()]
        for a, c in zip(lr, lw):
            for x, y in zip(a, c):
                assert x["packets"] == y["packets"] and x["crossings"] == y["crossings"]
                for key in ("emitted", "absorbed", "escaped", "truncated"):
                    assert abs(x[key] - y[key]) <= 1e-12 * x["emitted"], key
    for s, r in zip(sv, ref):
        f, fr = s.fetch(), r.fetch()
        assert np.max(PT.frac_err(f[1], fr[1], 1e-6)) <= 1e-9
        assert np.max(PT.deposit_err(f[7], fr[7])) <= 1e-9
    for s in ref + sv:
        s.release()
    for x in (ref_b, b1, b2):
        x.release()
