"""GPU parity of the one-bin instances that carry the served and batched
workload (monochromatic pure hydrogen: the tiled march, the per-packet march
and the fused steps of many solves) in the float32-march form against the
float64 oracle, and of the float64 form on inputs that are not float32
values.

Bars (Sec. 2, Eq. (1) deposits; the fractions the network makes of them):
* one frozen sub-step from an identical state: cell sequences, directions and
  sources bit-exact, fates equal outside the extinction guard band, deposits
  within 1e-5, fractions within 1e-4, ledger within 1e-5 of the emitted
  photons;
* several sub-steps: the state feeds back (each sub-step's absorbers come
  from fractions carrying the float32 form's 1e-4 bar), so deposits are held
  to the fraction bar, 1e-4;
* float64 form, full-precision inputs: traces bit-exact, deposits, fractions
  and temperature within 1e-9."""
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


MARCH = {"tiled": dict(), "direct": dict(direct=True)}


def f32_state(w):
    """The workload with its state rounded to float32 values, so that the
    float32 form and the oracle start from identical numbers."""
    r = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    return w.with_(n_h=r(w.n_h), x=r(w.x), temp=r(w.temp))


@pytest.mark.parametrize("march", list(MARCH))
def test_fp32_one_bin_single_substep(march):
    """The plain Stroemgren geometry (corner octant source, 13.6 eV, pure H,
    isothermal) in float32, one sub-step: histories and every field."""
    w = f32_state(W.stromgren_c1(n=16, packets=8000, steps=1, n_sub=1, fp64=False))
    print(f"fp32 one-bin single sub-step, {march}", flush=True)
    o, stats, fields, tr = PT.run_both(w, fp64=False, trace_n=3000, trace_len=64, **MARCH[march])
    g, r = stats[0]
    assert g["packets"] == r["packets"]
    assert abs(g["crossings"] - r["crossings"]) <= 1e-4 * r["crossings"]
    assert PT.ledger_close(g, r, 1e-5) <= 1e-6
    PT.compare_traces(w, o.kappa, tr, o.trace, exact=False)
    PT.compare_state(o, fields, w, frac_tol=1e-4, temp_tol=1e-4, dep_tol=1e-5)


@pytest.mark.parametrize("march", list(MARCH))
def test_fp32_one_bin_multistep(march):
    """Two steps of four frozen sub-steps in float32 against the oracle."""
    w = f32_state(W.stromgren_c1(n=16, packets=8000, steps=2, n_sub=4, fp64=False))
    print(f"fp32 one-bin two steps, {march}", flush=True)
    o, stats, fields, tr = PT.run_both(w, fp64=False, steps=2, **MARCH[march])
    for g, r in stats:
        assert g["packets"] == r["packets"]
        assert PT.ledger_close(g, r, 1e-5) <= 1e-6
    PT.compare_state(o, fields, w, frac_tol=1e-4, temp_tol=1e-4, dep_tol=1e-4)


def serving_requests(count, seed, steps, n_sub):
    reqs = W.serving_stream(count=count, rate_per_s=2000.0, seed=seed, steps=steps, n_sub=n_sub,
                            sides=(16, 24), log_packets=(3.5, 4.0), max_sources=6)
    for r in reqs:
        r.work = f32_state(r.work)
    return reqs


@pytest.mark.parametrize("steps,n_sub,dep_tol", [(1, 1, 1e-5), (2, 3, 1e-4)], ids=["one-substep", "multistep"])
def test_fp32_fused_batch_against_oracle(steps, n_sub, dep_tol):
    """Serving-shaped solves (uniform and lognormal gas, 1-6 sources, uneven
    sides) advanced together by fused float32 steps, each against the oracle
    run alone."""
    from paper_1101_4127_amd import rt
    reqs = serving_requests(4, 51, steps, n_sub)
    print(f"fp32 fused batch, {steps} steps of {n_sub} sub-steps", flush=True)
    pk = sum(-(-r.work.packets // r.work.n_sub) for r in reqs)
    b = rt.Batch(len(reqs), reqs[0].work, fp64=False, max_round_packets=pk,
                 max_tiles=sum(rt.tiles_of(r.work.n) for r in reqs), graph=True)
    solves = [rt.Solve(r.work, fp64=False, direct=True, brick_log2=3, stream=b.stream) for r in reqs]
    oracles = [O.OracleSolve(r.work) for r in reqs]
    for _ in range(steps):
        led = b.step(solves, stats=True)
        for o, g in zip(oracles, led):
            r = o.step()
            assert g["packets"] == r["packets"]
            assert abs(g["crossings"] - r["crossings"]) <= 1e-4 * r["crossings"]
            assert PT.ledger_close(g, r, 1e-5) <= 1e-6
    for r, s, o in zip(reqs, solves, oracles):
        PT.compare_state(o, s.fetch(), r.work, frac_tol=1e-4, temp_tol=1e-4, dep_tol=dep_tol)
        s.release()
    b.release()


def full_precision_case(n=(21, 18, 13), n_src=4, packets=10000, seed=61, y_he=0.0789, tau_kill=5.0):
    """H+He gas whose densities, fractions and temperatures use all 53 bits
    of float64 (no value is a float32 number), partly ionised and warm."""
    rng = np.random.default_rng(seed)
    nc = n[0] * n[1] * n[2]
    nh = 2e-4 * np.exp(rng.normal(0.0, 0.8, nc)) * (1.0 + 1e-12 * rng.random(nc))
    xi = 0.6 * rng.random(nc)
    x = np.zeros((5, nc))
    x[0] = 1.0 - xi
    x[1] = xi
    x[3] = 0.5 * xi * rng.random(nc)
    x[4] = 0.2 * xi * rng.random(nc)
    x[2] = 1.0 - x[3] - x[4]
    temp = 100.0 + 2e4 * rng.random(nc)
    assert not np.any(nh == nh.astype(np.float32)) and not np.all(x[1] == x[1].astype(np.float32))
    bins = W.blackbody_table(1e5)
    cells = rng.choice(nc, size=n_src, replace=False)
    return W.Workload(
        name="full_precision", n=n, cell_cm=6e22, y_he=y_he, bins=bins, redshift=9.0, n_h=nh, x=x,
        temp=temp, src_ijk=W.cells_to_ijk(cells, n),
        src_ndot=W.powerlaw_luminosities(n_src, 1e50, 1e53, rng), src_sed=np.tile(bins.sed, (n_src, 1)),
        dt_s=1e4 * W.YR_S, packets=packets, tau_kill=tau_kill, flags=W.FP64_MARCH, seed=9)


@pytest.mark.parametrize("march", list(MARCH))
def test_fp64_full_precision_inputs(march):
    w = full_precision_case()
    print(f"fp64 full-precision inputs, {march}", flush=True)
    o, stats, fields, tr = PT.run_both(w, fp64=True, trace_n=w.packets, trace_len=96, **MARCH[march])
    g, r = stats[0]
    assert g["crossings"] == r["crossings"] and g["n_truncated"] == r["n_truncated"] > 0
    PT.compare_traces(w, o.kappa, tr, o.trace, exact=True)
    assert PT.ledger_close(g, r, 1e-12) <= 1e-12
    PT.compare_state(o, fields, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)
