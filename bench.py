#!/usr/bin/env python3
"""Benchmark of the Monte-Carlo radiative-transfer hot path on one MI355X.

A step is one full pass of the path over the step's packets: absorber table
from the frozen state, the packet march (emission, traversal, Eq. (1)
attenuation, deposition), the ledger and the per-cell ionisation/temperature
update.  Workload: 256^3 lognormal H+He gas at z = 9, 1e4 black-body sources in
the densest 1 % of cells, 8 frequency bins, 1e8 packets per step; inputs are
seeded and synthetic and already resident in HBM when timing starts.

Prints one JSON line: whole-step cell crossings/s of the float32-march /
float64-accumulate form (tiled march, every packet of the step in flight),
the march kernel's roofline (algorithmic bytes per crossing over the
HIP-event duration of its launches on the library's stream), the plain
float64 form measured the same way, the float64 CPU oracle timed on a
bounded sample, and the serving workload: 512 independent pure-hydrogen
solves (sides 16-64, 5 steps each) arriving as a Poisson stream of 200/s,
served by continuous batching of fused steps (p50/p99 latency, throughput),
against the same solves run one at a time in the plain float64 form.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell crossings/s + HBM GB/s at 256^3; batched-solve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per crossing: absorber gather + four float64
# accumulator updates (H+He with heating)
BYTES_F32 = 3 * 4 + 4 * 8
BYTES_F64 = 3 * 8 + 4 * 8
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "march_traffic.json")
KERNELS = {False: "k_tmarch<float, 3, true, 8, 3, 2, false>", True: "k_march<float, 3, true, 8, 3, 2>"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def march_hash() -> str:
    h = hashlib.sha256()
    for name in ("rt_tiled.hip", "rt_march.hip", "rt_cross.h", "rt_device.h", "rt_internal.h"):
        with open(os.path.join(ROOT, "paper_1101_4127_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def workload(name: str, packets):
    from paper_1101_4127_amd import workloads as W
    if name == "lognormal_256":
        return W.lognormal_256(packets=packets or 100_000_000)
    if name == "lognormal_128":
        return W.lognormal_128(packets=packets or 10_000_000)
    if name == "lognormal_512":
        return W.lognormal_512(packets=packets or 500_000_000)
    raise SystemExit(f"unknown workload {name}")


def time_form(work, *, fp64: bool, steps: int, warmup: int, tiles: dict):
    import torch
    from paper_1101_4127_amd import rt
    tiles = dict(tiles)
    if not tiles.get("direct") and not tiles.get("inflight"):
        tiles["inflight"] = -(-work.packets // work.n_sub)        # every packet of a sub-step in flight
    s = rt.Solve(work, fp64=fp64, time_march=True, **tiles)
    for i in range(warmup):
        s.step(seed=1000 + i)
    torch.cuda.synchronize()
    cross = 0
    march_ms = kernel_ms = 0.0
    launches = 0
    resid = 0.0
    t0 = time.perf_counter()
    for i in range(steps):
        st = s.step(seed=1 + i)
        cross += st["crossings"]
        march_ms += st["march_ms"]
        kernel_ms += st["kernel_ms"]
        launches += st["kernel_launches"]
        resid = max(resid, abs(st["emitted"] - st["absorbed"] - st["escaped"] - st["truncated"]) / st["emitted"])
        if st["nonfinite"]:
            raise SystemExit("non-finite cell state")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.release()
    return dict(crossings=cross, wall_s=wall, march_ms=march_ms, kernel_ms=kernel_ms, launches=launches,
                resid=resid)


def copy_calibration(mib: int):
    """A plain device copy of known size, for scaling HBM counters (run under
    rocprofv3 --pmc next to the march)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {mib} MiB read + {mib} MiB written")
    del a, b


def cpu_baseline(work, target_s: float):
    """The float64 oracle on a bounded sample of the same step: packet ranges
    spread over all sources plus a random sample of cell updates, scaled to a
    full step."""
    import numpy as np
    from oracle import oracle as O
    o = O.OracleSolve(work)
    o.absorbers()
    P = work.packets
    nrange = 64
    per = 400
    acc = np.zeros((4, work.ncell))
    cross = 0
    used = 0
    t_march = 0.0
    k = 0
    while True:
        g0 = (k * 7919 % nrange) * (P // nrange) + (k // nrange) * per
        t0 = time.perf_counter()
        _, led, _ = o.march(g0, g0 + per, dt=work.dt_s, packets=P, seed=1, step_index=0, acc=acc,
                            absorbers=False)
        t_march += time.perf_counter() - t0
        cross += led["crossings"]
        used += per
        k += 1
        if t_march > 0.8 * target_s or used >= P:
            break
    rng = np.random.default_rng(0)
    nupd = min(work.ncell, 200_000)
    idx = np.sort(rng.choice(work.ncell, nupd, replace=False))
    t0 = time.perf_counter()
    o.update_cells(work.dt_s, acc, idx)
    t_upd = time.perf_counter() - t0
    full_cross = cross * P / used
    full_time = t_march * P / used + t_upd * work.ncell / nupd
    return {
        "value": full_cross / full_time, "unit": "crossings/s", "cores": 1, "kind": "oracle",
        "sample": (f"{used} packets in {k} ranges spread over all sources ({cross} crossings, "
                   f"{t_march:.1f} s) + {nupd} cell updates ({t_upd:.1f} s), scaled to one full step "
                   f"of {P} packets and {work.ncell} cells; single-threaded float64 C oracle"),
        "march_crossings_per_s": cross / t_march,
        "update_cells_per_s": nupd / t_upd,
    }


def traffic_for(launch_crossings: float):
    """HBM bytes per march launch from committed rocprofv3 counter runs, or
    None when the counters were taken on a different march kernel."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        t = json.load(f)
    if t.get("march_hash") != march_hash():
        return None
    return t.get("bytes_per_launch")


def serving_leg(count: int, accuracy_requests: int = 32):
    """The serving workload through the continuous-batching server (float32
    march, fused steps replayed as a hipGraph), in real time and with every
    request present at once, and the same requests one at a time in the plain
    float64 form; the served results of the first requests against their
    float64 results."""
    import numpy as np
    from paper_1101_4127_amd import serve
    from paper_1101_4127_amd import workloads as W
    t0 = time.perf_counter()
    reqs = W.serving_stream(count=count)
    log(f"serving: {count} requests ({time.perf_counter() - t0:.1f} s to generate), "
        f"arrivals over {reqs[-1].arrival_s:.2f} s")
    srv = serve.Server(max_slots=64, fp64=False, graph=True, keep_fields=False)
    srv.run(W.serving_stream(count=8, seed=99), realtime=False)           # capture and first launches
    srv.calls, srv.call_solves = 0, []
    t = time.perf_counter()
    got = srv.run(reqs)
    wall = time.perf_counter() - t
    calls, mean_batch = srv.calls, float(np.mean(srv.call_solves))
    t = time.perf_counter()
    sat = srv.run(reqs, realtime=False)
    wall_sat = time.perf_counter() - t
    srv.release()
    lat = [g.latency_s for g in got]
    cross = sum(g.crossings for g in got)
    cross_sat = sum(g.crossings for g in sat)
    base, wall_base = serve.run_alone(reqs, fp64=True, direct=True, keep_fields=False)
    cross_base = sum(g.crossings for g in base)
    # accuracy of the served form against the plain float64 form
    sub = reqs[:accuracy_requests]
    srv = serve.Server(max_slots=64, fp64=False, graph=True, keep_fields=True)
    acc32 = srv.run(sub, realtime=False)
    srv.release()
    acc64, _ = serve.run_alone(sub, fp64=True, direct=True, keep_fields=True)
    fx, dep = [], []
    for a, b in zip(acc32, acc64):
        for f in (1, 2):
            fx.append(np.abs(a.fields[f] - b.fields[f]) / np.maximum(b.fields[f], 1e-8))
        mean = float(np.mean(np.abs(b.fields[7])))
        dep.append(np.abs(a.fields[7] - b.fields[7]) / np.maximum(np.abs(b.fields[7]), 1e-12 * max(mean, 1e-300)))
    fx = np.concatenate(fx)
    dep = np.concatenate(dep)
    out = {
        "workload": f"poisson_{count}_pure_H_16-64^3", "requests": count, "rate_per_s": 200.0,
        "form": "float32 march, float64 accumulators; fused steps of up to 64 solves replayed as a hipGraph",
        "p50_latency_ms": 1e3 * serve.percentile(lat, 50), "p99_latency_ms": 1e3 * serve.percentile(lat, 99),
        "wall_s": wall, "solves_per_s": count / wall, "crossings_per_s": cross / wall,
        "fused_calls": calls, "mean_solves_per_call": mean_batch,
        "max_conservation_residual": max(g.residual for g in got),
        "all_present": {"wall_s": wall_sat, "solves_per_s": count / wall_sat, "crossings_per_s": cross_sat / wall_sat},
        "baseline_fp64_one_at_a_time": {"wall_s": wall_base, "solves_per_s": count / wall_base,
                                        "crossings_per_s": cross_base / wall_base, "march": "per-packet"},
        "speedup_all_present_vs_baseline": (cross_sat / wall_sat) / (cross_base / wall_base),
        "accuracy_vs_fp64": {"requests": len(sub), "fraction_err_max": float(fx.max()),
                             "fraction_err_p99": float(np.percentile(fx, 99)),
                             "deposit_err_max": float(dep.max()), "deposit_err_p99": float(np.percentile(dep, 99))},
    }
    log(f"serving: p50 {out['p50_latency_ms']:.1f} ms, p99 {out['p99_latency_ms']:.1f} ms, "
        f"{out['solves_per_s']:.0f} solves/s at 200/s arrivals; all present: {out['all_present']['crossings_per_s']:.3g} "
        f"crossings/s vs {out['baseline_fp64_one_at_a_time']['crossings_per_s']:.3g} one at a time in float64 "
        f"({out['speedup_all_present_vs_baseline']:.1f}x); fractions vs float64 max {fx.max():.2e}")
    return out


def reemit_leg(n: int, packets: int):
    """Recombination re-emission at scale: one step of an established H II
    region whose counters put about half of its cells over the threshold,
    with re-emission (float32 march) and, for the cost, the same step
    without it.  Each is timed on a fresh solve after a warm-up solve."""
    import torch
    from paper_1101_4127_amd import rt
    from paper_1101_4127_amd import workloads as W
    w, counters = W.hii_region_reemit(n=n, packets=packets)
    res = {}
    for tag, wk, rc in (("reemit", w, counters), ("plain", w.with_(recomb=None), None)):
        for timed in (False, True):
            s = rt.Solve(wk, time_march=True, counters=rc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.step(seed=7)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            s.release()
        res[tag] = dict(ms_per_step=1e3 * wall, crossings=st["crossings"], packets=st["packets"],
                        diffuse_packets=st["diffuse_packets"], march_ms=st["march_ms"],
                        kernel_ms=st["kernel_ms"],
                        residual=abs(st["emitted"] - st["absorbed"] - st["escaped"] - st["truncated"])
                        / st["emitted"])
    r, p = res["reemit"], res["plain"]
    log(f"re-emission: {r['ms_per_step']:.1f} ms/step ({r['diffuse_packets']} recombination packets, "
        f"{r['crossings']:.4g} crossings) vs {p['ms_per_step']:.1f} ms without")
    return {"workload": w.name, "grid": list(w.n), "source_packets": packets, "f_rec": w.recomb.f_rec,
            "form": "float32 march, float64 accumulators and cell update; case-A rates",
            "ms_per_step": r["ms_per_step"], "crossings_per_s": r["crossings"] / (r["ms_per_step"] * 1e-3),
            "recombination_packets": r["diffuse_packets"],
            "crossings_of_recombination_packets": r["crossings"] - p["crossings"],
            "march_ms": r["march_ms"], "march_kernel_ms": r["kernel_ms"],
            "conservation_residual": r["residual"],
            "without_reemission": {"ms_per_step": p["ms_per_step"], "march_ms": p["march_ms"],
                                   "crossings_per_s": p["crossings"] / (p["ms_per_step"] * 1e-3)}}


def periodic_leg(steps: int, packets):
    """The benchmark workload with periodic boundaries (a packet may cross 256
    cell faces along an axis) and a background field entering through the
    faces (a quarter of the sources' photon rate, a quarter as many packets,
    the sources' spectrum), float32 march; one warm-up step."""
    import numpy as np
    import torch
    from paper_1101_4127_amd import rt
    from paper_1101_4127_amd import workloads as W
    w = W.lognormal_256(packets=packets or 100_000_000)
    bg = W.Background(0.25 * float(np.sum(w.src_ndot)), w.bins.sed.copy(), w.packets // 4)
    w = w.with_(periodic=True, path_cells=256, background=bg)
    s = rt.Solve(w, time_march=True, inflight=w.packets)
    s.step(seed=500)
    torch.cuda.synchronize()
    cross = 0
    kernel_ms = march_ms = 0.0
    launches = 0
    resid = 0.0
    t0 = time.perf_counter()
    for i in range(steps):
        st = s.step(seed=501 + i)
        cross += st["crossings"]
        kernel_ms += st["kernel_ms"]
        march_ms += st["march_ms"]
        launches += st["kernel_launches"]
        resid = max(resid, abs(st["emitted"] - st["absorbed"] - st["escaped"] - st["truncated"]) / st["emitted"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.release()
    log(f"periodic + background: {1e3 * wall / steps:.1f} ms/step, {cross / wall:.4g} crossings/s, "
        f"{launches // steps} march launches per step")
    return {"workload": w.name + "_periodic_background", "grid": list(w.n), "source_packets": w.packets,
            "background_packets": bg.packets, "path_cells": 256, "steps": steps,
            "form": "float32 march, float64 accumulators and cell update",
            "ms_per_step": 1e3 * wall / steps, "crossings_per_s": cross / wall,
            "crossings_per_step": cross / steps, "march_ms_per_step": march_ms / steps,
            "march_kernel_ms_per_step": kernel_ms / steps, "march_launches_per_step": launches / steps,
            "conservation_residual": resid}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal_256")
    ap.add_argument("--packets", type=int, default=None)
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed steps of the plain float64 form")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--direct", action="store_true", help="per-packet march instead of the tiled one")
    ap.add_argument("--inflight", type=int, default=0)
    ap.add_argument("--run-len", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0)
    ap.add_argument("--bpcu", type=int, default=0)
    ap.add_argument("--serving-requests", type=int, default=512, help="0 skips the serving workload")
    ap.add_argument("--reemit-grid", type=int, default=256,
                    help="cells per axis of the re-emission workload (0 skips it)")
    ap.add_argument("--reemit-packets", type=int, default=10_000_000)
    ap.add_argument("--periodic-steps", type=int, default=1,
                    help="timed steps of the periodic-boundary + background variant (0 skips it)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the march's launch parameters by measurement first (tiled march)")
    ap.add_argument("--ceilings", action="store_true",
                    help="first measure the hardware ceilings (HBM copy/read, float64 atomics)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        raise SystemExit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()

    tiles = dict(direct=args.direct, inflight=args.inflight, run_len=args.run_len, refill_min=args.refill,
                 blocks_per_cu=args.bpcu)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
    ceil = None
    if args.ceilings:
        from paper_1101_4127_amd import ceilings
        ceil = ceilings.measure()
        log("ceilings: " + ", ".join(f"{k} {v:.4g}" for k, v in ceil.items()))
    t0 = time.perf_counter()
    work = workload(args.workload, args.packets)
    log(f"workload {work.name}: {work.ncell} cells, {len(work.src_ndot)} sources, "
        f"{work.packets} packets/step ({time.perf_counter() - t0:.1f} s to generate)")

    tuned = None
    if args.autotune:
        from paper_1101_4127_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.tune(work, fp64=False, kinds=("direct",) if args.direct else ("tiled",))
        tiles.update(tuned["config"])
        log(f"autotune: {tuned['config']} ({tuned['march_ms']:.1f} ms march, {len(tuned['trials'])} trials, "
            f"{time.perf_counter() - t0:.0f} s)")
    f32 = time_form(work, fp64=False, steps=args.steps, warmup=args.warmup, tiles=tiles)
    value = f32["crossings"] / f32["wall_s"]
    launches = max(f32["launches"], 1)
    per_launch = f32["crossings"] / launches
    avg_ms = f32["kernel_ms"] / launches
    achieved = BYTES_F32 * per_launch / (avg_ms * 1e-3) / 1e9
    log(f"float32 march: {value:.4g} crossings/s, march kernel {f32['kernel_ms'] / args.steps:.1f} ms/step "
        f"in {launches // args.steps} launches, {achieved:.0f} GB/s algorithmic, whole march "
        f"{f32['march_ms'] / args.steps:.1f} ms/step, conservation residual {f32['resid']:.2e}")
    out = {
        "metric": METRIC, "value": value, "unit": "crossings/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * f32["wall_s"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": work.name, "grid": list(work.n), "sources": len(work.src_ndot),
                   "packets_per_step": work.packets, "bins": work.bins.n_bins,
                   "form": "float32 march, float64 accumulators and cell update",
                   "march": "per-packet" if args.direct else "tiled",
                   "crossings_per_step": f32["crossings"] / args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(per_launch),
                     "kernel": KERNELS[args.direct], "bytes_per_crossing": BYTES_F32,
                     "crossings_per_launch": per_launch, "avg_launch_ms": avg_ms,
                     "whole_march_ms_per_step": f32["march_ms"] / args.steps,
                     "whole_march_gcross_per_s": f32["crossings"] / (f32["march_ms"] * 1e-3) / 1e9},
        "conservation_residual": f32["resid"],
    }
    if ceil is not None:
        out["ceilings"] = ceil
    if tuned is not None:
        out["config"]["autotuned"] = tuned["config"]
        out["config"]["autotune_trials"] = len(tuned["trials"])
    if args.fp64_steps > 0:
        f64 = time_form(work, fp64=True, steps=args.fp64_steps, warmup=1, tiles=tiles)
        v64 = f64["crossings"] / f64["wall_s"]
        l64 = max(f64["launches"], 1)
        ms64 = f64["kernel_ms"] / l64
        a64 = BYTES_F64 * (f64["crossings"] / l64) / (ms64 * 1e-3) / 1e9
        log(f"float64 plain: {v64:.4g} crossings/s, march kernel {f64['kernel_ms'] / args.fp64_steps:.1f} "
            f"ms/step, {a64:.0f} GB/s algorithmic")
        out["fp64_plain"] = {"value": v64, "unit": "crossings/s", "avg_launch_ms": ms64,
                             "achieved_gbs": a64, "bytes_per_crossing": BYTES_F64,
                             "ms_per_step": 1e3 * f64["wall_s"] / args.fp64_steps,
                             "speedup_of_fp32_form": value / v64, "conservation_residual": f64["resid"]}
    if args.serving_requests > 0:
        out["serving"] = serving_leg(args.serving_requests)
    if args.reemit_grid > 0:
        out["reemission"] = reemit_leg(args.reemit_grid, args.reemit_packets)
    if args.periodic_steps > 0:
        out["periodic_background"] = periodic_leg(args.periodic_steps, args.packets)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(work, args.cpu_seconds)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.4g} crossings/s "
            f"({time.perf_counter() - t0:.1f} s)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
