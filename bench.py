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
# VALU issue peak of MI355X for unpacked 32-bit operations: 256 compute units x
# 4 SIMDs x 16 lanes per cycle x 2.4 GHz (a wavefront instruction of 64 lanes
# every 4 cycles per SIMD; the build keeps packed float32 off)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic HBM bytes per crossing: absorber gather + four float64
# accumulator updates (H+He with heating)
BYTES_F32 = 3 * 4 + 4 * 8
BYTES_F64 = 3 * 8 + 4 * 8
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "march_traffic.json")
COUNTERS_JSON = os.path.join(ROOT, "profiles", "march_counters.json")
KERNELS = {False: "k_tmarch<float, 3, true, 8, 3, 2, false, false, false, false>", True: "k_march<float, 3, true, 8, 3, 2>"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C++ source without its comments and blank space (string and character
    literals kept whole), so that the march hash names the code alone."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            i = src.find("\n", i)
            i = n if i < 0 else i
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def march_hash() -> str:
    """Identifies the march kernel's code (its sources without comments): the
    committed counters apply while the code hashes to their march_hash."""
    h = hashlib.sha256()
    for name in ("rt_tiled.hip", "rt_march.hip", "rt_cross.h", "rt_device.h", "rt_internal.h"):
        with open(os.path.join(ROOT, "paper_1101_4127_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
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


def host_threads() -> int:
    """Host threads for the oracle: the cores this process may run on, at most
    16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model() -> str:
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return "unknown"
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return "unknown"


def oracle_step(work, threads: int):
    """One full step of the float64 oracle on `threads` host threads (the
    oracle's C routines release the interpreter lock): the packets of the
    step marched in ranges taken from a shared counter, each thread with its
    own accumulators (summed in thread order), then the cell update over
    ranges of cells.  Returns the solve (state after the step) and timings."""
    import threading
    import numpy as np
    from oracle import oracle as O
    o = O.OracleSolve(work)
    o.absorbers()
    P, nc = work.packets, work.ncell
    per = max(64, P // (threads * 64))
    ranges = [(g, min(P, g + per)) for g in range(0, P, per)]
    nxt = [0]
    lock = threading.Lock()
    accs = [np.zeros((4, nc)) for _ in range(threads)]
    leds = [[] for _ in range(threads)]

    def march(t):
        while True:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            if k >= len(ranges):
                return
            g0, g1 = ranges[k]
            _, led, _ = o.march(g0, g1, dt=work.dt_s / work.n_sub, packets=P, seed=work.seed, step_index=0,
                                acc=accs[t], absorbers=False)
            leds[t].append(led)

    t0 = time.perf_counter()
    ths = [threading.Thread(target=march, args=(t,)) for t in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    t_march = time.perf_counter() - t0
    acc = accs[0]
    for a in accs[1:]:
        acc += a
    del accs
    led = {}
    for ls in leds:
        for d in ls:
            for k, v in d.items():
                led[k] = led.get(k, 0) + v
    cells = np.array_split(np.arange(nc, dtype=np.int64), threads * 8)
    nxt[0] = 0

    def update(t):
        while True:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            if k >= len(cells):
                return
            o.update_cells(work.dt_s / work.n_sub, acc, cells[k])

    t0 = time.perf_counter()
    ths = [threading.Thread(target=update, args=(t,)) for t in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    t_upd = time.perf_counter() - t0
    o.acc = acc
    return o, led, t_march, t_upd


def field_errors(o, f, work, emitted):
    """Per-field errors of a GPU step against the oracle's: fractions
    relative to max(x, 1e-8), temperature relative, deposits and heat
    relative to max(|ref|, 1e-12 mean) after the photons the float32 form's
    bin dropping may move (e^-30 of those emitted; heat: times the largest
    photon energy above the HI threshold)."""
    import math
    import numpy as np
    from paper_1101_4127_amd import workloads as W
    out = {}
    names = ("x_HI", "x_HII", "x_HeI", "x_HeII", "x_HeIII")
    for i, n in enumerate(names):
        e = np.abs(f[1 + i] - o.x[i]) / np.maximum(o.x[i], 1e-8)
        out[n] = e
    out["T"] = np.abs(f[6] - o.T) / o.T
    drop = math.exp(-30.0) * emitted
    de = float(np.max(np.asarray(work.bins.e_ev) - W.E_TH_EV[0])) * W.EV_ERG
    for i, n in enumerate(("D_HI", "D_HeI", "D_HeII", "Q")):
        ref, allow = o.acc[i], (drop if i < 3 else drop * de)
        floor = 1e-12 * float(np.mean(np.abs(ref))) or 1e-300
        out[n] = np.maximum(np.abs(f[7 + i] - ref) - allow, 0.0) / np.maximum(np.abs(ref), floor)
    return {k: {"max": float(np.max(v)), "p99": float(np.percentile(v, 99))} for k, v in out.items()}


def oracle_leg(work, packets: int):
    """The float64 oracle on a bounded sample of the benchmark step (the same
    gas, sources and seed, `packets` packets: a fresh solve's first step) on
    the host's cores, and the same step of the float32-march form on the GPU,
    compared field by field.  Returns (cpu_baseline, accuracy)."""
    import torch
    from paper_1101_4127_amd import rt
    w = work.with_(packets=packets)
    threads = host_threads()
    o, led, t_march, t_upd = oracle_step(w, threads)
    s = rt.Solve(w, fp64=False, inflight=w.packets)
    st = s.step(seed=w.seed)
    f = s.fetch()
    s.release()
    torch.cuda.synchronize()
    acc = field_errors(o, f, w, st["emitted"])
    cross = led["crossings"]
    model = cpu_model()
    cpu = {
        "value": cross / (t_march + t_upd), "unit": "crossings/s", "cores": threads, "kind": "oracle",
        "cpu_model": model,
        "sample": (f"one full step of the benchmark gas and sources with {packets} packets ({cross} crossings, "
                   f"{cross / packets:.1f} per packet; the metric's step has {work.packets}): march "
                   f"{t_march:.1f} s + update of all {w.ncell} cells {t_upd:.1f} s on {threads} threads of "
                   f"{model}; float64 C oracle"),
        "march_crossings_per_s": cross / t_march, "update_cells_per_s": w.ncell / t_upd,
    }
    log(f"oracle: {cpu['value']:.4g} crossings/s on {threads} threads ({model}); march {t_march:.1f} s, "
        f"update {t_upd:.1f} s")
    accuracy = {"workload": w.name, "packets": packets, "against": "float64 oracle, same inputs and seed",
                "form": "float32 march, float64 accumulators and cell update", "fields": acc,
                "crossings_gpu": st["crossings"], "crossings_oracle": cross}
    log("accuracy vs oracle: " + ", ".join(f"{k} {v['max']:.2e}" for k, v in acc.items()))
    return cpu, accuracy


def counted_config(args) -> bool:
    """The committed counter runs are of the default benchmark: the 256^3
    workload, its packet count, the tiled march and default launch
    parameters.  Other workloads and launch shapes get no counter figures."""
    return (args.workload == "lognormal_256" and args.packets is None and not args.direct
            and args.inflight == 0 and args.run_len == 0 and args.refill == 0 and args.bpcu == 0)


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


def counters_for():
    """VALU counters of the march kernel per crossing from committed rocprofv3
    runs, or None when they were taken on a different march kernel."""
    if not os.path.exists(COUNTERS_JSON):
        return None
    with open(COUNTERS_JSON) as f:
        t = json.load(f)
    return t if t.get("march_hash") == march_hash() else None


# the server's fused calls: up to 256 solves, each sub-step's tile passes cut
# short after 4 by a finishing pass (the serving solves' packets cross few
# tiles; the passes after the fourth carry little work each)
SERVE_SLOTS = 256
SERVE_FINISH = 4


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
    srv = serve.Server(max_slots=SERVE_SLOTS, fp64=False, graph=True, keep_fields=False, finish_pass=SERVE_FINISH)
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
    srv = serve.Server(max_slots=SERVE_SLOTS, fp64=False, graph=True, keep_fields=True, finish_pass=SERVE_FINISH)
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
        "form": f"float32 march, float64 accumulators; fused tiled steps of up to {SERVE_SLOTS} solves (finishing "
                f"pass after {SERVE_FINISH} tile passes) replayed as a hipGraph",
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


def roofline(per_launch, avg_ms, achieved, args, f32):
    """The march kernel against its bound.  The kernel issues VALU
    instructions ~85 % of its time (committed counters), so its roofline is
    the VALU issue rate: VALU lane-operations per crossing (wavefront
    instructions x 64, from the counters) x crossings per launch / launch
    time, against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  Beside it the HBM
    roofline of the algorithmic bytes per crossing (absorber gather + float64
    accumulator updates) against the nominal 8 TB/s and the measured copy
    peak, and the HBM bytes the counters saw."""
    counted = counted_config(args)
    traffic = traffic_for(per_launch) if counted else None
    ctr = counters_for() if counted else None
    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "bytes_per_crossing": BYTES_F32, "traffic": traffic}
    if traffic is not None:
        hbm["measured_gbs"] = traffic / (avg_ms * 1e-3) / 1e9
        hbm["measured_frac"] = hbm["measured_gbs"] / HBM_PEAK_GBS
    out = {"kernel": KERNELS[args.direct], "crossings_per_launch": per_launch, "avg_launch_ms": avg_ms,
           "whole_march_ms_per_step": f32["march_ms"] / args.steps,
           "whole_march_gcross_per_s": f32["crossings"] / (f32["march_ms"] * 1e-3) / 1e9}
    if ctr is not None:
        ops = 64.0 * ctr["valu_insts_per_crossing"] * per_launch / (avg_ms * 1e-3) / 1e12
        out.update({"bound": "alu", "achieved": ops, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                    "frac": ops / VALU_PEAK_TOPS, "traffic": traffic,
                    "valu_insts_per_crossing": ctr["valu_insts_per_crossing"],
                    "lane_utilisation": ctr.get("lane_utilisation"), "hbm": hbm})
    else:
        out.update({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "hbm": hbm})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal_256")
    ap.add_argument("--packets", type=int, default=None)
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed steps of the plain float64 form")
    ap.add_argument("--oracle-packets", type=int, default=2_000_000,
                    help="packets of the step the oracle runs (CPU baseline and per-field errors)")
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
        "roofline": roofline(per_launch, avg_ms, achieved, args, f32),
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
        out["cpu_baseline"], out["accuracy_vs_oracle"] = oracle_leg(work, args.oracle_packets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
