"""rt_init_grid_static (the solve's workspace in the library's static
per-device array, for callers that cannot allocate device memory) against
rt_init_grid with a caller's workspace: the same packets and the same fields,
on two static solves in a row, the second on a smaller grid."""
import numpy as np
import pytest

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


def fields_of(work, dtype):
    import torch
    f = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=dtype, device="cuda").contiguous()
    return f(work.n_h), f(np.asarray(work.x).reshape(5, -1)), f(work.temp)


def run(work, static, seeds, trace_n=400, trace_len=64):
    """Two steps through the C ABI; returns (ledgers, fields, traces)."""
    import torch
    from paper_1101_4127_amd import rt
    desc = rt.desc_from_workload(work, trace_packets=trace_n, trace_len=trace_len,
                                 inflight=-(-work.packets // work.n_sub))
    nbytes = rt.rt_workspace_bytes(desc, len(work.src_ndot))
    nh, x, t = fields_of(work, torch.float64)
    if static:
        assert nbytes <= rt.RT_STATIC_WORKSPACE_BYTES
        h = rt.rt_init_grid_static(desc, len(work.src_ndot), nh, x, t)
    else:
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = rt.rt_init_grid(desc, ws, len(work.src_ndot), nh, x, t)
    rt.rt_add_sources(h, work.src_ijk, work.src_ndot, work.src_sed, work.src_flags)
    leds = [rt.rt_step(h, work.dt_s, work.packets, s, True) for s in seeds]
    f = rt.rt_fetch_fields(h, rt.RT_F_STATE, work.ncell)
    tr = rt.rt_fetch_trace(h, trace_n, trace_len)
    rt.rt_release(h)
    torch.cuda.synchronize()
    return leds, f, tr


def same(a, b, work):
    la, fa, ta = a
    lb, fb, tb = b
    for x, y in zip(la, lb):
        for k in ("packets", "crossings", "n_escaped", "n_truncated"):
            assert x[k] == y[k], k
        for k in ("emitted", "absorbed", "escaped", "truncated"):
            assert abs(x[k] - y[k]) <= 1e-12 * x["emitted"], k
    assert PT.traces_equal(ta, tb)
    # float64 both ways; the deposits may be summed in another order
    for k in range(1, 7):
        assert np.max(PT.frac_err(fb[k], fa[k], 1e-300)) <= 1e-12, k
    for k in range(7, 11):
        assert np.max(PT.deposit_err(fb[k], fa[k])) <= 1e-12, k


def test_static_workspace_equals_caller_workspace():
    from paper_1101_4127_amd import rt
    big = W.small_mixed(n=20, n_src=4, packets=8000, fp64=True)
    small = W.small_mixed(n=12, n_src=3, packets=3000, fp64=True, seed=9)
    for work, seeds in ((big, [3, 4]), (small, [5, 6])):
        print(f"static workspace: {work.n}, {work.packets} packets", flush=True)
        ref = run(work, False, seeds)
        got = run(work, True, seeds)
        same(ref, got, work)


def test_static_workspace_refusals():
    import torch
    from paper_1101_4127_amd import rt
    w = W.small_mixed(n=12, n_src=3, packets=3000, fp64=True, seed=9)
    nh, x, t = fields_of(w, torch.float64)
    desc = rt.desc_from_workload(w, inflight=w.packets)
    h = rt.rt_init_grid_static(desc, len(w.src_ndot), nh, x, t)
    with pytest.raises(rt.RTError) as e:                  # the device's static solve is taken
        rt.rt_init_grid_static(desc, len(w.src_ndot), nh, x, t)
    assert e.value.status == rt.RT_ESTATE
    rt.rt_release(h)
    big = rt.desc_from_workload(w, inflight=1 << 22)      # records alone exceed the static array
    assert rt.rt_workspace_bytes(big, len(w.src_ndot)) > rt.RT_STATIC_WORKSPACE_BYTES
    with pytest.raises(rt.RTError) as e:
        rt.rt_init_grid_static(big, len(w.src_ndot), nh, x, t)
    assert e.value.status == rt.RT_ESCRATCH
    timed = rt.desc_from_workload(w, inflight=w.packets, time_march=True)
    with pytest.raises(rt.RTError) as e:
        rt.rt_init_grid_static(timed, len(w.src_ndot), nh, x, t)
    assert e.value.status == rt.RT_EINVAL
    h = rt.rt_init_grid_static(desc, len(w.src_ndot), nh, x, t)   # free again after the refusals
    rt.rt_release(h)
