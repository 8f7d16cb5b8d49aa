"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rt_mcrt.h declares, its structs have the layout the
binding assumes, and the host-only calls validate their arguments."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1101_4127_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt_mcrt.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rt.LIB_PATH):
        from paper_1101_4127_amd import build
        build.build()
    return rt.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", rt.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (rt_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)
    assert set(rt.SIGNATURES) == set(names)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rt_grid_desc), offsetof(rt_grid_desc, solve_id),
         offsetof(rt_grid_desc, trace_stride), offsetof(rt_grid_desc, run_len),
         offsetof(rt_grid_desc, inflight), sizeof(rt_step_stats),
         offsetof(rt_step_stats, crossings), offsetof(rt_step_stats, nonfinite),
         offsetof(rt_step_stats, errors), offsetof(rt_step_stats, march_ms),
         offsetof(rt_step_stats, kernel_launches), offsetof(rt_grid_desc, path_cells),
         offsetof(rt_step_stats, diffuse_packets));
  return 0;
}}""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [C.sizeof(rt.GridDesc), rt.GridDesc.solve_id.offset, rt.GridDesc.trace_stride.offset,
                    rt.GridDesc.run_len.offset, rt.GridDesc.inflight.offset,
                    C.sizeof(rt.StepStats), rt.StepStats.crossings.offset, rt.StepStats.nonfinite.offset,
                    rt.StepStats.errors.offset, rt.StepStats.march_ms.offset,
                    rt.StepStats.kernel_launches.offset, rt.GridDesc.path_cells.offset,
                    rt.StepStats.diffuse_packets.offset]


def test_defaults_and_strerror(L):
    d = rt.rt_desc_defaults()
    assert list(d.n) == [1, 1, 1] and d.n_bins == 1 and d.tau_kill == 30.0 and d.n_chem == 8
    for st in (rt.RT_OK, rt.RT_EINVAL, rt.RT_ENOMEM, rt.RT_EDEVICE, rt.RT_ESTATE, rt.RT_EOVERFLOW,
               rt.RT_EINTERNAL):
        assert rt.rt_strerror(st)
    assert rt.rt_strerror(-99) == "unknown status"


def test_workspace_bytes_scales_and_validates(L):
    d = rt.rt_desc_defaults()
    d.flags = rt.RT_DIRECT_MARCH
    d.n[0] = d.n[1] = d.n[2] = 64
    d.cell_cm = 1e21
    b64 = rt.rt_workspace_bytes(d, 10)
    d.n[0] = d.n[1] = d.n[2] = 128
    b128 = rt.rt_workspace_bytes(d, 10)
    assert 7.5 < b128 / b64 < 8.5
    d.flags = rt.RT_FP64 | rt.RT_DIRECT_MARCH
    assert rt.rt_workspace_bytes(d, 10) > b128
    # invalid descriptions
    for field, bad in (("n_bins", 0), ("n_bins", 9), ("n_bins", 17), ("tau_kill", 0.0), ("n_sub", 0), ("n_chem", 0),
                       ("cell_cm", -1.0), ("brick_log2", 4), ("wave_chunk", 100), ("refill_min", 65),
                       ("flags", 0x40), ("flags", rt.RT_RECOMB | rt.RT_DIRECT_MARCH),
                       ("flags", rt.RT_PERIODIC | rt.RT_DIRECT_MARCH), ("path_cells", -1), ("path_cells", 2047), ("trace_stride", -1), ("brick_log2", 2), ("run_len", 10),
                       ("run_len", 65537), ("park_lanes", -1), ("park_lanes", 65), ("inflight", -1), ("inflight", 1 << 31)):
        e = rt.rt_desc_defaults()
        setattr(e, field, bad)
        with pytest.raises(rt.RTError) as ex:
            rt.rt_workspace_bytes(e, 1)
        assert ex.value.status == rt.RT_EINVAL, field
    # re-emission: counters, the spectrum table and a record per cell at least
    e = rt.rt_desc_defaults()
    e.n[0] = e.n[1] = e.n[2] = 64
    e.cell_cm = 1e21
    e.inflight = 1000
    plain = rt.rt_workspace_bytes(e, 1)
    e.flags = rt.RT_RECOMB
    assert rt.rt_workspace_bytes(e, 1) >= plain + 64 ** 3 * (8 + 32)
    e = rt.rt_desc_defaults()
    e.n[1] = 1025
    with pytest.raises(rt.RTError):
        rt.rt_workspace_bytes(e, 1)
    # bin counts: 1 or 8 only
    for nb in range(2, 8):
        e = rt.rt_desc_defaults()
        e.n_bins = nb
        for j in range(nb):
            e.e_bin_ev[j] = 14.0 + j
        with pytest.raises(rt.RTError) as ex:
            rt.rt_workspace_bytes(e, 1)
        assert ex.value.status == rt.RT_EINVAL, nb
    # H+He with 8 bins: the threshold-aligned table only, in either march
    e = rt.rt_desc_defaults()
    e.n_bins = 8
    e.y_he = 0.08
    for j in range(8):
        e.e_bin_ev[j] = 60.0 + j
        e.sigma_cm2[0][j] = 1e-19
        e.sigma_cm2[1][j] = 1e-19 if j >= 3 else 0.0
        e.sigma_cm2[2][j] = 1e-19 if j >= 5 else 0.0
    assert rt.rt_workspace_bytes(e, 1) > 0
    e.sigma_cm2[2][4] = 1e-19                     # HeII in bin 4: not the aligned layout
    for flags in (0, rt.RT_DIRECT_MARCH):
        e.flags = flags
        with pytest.raises(rt.RTError) as ex:
            rt.rt_workspace_bytes(e, 1)
        assert ex.value.status == rt.RT_EINVAL
    # a cross-section above zero below its threshold is rejected
    e = rt.rt_desc_defaults()
    e.e_bin_ev[0] = 20.0
    e.sigma_cm2[1][0] = 1e-18          # HeI below 24.6 eV
    with pytest.raises(rt.RTError):
        rt.rt_workspace_bytes(e, 1)


def test_tiled_workspace_holds_one_record_per_packet_in_flight(L):
    """The tiled march's workspace grows by a fixed record size per packet in
    flight (float32 H+He, 8 bins: 80-byte records on a 128-byte stride, so no
    record straddles a cache line, plus three list words)."""
    d = rt.rt_desc_defaults()
    d.n[0] = d.n[1] = d.n[2] = 64
    d.cell_cm = 1e21
    d.y_he = 0.08
    d.n_bins = 8
    for j in range(8):
        d.e_bin_ev[j] = 60.0 + j
    d.inflight = 1 << 20
    a = rt.rt_workspace_bytes(d, 10)
    d.inflight = 1 << 21
    b = rt.rt_workspace_bytes(d, 10)
    per = (b - a) / (1 << 20)
    assert 128 + 12 <= per <= 128 + 12 + 16 * 2      # record + lists (+ runs of 2048)
    d.flags = rt.RT_FP64
    c = rt.rt_workspace_bytes(d, 10)
    assert c > b
    # the direct march needs none of it
    d.flags = rt.RT_DIRECT_MARCH
    assert rt.rt_workspace_bytes(d, 10) < a


def test_init_rejects_bad_arguments_before_touching_the_device(L):
    d = rt.rt_desc_defaults()
    h = C.c_void_p()
    # misaligned or null workspace, null fields: EINVAL without a device call
    assert L.rt_init_grid(C.byref(d), None, 1 << 20, 1, 1, 1, 1, 0, None, C.byref(h)) == rt.RT_EINVAL
    assert L.rt_init_grid(C.byref(d), 0x1001, 1 << 20, 1, 256, 256, 256, 0, None, C.byref(h)) == rt.RT_EINVAL
    assert L.rt_init_grid(C.byref(d), 0x1000, 1 << 20, 1, None, 256, 256, 0, None, C.byref(h)) == rt.RT_EINVAL
    # too small a workspace
    assert L.rt_init_grid(C.byref(d), 0x1000, 16, 1, 256, 256, 256, 0, None, C.byref(h)) == rt.RT_ENOMEM
    # calls on a null handle
    assert L.rt_step(None, 1.0, 1, 1, None) == rt.RT_EINVAL
    assert L.rt_release(None) == rt.RT_EINVAL
    assert L.rt_fetch_fields(None, 1, None, 0, 1) == rt.RT_EINVAL


def test_batch_arguments_are_checked_before_the_device(L):
    out = C.c_size_t(0)
    shape = rt.rt_desc_defaults()
    for bad in (0, rt.RT_MAX_BATCH + 1):
        assert L.rt_batch_workspace_bytes(bad, C.byref(shape), 1000, 8, C.byref(out)) == rt.RT_EINVAL
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 1000, 8, None) == rt.RT_EINVAL
    assert L.rt_batch_workspace_bytes(1, None, 1000, 8, C.byref(out)) == rt.RT_EINVAL
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 0, 8, C.byref(out)) == rt.RT_EINVAL
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 1000, 0, C.byref(out)) == rt.RT_EINVAL
    assert L.rt_batch_workspace_bytes(64, C.byref(shape), 1000, 8, C.byref(out)) == rt.RT_OK
    big = out.value
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 1000, 8, C.byref(out)) == rt.RT_OK
    assert 0 < out.value < big
    # records for the packets of one round, lists for the tiles
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 1 << 20, 8, C.byref(out)) == rt.RT_OK
    more = out.value
    assert L.rt_batch_workspace_bytes(1, C.byref(shape), 1 << 21, 8, C.byref(out)) == rt.RT_OK
    per = (out.value - more) / (1 << 20)
    assert 64 + 12 <= per <= 64 + 12 + 16 * 2       # one-bin float32 record + lists (+ runs)
    bad_shape = rt.rt_desc_defaults()
    bad_shape.n_bins = 3
    assert L.rt_batch_workspace_bytes(1, C.byref(bad_shape), 1000, 8, C.byref(out)) == rt.RT_EINVAL
    for fin in (-2, rt.RT_MAX_FINISH_PASS + 1):
        bad_shape = rt.rt_desc_defaults()
        bad_shape.finish_pass = fin
        assert L.rt_batch_workspace_bytes(1, C.byref(bad_shape), 1000, 8, C.byref(out)) == rt.RT_EINVAL
        assert L.rt_workspace_bytes(C.byref(bad_shape), 1, C.byref(out)) == rt.RT_EINVAL
    for fin in (-1, 0, 1, rt.RT_MAX_FINISH_PASS):
        ok_shape = rt.rt_desc_defaults()
        ok_shape.finish_pass = fin
        assert L.rt_workspace_bytes(C.byref(ok_shape), 1, C.byref(out)) == rt.RT_OK
    b = C.c_void_p()
    s = C.byref(shape)
    assert L.rt_batch_init(0, s, 1000, 8, 0x1000, 1 << 30, 0x10, 0, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(rt.RT_MAX_BATCH + 1, s, 1000, 8, 0x1000, 1 << 30, 0x10, 0, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, 0x1000, 1 << 30, None, rt.RT_BATCH_GRAPH, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, 0x1000, 1 << 30, 0x10, 0x2, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, 0x1001, 1 << 30, 0x10, 0, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, None, 1 << 30, 0x10, 0, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, 0x1000, 16, 0x10, 0, C.byref(b)) == rt.RT_ENOMEM
    assert L.rt_batch_init(4, None, 1000, 8, 0x1000, 1 << 30, 0x10, 0, C.byref(b)) == rt.RT_EINVAL
    assert L.rt_batch_init(4, s, 1000, 8, 0x1000, 1 << 30, 0x10, 0, None) == rt.RT_EINVAL
    assert L.rt_step_many(None, None, 1, None, None, None, None) == rt.RT_EINVAL
    assert L.rt_batch_wait(None, 0, None) == rt.RT_EINVAL
    assert L.rt_batch_release(None) == rt.RT_EINVAL


def test_ceilings_library_exports_its_header():
    """The microbenchmark library (measured ceilings of the march) loads and
    exports every function include/rt_ceilings.h declares; invalid arguments
    are refused before any device call."""
    from paper_1101_4127_amd import ceilings
    if not os.path.exists(ceilings.LIB_PATH):
        from paper_1101_4127_amd import build
        build.build()
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "rt_ceilings.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(rtc_[a-z0-9_]+)\s*\(", text)))
    assert len(names) == 4 and set(names) == set(ceilings.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", ceilings.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n
    L = ceilings.lib()
    r = C.c_double(0)
    assert L.rtc_hbm_copy(None, None, 16, 1, None, C.byref(r)) == -1
    assert L.rtc_hbm_copy(0x1000, 0x2000, 17, 1, None, C.byref(r)) == -1
    assert L.rtc_global_atomic_f64(0x1000, 3, 1, None, C.byref(r)) == -1       # not a power of two
    assert L.rtc_lds_atomic_f64(5, 0, 1, 0x1000, None, C.byref(r)) == -1       # acc > 4
