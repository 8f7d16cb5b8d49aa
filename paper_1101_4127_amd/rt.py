"""Python binding of the C ABI in include/rt_mcrt.h (librt_mcrt.so).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the ABI.  PyTorch provides device memory (the workspace and the input
fields) and the stream.  Importing works without a GPU; any call that needs
the library raises if it has not been built.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librt_mcrt.so")

RT_MAX_BINS = 16
RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ESTATE, RT_EOVERFLOW, RT_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
RT_ESCRATCH = -7
RT_STATIC_WORKSPACE_BYTES = 64 << 20
RT_ISOTHERMAL, RT_FP64, RT_TIME_MARCH, RT_DIRECT_MARCH, RT_RECOMB, RT_PERIODIC = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
RT_MAX_PATH_CELLS = 2046
RT_MAX_FINISH_PASS = 65535
RT_SRC_CORNER_OCTANT = 0x1
RT_TRACE_HDR = 8
RT_FATE_TRUNC, RT_FATE_ESCAPE, RT_FATE_PATH = 1, 2, 3
RT_MAX_BATCH = 256
RT_BATCH_GRAPH = 0x1

FIELDS = ("nh", "x_hi", "x_hii", "x_hei", "x_heii", "x_heiii", "temp", "d_hi", "d_hei", "d_heii", "q",
          "r_hii", "r_heii", "r_heiii")
F = {name: 1 << i for i, name in enumerate(FIELDS)}
RT_F_ALL = (1 << len(FIELDS)) - 1
RT_F_STATE = (1 << 11) - 1          # every field but the recombination counters
RT_MAX_MILNE_T = 512


class GridDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("cell_cm", C.c_double), ("y_he", C.c_double),
        ("n_bins", C.c_int32), ("e_bin_ev", C.c_double * RT_MAX_BINS),
        ("sigma_cm2", (C.c_double * RT_MAX_BINS) * 3), ("redshift", C.c_double),
        ("tau_kill", C.c_double), ("n_sub", C.c_int32), ("n_chem", C.c_int32),
        ("flags", C.c_uint32), ("solve_id", C.c_uint64), ("step_index0", C.c_uint64),
        ("brick_log2", C.c_int32), ("wave_chunk", C.c_int32), ("refill_min", C.c_int32),
        ("blocks_per_cu", C.c_int32), ("trace_packets", C.c_int32), ("trace_len", C.c_int32),
        ("trace_stride", C.c_int32), ("run_len", C.c_int32), ("park_lanes", C.c_int32),
        ("inflight", C.c_int64), ("path_cells", C.c_int32), ("finish_pass", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [
        ("emitted", C.c_double), ("absorbed", C.c_double), ("escaped", C.c_double),
        ("truncated", C.c_double), ("crossings", C.c_int64), ("packets", C.c_int64),
        ("n_escaped", C.c_int64), ("n_truncated", C.c_int64), ("substeps", C.c_int64),
        ("nonfinite", C.c_uint32), ("errors", C.c_uint32), ("march_ms", C.c_double),
        ("kernel_ms", C.c_double), ("kernel_launches", C.c_int64),
        ("diffuse_emitted", C.c_double), ("diffuse_packets", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point
_VP, _I32, _I64, _U32, _U64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
SIGNATURES = {
    "rt_desc_defaults": (_I32, [C.POINTER(GridDesc)]),
    "rt_workspace_bytes": (_I32, [C.POINTER(GridDesc), _I64, C.POINTER(C.c_size_t)]),
    "rt_init_grid": (_I32, [C.POINTER(GridDesc), _VP, C.c_size_t, _I64, _VP, _VP, _VP, _I32, _VP,
                            C.POINTER(_VP)]),
    "rt_init_grid_static": (_I32, [C.POINTER(GridDesc), _I64, _VP, _VP, _VP, _I32, _VP, C.POINTER(_VP)]),
    "rt_add_sources": (_I32, [_VP, _I32, _VP, _VP, _VP, _U32]),
    "rt_step": (_I32, [_VP, _D, _I64, _U64, C.POINTER(StepStats)]),
    "rt_read_stats": (_I32, [_VP, C.POINTER(StepStats)]),
    "rt_fetch_fields": (_I32, [_VP, _U32, _VP, _I32, _I32]),
    "rt_fetch_trace": (_I32, [_VP, _VP, _I64]),
    "rt_trace_rays": (_I32, [_VP, _I32, _VP, _VP, _I32, _VP, _VP, _VP]),
    "rt_get_step_index": (_I32, [_VP, C.POINTER(_U64)]),
    "rt_set_recombination": (_I32, [_VP, _D, _I32, _D, _D, _VP, _VP, _I32]),
    "rt_set_background": (_I32, [_VP, _D, _VP, _I64]),
    "rt_release": (_I32, [_VP]),
    "rt_batch_workspace_bytes": (_I32, [_I32, C.POINTER(GridDesc), _I64, _I64, C.POINTER(C.c_size_t)]),
    "rt_batch_init": (_I32, [_I32, C.POINTER(GridDesc), _I64, _I64, _VP, C.c_size_t, _VP, _U32, C.POINTER(_VP)]),
    "rt_step_many": (_I32, [_VP, C.POINTER(_VP), _I32, C.POINTER(_D), C.POINTER(_I64), C.POINTER(_U64),
                            C.POINTER(StepStats)]),
    "rt_batch_wait": (_I32, [_VP, _I32, C.POINTER(StepStats)]),
    "rt_batch_release": (_I32, [_VP]),
    "rt_strerror": (C.c_char_p, [_I32]),
}

_lib = None


class RTError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {rt_strerror(status)} (status {status})")
        self.status = status


def lib():
    """Load the HIP library; raise if it was not built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1101_4127_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, status: int):
    if status != RT_OK:
        raise RTError(fn, status)


def rt_strerror(status: int) -> str:
    return lib().rt_strerror(int(status)).decode()


def rt_desc_defaults() -> GridDesc:
    d = GridDesc()
    _check("rt_desc_defaults", lib().rt_desc_defaults(C.byref(d)))
    return d


def rt_workspace_bytes(desc: GridDesc, max_sources: int) -> int:
    out = C.c_size_t(0)
    _check("rt_workspace_bytes", lib().rt_workspace_bytes(C.byref(desc), int(max_sources), C.byref(out)))
    return int(out.value)


def _ptr(t) -> int:
    return int(t.data_ptr())


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def rt_init_grid(desc: GridDesc, workspace, max_sources: int, nh, x, temp, stream=None):
    """workspace: uint8 device tensor; nh (ncell,), x (5, ncell), temp (ncell,) device
    tensors of one dtype (float64 or float32), contiguous, natural order."""
    import torch
    f64 = nh.dtype == torch.float64
    for t in (nh, x, temp):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == nh.dtype):
            raise ValueError("fields must be contiguous device tensors of one dtype")
    h = C.c_void_p()
    st = lib().rt_init_grid(C.byref(desc), _ptr(workspace), workspace.numel() * workspace.element_size(),
                            int(max_sources), _ptr(nh), _ptr(x), _ptr(temp), int(f64),
                            _stream_ptr(stream), C.byref(h))
    _check("rt_init_grid", st)
    return h


def rt_init_grid_static(desc: GridDesc, max_sources: int, nh, x, temp, stream=None):
    """rt_init_grid with the library's static per-device workspace (allocates
    nothing); the same field tensors as rt_init_grid."""
    import torch
    f64 = nh.dtype == torch.float64
    for t in (nh, x, temp):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == nh.dtype):
            raise ValueError("fields must be contiguous device tensors of one dtype")
    h = C.c_void_p()
    st = lib().rt_init_grid_static(C.byref(desc), int(max_sources), _ptr(nh), _ptr(x), _ptr(temp), int(f64),
                                   _stream_ptr(stream), C.byref(h))
    _check("rt_init_grid_static", st)
    return h


def rt_add_sources(h, ijk, ndot, sed, src_flags: int = 0):
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    ndot = np.ascontiguousarray(ndot, dtype=np.float64).reshape(-1)
    sed = np.ascontiguousarray(sed, dtype=np.float64).reshape(len(ndot), -1)
    _check("rt_add_sources", lib().rt_add_sources(h, len(ndot), ijk.ctypes.data, ndot.ctypes.data,
                                                  sed.ctypes.data, int(src_flags)))


def rt_step(h, dt_s: float, n_packets: int, seed: int, stats: bool = True) -> Optional[dict]:
    s = StepStats()
    _check("rt_step", lib().rt_step(h, float(dt_s), int(n_packets), int(seed),
                                    C.byref(s) if stats else None))
    return s.as_dict() if stats else None


def rt_read_stats(h) -> dict:
    s = StepStats()
    _check("rt_read_stats", lib().rt_read_stats(h, C.byref(s)))
    return s.as_dict()


def rt_fetch_fields(h, mask: int, ncell: int, as_fp64: bool = True, device_out=None) -> np.ndarray:
    """Fields in mask bit order as an array (nfields, ncell); with device_out
    (a device tensor of nfields*ncell elements) the copy stays on the device."""
    nf = bin(mask).count("1")
    if device_out is not None:
        _check("rt_fetch_fields", lib().rt_fetch_fields(h, int(mask), _ptr(device_out), 1, int(as_fp64)))
        return device_out.view(nf, ncell)
    out = np.empty((nf, ncell), dtype=np.float64 if as_fp64 else np.float32)
    _check("rt_fetch_fields", lib().rt_fetch_fields(h, int(mask), out.ctypes.data, 0, int(as_fp64)))
    return out


def rt_fetch_trace(h, count: int, trace_len: int) -> np.ndarray:
    out = np.zeros((count, RT_TRACE_HDR + trace_len), dtype=np.int32)
    _check("rt_fetch_trace", lib().rt_fetch_trace(h, out.ctypes.data, int(count)))
    return out


def rt_trace_rays(h, origins, dirs, max_len: int):
    """origins, dirs: (m, 3) int32 device tensors; returns device tensors
    (cells (m, max_len), count (m,), face (m,))."""
    import torch
    m = origins.shape[0]
    dev = origins.device
    cells = torch.full((m, max(max_len, 1)), -1, dtype=torch.int32, device=dev)
    count = torch.zeros(m, dtype=torch.int32, device=dev)
    face = torch.zeros(m, dtype=torch.int32, device=dev)
    _check("rt_trace_rays", lib().rt_trace_rays(h, int(m), _ptr(origins.contiguous()), _ptr(dirs.contiguous()),
                                                int(max_len), _ptr(cells), _ptr(count), _ptr(face)))
    return cells, count, face


def rt_get_step_index(h) -> int:
    v = C.c_uint64(0)
    _check("rt_get_step_index", lib().rt_get_step_index(h, C.byref(v)))
    return int(v.value)


def rt_set_recombination(h, f_rec: float, log10_t0: float, dlog10_t: float, milne, counters=None):
    """Threshold, spectrum table [3][n_t][n_bins] (host) and optional initial
    counters (device tensor [species][ncell], float64 or float32)."""
    tab = np.ascontiguousarray(milne, dtype=np.float64)
    if tab.ndim != 3 or tab.shape[0] != 3:
        raise ValueError("milne table must be [3][n_t][n_bins]")
    fp64 = 1
    cp = None
    if counters is not None:
        import torch
        fp64 = 1 if counters.dtype == torch.float64 else 0
        cp = _ptr(counters)
    _check("rt_set_recombination", lib().rt_set_recombination(
        h, float(f_rec), int(tab.shape[1]), float(log10_t0), float(dlog10_t),
        tab.ctypes.data_as(C.c_void_p), cp, fp64))


def rt_set_background(h, ndot: float, sed, packets_per_step: int):
    """Background field through the box faces: photons/s, spectrum, packets per step."""
    row = np.ascontiguousarray(sed, dtype=np.float64)
    _check("rt_set_background", lib().rt_set_background(h, float(ndot), row.ctypes.data_as(C.c_void_p),
                                                         int(packets_per_step)))


def rt_release(h):
    _check("rt_release", lib().rt_release(h))


def rt_batch_workspace_bytes(max_solves: int, shape: GridDesc, max_round_packets: int, max_tiles: int) -> int:
    out = C.c_size_t(0)
    _check("rt_batch_workspace_bytes", lib().rt_batch_workspace_bytes(
        int(max_solves), C.byref(shape), int(max_round_packets), int(max_tiles), C.byref(out)))
    return int(out.value)


def rt_batch_init(max_solves: int, shape: GridDesc, max_round_packets: int, max_tiles: int, workspace, stream,
                  flags: int = RT_BATCH_GRAPH):
    b = C.c_void_p()
    _check("rt_batch_init", lib().rt_batch_init(int(max_solves), C.byref(shape), int(max_round_packets),
                                                int(max_tiles), _ptr(workspace),
                                                workspace.numel() * workspace.element_size(),
                                                _stream_ptr(stream), int(flags), C.byref(b)))
    return b


def rt_step_many(b, handles, dt_s, n_packets, seeds, stats: bool = False):
    """One step of every solve in handles (fused); returns a list of ledger
    dicts when stats is true."""
    n = len(handles)
    hs = (_VP * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    dts = (_D * n)(*[float(v) for v in dt_s])
    pks = (_I64 * n)(*[int(v) for v in n_packets])
    sds = (_U64 * n)(*[int(v) for v in seeds])
    st = (StepStats * n)() if stats else None
    _check("rt_step_many", lib().rt_step_many(b, hs, int(n), dts, pks, sds, st))
    return [x.as_dict() for x in st] if stats else None


def rt_batch_wait(b, n: int):
    """Ledger dicts of the n solves of the batch's last fused call (waits for it)."""
    st = (StepStats * n)()
    _check("rt_batch_wait", lib().rt_batch_wait(b, int(n), st))
    return [x.as_dict() for x in st]


def rt_batch_release(b):
    _check("rt_batch_release", lib().rt_batch_release(b))


# ----------------------------------------------------------------------------
# Convenience owner of one solve: torch device memory for the workspace and
# the initial fields, built from a workload description.
# ----------------------------------------------------------------------------
def desc_from_workload(work, *, fp64: Optional[bool] = None, brick_log2: int = -1, wave_chunk: int = 0,
                       refill_min: int = 0, blocks_per_cu: int = 0, trace_packets: int = 0,
                       trace_len: int = 0, trace_stride: int = 1, time_march: bool = False,
                       direct: bool = False, run_len: int = 0, inflight: int = 0,
                       park_lanes: int = 0, finish_pass: int = 0) -> GridDesc:
    d = rt_desc_defaults()
    for a in range(3):
        d.n[a] = int(work.n[a])
    d.cell_cm = float(work.cell_cm)
    d.y_he = float(work.y_he)
    nb = work.bins.n_bins
    d.n_bins = nb
    for j in range(nb):
        d.e_bin_ev[j] = float(work.bins.e_ev[j])
        for s in range(3):
            d.sigma_cm2[s][j] = float(work.bins.sigma[s, j])
    d.redshift = float(work.redshift)
    d.tau_kill = float(work.tau_kill)
    d.n_sub = int(work.n_sub)
    d.n_chem = int(work.n_chem)
    f64 = bool(work.flags & 0x2) if fp64 is None else bool(fp64)
    d.flags = ((RT_ISOTHERMAL if work.flags & 0x1 else 0) | (RT_FP64 if f64 else 0)
               | (RT_TIME_MARCH if time_march else 0) | (RT_DIRECT_MARCH if direct else 0)
               | (RT_RECOMB if getattr(work, "recomb", None) is not None else 0)
               | (RT_PERIODIC if getattr(work, "periodic", False) else 0))
    d.solve_id = int(work.solve_id)
    d.brick_log2 = int(brick_log2)
    d.wave_chunk = int(wave_chunk)
    d.refill_min = int(refill_min)
    d.blocks_per_cu = int(blocks_per_cu)
    d.trace_packets = int(trace_packets)
    d.trace_len = int(trace_len)
    d.trace_stride = int(trace_stride)
    d.run_len = int(run_len)
    d.park_lanes = int(park_lanes)
    d.finish_pass = int(finish_pass)
    d.inflight = int(inflight)
    d.path_cells = int(getattr(work, "path_cells", 0) or 0)
    return d


class Solve:
    """One solve on the current GPU: workspace and fields in torch device memory."""

    def __init__(self, work, *, device: str = "cuda", stream=None, counters=None, **tiles):
        """counters: optional initial recombination counters [species][ncell]
        (numpy, float64) of a workload with recombination re-emission."""
        import torch
        self.work = work
        if not tiles.get("inflight"):
            # records for every packet of a sub-step, up to 2^24
            tiles["inflight"] = int(min(1 << 24, max(1, -(-int(work.packets) // int(work.n_sub)))))
        self.desc = desc_from_workload(work, **tiles)
        self.ncell = work.ncell
        self.fp64 = bool(self.desc.flags & RT_FP64)
        self.stream = stream
        nbytes = rt_workspace_bytes(self.desc, len(work.src_ndot))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        dt = torch.float64 if self.fp64 else torch.float32
        # the inputs go up on the solve's stream, which the import then follows
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            nh = torch.as_tensor(np.asarray(work.n_h), dtype=dt, device=device).contiguous()
            x = torch.as_tensor(np.asarray(work.x).reshape(5, -1), dtype=dt, device=device).contiguous()
            t = torch.as_tensor(np.asarray(work.temp), dtype=dt, device=device).contiguous()
        self.h = rt_init_grid(self.desc, self.workspace, len(work.src_ndot), nh, x, t, stream)
        if len(work.src_ndot):
            rt_add_sources(self.h, work.src_ijk, work.src_ndot, work.src_sed, work.src_flags)
        bg = getattr(work, "background", None)
        if bg is not None:
            rt_set_background(self.h, bg.ndot, bg.sed, bg.packets)
        self.recomb = getattr(work, "recomb", None) is not None
        if self.recomb:
            r = work.recomb
            rc = None
            if counters is not None:
                rc = torch.as_tensor(np.asarray(counters, np.float64), device=device).contiguous()
            rt_set_recombination(self.h, r.f_rec, r.log10_t0, r.dlog10_t, r.milne, rc)
            del rc
        # the import is stream-ordered: wait for it before the inputs are freed
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
        del nh, x, t

    def step(self, dt: Optional[float] = None, packets: Optional[int] = None, seed: Optional[int] = None,
             stats: bool = True):
        w = self.work
        return rt_step(self.h, w.dt_s if dt is None else dt, w.packets if packets is None else packets,
                       w.seed if seed is None else seed, stats)

    def fetch(self, mask: Optional[int] = None) -> np.ndarray:
        """Fields in FIELDS order (default: all, the recombination counters
        only for a solve with re-emission)."""
        if mask is None:
            mask = RT_F_ALL if self.recomb else RT_F_STATE
        return rt_fetch_fields(self.h, mask, self.ncell)

    def trace(self, count: Optional[int] = None) -> np.ndarray:
        n = self.desc.trace_packets if count is None else count
        return rt_fetch_trace(self.h, n, self.desc.trace_len)

    def release(self):
        if self.h is not None:
            rt_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def tiles_of(n) -> int:
    """Tiles of 8^3 cells of a grid with n cells per axis."""
    return int(np.prod([-(-int(v) // 8) for v in n]))


class Batch:
    """Fused steps of up to max_solves solves shaped like `shape` (a workload:
    precision from fp64, species, bins, thermal) on their own stream (torch
    device memory for the workspace); graph=True captures each call shape
    once.  max_round_packets: packets of one sub-step of all solves together;
    max_tiles: 8^3 tiles of all solves together."""

    def __init__(self, max_solves: int, shape, *, fp64: bool, max_round_packets: int, max_tiles: int,
                 graph: bool = True, stream=None, device: str = "cuda", **tiles):
        import torch
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.shape = desc_from_workload(shape, fp64=fp64, **tiles)
        nbytes = rt_batch_workspace_bytes(max_solves, self.shape, max_round_packets, max_tiles)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.b = rt_batch_init(max_solves, self.shape, max_round_packets, max_tiles, self.workspace, self.stream,
                               RT_BATCH_GRAPH if graph else 0)
        self.last_n = 0

    def step(self, solves, dt_s=None, packets=None, seeds=None, stats: bool = False):
        """One step of every Solve in solves; per-solve values default to the
        solve's workload (dt, packets per step, seed)."""
        dt_s = [s.work.dt_s for s in solves] if dt_s is None else dt_s
        packets = [s.work.packets for s in solves] if packets is None else packets
        seeds = [s.work.seed for s in solves] if seeds is None else seeds
        self.last_n = len(solves)
        return rt_step_many(self.b, [s.h for s in solves], dt_s, packets, seeds, stats)

    def launch(self, solves, dt_s=None, packets=None, seeds=None):
        """step() without waiting; wait() then returns the ledgers."""
        self.step(solves, dt_s, packets, seeds, stats=False)

    def wait(self):
        return rt_batch_wait(self.b, self.last_n)

    def synchronize(self):
        self.stream.synchronize()

    def release(self):
        if self.b is not None:
            rt_batch_release(self.b)
            self.b = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
