"""Python binding of the ceilings microbenchmarks (include/rt_ceilings.h,
librt_ceilings.so): HBM copy and read bandwidth, float64 atomic adds into
device memory and into LDS.  Argument marshalling only; torch provides the
buffers and the stream."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librt_ceilings.so")

_VP, _I32, _I64, _SZ, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
SIGNATURES = {
    "rtc_hbm_copy": (_I32, [_VP, _VP, _SZ, _I32, _VP, C.POINTER(_D)]),
    "rtc_hbm_read": (_I32, [_VP, _SZ, _I32, _VP, _VP, C.POINTER(_D)]),
    "rtc_global_atomic_f64": (_I32, [_VP, _SZ, _I64, _VP, C.POINTER(_D)]),
    "rtc_lds_atomic_f64": (_I32, [_I32, _I32, _I64, _VP, _VP, C.POINTER(_D)]),
}
_lib = None


def lib():
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


def _call(name, *args):
    out = C.c_double(0.0)
    st = getattr(lib(), name)(*args, C.byref(out))
    if st != 0:
        raise RuntimeError(f"{name}: status {st}")
    return out.value


def _stream():
    import torch
    return _VP(torch.cuda.current_stream().cuda_stream)


def measure(copy_mib: int = 4096, reps: int = 5) -> dict:
    """Every ceiling on the current device: HBM copy and read (GB/s) over
    copy_mib MiB, far beyond the last-level cache; float64 atomic adds
    (updates/s) into 1 MiB (cache-resident) and 1 GiB of device memory; float64
    atomic adds into LDS laid out as the tiled march's accumulators (4 values
    per cell) cell-major and value-major, and one value per cell."""
    import torch
    n = copy_mib << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    sink = torch.zeros(65536, dtype=torch.float64, device="cuda")
    st = _stream()
    out = {"copy_gbs": _call("rtc_hbm_copy", _VP(b.data_ptr()), _VP(a.data_ptr()), n, reps, st),
           "read_gbs": _call("rtc_hbm_read", _VP(a.data_ptr()), n, reps, _VP(sink.data_ptr()), st),
           "copy_bytes": n}
    del a, b
    for tag, cnt in (("l2", 1 << 17), ("hbm", 1 << 27)):
        buf = torch.zeros(cnt, dtype=torch.float64, device="cuda")
        out[f"atomic_f64_{tag}_per_s"] = _call("rtc_global_atomic_f64", _VP(buf.data_ptr()), cnt, 1 << 30, st)
        out[f"atomic_f64_{tag}_bytes"] = cnt * 8
        del buf
    for tag, acc, soa in (("lds_acc4_cellmajor", 4, 0), ("lds_acc4_valuemajor", 4, 1), ("lds_acc1", 1, 0)):
        out[f"atomic_f64_{tag}_per_s"] = _call("rtc_lds_atomic_f64", acc, soa, 1 << 33, _VP(sink.data_ptr()), st)
    torch.cuda.synchronize()
    return out
