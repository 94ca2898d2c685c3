"""ctypes binding of ``libxeng.so`` (argument marshalling only).

Every step of the correlation runs in the library's gfx950 kernels; this
module only turns PyTorch tensors and streams into the pointers and sizes
the C ABI takes.  PyTorch provides device memory and streams.  Importing
the binding fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxeng.so")

XENG_OK = 0
XENG_EINVAL = -1
XENG_EOVERFLOW = -2
XENG_ENOMEM = -3
XENG_EDEVICE = -4
XENG_EBUSY = -5
XENG_ENOTSUP = -6
XENG_NIBBLE_RE_LOW = 1
XENG_COUNTS = 4
XENG_RFI_MAX_BLOCK = 1024
XENG_BEAMS_MAX = 16
XENG_SERVER_STAGGER_EXPORTS = 2
XENG_KERNEL_AUTO = 0
XENG_KERNEL_GENERAL = 1
XENG_KERNEL_DMA4 = 2
XENG_KERNEL_FP8 = 3
XENG_TUNE_SETTINGS = 0
XENG_TUNE_MEASURED = 1
XENG_TUNE_CACHE_FILE = 2
XENG_PLAN_LINEAR = 0
XENG_PLAN_XCD = 1


class XengError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class _Config(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("device", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("mem_budget_bytes", ctypes.c_int64)]


class _RfiConfig(ctypes.Structure):
    _fields_ = [("block_len", ctypes.c_int32), ("den", ctypes.c_int32), ("lo_num", ctypes.c_int32),
                ("hi_num", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Job(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("slot", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("d_samples", ctypes.c_void_p), ("n_samples", ctypes.c_int64),
                ("row_stride", ctypes.c_int64)]


class _DumpJob(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("slot", ctypes.c_int32), ("reset", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("reserved", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("min_stages", ctypes.c_int32), ("plan_order", ctypes.c_int32),
                ("us_per_launch", ctypes.c_double), ("source", ctypes.c_int32),
                ("saved", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("device", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("frame_len", ctypes.c_int32), ("dump_frames", ctypes.c_int32),
                ("ring_frames", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_channels", ctypes.c_int32), ("frame_period_us", ctypes.c_double),
                ("launch_period_us", ctypes.c_double), ("mem_budget_bytes", ctypes.c_int64),
                ("reserved", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("frames_released", ctypes.c_int64), ("frames_done", ctypes.c_int64),
                ("frames_dropped", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("dumps", ctypes.c_int64), ("backlog_frames", ctypes.c_int64),
                ("channels_waiting", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("tcmacs", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("max_pass_ms", ctypes.c_double), ("max_launch_call_ms", ctypes.c_double),
                ("max_copy_call_ms", ctypes.c_double),
                ("frames_gathered", ctypes.c_int64)]


class _ServerChannel(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("slot", ctypes.c_int32), ("frames_done", ctypes.c_int64),
                ("dumps", ctypes.c_int64), ("last_dump_first_frame", ctypes.c_int64),
                ("admitted_s", ctypes.c_double)]


class _PieceInfo(ctypes.Structure):
    _fields_ = [("job", ctypes.c_int32), ("ti", ctypes.c_int32), ("tj", ctypes.c_int32),
                ("atomic", ctypes.c_int32), ("t0", ctypes.c_int64), ("t1", ctypes.c_int64),
                ("workgroup", ctypes.c_int32), ("n_tiles", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -m paper_2005_09481_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "xeng_create": (ctypes.c_int, [ctypes.POINTER(_Config), ctypes.POINTER(vp)]),
        "xeng_destroy": (ctypes.c_int, [vp]),
        "xeng_correlate": (ctypes.c_int, [vp, i32, vp, i64, i64, vp]),
        "xeng_correlate_batch": (ctypes.c_int, [ctypes.POINTER(_Job), i32, vp]),
        "xeng_dump": (ctypes.c_int, [vp, i32, vp, i32, vp]),
        "xeng_dump_batch": (ctypes.c_int, [ctypes.POINTER(_DumpJob), i32, vp]),
        "xeng_reset": (ctypes.c_int, [vp, i32, vp]),
        "xeng_samples_integrated": (i64, [vp, i32]),
        "xeng_max_integration": (i64, []),
        "xeng_slot_bytes": (i64, [i32]),
        "xeng_n_inputs": (i32, [vp]),
        "xeng_n_slots": (i32, [vp]),
        "xeng_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "xeng_correlate_reference": (ctypes.c_int, [vp, i64, i32, i64, u32, vp, vp]),
        "xeng_plan_inspect": (i64, [ctypes.POINTER(i32), ctypes.POINTER(i64), i32, i32, i32, i32,
                                    ctypes.POINTER(_PieceInfo), i64]),
        "xeng_set_tuning": (ctypes.c_int, [i32, i32, i32]),
        "xeng_clock_probe": (ctypes.c_int, [i32, vp]),
        "xeng_mfma_ceiling": (ctypes.c_int, [i32, i32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
        "xeng_batch_create": (ctypes.c_int, [ctypes.POINTER(_Job), i32, ctypes.POINTER(vp)]),
        "xeng_batch_launch": (ctypes.c_int, [vp, vp]),
        "xeng_batch_check": (ctypes.c_int, [vp]),
        "xeng_set_pad_chunk_bytes": (ctypes.c_int, [i64]),
        "xeng_set_plan_order": (ctypes.c_int, [i32]),
        "xeng_rfi_flags": (ctypes.c_int, [vp, i64, i32, i64, u32, ctypes.POINTER(_RfiConfig), vp, vp]),
        "xeng_correlate_flagged": (ctypes.c_int, [vp, i32, vp, i64, i64, vp, i32, vp]),
        "xeng_dump_counts": (ctypes.c_int, [vp, i32, vp, vp]),
        "xeng_correlate_presum": (ctypes.c_int, [vp, i32, vp, i64, i64, vp]),
        "xeng_beams_create": (ctypes.c_int, [i32, i32, i32, u32, vp, ctypes.POINTER(vp)]),
        "xeng_beams_set_weights": (ctypes.c_int, [vp, vp, vp]),
        "xeng_beams_destroy": (ctypes.c_int, [vp]),
        "xeng_beamform": (ctypes.c_int, [vp, vp, i64, i64, i32, vp, vp]),
        "xeng_correlate_static": (ctypes.c_int, [vp, i32, vp, i64, i64, vp]),
        "xeng_plan_inspect_static": (i64, [i32, i64, i32, i32, i32, ctypes.POINTER(_PieceInfo), i64]),
        "xeng_server_export_ring": (ctypes.c_int, [vp, i32, vp, i32]),
        "xeng_batch_destroy": (ctypes.c_int, [vp]),
        "xeng_autotune": (ctypes.c_int, [ctypes.POINTER(_Job), i32, i32, vp, ctypes.POINTER(_Tuning)]),
        "xeng_tuning_lookup": (ctypes.c_int, [ctypes.POINTER(_Job), i32, ctypes.POINTER(_Tuning)]),
        "xeng_tune_cache_path": (i32, [i32, ctypes.c_char_p, i32]),
        "xeng_server_create": (ctypes.c_int, [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]),
        "xeng_server_destroy": (ctypes.c_int, [vp]),
        "xeng_server_max_channels": (i32, [vp]),
        "xeng_server_admit": (ctypes.c_int, [vp, vp, i64, i32, ctypes.c_double, i64,
                                             ctypes.POINTER(i32)]),
        "xeng_server_run": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(_ServerStats)]),
        "xeng_server_channel_info": (ctypes.c_int, [vp, i32, ctypes.POINTER(_ServerChannel)]),
        "xeng_server_last_dump": (ctypes.c_int, [vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().xeng_strerror(status).decode()


def _check(status: int, what: str):
    if status != XENG_OK:
        raise XengError(status, what)


def tri(n: int) -> int:
    return n * (n + 1) // 2


def max_integration() -> int:
    return int(lib().xeng_max_integration())


def slot_bytes(n_inputs: int) -> int:
    return int(lib().xeng_slot_bytes(n_inputs))


def set_tuning(wgs_per_cu: int = 0, min_stages: int = 0, kernel: int = -1):
    """Launch tuning (results never depend on it): general-kernel workgroups
    per CU, minimum piece length in 64-sample stages, kernel selection
    (XENG_KERNEL_AUTO / XENG_KERNEL_GENERAL / XENG_KERNEL_DMA4 /
    XENG_KERNEL_FP8; -1 keeps the current one)."""
    _check(lib().xeng_set_tuning(wgs_per_cu, min_stages, kernel), "xeng_set_tuning")


def set_plan_order(order: int):
    """Work order of single-job launches: XENG_PLAN_XCD (default) or XENG_PLAN_LINEAR."""
    _check(lib().xeng_set_plan_order(order), "xeng_set_plan_order")


def set_pad_chunk_bytes(nbytes: int = 0):
    """Scratch bytes per padded chunk / per batched call (0: the default)."""
    _check(lib().xeng_set_pad_chunk_bytes(nbytes), "xeng_set_pad_chunk_bytes")


def clock_probe(buf=None, device: int = 0):
    """Clock probe (``xeng_clock_probe``, measurement only): while set, every
    wide-kernel launch on ``device`` stores, from its workgroup 0, the shader
    cycle counter and the 100 MHz real-time counter at the workgroup's start
    and end into ``buf`` (an int64 device tensor of >= 4 elements); None
    stops it.  ``sclk_ghz(buf)`` turns the four values into a clock."""
    if buf is not None:
        import torch
        if buf.dtype != torch.int64 or buf.numel() < 4 or not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("clock_probe needs a contiguous int64 device tensor of >= 4 elements")
        ptr = ctypes.c_void_p(buf.data_ptr())
    else:
        ptr = ctypes.c_void_p(0)
    _check(lib().xeng_clock_probe(device, ptr), "xeng_clock_probe")


def mfma_ceiling(ms: int = 400, device: int = 0):
    """Matrix-core ceiling (``xeng_mfma_ceiling``, measurement only): runs a
    loop of nothing but int8 MFMAs on every CU for about ``ms`` ms and
    returns (int8 MAC/s of its second half, shader clock in GHz then)."""
    mac, ghz = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().xeng_mfma_ceiling(device, ms, ctypes.byref(mac), ctypes.byref(ghz)), "xeng_mfma_ceiling")
    return mac.value, ghz.value


def sclk_ghz(buf) -> float:
    """Shader clock of the probed launch from its four counter values."""
    c = [int(v) for v in buf[:4].tolist()]
    dt_s = (c[3] - c[1]) / 1e8
    return (c[2] - c[0]) / dt_s / 1e9 if dt_s > 0 else float("nan")


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _samples_args(samples, n_inputs: int, device: int):
    import torch
    if not isinstance(samples, torch.Tensor) or samples.dtype != torch.uint8:
        raise TypeError("samples must be a torch.uint8 tensor")
    if samples.dim() != 2:
        raise ValueError("samples must be 2-D [T, >=N]")
    if samples.shape[0] == 0:
        return None, 0, max(n_inputs, samples.shape[1])
    if samples.device.type != "cuda" or samples.device.index != device:
        raise ValueError(f"samples must live on cuda:{device}")
    if samples.shape[1] < n_inputs or samples.stride(1) != 1:
        raise ValueError("samples must be [T, >=N] with unit stride along inputs")
    row_stride = samples.stride(0) if samples.shape[0] > 1 else max(samples.stride(0), n_inputs)
    return ctypes.c_void_p(samples.data_ptr()), samples.shape[0], row_stride


class Correlator:
    """N-input correlator with ``n_slots`` device-resident int32 accumulators."""

    def __init__(self, n_inputs: int, n_slots: int = 1, device: int | None = None,
                 re_low: bool = False, mem_budget_bytes: int = 0, counts: bool = False):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        flags = (XENG_NIBBLE_RE_LOW if re_low else 0) | (XENG_COUNTS if counts else 0)
        cfg = _Config(n_inputs, n_slots, self.device, flags, mem_budget_bytes)
        h = ctypes.c_void_p()
        _check(lib().xeng_create(ctypes.byref(cfg), ctypes.byref(h)), "xeng_create")
        self._h = h
        self.n_inputs = n_inputs
        self.n_slots = n_slots

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("correlator is closed")
        return self._h

    def correlate(self, slot: int, samples, stream=None):
        """acc[slot] += V(samples); ``samples`` is uint8 [T, >=N] on the device."""
        ptr, t, row_stride = _samples_args(samples, self.n_inputs, self.device)
        _check(lib().xeng_correlate(self.handle, slot, ptr, t, row_stride,
                                    _stream_handle(stream, self.device)), "xeng_correlate")

    def correlate_presum(self, slot: int, samples, stream=None):
        """acc[slot] += V(samples) by the unsigned-nibble form with pre-sums."""
        ptr, t, row_stride = _samples_args(samples, self.n_inputs, self.device)
        _check(lib().xeng_correlate_presum(self.handle, slot, ptr, t, row_stride,
                                           _stream_handle(stream, self.device)), "xeng_correlate_presum")

    def correlate_flagged(self, slot: int, samples, flags, block_len: int, stream=None):
        """acc[slot] += V over unflagged samples, counts[slot] += n_ij;
        ``flags`` uint8 [ceil(T / block_len), N] on the device (nonzero = flagged)."""
        import torch
        ptr, t, row_stride = _samples_args(samples, self.n_inputs, self.device)
        nb = -(-t // block_len) if block_len > 0 else 0
        if not isinstance(flags, torch.Tensor) or flags.dtype != torch.uint8 or not flags.is_contiguous() \
                or (t > 0 and (tuple(flags.shape) != (nb, self.n_inputs) or not flags.is_cuda)):
            raise ValueError("flags must be a contiguous uint8 device tensor [ceil(T/block_len), N]")
        fptr = ctypes.c_void_p(flags.data_ptr()) if t > 0 else None
        _check(lib().xeng_correlate_flagged(self.handle, slot, ptr, t, row_stride, fptr, block_len,
                                            _stream_handle(stream, self.device)), "xeng_correlate_flagged")

    def dump_counts(self, slot: int, out=None, stream=None):
        """Per-pair sample counts int32 [N(N+1)/2] (pairs in the order of dump)."""
        import torch
        if out is None:
            out = torch.empty(tri(self.n_inputs), dtype=torch.int32, device=f"cuda:{self.device}")
        if out.dtype != torch.int32 or out.numel() != tri(self.n_inputs) or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of N(N+1)/2")
        _check(lib().xeng_dump_counts(self.handle, slot, ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(stream, self.device)), "xeng_dump_counts")
        return out

    def _dump_out(self, out):
        import torch
        if out is None:
            out = torch.empty((tri(self.n_inputs), 2), dtype=torch.int32,
                              device=f"cuda:{self.device}")
        if out.dtype != torch.int32 or out.numel() != 2 * tri(self.n_inputs) or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of N(N+1)/2 x 2")
        return out

    def dump(self, slot: int, out=None, reset: bool = True, stream=None):
        """Integrated visibilities int32 [N(N+1)/2, 2] (Re, Im), upper triangle row-major."""
        out = self._dump_out(out)
        _check(lib().xeng_dump(self.handle, slot, ctypes.c_void_p(out.data_ptr()), int(bool(reset)),
                               _stream_handle(stream, self.device)), "xeng_dump")
        return out

    def reset(self, slot: int, stream=None):
        _check(lib().xeng_reset(self.handle, slot, _stream_handle(stream, self.device)),
               "xeng_reset")

    def samples_integrated(self, slot: int) -> int:
        v = int(lib().xeng_samples_integrated(self.handle, slot))
        if v < 0:
            raise XengError(XENG_EINVAL, "xeng_samples_integrated")
        return v

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib().xeng_destroy(self._h), "xeng_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _job_array(jobs):
    arr = (_Job * len(jobs))()
    for k, (corr, slot, samples) in enumerate(jobs):
        ptr, t, row_stride = _samples_args(samples, corr.n_inputs, corr.device)
        arr[k] = _Job(corr.handle, slot, 0, ptr, t, row_stride)
    return arr


def correlate_batch(jobs, stream=None):
    """One persistent launch per kernel kind over ``jobs`` = [(correlator, slot, samples), ...]."""
    if not jobs:
        return
    _check(lib().xeng_correlate_batch(_job_array(jobs), len(jobs),
                                      _stream_handle(stream, jobs[0][0].device)),
           "xeng_correlate_batch")


def dump_batch(jobs, stream=None):
    """Export many slots in two launches: ``jobs`` = [(correlator, slot), ...]
    or [(correlator, slot, out, reset), ...] (out None: allocated; reset
    default True).  Returns the output tensors in job order."""
    if not jobs:
        return []
    arr = (_DumpJob * len(jobs))()
    outs = []
    for k, j in enumerate(jobs):
        c, slot = j[0], j[1]
        out = c._dump_out(j[2] if len(j) > 2 else None)
        reset = bool(j[3]) if len(j) > 3 else True
        arr[k] = _DumpJob(c.handle, slot, int(reset), out.data_ptr(), 0, 0)
        outs.append(out)
    _check(lib().xeng_dump_batch(arr, len(jobs), _stream_handle(stream, jobs[0][0].device)),
           "xeng_dump_batch")
    return outs


class Batch:
    """Prepared batch (``xeng_batch_*``): plan and job table resident on the
    device, launches that only enqueue kernels (graph-capturable).  The
    sample tensors named by ``jobs`` are kept alive by the batch."""

    def __init__(self, jobs):
        self._keep = [j[2] for j in jobs] + [j[0] for j in jobs]
        self.device = jobs[0][0].device
        h = ctypes.c_void_p()
        _check(lib().xeng_batch_create(_job_array(jobs), len(jobs), ctypes.byref(h)),
               "xeng_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().xeng_batch_launch(self._h, _stream_handle(stream, self.device)),
               "xeng_batch_launch")

    def check(self) -> int:
        """Wait for the device; XENG_EOVERFLOW if a launch or replay since
        the previous check was refused by the device-side integration guard
        (it then integrated nothing), else XENG_OK."""
        return int(lib().xeng_batch_check(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().xeng_batch_destroy(self._h), "xeng_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Tuning:
    kernel: int
    wgs_per_cu: int
    min_stages: int
    plan_order: int
    us_per_launch: float
    source: int
    saved: bool


def _tuning(t) -> Tuning:
    return Tuning(t.kernel, t.wgs_per_cu, t.min_stages, t.plan_order, t.us_per_launch, t.source, bool(t.saved))


def autotune(jobs, iters: int = 5, stream=None) -> Tuning:
    """Time the candidate launch configurations on ``jobs`` (on scratch
    accumulators: the jobs' slots are untouched), keep the best for later
    calls of the same job class and write it to the tune-cache file."""
    t = _Tuning()
    _check(lib().xeng_autotune(_job_array(jobs), len(jobs), iters,
                               _stream_handle(stream, jobs[0][0].device), ctypes.byref(t)),
           "xeng_autotune")
    return _tuning(t)


def tuning_lookup(jobs) -> Tuning:
    """The configuration a batched call of ``jobs`` would launch with now."""
    t = _Tuning()
    _check(lib().xeng_tuning_lookup(_job_array(jobs), len(jobs), ctypes.byref(t)), "xeng_tuning_lookup")
    return _tuning(t)


def tune_cache_path(device: int = 0) -> str:
    """Path of the tune-cache file of ``device``'s architecture."""
    n = int(lib().xeng_tune_cache_path(device, None, 0))
    if n < 0:
        _check(n, "xeng_tune_cache_path")
    buf = ctypes.create_string_buffer(n + 1)
    _check(min(0, int(lib().xeng_tune_cache_path(device, buf, n + 1))), "xeng_tune_cache_path")
    return buf.value.decode()


def rfi_flags(samples, n_inputs: int | None = None, block_len: int = 256, lo_num: int = 625,
              hi_num: int = 1375, den: int = 1000, re_low: bool = False, out=None, stream=None):
    """Spectral-kurtosis RFI flags uint8 [ceil(T / block_len), N] (1 = flagged)."""
    import torch
    n = samples.shape[1] if n_inputs is None else n_inputs
    dev = samples.device.index if samples.device.type == "cuda" else torch.cuda.current_device()
    ptr, t, row_stride = _samples_args(samples, n, dev)
    nb = -(-t // block_len)
    if out is None:
        out = torch.empty((nb, n), dtype=torch.uint8, device=f"cuda:{dev}")
    if out.dtype != torch.uint8 or tuple(out.shape) != (nb, n) or not out.is_contiguous():
        raise ValueError("out must be a contiguous uint8 tensor [ceil(T/block_len), N]")
    cfg = _RfiConfig(block_len, den, lo_num, hi_num, 0)
    _check(lib().xeng_rfi_flags(ptr, t, n, row_stride, XENG_NIBBLE_RE_LOW if re_low else 0, ctypes.byref(cfg),
                                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream, dev)), "xeng_rfi_flags")
    return out


class Beams:
    """A beam set (``xeng_beams_*``): complex int8 weights [B][N][2] held on
    the device; ``form`` computes y_b(t) = sum_i w_bi x_i(t)."""

    def __init__(self, weights, device: int = 0, re_low: bool = False):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.int8)
        if w.ndim != 3 or w.shape[2] != 2:
            raise ValueError("weights must be int8 [B][N][2]")
        self.n_beams, self.n_inputs, self.device = w.shape[0], w.shape[1], device
        h = ctypes.c_void_p()
        _check(lib().xeng_beams_create(self.n_inputs, self.n_beams, device, XENG_NIBBLE_RE_LOW if re_low else 0,
                                       w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)), "xeng_beams_create")
        self._h = h

    def set_weights(self, weights, stream=None):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.int8)
        if w.shape != (self.n_beams, self.n_inputs, 2):
            raise ValueError("weights must keep the beam set's [B][N][2] shape")
        _check(lib().xeng_beams_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p),
                                            _stream_handle(stream, self.device)), "xeng_beams_set_weights")

    def form(self, samples, shift: int = -1, out=None, stream=None):
        """int32 [T][B][2] (shift -1) or int8 [T][B][2] (8-bit export)."""
        import torch
        ptr, t, row_stride = _samples_args(samples, self.n_inputs, self.device)
        dtype = torch.int32 if shift < 0 else torch.int8
        if out is None:
            out = torch.empty((t, self.n_beams, 2), dtype=dtype, device=f"cuda:{self.device}")
        if out.dtype != dtype or tuple(out.shape) != (t, self.n_beams, 2) or not out.is_contiguous():
            raise ValueError("out must be a contiguous [T][B][2] tensor of the export's dtype")
        _check(lib().xeng_beamform(self._h, ptr, t, row_stride, shift, ctypes.c_void_p(out.data_ptr()),
                                   _stream_handle(stream, self.device)), "xeng_beamform")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().xeng_beams_destroy(self._h), "xeng_beams_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def beamform(samples, weights, shift: int = -1, re_low: bool = False, stream=None):
    """One-off beams of ``samples`` with ``weights`` (a beam set made for the call)."""
    dev = samples.device.index if samples.device.type == "cuda" else 0
    bm = Beams(weights, device=dev, re_low=re_low)
    try:
        return bm.form(samples, shift=shift, stream=stream)
    finally:
        import torch
        torch.cuda.synchronize(dev)
        bm.close()


def correlate_reference(samples, n_inputs: int | None = None, re_low: bool = False, stream=None):
    """Scalar GPU reference kernel; returns int32 [N(N+1)/2, 2] for one call."""
    import torch
    n = samples.shape[1] if n_inputs is None else n_inputs
    dev = samples.device.index if samples.device.type == "cuda" else torch.cuda.current_device()
    ptr, t, row_stride = _samples_args(samples, n, dev)
    out = torch.empty((tri(n), 2), dtype=torch.int32, device=f"cuda:{dev}")
    _check(lib().xeng_correlate_reference(ptr, t, n, row_stride,
                                          XENG_NIBBLE_RE_LOW if re_low else 0,
                                          ctypes.c_void_p(out.data_ptr()),
                                          _stream_handle(stream, dev)), "xeng_correlate_reference")
    return out


@dataclass
class PieceInfo:
    job: int
    ti: int
    tj: int
    atomic: bool
    t0: int
    t1: int
    workgroup: int
    n_tiles: int


def plan_inspect(n_inputs, n_samples, n_workgroups: int, min_stages: int = 0, wide=False):
    """Pieces the library would launch for jobs of these sizes (host only);
    ``wide``: False / 0 square tiles, True / 1 wide, 2 narrow (N <= 64)."""
    n = len(n_inputs)
    ni = (ctypes.c_int32 * n)(*n_inputs)
    ns = (ctypes.c_int64 * n)(*n_samples)
    cnt = lib().xeng_plan_inspect(ni, ns, n, n_workgroups, min_stages, int(wide), None, 0)
    if cnt < 0:
        raise XengError(int(cnt), "xeng_plan_inspect")
    out = (_PieceInfo * max(cnt, 1))()
    cnt2 = lib().xeng_plan_inspect(ni, ns, n, n_workgroups, min_stages, int(wide), out, cnt)
    assert cnt2 == cnt
    return [PieceInfo(p.job, p.ti, p.tj, bool(p.atomic), p.t0, p.t1, p.workgroup, p.n_tiles)
            for p in out[:cnt]]


def plan_inspect_static(n_inputs: int, n_samples: int, n_workgroups: int, min_stages: int = 0,
                        wide: bool = False):
    """Pieces of the allocation-free path's device planner (host copy)."""
    cnt = lib().xeng_plan_inspect_static(n_inputs, n_samples, n_workgroups, min_stages, int(wide), None, 0)
    if cnt < 0:
        raise XengError(int(cnt), "xeng_plan_inspect_static")
    out = (_PieceInfo * max(cnt, 1))()
    cnt2 = lib().xeng_plan_inspect_static(n_inputs, n_samples, n_workgroups, min_stages, int(wide), out, cnt)
    assert cnt2 == cnt
    return [PieceInfo(p.job, p.ti, p.tj, bool(p.atomic), p.t0, p.t1, p.workgroup, p.n_tiles)
            for p in out[:cnt]]


class Server:
    """Streaming server (``xeng_server_*``): channels of N inputs ingest
    frames at a fixed cadence; one batched launch about every
    ``launch_period_us`` integrates every channel's new frames; each channel
    is exported every ``dump_frames`` frames (``stagger_exports``: at frame
    counts offset per slot, XENG_SERVER_STAGGER_EXPORTS)."""

    def __init__(self, n_inputs: int, device: int = 0, frame_len: int = 256, dump_frames: int = 128,
                 ring_frames: int = 64, max_inflight: int = 2, max_channels: int = 0,
                 frame_period_us: float = 655.36, launch_period_us: float = 5000.0,
                 mem_budget_bytes: int = 0, re_low: bool = False, stagger_exports: bool = False):
        flags = (XENG_NIBBLE_RE_LOW if re_low else 0) | (XENG_SERVER_STAGGER_EXPORTS if stagger_exports else 0)
        self.dump_frames = dump_frames
        cfg = _ServerConfig(n_inputs, device, flags, frame_len,
                            dump_frames, ring_frames, max_inflight, max_channels, frame_period_us,
                            launch_period_us, mem_budget_bytes, 0)
        h = ctypes.c_void_p()
        _check(lib().xeng_server_create(ctypes.byref(cfg), ctypes.byref(h)), "xeng_server_create")
        self._h = h
        self.n_inputs, self.device, self.frame_len = n_inputs, device, frame_len
        self._keep = []

    @property
    def max_channels(self) -> int:
        return int(lib().xeng_server_max_channels(self._h))

    def admit(self, frames, start_s: float = 0.0, total_frames: int = 0) -> int:
        """``frames``: uint8 [F][frame_len][N], on the device or in pinned host memory."""
        import torch
        if frames.dtype != torch.uint8 or frames.dim() != 3 or not frames.is_contiguous() or \
                frames.shape[1] != self.frame_len or frames.shape[2] != self.n_inputs:
            raise ValueError("frames must be contiguous uint8 [F][frame_len][N]")
        host = 0 if frames.is_cuda else 1
        if host and not frames.is_pinned():
            raise ValueError("host frames must be in pinned memory")
        ch = ctypes.c_int32()
        _check(lib().xeng_server_admit(self._h, ctypes.c_void_p(frames.data_ptr()), frames.shape[0], host,
                                       start_s, total_frames, ctypes.byref(ch)), "xeng_server_admit")
        self._keep.append(frames)
        return ch.value

    def run(self, seconds: float) -> dict:
        st = _ServerStats()
        _check(lib().xeng_server_run(self._h, seconds, ctypes.byref(st)), "xeng_server_run")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def channel_info(self, channel: int) -> dict:
        ci = _ServerChannel()
        _check(lib().xeng_server_channel_info(self._h, channel, ctypes.byref(ci)), "xeng_server_channel_info")
        return {f: getattr(ci, f) for f, _ in _ServerChannel._fields_}

    def export_ring(self, channel: int, ring):
        """Every export of ``channel`` goes to ``ring`` [n][N(N+1)/2][2] int32
        (device or pinned host), entry k % n for its k-th export."""
        import torch
        if ring.dtype != torch.int32 or ring.dim() != 3 or not ring.is_contiguous() or \
                ring.shape[1] != tri(self.n_inputs) or ring.shape[2] != 2:
            raise ValueError("ring must be contiguous int32 [n][N(N+1)/2][2]")
        if not ring.is_cuda and not ring.is_pinned():
            raise ValueError("a host ring must be in pinned memory")
        _check(lib().xeng_server_export_ring(self._h, channel, ctypes.c_void_p(ring.data_ptr()), ring.shape[0]),
               "xeng_server_export_ring")
        self._keep.append(ring)

    def last_dump(self, channel: int):
        import torch
        out = torch.empty((tri(self.n_inputs), 2), dtype=torch.int32, device=f"cuda:{self.device}")
        _check(lib().xeng_server_last_dump(self._h, channel, ctypes.c_void_p(out.data_ptr())),
               "xeng_server_last_dump")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().xeng_server_destroy(self._h), "xeng_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
