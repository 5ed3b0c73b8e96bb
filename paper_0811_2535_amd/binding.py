"""ctypes binding of libliftfft.so (argument marshalling only).

Every transform runs in the HIP library; this module only converts Python
arguments into the C ABI of ``include/liftfft.h``.  If the library is not
built the calls raise :class:`LibraryNotBuilt` -- there is no fallback.

PyTorch is imported before the library is loaded so that the library binds to
the HIP runtime PyTorch already carries (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  -- must precede loading the HIP library

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libliftfft.so")

FFT_C64, FFT_C128 = 0, 1
FFT_OK = 0
STATUS = {
    0: "FFT_OK", -1: "FFT_E_SIZE", -2: "FFT_E_DTYPE", -3: "FFT_E_SIGN", -4: "FFT_E_NULL",
    -5: "FFT_E_ALIGN", -6: "FFT_E_OOM", -7: "FFT_E_HIP", -8: "FFT_E_UNSUPPORTED",
    -9: "FFT_E_ARG", -10: "FFT_E_CAPACITY",
}
EXPORTED = [
    "fft_plan_create", "fft_plan_create_ex", "fft_execute", "fft_plan_destroy",
    "fft_strerror", "fft_plan_get_info", "fft_plan_set_timing", "fft_plan_read_timing",
    "fft_abi_version", "fft_plan_create_many", "fft_plan_create_tuned", "fft_plan_set_precision",
    "fft_plan_create_paper", "fft_execute_static",
]


class LibraryNotBuilt(RuntimeError):
    pass


class FFTError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__("%s: %s (%s)" % (what, strerror(code), self.name))


FFT_OPT_NO_XCD_REMAP = 1
FFT_OPT_SPLIT_EXCHANGE = 2
FFT_OPT_FULL_EXCHANGE = 4
FFT_OPT_PERSISTENT = 8
FFT_OPT_ONE_TILE = 16
FFT_OPT_DENSE = 32
FFT_OPT_GRAPH = 64
FFT_OPT_TWO_LEVEL = 128
FFT_OPT_THREE_LEVEL = 256
FFT_OPT_SHUFFLE_EXCHANGE = 512
FFT_OPT_AUTOTUNE = 1024
FFT_OPT_LDS_PREFETCH = 2048
FFT_OPT_DEBUG_CANARY = 4096
FFT_OPT_TILE_ORDER = 8192
FFT_OPT_ROW_LANES = 16384


class PlanOpts(ctypes.Structure):
    _fields_ = [("log2_p", ctypes.c_int32), ("radix", ctypes.c_int32),
                ("lines_per_block", ctypes.c_int32), ("lines_per_block2", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("values_per_thread", ctypes.c_int32),
                ("values_per_thread2", ctypes.c_int32), ("scratch_width", ctypes.c_int32),
                ("tile_order", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("opts", PlanOpts), ("ms", ctypes.c_double), ("ms_default", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("rejected", ctypes.c_int32)]

    def as_dict(self) -> dict:
        o = self.opts
        return {"opts": {"log2_p": o.log2_p, "radix": o.radix, "lines_per_block": o.lines_per_block,
                         "lines_per_block2": o.lines_per_block2, "flags": o.flags,
                         "values_per_thread": o.values_per_thread,
                         "values_per_thread2": o.values_per_thread2, "scratch_width": o.scratch_width,
                         "tile_order": o.tile_order},
                "ms": self.ms, "ms_default": self.ms_default, "candidates": self.candidates,
                "rejected": self.rejected}


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("batch", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("log2_p", ctypes.c_int32), ("log2_q", ctypes.c_int32),
                ("radix", ctypes.c_int32), ("lines_per_block_pass1", ctypes.c_int32),
                ("lines_per_block_pass2", ctypes.c_int32),
                ("grid_pass1", ctypes.c_int32), ("grid_pass2", ctypes.c_int32),
                ("threads_pass1", ctypes.c_int32), ("threads_pass2", ctypes.c_int32),
                ("lds_bytes_pass1", ctypes.c_int64), ("lds_bytes_pass2", ctypes.c_int64),
                ("scratch_bytes", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("variant_pass1", ctypes.c_int32), ("variant_pass2", ctypes.c_int32),
                ("length_classes", ctypes.c_int32), ("graph_launch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("log2_n1", ctypes.c_int32),
                ("log2_n2", ctypes.c_int32), ("log2_n3", ctypes.c_int32),
                ("lines_per_block_pass3", ctypes.c_int32), ("grid_pass3", ctypes.c_int32),
                ("threads_pass3", ctypes.c_int32), ("paper_breakpoint", ctypes.c_int32),
                ("lds_bytes_pass3", ctypes.c_int64),
                ("streams", ctypes.c_int32), ("reserved2", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded library (raises :class:`LibraryNotBuilt` if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise LibraryNotBuilt(
                    "%s is not built; run `python -c \"import __graft_entry__ as g; g.build()\"` "
                    "or `python -m paper_0811_2535_amd._build`" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
            L.fft_plan_create.argtypes = [i64, i64, i32, ctypes.POINTER(vp)]
            L.fft_plan_create_ex.argtypes = [i64, i64, i32, ctypes.POINTER(PlanOpts),
                                             ctypes.POINTER(vp)]
            L.fft_plan_create_many.argtypes = [ctypes.POINTER(i64), i64, i32, ctypes.c_uint32,
                                               ctypes.POINTER(vp)]
            L.fft_plan_create_tuned.argtypes = [i64, i64, i32, ctypes.c_int32, ctypes.POINTER(vp),
                                                ctypes.POINTER(TuneResult)]
            L.fft_plan_create_paper.argtypes = [i64, i64, i32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(vp)]
            L.fft_execute.argtypes = [vp, vp, vp, i32, vp]
            L.fft_execute_static.argtypes = [i64, i64, i32, vp, vp, i32, vp]
            L.fft_plan_destroy.argtypes = [vp]
            L.fft_strerror.argtypes = [i32]
            L.fft_strerror.restype = ctypes.c_char_p
            L.fft_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
            L.fft_plan_set_timing.argtypes = [vp, i32]
            L.fft_plan_set_precision.argtypes = [vp, i32]
            L.fft_plan_read_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double * 3),
                                               ctypes.POINTER(ctypes.c_int64 * 3), i32]
            for name in ("fft_plan_create", "fft_plan_create_ex", "fft_plan_create_many", "fft_plan_create_paper",
                         "fft_plan_create_tuned", "fft_plan_set_precision", "fft_execute",
                         "fft_plan_destroy", "fft_plan_get_info", "fft_plan_set_timing",
                         "fft_plan_read_timing", "fft_abi_version", "fft_execute_static"):
                getattr(L, name).restype = i32
            _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().fft_strerror(int(code)).decode()
    except LibraryNotBuilt:
        return STATUS.get(code, "unknown")


def _check(rc: int, what: str) -> None:
    if rc != FFT_OK:
        raise FFTError(rc, what)


def dtype_code(dtype) -> int:
    if dtype in (torch.complex64, "c64", "complex64"):
        return FFT_C64
    if dtype in (torch.complex128, "c128", "complex128"):
        return FFT_C128
    raise FFTError(-2, "unsupported dtype %r" % (dtype,))


class Plan:
    """A plan for ``batch`` transforms of length ``n`` (owns device memory).

    Thin wrapper over fft_plan_create_ex / fft_execute / fft_plan_destroy."""

    @classmethod
    def tuned(cls, n: int, batch: int = 1, dtype=torch.complex64, max_candidates: int = 0):
        """The fastest of the configurations fft_plan_create_tuned times for
        this shape; returns (plan, result dict)."""
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        self.n, self.batch = int(n), int(batch)
        self.dtype_code = dtype_code(dtype)
        self.torch_dtype = torch.complex64 if self.dtype_code == FFT_C64 else torch.complex128
        res = TuneResult()
        rc = lib().fft_plan_create_tuned(self.n, self.batch, self.dtype_code, int(max_candidates),
                                         ctypes.byref(self._h), ctypes.byref(res))
        _check(rc, "fft_plan_create_tuned(n=%d, batch=%d)" % (self.n, self.batch))
        return self, res.as_dict()

    @classmethod
    def paper(cls, n: int, batch: int = 1, dtype=torch.complex64, log2_m: int = 1,
              breakpoint: int = 2) -> "Plan":
        """The paper's partitioned radix-2 plan with m = 2^log2_m processors
        (workgroups) split at ``breakpoint`` (fft_plan_create_paper)."""
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        self.n, self.batch = int(n), int(batch)
        self.dtype_code = dtype_code(dtype)
        self.torch_dtype = torch.complex64 if self.dtype_code == FFT_C64 else torch.complex128
        rc = lib().fft_plan_create_paper(self.n, self.batch, self.dtype_code, int(log2_m), int(breakpoint),
                                         ctypes.byref(self._h))
        _check(rc, "fft_plan_create_paper(n=%d, log2_m=%d, breakpoint=%d)" % (self.n, log2_m, breakpoint))
        return self

    @classmethod
    def uneven(cls, lengths, dtype=torch.complex64, graph: bool = False, persistent: bool = False,
               autotune: bool = False) -> "Plan":
        """A plan for transforms of the given power-of-two lengths packed back
        to back in one buffer (fft_plan_create_many); ``self.offsets`` holds
        each transform's first element.  ``persistent`` selects the
        persistent-launch form, ``autotune`` tunes every length class."""
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        lens = [int(v) for v in lengths]
        arr = (ctypes.c_int64 * max(1, len(lens)))(*lens)
        self.dtype_code = dtype_code(dtype)
        self.torch_dtype = torch.complex64 if self.dtype_code == FFT_C64 else torch.complex128
        flags = (FFT_OPT_GRAPH if graph else 0) | (FFT_OPT_PERSISTENT if persistent else 0) | \
            (FFT_OPT_AUTOTUNE if autotune else 0)
        rc = lib().fft_plan_create_many(arr, len(lens), self.dtype_code, flags, ctypes.byref(self._h))
        _check(rc, "fft_plan_create_many(count=%d)" % len(lens))
        self.lengths = lens
        self.offsets = [0] * len(lens)
        acc = 0
        for i, v in enumerate(lens):
            self.offsets[i] = acc
            acc += v
        self.n, self.batch = acc, 1  # execute() checks the packed element count
        return self

    def __init__(self, n: int, batch: int = 1, dtype=torch.complex64, log2_p: int = 0,
                 radix: int = 0, lines_per_block: int = 0, lines_per_block2: int = 0,
                 flags: int = 0, values_per_thread: int = 0, values_per_thread2: int = 0,
                 scratch_width: int = 0, tile_order: int = 0):
        self._h = ctypes.c_void_p()
        self.n, self.batch = int(n), int(batch)
        self.dtype_code = dtype_code(dtype)
        self.torch_dtype = torch.complex64 if self.dtype_code == FFT_C64 else torch.complex128
        opts = PlanOpts(int(log2_p), int(radix), int(lines_per_block), int(lines_per_block2),
                        int(flags), int(values_per_thread), int(values_per_thread2), int(scratch_width),
                        int(tile_order))
        rc = lib().fft_plan_create_ex(self.n, self.batch, self.dtype_code, ctypes.byref(opts),
                                      ctypes.byref(self._h))
        _check(rc, "fft_plan_create_ex(n=%d, batch=%d)" % (self.n, self.batch))

    @property
    def handle(self) -> int:
        if not self._h:
            raise FFTError(-4, "plan already destroyed")
        return self._h.value

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().fft_plan_get_info(self.handle, ctypes.byref(inf)), "fft_plan_get_info")
        return inf.as_dict()

    def execute_ptr(self, in_ptr: int, out_ptr: int, sign: int, stream: int) -> None:
        rc = lib().fft_execute(self.handle, in_ptr, out_ptr, int(sign), stream)
        _check(rc, "fft_execute")

    def execute(self, x: torch.Tensor, out: torch.Tensor, sign: int = -1, stream=None) -> None:
        """out <- F_sign(x); tensors on the plan's device, dtype and size."""
        for t, nm in ((x, "input"), (out, "output")):
            if t.dtype != self.torch_dtype:
                raise FFTError(-2, "%s dtype %s != plan dtype %s" % (nm, t.dtype, self.torch_dtype))
            if not t.is_cuda:
                raise FFTError(-9, "%s must be a GPU tensor" % nm)
            if not t.is_contiguous():
                raise FFTError(-9, "%s must be contiguous" % nm)
            if t.numel() != self.n * self.batch:
                raise FFTError(-1, "%s has %d elements, plan needs %d"
                               % (nm, t.numel(), self.n * self.batch))
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        self.execute_ptr(x.data_ptr(), out.data_ptr(), sign, stream.cuda_stream)

    def set_precision(self, mode) -> None:
        """'fp32' (default), 'f16x2' or 'bf16x2' (radix-16 stages on the matrix cores)."""
        code = {"fp32": 0, "f16x2": 1, "bf16x2": 2}.get(mode, mode)
        _check(lib().fft_plan_set_precision(self.handle, int(code)), "fft_plan_set_precision(%r)" % (mode,))

    def set_timing(self, enable: bool) -> None:
        _check(lib().fft_plan_set_timing(self.handle, int(bool(enable))), "fft_plan_set_timing")

    def read_timing(self, reset: bool = True):
        """([ms per pass] , [launches per pass]) summed since the last reset,
        three entries each (passes the plan does not have read zero)."""
        ms = (ctypes.c_double * 3)()
        cnt = (ctypes.c_int64 * 3)()
        _check(lib().fft_plan_read_timing(self.handle, ctypes.byref(ms), ctypes.byref(cnt),
                                          int(bool(reset))), "fft_plan_read_timing")
        return list(ms), list(cnt)

    def destroy(self) -> None:
        if self._h:
            lib().fft_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


_plans: dict = {}
_plans_lock = threading.Lock()


def cached_plan(n: int, batch: int, dtype, device: torch.device, stream=None) -> Plan:
    """One plan per (n, batch, dtype, device, stream), created on first use.
    A plan's executes share its scratch array, so they must be ordered on one
    stream: work on another stream gets a plan of its own.  Host threads that
    share a stream (the autograd engine runs backward on a thread of its own,
    on the forward's stream) share the plan; :func:`fft` serialises their
    execute calls with the plan's lock."""
    if stream is None:
        stream = torch.cuda.current_stream(device)
    key = (int(n), int(batch), dtype, device.index, int(stream.cuda_stream))
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            with torch.cuda.device(device):
                p = Plan(n, batch, dtype)
            p.lock = threading.Lock()
            _plans[key] = p
    return p


def clear_plan_cache() -> None:
    torch.cuda.synchronize()
    for p in _plans.values():
        p.destroy()
    _plans.clear()


def fft(x: torch.Tensor, sign: int = -1, out: torch.Tensor | None = None) -> torch.Tensor:
    """Unnormalized transform along the last dimension of a complex GPU tensor:
    out[..., k] = sum_j x[..., j] exp(sign 2 pi i j k / n)."""
    if x.dtype not in (torch.complex64, torch.complex128):
        raise FFTError(-2, "fft needs complex64 or complex128, got %s" % x.dtype)
    if not x.is_cuda:
        raise FFTError(-9, "fft runs on the GPU only; got a %s tensor" % x.device)
    n = x.shape[-1] if x.dim() else 0
    x = x.contiguous()
    batch = x.numel() // n if n else 0
    if out is None:
        out = torch.empty_like(x)
    if batch == 0:
        return out
    stream = torch.cuda.current_stream(x.device)
    plan = cached_plan(n, batch, x.dtype, x.device, stream)
    with plan.lock:
        plan.execute(x, out, sign, stream)
    return out
