"""Python binding of libgtt.so (argument marshalling only).

Every step of the transform runs in the HIP kernels of libgtt.so; this module
passes device pointers, sizes and the current HIP stream of torch through the
C ABI of include/gtt.h, and raises if the library is missing.  torch is used
for device memory and streams only.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtt.so")

# gtt_status
OK = 0
STATUS_NAMES = {0: "GTT_OK", 1: "GTT_ERR_INVALID_VALUE", 2: "GTT_ERR_SHAPE", 3: "GTT_ERR_DTYPE",
                4: "GTT_ERR_ALIGNMENT", 5: "GTT_ERR_WORKSPACE", 6: "GTT_ERR_UNSUPPORTED",
                7: "GTT_ERR_HIP", 8: "GTT_ERR_INTERNAL", 9: "GTT_ERR_TIMEOUT"}
ERR_UNSUPPORTED = 6
ERR_TIMEOUT = 9
# gtt_dtype
F64, F32, C128, C64, BF16, F16, I32 = range(7)
FLAG_FP32_INTERMEDIATE = 0x1
FLAG_NO_TUNE = 0x2
FLAG_PERSISTENT = 0x4
FLAG_PER_INSTANCE = 0x8

TORCH_TO_GTT = {torch.float64: F64, torch.float32: F32, torch.complex128: C128,
                torch.complex64: C64, torch.bfloat16: BF16, torch.float16: F16, torch.int32: I32}
# dtype of W (the compute dtype) for each storage dtype
W_DTYPE = {torch.float64: torch.float64, torch.float32: torch.float32,
           torch.complex128: torch.complex128, torch.complex64: torch.complex64,
           torch.bfloat16: torch.float32, torch.float16: torch.float32, torch.int32: torch.int32}

# every symbol declared in include/gtt.h
EXPORTS = ["gtt_plan", "gtt_plan_mixed", "gtt_workspace_size", "gtt_forward", "gtt_inverse",
           "gtt_backward", "gtt_filter", "gtt_compress", "gtt_compress_workspace_size", "gtt_plan_destroy",
           "gtt_status_string",
           "gtt_plan_describe", "gtt_plan_timing", "gtt_plan_timing_read", "gtt_plan_timing_filter", "gtt_set_tuning",
           "gtt_selftest", "gtt_plan_check", "gtt_plan_barrier_limit", "gtt_backward_noalloc"]


# plans whose destruction was deferred because a graph capture was running
_DEFERRED: list = []


def _capturing() -> bool:
    """True while the current stream is capturing a graph."""
    try:
        return bool(torch.cuda.is_available() and torch.cuda.is_current_stream_capturing())
    except Exception:  # interpreter shutdown, no device
        return False


def _destroy_deferred():
    while _DEFERRED and _lib is not None and not _capturing():
        _lib.gtt_plan_destroy(_DEFERRED.pop())


class GTTError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgtt.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2507_02420_amd.build` "
                           "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    P32, P64 = ctypes.POINTER(i32), ctypes.POINTER(i64)
    L.gtt_plan.argtypes = [ctypes.POINTER(vp), i32, P32, P32, i64, P64, P32, ctypes.c_int, u32]
    L.gtt_plan_mixed.argtypes = [ctypes.POINTER(vp), i32, P32, i64, ctypes.c_int, u32]
    L.gtt_workspace_size.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.gtt_forward.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.gtt_inverse.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.gtt_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.gtt_filter.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.gtt_compress.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
    L.gtt_compress_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.gtt_plan_destroy.argtypes = [vp]
    L.gtt_status_string.argtypes = [ctypes.c_int]
    L.gtt_status_string.restype = ctypes.c_char_p
    L.gtt_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    L.gtt_plan_timing.argtypes = [vp, i32]
    L.gtt_plan_timing_read.argtypes = [vp, ctypes.c_char_p, sz]
    L.gtt_plan_timing_filter.argtypes = [vp, ctypes.c_char_p]
    L.gtt_set_tuning.argtypes = [i32, i32, ctypes.c_int, i32, i32, i32, i32]
    L.gtt_selftest.argtypes = []
    L.gtt_plan_check.argtypes = [vp, vp]
    L.gtt_plan_barrier_limit.argtypes = [vp, u32]
    L.gtt_backward_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        if name != "gtt_status_string":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    if not os.environ.get("GTT_NO_TUNE"):
        load_tuning()
    return L


TUNE_PATH = os.path.join(_HERE, "tuned_gfx950.json")
_NAME_TO_GTT = {"f64": F64, "f32": F32, "c128": C128, "c64": C64, "bf16": BF16, "f16": F16, "i32": I32}


def load_tuning(path: Optional[str] = None) -> int:
    """Apply the autotuner's table (tile budget and least row width per radix
    and dtype) to plans created afterwards; returns the number of entries."""
    path = path or os.environ.get("GTT_TUNE_FILE") or TUNE_PATH
    if not os.path.exists(path):
        return 0
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return 0
    n = 0
    for e in table.get("entries", []):
        if not e.get("override", True):
            continue
        st = _lib.gtt_set_tuning(int(e["b"]), int(e.get("n", 0)), _NAME_TO_GTT[e["dtype"]], int(e["lds_budget"]),
                                 int(e["min_row_bytes"]), int(e.get("max_group_digits", 0)), int(e.get("bwd_lds", 0)))
        n += st == OK
    return n


def _check(st: int, where: str):
    if st != OK:
        raise GTTError(st, where)


def _ptr(t: Optional[torch.Tensor]):
    """Device address of a dense tensor.  The library reads memory in plain
    row-major order, so a strided view (a transpose, the column-major result
    of a LAPACK-backed op) or a host tensor is refused rather than misread."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"tensor of shape {tuple(t.shape)} is not on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"tensor of shape {tuple(t.shape)} and strides {t.stride()} is not contiguous; "
                         "call .contiguous() first")
    if t.is_conj() or t.is_neg():
        raise ValueError("lazy conjugate/negative view: call .resolve_conj() / .resolve_neg() first")
    return ctypes.c_void_p(t.data_ptr())


# the current stream's raw handle for the device of `t` (torch's C-level
# query; torch.cuda.current_stream() builds a Stream object, a few
# microseconds, which at one 1024-element vector is a third of a call)
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(t: Optional[torch.Tensor] = None):
    if t is not None and _raw_stream is not None:
        return ctypes.c_void_p(_raw_stream(t.device.index))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _arr(ctype, seq):
    return (ctype * len(seq))(*seq)


class Plan:
    """An execution plan (gtt_plan / gtt_plan_mixed).

    Plan(b, n, batch, dtype)                       uniform batch
    Plan(b=[...], n=[...], dtype=..., x_off=..., w_idx=...)   ragged batch
    Plan.mixed(radices, batch, dtype)             heterogeneous factors
    """

    def __init__(self, b, n, batch: int = 1, dtype=torch.float32, flags: int = 0,
                 x_off: Optional[Sequence[int]] = None, w_idx: Optional[Sequence[int]] = None,
                 _handle=None):
        L = lib()
        self.dtype = dtype
        self.flags = flags
        self._wsz = None
        if _handle is not None:
            self._h = _handle
            return
        bs = list(b) if isinstance(b, (list, tuple)) else [int(b)]
        ns = list(n) if isinstance(n, (list, tuple)) else [int(n)]
        if len(bs) != len(ns):
            raise ValueError("b and n must have the same length")
        self.b, self.n, self.batch = bs, ns, batch
        _destroy_deferred()
        h = ctypes.c_void_p()
        st = L.gtt_plan(ctypes.byref(h), len(bs), _arr(ctypes.c_int32, bs), _arr(ctypes.c_int32, ns),
                        batch, None if x_off is None else _arr(ctypes.c_int64, list(x_off)),
                        None if w_idx is None else _arr(ctypes.c_int32, list(w_idx)),
                        TORCH_TO_GTT[dtype], flags)
        _check(st, "gtt_plan")
        self._h = h

    @classmethod
    def mixed(cls, radices: Sequence[int], batch: int = 1, dtype=torch.complex64, flags: int = 0):
        L = lib()
        h = ctypes.c_void_p()
        st = L.gtt_plan_mixed(ctypes.byref(h), len(radices), _arr(ctypes.c_int32, list(radices)), batch,
                              TORCH_TO_GTT[dtype], flags)
        _check(st, "gtt_plan_mixed")
        p = cls(None, None, batch, dtype, flags, _handle=h)
        p.radices = list(radices)
        p.batch = batch
        return p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            self._h = None
            if _capturing():
                # the garbage collector can run this inside a graph capture;
                # freeing the plan's device memory there would invalidate
                # the capture, so the plan is freed after it
                _DEFERRED.append(h)
            else:
                _lib.gtt_plan_destroy(h)
                _destroy_deferred()

    @property
    def handle(self):
        return self._h

    def workspace_size(self):
        """(forward, backward, saved) workspace bytes: fixed when the plan is
        made, so asked once."""
        if self._wsz is None:
            f, b, s = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
            _check(lib().gtt_workspace_size(self._h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(s)),
                   "gtt_workspace_size")
            self._wsz = (f.value, b.value, s.value)
        return self._wsz

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().gtt_plan_describe(self._h, buf, len(buf)), "gtt_plan_describe")
        return json.loads(buf.value.decode())

    def timing(self, enable: bool = True):
        """Bracket every kernel launch of this plan with HIP events."""
        _check(lib().gtt_plan_timing(self._h, 1 if enable else 0), "gtt_plan_timing")

    def timing_filter(self, prefix: Optional[str] = None):
        """Time only the launches whose name starts with prefix (None: all)."""
        _check(lib().gtt_plan_timing_filter(self._h, None if not prefix else prefix.encode()),
               "gtt_plan_timing_filter")

    def timing_read(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().gtt_plan_timing_read(self._h, buf, len(buf)), "gtt_plan_timing_read")
        return json.loads(buf.value.decode())

    def check(self):
        """Wait for the current stream; raise GTTError(GTT_ERR_TIMEOUT) if a
        persistent ragged launch of this plan gave up at a grid barrier since
        the last check (and clear that record)."""
        _check(lib().gtt_plan_check(self._h, _stream()), "gtt_plan_check")

    def barrier_limit(self, polls: int):
        """Polls a work-group of a persistent ragged launch makes at a grid
        barrier before it gives up (default 2**24)."""
        _check(lib().gtt_plan_barrier_limit(self._h, int(polls)), "gtt_plan_barrier_limit")

    # -- calls ---------------------------------------------------------------
    def _ws(self, nbytes: int, device) -> Optional[torch.Tensor]:
        if nbytes == 0:
            return None
        return torch.empty(nbytes, dtype=torch.uint8, device=device)

    def forward(self, W: torch.Tensor, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                saved: Optional[torch.Tensor] = None) -> torch.Tensor:
        if y is None:
            y = torch.empty_like(x)
        fwd, _, _ = self.workspace_size()
        ws = self._ws(fwd, x.device)
        _check(lib().gtt_forward(self._h, _ptr(W), _ptr(x), _ptr(y), _ptr(saved), _ptr(ws), fwd, _stream(x)),
               "gtt_forward")
        return y

    def inverse(self, W: torch.Tensor, y: torch.Tensor, x: Optional[torch.Tensor] = None) -> torch.Tensor:
        if x is None:
            x = torch.empty_like(y)
        fwd, _, _ = self.workspace_size()
        ws = self._ws(fwd, y.device)
        _check(lib().gtt_inverse(self._h, _ptr(W), _ptr(y), _ptr(x), _ptr(ws), fwd, _stream(y)), "gtt_inverse")
        return x

    def backward(self, W: torch.Tensor, x: torch.Tensor, gy: torch.Tensor, saved: Optional[torch.Tensor] = None,
                 want_gx: bool = True, want_gW: bool = True, gx: Optional[torch.Tensor] = None,
                 gW: Optional[torch.Tensor] = None):
        if want_gx and gx is None:
            gx = torch.empty_like(gy)
        if want_gW and gW is None:
            gW = torch.empty_like(W)
        _, bwd, sv = self.workspace_size()
        need = bwd - sv if saved is not None else bwd
        ws = self._ws(need, x.device)
        _check(lib().gtt_backward(self._h, _ptr(W), _ptr(x), _ptr(saved), _ptr(gy),
                                  _ptr(gx) if want_gx else None, _ptr(gW) if want_gW else None,
                                  _ptr(ws), need, _stream(x)), "gtt_backward")
        return (gx if want_gx else None), (gW if want_gW else None)

    def filter(self, W: torch.Tensor, x: torch.Tensor, cutoff: int, low=True, high=True):
        lo = torch.empty_like(x) if low else None
        hi = torch.empty_like(x) if high else None
        fwd, _, _ = self.workspace_size()
        need = fwd + x.numel() * x.element_size()
        ws = self._ws(need, x.device)
        _check(lib().gtt_filter(self._h, _ptr(W), _ptr(x), int(cutoff), _ptr(lo), _ptr(hi), _ptr(ws), need,
                                _stream(x)), "gtt_filter")
        return lo, hi


def _compress(self, W: torch.Tensor, x: torch.Tensor, k: int, reconstruct: bool = True):
    """(idx, val, recon): the k dominant coefficients of every instance
    (ascending indices) and, optionally, the reconstruction from them."""
    batch = x.numel() // x.shape[-1]
    idx = torch.empty(batch, k, dtype=torch.int64, device=x.device)
    val = torch.empty(batch, k, dtype=x.dtype, device=x.device)
    recon = torch.empty_like(x) if reconstruct else None
    nb = ctypes.c_size_t()
    _check(lib().gtt_compress_workspace_size(self._h, ctypes.byref(nb)), "gtt_compress_workspace_size")
    need = nb.value
    ws = self._ws(need, x.device)
    _check(lib().gtt_compress(self._h, _ptr(W), _ptr(x), int(k), _ptr(idx), _ptr(val), _ptr(recon), _ptr(ws), need,
                              _stream(x)), "gtt_compress")
    return idx, val, recon


Plan.compress = _compress


def set_tuning(b: int, dtype, lds_budget_bytes: int, min_row_bytes: int, max_group_digits: int = 0, n: int = 0,
               bwd_lds_bytes: int = 0):
    """Tiling overrides for plans created afterwards (radix b, n digits or
    every n when n == 0, storage dtype); all zeros restore the defaults."""
    _check(lib().gtt_set_tuning(int(b), int(n), TORCH_TO_GTT[dtype], int(lds_budget_bytes), int(min_row_bytes),
                                int(max_group_digits), int(bwd_lds_bytes)), "gtt_set_tuning")


def selftest() -> int:
    return lib().gtt_selftest()


def forward(W: torch.Tensor, x: torch.Tensor, b: int, n: int) -> torch.Tensor:
    """y = (W kron ... kron W) x along the last dimension of x (N = b**n)."""
    xs = x.reshape(-1, b ** n).contiguous()
    p = Plan(b, n, xs.shape[0], x.dtype)
    return p.forward(W.contiguous(), xs).reshape(x.shape)


def inverse(W: torch.Tensor, y: torch.Tensor, b: int, n: int) -> torch.Tensor:
    ys = y.reshape(-1, b ** n).contiguous()
    p = Plan(b, n, ys.shape[0], y.dtype)
    return p.inverse(W.contiguous(), ys).reshape(y.shape)


class GTTFunction(torch.autograd.Function):
    """y = G_N x with gradients for x and W through gtt_backward.

    forward(x, W, b, n): x is (batch, b**n) on the GPU, W is b x b in the
    compute dtype.  The activations between digit groups are kept from the
    forward call for the backward call.
    """

    @staticmethod
    def forward(ctx, x, W, b: int, n: int):
        xs = x.contiguous()
        batch = xs.numel() // (b ** n)
        plan = Plan(b, n, batch, xs.dtype)
        _, _, sv = plan.workspace_size()
        saved = torch.empty(sv, dtype=torch.uint8, device=xs.device) if sv else None
        y = plan.forward(W.contiguous(), xs, saved=saved)
        ctx.plan = plan
        ctx.save_for_backward(xs, W)
        ctx.saved_act = saved
        return y

    @staticmethod
    def backward(ctx, gy):
        xs, W = ctx.saved_tensors
        gx, gW = ctx.plan.backward(W.contiguous(), xs, gy.contiguous(), saved=ctx.saved_act,
                                   want_gx=ctx.needs_input_grad[0], want_gW=ctx.needs_input_grad[1])
        return gx, gW, None, None


def gtt(x: torch.Tensor, W: torch.Tensor, b: int, n: int) -> torch.Tensor:
    return GTTFunction.apply(x, W, b, n)
