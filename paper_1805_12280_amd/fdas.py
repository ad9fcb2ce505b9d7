"""ctypes binding of libfdas.so (include/fdas.h): argument marshalling only.

Every step of the FT convolution runs in the library's HIP kernels; torch is
used here for device memory and the current stream.  Loading fails loudly
when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfdas.so")

FDAS_OK, FDAS_EINVAL, FDAS_ENOMEM, FDAS_EHIP, FDAS_EUNSUPPORTED = 0, 1, 2, 3, 4
FDAS_FP32 = 0
FDAS_TAPS_ON_DEVICE = 1
FDAS_FP16 = 2
FDAS_BF16 = 4
PRECISIONS = {"fp32": FDAS_FP32, "fp16": FDAS_FP16, "bf16": FDAS_BF16}

MAX_BATCH = 128
MAX_TOPK = 32
STATIC_WORKSPACE_BYTES = 32 << 20

EXPORTED = ("fdas_plan_create", "fdas_plan_set_workgroups_per_cu", "fdas_plan_set_direct_templates",
            "fdas_convolve", "fdas_tdfir",
            "fdas_batched_workspace_bytes",
            "fdas_convolve_batched", "fdas_convolve_batched_static", "fdas_segment_fft",
            "fdas_plan_template_spectra", "fdas_plan_info", "fdas_plan_destroy",
            "fdas_strerror", "fdas_last_error", "fdas_variant_name")


class FdasError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdas error {code}: {msg}")
        self.code = code
        self.msg = msg


class PlanInfo(ctypes.Structure):
    _fields_ = [("seg_fft", ctypes.c_int32), ("valid_per_seg", ctypes.c_int32),
                ("num_segments", ctypes.c_int64), ("k_max", ctypes.c_int32),
                ("num_templates", ctypes.c_int32), ("input_len", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("threads_per_fft", ctypes.c_int32),
                ("fused_grid", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("device", ctypes.c_int32), ("wg_per_cu_max", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("direct_templates", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfdas.so and declare its signatures (raises if it is missing)."""
    global _lib
    if not os.path.exists(path):
        raise FdasError(FDAS_EHIP, f"{path} is not built; run __graft_entry__.build()")
    if _lib is not None and path == LIB_PATH:
        return _lib
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.fdas_plan_create.argtypes = [ctypes.POINTER(vp), vp, vp, i32, i32, i64, i32, ctypes.c_uint32, vp]
    lib.fdas_plan_create.restype = ctypes.c_int
    for name in ("fdas_convolve", "fdas_tdfir"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i64, vp, i64, vp]
        f.restype = ctypes.c_int
    lib.fdas_batched_workspace_bytes.argtypes = [vp, vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdas_batched_workspace_bytes.restype = ctypes.c_int
    lib.fdas_convolve_batched.argtypes = [vp, vp, vp, i32, i32, vp, vp, ctypes.c_size_t, vp]
    lib.fdas_convolve_batched.restype = ctypes.c_int
    lib.fdas_convolve_batched_static.argtypes = [vp, vp, vp, i32, i32, vp, vp]
    lib.fdas_convolve_batched_static.restype = ctypes.c_int
    lib.fdas_segment_fft.argtypes = [vp, vp, vp, i64, i32, vp]
    lib.fdas_segment_fft.restype = ctypes.c_int
    lib.fdas_plan_template_spectra.argtypes = [vp, vp]
    lib.fdas_plan_template_spectra.restype = ctypes.c_int
    lib.fdas_plan_set_workgroups_per_cu.argtypes = [vp, i32]
    lib.fdas_plan_set_workgroups_per_cu.restype = ctypes.c_int
    lib.fdas_plan_set_direct_templates.argtypes = [vp, i32]
    lib.fdas_plan_set_direct_templates.restype = ctypes.c_int
    lib.fdas_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.fdas_plan_info.restype = ctypes.c_int
    lib.fdas_plan_destroy.argtypes = [vp]
    lib.fdas_plan_destroy.restype = None
    lib.fdas_strerror.argtypes = [ctypes.c_int]
    lib.fdas_strerror.restype = ctypes.c_char_p
    lib.fdas_last_error.argtypes = []
    lib.fdas_last_error.restype = ctypes.c_char_p
    lib.fdas_variant_name.argtypes = [i32]
    lib.fdas_variant_name.restype = ctypes.c_char_p
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(rc: int):
    if rc != FDAS_OK:
        lib = load_library()
        raise FdasError(rc, f"{lib.fdas_strerror(rc).decode()}: {lib.fdas_last_error().decode()}")


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _on_stream(stream):
    """Context in which torch allocates buffers for a call enqueued on
    `stream` (None: the current stream), so the caching allocator does not
    hand their memory out again while that stream may still use it."""
    import contextlib
    import torch
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


def split_candidates(raw):
    """(t, bin, p) views of a [count, topk, 3] candidate tensor."""
    import torch
    return raw[..., 0], raw[..., 1], raw[..., 2].view(torch.float32)


class Plan:
    """A template bank resident on the GPU, ready to filter spectra.

    taps:     complex64 [M, K_max] (numpy, CPU or CUDA torch), zero beyond tap_len
    tap_len:  int32 [M] or None (all K_max)
    input_len: largest spectrum length that will be filtered
    seg_fft:  segment transform length L in {1024, 2048, 4096, 8192}
    precision: "fp32", or "fp16" / "bf16" for the mixed plans (16-bit input
               and template spectra, matrix-core inverse transforms, float32
               accumulation and power; L = 2048; convolve() and
               convolve_batched() only, inputs as [n, 2] 16-bit tensors)
    """

    def __init__(self, taps, tap_len=None, input_len: int = 1 << 22, seg_fft: int = 2048,
                 precision: str = "fp32", stream=None):
        import torch
        if precision not in PRECISIONS:
            raise FdasError(FDAS_EINVAL, f"precision {precision!r}: one of {sorted(PRECISIONS)}")
        lib = load_library()
        flags = PRECISIONS[precision]
        self.precision = precision
        keep = []
        if isinstance(taps, torch.Tensor) and taps.is_cuda:
            taps_t = taps.to(torch.complex64).contiguous()
            keep.append(taps_t)
            taps_p = _ptr(taps_t)
            flags |= FDAS_TAPS_ON_DEVICE
            m, k_max = taps_t.shape
            if tap_len is not None:
                tl = torch.as_tensor(tap_len, dtype=torch.int32, device=taps_t.device).contiguous()
                keep.append(tl)
                len_p = _ptr(tl)
            else:
                len_p = None
        else:
            if isinstance(taps, torch.Tensor):
                taps = taps.numpy()
            taps_np = np.ascontiguousarray(np.asarray(taps, dtype=np.complex64))
            if taps_np.ndim != 2:
                raise FdasError(FDAS_EINVAL, "taps must be [M, K_max]")
            keep.append(taps_np)
            taps_p = ctypes.c_void_p(taps_np.ctypes.data)
            m, k_max = taps_np.shape
            if tap_len is not None:
                tl = np.ascontiguousarray(np.asarray(tap_len, dtype=np.int32))
                if tl.shape != (m,):
                    raise FdasError(FDAS_EINVAL, "tap_len must be [M]")
                keep.append(tl)
                len_p = ctypes.c_void_p(tl.ctypes.data)
            else:
                len_p = None
        handle = ctypes.c_void_p()
        check(lib.fdas_plan_create(ctypes.byref(handle), taps_p, len_p, int(m), int(k_max),
                                   int(input_len), int(seg_fft), flags, _stream_handle(stream)))
        self._h = handle
        self._lib = lib
        self.num_templates = int(m)
        self.k_max = int(k_max)
        self.input_len = int(input_len)
        info = self.info
        self.seg_fft = info.seg_fft
        self.device = info.device

    # -- properties ---------------------------------------------------------
    @property
    def info(self) -> PlanInfo:
        out = PlanInfo()
        check(self._lib.fdas_plan_info(self._h, ctypes.byref(out)))
        return out

    @property
    def variant(self) -> str:
        return self._lib.fdas_variant_name(self.info.variant).decode()

    def set_workgroups_per_cu(self, per_cu: int):
        """Cap the persistent grids at per_cu workgroups per CU (0: no cap)."""
        check(self._lib.fdas_plan_set_workgroups_per_cu(self._h, int(per_cu)))

    def set_direct_templates(self, m: int):
        """Run the m shortest templates (whole blocks of 8) by direct
        convolution on the matrix cores and the rest by overlap-save
        (float32 plans; 0: all by overlap-save, -1: the plan's default)."""
        check(self._lib.fdas_plan_set_direct_templates(self._h, int(m)))

    # -- calls --------------------------------------------------------------
    def input_dtype(self):
        """torch dtype of one real component of the input spectrum."""
        import torch
        return {"fp32": torch.float32, "fp16": torch.float16, "bf16": torch.bfloat16}[self.precision]

    def _io(self, x, out, stream=None):
        import torch
        if self.precision == "fp32":
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64):
                raise FdasError(FDAS_EINVAL, "x must be a CUDA complex64 tensor")
            if x.dim() != 1 or not x.is_contiguous():
                raise FdasError(FDAS_EINVAL, "x must be 1-D and contiguous")
        else:
            want = self.input_dtype()
            if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want and x.dim() == 2
                    and x.shape[1] == 2 and x.is_contiguous()):
                raise FdasError(FDAS_EINVAL, f"x must be a contiguous CUDA {want} tensor [n, 2] (re, im)")
        n = x.shape[0]
        if out is None:
            with _on_stream(stream):
                out = torch.empty((self.num_templates, n), dtype=torch.float32, device=x.device)
        if out.dtype != torch.float32 or not out.is_cuda or out.dim() != 2 or out.stride(1) != 1 \
                or out.shape[0] != self.num_templates or out.shape[1] < n:
            raise FdasError(FDAS_EINVAL, "out must be CUDA float32 [M, >=n] with unit column stride")
        return n, out

    def convolve(self, x, out=None, stream=None):
        """Power plane P[t, i] = |sum_k x[i-k] h_t[k]|^2 via overlap-save FDFIR."""
        n, out = self._io(x, out, stream)
        check(self._lib.fdas_convolve(self._h, _ptr(x), n, _ptr(out), out.stride(0),
                                      _stream_handle(stream)))
        return out

    def tdfir(self, x, out=None, stream=None):
        """The same power plane by direct time-domain FIR."""
        n, out = self._io(x, out, stream)
        check(self._lib.fdas_tdfir(self._h, _ptr(x), n, _ptr(out), out.stride(0),
                                   _stream_handle(stream)))
        return out

    def batched_workspace_bytes(self, lengths, topk: int = 16) -> int:
        ns = (ctypes.c_int64 * len(lengths))(*[int(v) for v in lengths])
        out = ctypes.c_size_t()
        check(self._lib.fdas_batched_workspace_bytes(self._h, ns, len(lengths), int(topk),
                                                     ctypes.byref(out)))
        return int(out.value)

    def convolve_batched(self, xs, topk: int = 16, out=None, workspace=None, stream=None):
        """Top-`topk` cells (t, bin, P) of each array's power plane, computed in
        one persistent launch without writing the planes.

        Returns an int32 tensor [count, topk, 3]; use `split_candidates` to
        view it as (t, bin, p)."""
        import torch
        xs = list(xs)
        for x in xs:
            if self.precision == "fp32":
                ok = (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64
                      and x.dim() == 1 and x.is_contiguous())
                what = "a contiguous CUDA complex64 vector"
            else:
                ok = (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == self.input_dtype()
                      and x.dim() == 2 and x.shape[1] == 2 and x.is_contiguous())
                what = f"a contiguous CUDA {self.input_dtype()} tensor [n, 2]"
            if not ok:
                raise FdasError(FDAS_EINVAL, f"each array must be {what}")
        count = len(xs)
        if count < 1 or count > MAX_BATCH:
            raise FdasError(FDAS_EINVAL, f"batch of {count} arrays; 1..{MAX_BATCH} supported")
        lengths = [x.shape[0] for x in xs]
        need = self.batched_workspace_bytes(lengths, topk)
        dev = xs[0].device
        with _on_stream(stream):
            if workspace is None:
                workspace = torch.empty(need, dtype=torch.uint8, device=dev)
            if out is None:
                out = torch.empty((count, topk, 3), dtype=torch.int32, device=dev)
        if out.dtype != torch.int32 or tuple(out.shape) != (count, topk, 3) or not out.is_contiguous():
            raise FdasError(FDAS_EINVAL, "out must be a contiguous int32 [count, topk, 3] tensor")
        ptrs = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
        ns = (ctypes.c_int64 * count)(*lengths)
        check(self._lib.fdas_convolve_batched(self._h, ptrs, ns, count, int(topk), _ptr(out),
                                              _ptr(workspace), workspace.numel(), _stream_handle(stream)))
        return out

    def convolve_batched_static(self, xs, topk: int = 16, out=None, stream=None):
        """convolve_batched with the library's static workspace: the call
        allocates no device memory (pass `out` to allocate none here either).
        Calls that overlap on one GPU race on that workspace."""
        import torch
        xs = list(xs)
        count = len(xs)
        if count < 1 or count > MAX_BATCH:
            raise FdasError(FDAS_EINVAL, f"batch of {count} arrays; 1..{MAX_BATCH} supported")
        if out is None:
            with _on_stream(stream):
                out = torch.empty((count, topk, 3), dtype=torch.int32, device=xs[0].device)
        if out.dtype != torch.int32 or tuple(out.shape) != (count, topk, 3) or not out.is_contiguous():
            raise FdasError(FDAS_EINVAL, "out must be a contiguous int32 [count, topk, 3] tensor")
        ptrs = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
        ns = (ctypes.c_int64 * count)(*[int(x.shape[0]) for x in xs])
        check(self._lib.fdas_convolve_batched_static(self._h, ptrs, ns, count, int(topk), _ptr(out),
                                                     _stream_handle(stream)))
        return out

    def segment_fft(self, x, direction: int = -1, stream=None):
        """The plan's L-point transform on each row of x [count, L] (natural order)."""
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64
                and x.dim() == 2 and x.shape[1] == self.seg_fft and x.is_contiguous()):
            raise FdasError(FDAS_EINVAL, "x must be CUDA complex64 [count, L], contiguous")
        with _on_stream(stream):
            out = torch.empty_like(x)
        check(self._lib.fdas_segment_fft(self._h, _ptr(x), _ptr(out), x.shape[0], int(direction),
                                         _stream_handle(stream)))
        return out

    def template_spectra(self) -> np.ndarray:
        """H_t[q] (1/L folded in), complex64 [M, L], natural order, on the host."""
        out = np.empty((self.num_templates, self.seg_fft), dtype=np.complex64)
        check(self._lib.fdas_plan_template_spectra(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fdas_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
