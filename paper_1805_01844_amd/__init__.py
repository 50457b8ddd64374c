"""MI355X (gfx950) polynomial lossless compressor -- Python binding.

Thin ctypes marshalling over ``libpcomp.so`` (see ``include/pcomp.h``): every step of
compression and decompression runs in the library's HIP kernels; PyTorch only
provides device memory and the current stream. There is no CPU fallback: if the
library is missing the import of the binding fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcomp.so")

SELECT_EXHAUSTIVE = 0x100
SELECT_LEARNED = 0x200
OK, EINVAL, ENOSPC, ECORRUPT, ENOMODEL, EHIP, ENOWS, ENOINIT = 0, -1, -2, -3, -4, -5, -6, -7
_ERR = {EINVAL: "EINVAL", ENOSPC: "ENOSPC", ECORRUPT: "ECORRUPT", ENOMODEL: "ENOMODEL", EHIP: "EHIP",
        ENOWS: "ENOWS", ENOINIT: "ENOINIT"}
SCRATCH_BYTES = 32 << 20  # PCOMP_SCRATCH_BYTES

_DT = {torch.uint8: 1, torch.uint16: 2, torch.uint32: 4}
_TORCH = {1: torch.uint8, 2: torch.uint16, 4: torch.uint32}

_lib = None


class PcompError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, _ERR.get(code, "?"), code))
        self.code = code


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpcomp.so is not built (run __graft_entry__.build()): " + LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        u64, i32, u32, sz, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_void_p
        L.pcomp_init.restype = i32
        L.pcomp_init.argtypes = []
        L.pcomp_bound.restype = sz
        L.pcomp_bound.argtypes = [u64, i32, u32, i32]
        L.pcomp_workspace_size.restype = sz
        L.pcomp_workspace_size.argtypes = [u64, i32, u32, i32]
        L.pcomp_compress.restype = i32
        L.pcomp_compress.argtypes = [vp, u64, i32, u32, i32, vp, sz, vp, vp, sz, vp]
        L.pcomp_compress_noalloc.restype = i32
        L.pcomp_compress_noalloc.argtypes = [vp, u64, i32, u32, i32, vp, sz, vp, vp]
        L.pcomp_decompress.restype = i32
        L.pcomp_decompress.argtypes = [vp, sz, vp, sz, vp, vp]
        L.pcomp_decompress_typed.restype = i32
        L.pcomp_decompress_typed.argtypes = [vp, sz, i32, u32, vp, sz, vp, vp]
        L.pcomp_integrate.restype = i32
        L.pcomp_integrate.argtypes = [vp, i32, u64, u32, vp, vp]
        L.pcomp_compress_transposed.restype = i32
        L.pcomp_compress_transposed.argtypes = [vp, u64, u32, u32, i32, u32, i32, vp, sz, vp, vp, sz, vp]
        L.pcomp_decompress_transposed.restype = i32
        L.pcomp_decompress_transposed.argtypes = [vp, sz, i32, u32, u64, u32, u32, vp, sz, vp, vp]
        L.pcomp_stream_info.restype = i32
        L.pcomp_stream_info.argtypes = [vp, vp, vp, vp, vp]
        L.pcomp_atlas_info.restype = i32
        L.pcomp_atlas_info.argtypes = [u64, vp, vp, vp, vp]
        L.pcomp_atlas_word.restype = i32
        L.pcomp_atlas_word.argtypes = [u64, u32, vp, vp, vp, vp]
        L.pcomp_batch_plan_bytes.restype = sz
        L.pcomp_batch_plan_bytes.argtypes = [vp, u32, vp, i32]
        L.pcomp_batch_plan.restype = i32
        L.pcomp_batch_plan.argtypes = [vp, u32, vp, i32, vp, sz]
        L.pcomp_batch_info.restype = i32
        L.pcomp_batch_info.argtypes = [vp, vp, vp, vp]
        L.pcomp_compress_batch.restype = i32
        L.pcomp_compress_batch.argtypes = [vp, vp, vp, sz, vp, vp, vp, sz, u32, vp]
        L.pcomp_decompress_batch.restype = i32
        L.pcomp_decompress_batch.argtypes = [vp, vp, vp, sz, vp, vp, u32, vp]
        L.pcomp_set_model.restype = i32
        L.pcomp_set_model.argtypes = [vp, sz]
        L.pcomp_block_features.restype = i32
        L.pcomp_block_features.argtypes = [vp, u64, i32, u32, vp, vp, vp, vp, sz, vp]
        L.pcomp_mlp_scores.restype = i32
        L.pcomp_mlp_scores.argtypes = [vp, vp, u64, vp, vp]
        L.pcomp_mlp_workspace_size.restype = sz
        L.pcomp_mlp_workspace_size.argtypes = [u64]
        L.pcomp_mlp_loss_grad.restype = i32
        L.pcomp_mlp_loss_grad.argtypes = [vp, vp, vp, u64, vp, vp, vp, sz, vp]
        L.pcomp_mlp_adam.restype = i32
        L.pcomp_mlp_adam.argtypes = [vp, vp, vp, vp, u32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, vp]
        L.pcomp_bound32.restype = sz
        L.pcomp_bound32.argtypes = [u64, i32, u32, i32]
        L.pcomp_workspace_size32.restype = sz
        L.pcomp_workspace_size32.argtypes = [u64, i32, u32, i32]
        L.pcomp_compress32.restype = i32
        L.pcomp_compress32.argtypes = [vp, u64, i32, u32, i32, vp, sz, vp, vp, sz, vp]
        L.pcomp_decompress32.restype = i32
        L.pcomp_decompress32.argtypes = [vp, sz, i32, u32, vp, sz, vp, vp]
        _lib = L
    return _lib


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise PcompError(rc, what)


def _require(cond, what):
    """Argument checks of the binding (kept under ``python -O``, unlike assert)."""
    if not cond:
        raise ValueError(what)


def _is_values(t: torch.Tensor) -> bool:
    return t.is_cuda and t.is_contiguous() and t.dtype in _DT


def init() -> None:
    _check(lib().pcomp_init(), "pcomp_init")


def bound(n: int, dtype_bytes: int, block_len: int, variant: int) -> int:
    return lib().pcomp_bound(n, dtype_bytes, block_len, variant)


def workspace_size(n: int, dtype_bytes: int, block_len: int, variant: int) -> int:
    return lib().pcomp_workspace_size(n, dtype_bytes, block_len, variant)


class Compressor:
    """Reusable buffers for repeated compression of same-shaped inputs (no allocation per call)."""

    def __init__(self, n: int, dtype: torch.dtype, block_len: int, variant: int, device="cuda"):
        self.n, self.w, self.L, self.variant = int(n), _DT[dtype], int(block_len), int(variant)
        cap = bound(self.n, self.w, self.L, self.variant)
        if cap == 0:
            raise PcompError(EINVAL, "pcomp_bound")
        self.out = torch.empty(cap, dtype=torch.uint8, device=device)
        self.ws = torch.empty(max(8, workspace_size(self.n, self.w, self.L, self.variant)), dtype=torch.uint8,
                              device=device)
        self.size = torch.zeros(1, dtype=torch.int64, device=device)

    def __call__(self, x: torch.Tensor) -> None:
        """Enqueues compression of x on the current stream (asynchronous)."""
        _require(_is_values(x) and x.numel() == self.n and _DT[x.dtype] == self.w and x.device == self.out.device,
                 "x is a contiguous CUDA tensor of the compressor's size, dtype and device")
        rc = lib().pcomp_compress(ctypes.c_void_p(x.data_ptr()), self.n, self.w, self.L, self.variant,
                                  ctypes.c_void_p(self.out.data_ptr()), self.out.numel(),
                                  ctypes.c_void_p(self.size.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                  self.ws.numel(), _stream_handle())
        _check(rc, "pcomp_compress")

    def error_flag(self) -> int:
        """Internal error word of the last call (0 = none; synchronises)."""
        return int(self.ws[:4].view(torch.int32).item())

    def stream(self) -> torch.Tensor:
        """The compressed stream of the last call (synchronises to read its size)."""
        n = int(self.size.item())
        err = self.error_flag()
        if err:
            raise PcompError(EHIP, "pcomp_compress (device error word %d)" % err)
        return self.out[:n]


def compress(x: torch.Tensor, block_len: int, variant: int = 0) -> torch.Tensor:
    """Compresses a contiguous u8/u16/u32 CUDA tensor; returns the stream as a u8 CUDA tensor."""
    x = x.contiguous().reshape(-1)
    c = Compressor(x.numel(), x.dtype, block_len, variant, device=x.device)
    c(x)
    return c.stream()


def stream_info(stream: torch.Tensor):
    """(n, dtype bytes, block_len, total bytes) from the stream header."""
    h = stream[:64].cpu().numpy().tobytes() if stream.is_cuda else bytes(stream[:64].numpy())
    if len(h) < 64:
        raise PcompError(ECORRUPT, "pcomp_stream_info")
    buf = ctypes.create_string_buffer(h, 64)
    n, w, L, tot = ctypes.c_uint64(), ctypes.c_int(), ctypes.c_uint32(), ctypes.c_uint64()
    _check(lib().pcomp_stream_info(buf, ctypes.byref(n), ctypes.byref(w), ctypes.byref(L), ctypes.byref(tot)),
           "pcomp_stream_info")
    return n.value, w.value, L.value, tot.value


def _check_decode_args(stream, out, status):
    _require(stream.is_cuda and stream.dtype == torch.uint8 and stream.is_contiguous(),
             "stream is a contiguous u8 CUDA tensor")
    _require(_is_values(out), "out is a contiguous u8/u16/u32 CUDA tensor")
    _require(status.is_cuda and status.dtype == torch.int32 and status.numel() >= 1, "status is an i32 CUDA tensor")
    _require(stream.device == out.device == status.device, "stream, out and status are on one device")


def decompress_into(stream: torch.Tensor, out: torch.Tensor, status: torch.Tensor, dtype_bytes: int = None,
                    block_len: int = None) -> None:
    """Enqueues decompression into `out` on the current stream (asynchronous); status is i32[1].

    `out` must have the stream's dtype: the library takes its capacity in values of that dtype.
    Without `dtype_bytes` the header is read to check it (a 64-byte copy that synchronises);
    a caller that already knows the stream's element size (from ``stream_info``) passes it, and
    with the block length as well only the matching decoder is launched
    (``pcomp_decompress_typed``)."""
    _check_decode_args(stream, out, status)
    w = stream_info(stream)[1] if dtype_bytes is None else int(dtype_bytes)
    _require(_DT[out.dtype] == w, "out has the stream's dtype (%d bytes per value)" % w)
    if block_len is not None:
        rc = lib().pcomp_decompress_typed(ctypes.c_void_p(stream.data_ptr()), stream.numel(), w, int(block_len),
                                          ctypes.c_void_p(out.data_ptr()), out.numel(),
                                          ctypes.c_void_p(status.data_ptr()), _stream_handle())
        _check(rc, "pcomp_decompress_typed")
        return
    rc = lib().pcomp_decompress(ctypes.c_void_p(stream.data_ptr()), stream.numel(), ctypes.c_void_p(out.data_ptr()),
                                out.numel(), ctypes.c_void_p(status.data_ptr()), _stream_handle())
    _check(rc, "pcomp_decompress")


def decompress(stream: torch.Tensor) -> torch.Tensor:
    n, w, L, tot = stream_info(stream)
    out = torch.empty(max(n, 1), dtype=_TORCH[w], device=stream.device)
    status = torch.zeros(1, dtype=torch.int32, device=stream.device)
    decompress_into(stream, out, status, dtype_bytes=w, block_len=L)
    st = int(status.item())
    if st != OK:
        raise PcompError(st, "pcomp_decompress (device status)")
    return out[:n]


# ---- streams of 32-bit words ---------------------------------------------------------------

class Compressor32:
    """Reusable buffers for streams of 32-bit words (``pcomp_compress32``): variant 0 (basic),
    8 (advanced, u8/u16 data) or SELECT_EXHAUSTIVE (the smaller of the two per block)."""

    def __init__(self, n: int, dtype: torch.dtype, block_len: int, variant: int, device="cuda"):
        self.n, self.w, self.L, self.variant = int(n), _DT[dtype], int(block_len), int(variant)
        cap = lib().pcomp_bound32(self.n, self.w, self.L, self.variant)
        if cap == 0:
            raise PcompError(EINVAL, "pcomp_bound32")
        self.out = torch.empty(cap, dtype=torch.uint8, device=device)
        ws = lib().pcomp_workspace_size32(self.n, self.w, self.L, self.variant)
        self.ws = torch.empty(max(8, ws), dtype=torch.uint8, device=device)
        self.size = torch.zeros(1, dtype=torch.int64, device=device)

    def __call__(self, x: torch.Tensor) -> None:
        _require(_is_values(x) and x.numel() == self.n and _DT[x.dtype] == self.w and x.device == self.out.device,
                 "x is a contiguous CUDA tensor of the compressor's size, dtype and device")
        rc = lib().pcomp_compress32(ctypes.c_void_p(x.data_ptr()), self.n, self.w, self.L, self.variant,
                                    ctypes.c_void_p(self.out.data_ptr()), self.out.numel(),
                                    ctypes.c_void_p(self.size.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                    self.ws.numel(), _stream_handle())
        _check(rc, "pcomp_compress32")

    def error_flag(self) -> int:
        return int(self.ws[:4].view(torch.int32).item())

    def stream(self) -> torch.Tensor:
        n = int(self.size.item())
        err = self.error_flag()
        if err:
            raise PcompError(EHIP, "pcomp_compress32 (device error word %d)" % err)
        return self.out[:n]


def compress32(x: torch.Tensor, block_len: int, variant: int = 0) -> torch.Tensor:
    """Stream of 32-bit words of a contiguous u8/u16/u32 CUDA tensor (a u8 CUDA tensor)."""
    x = x.contiguous().reshape(-1)
    c = Compressor32(x.numel(), x.dtype, block_len, variant, device=x.device)
    c(x)
    return c.stream()


def decompress32_into(stream: torch.Tensor, out: torch.Tensor, status: torch.Tensor, block_len: int) -> None:
    """Enqueues decompression of a stream of 32-bit words into `out` (its dtype is the stream's)."""
    _check_decode_args(stream, out, status)
    rc = lib().pcomp_decompress32(ctypes.c_void_p(stream.data_ptr()), stream.numel(), _DT[out.dtype],
                                  int(block_len), ctypes.c_void_p(out.data_ptr()), out.numel(),
                                  ctypes.c_void_p(status.data_ptr()), _stream_handle())
    _check(rc, "pcomp_decompress32")


def decompress32(stream: torch.Tensor) -> torch.Tensor:
    n, w, L, tot = stream_info(stream)
    out = torch.empty(max(n, 1), dtype=_TORCH[w], device=stream.device)
    status = torch.zeros(1, dtype=torch.int32, device=stream.device)
    decompress32_into(stream, out, status, L)
    st = int(status.item())
    if st != OK:
        raise PcompError(st, "pcomp_decompress32 (device status)")
    return out[:n]


class CompressorTransposed(Compressor):
    """Reusable buffers for time-major blocking of same-shaped matrices [n_mat, rows, cols]
    (``pcomp_compress_transposed``; no allocation per call)."""

    def __init__(self, shape, dtype: torch.dtype, block_len: int, variant: int, device="cuda"):
        n_mat, rows, cols = (int(v) for v in shape)
        _require(rows > 0 and cols > 0, "rows and cols are positive")
        super().__init__(n_mat * rows * cols, dtype, block_len, variant, device=device)
        self.shape = (n_mat, rows, cols)

    def __call__(self, x: torch.Tensor) -> None:
        _require(_is_values(x) and tuple(x.shape) == self.shape and _DT[x.dtype] == self.w and
                 x.device == self.out.device, "x is a contiguous CUDA tensor of the compressor's shape and dtype")
        n_mat, rows, cols = self.shape
        rc = lib().pcomp_compress_transposed(ctypes.c_void_p(x.data_ptr()), n_mat, rows, cols, self.w, self.L,
                                             self.variant, ctypes.c_void_p(self.out.data_ptr()), self.out.numel(),
                                             ctypes.c_void_p(self.size.data_ptr()),
                                             ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream_handle())
        _check(rc, "pcomp_compress_transposed")


def compress_transposed(x: torch.Tensor, block_len: int, variant: int = 0) -> torch.Tensor:
    """Time-major blocking of matrices x [n_mat, rows, cols] (e.g. camera events [events,
    pixels, samples]): the stream of their transposes, read without a transposed copy
    (``pcomp_compress_transposed``)."""
    _require(_is_values(x) and x.dim() == 3 and x.shape[1] > 0 and x.shape[2] > 0,
             "x is a contiguous [n_mat, rows, cols] u8/u16/u32 CUDA tensor")
    n_mat, rows, cols = x.shape
    n, w = x.numel(), _DT[x.dtype]
    cap = bound(n, w, block_len, variant)
    if cap == 0:
        raise PcompError(EINVAL, "pcomp_bound")
    out = torch.empty(cap, dtype=torch.uint8, device=x.device)
    ws = torch.empty(max(8, workspace_size(n, w, block_len, variant)), dtype=torch.uint8, device=x.device)
    size = torch.zeros(1, dtype=torch.int64, device=x.device)
    rc = lib().pcomp_compress_transposed(ctypes.c_void_p(x.data_ptr()), n_mat, rows, cols, w, block_len, variant,
                                         ctypes.c_void_p(out.data_ptr()), cap, ctypes.c_void_p(size.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle())
    _check(rc, "pcomp_compress_transposed")
    err = int(ws[:4].view(torch.int32).item())
    if err:
        raise PcompError(EHIP, "pcomp_compress_transposed (device error word %d)" % err)
    return out[:int(size.item())]


def integrate(traces: torch.Tensor) -> torch.Tensor:
    """Integrated signal (``pcomp_integrate``): the u32 sum of every trace of traces [..., samples]."""
    _require(_is_values(traces) and traces.dim() >= 1 and traces.shape[-1] > 0,
             "traces is a contiguous [..., samples] u8/u16/u32 CUDA tensor")
    samples = traces.shape[-1]
    n = traces.numel() // samples
    out = torch.empty(traces.shape[:-1], dtype=torch.uint32, device=traces.device)
    rc = lib().pcomp_integrate(ctypes.c_void_p(traces.data_ptr()), _DT[traces.dtype], n, samples,
                               ctypes.c_void_p(out.data_ptr()), _stream_handle())
    _check(rc, "pcomp_integrate")
    return out


def decompress_transposed_into(stream: torch.Tensor, out: torch.Tensor, status: torch.Tensor, block_len: int) -> None:
    """Enqueues decompression of a time-major stream back into matrices out [n_mat, rows, cols]."""
    _check_decode_args(stream, out, status)
    _require(out.dim() == 3, "out is [n_mat, rows, cols]")
    n_mat, rows, cols = out.shape
    rc = lib().pcomp_decompress_transposed(ctypes.c_void_p(stream.data_ptr()), stream.numel(), _DT[out.dtype],
                                           int(block_len), n_mat, rows, cols, ctypes.c_void_p(out.data_ptr()),
                                           out.numel(), ctypes.c_void_p(status.data_ptr()), _stream_handle())
    _check(rc, "pcomp_decompress_transposed")


def atlas_info(B: int):
    k, mu, lam, V = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().pcomp_atlas_info(B, ctypes.byref(k), ctypes.byref(mu), ctypes.byref(lam), ctypes.byref(V)),
           "pcomp_atlas_info")
    return k.value, mu.value, lam.value, V.value


def atlas_word(B: int, i: int):
    s, p, R, q = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().pcomp_atlas_word(B, i, ctypes.byref(s), ctypes.byref(p), ctypes.byref(R), ctypes.byref(q)),
           "pcomp_atlas_word")
    return s.value, p.value, R.value, q.value


# ---- batches ---------------------------------------------------------------------------

class _Segment(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("n", ctypes.c_uint64), ("dtype", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


def _block_lens(block_len):
    """Block length per width group (u8, u16, u32) from an int or a 3-sequence."""
    if isinstance(block_len, int):
        return (block_len, block_len, block_len)
    bl = tuple(int(x) for x in block_len)
    _require(len(bl) == 3, "block_len is an int or one length per width group (u8, u16, u32)")
    return bl


class _Plan:
    """A batch plan: host copy (ctypes buffer) and device copy (u8 tensor)."""

    def __init__(self, tensors, block_len, variant, device):
        for t in tensors:
            _require(_is_values(t), "segments are contiguous u8/u16/u32 CUDA tensors")
        self.n_segs = len(tensors)
        self.segs = (_Segment * max(1, self.n_segs))()
        for i, t in enumerate(tensors):
            self.segs[i] = _Segment(t.data_ptr(), t.numel(), _DT[t.dtype], 0)
        self.L = (ctypes.c_uint32 * 3)(*_block_lens(block_len))
        self.variant = int(variant)
        nb = lib().pcomp_batch_plan_bytes(self.segs, self.n_segs, self.L, self.variant)
        if nb == 0:
            raise PcompError(EINVAL, "pcomp_batch_plan_bytes")
        self.host = (ctypes.c_uint64 * ((nb + 7) // 8))()
        _check(lib().pcomp_batch_plan(self.segs, self.n_segs, self.L, self.variant, self.host, nb), "pcomp_batch_plan")
        ob, wb, nt = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pcomp_batch_info(self.host, ctypes.byref(ob), ctypes.byref(wb), ctypes.byref(nt)),
               "pcomp_batch_info")
        self.out_capacity, self.ws_bytes, self.n_tiles = ob.value, wb.value, nt.value
        raw = bytes(memoryview(self.host).cast("B")[:nb])
        self.device = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


class Batch:
    """Compression of a list of segments (any mix of u8/u16/u32 CUDA tensors and lengths) by one
    fixed sequence of launches. Buffers are allocated once; ``compress()`` enqueues the launches
    on the current stream and allocates nothing, so it can be captured in a HIP graph
    (``capture()``). Each segment becomes its own stream, identical to ``compress(segment)``;
    the streams follow one another in ``out`` in the segments' order, ``seg_offsets`` (device)
    says where each starts and ``total`` (device) how many bytes they take together.
    ``grid`` = 0 runs one workgroup per tile; otherwise the per-tile launches are persistent
    with that many workgroups."""

    def __init__(self, tensors, block_len=1024, variant=0, grid=0, device="cuda"):
        self.tensors = list(tensors)
        self.variant, self.grid = int(variant), int(grid)
        self.block_len = _block_lens(block_len)
        self.plan = _Plan(self.tensors, self.block_len, self.variant, device)
        self.out = torch.empty(max(8, self.plan.out_capacity), dtype=torch.uint8, device=device)
        self.ws = torch.empty(max(8, self.plan.ws_bytes), dtype=torch.uint8, device=device)
        self.seg_offsets = torch.zeros(max(1, self.plan.n_segs), dtype=torch.int64, device=device)
        self.total = torch.zeros(1, dtype=torch.int64, device=device)
        self.graph = None

    def compress(self) -> None:
        rc = lib().pcomp_compress_batch(self.plan.host, ctypes.c_void_p(self.plan.device.data_ptr()),
                                        ctypes.c_void_p(self.out.data_ptr()), self.out.numel(),
                                        ctypes.c_void_p(self.seg_offsets.data_ptr()),
                                        ctypes.c_void_p(self.total.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                        self.ws.numel(), self.grid, _stream_handle())
        _check(rc, "pcomp_compress_batch")

    def capture(self):
        """Captures compress() in a CUDA/HIP graph (after one eager warm-up call); returns the graph,
        whose replay() re-runs the whole batch."""
        self.compress()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.compress()
        self.graph = g
        return g

    def error_flag(self) -> int:
        return int(self.ws[:4].view(torch.int32).item())

    def total_bytes(self) -> int:
        return int(self.total.item())

    def offsets(self):
        """Where every segment's stream starts in ``out`` (synchronises)."""
        return self.seg_offsets[:self.plan.n_segs].tolist()

    def file(self) -> torch.Tensor:
        """The whole compressed batch: the first ``total`` bytes of ``out`` (synchronises)."""
        err = self.error_flag()
        if err:
            raise PcompError(EHIP, "pcomp_compress_batch (device error word %d)" % err)
        return self.out[:self.total_bytes()]

    def streams(self):
        """Views of every segment's stream (synchronises)."""
        f = self.file()
        offs = self.offsets() + [f.numel()]
        return [f[offs[i]:offs[i + 1]] for i in range(self.plan.n_segs)]


class BatchDecoder:
    """Decompression of a compressed batch (a Batch's ``out``, or a copy of its first ``total``
    bytes, with its ``seg_offsets``) into destination tensors shaped like its segments."""

    def __init__(self, batch: Batch, outs, grid=0):
        _require(len(outs) == len(batch.tensors), "one destination per segment")
        for t, o in zip(batch.tensors, outs):
            _require(o.numel() == t.numel() and o.dtype == t.dtype, "destinations are shaped like the segments")
        self.batch, self.outs, self.grid = batch, list(outs), int(grid)
        self.plan = _Plan(self.outs, batch.block_len, batch.variant, batch.out.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=batch.out.device)

    def __call__(self, buf: torch.Tensor = None, seg_offsets: torch.Tensor = None) -> None:
        buf = self.batch.out if buf is None else buf
        offs = self.batch.seg_offsets if seg_offsets is None else seg_offsets
        _require(buf.is_cuda and buf.dtype == torch.uint8 and buf.is_contiguous(), "buf is a contiguous u8 CUDA tensor")
        _require(offs.is_cuda and offs.dtype == torch.int64 and offs.is_contiguous() and
                 offs.numel() >= self.plan.n_segs and offs.device == buf.device,
                 "seg_offsets holds one i64 per segment, on the device of buf")
        rc = lib().pcomp_decompress_batch(self.plan.host, ctypes.c_void_p(self.plan.device.data_ptr()),
                                          ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                          ctypes.c_void_p(offs.data_ptr()),
                                          ctypes.c_void_p(self.status.data_ptr()), self.grid, _stream_handle())
        _check(rc, "pcomp_decompress_batch")

    def check(self) -> None:
        st = int(self.status.item())
        if st != OK:
            raise PcompError(st, "pcomp_decompress_batch (device status)")


# ---- learned class selector -----------------------------------------------------------

MLP_PARAMS = 2320
MLP_IN, MLP_OUT = 19, 16


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def set_model(params) -> None:
    """Loads the selector's parameters (2320 floats: tensor, array or sequence; None
    unloads) on the current device."""
    if params is None:
        _check(lib().pcomp_set_model(None, 0), "pcomp_set_model")
        return
    p = torch.as_tensor(params, dtype=torch.float32).detach().cpu().contiguous().reshape(-1)
    _check(lib().pcomp_set_model(ctypes.c_void_p(p.data_ptr()), p.numel()), "pcomp_set_model")


def block_features(x: torch.Tensor, block_len: int, want_x=True, want_words=True, want_label=True):
    """(features [nb, 19] f32, class words [nb, 16] u32-as-int32, labels [nb] u8) of a CUDA
    array, computed on the GPU; entries not wanted are None."""
    _require(x.is_cuda and x.dtype in _DT, "x is a u8/u16/u32 CUDA tensor")
    x = x.contiguous().reshape(-1)
    n, w = x.numel(), _DT[x.dtype]
    nb = (n + block_len - 1) // block_len
    dev = x.device
    fx = torch.empty((max(nb, 1), MLP_IN), dtype=torch.float32, device=dev) if want_x else None
    words = torch.empty((max(nb, 1), 16), dtype=torch.int32, device=dev) if want_words else None
    lab = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if want_label else None
    ws = torch.empty(1024, dtype=torch.uint8, device=dev)
    rc = lib().pcomp_block_features(_vp(x), n, w, block_len, _vp(fx), _vp(words), _vp(lab), _vp(ws), ws.numel(),
                                    _stream_handle())
    _check(rc, "pcomp_block_features")
    cut = lambda t: None if t is None else t[:nb]
    return cut(fx), cut(words), cut(lab)


def _require_mlp_inputs(params: torch.Tensor, X: torch.Tensor):
    _require(params.is_cuda and params.dtype == torch.float32 and params.is_contiguous() and
             params.numel() == MLP_PARAMS, "params is a contiguous f32 CUDA tensor of %d values" % MLP_PARAMS)
    _require(X.is_cuda and X.dtype == torch.float32 and X.is_contiguous() and X.dim() == 2 and
             X.shape[1] == MLP_IN and X.device == params.device,
             "X is a contiguous f32 [n, %d] tensor on the device of params" % MLP_IN)


def mlp_scores(params: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    _require_mlp_inputs(params, X)
    n = X.shape[0]
    S = torch.empty((max(n, 1), MLP_OUT), dtype=torch.float32, device=X.device)
    _check(lib().pcomp_mlp_scores(_vp(params), _vp(X), n, _vp(S), _stream_handle()), "pcomp_mlp_scores")
    return S[:n]


class MLPTrainer:
    """Adam training of the selector on the GPU through the library's kernels."""

    def __init__(self, params: torch.Tensor, max_batch: int, lr=3e-3, betas=(0.9, 0.999), eps=1e-8):
        self.params = params.detach().to(torch.float32).contiguous().clone()
        dev = self.params.device
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.ws = torch.empty(lib().pcomp_mlp_workspace_size(max_batch), dtype=torch.uint8, device=dev)
        self.max_batch, self.lr, self.betas, self.eps, self.step_no = max_batch, lr, betas, eps, 0

    def loss_grad(self, X: torch.Tensor, y: torch.Tensor) -> None:
        _require_mlp_inputs(self.params, X)
        n = X.shape[0]
        _require(0 < n <= self.max_batch, "1 <= batch <= max_batch")
        _require(y.device == X.device and y.dtype == torch.uint8 and y.is_contiguous() and y.numel() >= n,
                 "y holds one u8 label per row of X, on its device")
        rc = lib().pcomp_mlp_loss_grad(_vp(self.params), _vp(X), _vp(y), n, _vp(self.grad), _vp(self.loss),
                                       _vp(self.ws), self.ws.numel(), _stream_handle())
        _check(rc, "pcomp_mlp_loss_grad")

    def step(self, X: torch.Tensor, y: torch.Tensor) -> None:
        self.loss_grad(X, y)
        self.step_no += 1
        rc = lib().pcomp_mlp_adam(_vp(self.params), _vp(self.grad), _vp(self.m), _vp(self.v), self.step_no,
                                  self.lr, self.betas[0], self.betas[1], self.eps, _stream_handle())
        _check(rc, "pcomp_mlp_adam")
