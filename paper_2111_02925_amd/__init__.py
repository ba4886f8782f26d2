"""MI355X-native interpolation compressor (SZ3-Interp hot path) -- Python binding.

Thin ctypes binding of ``libszg.so`` (C ABI in ``include/szg.h``).  It only
marshals arguments: every stage of compression and decompression runs in the
library's HIP kernels on the GPU.  PyTorch is used for device memory and the
current stream.  If the library has not been built, every entry point raises
``SzLibraryMissing`` -- there is no fallback.

Paper: "SZ3: A Modular Framework for Composing Prediction-Based Error-Bounded
Lossy Compressors" (arXiv 2111.02925), Section 6.2 (SZ3-Interp), Section 3.2
(linear-scaling quantizer, Huffman encoder), Algorithm 1 (stage order).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libszg.so")

F32, F64 = 0, 1
ABS, REL, PWREL = 0, 1, 2
LINEAR, CUBIC, ADAPTIVE, LORENZO = 0, 1, 2, 3
OK, ERR_ARG, ERR_DTYPE, ERR_CAPACITY, ERR_CORRUPT, ERR_DEVICE, ERR_NOMEM, ERR_UNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "SZ_OK", -1: "SZ_ERR_ARG", -2: "SZ_ERR_DTYPE", -3: "SZ_ERR_CAPACITY",
                -4: "SZ_ERR_CORRUPT", -5: "SZ_ERR_DEVICE", -6: "SZ_ERR_NOMEM",
                -7: "SZ_ERR_UNSUPPORTED"}
HEADER_BYTES = 128

# every function declared in include/szg.h
EXPORTS = ("sz_ctx_create", "sz_ctx_destroy", "sz_last_error", "sz_default_options",
           "sz_compress_bound", "sz_compress_bound_pwrel", "sz_compress", "sz_decompress",
           "sz_inspect",
           "sz_compress_batch", "sz_set_timing", "sz_set_timing_family", "sz_timing_get",
           "sz_timing_reset",
           "sz_debug_codes", "sz_server_create", "sz_server_submit", "sz_server_poll",
           "sz_server_wait", "sz_server_used_bytes", "sz_server_destroy",
           "sz_lossless_bound", "sz_lossless_pack", "sz_lossless_unpack",
           "sz_compress_noalloc")

# the static scratch of sz_compress_noalloc (SZ_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class SzLibraryMissing(ImportError):
    pass


class SzError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("dim_order", ctypes.c_uint8 * 4), ("subchunks", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("ndim", ctypes.c_int), ("dims", ctypes.c_uint64 * 4),
                ("n", ctypes.c_uint64), ("predictor", ctypes.c_int),
                ("dim_order", ctypes.c_uint8 * 4), ("eb_mode", ctypes.c_int),
                ("eb_user", ctypes.c_double), ("eb", ctypes.c_double),
                ("radius", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("sub", ctypes.c_uint32), ("n_unpred", ctypes.c_uint64), ("nsym", ctypes.c_uint32),
                ("total_words", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64),
                ("coded_dtype", ctypes.c_int), ("signs", ctypes.c_int),
                ("off_signs", ctypes.c_uint64), ("level_mask", ctypes.c_uint32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("d_in", ctypes.c_void_p), ("in_size", ctypes.c_size_t),
                ("dtype", ctypes.c_int), ("ndim", ctypes.c_int), ("dims", ctypes.c_uint64 * 4),
                ("eb_mode", ctypes.c_int), ("eb", ctypes.c_double), ("predictor", ctypes.c_int),
                ("has_options", ctypes.c_int), ("options", Options), ("d_out", ctypes.c_void_p),
                ("out_capacity", ctypes.c_size_t), ("wait_event", ctypes.c_void_p)]


REQ_COMPRESS, REQ_DECOMPRESS = 0, 1


class Field(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("dtype", ctypes.c_int), ("ndim", ctypes.c_int),
                ("dims", ctypes.c_uint64 * 4), ("eb_mode", ctypes.c_int), ("eb", ctypes.c_double),
                ("predictor", ctypes.c_int), ("d_out", ctypes.c_void_p),
                ("out_capacity", ctypes.c_size_t), ("out_size", ctypes.c_size_t),
                ("status", ctypes.c_int)]


_lib = None


def lib():
    """Load libszg.so (raises SzLibraryMissing if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SzLibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    U64P = ctypes.POINTER(ctypes.c_uint64)
    L.sz_ctx_create.argtypes = [I]
    L.sz_ctx_create.restype = P
    L.sz_ctx_destroy.argtypes = [P]
    L.sz_ctx_destroy.restype = None
    L.sz_last_error.argtypes = [P]
    L.sz_last_error.restype = ctypes.c_char_p
    L.sz_default_options.argtypes = [ctypes.POINTER(Options)]
    L.sz_default_options.restype = None
    L.sz_compress_bound.argtypes = [I, I, U64P, ctypes.POINTER(Options)]
    L.sz_compress_bound.restype = SZ
    L.sz_compress_bound_pwrel.argtypes = [I, I, U64P, ctypes.POINTER(Options)]
    L.sz_compress_bound_pwrel.restype = SZ
    L.sz_compress.argtypes = [P, P, I, I, U64P, I, D, I, ctypes.POINTER(Options), P, SZ,
                              ctypes.POINTER(SZ), P]
    L.sz_compress.restype = I
    L.sz_compress_noalloc.argtypes = L.sz_compress.argtypes
    L.sz_compress_noalloc.restype = I
    L.sz_decompress.argtypes = [P, P, SZ, P, SZ, P]
    L.sz_decompress.restype = I
    L.sz_inspect.argtypes = [P, SZ, ctypes.POINTER(Info)]
    L.sz_inspect.restype = I
    L.sz_compress_batch.argtypes = [P, ctypes.POINTER(Field), I, ctypes.POINTER(Options), P]
    L.sz_compress_batch.restype = I
    L.sz_set_timing.argtypes = [P, I]
    L.sz_set_timing.restype = I
    L.sz_set_timing_family.argtypes = [P, ctypes.c_char_p]
    L.sz_set_timing_family.restype = I
    L.sz_timing_get.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(D), U64P]
    L.sz_timing_get.restype = I
    L.sz_timing_reset.argtypes = [P]
    L.sz_timing_reset.restype = I
    L.sz_debug_codes.argtypes = [P, P, SZ, P]
    L.sz_debug_codes.restype = I
    L.sz_server_create.argtypes = [I, SZ, I]
    L.sz_server_create.restype = P
    L.sz_server_submit.argtypes = [P, ctypes.POINTER(Request), U64P]
    L.sz_server_submit.restype = I
    L.sz_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I), ctypes.POINTER(I),
                                 ctypes.POINTER(SZ)]
    L.sz_server_poll.restype = I
    L.sz_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I), ctypes.POINTER(SZ)]
    L.sz_server_wait.restype = I
    L.sz_server_used_bytes.argtypes = [P]
    L.sz_server_used_bytes.restype = SZ
    L.sz_server_destroy.argtypes = [P]
    L.sz_server_destroy.restype = None
    L.sz_lossless_bound.argtypes = [SZ]
    L.sz_lossless_bound.restype = SZ
    L.sz_lossless_pack.argtypes = [ctypes.c_char_p, SZ, P, SZ, ctypes.POINTER(SZ), I]
    L.sz_lossless_pack.restype = I
    L.sz_lossless_unpack.argtypes = [ctypes.c_char_p, SZ, P, SZ, ctypes.POINTER(SZ)]
    L.sz_lossless_unpack.restype = I
    _lib = L
    return L


def _mode(v) -> int:
    if isinstance(v, str):
        return {"abs": ABS, "rel": REL, "pwrel": PWREL}[v.lower()]
    return int(v)


def _pred(v) -> int:
    if isinstance(v, str):
        return {"linear": LINEAR, "cubic": CUBIC, "adaptive": ADAPTIVE, "lorenzo": LORENZO}[v.lower()]
    return int(v)


def make_options(radius: int = 32768, chunk: int = 4096, dim_order=None, ndim: int = 4,
                 subchunks: int = 0) -> Options:
    o = Options()
    o.radius = radius
    o.chunk = chunk
    o.subchunks = subchunks
    order = list(dim_order) if dim_order is not None else list(range(ndim))
    order += list(range(len(order), 4))
    for j in range(4):
        o.dim_order[j] = order[j]
    return o


def _dims(shape):
    d = (ctypes.c_uint64 * 4)(1, 1, 1, 1)
    for i, s in enumerate(shape):
        d[i] = int(s)
    return d


def compress_bound(shape, dtype: int = F32, radius: int = 32768, chunk: int = 4096,
                   dim_order=None, subchunks: int = 0, eb_mode=ABS) -> int:
    o = make_options(radius, chunk, dim_order, len(shape), subchunks)
    fn = lib().sz_compress_bound_pwrel if _mode(eb_mode) == PWREL else lib().sz_compress_bound
    return int(fn(dtype, len(shape), _dims(shape), ctypes.byref(o)))


def inspect(stream) -> dict:
    """Decode a stream header held in host memory (bytes / numpy / CPU tensor)."""
    b = bytes(stream[:HEADER_BYTES]) if not hasattr(stream, "cpu") else bytes(
        stream[:HEADER_BYTES].cpu().numpy().tobytes())
    buf = ctypes.create_string_buffer(b, len(b))
    info = Info()
    rc = lib().sz_inspect(ctypes.cast(buf, ctypes.c_void_p), len(b), ctypes.byref(info))
    if rc:
        raise SzError(rc, "sz_inspect")
    return {f: (list(getattr(info, f))[: info.ndim] if f in ("dims", "dim_order") else getattr(info, f))
            for f, _ in Info._fields_}


def lossless_pack(data, level: int = 1) -> bytes:
    """The host lossless stage: zlib stream of `data` (bytes, numpy or a CPU
    uint8 tensor) at zlib level 0..9."""
    b = _host_bytes(data)
    cap = int(lib().sz_lossless_bound(ctypes.c_size_t(len(b))))
    out = ctypes.create_string_buffer(max(cap, 1))
    size = ctypes.c_size_t(0)
    rc = lib().sz_lossless_pack(b, ctypes.c_size_t(len(b)), out, ctypes.c_size_t(cap),
                                ctypes.byref(size), int(level))
    if rc:
        raise SzError(rc, "sz_lossless_pack")
    return out.raw[: size.value]


def lossless_unpack(data, size_hint: int = 0) -> bytes:
    """Inverse of lossless_pack; the output buffer grows until it fits."""
    b = _host_bytes(data)
    cap = max(size_hint, 4 * len(b) + 4096)
    while True:
        out = ctypes.create_string_buffer(cap)
        size = ctypes.c_size_t(0)
        rc = lib().sz_lossless_unpack(b, ctypes.c_size_t(len(b)), out, ctypes.c_size_t(cap),
                                      ctypes.byref(size))
        if rc == -3:  # SZ_ERR_CAPACITY
            cap *= 2
            continue
        if rc:
            raise SzError(rc, "sz_lossless_unpack")
        return out.raw[: size.value]


def _host_bytes(data) -> bytes:
    if isinstance(data, (bytes, bytearray)):
        return bytes(data)
    if hasattr(data, "is_cuda"):
        if data.is_cuda:
            raise ValueError("the lossless stage works on host memory")
        return data.numpy().tobytes()
    return bytes(memoryview(data).cast("B"))


def _torch():
    import torch

    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


class Context:
    """A library context on one GPU (owns the scratch memory)."""

    def __init__(self, device: int = 0):
        self._lib = lib()
        self.device = device
        self._h = self._lib.sz_ctx_create(device)
        if not self._h:
            raise SzError(ERR_DEVICE, f"sz_ctx_create({device}) failed")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sz_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc, what):
        msg = self._lib.sz_last_error(self._h)
        return SzError(rc, f"{what}: {msg.decode() if msg else ''}")

    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def compress(self, x, eb_mode="rel", eb: float = 1e-3, predictor="cubic",
                 radius: int = 32768, chunk: int = 4096, dim_order=None, subchunks: int = 0,
                 out=None, stream=None):
        """Compress a contiguous float32/float64 CUDA tensor; returns a uint8
        CUDA tensor holding the stream (a view of `out` if given)."""
        return self._compress("sz_compress", x, eb_mode, eb, predictor, radius, chunk,
                              dim_order, subchunks, out, stream)

    def compress_noalloc(self, x, out, eb_mode="rel", eb: float = 1e-3, predictor="cubic",
                         radius: int = 32768, chunk: int = 4096, dim_order=None,
                         subchunks: int = 0, stream=None):
        """sz_compress_noalloc: as compress, into the caller's `out` (uint8
        CUDA tensor); the library allocates no device memory for the call."""
        if out is None:
            raise ValueError("compress_noalloc needs the output buffer")
        return self._compress("sz_compress_noalloc", x, eb_mode, eb, predictor, radius, chunk,
                              dim_order, subchunks, out, stream)

    def _compress(self, entry, x, eb_mode, eb, predictor, radius, chunk, dim_order, subchunks,
                  out, stream):
        torch = _torch()
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor")
        opts = make_options(radius, chunk, dim_order, x.dim(), subchunks)
        dims = _dims(x.shape)
        if out is None:
            fn = (self._lib.sz_compress_bound_pwrel if _mode(eb_mode) == PWREL
                  else self._lib.sz_compress_bound)
            cap = int(fn(_dtype_code(x), x.dim(), dims, ctypes.byref(opts)))
            out = torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device)
        elif not out.is_cuda or out.dtype != torch.uint8 or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 CUDA tensor")
        size = ctypes.c_size_t(0)
        rc = getattr(self._lib, entry)(self._h, ctypes.c_void_p(x.data_ptr()), _dtype_code(x),
                                       x.dim(), dims, _mode(eb_mode), float(eb), _pred(predictor),
                                       ctypes.byref(opts), ctypes.c_void_p(out.data_ptr()),
                                       out.numel(), ctypes.byref(size), self._stream(stream))
        if rc:
            err = self._err(rc, entry)
            err.required = size.value
            raise err
        return out[: size.value]

    def decompress(self, stream_t, out=None, stream=None):
        """Decompress a uint8 CUDA tensor holding a stream; returns the field."""
        torch = _torch()
        if not stream_t.is_cuda or stream_t.dtype != torch.uint8:
            raise ValueError("stream must be a uint8 CUDA tensor")
        if out is None:  # (with `out` given, the library reads the header itself)
            info = inspect(stream_t[:HEADER_BYTES].cpu())
            dt = torch.float64 if info["dtype"] == F64 else torch.float32
            out = torch.empty(tuple(info["dims"]), dtype=dt, device=stream_t.device)
        elif not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA tensor")
        rc = self._lib.sz_decompress(self._h, ctypes.c_void_p(stream_t.data_ptr()),
                                     stream_t.numel(), ctypes.c_void_p(out.data_ptr()),
                                     out.numel() * out.element_size(), self._stream(stream))
        if rc:
            raise self._err(rc, "sz_decompress")
        return out

    def compress_batch(self, fields, radius: int = 32768, chunk: int = 4096, subchunks: int = 0,
                       stream=None):
        """fields: list of (tensor, eb_mode, eb, predictor).  Returns the list
        of stream tensors (views of per-field output buffers)."""
        return self.prepare_batch(fields, radius, chunk, subchunks).run(stream)

    def prepare_batch(self, fields, radius: int = 32768, chunk: int = 4096, subchunks: int = 0):
        """A batch whose argument array and output buffers are built once, for
        calls repeated on the same inputs (BatchCall.run)."""
        return BatchCall(self, fields, radius, chunk, subchunks)

    def debug_codes(self, n: int, device="cuda"):
        torch = _torch()
        t = torch.empty(max(n, 1), dtype=torch.int16, device=device)
        rc = self._lib.sz_debug_codes(self._h, ctypes.c_void_p(t.data_ptr()), 2 * n,
                                      self._stream(None))
        if rc:
            raise self._err(rc, "sz_debug_codes")
        return t[:n]

    def set_timing(self, on: bool = True):
        self._lib.sz_set_timing(self._h, 1 if on else 0)

    def set_timing_family(self, name=None):
        """Time only the kernel family `name` (None: every family)."""
        self._lib.sz_set_timing_family(self._h, name.encode() if name else None)

    def timing_reset(self):
        self._lib.sz_timing_reset(self._h)

    def timing(self, name: str):
        ms = ctypes.c_double(0)
        cnt = ctypes.c_uint64(0)
        self._lib.sz_timing_get(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(cnt))
        return ms.value, cnt.value


class BatchCall:
    """The arguments of one sz_compress_batch call (field array, options,
    output buffers sized by the compression bound), kept for repeated runs."""

    def __init__(self, ctx: "Context", fields, radius: int, chunk: int, subchunks: int):
        torch = _torch()
        self._ctx = ctx
        self._arr = (Field * len(fields))()
        self._opts = make_options(radius, chunk, None, 4, subchunks)
        self.outs = []
        for i, (x, mode, eb, pred) in enumerate(fields):
            if not x.is_cuda or not x.is_contiguous():
                raise ValueError("fields must be contiguous CUDA tensors")
            o1 = make_options(radius, chunk, None, x.dim(), subchunks)
            fn = (ctx._lib.sz_compress_bound_pwrel if _mode(mode) == PWREL
                  else ctx._lib.sz_compress_bound)
            cap = int(fn(_dtype_code(x), x.dim(), _dims(x.shape), ctypes.byref(o1)))
            out = torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device)
            self.outs.append(out)
            f = self._arr[i]
            f.d_in = x.data_ptr()
            f.dtype = _dtype_code(x)
            f.ndim = x.dim()
            for d in range(4):
                f.dims[d] = int(x.shape[d]) if d < x.dim() else 1
            f.eb_mode = _mode(mode)
            f.eb = float(eb)
            f.predictor = _pred(pred)
            f.d_out = out.data_ptr()
            f.out_capacity = out.numel()
        self._keep = [x for x, *_ in fields]  # the inputs stay alive with the call

    def run(self, stream=None):
        ctx = self._ctx
        rc = ctx._lib.sz_compress_batch(ctx._h, self._arr, len(self.outs), ctypes.byref(self._opts),
                                        ctx._stream(stream))
        if rc:
            raise ctx._err(rc, "sz_compress_batch")
        return [self.outs[i][: self._arr[i].out_size] for i in range(len(self.outs))]


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def compress(x, eb_mode="rel", eb: float = 1e-3, predictor="cubic", **kw):
    return default_context(x.device.index or 0).compress(x, eb_mode, eb, predictor, **kw)


def decompress(stream_t, **kw):
    return default_context(stream_t.device.index or 0).decompress(stream_t, **kw)


class Server:
    """Request server on one GPU: compression / decompression requests run
    concurrently by `workers` threads within a device-memory budget.  The
    tensors of a request are kept referenced until it is done."""

    def __init__(self, device: int = 0, budget_bytes: int = 8 << 30, workers: int = 4):
        self._lib = lib()
        self.device = device
        self._h = self._lib.sz_server_create(device, int(budget_bytes), int(workers))
        if not self._h:
            raise SzError(ERR_DEVICE, f"sz_server_create({device}, {budget_bytes}, {workers}) failed")
        self._keep = {}

    def submit_compress(self, x, eb_mode="rel", eb: float = 1e-3, predictor="cubic",
                        radius: int = 32768, chunk: int = 4096, dim_order=None, subchunks: int = 0,
                        out=None) -> int:
        torch = _torch()
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous CUDA tensor")
        opts = make_options(radius, chunk, dim_order, x.dim(), subchunks)
        if out is None:
            cap = compress_bound(tuple(x.shape), _dtype_code(x), radius, chunk, dim_order, subchunks,
                                 eb_mode)
            out = torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device)
        r = Request()
        r.kind = REQ_COMPRESS
        r.d_in = x.data_ptr()
        r.dtype = _dtype_code(x)
        r.ndim = x.dim()
        for d in range(4):
            r.dims[d] = int(x.shape[d]) if d < x.dim() else 1
        r.eb_mode = _mode(eb_mode)
        r.eb = float(eb)
        r.predictor = _pred(predictor)
        r.has_options = 1
        r.options = opts
        r.d_out = out.data_ptr()
        r.out_capacity = out.numel()
        return self._submit(r, (x, out))

    def submit_decompress(self, stream_t, out=None) -> int:
        torch = _torch()
        info = inspect(stream_t[:HEADER_BYTES].cpu())
        if out is None:
            dt = torch.float64 if info["dtype"] == F64 else torch.float32
            out = torch.empty(tuple(info["dims"]), dtype=dt, device=stream_t.device)
        r = Request()
        r.kind = REQ_DECOMPRESS
        r.d_in = stream_t.data_ptr()
        r.in_size = stream_t.numel()
        r.d_out = out.data_ptr()
        r.out_capacity = out.numel() * out.element_size()
        return self._submit(r, (stream_t, out))

    def _submit(self, r, keep) -> int:
        # the request's work waits, on the device, for what torch's current
        # stream has queued so far: the input's producer and the output's
        # earlier users
        torch = _torch()
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        r.wait_event = ev.cuda_event
        t = ctypes.c_uint64(0)
        rc = self._lib.sz_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if rc:
            raise SzError(rc, "sz_server_submit")
        self._keep[t.value] = keep + (ev,)
        return t.value

    def poll(self, ticket: int):
        """None while running; else (status, output tensor view)."""
        done, st, sz = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_size_t(0)
        rc = self._lib.sz_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st),
                                      ctypes.byref(sz))
        if rc:
            raise SzError(rc, "sz_server_poll")
        if not done.value:
            return None
        return self._finish(ticket, st.value, sz.value)

    def wait(self, ticket: int):
        st, sz = ctypes.c_int(0), ctypes.c_size_t(0)
        rc = self._lib.sz_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(sz))
        if rc:
            raise SzError(rc, "sz_server_wait")
        return self._finish(ticket, st.value, sz.value)

    def _finish(self, ticket, status, size):
        x, out, _ev = self._keep.pop(ticket)
        if status:
            return status, None
        if out.dtype == _torch().uint8:
            return status, out[:size]
        return status, out

    def used_bytes(self) -> int:
        return int(self._lib.sz_server_used_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sz_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
