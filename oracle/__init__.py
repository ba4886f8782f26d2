"""CPU oracle for the interpolation compressor hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and
shares no code with it.  The arithmetic lives in ``szo.c`` / ``szo_typed.inc``
(plain single-threaded C); this module only marshals numpy arrays through
ctypes.

Parity pins: see ``tests/test_oracle_pins.py`` and ``tests/golden/``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "szo.c")]
DEPS = SOURCES + [os.path.join(_HERE, "szo.h"), os.path.join(_HERE, "szo_typed.inc")]

F32, F64 = 0, 1
ABS, REL, PWREL = 0, 1, 2
LINEAR, CUBIC, ADAPTIVE, LORENZO = 0, 1, 2, 3
OK, ERR_ARG, ERR_CAPACITY, ERR_CORRUPT, ERR_NOMEM = 0, -1, -3, -4, -6
HEADER_BYTES = 128


def build(force: bool = True) -> str:
    """Compile the oracle with strict IEEE settings (no contraction, no fast
    math, no -march so no FMA)."""
    if not force and os.path.exists(LIB_PATH) and all(
        os.path.getmtime(LIB_PATH) >= os.path.getmtime(p) for p in DEPS
    ):
        return LIB_PATH
    cmd = [
        "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
        "-fno-strict-aliasing", "-Wall", "-Wextra", "-fPIC", "-shared",
        "-o", LIB_PATH + ".tmp", *SOURCES, "-lm",
    ]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, U64, I, D = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        U32 = ctypes.c_uint32
        L.szo_resolve_eb.argtypes = [P, U64, I, I, D, ctypes.POINTER(D)]
        L.szo_predict_quantize.argtypes = [P, I, I, P, P, I, D, U32, P, P]
        L.szo_reconstruct.argtypes = [P, P, U64, I, I, P, P, I, D, U32, P]
        L.szo_quantize_one.argtypes = [I, P, P, D, U32, P, P]
        L.szo_check_traversal.argtypes = [I, P, P, I, P, ctypes.POINTER(U64)]
        L.szo_histogram.argtypes = [P, U64, U32, P]
        L.szo_huffman_lengths.argtypes = [P, U32, P]
        L.szo_canonical_codes.argtypes = [P, U32, P]
        L.szo_check_sub.argtypes = [U32, U32]
        L.szo_pack.argtypes = [P, U64, P, P, U32, U32, P, P, P, ctypes.POINTER(U64)]
        L.szo_unpack.argtypes = [P, U64, P, U64, U32, U32, P, P, U32, P]
        L.szo_compress.argtypes = [P, I, I, P, I, D, I, U32, U32, U32, P,
                                   ctypes.POINTER(ctypes.POINTER(ctypes.c_uint8)),
                                   ctypes.POINTER(U64), P, P]
        L.szo_decompress.argtypes = [P, U64, P, U64, P]
        L.szo_free.argtypes = [P]
        for name in ("szo_log2", "szo_exp2"):
            getattr(L, name).argtypes = [D]
            getattr(L, name).restype = D
        L.szo_pwrel_delta.argtypes = [D, I]
        L.szo_pwrel_delta.restype = D
        for name in ("szo_resolve_eb", "szo_predict_quantize", "szo_reconstruct",
                     "szo_quantize_one", "szo_check_traversal", "szo_histogram",
                     "szo_huffman_lengths", "szo_canonical_codes", "szo_check_sub", "szo_pack",
                     "szo_unpack", "szo_compress", "szo_decompress"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dtype_code(x: np.ndarray) -> int:
    if x.dtype == np.float32:
        return F32
    if x.dtype == np.float64:
        return F64
    raise TypeError(f"unsupported dtype {x.dtype}")


def _dims(shape):
    return np.ascontiguousarray(np.array(shape, dtype=np.uint64))


def _order(order, ndim):
    if order is None:
        return None
    o = np.ascontiguousarray(np.array(order, dtype=np.uint8))
    assert o.size == ndim
    return o


def resolve_eb(x: np.ndarray, mode: int, value: float) -> float:
    x = np.ascontiguousarray(x)
    out = ctypes.c_double()
    rc = lib().szo_resolve_eb(_ptr(x), x.size, _dtype_code(x), mode, value, ctypes.byref(out))
    if rc:
        raise OracleError(rc, "resolve_eb")
    return out.value


def predict_quantize(x: np.ndarray, eb_t: float, predictor: int = LINEAR,
                     radius: int = 32768, order=None):
    """Returns (codes u16, recon T) for the whole field."""
    x = np.ascontiguousarray(x)
    codes = np.empty(x.shape, dtype=np.uint16)
    recon = np.empty_like(x)
    d = _dims(x.shape)
    o = _order(order, x.ndim)
    rc = lib().szo_predict_quantize(_ptr(x), _dtype_code(x), x.ndim, _ptr(d), _ptr(o),
                                    predictor, eb_t, radius, _ptr(codes), _ptr(recon))
    if rc:
        raise OracleError(rc, "predict_quantize")
    return codes, recon


def reconstruct(codes: np.ndarray, unpred: np.ndarray, eb_t: float, predictor: int = LINEAR,
                radius: int = 32768, order=None) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    unpred = np.ascontiguousarray(unpred)
    out = np.empty(codes.shape, dtype=unpred.dtype)
    d = _dims(codes.shape)
    o = _order(order, codes.ndim)
    rc = lib().szo_reconstruct(_ptr(codes), _ptr(unpred), unpred.size, _dtype_code(unpred),
                               codes.ndim, _ptr(d), _ptr(o), predictor, eb_t, radius, _ptr(out))
    if rc:
        raise OracleError(rc, "reconstruct")
    return out


def quantize_one(x, pred, eb_t: float, radius: int = 32768, dtype=np.float32):
    xa = np.array([x], dtype=dtype)
    pa = np.array([pred], dtype=dtype)
    code = np.zeros(1, dtype=np.uint16)
    rec = np.zeros(1, dtype=dtype)
    rc = lib().szo_quantize_one(_dtype_code(xa), _ptr(xa), _ptr(pa), eb_t, radius,
                                _ptr(code), _ptr(rec))
    if rc:
        raise OracleError(rc, "quantize_one")
    return int(code[0]), rec[0]


def check_traversal(shape, predictor: int = CUBIC, order=None):
    """Returns (visit counts array, number of stencil reads of non-final points)."""
    d = _dims(shape)
    n = int(np.prod(shape)) if len(shape) else 0
    visits = np.zeros(max(n, 1), dtype=np.uint32)
    early = ctypes.c_uint64()
    o = _order(order, len(shape))
    rc = lib().szo_check_traversal(len(shape), _ptr(d), _ptr(o), predictor, _ptr(visits),
                                   ctypes.byref(early))
    if rc:
        raise OracleError(rc, "check_traversal")
    return visits[:n].reshape(shape), early.value


def histogram(codes: np.ndarray, nsym: int) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint16).ravel()
    h = np.zeros(nsym, dtype=np.uint64)
    rc = lib().szo_histogram(_ptr(codes), codes.size, nsym, _ptr(h))
    if rc:
        raise OracleError(rc, "histogram")
    return h


def huffman_lengths(hist: np.ndarray) -> np.ndarray:
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    lens = np.zeros(hist.size, dtype=np.uint8)
    rc = lib().szo_huffman_lengths(_ptr(hist), hist.size, _ptr(lens))
    if rc < 0:
        raise OracleError(rc, "huffman_lengths")
    return lens


def canonical_codes(lens: np.ndarray) -> np.ndarray:
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    cw = np.zeros(lens.size, dtype=np.uint64)
    rc = lib().szo_canonical_codes(_ptr(lens), lens.size, _ptr(cw))
    if rc:
        raise OracleError(rc, "canonical_codes")
    return cw


def check_sub(chunk: int, sub: int) -> bool:
    return lib().szo_check_sub(chunk, sub) == 0


def pack(codes: np.ndarray, lens: np.ndarray, cw: np.ndarray, chunk: int, sub: int = 1):
    """Returns (words u32, chunk_words u32), plus the sub-chunk bit offsets
    (u32, (sub - 1) per chunk) when sub > 1."""
    codes = np.ascontiguousarray(codes, dtype=np.uint16).ravel()
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    cw = np.ascontiguousarray(cw, dtype=np.uint64)
    nchunks = (codes.size + chunk - 1) // chunk
    cwords = np.zeros(max(nchunks, 1), dtype=np.uint32)
    sbits = np.zeros(max(nchunks * (sub - 1), 1), dtype=np.uint32)
    total = ctypes.c_uint64()
    rc = lib().szo_pack(_ptr(codes), codes.size, _ptr(lens), _ptr(cw), chunk, sub, None,
                        _ptr(cwords), _ptr(sbits), ctypes.byref(total))
    if rc:
        raise OracleError(rc, "pack(count)")
    words = np.zeros(max(total.value, 1), dtype=np.uint32)
    rc = lib().szo_pack(_ptr(codes), codes.size, _ptr(lens), _ptr(cw), chunk, sub, _ptr(words),
                        _ptr(cwords), _ptr(sbits), ctypes.byref(total))
    if rc:
        raise OracleError(rc, "pack")
    if sub > 1:
        return words[: total.value], cwords[:nchunks], sbits[: nchunks * (sub - 1)]
    return words[: total.value], cwords[:nchunks]


def unpack(words: np.ndarray, chunk_words: np.ndarray, n: int, chunk: int,
           lens: np.ndarray, sub: int = 1, sub_bits=None) -> np.ndarray:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    chunk_words = np.ascontiguousarray(chunk_words, dtype=np.uint32)
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    codes = np.zeros(max(n, 1), dtype=np.uint16)
    w = words if words.size else np.zeros(1, dtype=np.uint32)
    cwd = chunk_words if chunk_words.size else np.zeros(1, dtype=np.uint32)
    sb = None
    if sub > 1:
        sb = np.ascontiguousarray(sub_bits, dtype=np.uint32)
        sb = sb if sb.size else np.zeros(1, dtype=np.uint32)
    rc = lib().szo_unpack(_ptr(w), words.size, _ptr(cwd), n, chunk, sub, _ptr(sb), _ptr(lens),
                          lens.size, _ptr(codes))
    if rc:
        raise OracleError(rc, "unpack")
    return codes[:n]


def default_sub(chunk: int) -> int:
    """The sub-chunk count used by default: 4, or fewer when the chunk is too
    short to split that far."""
    for s in (4, 2, 1):
        if check_sub(chunk, s):
            return s
    return 1


def compress(x: np.ndarray, eb_mode: int, eb: float, predictor: int = LINEAR,
             radius: int = 32768, chunk: int = 4096, order=None, want_debug: bool = False,
             sub: int = None):
    """Whole pipeline.  Returns the stream bytes, or (stream, codes, recon)."""
    x = np.ascontiguousarray(x)
    d = _dims(x.shape)
    o = _order(order, x.ndim)
    out = ctypes.POINTER(ctypes.c_uint8)()
    size = ctypes.c_uint64()
    codes = np.empty(x.shape, dtype=np.uint16) if want_debug else None
    recon = np.empty_like(x) if want_debug else None
    xin = x if x.size else np.zeros(1, dtype=x.dtype)
    if sub is None:
        sub = default_sub(chunk)
    rc = lib().szo_compress(_ptr(xin), _dtype_code(x), x.ndim, _ptr(d), eb_mode, eb, predictor,
                            radius, chunk, sub, _ptr(o), ctypes.byref(out), ctypes.byref(size),
                            _ptr(codes), _ptr(recon))
    if rc:
        raise OracleError(rc, "compress")
    try:
        stream = bytes(ctypes.string_at(out, size.value))
    finally:
        lib().szo_free(out)
    if want_debug:
        return stream, codes, recon
    return stream


def log2(a: float) -> float:
    """The point-wise relative mode's logarithm (series in szo.c)."""
    return lib().szo_log2(float(a))


def exp2(y: float) -> float:
    return lib().szo_exp2(float(y))


def pwrel_delta(eps: float, dtype: int = F32) -> float:
    return lib().szo_pwrel_delta(float(eps), dtype)


def parse_header(stream: bytes) -> dict:
    """Decode the fixed 128-byte header (layout documented in szo.c)."""
    b = stream
    if len(b) < HEADER_BYTES:
        raise ValueError("short stream")
    u16 = lambda o: int.from_bytes(b[o:o + 2], "little")
    u32 = lambda o: int.from_bytes(b[o:o + 4], "little")
    u64 = lambda o: int.from_bytes(b[o:o + 8], "little")
    ndim = b[7]
    return dict(
        magic=bytes(b[0:4]), version=u16(4), dtype=b[6], ndim=ndim,
        dims=tuple(u64(8 + 8 * d) for d in range(ndim)), predictor=b[40],
        order=tuple(b[41:41 + ndim]), eb_mode=b[45],
        eb_user=np.frombuffer(b[48:56], dtype="<f8")[0],
        eb=np.frombuffer(b[56:64], dtype="<f8")[0],
        radius=u32(64), chunk=u32(68), n_unpred=u64(72), nsym=u32(80), sub=u32(84),
        total_words=u64(88), stream_bytes=u64(96),
        out_dtype=b[104] if b[45] == PWREL else b[6], signs=b[105], off_signs=u64(112),
        level_mask=u32(124),
    )


def decompress(stream: bytes, want_codes: bool = False):
    h = parse_header(stream)
    dt = np.float64 if h["out_dtype"] == F64 else np.float32
    shape = h["dims"]
    out = np.empty(shape, dtype=dt)
    codes = np.empty(shape, dtype=np.uint16) if want_codes else None
    buf = np.frombuffer(stream, dtype=np.uint8)
    o = out if out.size else np.zeros(1, dtype=dt)
    rc = lib().szo_decompress(_ptr(buf), buf.size, _ptr(o), out.nbytes, _ptr(codes))
    if rc:
        raise OracleError(rc, "decompress")
    return (out, codes) if want_codes else out


def lossless_pack(stream: bytes, level: int = 1) -> bytes:
    """The pipeline's last, lossless stage on a finished stream (paper
    Section 3; SZ3-Interp ends with zstd, Section 6.2).  zlib stands in for
    zstd: Python's zlib module (RFC 1950 framing around deflate) at the given
    level, the stream taken as opaque bytes."""
    import zlib

    return zlib.compress(bytes(stream), level)


def lossless_unpack(packed: bytes) -> bytes:
    """Inverse of lossless_pack."""
    import zlib

    return zlib.decompress(bytes(packed))
