"""The host lossless stage (zlib standing in for the paper's zstd) through
the C ABI, against the oracle's (Python's zlib module) on oracle streams.
Host only: no GPU needed."""
import ctypes
import zlib

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def szg():
    import paper_2111_02925_amd as m

    try:
        m.lib()
    except Exception as e:  # pragma: no cover - the library must build here
        pytest.fail(f"library not loadable: {e}")
    return m


@pytest.fixture(scope="module")
def stream(orc):
    x = synth.lognormal_grf((40, 36, 30), seed=5)
    return orc.compress(x, orc.REL, 1e-3, orc.CUBIC, 32768, 4096)


@pytest.mark.parametrize("level", [0, 1, 6, 9])
def test_pack_matches_oracle(szg, orc, stream, level):
    p = szg.lossless_pack(stream, level)
    assert p == orc.lossless_pack(stream, level)
    assert szg.lossless_unpack(p) == stream
    # the zlib framing: any RFC 1950 decoder restores the stream
    assert zlib.decompress(p) == stream


def test_pack_shrinks_a_stream(szg, orc, stream):
    p = szg.lossless_pack(stream, 6)
    assert len(p) < len(stream)
    # the unpacked stream still decodes to the same reconstruction
    back = orc.decompress(szg.lossless_unpack(p))
    assert back.tobytes() == orc.decompress(stream).tobytes()


def test_empty_and_tiny(szg):
    for d in (b"", b"a", bytes(range(256)) * 3):
        p = szg.lossless_pack(d, 1)
        assert p == zlib.compress(d, 1)
        assert szg.lossless_unpack(p) == d


def _raw_unpack(szg, data, cap):
    L = szg.lib()
    out = ctypes.create_string_buffer(max(cap, 1))
    size = ctypes.c_size_t(0)
    rc = L.sz_lossless_unpack(data, len(data), out, cap, ctypes.byref(size))
    return rc, size.value


def test_errors(szg, stream):
    L = szg.lib()
    p = szg.lossless_pack(stream, 1)
    # output too small to pack: capacity error with the bound as the required size
    out = ctypes.create_string_buffer(16)
    size = ctypes.c_size_t(0)
    rc = L.sz_lossless_pack(stream, len(stream), out, 16, ctypes.byref(size), 1)
    assert rc == -3 and size.value == L.sz_lossless_bound(len(stream))
    # bad level, null output
    assert L.sz_lossless_pack(stream, len(stream), out, 16, ctypes.byref(size), 10) == -1
    assert L.sz_lossless_pack(stream, len(stream), None, 16, ctypes.byref(size), 1) == -1
    # restored bytes that do not fit
    assert _raw_unpack(szg, p, len(stream) - 1)[0] == -3
    assert _raw_unpack(szg, p, len(stream)) == (0, len(stream))
    # truncated input, trailing bytes, damaged data
    assert _raw_unpack(szg, p[:-7], len(stream))[0] == -4
    assert _raw_unpack(szg, p + b"xx", len(stream))[0] == -4
    bad = bytearray(p)
    bad[len(bad) // 2] ^= 0xFF
    bad[len(bad) // 2 + 1] ^= 0x5A
    rc, _ = _raw_unpack(szg, bytes(bad), 2 * len(stream))
    assert rc == -4
