"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/szg.h declares, and its host-only entry points
(bound, header inspection, argument validation) behave."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2111_02925_amd as szg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "szg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sz_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = szg.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(szg.EXPORTS) == names


def test_compress_bound_covers_streams(orc):
    rng = np.random.default_rng(0)
    for shape, dt in (((33, 20, 7), np.float32), ((1000,), np.float64), ((5, 1, 9, 4), np.float32)):
        x = rng.standard_normal(shape).astype(dt)
        for rel in (1e-1, 1e-6):
            s = orc.compress(x, orc.REL, rel, orc.CUBIC, 32768, 256)
            b = szg.compress_bound(shape, szg.F64 if dt == np.float64 else szg.F32, 32768, 256)
            assert len(s) <= b
    # every value unpredictable (radius 1 keeps only exact predictions)
    x = rng.standard_normal((64, 64)).astype(np.float32)
    s = orc.compress(x, orc.ABS, 0.0, orc.LINEAR, 1, 64)
    assert len(s) <= szg.compress_bound((64, 64), szg.F32, 1, 64)
    assert szg.compress_bound((0, 4), szg.F32) >= 128
    assert szg.compress_bound((4, 4), 7) == 0
    assert szg.compress_bound((4, 4), szg.F32, 0) == 0
    assert szg.compress_bound((4, 4), szg.F32, 32768, 100) == 0  # chunk not a multiple of 64
    assert szg.compress_bound((1 << 20, 1 << 13), szg.F32) == 0  # more than 2^32-1 points


def test_inspect_matches_oracle_header(orc):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((12, 34, 5)).astype(np.float64)
    s = orc.compress(x, orc.REL, 1e-3, orc.CUBIC, 512, 128, (2, 0, 1))
    h = orc.parse_header(s)
    info = szg.inspect(s)
    assert info["dims"] == [12, 34, 5] and info["dtype"] == szg.F64
    assert info["dim_order"] == [2, 0, 1] and info["radius"] == 512 and info["chunk"] == 128
    for k in ("n_unpred", "nsym", "total_words", "stream_bytes", "eb", "eb_mode", "predictor",
              "sub"):
        assert info[k] == h[k], k
    assert info["n"] == x.size and info["sub"] == 4


@pytest.mark.parametrize("chunk,sub,ok", [(4096, 0, True), (4096, 8, True), (4096, 3, False),
                                          (64, 4, False), (64, 2, True), (128, 4, True),
                                          (192, 4, False), (192, 2, True), (65536, 8, True), (1024, 16, False)])
def test_subchunk_option_validation(chunk, sub, ok):
    b = szg.compress_bound((1000,), szg.F32, chunk=chunk, subchunks=sub)
    assert (b > 0) == ok
    if ok:
        # the bound grows with the sub-chunk table: 4 bytes per extra run
        base = szg.compress_bound((1000,), szg.F32, chunk=chunk, subchunks=1)
        S = sub or 4
        nch = (1000 + chunk - 1) // chunk
        assert b - base == ((4 * (S - 1) * nch + 7) & ~7)


def test_inspect_rejects_bad_subchunk_count(orc):
    x = np.linspace(0, 1, 3000).astype(np.float32)
    s = orc.compress(x, orc.REL, 1e-2, chunk=1024, sub=2)
    assert szg.inspect(s)["sub"] == 2
    for v in (0, 3, 16, 1):  # invalid counts, and 1: valid but the layout no longer adds up
        bad = bytearray(s)
        bad[84:88] = int(v).to_bytes(4, "little")
        with pytest.raises(szg.SzError):
            szg.inspect(bytes(bad))


def test_inspect_rejects_bad_headers(orc):
    x = np.linspace(0, 1, 300).astype(np.float32)
    s = orc.compress(x, orc.REL, 1e-2)
    # fields whose corruption the header alone reveals (a changed extent or
    # chunk size that keeps the layout consistent is caught while decoding)
    for pos in (0, 4, 6, 7, 40, 41, 45, 56, 64, 72, 80, 96):
        bad = bytearray(s)
        bad[pos] ^= 0x80
        with pytest.raises(szg.SzError):
            szg.inspect(bytes(bad))
    with pytest.raises(szg.SzError):
        szg.inspect(s[:100])


def test_null_context_is_rejected():
    L = szg.lib()
    size = ctypes.c_size_t(0)
    dims = (ctypes.c_uint64 * 4)(4, 4, 1, 1)
    rc = L.sz_compress(None, None, 0, 2, dims, 0, 0.1, 0, None, None, 0, ctypes.byref(size), None)
    assert rc == szg.ERR_ARG
    assert L.sz_decompress(None, None, 0, None, 0, None) == szg.ERR_ARG
    assert L.sz_last_error(None) == b"no context"


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the C header's sizes and offsets."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    fields = {
        "sz_options": (szg.Options, ["radius", "chunk", "dim_order", "subchunks"]),
        "sz_info": (szg.Info, ["dtype", "dims", "n", "eb", "chunk", "sub", "n_unpred", "stream_bytes"]),
        "sz_request": (szg.Request, ["kind", "d_in", "in_size", "dims", "eb", "options", "d_out",
                                     "out_capacity", "wait_event"]),
        "sz_field": (szg.Field, ["d_in", "dims", "eb", "d_out", "out_size", "status"]),
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "szg.h"', "int main(void) {"]
    for st, (_, names) in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in names:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for st, (cls, names) in fields.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in names:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def test_server_create_fails_cleanly_without_device():
    # an absent device index yields NULL rather than a crash
    assert not szg.lib().sz_server_create(10_000, 1 << 30, 2)
    assert not szg.lib().sz_server_create(0, 1 << 30, 0)
