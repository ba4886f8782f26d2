"""sz_compress_noalloc, the compression entry point for callers that cannot
allocate device memory, called through the C ABI and checked against
sz_compress on the same inputs: several calls in a row on one context, each
smaller than or unlike the one before (the static scratch keeps the previous
call's contents), every stream byte-identical to sz_compress's and the first
small one also to the oracle's; a field too large for the static scratch is
refused before any work is enqueued."""
import numpy as np
import pytest

import paper_2111_02925_amd as szg
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = szg.Context(0)
    yield c
    c.close()


def _bound(x, eb_mode="rel"):
    dt = szg.F64 if x.dtype == np.float64 else szg.F32
    return szg.compress_bound(x.shape, dt)


# (label, field, eb mode, eb, predictor); each call's field is smaller than
# the first one's, and the sequence changes dtype, rank and predictor
SEQUENCE = [
    ("lognormal 150x130x118 f32 cubic", lambda: synth.lognormal_grf((150, 130, 118), seed=61),
     "rel", 1e-3, "cubic"),
    ("lognormal 41x35x29 f32 cubic", lambda: synth.lognormal_grf((41, 35, 29), seed=62),
     "rel", 1e-3, "cubic"),
    ("climate 181x362 f64 linear", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float64),
     "rel", 1e-4, "linear"),
    ("lognormal 64x60x50 f32 adaptive", lambda: synth.lognormal_grf((64, 60, 50), seed=63),
     "rel", 1e-3, "adaptive"),
    # the order choice of two and four dimensions (rows sampled in the kernel)
    ("climate 181x362 f32 adaptive", lambda: synth.climate_2d((181, 362), seed=4, dtype=np.float32),
     "rel", 1e-3, "adaptive"),
    ("random 6x10x8x40 f32 adaptive", lambda: synth.random_field((6, 10, 8, 40), seed=69),
     "rel", 1e-3, "adaptive"),
    ("lognormal 30x20x26 f32 lorenzo abs", lambda: synth.lognormal_grf((30, 20, 26), seed=64),
     "abs", 1e-2, "lorenzo"),
]


def test_noalloc_streams_equal_compress(ctx, orc):
    for i, (label, gen, mode, eb, pred) in enumerate(SEQUENCE):
        print(f"[noalloc] call {i}: {label}", flush=True)
        x = gen()
        xt = torch.from_numpy(x).cuda()
        out = torch.empty(_bound(x), dtype=torch.uint8, device="cuda")
        got = bytes(ctx.compress_noalloc(xt, out, mode, eb, pred).cpu().numpy().tobytes())
        n = x.size
        codes_noalloc = ctx.debug_codes(n).cpu().numpy().copy()
        ref = bytes(ctx.compress(xt, mode, eb, pred).cpu().numpy().tobytes())
        assert got == ref, f"{label}: noalloc stream differs from sz_compress's"
        assert np.array_equal(codes_noalloc, ctx.debug_codes(n).cpu().numpy()), label
        if i == 1:
            omode = orc.REL if mode == "rel" else orc.ABS
            oref = orc.compress(x, omode, eb, orc.CUBIC)
            assert got == oref, f"{label}: noalloc stream differs from the oracle's"
        back = ctx.decompress(torch.frombuffer(bytearray(got), dtype=torch.uint8).cuda())
        err = np.abs(back.cpu().numpy().astype(np.float64) - x.astype(np.float64)).max()
        assert err <= szg.inspect(got)["eb"], label


def test_noalloc_refuses_fields_beyond_its_scratch(ctx):
    # 256^3 f32 needs about 109 MB (reconstruction 4n, codes 2n, lattice n/2):
    # more than the 64 MiB array; nothing is enqueued
    x = torch.zeros((256, 256, 256), dtype=torch.float32, device="cuda")
    out = torch.empty(szg.compress_bound(x.shape, szg.F32), dtype=torch.uint8, device="cuda")
    with pytest.raises(szg.SzError) as e:
        ctx.compress_noalloc(x, out, "abs", 1e-3, "cubic")
    assert e.value.status == szg.ERR_NOMEM
    assert "static buffer" in str(e.value)
    # a field that fits still compresses afterwards, equal to sz_compress
    y = torch.from_numpy(synth.lognormal_grf((33, 47, 21), seed=65)).cuda()
    out2 = torch.empty(szg.compress_bound(y.shape, szg.F32), dtype=torch.uint8, device="cuda")
    got = bytes(ctx.compress_noalloc(y, out2, "rel", 1e-3, "cubic").cpu().numpy().tobytes())
    assert got == bytes(ctx.compress(y, "rel", 1e-3, "cubic").cpu().numpy().tobytes())


def test_noalloc_rejects_pointwise_relative(ctx):
    y = torch.from_numpy(synth.lognormal_grf((16, 16, 16), seed=66)).cuda()
    out = torch.empty(szg.compress_bound(y.shape, szg.F32, eb_mode="pwrel"), dtype=torch.uint8,
                      device="cuda")
    with pytest.raises(szg.SzError) as e:
        ctx.compress_noalloc(y, out, "pwrel", 1e-3, "cubic")
    assert e.value.status == szg.ERR_UNSUPPORTED
