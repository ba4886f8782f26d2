"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact on everything: quantization codes, stream bytes (hence the
compression ratio), and reconstructed values.  Cases span several chunks and
levels with ragged extents, 1-D to 4-D, every predictor (linear, cubic,
adaptive, Lorenzo) and both dtypes, the three error-bound modes, small radii
(unpredictable path), dimension orders, chunk sizes, special values and
degenerate shapes."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2111_02925_amd as szg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = szg.Context(0)
    yield c
    c.close()


def gpu_roundtrip(ctx, x, mode, eb, pred, radius=32768, chunk=4096, order=None, sub=None):
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    s = ctx.compress(xt, mode, eb, pred, radius=radius, chunk=chunk, dim_order=order,
                     subchunks=sub or 0)
    stream = bytes(s.cpu().numpy().tobytes())
    codes = ctx.debug_codes(x.size).cpu().numpy().view(np.uint16).reshape(x.shape)
    back = ctx.decompress(s).cpu().numpy()
    return stream, codes, back


def check_case(ctx, orc, x, mode, eb, pred, radius=32768, chunk=4096, order=None, label="",
               sub=None):
    print(f"[case] {label} shape={x.shape} dtype={x.dtype} mode={mode} eb={eb} pred={pred} "
          f"R={radius} C={chunk} S={sub} order={order}", flush=True)
    omode = {"abs": orc.ABS, "rel": orc.REL, "pwrel": orc.PWREL}[mode]
    ref, rcodes, rrec = orc.compress(x, omode, eb, pred, radius, chunk, order, want_debug=True,
                                     sub=sub)
    stream, codes, back = gpu_roundtrip(ctx, x, mode, eb, pred, radius, chunk, order, sub)
    assert np.array_equal(codes, rcodes), f"codes differ at {np.argwhere(codes != rcodes)[:5]}"
    assert len(stream) == len(ref), (len(stream), len(ref))
    if stream != ref:
        diff = np.flatnonzero(np.frombuffer(stream, np.uint8) != np.frombuffer(ref, np.uint8))
        raise AssertionError(f"stream bytes differ at {diff[:10]}")
    assert back.tobytes() == rrec.tobytes(), "GPU decompress != oracle reconstruction"
    # the GPU decoder also accepts the oracle's stream
    st = torch.frombuffer(bytearray(ref), dtype=torch.uint8).cuda()
    assert ctx.decompress(st).cpu().numpy().tobytes() == rrec.tobytes()


def lognormal(shape, seed):
    return synth.lognormal_grf(shape, seed=seed)


CASES = [
    # label, generator, mode, eb, pred, radius, chunk, order
    ("cfg1-64^3-linear-abs", lambda: synth.sinusoid_field()[0], "abs", None, 0, 32768, 4096, None),
    ("lognormal-ragged-cubic-1e-2", lambda: lognormal((97, 80, 71), 21), "rel", 1e-2, 1, 32768, 4096, None),
    ("lognormal-ragged-cubic-1e-3", lambda: lognormal((97, 80, 71), 22), "rel", 1e-3, 1, 32768, 4096, None),
    ("lognormal-ragged-cubic-1e-4", lambda: lognormal((97, 80, 71), 23), "rel", 1e-4, 1, 32768, 1024, None),
    ("lognormal-linear-order", lambda: lognormal((33, 70, 45), 24), "rel", 1e-3, 0, 32768, 256, (2, 0, 1)),
    ("climate-f64-cubic", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float64), "rel", 1e-4, 1, 32768, 4096, None),
    ("climate-f32-linear", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float32), "rel", 1e-4, 0, 32768, 4096, None),
    ("climate-f64-cubic-R512", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float64), "rel", 1e-4, 1, 512, 4096, None),
    ("climate-f32-linear-R512", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float32), "rel", 1e-4, 0, 512, 64, None),
    ("1d-long", lambda: np.cumsum(np.random.default_rng(5).standard_normal(100003)).astype(np.float32), "rel", 1e-3, 1, 32768, 65536, None),
    ("4d", lambda: synth.random_field((9, 12, 7, 10), seed=6), "rel", 1e-3, 1, 32768, 512, (3, 1, 0, 2)),
    ("tiny-radius", lambda: synth.random_field((40, 40), seed=7), "rel", 1e-3, 0, 4, 64, None),
    # wide code histograms: thousands of coded symbols (the codebook's global
    # path), codes far from the radius (the histogram's far path), and many
    # unpredictable values
    ("wide-hist-1e-6", lambda: synth.random_field((64, 64, 32), seed=17), "rel", 1e-6, 1, 32768, 4096, None),
    ("wide-hist-1e-5", lambda: lognormal((64, 64, 64), 3), "rel", 1e-5, 1, 32768, 4096, None),
    # more than 65536 chunks: the chunk-size scans take the multi-launch path
    ("many-chunks", lambda: lognormal((200, 150, 141), 40), "rel", 1e-3, 1, 32768, 64, None),
]


# The stride-1 level of 3-D fields with an even last extent runs as row strips
# (one to four waves of 128 columns, one or more column windows, runs of rows
# and groups of planes with ragged ends).
FINE_CASES = [
    ("fine-2win-ragged", lambda: lognormal((20, 37, 600), 31), "rel", 1e-3, 1, 32768, 4096, None),
    ("fine-3win", lambda: lognormal((9, 130, 1030), 32), "rel", 1e-4, 1, 32768, 4096, None),
    ("fine-3wave-f64-linear", lambda: synth.random_field((11, 50, 260), seed=33, dtype=np.float64), "rel", 1e-4, 0, 32768, 4096, None),
    ("fine-2wave-f64-cubic", lambda: synth.random_field((13, 41, 200), seed=34, dtype=np.float64), "rel", 1e-3, 1, 32768, 4096, None),
    ("fine-3planes", lambda: lognormal((3, 16, 200), 35), "rel", 1e-2, 1, 32768, 4096, None),
    ("fine-2planes", lambda: lognormal((2, 300, 256), 36), "rel", 1e-3, 1, 32768, 4096, None),
    ("fine-unpred", lambda: synth.random_field((16, 40, 300), seed=37), "rel", 1e-6, 1, 32768, 4096, None),
    ("fine-unpred-R2", lambda: synth.random_field((10, 33, 140), seed=38), "rel", 1e-3, 0, 2, 1024, None),
    ("fine-4col", lambda: lognormal((12, 10, 4), 39), "rel", 1e-3, 1, 32768, 256, None),
    # an order that swaps the outer dimensions keeps the contiguous pass last
    # but not the planes outermost: the fixed-pitch kernel takes it
    ("fine-swapped-order", lambda: lognormal((20, 37, 600), 31), "rel", 1e-3, 1, 32768, 4096, (1, 0, 2)),
]


def mixed_signs(shape, seed, dtype=np.float32):
    """Both signs, exact zeros and six decades of magnitude."""
    x = synth.random_field(shape, seed=seed, dtype=dtype)
    x = (np.sign(x - np.median(x)) * np.exp(3 * x)).astype(dtype)
    x.flat[::53] = 0
    return x


def specials(shape, seed):
    x = lognormal(shape, seed)
    x.flat[5] = np.inf
    x.flat[77] = -np.inf
    x.flat[123] = np.nan
    x.flat[200] = np.float32(1e-40)
    x.flat[201] = -0.0
    x.flat[300] = -x.flat[300]
    return x


# The point-wise relative mode: the logarithmic preprocessor, the double log
# field through the same kernels (the strip kernel's f64 variant where the
# last extent is even), and the inverse transform with the sign section.
PW_CASES = [
    ("pw-lognormal-cubic-1e-3", lambda: lognormal((40, 36, 46), 51), "pwrel", 1e-3, 1, 32768, 4096, None),
    ("pw-lognormal-linear-1e-2", lambda: lognormal((33, 27, 31), 52), "pwrel", 1e-2, 0, 32768, 4096, None),
    ("pw-mixed-signs-zeros", lambda: mixed_signs((30, 28, 26), 53), "pwrel", 1e-3, 1, 32768, 4096, None),
    ("pw-f64-2d", lambda: synth.climate_2d((91, 77), seed=54, dtype=np.float64), "pwrel", 1e-6, 1, 32768, 4096, None),
    ("pw-specials", lambda: specials((20, 22, 24), 55), "pwrel", 1e-2, 1, 32768, 4096, None),
    ("pw-R512-unpred", lambda: mixed_signs((24, 20, 18), 56), "pwrel", 1e-4, 1, 512, 1024, None),
]


def step_1d(n, at):
    x = np.cumsum(np.random.default_rng(at).standard_normal(n) * 0.01).astype(np.float32)
    x[at:] += 5.0
    return x


# Adaptive interpolation: each level's predictor chosen from the two cost
# sums on the GPU, the level mask in the header, and the per-level predictor
# in every kernel (fused levels, the strip kernel, the decoder side).
ADAPT_CASES = [
    ("ad-lognormal-ragged", lambda: lognormal((97, 80, 71), 61), "rel", 1e-3, 2, 32768, 4096, None),
    ("ad-climate-f32", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float32), "rel", 1e-3, 2, 32768, 4096, None),
    ("ad-climate-f64-1e-5", lambda: synth.climate_2d((181, 362), seed=62, dtype=np.float64), "rel", 1e-5, 2, 32768, 4096, None),
    ("ad-step-1d", lambda: step_1d(70001, 23456), "abs", 1e-3, 2, 32768, 4096, None),
    ("ad-4d-order", lambda: synth.random_field((9, 12, 7, 10), seed=63), "rel", 1e-3, 2, 32768, 512, (3, 1, 0, 2)),
    ("ad-fine-3win", lambda: lognormal((9, 130, 1030), 64), "rel", 1e-4, 2, 32768, 4096, None),
    ("ad-eb0", lambda: synth.random_field((20, 30, 18), seed=65), "abs", 0.0, 2, 32768, 4096, None),
    ("ad-R2-unpred", lambda: synth.random_field((10, 33, 140), seed=66), "rel", 1e-3, 2, 2, 1024, None),
    ("ad-pw-mixed-signs", lambda: mixed_signs((30, 28, 26), 67), "pwrel", 1e-3, 2, 32768, 4096, None),
    ("ad-specials", lambda: specials((20, 22, 24), 68), "rel", 1e-2, 2, 32768, 4096, None),
    # the default order chosen among 24 (four dimensions, on the host) and
    # among six in f64 (on the device); the oracle picks (1, 0, 2, 3) and
    # (2, 1, 0) here
    ("ad-4d-default", lambda: synth.random_field((6, 10, 8, 40), seed=69), "rel", 1e-3, 2, 32768, 1024, None),
    ("ad-f64-order", lambda: synth.random_field((21, 40, 70), seed=70, dtype=np.float64), "rel", 1e-3, 2, 32768, 1024, None),
]


# The Lorenzo predictor: wavefronts of blocks (several block diagonals and
# ragged blocks in every dimension), 1-D to 4-D, both dtypes, eb = 0, the
# unpredictable path, special values and the point-wise relative mode.
LOR_CASES = [
    ("lor-lognormal-ragged", lambda: lognormal((97, 80, 71), 71), "rel", 1e-3, 3, 32768, 4096, None),
    ("lor-f64-3d", lambda: synth.random_field((33, 40, 37), seed=72, dtype=np.float64), "rel", 1e-4, 3, 32768, 4096, None),
    ("lor-climate-f32", lambda: synth.climate_2d((181, 362), seed=3, dtype=np.float32), "rel", 1e-4, 3, 32768, 4096, None),
    ("lor-climate-f64", lambda: synth.climate_2d((181, 362), seed=73, dtype=np.float64), "rel", 1e-3, 3, 32768, 4096, None),
    ("lor-1d", lambda: np.cumsum(np.random.default_rng(74).standard_normal(20003)).astype(np.float32), "rel", 1e-3, 3, 32768, 4096, None),
    ("lor-4d", lambda: synth.random_field((9, 12, 7, 10), seed=75), "rel", 1e-3, 3, 32768, 512, None),
    ("lor-4d-f64", lambda: synth.random_field((5, 20, 9, 18), seed=76, dtype=np.float64), "rel", 1e-3, 3, 32768, 512, None),
    ("lor-eb0", lambda: synth.random_field((20, 30, 18), seed=77), "abs", 0.0, 3, 32768, 4096, None),
    ("lor-R4-unpred", lambda: synth.random_field((30, 33, 40), seed=78), "rel", 1e-3, 3, 4, 1024, None),
    ("lor-specials", lambda: specials((20, 22, 24), 79), "rel", 1e-2, 3, 32768, 4096, None),
    ("lor-pwrel", lambda: mixed_signs((30, 28, 26), 80), "pwrel", 1e-3, 3, 32768, 4096, None),
]


@pytest.mark.parametrize("case", CASES + FINE_CASES + PW_CASES + ADAPT_CASES + LOR_CASES,
                         ids=[c[0] for c in CASES + FINE_CASES + PW_CASES + ADAPT_CASES + LOR_CASES])
def test_parity(ctx, orc, case):
    label, gen, mode, eb, pred, radius, chunk, order = case
    x = gen()
    if eb is None:
        eb = synth.sinusoid_field()[1]
    check_case(ctx, orc, x, mode, eb, pred, radius, chunk, order, label)


# Sub-chunk splits: S lanes decode one chunk from the stored run offsets.
# Ragged tails leave the last chunk's later runs short or empty; small radii
# put many unpredictable values in each run (their per-run lists and scatter).
SUB_CASES = [
    # label, generator, eb, pred, radius, chunk, sub
    ("S1", lambda: lognormal((97, 80, 71), 41), 1e-3, 1, 32768, 4096, 1),
    ("S2", lambda: lognormal((97, 80, 71), 41), 1e-3, 1, 32768, 4096, 2),
    ("S8", lambda: lognormal((97, 80, 71), 41), 1e-3, 1, 32768, 4096, 8),
    ("S8-1d-tail", lambda: np.cumsum(np.random.default_rng(9).standard_normal(3 * 2048 + 300)).astype(np.float32), 1e-3, 0, 32768, 2048, 8),
    ("S2-C64", lambda: synth.random_field((45, 37), seed=12), 1e-3, 1, 32768, 64, 2),
    ("S8-R2-unpred", lambda: synth.random_field((130, 70), seed=13), 1e-3, 0, 2, 1024, 8),
    ("S4-R3-f64-unpred", lambda: synth.climate_2d((91, 77), seed=14, dtype=np.float64), 1e-5, 1, 3, 512, 4),
    ("S4-C65536", lambda: lognormal((67, 61, 59), 15), 1e-4, 1, 32768, 65536, 4),
]


@pytest.mark.parametrize("case", SUB_CASES, ids=[c[0] for c in SUB_CASES])
def test_parity_subchunks(ctx, orc, case):
    label, gen, eb, pred, radius, chunk, sub = case
    check_case(ctx, orc, gen(), "rel", eb, pred, radius, chunk, None, "sub:" + label, sub)


@pytest.fixture(scope="module")
def ctx_passes():
    """A context that runs one kernel per (level, dimension) pass instead of
    one fused kernel per level (the path taken for four dimensions)."""
    import paper_2111_02925_amd as szg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    os.environ["SZG_FUSED_LEVELS"] = "0"
    try:
        c = szg.Context(0)
    finally:
        del os.environ["SZG_FUSED_LEVELS"]
    yield c
    c.close()


PASS_CASES = [CASES[i] for i in (0, 2, 4, 6, 9)] + [ADAPT_CASES[i] for i in (0, 3)]


@pytest.mark.parametrize("case", PASS_CASES, ids=[c[0] for c in PASS_CASES])
def test_parity_pass_kernels(ctx_passes, orc, case):
    label, gen, mode, eb, pred, radius, chunk, order = case
    x = gen()
    if eb is None:
        eb = synth.sinusoid_field()[1]
    check_case(ctx_passes, orc, x, mode, eb, pred, radius, chunk, order, "passes:" + label)


def test_parity_special_values(ctx, orc):
    x = synth.random_field((30, 41), seed=8)
    x[3, 7] = np.nan
    x[5, 5] = np.inf
    x[6, 6] = -np.inf
    x[7, 0] = np.float32(1e-42)
    x[2, 2] = -0.0
    x[20, 30] = 3e38
    check_case(ctx, orc, x, "rel", 1e-3, 1, label="special-values")


@pytest.mark.parametrize("shape", [(1,), (2,), (3,), (1, 1, 1), (1, 1, 5), (2, 3, 1, 2), (65,), (64, 1)])
def test_parity_tiny_shapes(ctx, orc, shape):
    x = (np.arange(int(np.prod(shape)), dtype=np.float32) * 0.37 + 1).reshape(shape)
    check_case(ctx, orc, x, "rel", 1e-2, 1, chunk=64, label=f"tiny{shape}")
    check_case(ctx, orc, x, "rel", 1e-2, 3, chunk=64, label=f"tiny-lorenzo{shape}")


def test_lorenzo_rejects_dim_order(ctx):
    import paper_2111_02925_amd as szg

    xt = torch.from_numpy(synth.random_field((10, 12), seed=3)).cuda()
    with pytest.raises(szg.SzError):
        ctx.compress(xt, "rel", 1e-3, "lorenzo", dim_order=(1, 0))


def test_parity_degenerate_bounds(ctx, orc):
    const = np.full((17, 9, 5), 2.5, dtype=np.float32)
    check_case(ctx, orc, const, "rel", 1e-3, 1, label="constant (eb = 0 via range)")
    x = synth.random_field((20, 20), seed=9, dtype=np.float64)
    check_case(ctx, orc, x, "abs", 0.0, 0, label="abs eb = 0")
    allnan = np.full((8, 8), np.nan, dtype=np.float32)
    check_case(ctx, orc, allnan, "rel", 1e-3, 1, label="no finite value")


def test_empty_field(ctx, orc):
    x = np.zeros((4, 0, 3), dtype=np.float32)
    ref = orc.compress(x, orc.REL, 1e-3, orc.CUBIC)
    xt = torch.zeros((4, 0, 3), dtype=torch.float32, device="cuda")
    s = ctx.compress(xt, "rel", 1e-3, "cubic")
    assert bytes(s.cpu().numpy().tobytes()) == ref
    back = ctx.decompress(s)
    assert tuple(back.shape) == (4, 0, 3)


def test_capacity_and_corruption(ctx, orc):
    import paper_2111_02925_amd as szg

    x = synth.random_field((50, 60), seed=10)
    xt = torch.from_numpy(x).cuda()
    s = ctx.compress(xt, "rel", 1e-3, "cubic")
    small = torch.zeros(len(s) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(szg.SzError) as ei:
        ctx.compress(xt, "rel", 1e-3, "cubic", out=small)
    assert ei.value.status == szg.ERR_CAPACITY and ei.value.required == len(s)
    good = ctx.decompress(s).cpu().numpy()
    h = szg.inspect(s.cpu())
    K = h["nsym"]
    sym_pos = 128 + 2                      # a symbol-table length byte
    chunk_pos = 128 + ((4 * K + 7) & ~7)   # first chunk's word count
    assert h["sub"] == 4
    sub_pos = chunk_pos + 8                # the single chunk's run offsets
    for pos in (6, 45, sym_pos, chunk_pos, sub_pos, sub_pos + 4, sub_pos + 8, sub_pos + 9):
        bad = s.clone()
        bad[pos] ^= 0x5A
        with pytest.raises(szg.SzError) as ei:
            ctx.decompress(bad)
        assert ei.value.status == szg.ERR_CORRUPT
    # flipped bitstream bits: detected, or a different (still finite-time) result
    rng = np.random.default_rng(0)
    nb = 4 * h["total_words"]
    for pos in rng.integers(len(s) - nb, len(s), size=8):
        bad = s.clone()
        bad[int(pos)] ^= 0x08
        try:
            out = ctx.decompress(bad).cpu().numpy()
        except szg.SzError as e:
            assert e.status == szg.ERR_CORRUPT
            continue
        assert out.tobytes() != good.tobytes()
    with pytest.raises(szg.SzError):
        ctx.decompress(s[:-4])


def test_lossless_stage_roundtrip(ctx, orc):
    """GPU stream -> host lossless stage -> back -> GPU decompress: the same
    bytes and the oracle's reconstruction."""
    import paper_2111_02925_amd as szg

    x = lognormal((48, 40, 64), 42)
    ref = orc.compress(x, orc.REL, 1e-3, orc.CUBIC, 32768, 4096)
    s = ctx.compress(torch.from_numpy(x).cuda(), "rel", 1e-3, "cubic")
    host = bytes(s.cpu().numpy().tobytes())
    assert host == ref
    packed = szg.lossless_pack(host, 1)
    assert packed == orc.lossless_pack(ref, 1)
    back = szg.lossless_unpack(packed)
    st = torch.frombuffer(bytearray(back), dtype=torch.uint8).cuda()
    assert ctx.decompress(st).cpu().numpy().tobytes() == orc.decompress(ref).tobytes()
