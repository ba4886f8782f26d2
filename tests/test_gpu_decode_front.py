"""The decompressor's front (decoding tables, the chunk table's scans and the
stream's prefetch in one launch) on its three routes, each checked byte for
byte against the oracle's reconstruction:

- a fresh context (no chunk buffers yet): the host launches the front once it
  has parsed the header;
- a context whose buffers hold the stream's chunks: the front starts from the
  header in device memory before the host has it;
- a context whose buffers are too small: that launch does nothing, the
  buffers grow and the host launches the front again.

The chunk table is scanned in slices of 2048 entries by at most 256 blocks:
one case has more slices than blocks (each block takes several, the carries
span all of them).  Corrupted headers decoded by a warm context are rejected
and leave it able to decode the next stream."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def szg():
    import paper_2111_02925_amd as m

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return m


def oracle_case(orc, shape, dtype, chunk, seed):
    x = synth.random_field(shape, seed=seed, dtype=dtype)
    ref = orc.compress(x, orc.REL, 1e-3, orc.CUBIC, 32768, chunk)
    rec = orc.decompress(ref)
    return x, ref, np.ascontiguousarray(rec)


def decode(ctx, stream_bytes, like):
    st = torch.frombuffer(bytearray(stream_bytes), dtype=torch.uint8).cuda()
    out = torch.empty(like.shape, dtype=torch.float64 if like.dtype == np.float64 else torch.float32,
                      device="cuda")
    ctx.decompress(st, out=out)
    return out.cpu().numpy()


def test_front_routes(szg, orc):
    cases = [
        ((40, 50, 60), np.float32, 1024, 1),     # 118 chunks
        ((96, 100, 130), np.float32, 512, 2),     # 2438 chunks: two slices
        ((33, 47, 21), np.float64, 4096, 3),      # one ragged chunk
    ]
    data = [oracle_case(orc, *c) for c in cases]
    ctx = szg.Context(0)
    try:
        # fresh, too small (grows), then warm for every case, in both orders
        for k in (0, 1, 0, 2, 1, 2, 0):
            x, ref, rec = data[k]
            print(f"[front] case {k} shape={x.shape} dtype={x.dtype}", flush=True)
            assert decode(ctx, ref, rec).tobytes() == rec.tobytes(), f"case {k}"
    finally:
        ctx.close()


def test_front_more_slices_than_blocks(szg, orc):
    # 512 x 512 x 520 points in chunks of 256: 532 480 chunks, 260 slices
    x = synth.lognormal_grf((520, 512, 512), seed=21)
    ref = orc.compress(x, orc.REL, 1e-3, orc.CUBIC, 32768, 256)
    rec = np.ascontiguousarray(orc.decompress(ref))
    print(f"[front] {len(ref)} stream bytes, {(x.size + 255) // 256} chunks", flush=True)
    ctx = szg.Context(0)
    try:
        for _ in range(2):  # host route, then the early one
            assert decode(ctx, ref, rec).tobytes() == rec.tobytes()
    finally:
        ctx.close()


def test_front_corrupt_headers_warm(szg, orc):
    x, ref, rec = oracle_case(orc, (96, 100, 130), np.float32, 512, 2)
    ctx = szg.Context(0)
    try:
        assert decode(ctx, ref, rec).tobytes() == rec.tobytes()  # warm: buffers for 2438 chunks
        small_x, small_ref, small_rec = oracle_case(orc, (40, 50, 60), np.float32, 1024, 1)
        # header fields the device reads: dims, radius, chunk, unpredictable
        # count, coded symbols, bit-stream words
        for pos in (8, 16, 24, 64, 68, 72, 80, 88):
            bad = bytearray(small_ref)
            bad[pos] ^= 0x21
            print(f"[front] corrupt byte {pos}", flush=True)
            with pytest.raises(szg.SzError) as ei:
                decode(ctx, bytes(bad), small_rec)
            assert ei.value.status == szg.ERR_CORRUPT
            assert decode(ctx, small_ref, small_rec).tobytes() == small_rec.tobytes()
    finally:
        ctx.close()
