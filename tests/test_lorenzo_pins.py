"""Pins of the oracle's Lorenzo predictor against what fixes it from
outside: the prediction error of the first-order Lorenzo predictor is the
N-th mixed backward difference of the reconstructed field (zero outside the
grid), so on integer-valued fields at eb = 1/2, where every reconstruction is
exact, the codes are R plus that difference, computed here in exact integer
arithmetic; in 1-D it is the previous value.  Also the error bound, round
trips, eb = 0, the unpredictable path, and the rejected forms."""
import numpy as np
import pytest

import synth


def mixed_difference(x):
    """prod_e (1 - shift_e) x with zero extension, in exact integers."""
    d = x.astype(np.int64)
    for e in range(x.ndim):
        pad = np.zeros_like(d)
        idx = [slice(None)] * x.ndim
        src = [slice(None)] * x.ndim
        idx[e] = slice(1, None)
        src[e] = slice(0, -1)
        pad[tuple(idx)] = d[tuple(src)]
        d = d - pad
    return d


@pytest.mark.parametrize("shape", [(1,), (50,), (7, 9), (5, 6, 7), (3, 4, 5, 6), (1, 1, 13),
                                   (9, 1, 4)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_codes_are_the_mixed_difference(orc, shape, dtype):
    rng = np.random.default_rng(sum(shape))
    xi = rng.integers(-40, 40, size=shape)
    x = xi.astype(dtype)
    s, codes, rec = orc.compress(x, orc.ABS, 0.5, orc.LORENZO, want_debug=True)
    assert rec.tobytes() == x.tobytes()
    want = 32768 + mixed_difference(xi)
    assert np.array_equal(codes.astype(np.int64), want)
    assert orc.decompress(s).tobytes() == x.tobytes()


def test_one_dimension_is_previous_value(orc):
    xi = np.cumsum(np.random.default_rng(3).integers(-5, 6, size=1000))
    s, codes, _ = orc.compress(xi.astype(np.float32), orc.ABS, 0.5, orc.LORENZO, want_debug=True)
    prev = np.concatenate([[0], xi[:-1]])
    assert np.array_equal(codes.astype(np.int64) - 32768, xi - prev)


def test_polynomial_of_degree_one_per_dimension_is_exact(orc):
    # f = (1+i)(2+j)(3+k) has a nonzero third mixed difference only at the
    # origin's faces; with eb = 1/2 interior codes are R + 1 (the product of
    # unit steps) and the field comes back exactly
    i, j, k = np.meshgrid(np.arange(6), np.arange(7), np.arange(8), indexing="ij")
    xi = (1 + i) * (2 + j) * (3 + k)
    _, codes, rec = orc.compress(xi.astype(np.float64), orc.ABS, 0.5, orc.LORENZO,
                                 want_debug=True)
    assert np.all(codes[1:, 1:, 1:] == 32768 + 1)
    assert np.array_equal(rec, xi)


@pytest.mark.parametrize("mode,eb", [("rel", 1e-2), ("rel", 1e-4), ("abs", 0.0)])
def test_bound_and_round_trip(orc, mode, eb):
    x = synth.lognormal_grf((21, 18, 23), seed=5)
    m = {"rel": orc.REL, "abs": orc.ABS}[mode]
    s, codes, rec = orc.compress(x, m, eb, orc.LORENZO, want_debug=True)
    back = orc.decompress(s)
    assert back.tobytes() == rec.tobytes()
    ebt = orc.parse_header(s)["eb"]
    assert np.all(np.abs(back.astype(np.float64) - x) <= ebt)
    if eb == 0:
        assert back.tobytes() == x.tobytes()


def test_unpredictable_path(orc):
    x = synth.random_field((30, 40), seed=9)
    s, codes, rec = orc.compress(x, orc.REL, 1e-3, orc.LORENZO, radius=4, want_debug=True)
    assert (codes == 0).sum() > 100
    assert orc.decompress(s).tobytes() == rec.tobytes()


def test_rejected_forms(orc):
    x = synth.random_field((10, 12), seed=2)
    with pytest.raises(Exception):
        orc.compress(x, orc.REL, 1e-3, orc.LORENZO, order=(1, 0))
    s = bytearray(orc.compress(x, orc.REL, 1e-3, orc.LORENZO))
    bad = bytearray(s)
    bad[124] = 1  # a level mask on a Lorenzo stream
    with pytest.raises(Exception):
        orc.decompress(bytes(bad))
    bad = bytearray(s)
    bad[41], bad[42] = 1, 0  # a dimension order
    with pytest.raises(Exception):
        orc.decompress(bytes(bad))
    bad = bytearray(s)
    bad[40] = 4
    with pytest.raises(Exception):
        orc.decompress(bytes(bad))


def test_fibonacci_steps_give_33_bit_codes(orc):
    """Codes longer than 32 bits, fixed from outside.  On the integer field of
    synth.fibonacci_steps_field at eb = 1/2 the codes are R plus the steps
    (the mixed difference of a triple cumulative sum is the summand).  The
    steps' counts are the Fibonacci numbers F1..F34, the last raised, so the
    two-queue Huffman merge joins the running internal node with the next
    leaf at every step (the sum of F1..Fk is F(k+2) - 1, below the leaf after
    next): a caterpillar tree whose leaves, by increasing count, have depths
    33, 33, 32, ..., 2, 1.  Round trip exact."""
    x, steps = synth.fibonacci_steps_field((256, 256, 256), nsym=34, seed=41)
    s, codes, rec = orc.compress(x, orc.ABS, 0.5, orc.LORENZO, want_debug=True)
    assert np.array_equal(codes.astype(np.int64), 32768 + steps)
    hist = np.bincount(codes.ravel(), minlength=65536)
    lens = orc.huffman_lengths(hist)
    used = np.flatnonzero(hist)
    by_count = used[np.lexsort((used, hist[used]))]
    m = len(used)
    want = np.array([m - 1] + [m - k for k in range(1, m)])
    assert np.array_equal(lens[by_count], want)
    h = orc.parse_header(s)
    table = np.frombuffer(s[128:128 + 4 * h["nsym"]], np.uint32)
    assert int((table >> 16).max()) == 33
    assert orc.decompress(s).tobytes() == x.tobytes()
