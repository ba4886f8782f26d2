"""Pins for the CPU oracle: checks against what the paper and mathematics fix,
not against the oracle's own formulas.

* hand-worked examples (tests/golden/) -- traversal, stencils, quantizer,
  Huffman tie rule, canonical codes, bit packing;
* the error bound |x - x'| <= eb, checked exactly with rationals near the
  bound (Section 1 and Section 3.2 "Quantizer");
* visit-once and dependency order of the multilevel traversal;
* closed-form code arrays on constant and linear fields, and exactness of the
  cubic/quadratic stencils on polynomials (Section 6.2: constant-coefficient
  interpolation);
* Huffman optimality by brute force, Kraft equality, entropy bounds
  (Section 3.2 "Encoder");
* codec, pipeline and format round trips; corruption is detected.
"""
from fractions import Fraction
import itertools
import math

import numpy as np
import pytest

from tests import golden_io


# ----------------------------------------------------------------- helpers

def exact_within(x, r, eb):
    """max |x - r| <= eb, exactly (rationals for the points near the bound)."""
    x = np.asarray(x).ravel()
    r = np.asarray(r).ravel()
    fin = np.isfinite(x)
    with np.errstate(invalid="ignore"):
        d = np.abs(x.astype(np.float64) - r.astype(np.float64))
    assert np.array_equal(np.isnan(x), np.isnan(r))
    # non-finite inputs must come back bit-identical (stored verbatim)
    nf = ~fin
    assert x[nf].tobytes() == r[nf].tobytes()
    near = fin & ~(d < eb * (1 - 1e-9))
    for i in np.flatnonzero(near):
        assert abs(Fraction(float(x[i])) - Fraction(float(r[i]))) <= Fraction(float(eb)), i
    return float(d[fin].max() / eb) if fin.any() and eb > 0 else 0.0


def v2(v):
    return (v & -v).bit_length() - 1


def pass_of(p, order):
    """Closed form of the pass holding point p (O4): level stride s = 2^m with
    m the smallest 2-adic valuation among nonzero coordinates; dimension = the
    last one in the visiting order whose coordinate is an odd multiple of s."""
    m = min(v2(c) for c in p if c)
    s = 1 << m
    d = [e for e in order if p[e] % (2 * s) == s][-1]
    return s, d


def run_golden(orc, name, dtype):
    g = golden_io.load(name)
    shape = tuple(golden_io.ints(g["shape"]))
    order = golden_io.ints(g["order"])
    pred = orc.CUBIC if g["predictor"][0] == "cubic" else orc.LINEAR
    x = np.array(golden_io.floats(g["x"]), dtype=dtype).reshape(shape)
    codes, recon = orc.predict_quantize(x, float(g["eb"][0]), pred,
                                        int(g["radius"][0]), order=order)
    exp_codes = np.array(golden_io.ints(g["codes"]), dtype=np.uint16).reshape(shape)
    exp_recon = np.array(golden_io.floats(g["recon"]), dtype=dtype).reshape(shape)
    assert np.array_equal(codes, exp_codes), (codes.ravel(), exp_codes.ravel())
    assert np.array_equal(recon, exp_recon), (recon.ravel(), exp_recon.ravel())
    # the decompressor's mirror rebuilds the same values from codes + verbatim values
    unpred = x.ravel()[codes.ravel() == 0]
    back = orc.reconstruct(codes, unpred, float(g["eb"][0]), pred, int(g["radius"][0]), order)
    assert np.array_equal(back, exp_recon)


# ----------------------------------------------------------------- goldens

GOLDEN_INTERP = [
    "interp_1d_linear_n9.txt",
    "interp_1d_linear_n9_r4.txt",
    "interp_1d_linear_n8.txt",
    "interp_2d_linear_3x5_order01.txt",
    "interp_2d_linear_3x5_order10.txt",
    "interp_1d_cubic_n9.txt",
]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("name", GOLDEN_INTERP)
def test_golden_interp(orc, name, dtype):
    run_golden(orc, name, dtype)


def test_golden_huffman(orc):
    g = golden_io.load("huffman_ties.txt")
    hist = np.array(golden_io.ints(g["hist"]), dtype=np.uint64)
    lens = orc.huffman_lengths(hist)
    assert lens.tolist() == golden_io.ints(g["lens"])
    cw = orc.canonical_codes(lens)
    assert cw.tolist() == golden_io.ints(g["codewords"])
    syms = np.array(golden_io.ints(g["symbols"]), dtype=np.uint16)
    words, cwords = orc.pack(syms, lens, cw, 4)
    assert words.tolist() == golden_io.ints(g["chunk4_words"])
    assert cwords.tolist() == golden_io.ints(g["chunk4_chunk_words"])
    words2, cw2 = orc.pack(np.concatenate([syms, syms]), lens, cw, 32)
    assert words2.tolist() == golden_io.ints(g["double_chunk32_words"])
    assert cw2.tolist() == [2]
    assert orc.unpack(words, cwords, syms.size, 4, lens).tolist() == syms.tolist()


# ------------------------------------------------------------ error bound

BOUND_CASES = [
    ((37,), np.float32, 0, 1e-2, 32768, None),
    ((16, 23), np.float64, 1, 1e-3, 32768, (1, 0)),
    ((9, 17, 12), np.float32, 1, 1e-4, 32768, (2, 0, 1)),
    ((5, 6, 7, 8), np.float32, 0, 1e-3, 32768, (3, 1, 0, 2)),
    ((33, 40, 31), np.float64, 1, 1e-5, 512, None),
    ((64, 64), np.float32, 1, 1e-2, 8, None),
]


@pytest.mark.parametrize("shape,dtype,pred,rel,radius,order", BOUND_CASES)
def test_error_bound_and_roundtrip(orc, shape, dtype, pred, rel, radius, order):
    rng = np.random.default_rng(abs(hash((shape, rel))) % 2**32)
    x = np.cumsum(rng.standard_normal(shape), axis=-1)
    x += rng.standard_normal(shape) * 0.01
    x = x.astype(dtype)
    if x.size > 10:
        x.ravel()[rng.choice(x.size, 3, replace=False)] *= 1000.0  # spikes
    stream, codes, recon = orc.compress(x, orc.REL, rel, pred, radius, 64, order, want_debug=True)
    eb = orc.parse_header(stream)["eb"]
    r = exact_within(x, recon, eb)
    assert r <= 1.0
    # unpredictable points are stored verbatim
    assert np.array_equal(recon[codes == 0].view(np.uint8), x[codes == 0].view(np.uint8))
    back, bcodes = orc.decompress(stream, want_codes=True)
    assert np.array_equal(back.view(np.uint8), recon.view(np.uint8))  # bitwise (P8)
    assert np.array_equal(bcodes, codes)


def test_error_bound_special_values(orc):
    x = np.linspace(-3, 3, 1000).astype(np.float32).reshape(10, 100)
    x[3, 7] = np.nan
    x[5, 50] = np.inf
    x[6, 51] = -np.inf
    x[7, 0] = np.float32(1e-42)  # subnormal
    x[2, 2] = -0.0
    stream, codes, recon = orc.compress(x, orc.REL, 1e-3, orc.CUBIC, want_debug=True)
    eb = orc.parse_header(stream)["eb"]
    # the range uses finite values only
    assert eb == np.float32(1e-3 * 6.0)
    assert codes[3, 7] == 0 and codes[5, 50] == 0 and codes[6, 51] == 0
    exact_within(x, recon, eb)
    back = orc.decompress(stream)
    assert np.array_equal(back.view(np.uint32), recon.view(np.uint32))


# ------------------------------------------------------------- traversal

TRAV_SHAPES = [(1,), (2,), (3,), (17,), (1, 1), (2, 9), (5, 1, 3), (16, 16, 16),
               (9, 13, 6), (33, 2, 5), (3, 4, 5, 6), (1, 7, 1, 9)]


@pytest.mark.parametrize("shape", TRAV_SHAPES)
@pytest.mark.parametrize("pred", [0, 1])
def test_traversal_visits_once_in_dependency_order(orc, shape, pred):
    orders = [None] + ([tuple(reversed(range(len(shape))))] if len(shape) > 1 else [])
    for order in orders:
        visits, early = orc.check_traversal(shape, pred, order)
        assert early == 0
        assert np.all(visits == 1)


# ------------------------------------------- constant / polynomial fields

def exception_points(shape, order):
    """Points whose stencil holds a single known neighbour: on the pass of dim
    d at level stride s = 2^(L_d - 1) (L_d = ceil(log2 n_d)), coordinate
    p_d = s, with s < n_d <= 2s.  Derived from the level structure, not from
    the oracle."""
    pts = set()
    nd = len(shape)
    order = list(order)
    for j, d in enumerate(order):
        n = shape[d]
        if n < 2:
            continue
        s = 1 << (math.ceil(math.log2(n)) - 1)
        ranges = []
        for e in range(nd):
            if e == d:
                ranges.append([s])
            elif order.index(e) < j:
                ranges.append(range(0, shape[e], s))
            else:
                ranges.append(range(0, shape[e], 2 * s))
        for p in itertools.product(*ranges):
            pts.add((p, d, s))
    return pts


@pytest.mark.parametrize("shape,order", [((13,), (0,)), ((6, 11), (0, 1)), ((6, 11), (1, 0)),
                                         ((5, 9, 4), (0, 1, 2)), ((5, 9, 4), (2, 0, 1)),
                                         ((3, 5, 2, 6), (0, 1, 2, 3))])
@pytest.mark.parametrize("pred", [0, 1])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_linear_field_closed_form(orc, shape, order, pred, dtype):
    """x = a + sum_d b_d p_d with integers, eb = 1/2: every prediction with two
    neighbours (interpolation or extrapolation) is exact, so the code array
    is R everywhere except the origin (R + a) and the single-neighbour points
    (R + b_d * s)."""
    R = 32768
    a = 7
    b = [3, -2, 5, 1][: len(shape)]
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    x = (a + sum(bd * g for bd, g in zip(b, grids))).astype(dtype)
    codes, recon = orc.predict_quantize(x, 0.5, pred, R, order)
    exp = np.full(shape, R, dtype=np.int64)
    exp[(0,) * len(shape)] = R + a
    for p, d, s in exception_points(shape, order):
        exp[p] = R + b[d] * s
    assert np.array_equal(codes.astype(np.int64), exp)
    assert np.array_equal(recon, x)


@pytest.mark.parametrize("pred", [0, 1])
def test_constant_field(orc, pred):
    x = np.full((7, 10, 5), 3.25, dtype=np.float32)
    codes, recon = orc.predict_quantize(x, 0.125, pred)
    assert codes[0, 0, 0] == 32768 + 13  # 3.25 / 0.25
    assert np.all(codes.ravel()[1:] == 32768)
    assert np.array_equal(recon, x)


def stencil_case(i, s, n):
    has_a, has_c, has_e = i >= 3 * s, i + s < n, i + 3 * s < n
    if not has_c:
        return "edge"
    if has_a and has_e:
        return "four"
    if has_a or has_e:
        return "quad"
    return "two"


@pytest.mark.parametrize("shape,order", [((23,), (0,)), ((11, 14), (0, 1)),
                                         ((9, 7, 12), (1, 2, 0))])
def test_cubic_polynomial_exactness(orc, shape, order):
    """Cubic interpolation reproduces cubics with the 4-point rule and
    quadratics with the 3-point boundary rules.  With integer data and a tiny
    dyadic eb every operation is exact in f64, so a code is R exactly where
    the stencil is exact for the polynomial."""
    R = 32768
    eb = 2.0 ** -30
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    cub = sum((g - 3) ** 3 - 2 * g * g for g in grids) + 5.0
    quad = sum(2 * g * g - 3 * g for g in grids) + 1.0
    for field, exact_cases in ((cub, {"four"}), (quad, {"four", "quad"})):
        codes, recon = orc.predict_quantize(field, eb, orc.CUBIC, R, order)
        assert np.array_equal(recon, field)
        for p in itertools.product(*[range(n) for n in shape]):
            if not any(p):
                continue
            s, d = pass_of(p, order)
            if stencil_case(p[d], s, shape[d]) in exact_cases:
                assert codes[p] == R, (p, s, d)


# ----------------------------------------------------------------- Huffman

def brute_min_cost(h):
    """Minimum sum h_i * len_i over all complete prefix codes (Kraft
    equality), by enumerating length vectors."""
    K = len(h)
    best = None
    for lens in itertools.product(range(1, K), repeat=K):
        if sum(Fraction(1, 2 ** l) for l in lens) != 1:
            continue
        c = sum(a * b for a, b in zip(h, lens))
        best = c if best is None else min(best, c)
    return best


def test_huffman_bruteforce_small(orc):
    rng = np.random.default_rng(11)
    for trial in range(60):
        K = int(rng.integers(2, 7))
        h = [int(v) for v in rng.integers(1, 30, size=K)]
        if trial % 3 == 0:
            h = [int(v) for v in rng.integers(1, 4, size=K)]  # many ties
        hist = np.zeros(16, dtype=np.uint64)
        syms = rng.choice(16, size=K, replace=False)
        hist[syms] = h
        lens = orc.huffman_lengths(hist)
        assert np.all((lens > 0) == (hist > 0))
        assert sum(Fraction(1, 2 ** int(lens[s])) for s in syms) == 1
        assert sum(int(hist[s]) * int(lens[s]) for s in syms) == brute_min_cost(h)


def test_huffman_entropy_bounds_and_kraft(orc):
    rng = np.random.default_rng(5)
    for _ in range(20):
        k = rng.integers(2, 3000)
        hist = np.zeros(65536, dtype=np.uint64)
        idx = rng.choice(65536, size=k, replace=False)
        hist[idx] = (rng.pareto(1.2, size=k) * 50 + 1).astype(np.uint64)
        lens = orc.huffman_lengths(hist)
        used = hist > 0
        kraft = sum(Fraction(1, 2 ** int(l)) for l in lens[used])
        assert kraft == 1
        n = hist.sum(dtype=np.float64)
        p = hist[used] / n
        H = -(p * np.log2(p)).sum()
        bits = (hist[used].astype(np.float64) * lens[used]).sum()
        assert n * H <= bits + 1e-6 and bits < n * (H + 1)


def test_huffman_single_symbol_and_empty(orc):
    hist = np.zeros(8, dtype=np.uint64)
    assert orc.huffman_lengths(hist).tolist() == [0] * 8
    hist[5] = 100
    lens = orc.huffman_lengths(hist)
    assert lens.tolist() == [0, 0, 0, 0, 0, 1, 0, 0]
    cw = orc.canonical_codes(lens)
    syms = np.full(70, 5, dtype=np.uint16)
    words, cwords = orc.pack(syms, lens, cw, 64)
    assert cwords.tolist() == [2, 1]  # 64 zero bits, then 6 bits -> one word
    assert np.all(words == 0)
    assert np.array_equal(orc.unpack(words, cwords, 70, 64, lens), syms)


def test_codec_roundtrip_long_codes(orc):
    """Fibonacci frequencies give the deepest tree: 65 symbols reach 64 bits."""
    fib = [1, 1]
    while len(fib) < 65:
        fib.append(fib[-1] + fib[-2])
    hist = np.zeros(128, dtype=np.uint64)
    hist[:65] = fib
    lens = orc.huffman_lengths(hist)
    assert lens.max() == 64
    cw = orc.canonical_codes(lens)
    rng = np.random.default_rng(3)
    syms = rng.permutation(np.repeat(np.arange(65, dtype=np.uint16), 3))
    for chunk in (1, 7, 64, 1000):
        words, cwords = orc.pack(syms, lens, cw, chunk)
        assert np.array_equal(orc.unpack(words, cwords, syms.size, chunk, lens), syms)


def test_codec_roundtrip_random(orc):
    rng = np.random.default_rng(8)
    for n, chunk in ((1, 4096), (4095, 4096), (4097, 4096), (50000, 1000), (3333, 512)):
        codes = np.clip(np.round(rng.laplace(0, 20, size=n)) + 300, 1, 599).astype(np.uint16)
        hist = orc.histogram(codes, 600)
        lens = orc.huffman_lengths(hist)
        cw = orc.canonical_codes(lens)
        words, cwords = orc.pack(codes, lens, cw, chunk)
        assert cwords.size == (n + chunk - 1) // chunk
        assert np.array_equal(orc.unpack(words, cwords, n, chunk, lens), codes)


def _sub_layout_rule(chunk, sub):
    # the sub-chunk rule of the stream format, written out: S in {1, 2, 4, 8}
    # equal runs, each a whole number of the encoder's per-lane runs of
    # max(32, chunk / 64) symbols
    if sub == 1:
        return True
    if sub not in (2, 4, 8) or chunk % sub:
        return False
    return (chunk // sub) % max(32, chunk // 64) == 0


def test_subchunk_rule_and_default(orc):
    for chunk in (1, 7, 32, 64, 96, 128, 256, 1000, 1024, 4096, 4160, 8192, 65536):
        for sub in range(0, 10):
            assert orc.check_sub(chunk, sub) == _sub_layout_rule(chunk, sub), (chunk, sub)
    assert orc.default_sub(4096) == 4 and orc.default_sub(65536) == 4
    assert orc.default_sub(64) == 2 and orc.default_sub(128) == 4 and orc.default_sub(96) == 1
    assert orc.default_sub(100) == 1


def test_subchunk_offsets_are_code_length_prefix_sums(orc):
    """A sub-chunk starts at the sum of the code lengths of the chunk's
    symbols before it (counted directly from the lengths here); symbols,
    words and decoding do not depend on the split; a wrong offset is caught."""
    rng = np.random.default_rng(31)
    n = 3 * 4096 + 1234  # a partial last chunk whose last two runs are empty
    codes = np.clip(np.round(rng.laplace(0, 9, size=n)) + 200, 0, 399).astype(np.uint16)
    codes[rng.integers(0, n, size=50)] = 0
    hist = orc.histogram(codes, 400)
    lens = orc.huffman_lengths(hist)
    cw = orc.canonical_codes(lens)
    chunk = 4096
    w1, cw1 = orc.pack(codes, lens, cw, chunk)
    L = lens[codes].astype(np.int64)
    for sub in (2, 4, 8):
        words, cwords, sbits = orc.pack(codes, lens, cw, chunk, sub)
        assert np.array_equal(words, w1) and np.array_equal(cwords, cw1)
        span = chunk // sub
        want = []
        for c in range((n + chunk - 1) // chunk):
            lo, hi = c * chunk, min(n, (c + 1) * chunk)
            for k in range(1, sub):
                want.append(int(L[lo:min(hi, lo + k * span)].sum()))
        assert sbits.tolist() == want
        assert np.array_equal(orc.unpack(words, cwords, n, chunk, lens, sub, sbits), codes)
        for j in (0, len(want) - 1, len(want) // 2):
            for dlt in (-1, 1):
                bad = sbits.copy()
                bad[j] = np.uint32(int(bad[j]) + dlt)
                with pytest.raises(Exception):
                    orc.unpack(words, cwords, n, chunk, lens, sub, bad)


# ------------------------------------------------------------ quantizer

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_quantizer_near_ties(orc, dtype):
    """diff = (k + 1/2) * 2eb +- 1 ulp: the code differs from exact rational
    rounding by at most one bin and the bound always holds exactly."""
    rng = np.random.default_rng(17)
    R = 32768
    for _ in range(400):
        eb = dtype(10.0 ** rng.uniform(-6, 2))
        pred = dtype(rng.uniform(-100, 100))
        k = int(rng.integers(-40, 40))
        x0 = pred + dtype((k + 0.5) * 2.0 * float(eb))
        for x in (np.nextafter(x0, -np.inf, dtype=dtype), x0, np.nextafter(x0, np.inf, dtype=dtype)):
            code, rec = orc.quantize_one(x, pred, float(eb), R, dtype)
            if code == 0:
                assert rec.tobytes() == dtype(x).tobytes()
                continue
            kq = code - R
            exact = (Fraction(float(x)) - Fraction(float(pred))) / (2 * Fraction(float(eb)))
            assert abs(kq - exact) <= Fraction(3, 2)
            assert abs(Fraction(float(x)) - Fraction(float(rec))) <= Fraction(float(eb))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_quantizer_special_values(orc, dtype):
    big = np.finfo(dtype).max
    tiny = np.finfo(dtype).smallest_subnormal
    for x, pred, eb in ((np.nan, 0.0, 1.0), (np.inf, 0.0, 1.0), (-np.inf, 1.0, 1.0),
                        (1.0, np.nan, 1.0), (big, -big, 1.0), (1.0, 0.0, 1e-30),
                        (tiny * 5, 0.0, tiny), (tiny, -tiny, tiny), (0.0, 0.0, 0.0),
                        (1.0, 1.0, 0.0), (1.0, 0.5, 0.0)):
        code, rec = orc.quantize_one(x, pred, float(dtype(eb)), 32768, dtype)
        xv = dtype(x)
        if code == 0:
            assert rec.tobytes() == xv.tobytes()
        else:
            assert abs(Fraction(float(xv)) - Fraction(float(rec))) <= Fraction(float(dtype(eb)))
    # eb = 0: only an exact prediction is coded
    assert orc.quantize_one(1.0, 1.0, 0.0, 32768, dtype)[0] == 32768
    assert orc.quantize_one(1.0, 0.5, 0.0, 32768, dtype)[0] == 0
    # subnormal bound (half the smallest normal, so 1/(2 eb) is finite): exact
    sub = dtype(np.finfo(dtype).tiny / 2)
    code, rec = orc.quantize_one(sub * 6, 0.0, float(sub), 32768, dtype)
    assert code == 32768 + 3 and rec == dtype(sub * 6)
    # with the smallest subnormal bound 1/(2 eb) overflows: stored verbatim
    code, rec = orc.quantize_one(tiny * 6, 0.0, float(tiny), 32768, dtype)
    assert code == 0 and rec == dtype(tiny * 6)


def test_exact_bound_check_rejects_rounded_difference(orc):
    """A difference that rounds to exactly eb but exceeds it must be rejected.
    f32, eb = 1, pred = -2^-30, x = 1: fl(x - pred) = 1, so k = rint(0.5) = 0
    and x' = pred; fl(x - x') == eb while the exact difference is 1 + 2^-30."""
    f = np.float32
    eb = f(1.0)
    pred = f(-2.0 ** -30)
    x = f(1.0)
    code, rec = orc.quantize_one(x, pred, float(eb), 32768, f)
    assert code == 0 and rec == x


# --------------------------------------------------------- error bounds

def test_resolve_eb(orc):
    x = np.array([1.0, np.nan, -3.0, np.inf, 5.0], dtype=np.float32)
    assert orc.resolve_eb(x, orc.REL, 0.5) == np.float32(0.5 * 8.0)
    assert orc.resolve_eb(x, orc.ABS, 0.1) == float(np.float32(0.1))
    assert orc.resolve_eb(np.array([np.nan, np.inf], dtype=np.float64), orc.REL, 0.1) == 0.0
    with pytest.raises(Exception):
        orc.resolve_eb(x, orc.ABS, -1.0)
    with pytest.raises(Exception):
        orc.resolve_eb(x, orc.ABS, 1e300)  # not representable in f32


# ------------------------------------------------------------- format

@pytest.mark.parametrize("chunk,sub", [(100, None), (128, 4), (64, 2), (256, 8), (256, 1)])
def test_format_roundtrip_and_sections(orc, chunk, sub):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((20, 30)).astype(np.float64)
    x[4, 4] = 1e30
    s = orc.compress(x, orc.REL, 1e-4, orc.CUBIC, 512, chunk, sub=sub)
    h = orc.parse_header(s)
    assert h["magic"] == b"SZG1" and h["version"] == 1 and h["dims"] == (20, 30)
    assert h["stream_bytes"] == len(s)
    assert h["sub"] == (orc.default_sub(chunk) if sub is None else sub)
    K, nch, S = h["nsym"], (600 + chunk - 1) // chunk, h["sub"]
    pad8 = lambda v: (v + 7) & ~7
    off_bits = 128 + pad8(4 * K) + 8 * nch + pad8(4 * (S - 1) * nch) + pad8(8 * h["n_unpred"])
    assert off_bits + 4 * h["total_words"] == len(s)
    assert h["n_unpred"] >= 1
    # identical input -> identical bytes (deterministic)
    assert orc.compress(x, orc.REL, 1e-4, orc.CUBIC, 512, chunk, sub=sub) == s
    # the split changes only the header field and the sub-chunk table
    one = orc.compress(x, orc.REL, 1e-4, orc.CUBIC, 512, chunk, sub=1)
    assert np.array_equal(orc.decompress(one), orc.decompress(s))
    assert s[-4 * h["total_words"]:] == one[-4 * h["total_words"]:]


def test_corruption_detected(orc):
    rng = np.random.default_rng(9)
    x = np.cumsum(rng.standard_normal((40, 50)), axis=1).astype(np.float32)
    s = orc.compress(x, orc.REL, 1e-3, orc.LINEAR, 32768, 256)
    ref = orc.decompress(s)
    h = orc.parse_header(s)
    K = h["nsym"]
    nch = (2000 + 255) // 256
    assert h["sub"] == 4
    off_sub = 128 + ((4 * K + 7) & ~7) + 8 * nch
    # header fields, symbol table, chunk table and sub-chunk table entries are
    # all checked
    for pos in list(range(0, 12)) + [40, 41, 45, 64, 68, 72, 80, 84, 88, 96] + \
            [128 + 4 * i + 2 for i in range(min(K, 8))] + [128 + ((4 * K + 7) & ~7) + 3] + \
            [off_sub, off_sub + 4 * 3 * (nch - 1) + 8]:
        bad = bytearray(s)
        bad[pos] ^= 0x5A
        with pytest.raises(Exception):
            orc.decompress(bytes(bad))
    # a flipped bitstream bit is detected or changes the output
    for pos in rng.integers(len(s) - 4 * h["total_words"], len(s), size=20):
        bad = bytearray(s)
        bad[int(pos)] ^= 0x10
        try:
            out = orc.decompress(bytes(bad))
        except Exception:
            continue
        assert not np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    with pytest.raises(Exception):
        orc.decompress(s[:-4])


# ------------------------------------------------------------- edge shapes

@pytest.mark.parametrize("shape", [(1,), (2,), (1, 1, 1), (0,), (4, 0, 3), (1, 1, 5), (2, 3, 1, 2)])
def test_edge_shapes(orc, shape):
    x = (np.arange(int(np.prod(shape)), dtype=np.float32) * 0.37).reshape(shape)
    s, codes, recon = orc.compress(x, orc.REL, 1e-2, orc.CUBIC, want_debug=True)
    back = orc.decompress(s)
    assert back.shape == shape
    assert np.array_equal(back, recon)
    if x.size:
        exact_within(x, back, orc.parse_header(s)["eb"])


def test_bad_arguments(orc):
    x = np.zeros((4, 4), dtype=np.float32)
    for kw in (dict(radius=0), dict(radius=40000), dict(chunk=0), dict(predictor=7),
               dict(order=(0, 0))):
        args = dict(predictor=orc.LINEAR, radius=32768, chunk=64, order=None)
        args.update(kw)
        with pytest.raises(Exception):
            orc.compress(x, orc.ABS, 0.1, **args)


@pytest.mark.parametrize("n,nsym,seed", [(1, 2, 0), (7, 8, 1), (4099, 65536, 2), (100000, 17, 3)])
def test_histogram_is_a_direct_count(orc, n, nsym, seed):
    """The histogram against an independent count (numpy's bincount), with
    symbol 0 at the first position, the largest symbol nsym - 1 at the last
    and a symbol that occurs only there, so that a skipped first or last
    element or an off-by-one in the symbol index changes the counts."""
    rng = np.random.default_rng(seed)
    codes = rng.integers(1, max(nsym - 1, 2), size=n).astype(np.uint16)
    codes[0] = 0
    codes[-1] = nsym - 1
    codes[1:-1][codes[1:-1] == nsym - 1] = 1
    h = orc.histogram(codes, nsym)
    want = np.bincount(codes, minlength=nsym)
    assert h.dtype == np.uint64 and h.shape == (nsym,)
    assert np.array_equal(h.astype(np.int64), want)
    assert int(h.sum()) == n
    with pytest.raises(Exception):
        orc.histogram(np.array([nsym], dtype=np.uint16), nsym)
