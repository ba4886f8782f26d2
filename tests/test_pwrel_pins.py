"""Pins of the point-wise relative mode's oracle (the logarithmic
preprocessor): its log2/exp2 series against 60-digit references, the log
field's bound, the point-wise bound on every normal value, the special
values, and the stream's sign section."""
import math
import random
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import synth

getcontext().prec = 60


def _ulps(got: float, ref: Decimal) -> float:
    return float(abs(Decimal(got) - ref) / Decimal(math.ulp(float(ref))))


def test_log2_series_within_one_ulp(orc):
    rng = random.Random(11)
    worst = 0.0
    for _ in range(2000):
        a = math.ldexp(rng.uniform(0.5, 1.0), rng.randint(-1074, 1023))
        if a == 0.0:
            continue
        ref = Decimal(a).ln() / Decimal(2).ln()
        worst = max(worst, _ulps(orc.log2(a), ref))
    assert worst <= 1.0, worst
    # exact at powers of two, and at 1
    for k in (-1074, -1022, -126, -1, 0, 1, 52, 1023):
        assert orc.log2(math.ldexp(1.0, k)) == float(k)


def test_exp2_series_within_two_ulps(orc):
    rng = random.Random(12)
    worst = 0.0
    for _ in range(2000):
        y = rng.uniform(-1020.0, 1023.0)
        ref = Decimal(2) ** Decimal(y)
        worst = max(worst, _ulps(orc.exp2(y), ref))
    assert worst <= 2.0, worst
    for k in (-1022, -126, -1, 0, 1, 100, 1023):
        assert orc.exp2(float(k)) == math.ldexp(1.0, k)


@pytest.mark.parametrize("dtype,u,e_log", [(0, 2.0 ** -24, 2.0 ** -45), (1, 2.0 ** -53, 2.0 ** -42)])
def test_delta_formula(orc, dtype, u, e_log):
    for eps in (0.5, 1e-1, 1e-3, 1e-6) + ((1e-9, 1e-12) if dtype == 1 else ()):
        d = orc.pwrel_delta(eps, dtype)
        # the definition's double roundings (1 + eps, its quotient), then the
        # logarithm to 60 digits, the margin factor and the absolute margin
        r = (1.0 + eps) / (1.0 + 4.0 * u)
        ref = (Decimal(r).ln() / Decimal(2).ln() * (1 - Decimal(2) ** -20)
               - Decimal(e_log) - Decimal(2) ** -50)
        assert abs(Decimal(d) - ref) <= 2 * Decimal(math.ulp(float(ref)))
        # and the margins are real: with the log's largest rounding error E
        # added back, 2^(d + E) (1 + 4u) stays below 1 + eps (the exact
        # 1 + eps, not its double)
        assert Decimal(2) ** (Decimal(d) + Decimal(e_log)) * (1 + 4 * Decimal(u)) < 1 + Decimal(eps)
    # unusable bounds: too small for the type (the absolute margin alone
    # needs eps above about 2^-42 ln 2 = 1.6e-13 for doubles), or outside (0, 1)
    assert orc.pwrel_delta(1e-9 if dtype == 0 else 1e-18, dtype) <= 0
    if dtype == 1:
        assert orc.pwrel_delta(1e-13, dtype) <= 0 and orc.pwrel_delta(1e-14, dtype) <= 0
    for bad in (0.0, -1e-3, 1.0, 2.0, float("nan")):
        assert orc.pwrel_delta(bad, dtype) <= 0


def _field(dtype, seed):
    x = synth.random_field((26, 24, 22), seed=seed, dtype=dtype)
    x = (np.sign(x - np.median(x)) * np.exp(3 * x)).astype(dtype)  # mixed signs, wide range
    x.flat[::97] = 0
    return x


def _check_pointwise(x, back, eps):
    tiny = np.finfo(x.dtype).tiny
    normal = np.isfinite(x) & (np.abs(x) >= tiny)
    # exact rational check on every normal value
    for a, b in zip(x[normal].ravel().tolist(), back[normal].ravel().tolist()):
        assert abs(Fraction(a) - Fraction(b)) <= Fraction(eps) * abs(Fraction(a)), (a, b)


@pytest.mark.parametrize("dtype,eps", [(np.float32, 1e-1), (np.float32, 1e-3), (np.float32, 1e-6),
                                       (np.float64, 1e-3), (np.float64, 1e-12)])
def test_pointwise_bound_holds(orc, dtype, eps):
    x = _field(dtype, 21)
    s, codes, rec = orc.compress(x, orc.PWREL, eps, orc.CUBIC, want_debug=True)
    back = orc.decompress(s)
    assert back.tobytes() == rec.tobytes()
    _check_pointwise(x, back, eps)
    h = orc.parse_header(s)
    assert h["eb_mode"] == orc.PWREL and h["dtype"] == orc.F64
    assert h["out_dtype"] == (orc.F64 if dtype == np.float64 else orc.F32)
    assert h["eb_user"] == eps and h["eb"] == orc.pwrel_delta(eps, h["out_dtype"])


def test_special_values(orc):
    x = np.full((9, 10, 11), 3.0, dtype=np.float32)
    x[0, 0, 0] = 0.0
    x[0, 0, 1] = -0.0
    x[1, 1, 1] = np.float32(1e-40)   # subnormal: back as a signed zero
    x[1, 1, 2] = -np.float32(1e-41)
    x[2, 2, 2] = np.inf
    x[2, 2, 3] = -np.inf
    x[3, 3, 3] = np.nan
    x[4, 4, 4] = -2.5
    x[5, 5, 5] = np.finfo(np.float32).max
    x[5, 5, 6] = np.finfo(np.float32).tiny
    back = orc.decompress(orc.compress(x, orc.PWREL, 1e-3, orc.LINEAR))
    assert back[0, 0, 0] == 0 and not np.signbit(back[0, 0, 0])
    assert back[0, 0, 1] == 0 and np.signbit(back[0, 0, 1])
    assert back[1, 1, 1] == 0 and not np.signbit(back[1, 1, 1])
    assert back[1, 1, 2] == 0 and np.signbit(back[1, 1, 2])
    assert back[2, 2, 2] == np.inf and back[2, 2, 3] == -np.inf
    assert np.isnan(back[3, 3, 3])
    assert np.isfinite(back[5, 5, 5])  # clamped to the largest float
    _check_pointwise(x, back, 1e-3)


def test_sign_section(orc):
    pos = np.abs(synth.random_field((20, 30), seed=4)) + 1
    s = orc.compress(pos, orc.PWREL, 1e-2, orc.CUBIC)
    h = orc.parse_header(s)
    assert h["signs"] == 0 and h["off_signs"] == 0 and h["stream_bytes"] == len(s)
    neg = pos.copy()
    neg[3, 4] = -neg[3, 4]
    s2 = orc.compress(neg, orc.PWREL, 1e-2, orc.CUBIC)
    h2 = orc.parse_header(s2)
    n = neg.size
    assert h2["signs"] == 1 and h2["off_signs"] % 8 == 0
    assert h2["stream_bytes"] == len(s2) == h2["off_signs"] + 8 * ((n + 63) // 64)
    words = np.frombuffer(s2[h2["off_signs"]:], dtype="<u8")
    i = 3 * 30 + 4
    assert words[i // 64] == 1 << (i % 64) and words.sum() == words[i // 64]
    assert orc.decompress(s2)[3, 4] < 0


def test_corrupt_extension_rejected(orc):
    x = -np.abs(synth.random_field((12, 14), seed=6)) - 1
    s = bytearray(orc.compress(x, orc.PWREL, 1e-2, orc.CUBIC))
    for off, v in ((104, 7), (105, 2), (106, 1), (112, s[112] ^ 0x40), (6, 0), (120, 1)):
        bad = bytearray(s)
        bad[off] = v
        with pytest.raises(Exception):
            orc.decompress(bytes(bad))
    with pytest.raises(Exception):
        orc.decompress(bytes(s[:-8]))


def _extreme(dtype, mag, seed):
    """A positive field spanning a factor e^6 around `mag`, with both signs."""
    x = synth.random_field((14, 12, 10), seed=seed, dtype=np.float64)
    v = mag * np.exp(x) * np.where(x > 0, 1.0, -1.0)
    return v.astype(dtype)


@pytest.mark.parametrize("dtype,mag,eps", [
    (np.float64, 1e300, 1e-12), (np.float64, 1e-300, 1e-12), (np.float64, 1e100, 2e-13),
    (np.float64, 1e-300, 2e-13), (np.float64, 1e300, 1e-6), (np.float32, 1e36, 1e-6),
    (np.float32, 1e-36, 1e-6), (np.float32, 1e36, 3e-7),
])
def test_pointwise_bound_at_extreme_exponents(orc, dtype, mag, eps):
    """Near the ends of the exponent range |log2|x|| approaches 1024 (128),
    where the rounding of the logarithm is largest: the bound still holds at
    every point, in exact rationals, down to the smallest accepted eps."""
    x = _extreme(dtype, mag, seed=int(abs(math.log10(mag))))
    assert np.all(np.isfinite(x)) and np.all(np.abs(x) >= np.finfo(dtype).tiny)
    back = orc.decompress(orc.compress(x, orc.PWREL, eps, orc.CUBIC))
    _check_pointwise(x, back, eps)


@pytest.mark.parametrize("eps", [1e-13, 1e-14])
def test_too_small_bound_rejected_for_doubles(orc, eps):
    """A double field of values near 1e300 at eps = 1e-14 would break the
    bound (the rounding of log2|x| alone is about 4e-14 relative there), so
    bounds below the absolute margin are refused."""
    x = _extreme(np.float64, 1e300, seed=300)
    with pytest.raises(Exception):
        orc.compress(x, orc.PWREL, eps, orc.CUBIC)
