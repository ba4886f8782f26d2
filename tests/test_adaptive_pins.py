"""Pins of adaptive interpolation in the oracle: exact polynomial fields
(cubic reproduces them, so every level takes cubic), a step (linear wins at
the fine levels), a brute-force computation of the level costs on small 1-D
fields, consistency with the fixed predictors, and the stored level mask."""
import numpy as np
import pytest

import synth


def _mask(orc, s):
    return orc.parse_header(s)["level_mask"]


@pytest.mark.parametrize("shape", [(300,), (40, 37), (17, 20, 23)])
def test_polynomials_take_cubic(orc, shape):
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    L = max(int(np.ceil(np.log2(n))) for n in shape)
    for x in (sum(0.5 * g for g in grids) + 3.0,           # linear
              sum(0.01 * g * g for g in grids),            # quadratic: linear errs, cubic exact
              sum(1e-4 * g ** 3 - 0.02 * g for g in grids)):  # cubic
        x = x.astype(np.float64)
        s = orc.compress(x, orc.ABS, 1e-6, orc.ADAPTIVE)
        assert _mask(orc, s) == (1 << L) - 1
        # then the stream equals the cubic one (in the chosen dimension order)
        # apart from the predictor byte and the mask
        order = tuple(s[41:41 + x.ndim])
        c = orc.compress(x, orc.ABS, 1e-6, orc.CUBIC, order=order)
        a = bytearray(s)
        a[40] = orc.CUBIC
        a[124:128] = b"\0\0\0\0"
        assert bytes(a) == c


def _costs_1d(x, eb, R, L):
    """Level costs of a 1-D field, straight from the definitions: every point
    of level l predicted both ways from the original values, cost min(|k|, R)."""
    x = x.astype(np.float32)
    two = np.float32(2) * np.float32(eb)
    inv = np.float32(1) / two
    n = x.size
    cost = {}
    for l in range(L, 0, -1):
        s = 1 << (l - 1)
        c = [0, 0]
        for i in range(s, n, 2 * s):
            b = x[i - s]
            has_a, has_c, has_e = i >= 3 * s, i + s < n, i + 3 * s < n
            for k in (0, 1):
                if not has_c:
                    p = (np.float32(3) * b - x[i - 3 * s]) * np.float32(0.5) if has_a else b
                elif k == 0:
                    p = (b + x[i + s]) * np.float32(0.5)
                elif has_a and has_e:
                    p = (np.float32(9) * (b + x[i + s]) - (x[i - 3 * s] + x[i + 3 * s])) * np.float32(0.0625)
                elif has_e:
                    p = ((np.float32(3) * b + np.float32(6) * x[i + s]) - x[i + 3 * s]) * np.float32(0.125)
                elif has_a:
                    p = ((np.float32(6) * b + np.float32(3) * x[i + s]) - x[i - 3 * s]) * np.float32(0.125)
                else:
                    p = (b + x[i + s]) * np.float32(0.5)
                kf = np.rint(np.abs(np.float32(x[i] - p)) * inv)
                c[k] += int(kf) if kf < R else R
        cost[l] = c
    return cost


@pytest.mark.parametrize("seed,n", [(1, 97), (2, 256), (3, 1000)])
def test_level_costs_brute_force(orc, seed, n):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.standard_normal(n)).astype(np.float32)
    x[n // 3:] += 7.0  # a step
    eb = 0.05
    L = int(np.ceil(np.log2(n)))
    cost = _costs_1d(x, eb, 32768, L)
    want = sum(1 << (l - 1) for l in range(1, L + 1) if cost[l][1] <= cost[l][0])
    s = orc.compress(x, orc.ABS, eb, orc.ADAPTIVE)
    assert _mask(orc, s) == want


def test_step_prefers_linear_at_fine_levels(orc):
    x = (np.arange(512) > 200.5).astype(np.float32) * 5 + 1
    m = _mask(orc, orc.compress(x, orc.ABS, 1e-4, orc.ADAPTIVE))
    assert m & 1 == 0  # the finest level: linear errs at one point, cubic overshoots at more


def test_roundtrip_and_mixed_mask(orc):
    x = synth.climate_2d((181, 362), seed=3, dtype=np.float32)
    s, codes, rec = orc.compress(x, orc.REL, 1e-3, orc.ADAPTIVE, want_debug=True)
    assert orc.decompress(s).tobytes() == rec.tobytes()
    m = _mask(orc, s)
    L = 9
    assert 0 < m < (1 << L) - 1 and m >> L == 0
    err = np.abs(orc.decompress(s).astype(np.float64) - x)
    assert err.max() <= orc.parse_header(s)["eb"]


def test_bad_masks_rejected(orc):
    x = synth.random_field((30, 20), seed=2)
    s = bytearray(orc.compress(x, orc.REL, 1e-3, orc.ADAPTIVE))
    bad = bytearray(s)
    bad[124 + 3] |= 0x80  # a level the field does not have
    with pytest.raises(Exception):
        orc.decompress(bytes(bad))
    fixed = bytearray(orc.compress(x, orc.REL, 1e-3, orc.CUBIC))
    fixed[124] = 1  # a mask on a fixed-predictor stream
    with pytest.raises(Exception):
        orc.decompress(bytes(fixed))


def _row_sampled(r):
    return ((r * 0x9E3779B1) & 0xFFFFFFFF) >> 29 == 0


def _ctz(v):
    return 64 if v == 0 else (v & -v).bit_length() - 1


def _predict(xf, q, d, s, dims, strides, cubic):
    """The interpolation rules written out (Section 6.2 stencils, the edge
    cases of the cubic and linear rules), in float32."""
    i, nd = q[d], dims[d]
    f = sum(qe * st for qe, st in zip(q, strides))
    sd = s * strides[d]
    b = xf[f - sd]
    has_a, has_c, has_e = i >= 3 * s, i + s < nd, i + 3 * s < nd
    h = np.float32
    if not has_c:
        return (h(3) * b - xf[f - 3 * sd]) * h(0.5) if has_a else b
    c = xf[f + sd]
    if not cubic:
        return (b + c) * h(0.5)
    if has_a and has_e:
        return (h(9) * (b + c) - (xf[f - 3 * sd] + xf[f + 3 * sd])) * h(0.0625)
    if has_e:
        return ((h(3) * b + h(6) * c) - xf[f + 3 * sd]) * h(0.125)
    if has_a:
        return ((h(6) * b + h(3) * c) - xf[f - 3 * sd]) * h(0.125)
    return (b + c) * h(0.5)


def _order_total(x, order, eb, R):
    """Sampled price of one dimension order: per level, the cheaper of the
    two cost sums over the points of sampled rows; every point's level and
    pass found from its coordinates (fewest trailing zeros, last dimension
    of the order with that many)."""
    dims = x.shape
    strides = [int(np.prod(dims[e + 1:])) for e in range(len(dims))]
    xf = x.reshape(-1).astype(np.float32)
    pos = {e: j for j, e in enumerate(order)}
    inv = np.float32(1) / (np.float32(2) * np.float32(eb))
    cost = {}
    for q in np.ndindex(*dims):
        t = min(_ctz(v) for v in q)
        if t == 64:
            continue
        f = sum(qe * st for qe, st in zip(q, strides))
        if not _row_sampled(f // dims[-1]):
            continue
        d = max((e for e in range(len(dims)) if _ctz(q[e]) == t), key=lambda e: pos[e])
        for k in (0, 1):
            p = _predict(xf, q, d, 1 << t, dims, strides, k == 1)
            kf = np.rint(np.abs(np.float32(xf[f] - p)) * inv)
            cost.setdefault(t, [0, 0])[k] += int(kf) if kf < R else R
    return sum(min(c) for c in cost.values())


@pytest.mark.parametrize("shape,seed", [((24, 40), 1), ((9, 11, 14), 2), ((30, 7, 12), 3),
                                        ((5, 6, 4, 7), 4)])
def test_order_is_the_cheapest_by_brute_force(orc, shape, seed):
    import itertools

    x = synth.random_field(shape, seed=seed)
    x = x + np.linspace(0, 3, shape[-1], dtype=np.float32)  # a trend along the last axis
    eb = 1e-2
    s = orc.compress(x, orc.ABS, eb, orc.ADAPTIVE)
    chosen = tuple(s[41:41 + x.ndim])
    totals = {p: _order_total(x, p, eb, 32768) for p in itertools.permutations(range(x.ndim))}
    best = min(totals.values())
    first = next(p for p in sorted(totals) if totals[p] == best)
    assert chosen == first, (chosen, first, totals)
    # the stream decodes in that order within the bound
    back = orc.decompress(s)
    assert np.abs(back.astype(np.float64) - x).max() <= orc.parse_header(s)["eb"]


def test_given_order_is_kept(orc):
    x = synth.random_field((20, 30), seed=5)
    s = orc.compress(x, orc.REL, 1e-3, orc.ADAPTIVE, order=(1, 0))
    assert tuple(s[41:43]) == (1, 0)


def _rough_smooth_field(shape, rough_axis, slopes, seed):
    """Integer-valued float32 field: seeded multiples of 16 in [-3200, 3200]
    along `rough_axis` (the same at every position of the other axes) plus an
    exactly linear trend slopes[e] * index along every other axis."""
    rng = np.random.default_rng(seed)
    r = 16.0 * rng.integers(-200, 201, size=shape[rough_axis])
    sh = [1] * len(shape)
    sh[rough_axis] = shape[rough_axis]
    x = np.broadcast_to(r.reshape(sh), shape).copy()
    for e, a in enumerate(slopes):
        if e != rough_axis and a:
            she = [1] * len(shape)
            she[e] = shape[e]
            x = x + a * np.arange(shape[e], dtype=np.float64).reshape(she)
    return x.astype(np.float32)


@pytest.mark.parametrize("shape,rough,slopes,want", [
    ((40, 36), 0, (0, 0), (0, 1)),
    ((40, 36), 1, (0, 0), (1, 0)),
    ((40, 36), 0, (0, 1), (0, 1)),
    ((33, 45), 1, (3, 0), (1, 0)),
    ((21, 17, 22), 2, (0, 0, 0), (2, 0, 1)),
    ((21, 17, 22), 0, (0, 0, 0), (0, 1, 2)),
    ((21, 17, 22), 1, (0, 0, 0), (1, 0, 2)),
    ((19, 21, 23), 1, (2, 0, 1), (1, 0, 2)),
])
def test_order_puts_the_rough_axis_first(orc, shape, rough, slopes, want):
    """What the order's definition fixes, independently of its sampling.

    At abs eb 1/2 every operation on these integer fields is exact: the
    stencils' weights have denominators 2, 8 and 16, the rough values are
    multiples of 16 and the trends are constant along the rough axis, so
    every prediction is an integer and every reconstruction equals the
    field.  Along an axis where the field is linear
    (slope 0 or not) both stencils are exact wherever the stencil has two
    points, so such passes cost nothing.  Only a point with a single known
    neighbour (p_d = s with s < n_d <= 2s) costs the slope times s, and only
    when the slope is not 0.  Along the rough axis a point's cost depends on
    its rough coordinate and the level alone.

    At stride s a pass along d takes the points whose coordinate along d is
    an odd multiple of s.  Their coordinates along the dimensions before d
    in the order are multiples of s, and along those after d multiples of 2s.
    In 2-D the first pass of a level therefore holds about (n/2s)^2 points
    and the second about n^2/(2s^2), twice as many.  In 3-D the three passes
    hold in the ratio 1 : 2 : 4.  The sampled rows are the same for every
    order, so the rough axis's pass holds a subset of its points when it
    comes first.  The order that puts the rough axis first is therefore
    never dearer.  It is strictly cheaper when, for every smooth axis e, a
    sampled row holds a stride-1 point with odd coordinates along the rough
    axis and along e and even ones elsewhere: every order that puts e before
    the rough axis prices that point's rough prediction and the rough-first
    order does not (checked below; it depends on the shape through the row
    sampling, a reading).  With the smooth axes at slope 0 the orders that
    start with the rough axis cost the same, and the first in lexicographic
    order wins.  A reversed tie rule, or a pass counted at the wrong
    position, picks another order."""
    nd = len(shape)
    for e in range(nd):
        if e == rough:
            continue
        assert any(_row_sampled(int(np.ravel_multi_index(q, shape)) // shape[-1])
                   for q in np.ndindex(*shape)
                   if q[rough] % 2 == 1 and q[e] % 2 == 1
                   and all(q[f] % 2 == 0 for f in range(nd) if f not in (rough, e)))
    x = _rough_smooth_field(shape, rough, slopes, seed=sum(shape) + rough)
    s = orc.compress(x, orc.ABS, 0.5, orc.ADAPTIVE)
    assert tuple(s[41:41 + x.ndim]) == want
    assert orc.decompress(s).tobytes() == x.tobytes()
