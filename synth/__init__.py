"""Seeded synthetic fields standing in for the paper's datasets.

This module only draws inputs; it holds none of the compressor's arithmetic.
Both the GPU path and the CPU oracle are fed the exact bytes it returns.

The paper's evaluation data (Section 6.2, Table "Dataset Information": NYX
512^3 cosmology, ATM 1800x3600 climate, Hurricane 13 x 100x500x500) is not
available, so each workload is a seeded field of the same shape with a
comparable value distribution:

* ``sinusoid_field``  -- 64^3 sum of 8 random sinusoids plus small noise.
* ``lognormal_grf``   -- exp of a Gaussian random field with P(k) ~ k^-3
                          (density-like, heavy tailed; NYX stand-in).
* ``climate_2d``      -- smooth large-scale modes + tanh fronts + 0.1%
                          spikes (ATM stand-in).
* ``batch_fields``    -- 13 offset/scaled GRFs of 100x500x500 plus 64 small
                          fields (Hurricane-like variables).
* ``serving_pool``    -- base fields (GRFs of 256x512x512, slopes spread over
                          [-4, -2]) that serving requests crop.
* ``serving_requests``-- the serving workload's requests: size, aspect ratio,
                          base field, crop origin and bound of each.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

try:  # multithreaded FFTs when scipy is present
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _fft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def grf(shape, alpha: float, rng: np.random.Generator, dtype=np.float64) -> np.ndarray:
    """Gaussian random field with power spectrum P(k) ~ |k|^alpha.

    White noise -> rFFT -> multiply by |k|^(alpha/2) (k in cycles/cell from
    fftfreq, the k=0 mode zeroed) -> inverse rFFT -> standardise to mean 0,
    std 1.  ``dtype`` selects the FFT precision (float32 halves memory for the
    largest fields).
    """
    shape = tuple(int(s) for s in shape)
    w = rng.standard_normal(shape, dtype=np.float64).astype(dtype, copy=False)
    spec = _rfftn(w)
    del w
    k2 = None
    for ax, n in enumerate(shape):
        f = np.fft.rfftfreq(n) if ax == len(shape) - 1 else np.fft.fftfreq(n)
        f = f.astype(dtype)
        sh = [1] * len(shape)
        sh[ax] = f.size
        f2 = (f * f).reshape(sh)
        k2 = f2 if k2 is None else k2 + f2
    with np.errstate(divide="ignore"):
        amp = np.power(k2, dtype(alpha / 4.0)) if k2.dtype == np.float32 else np.power(k2, alpha / 4.0)
    amp[(0,) * len(shape)] = 0.0
    spec *= amp
    del amp, k2
    out = _irfftn(spec, s=shape)
    del spec
    out = out.astype(np.float64, copy=False) if dtype == np.float64 else out
    m = out.mean(dtype=np.float64)
    sd = out.std(dtype=np.float64)
    out -= out.dtype.type(m)
    out *= out.dtype.type(1.0 / sd if sd > 0 else 1.0)
    return out


def sinusoid_field(n: int = 64, seed: int = 1) -> tuple[np.ndarray, float]:
    """Sum of 8 sinusoids (wavevector components U[0.5,4]*2pi/n, amplitudes
    U[0,1], phases U[0,2pi)) plus N(0, (1e-3 * range)^2) noise, as float32.

    Returns (field, abs_eb) with abs_eb = 1e-3 * (max - min) of the final
    float32 field, computed in double by the harness (absolute-bound mode)."""
    rng = np.random.default_rng(seed)
    ax = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    f = np.zeros((n, n, n), dtype=np.float64)
    for _ in range(8):
        kv = rng.uniform(0.5, 4.0, size=3) * 2.0 * math.pi / n
        a = rng.uniform(0.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        f += a * np.sin(kv[0] * z + kv[1] * y + kv[2] * x + ph)
    rng0 = float(f.max() - f.min())
    f += rng.normal(0.0, 1e-3 * rng0, size=f.shape)
    f32 = f.astype(np.float32)
    eb = 1e-3 * (float(f32.max()) - float(f32.min()))
    return f32, eb


def lognormal_grf(shape=(512, 512, 512), seed: int = 2, alpha: float = -3.0,
                  sigma: float = 1.0) -> np.ndarray:
    """exp(sigma * GRF(shape, alpha)) as float32: log-normal, density-like."""
    rng = np.random.default_rng(seed)
    big = int(np.prod(shape)) >= (1 << 24)
    g = grf(shape, alpha, rng, dtype=np.float32 if big else np.float64)
    g *= g.dtype.type(sigma)
    np.exp(g, out=g)
    return g.astype(np.float32, copy=False)


def climate_2d(shape=(1800, 3600), seed: int = 3, dtype=np.float64) -> np.ndarray:
    """Smooth large-scale part (16 terms a*cos(l*theta)*sin(q*lambda+phi),
    l, q in 0..8) + 20 tanh fronts (width U[2,10] cells, uniform orientation
    and position, height U[0.5,1.5]*std) + 0.1% isolated spikes of +-100x the
    local (9x9) standard deviation."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    th = math.pi * (np.arange(ny, dtype=np.float64) + 0.5) / ny
    lam = 2.0 * math.pi * np.arange(nx, dtype=np.float64) / nx
    f = np.zeros(shape, dtype=np.float64)
    for _ in range(16):
        l = rng.integers(0, 9)
        q = rng.integers(0, 9)
        a = rng.normal()
        ph = rng.uniform(0, 2 * math.pi)
        f += a * np.cos(l * th)[:, None] * np.sin(q * lam + ph)[None, :]
    sd = float(f.std()) or 1.0
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    for _ in range(20):
        w = rng.uniform(2.0, 10.0)
        ang = rng.uniform(0, 2 * math.pi)
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        b = rng.uniform(0.5, 1.5) * sd
        f += b * np.tanh(((yy - cy) * math.sin(ang) + (xx - cx) * math.cos(ang)) / w)
    del yy, xx
    npk = max(1, int(round(1e-3 * f.size)))
    idx = rng.choice(f.size, size=npk, replace=False)
    # local std over a 9x9 window (box filter of f and f^2 via cumulative sums)
    pad = np.pad(f, 4, mode="edge")
    c1 = pad.cumsum(0).cumsum(1)
    c2 = (pad * pad).cumsum(0).cumsum(1)
    c1 = np.pad(c1, ((1, 0), (1, 0)))
    c2 = np.pad(c2, ((1, 0), (1, 0)))

    def box(c):
        return c[9:, 9:] - c[:-9, 9:] - c[9:, :-9] + c[:-9, :-9]

    s1, s2 = box(c1) / 81.0, box(c2) / 81.0
    lsd = np.sqrt(np.maximum(s2 - s1 * s1, 0.0)) + 1e-12 * sd
    sign = rng.choice([-1.0, 1.0], size=npk)
    flat = f.reshape(-1)
    flat[idx] += sign * 100.0 * lsd.reshape(-1)[idx]
    return f.astype(dtype)


def batch_fields(seed: int = 4, n_large: int = 13, large_shape=(100, 500, 500),
                 n_small: int = 64, small_lo: int = 16, small_hi: int = 96):
    """The batching workload: ``n_large`` fields offset + scale * GRF with
    slope U[-4,-2] and offset, scale log-uniform over [1e-3, 1e6], plus
    ``n_small`` small fields with each dimension uniform in [lo, hi].
    Returns a list of (float32 field, rel_eb) with rel_eb log-uniform over
    [1e-5, 1e-2]."""
    rng = np.random.default_rng(seed)
    out = []
    shapes = [tuple(large_shape)] * n_large + [
        tuple(int(v) for v in rng.integers(small_lo, small_hi + 1, size=3)) for _ in range(n_small)
    ]
    for shp in shapes:
        alpha = rng.uniform(-4.0, -2.0)
        off = 10.0 ** rng.uniform(-3.0, 6.0)
        scale = 10.0 ** rng.uniform(-3.0, 6.0)
        rel = 10.0 ** rng.uniform(-5.0, -2.0)
        g = grf(shp, alpha, rng, dtype=np.float32 if int(np.prod(shp)) >= (1 << 24) else np.float64)
        f = (off + scale * g.astype(np.float64)).astype(np.float32)
        out.append((f, rel))
    return out


def serving_pool(seed: int = 5, n_base: int = 5, shape=(256, 512, 512)):
    """The base fields serving requests are cropped from: ``n_base`` float32
    GRFs of ``shape`` whose spectral slopes are spread evenly over [-4, -2].
    Returns a list of (field, slope)."""
    rng = np.random.default_rng(seed)
    slopes = np.linspace(-4.0, -2.0, n_base)
    return [(grf(shape, float(a), rng, dtype=np.float32).astype(np.float32, copy=False), float(a))
            for a in slopes]


def serving_requests(n: int = 10000, seed: int = 6, base_shape=(256, 512, 512), n_base: int = 5,
                     lo: int = 16 ** 3, hi: int = 256 * 512 * 512):
    """The serving workload: ``n`` compression requests, each a crop of a
    base field of ``serving_pool``.

    * size N log-uniform over [lo, hi] points;
    * aspect ratio: log n_d = w_d log N with w ~ Dirichlet(2, 2, 2); an
      extent above the base field's is clipped and its excess exponent shared
      among the other dimensions (extents at least 4);
    * spectral slope U[-4, -2], served by the base field of nearest slope;
    * crop origin uniform over the positions that fit;
    * range-relative bound log-uniform over [1e-5, 1e-2].

    Returns a list of dicts: shape, base, origin, slope, rel_eb."""
    rng = np.random.default_rng(seed)
    slopes = np.linspace(-4.0, -2.0, n_base)
    cap = np.log(np.asarray(base_shape, dtype=np.float64))
    out = []
    for _ in range(n):
        logn = rng.uniform(math.log(lo), math.log(hi))
        w = rng.dirichlet([2.0, 2.0, 2.0])
        ld = w * logn
        free = np.ones(3, dtype=bool)
        for _ in range(3):  # clip and share the excess among the others
            over = free & (ld > cap)
            if not over.any():
                break
            excess = float((ld[over] - cap[over]).sum())
            ld[over] = cap[over]
            free &= ~over
            if free.any():
                ld[free] += excess * w[free] / w[free].sum()
        dims = tuple(int(min(base_shape[d], max(4, round(math.exp(ld[d]))))) for d in range(3))
        slope = float(rng.uniform(-4.0, -2.0))
        base = int(np.argmin(np.abs(slopes - slope)))
        origin = tuple(int(rng.integers(0, base_shape[d] - dims[d] + 1)) for d in range(3))
        rel = float(10.0 ** rng.uniform(-5.0, -2.0))
        out.append({"shape": dims, "base": base, "origin": origin, "slope": slope, "rel_eb": rel})
    return out


def random_field(shape, seed: int, alpha: float = -3.0, dtype=np.float32) -> np.ndarray:
    """A plain seeded GRF of any shape (used for parity cases)."""
    rng = np.random.default_rng(seed)
    return grf(shape, alpha, rng).astype(dtype)


def fibonacci_counts(m: int) -> list[int]:
    """The first m Fibonacci numbers 1, 1, 2, 3, 5, ..."""
    f = [1, 1]
    while len(f) < m:
        f.append(f[-1] + f[-2])
    return f[:m]


def fibonacci_steps_field(shape=(256, 256, 256), nsym: int = 34, seed: int = 41):
    """An integer-valued float64 field whose mixed differences are steps with
    Fibonacci frequencies.

    The steps take the nsym integer values -nsym/2 .. nsym/2 - 1 (assigned to
    the Fibonacci counts 1, 1, 2, 3, ... in a seeded order; the most frequent
    value also takes the points left over), are placed at seeded random
    positions, and are summed along every axis.  Returns (field, steps): the
    steps array has the field's shape and int64 values."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    counts = fibonacci_counts(nsym)
    if sum(counts) > n:
        raise ValueError("field too small for the Fibonacci counts")
    counts[-1] += n - sum(counts)
    vals = np.arange(-(nsym // 2), nsym - nsym // 2, dtype=np.int64)
    rng.shuffle(vals)
    steps = np.repeat(vals, counts)[rng.permutation(n)].reshape(shape)
    x = steps
    for ax in range(len(shape)):
        x = np.cumsum(x, axis=ax)
    return x.astype(np.float64), steps
