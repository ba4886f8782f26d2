"""GPU parity at the workloads' full sizes and on codes longer than 32 bits.

* Codes of 33 bits: an integer field whose Lorenzo residuals have Fibonacci
  frequencies (synth.fibonacci_steps_field, 256^3 f64, abs eb 1/2).  The
  Huffman tree is a caterpillar 33 deep, so the codebook's deep path, the
  encoder's global-codebook variant (codes over 32 bits) and the decoder's
  exact long-code read all run.  The GPU compresses against the oracle and
  decodes the oracle's stream.
* The climate-like 1800 x 3600 field (the paper's ATM shape, Section 6.2
  dataset table) in f32 and f64, linear and cubic interpolation at rel 1e-4,
  and the radius-512 variant whose out-of-range errors take the
  unpredictable path.
* The 512^3 log-normal field (the NYX shape) at rel 1e-2, 1e-3 and 1e-4 with
  cubic interpolation: at 1e-4 the codebook holds thousands of symbols.

Every case is bit-exact: codes, stream bytes and reconstruction."""
import functools

import numpy as np
import pytest

import synth
from tests.test_gpu_parity import check_case

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


def max_code_length(stream: bytes, orc) -> int:
    h = orc.parse_header(stream)
    table = np.frombuffer(stream[128:128 + 4 * h["nsym"]], np.uint32)
    return int((table >> 16).max())


@pytest.mark.parametrize("sub", [4, 1])
def test_long_codes_33_bits(ctx, orc, sub):
    x, _steps = synth.fibonacci_steps_field((256, 256, 256), nsym=34, seed=41)
    ref = orc.compress(x, orc.ABS, 0.5, orc.LORENZO, 32768, 4096, sub=sub)
    assert max_code_length(ref, orc) == 33
    check_case(ctx, orc, x, "abs", 0.5, 3, label=f"long-codes-33bit-S{sub}", sub=sub)


@functools.lru_cache(maxsize=2)
def climate(dtype):
    return synth.climate_2d((1800, 3600), seed=3, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
@pytest.mark.parametrize("pred,radius", [(0, 32768), (1, 32768), (0, 512), (1, 512)],
                         ids=["linear", "cubic", "linear-R512", "cubic-R512"])
def test_climate_full_size(ctx, orc, dtype, pred, radius):
    check_case(ctx, orc, climate(dtype), "rel", 1e-4, pred, radius,
               label=f"climate-1800x3600-{np.dtype(dtype).name}")


@functools.lru_cache(maxsize=1)
def nyx_like():
    return synth.lognormal_grf((512, 512, 512), seed=2)


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_lognormal_512_cubed(ctx, orc, eb):
    check_case(ctx, orc, nyx_like(), "rel", eb, 1, label="lognormal-512^3")
