"""The request server through the C ABI: outputs byte-identical to the same
calls alone, the memory budget respected and enforced, unknown tickets."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def szg():
    import paper_2111_02925_amd as szg

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return szg


def fields():
    return [
        ("lognormal-3d", synth.lognormal_grf((48, 40, 36), seed=31), "rel", 1e-3, "cubic", 4096),
        ("climate-f64", synth.climate_2d((91, 180), seed=32, dtype=np.float64), "rel", 1e-4, "linear", 1024),
        ("1d", np.cumsum(np.random.default_rng(33).standard_normal(20011)).astype(np.float32), "abs", 0.05, "cubic", 2048),
        ("tiny", synth.random_field((5, 7), seed=34), "rel", 1e-2, "cubic", 64),
        ("lognormal-2", synth.lognormal_grf((33, 70, 45), seed=35), "rel", 1e-4, "linear", 4096),
        ("adaptive", synth.lognormal_grf((40, 36, 46), seed=36), "rel", 1e-3, "adaptive", 4096),
        ("lorenzo-f64", synth.climate_2d((61, 90), seed=37, dtype=np.float64), "rel", 1e-3, "lorenzo", 1024),
        ("pwrel", synth.lognormal_grf((30, 28, 26), seed=38), "pwrel", 1e-3, "cubic", 4096),
    ]


def test_server_outputs_equal_calls_alone(szg):
    print("[case] server: 8 fields x 3 repeats, 3 workers", flush=True)
    ctx = szg.Context(0)
    cases = []
    for label, x, mode, eb, pred, chunk in fields():
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        alone = ctx.compress(xt, mode, eb, pred, chunk=chunk)
        cases.append((label, xt, mode, eb, pred, chunk, bytes(alone.cpu().numpy().tobytes()),
                      ctx.decompress(alone).cpu().numpy().tobytes()))
    ctx.close()
    srv = szg.Server(0, budget_bytes=2 << 30, workers=3)
    try:
        tickets = []
        for rep in range(3):
            for c in cases:
                label, xt, mode, eb, pred, chunk = c[:6]
                tickets.append((c, srv.submit_compress(xt, mode, eb, pred, chunk=chunk)))
        streams = []
        for c, t in tickets:
            st, out = srv.wait(t)
            assert st == 0, (c[0], st)
            assert bytes(out.cpu().numpy().tobytes()) == c[6], c[0]
            streams.append((c, out))
        dts = [(c, srv.submit_decompress(s)) for c, s in streams]
        for c, t in dts:
            st, out = srv.wait(t)
            assert st == 0, (c[0], st)
            assert out.cpu().numpy().tobytes() == c[7], c[0]
    finally:
        srv.close()


def test_server_budget_respected_and_enforced(szg):
    print("[case] server: budget", flush=True)
    probe = szg.Server(0, budget_bytes=1 << 30, workers=2)
    fixed = probe.used_bytes()  # idle, nothing held: the two contexts' fixed part
    probe.close()
    assert fixed > 0
    # room for one 32^3 f32 compression's scratch (about 0.3 MB), not for 64^3 (about 1.7 MB)
    srv = szg.Server(0, budget_bytes=fixed + (1 << 20), workers=2)
    try:
        small = [torch.from_numpy(synth.random_field((32, 32, 32), seed=40 + k)).cuda() for k in range(6)]
        big = torch.from_numpy(synth.random_field((64, 64, 64), seed=50)).cuda()
        with pytest.raises(szg.SzError) as ei:
            srv.submit_compress(big, "rel", 1e-3, "cubic")
        assert ei.value.status == szg.ERR_NOMEM
        ts = [srv.submit_compress(x, "rel", 1e-3, "cubic") for x in small]
        peak = 0
        pending = set(ts)
        results = {}
        while pending:
            peak = max(peak, srv.used_bytes())
            for t in list(pending):
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
                    pending.discard(t)
        assert peak <= fixed + (1 << 20)
        ctx = szg.Context(0)
        for x, t in zip(small, ts):
            st, out = results[t]
            assert st == 0
            assert bytes(out.cpu().numpy().tobytes()) == bytes(ctx.compress(x, "rel", 1e-3, "cubic").cpu().numpy().tobytes())
        ctx.close()
        with pytest.raises(szg.SzError) as ei:
            srv.poll(123456789)
        assert ei.value.status == szg.ERR_ARG
    finally:
        srv.close()


def test_server_waits_for_the_callers_stream(szg):
    """A request submitted while torch's stream is still producing its input:
    the server's work waits for that stream on the device, so the stream is
    the one of the finished input."""
    print("[case] server: input produced asynchronously just before submit", flush=True)
    base = torch.from_numpy(synth.lognormal_grf((96, 96, 96), seed=39)).cuda()

    def produce(out):
        out.copy_(base)
        for _ in range(300):  # a queue of kernels still running at submit time
            out.mul_(1.0001)
        return out

    ctx = szg.Context(0)
    ref_in = produce(torch.empty_like(base))
    torch.cuda.synchronize()
    ref = bytes(ctx.compress(ref_in, "rel", 1e-3, "cubic").cpu().numpy().tobytes())
    ctx.close()
    srv = szg.Server(0, budget_bytes=2 << 30, workers=2)
    try:
        for _ in range(3):
            x = produce(torch.empty_like(base))
            t = srv.submit_compress(x, "rel", 1e-3, "cubic")
            st, out = srv.wait(t)
            assert st == 0
            assert bytes(out.cpu().numpy().tobytes()) == ref
    finally:
        srv.close()
