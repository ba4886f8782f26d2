"""Batched compression (sz_compress_batch): every field's stream is
byte-identical to sz_compress of that field alone, and a seeded sample is
byte-identical to the oracle's.

The batch mixes what the shared launches must keep apart: f32 and f64, one to
three dimensions, linear and cubic interpolation, absolute and range-relative
bounds drawn per field, ragged extents (strip kernel with one to four waves,
odd last extents on the fixed-pitch kernel, the compact stride-2 lattice),
and fields the batched path does not take (adaptive, Lorenzo, point-wise
relative, four dimensions, empty), which go through single calls inside the
same batch.  The plan's graph is replayed several times with other GPU work
in between, every replay checked; every tiling the autotuner may pick gives
the same bytes; a field whose buffer is too small reports its size."""
import os

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


@pytest.fixture()
def ctx(szg):
    c = szg.Context(0)
    yield c
    c.close()


def mixed_batch():
    rng = np.random.default_rng(77)
    fields = []
    # (shape, dtype, mode, predictor); the bound is drawn per field
    specs = [
        ((100, 120, 130), np.float32, "rel", "cubic"),    # strip kernel, 2 waves, lattice
        ((64, 70, 514), np.float32, "rel", "cubic"),      # 4 waves, two column windows
        ((33, 47, 21), np.float32, "abs", "linear"),      # odd last extent
        ((40, 36, 60), np.float64, "rel", "cubic"),       # f64 strip kernel
        ((17, 90, 96), np.float64, "abs", "linear"),
        ((181, 362), np.float32, "rel", "cubic"),         # 2-D
        ((5000,), np.float64, "rel", "linear"),           # 1-D
        ((16, 16, 16), np.float32, "rel", "cubic"),
        ((1, 1, 1), np.float32, "abs", "cubic"),          # a single point
        ((96, 17, 50), np.float32, "rel", "linear"),
        ((30, 40, 50), np.float32, "rel", "adaptive"),    # single calls from here
        ((20, 30, 40), np.float32, "abs", "lorenzo"),
        ((24, 25, 26), np.float32, "pwrel", "cubic"),
        ((6, 7, 8, 9), np.float32, "rel", "cubic"),
        ((0, 5, 5), np.float32, "rel", "cubic"),
    ]
    for k, (shape, dt, mode, pred) in enumerate(specs):
        if 0 in shape:
            x = np.zeros(shape, dt)
        else:
            x = synth.random_field(shape, seed=100 + k, dtype=dt)
            if k % 3 == 0:
                x = np.exp(x).astype(dt)  # heavy tails, unpredictable values at R = 512
        if mode == "abs":
            eb = float(10.0 ** rng.uniform(-4, -1)) * float(np.ptp(x) if x.size else 1.0)
        elif mode == "pwrel":
            eb = 1e-2
        else:
            eb = float(10.0 ** rng.uniform(-5, -2))
        fields.append((x, mode, eb, pred))
    return fields


def singles(ctx, tensors, fields, radius=32768, chunk=4096):
    out = []
    for t, (x, mode, eb, pred) in zip(tensors, fields):
        out.append(bytes(ctx.compress(t, mode, eb, pred, radius=radius, chunk=chunk)
                         .cpu().numpy().tobytes()))
    return out


@pytest.mark.parametrize("radius,chunk", [(32768, 4096), (512, 1024)])
def test_batch_equals_single_calls_and_oracle(ctx, orc, radius, chunk):
    fields = mixed_batch()
    tensors = [torch.from_numpy(x).cuda() for x, *_ in fields]
    ref = singles(ctx, tensors, fields, radius, chunk)
    for rep in range(3):
        print(f"[batch] R={radius} C={chunk} replay {rep}", flush=True)
        got = ctx.compress_batch([(t, m, e, p) for t, (_, m, e, p) in zip(tensors, fields)],
                                 radius=radius, chunk=chunk)
        for k, (g, r) in enumerate(zip(got, ref)):
            assert bytes(g.cpu().numpy().tobytes()) == r, f"field {k} differs from its single call"
        # other work on the device between replays
        z = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del z
    # a seeded sample against the oracle (the batched fields)
    omode = {"abs": orc.ABS, "rel": orc.REL}
    opred = {"linear": orc.LINEAR, "cubic": orc.CUBIC}
    for k in (0, 2, 3, 5, 6, 8):
        x, mode, eb, pred = fields[k]
        o = orc.compress(x, omode[mode], eb, opred[pred], radius, chunk)
        assert o == ref[k], f"field {k}: single call differs from the oracle"


@pytest.mark.parametrize("tiling", [0, 1, 2, 3])
def test_every_tiling_writes_the_same_bytes(ctx, tiling, monkeypatch):
    fields = [f for f in mixed_batch()[:10]]
    tensors = [torch.from_numpy(x).cuda() for x, *_ in fields]
    ref = singles(ctx, tensors, fields)
    monkeypatch.setenv("SZG_BATCH_TILING", str(tiling))
    got = ctx.compress_batch([(t, m, e, p) for t, (_, m, e, p) in zip(tensors, fields)])
    for k, (g, r) in enumerate(zip(got, ref)):
        assert bytes(g.cpu().numpy().tobytes()) == r, f"tiling {tiling}: field {k} differs"


def test_batch_without_graph_and_shape_changes(ctx, monkeypatch):
    fields = mixed_batch()[:6]
    tensors = [torch.from_numpy(x).cuda() for x, *_ in fields]
    ref = singles(ctx, tensors, fields)
    monkeypatch.setenv("SZG_BATCH_GRAPH", "0")
    got = ctx.compress_batch([(t, m, e, p) for t, (_, m, e, p) in zip(tensors, fields)])
    assert [bytes(g.cpu().numpy().tobytes()) for g in got] == ref
    monkeypatch.delenv("SZG_BATCH_GRAPH")
    # a different batch (new plan), then the first again (plan rebuilt)
    sub = fields[1:4]
    got = ctx.compress_batch([(t, m, e, p) for t, (_, m, e, p) in zip(tensors[1:4], sub)])
    assert [bytes(g.cpu().numpy().tobytes()) for g in got] == ref[1:4]
    got = ctx.compress_batch([(t, m, e, p) for t, (_, m, e, p) in zip(tensors, fields)])
    assert [bytes(g.cpu().numpy().tobytes()) for g in got] == ref


def test_batch_reports_capacity_per_field(ctx, szg):
    import ctypes

    fields = mixed_batch()[:3]
    tensors = [torch.from_numpy(x).cuda() for x, *_ in fields]
    ref = singles(ctx, tensors, fields)
    L = szg.lib()
    arr = (szg.Field * 3)()
    outs = []
    for i, (t, (x, mode, eb, pred)) in enumerate(zip(tensors, fields)):
        cap = len(ref[i]) if i != 1 else len(ref[i]) - 8
        o = torch.empty(max(cap, 1), dtype=torch.uint8, device="cuda")
        outs.append(o)
        f = arr[i]
        f.d_in = t.data_ptr()
        f.dtype = szg.F32 if x.dtype == np.float32 else szg.F64
        f.ndim = x.ndim
        for d in range(4):
            f.dims[d] = x.shape[d] if d < x.ndim else 1
        f.eb_mode = {"abs": szg.ABS, "rel": szg.REL}[mode]
        f.eb = eb
        f.predictor = {"linear": szg.LINEAR, "cubic": szg.CUBIC}[pred]
        f.d_out = o.data_ptr()
        f.out_capacity = cap
    opts = szg.make_options(32768, 4096, None, 4, 0)
    rc = L.sz_compress_batch(ctx._h, arr, 3, ctypes.byref(opts),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == szg.ERR_CAPACITY
    assert arr[0].status == 0 and arr[2].status == 0
    assert arr[1].status == szg.ERR_CAPACITY and arr[1].out_size == len(ref[1])
    for i in (0, 2):
        assert bytes(outs[i][: arr[i].out_size].cpu().numpy().tobytes()) == ref[i]
