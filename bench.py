"""Throughput of the interpolation compressor hot path on one MI355X.

One step = one sz_compress + one sz_decompress of the 512^3 float32
log-normal field (cubic interpolation, range-relative bound 1e-3, radius
32768): every stage of the path -- bound resolution, multilevel prediction and
quantization, histogram, codebook, encode, decode, reconstruction.  Inputs are
resident in HBM before timing.  Prints one JSON line.

value = input bytes per step / step time (GB/s, 1e9 B/s), the paper's MB/s
convention (original bytes over time) applied to a compress+decompress round
trip; compress-only and decompress-only rates are reported beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


FAMILIES = ("minmax", "interp", "histogram", "codebook", "encode", "other",
            "decode_tables", "chunk_scan", "decode", "recon")


def algorithmic_bytes(n, s_t, stream_bytes, nchunks):
    """Bytes each kernel family must move per step (reads + writes of its
    inputs and outputs, once), n points of s_t bytes, u16 codes."""
    return {
        "minmax": n * s_t,                          # read x
        "interp": n * s_t + 2 * n,                  # read x, write codes
        "histogram": 2 * n,                         # read codes
        "codebook": 0,
        "encode": 2 * n + stream_bytes,             # read codes, write the stream
        "other": 0,
        "decode_tables": 0,
        "chunk_scan": 8 * nchunks,                  # read the chunk table
        "decode": stream_bytes + 2 * n,             # read the stream, write codes
        "recon": 2 * n + n * s_t,                   # read codes, write the field
    }


def measured_traffic(family, shape, args, sub):
    """HBM bytes per step of `family` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's readings), when it was
    taken on this workload and on the kernel sources as they are now."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    doc = json.loads(m.group(1))
    ent = doc.get("families", {}).get(family)
    if not ent or doc.get("workload") != workload_name(shape, args, sub):
        return None
    h = hashlib.sha256()
    for src in ent["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != ent["sources_sha256"]:
        return None  # the kernel changed since the counters were taken
    return ent["hbm_bytes_per_step"]


def workload_name(shape, args, sub):
    return (f"log-normal GRF (P(k)~k^-3) {'x'.join(map(str, shape))} f32, cubic "
            f"interpolation, rel eb {args.rel:g}, radius 32768, chunk {args.chunk}, "
            f"{sub} sub-chunks")


def pwrel_measurement(szg, torch, np, ctx, xt, in_bytes, eps=1e-3, reps=3):
    """The point-wise relative mode on the same field (logarithmic
    preprocessor, the double log field through the same kernels, inverse
    transform), outside the timed region: throughput of compress and of
    decompress, ratio, and the largest point-wise relative error over the
    normal values, which must not exceed eps.  (The CPU-baseline leg adds
    a byte-for-byte comparison with the oracle on a 128^3 corner.)"""
    cap = szg.compress_bound(tuple(xt.shape), szg.F32, eb_mode="pwrel")
    out = torch.empty(cap, dtype=torch.uint8, device=xt.device)
    rec = torch.empty_like(xt)
    s = ctx.compress(xt, "pwrel", eps, "cubic", out=out)
    ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s = ctx.compress(xt, "pwrel", eps, "cubic", out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xd, rd = xt.double(), rec.double()
    normal = torch.isfinite(xd) & (xd.abs() >= float(np.finfo(np.float32).tiny))
    rel = float(((xd - rd).abs() / xd.abs())[normal].max().item())
    del xd, rd
    res = {"eps": eps, "workload": "the same field, point-wise relative bound, cubic",
           "ratio": round(in_bytes / s.numel(), 4),
           "compress_GBps": round(in_bytes * reps / (t1 - t0) / 1e9, 3),
           "decompress_GBps": round(in_bytes * reps / (t2 - t1) / 1e9, 3),
           "max_pointwise_rel_err": rel, "bound_holds": rel <= eps}
    return res


def adaptive_measurement(szg, torch, ctx, xt, in_bytes, rel, chunk, reps=3):
    """Adaptive interpolation on the same field and bound, outside the timed
    region: each level's predictor chosen from the two cost sums, throughput
    of compress (estimation included) and of decompress, ratio, the level
    mask, and the largest error over the bound."""
    cap = szg.compress_bound(tuple(xt.shape), szg.F32, 32768, chunk)
    out = torch.empty(cap, dtype=torch.uint8, device=xt.device)
    rec = torch.empty_like(xt)
    s = ctx.compress(xt, "rel", rel, "adaptive", chunk=chunk, out=out)
    ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s = ctx.compress(xt, "rel", rel, "adaptive", chunk=chunk, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = szg.inspect(s[:128].cpu())
    err = float((xt.double() - rec.double()).abs().max().item())
    return {"workload": "the same field and bound, adaptive linear/cubic per level",
            "ratio": round(in_bytes / s.numel(), 4),
            "level_mask": bin(info["level_mask"]),
            "dim_order": list(info["dim_order"]),
            "compress_GBps": round(in_bytes * reps / (t1 - t0) / 1e9, 3),
            "decompress_GBps": round(in_bytes * reps / (t2 - t1) / 1e9, 3),
            "max_abs_err_over_eb": err / info["eb"] if info["eb"] > 0 else 0.0}


def lorenzo_measurement(szg, torch, ctx, xt, in_bytes, rel, chunk, reps=3):
    """The Lorenzo predictor on the same field and bound, outside the timed
    region: throughput of compress and decompress (wavefronts of blocks),
    ratio, and the largest error over the bound."""
    cap = szg.compress_bound(tuple(xt.shape), szg.F32, 32768, chunk)
    out = torch.empty(cap, dtype=torch.uint8, device=xt.device)
    rec = torch.empty_like(xt)
    s = ctx.compress(xt, "rel", rel, "lorenzo", chunk=chunk, out=out)
    ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s = ctx.compress(xt, "rel", rel, "lorenzo", chunk=chunk, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = szg.inspect(s[:128].cpu())
    err = float((xt.double() - rec.double()).abs().max().item())
    return {"workload": "the same field and bound, first-order Lorenzo predictor",
            "ratio": round(in_bytes / s.numel(), 4),
            "compress_GBps": round(in_bytes * reps / (t1 - t0) / 1e9, 3),
            "decompress_GBps": round(in_bytes * reps / (t2 - t1) / 1e9, 3),
            "max_abs_err_over_eb": err / info["eb"] if info["eb"] > 0 else 0.0}


def lossless_measurement(szg, s, in_bytes, level=1):
    """The host lossless stage (zlib standing in for zstd) on the step's
    stream, outside the timed region: one thread of the host, the stream
    already in host memory.  Checked to restore the stream exactly."""
    host = bytes(s.cpu().numpy().tobytes())
    t0 = time.perf_counter()
    packed = szg.lossless_pack(host, level)
    t1 = time.perf_counter()
    back = szg.lossless_unpack(packed, len(host))
    t2 = time.perf_counter()
    return {"codec": "zlib (stand-in for zstd)", "level": level, "host_threads": 1,
            "stream_bytes": len(host), "packed_bytes": len(packed),
            "ratio_with_stage": round(in_bytes / len(packed), 4),
            "gain": round(len(host) / len(packed), 4),
            "pack_MBps": round(len(host) / (t1 - t0) / 1e6, 1),
            "unpack_MBps": round(len(host) / (t2 - t1) / 1e6, 1),
            "restored": back == host}


def copy_ceiling(torch, xt, reps=5):
    """The practical streaming ceiling of the box: plain device-to-device
    copies of the input, timed with HIP events on the current stream.  Two
    copies: the HIP runtime's (hipMemcpyDtoDAsync) and torch's elementwise
    kernel.  GB/s counts the bytes read plus the bytes written."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyDtoDAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p]
    st = torch.cuda.current_stream()
    nbytes = xt.numel() * xt.element_size()
    dst = torch.empty_like(xt)
    out = {}
    for name in ("hipMemcpyDtoD", "torch_copy"):
        ms = []
        for _ in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            if name == "hipMemcpyDtoD":
                rc = hip.hipMemcpyDtoDAsync(dst.data_ptr(), xt.data_ptr(), nbytes, st.cuda_stream)
                if rc != 0:
                    raise RuntimeError(f"hipMemcpyDtoDAsync failed ({rc})")
            else:
                dst.copy_(xt)
            b.record(st)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        out[name] = round(2 * nbytes / (min(ms[1:]) * 1e-3) / 1e9, 1)
    del dst
    return out


def bound_measurement(szg, torch, ctx, xt, rels, chunk, flush, reps=3):
    """The same field at other range-relative bounds (cubic): event-timed
    compress and decompress (the Infinity Cache flushed before each), the
    ratio, and the streams and reconstructions kept for the oracle check."""
    st = torch.cuda.current_stream()
    in_bytes = xt.numel() * xt.element_size()
    cap = szg.compress_bound(tuple(xt.shape), szg.F32, 32768, chunk)
    out = torch.empty(cap, dtype=torch.uint8, device=xt.device)
    rec = torch.empty_like(xt)
    res = {}
    for rel in rels:
        s = ctx.compress(xt, "rel", rel, "cubic", chunk=chunk, out=out)
        ctx.decompress(s, out=rec)
        mc, md = [], []
        for _ in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            flush()
            e[0].record(st)
            s = ctx.compress(xt, "rel", rel, "cubic", chunk=chunk, out=out)
            e[1].record(st)
            flush()
            e[2].record(st)
            ctx.decompress(s, out=rec)
            e[3].record(st)
            torch.cuda.synchronize()
            mc.append(e[0].elapsed_time(e[1]))
            md.append(e[2].elapsed_time(e[3]))
        mc.sort()
        md.sort()
        res[f"{rel:g}"] = {
            "compress_GBps": round(in_bytes / (mc[len(mc) // 2] * 1e-3) / 1e9, 3),
            "decompress_GBps": round(in_bytes / (md[len(md) // 2] * 1e-3) / 1e9, 3),
            "ratio": round(in_bytes / s.numel(), 4),
            "_stream": bytes(s.cpu().numpy().tobytes()),
            "_rec": rec.cpu().numpy().tobytes(),
        }
    return res


def batch_measurement(szg, torch, np, synth, workers, reps=5):
    """The batching workload (13 x 100x500x500 f32 plus 64 fields of dims
    U{16..96}^3): sz_compress_batch (shared launches, graph replay) against a
    loop of sz_compress calls on one stream and against the request server,
    once with each field's drawn rel eb (log-uniform over 1e-5..1e-2) and once
    with every field at rel 1e-3.  All three must write the same bytes (the
    oracle checks them in the CPU-baseline leg: every field of the drawn
    bounds, a seeded sample at 1e-3).  Times are medians over `reps` runs,
    each preceded by an Infinity Cache flush."""
    flds = synth.batch_fields(seed=4, n_large=13)
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(f).to(dev) for f, _ in flds]
    total = sum(x.numel() * x.element_size() for x in xs)
    npts = [x.numel() for x in xs]
    outs = [torch.empty(szg.compress_bound(tuple(x.shape), szg.F32), dtype=torch.uint8, device=dev)
            for x in xs]
    flush_buf = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    ctx = szg.Context(0)
    srv = szg.Server(0, budget_bytes=64 << 30, workers=workers)
    souts = [torch.empty_like(o) for o in outs]
    rng = np.random.default_rng(12)
    sample = sorted(set([0] + [13 + int(k) for k in rng.choice(64, size=6, replace=False)]))

    def timed(fn):
        ts = []
        for _ in range(reps):
            flush_buf.max()  # evict the cache with clean lines (see `flush` in main)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    res = {"workload": "13 x 100x500x500 + 64 fields of dims U{16..96}^3 f32, offset + scale * "
                       "GRF (slope U[-4,-2], offset and scale log-uniform over 1e-3..1e6), cubic",
           "fields": len(xs), "input_bytes": total, "server_workers": workers}
    for label, ebs in (("drawn_eb", [e for _, e in flds]), ("rel_1e-3", [1e-3] * len(flds))):
        def per_field():
            return [int(ctx.compress(x, "rel", e, "cubic", out=o).numel())
                    for x, o, e in zip(xs, outs, ebs)]

        sizes = per_field()
        torch.cuda.synchronize()
        ref = [bytes(o[:n].cpu().numpy().tobytes()) for o, n in zip(outs, sizes)]
        call = ctx.prepare_batch([(x, "rel", e, "cubic") for x, e in zip(xs, ebs)])
        t_first = time.perf_counter()
        got = call.run()  # builds the plan, tunes the tiles, captures the graph
        t_first = time.perf_counter() - t_first
        same_batch = all(bytes(g.cpu().numpy().tobytes()) == r for g, r in zip(got, ref))
        del got

        def served():
            ts = [srv.submit_compress(x, "rel", e, "cubic", out=o) for x, o, e in zip(xs, souts, ebs)]
            return [srv.wait(t) for t in ts]

        sres = served()
        same_server = all(st == 0 and bytes(v.cpu().numpy().tobytes()) == r
                          for (st, v), r in zip(sres, ref))
        t_b = timed(call.run)
        t_pf = timed(per_field)
        t_sv = timed(served)
        stream_bytes = sum(len(r) for r in ref)
        # compress: read x twice (range, then prediction), write and read the
        # u16 codes, write the stream
        alg = sum(n * 4 * 2 + 4 * n for n in npts) + stream_bytes
        res[label] = {
            "batched_GBps": round(total / t_b / 1e9, 2), "batched_ms": round(t_b * 1e3, 3),
            "per_field_GBps": round(total / t_pf / 1e9, 2), "per_field_ms": round(t_pf * 1e3, 3),
            "server_GBps": round(total / t_sv / 1e9, 2), "server_ms": round(t_sv * 1e3, 3),
            "batched_over_per_field": round(t_pf / t_b, 2),
            "batched_alg_bytes": alg, "batched_alg_GBps": round(alg / t_b / 1e9, 1),
            "batched_frac": round(alg / t_b / 1e9 / HBM_PEAK_GBPS, 4),
            "ratio": round(total / stream_bytes, 3),
            "first_call_ms": round(t_first * 1e3, 1),
            "batch_identical_to_per_field": same_batch,
            "server_identical_to_per_field": same_server,
            "_streams": ref if label == "drawn_eb" else {k: ref[k] for k in sample},
            "_ebs": ebs,
        }
    srv.close()
    ctx.close()
    res["_fields"] = [f for f, _ in flds]
    res["_sample"] = sample
    return res


def serving_measurement(szg, torch, np, synth, workers, n_req, budget=200 << 30, window=32,
                        loads=(0.5, 0.8, 1.2), n_sample=100):
    """The serving workload: ``n_req`` compression requests (synth.serving_requests:
    sizes log-uniform over 16^3..256x512x512 points, random aspect ratios,
    slopes U[-4,-2], rel eb log-uniform over 1e-5..1e-2), each a crop of a
    device-resident base field, served by the request server under an HBM
    budget.

    1. saturated rate: a closed loop keeping ``window`` requests outstanding;
    2. at each offered load, Poisson arrivals at load x the saturated rate;
       a request's latency runs from its scheduled arrival to the client's
       observation that it is done (the client polls the oldest 64
       outstanding tickets between arrivals; the server starts requests in
       arrival order, so later ones cannot be done first unless those are);
    3. every request is served again in a mix (closed loop) and compared on
       the device with the same request compressed alone; a seeded sample
       keeps its bytes for the oracle (CPU-baseline leg)."""
    pool = synth.serving_pool(seed=5)
    reqs = synth.serving_requests(n_req, seed=6)
    dev = torch.device("cuda:0")
    bases = [torch.from_numpy(f).to(dev) for f, _ in pool]
    srv = szg.Server(0, budget_bytes=budget, workers=workers)
    caps = [szg.compress_bound(r["shape"], szg.F32) for r in reqs]
    nbytes = [4 * int(np.prod(r["shape"])) for r in reqs]
    total = sum(nbytes)

    def crop(k):
        r = reqs[k]
        (a, b, c), (na, nb, nc) = r["origin"], r["shape"]
        return bases[r["base"]][a:a + na, b:b + nb, c:c + nc].contiguous()

    def issue(k):
        out = torch.empty(caps[k], dtype=torch.uint8, device=dev)
        return srv.submit_compress(crop(k), "rel", reqs[k]["rel_eb"], "cubic", out=out)

    def sweep(outstanding, on_done, limit=64):
        done = []
        for t in list(outstanding)[:limit]:
            res = srv.poll(t)
            if res is not None:
                done.append((t, res))
        for t, res in done:
            on_done(outstanding.pop(t), res)

    # 1. saturated rate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outstanding, nxt = {}, 0
    while nxt < n_req or outstanding:
        while nxt < n_req and len(outstanding) < window:
            outstanding[issue(nxt)] = nxt
            nxt += 1
        sweep(outstanding, lambda k, res: None)
    t_sat = time.perf_counter() - t0
    sat_rate = n_req / t_sat
    res = {"workload": f"{n_req} compression requests, 3-D f32 crops of {len(pool)} base GRFs "
                       "of 256x512x512 (slopes -4..-2), sizes log-uniform 16^3..256x512x512, "
                       "random aspect ratios, rel eb log-uniform 1e-5..1e-2, cubic",
           "requests": n_req, "input_bytes": total, "budget_bytes": budget, "workers": workers,
           "saturated": {"req_per_s": round(sat_rate, 1), "GBps": round(total / t_sat / 1e9, 2),
                         "window": window, "seconds": round(t_sat, 3)}}
    # 2. Poisson arrivals at each offered load
    rng = np.random.default_rng(7)
    for load in loads:
        lam = load * sat_rate
        arr = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
        lat = np.zeros(n_req)
        last = [0.0]
        outstanding, i = {}, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def on_done(k, r):
            now = time.perf_counter() - t0
            lat[k] = now - arr[k]
            last[0] = now
            if r[0] != 0:
                raise RuntimeError(f"request {k} failed with status {r[0]}")

        while i < n_req or outstanding:
            now = time.perf_counter() - t0
            while i < n_req and arr[i] <= now:
                outstanding[issue(i)] = i
                i += 1
            sweep(outstanding, on_done)
        span = last[0] - arr[0]
        res[f"load_{load:g}"] = {
            "offered_req_per_s": round(lam, 1),
            "achieved_GBps": round(total / span / 1e9, 2),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3),
        }
    # 3. in a mix (closed loop) against alone, every request
    ctx = szg.Context(0)
    sample = sorted(int(k) for k in np.random.default_rng(8).choice(n_req, size=min(n_sample, n_req),
                                                                    replace=False))
    keep = {}
    bad = []

    def check(k, r):
        alone = ctx.compress(crop(k), "rel", reqs[k]["rel_eb"], "cubic")
        if r[0] != 0 or r[1].numel() != alone.numel() or not torch.equal(r[1], alone):
            bad.append(k)
        if k in sample_set:
            keep[k] = bytes(r[1].cpu().numpy().tobytes())

    sample_set = set(sample)
    outstanding, nxt = {}, 0
    while nxt < n_req or outstanding:
        while nxt < n_req and len(outstanding) < window:
            outstanding[issue(nxt)] = nxt
            nxt += 1
        sweep(outstanding, check)
    srv.close()
    ctx.close()
    res["alone_equals_in_mix"] = {"requests": n_req, "mismatches": len(bad)}
    res["_sample"] = keep
    res["_reqs"] = reqs
    res["_pool"] = [f for f, _ in pool]
    return res


def serving_oracle_leg(orc, serving, threads):
    """The oracle on a seeded sample of the serving requests (host crops of
    the same base fields), byte for byte against the served streams."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    reqs, pool, sample = serving["_reqs"], serving["_pool"], serving["_sample"]

    def one(k):
        r = reqs[k]
        (a, b, c), (na, nb, nc) = r["origin"], r["shape"]
        x = np.ascontiguousarray(pool[r["base"]][a:a + na, b:b + nb, c:c + nc])
        return orc.compress(x, orc.REL, r["rel_eb"], orc.CUBIC) == sample[k]

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        ok = list(ex.map(one, sorted(sample)))
    serving["parity_with_oracle_sample"] = {"requests": len(ok), "identical": all(ok),
                                            "seconds": round(time.perf_counter() - t0, 2)}


def strip_private(d):
    """The object without its private (underscore) entries, recursively."""
    if not isinstance(d, dict):
        return d
    return {k: strip_private(v) for k, v in d.items() if not k.startswith("_")}


def batch_oracle_leg(orc, batched, threads):
    """The oracle on the batching workload: every field at its drawn bound,
    one field per thread (the oracle is reentrant C; ctypes releases the
    interpreter lock) across `threads` host threads, checked byte for byte
    against the GPU's streams, timed as the CPU baseline of that workload; and
    the seeded sample at rel 1e-3."""
    from concurrent.futures import ThreadPoolExecutor

    fields = batched["_fields"]
    d = batched["drawn_eb"]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        streams = list(ex.map(lambda k: orc.compress(fields[k], orc.REL, d["_ebs"][k], orc.CUBIC),
                              range(len(fields))))
    wall = time.perf_counter() - t0
    d["parity_with_oracle_all_fields"] = all(a == b for a, b in zip(streams, d["_streams"]))
    e = batched["rel_1e-3"]
    e["parity_with_oracle_sample"] = all(
        orc.compress(fields[k], orc.REL, 1e-3, orc.CUBIC) == v for k, v in e["_streams"].items())
    e["oracle_sample_fields"] = batched["_sample"]
    batched["cpu_baseline"] = {
        "value": round(batched["input_bytes"] / wall / 1e9, 4), "unit": "GB/s (compress)",
        "cores": threads, "kind": "oracle",
        "sample": f"all {len(fields)} fields at their drawn bounds, compress only, one field per "
                  f"thread on {threads} host threads ({wall:.1f}s wall)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shape", default="512,512,512")
    ap.add_argument("--rel", type=float, default=1e-3)
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--subchunks", type=int, default=0,
                    help="runs per chunk decoded by separate lanes (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched vs per-field measurement")
    ap.add_argument("--batch-workers", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving measurement (Poisson arrivals, p50/p99)")
    ap.add_argument("--serving-requests", type=int, default=10000)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the lossless, point-wise relative and adaptive measurements "
                         "(for profiler runs that count the step's kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy the input once on the device "
                         "(a plain copy of known size, to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the path shards as independent fields with no exchange, see DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2111_02925_amd as szg
    import synth

    shape = tuple(int(v) for v in args.shape.split(","))
    t0 = time.time()
    x = synth.lognormal_grf(shape, seed=2)
    print(f"[bench] generated {shape} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    n = x.size
    in_bytes = x.nbytes
    dev = torch.device("cuda:0")
    ctx = szg.Context(0)
    xt = torch.from_numpy(x).to(dev)
    cap = szg.compress_bound(shape, szg.F32, 32768, args.chunk, subchunks=args.subchunks)
    out = torch.empty(cap, dtype=torch.uint8, device=dev)
    rec = torch.empty(shape, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream(dev)

    def step():
        s = ctx.compress(xt, "rel", args.rel, "cubic", chunk=args.chunk,
                         subchunks=args.subchunks, out=out)
        ctx.decompress(s, out=rec)
        return s

    for _ in range(args.warmup):
        s = step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    # Infinity Cache flush between the phases, so that no phase reads what the
    # previous one left in the 256 MB cache (the stream the compression just
    # wrote, in particular): a read of 512 MiB, which leaves the cache holding
    # clean lines (a write would leave 256 MB of dirty lines for the next
    # phase to write back inside its timed region)
    flush_buf = torch.empty(1 << 29, dtype=torch.uint8, device=dev)

    def flush():
        flush_buf.max()

    # per-family breakdown (HIP events around every family), outside the
    # timed region (the events cost about a tenth of a step), flushed like it
    ctx.timing_reset()
    ctx.set_timing(True)
    ctx.set_timing_family(None)
    for _ in range(args.steps):
        flush()
        s = ctx.compress(xt, "rel", args.rel, "cubic", chunk=args.chunk,
                         subchunks=args.subchunks, out=out)
        flush()
        ctx.decompress(s, out=rec)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    fam = {k: ctx.timing(k) for k in FAMILIES}
    per_step = {k: (v[0] / args.steps, v[1] / args.steps) for k, v in fam.items()}
    dom = max(per_step, key=lambda k: per_step[k][0])

    # timed region: every step's compress and decompress between HIP events,
    # the cache flushed before each (outside the events); HIP events around
    # the dominant family as well
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(4))
          for _ in range(args.steps)]
    ctx.timing_reset()
    ctx.set_timing(True)
    ctx.set_timing_family(dom)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        flush()
        ev[i][0].record(st)
        s = ctx.compress(xt, "rel", args.rel, "cubic", chunk=args.chunk,
                         subchunks=args.subchunks, out=out)
        ev[i][1].record(st)
        flush()
        ev[i][2].record(st)
        ctx.decompress(s, out=rec)
        ev[i][3].record(st)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ctx.set_timing(False)
    dom_ms_live, dom_regions = ctx.timing(dom)
    ctx.set_timing_family(None)
    comp = [a.elapsed_time(b) for a, b, _, _ in ev]
    decomp = [c.elapsed_time(d) for _, _, c, d in ev]
    ms_c = float(np.median(comp))
    ms_d = float(np.median(decomp))
    # a step: one compress and one decompress, the flushes between them left out
    ms_step = float(np.mean([a + b for a, b in zip(comp, decomp)]))
    wall_ms_step = t_total * 1e3 / args.steps
    size = int(s.numel())

    # quality (measurement only, after the timed region)
    diff = (rec.double() - xt.double()).abs()
    vr = float(xt.max() - xt.min())
    mse = float((diff * diff).mean())
    psnr = 20 * np.log10(vr) - 10 * np.log10(mse) if mse > 0 else float("inf")
    info = szg.inspect(s[:128].cpu())
    maxerr_over_eb = float(diff.max()) / info["eb"] if info["eb"] > 0 else 0.0

    if args.copy_calibration:
        # plain device-to-device copies of the input (known size): the HIP
        # runtime's copy kernel, then torch's elementwise copy
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        calib = torch.empty_like(xt)
        torch.cuda.synchronize()
        rc = hip.hipMemcpyDtoD(ctypes.c_void_p(calib.data_ptr()), ctypes.c_void_p(xt.data_ptr()),
                               ctypes.c_size_t(in_bytes))
        if rc != 0:
            raise RuntimeError(f"hipMemcpyDtoD failed ({rc})")
        calib.copy_(xt)
        torch.cuda.synchronize()
        del calib

    # roofline of the dominant kernel family (largest time per step), from
    # its events in the timed region; the algorithmic bytes of each family
    alg = algorithmic_bytes(n, 4, size, -(-n // args.chunk))
    dom_ms = dom_ms_live / args.steps
    achieved = alg[dom] / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": measured_traffic(dom, shape, args, info["sub"]),
                "timed_regions_per_step": dom_regions / args.steps,
                "ms_per_step": round(dom_ms, 4),
                "alg_bytes_per_step": alg[dom]}

    # the whole step's algorithmic bytes: compression reads the field twice
    # (range, then prediction), writes and reads the codes, writes the
    # stream; decompression reads the stream, writes and reads the codes,
    # writes the field
    b_c = 2 * n * 4 + 4 * n + size
    b_d = size + 4 * n + n * 4
    step_alg = {"compress_bytes": b_c, "decompress_bytes": b_d,
                "GBps": round((b_c + b_d) / (ms_step * 1e-3) / 1e9, 1),
                "frac": round((b_c + b_d) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "compress_frac": round(b_c / (ms_c * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "decompress_frac": round(b_d / (ms_d * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    copy = copy_ceiling(torch, xt)
    bounds = None if args.no_extras else bound_measurement(
        szg, torch, ctx, xt, [1e-2, 1e-4], args.chunk, flush)

    batched = None if args.no_batch else batch_measurement(szg, torch, np, synth,
                                                           args.batch_workers)
    serving = None if args.no_serving else serving_measurement(
        szg, torch, np, synth, args.batch_workers, args.serving_requests)
    lossless = pwrel = adaptive = lorenzo = None
    if not args.no_extras:
        lossless = lossless_measurement(szg, s, in_bytes)
        pwrel = pwrel_measurement(szg, torch, np, ctx, xt, in_bytes)
        adaptive = adaptive_measurement(szg, torch, ctx, xt, in_bytes, args.rel, args.chunk)
        lorenzo = lorenzo_measurement(szg, torch, ctx, xt, in_bytes, args.rel, args.chunk)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t1 = time.perf_counter()
        ref = oracle.compress(x, oracle.REL, args.rel, oracle.CUBIC, 32768, args.chunk,
                              sub=info["sub"])
        t2 = time.perf_counter()
        back = oracle.decompress(ref)
        t3 = time.perf_counter()
        parity = (ref == bytes(s.cpu().numpy().tobytes())) and (
            back.tobytes() == rec.cpu().numpy().tobytes())
        # the other bounds of the same field, byte for byte (streams and
        # reconstructions kept from their GPU runs)
        if batched is not None:
            batch_oracle_leg(oracle, batched, min(16, os.cpu_count() or 1))
        if serving is not None:
            serving_oracle_leg(oracle, serving, min(16, os.cpu_count() or 1))
        if bounds is not None:
            for key, b in bounds.items():
                bref = oracle.compress(x, oracle.REL, float(key), oracle.CUBIC, 32768, args.chunk,
                                       sub=info["sub"])
                b["parity_with_oracle"] = (bref == b["_stream"]) and (
                    oracle.decompress(bref).tobytes() == b["_rec"])
        # the point-wise relative and adaptive modes on a 128^3 corner, byte for byte
        corner = np.ascontiguousarray(x[:128, :128, :128])
        if pwrel is not None:
            pref = oracle.compress(corner, oracle.PWREL, pwrel["eps"], oracle.CUBIC)
            sc = ctx.compress(torch.from_numpy(corner).to(dev), "pwrel", pwrel["eps"], "cubic")
            pback = ctx.decompress(sc)
            pwrel["parity_with_oracle_128cubed"] = (
                bytes(sc.cpu().numpy().tobytes()) == pref
                and pback.cpu().numpy().tobytes() == oracle.decompress(pref).tobytes())
        if lorenzo is not None:
            lref = oracle.compress(corner, oracle.REL, args.rel, oracle.LORENZO, 32768, args.chunk)
            sl = ctx.compress(torch.from_numpy(corner).to(dev), "rel", args.rel, "lorenzo",
                              chunk=args.chunk)
            lback = ctx.decompress(sl)
            lorenzo["parity_with_oracle_128cubed"] = (
                bytes(sl.cpu().numpy().tobytes()) == lref
                and lback.cpu().numpy().tobytes() == oracle.decompress(lref).tobytes())
        if adaptive is not None:
            aref = oracle.compress(corner, oracle.REL, args.rel, oracle.ADAPTIVE, 32768, args.chunk)
            sa = ctx.compress(torch.from_numpy(corner).to(dev), "rel", args.rel, "adaptive",
                              chunk=args.chunk)
            aback = ctx.decompress(sa)
            adaptive["parity_with_oracle_128cubed"] = (
                bytes(sa.cpu().numpy().tobytes()) == aref
                and aback.cpu().numpy().tobytes() == oracle.decompress(aref).tobytes())
        cpu = {"value": round(in_bytes / (t3 - t1) / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full {shape} field: one compress ({t2 - t1:.1f}s) + one "
                         f"decompress ({t3 - t2:.1f}s), single thread, host "
                         f"{os.cpu_count()} logical CPUs"}

    res = {
        "metric": "compress/decompress GB/s at rel eb 1e-3 (ratio fixed), % HBM roofline; batched vs per-field",
        "value": round(in_bytes / (ms_step * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_name(shape, args, info["sub"]),
                   "shape": list(shape), "eb_mode": "rel", "eb": args.rel, "predictor": "cubic"},
        "compress_GBps": round(in_bytes / (ms_c * 1e-3) / 1e9, 3),
        "decompress_GBps": round(in_bytes / (ms_d * 1e-3) / 1e9, 3),
        "compress_ms": round(ms_c, 4),
        "decompress_ms": round(ms_d, 4),
        "ratio": round(in_bytes / size, 4),
        "bit_rate": round(32.0 * size / in_bytes, 4),
        "psnr_db": round(psnr, 3),
        "max_err_over_eb": round(maxerr_over_eb, 6),
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in per_step.items()},
        "kernel_ms_note": "per family, from a separate run of the same steps with events around every family",
        "roofline": roofline,
        "step_algorithmic": step_alg,
        "copy_GBps": copy,
        "timing_note": "ms_per_step and the compress/decompress rates are event-timed per phase "
                       "with a 512 MiB Infinity Cache flush (a read) before each phase, outside the events; "
                       "wall_ms_per_step includes the flushes",
        "wall_ms_per_step": round(wall_ms_step, 4),
        "bounds": None if bounds is None else {
            k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")} for k, v in bounds.items()},
        "cpu_baseline": cpu,
        "batched": strip_private(batched),
        "serving": strip_private(serving),
        "lossless": lossless,
        "pwrel": pwrel,
        "adaptive": adaptive,
        "lorenzo": lorenzo,
        "parity_with_oracle": parity,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
