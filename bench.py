#!/usr/bin/env python3
"""Throughput of the chunk codec hot path on one MI355X.

Workload: 1080p chunks of T = 8 frames (1920x1080, padded to 1088 inside the
codec), C = 128 latent channels, synthetic textured video (4 distinct seeded
chunks cycled so the 199 MB input of a step is not cache resident), inputs
resident in HBM.  One step = encode one chunk to a bit-stream (exact length
read back to the host) + decode that bit-stream to T frames.

Prints one JSON line: BF16 encode+decode frames/s (the headline), the FP32
plain path on the same GPU, the BF16-vs-FP32 PSNR delta, per-step latency
p50/p99, the dominant kernel against its roofline (average launch duration
from HIP events recorded by the library around each launch, on the stream
the kernel runs on, during the timed region), and the CPU oracle timed on
this host as a baseline.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "1080p frames/s enc+dec, BF16 vs FP32 at <=0.05 dB PSNR delta; p99 latency"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}

# HBM bytes per launch of the two largest convs at 1080p, T = 8, C = 128 (a1,
# the patchify-fused analysis conv, and k3, the frame heads with the
# pixel-shuffle store), from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
# script, each scaled by the same counter's reading for plain 256 MiB device
# copies in the same run, per tile configuration index.  They hold only for
# the conv sources they were taken with: bench reports them while the SHA-256
# of ufvc_conv.hip followed by ufvc_common.h still matches, and null otherwise.
TRAFFIC_SHA256 = "a8980a151be0ef47c99be958c8be53f52f8443a650c624de9fd941f1477e416b"
TRAFFIC = {  # (stage, tile configuration): (read bytes, write bytes)
    ("a1_conv", 31): (251.15e6, 8.36e6),
    ("a1_conv", 32): (251.12e6, 8.36e6),
    ("k3_conv", 12): (103.35e6, 199.07e6),
    ("k3_conv", 13): (115.67e6, 199.07e6),
    ("k3_conv", 15): (116.07e6, 199.07e6),
    ("k3_conv", 16): (102.59e6, 199.07e6),
    ("k3_conv", 17): (102.39e6, 199.07e6),
    ("k3_conv", 18): (115.12e6, 199.07e6),
    ("k3_conv", 19): (103.49e6, 199.07e6),
    ("k3_conv", 25): (82.98e6, 199.1e6),
    ("k3_conv", 26): (74.58e6, 199.07e6),
    ("k3_conv", 27): (115.15e6, 199.07e6),
    ("k3_conv", 28): (103.25e6, 199.07e6),
    ("k3_conv", 29): (84.16e6, 199.11e6),
    ("k3_conv", 30): (72.97e6, 199.07e6),
    ("k3_conv", 33): (102.4e6, 199.07e6),
    ("k3_conv", 34): (76.81e6, 199.07e6),
    ("k3_conv", 35): (102.98e6, 199.07e6),
    ("k3_conv", 36): (78.94e6, 199.27e6),
}


def conv_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2606_04410_amd", "csrc")
    for name in ("ufvc_conv.hip", "ufvc_common.h"):
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def conv_flops(T, C, h, w):
    """Algorithmic FLOPs (2 per MAC) of every conv stage for one chunk."""
    npos = h * w
    hz, wz = (h + 1) // 2, (w + 1) // 2
    f = lambda cin, cout, pos: 2.0 * 9 * cin * cout * pos  # noqa: E731
    return {
        "a1_conv": f(192 * T, C, npos), "a2_conv": f(C, C, npos), "a3_conv": f(C, C, npos),
        "hyper_conv": f(C, 32, hz * wz), "params_conv_enc": f(32, 2 * C, npos),
        "params_conv_dec": f(32, 2 * C, npos), "d1_conv": f(C, C, npos), "d2_conv": f(C, C, npos),
        "d3_conv": f(C, C, npos), "k1_conv": f(C, T * C, npos), "k2_conv": T * f(C, C, npos),
        "k3_conv": T * f(C, 192, npos),
    }


def mean_step_flops(C, h, w):
    """Algorithmic FLOPs of the three quadtree mean steps of one side: step k
    gives C / 4 outputs per position from the k earlier partitions (k C / 4
    input channels per tap)."""
    return sum(2.0 * h * w * (C // 4) * 9 * k * (C // 4) for k in (1, 2, 3))


def a1_algorithmic_bytes(T, C, H, W, h, w):
    """Bytes a1 must move once: the float32 frames and its bf16 weights read,
    its bf16 activation written."""
    return T * 3 * H * W * 4 + 9 * (T * 192) * C * 2 + h * w * C * 2


def k3_algorithmic_bytes(T, C, H, W, h, w):
    """Bytes the frame heads' last conv must move once: k2's bf16 activation
    and the bf16 weights read, the float32 frames written."""
    return h * w * T * C * 2 + 9 * C * 192 * T * 2 + T * 3 * H * W * 4


def stage_bytes(h, w, C, r):
    """Algorithmic HBM bytes of the entropy-coding stages for one chunk."""
    ny = h * w * C
    nz = ((h + 1) // 2) * ((w + 1) // 2) * 32
    stream_bytes = r["bytes"]
    return {
        # symbol + index read, stream words written
        "rans_encode": 2.0 * ny + nz + r["y_bytes"] + r["z_bytes"],
        # stream read, index read, symbol written
        "rans_decode_y": r["y_bytes"] + 2.0 * ny,
        # stream read, symbol written
        "rans_decode_z": r["z_bytes"] + 1.0 * nz,
        # scale logit + mean + y read (4 B each), index + symbol written
        "params_epilogue_enc": 14.0 * ny,
        # scale logit read, index written
        "params_epilogue_dec": 5.0 * ny,
        # slots read, container written
        "compact": 2.0 * stream_bytes,
    }


def run_codec(torch, ufvc, weights, prec, chunks, H, W, steps, warmup, seg_log2, seg_log2_z,
              profile, autotune=True):
    T = chunks[0].shape[0]
    c = ufvc.Codec(T, 128, weights, precision=prec, seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                   model_tag=0x0800_1080, autotune=autotune)
    cap = c.max_bitstream_bytes(H, W)
    bufs = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in chunks]
    out = torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    lens = [0] * len(chunks)

    def step(i):
        k = i % len(chunks)
        _, n = c.encode(chunks[k], out=bufs[k], stream=stream)
        lens[k] = n
        c.decode(bufs[k], n, H, W, out=out, stream=stream, check=False)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if c.status(stream) != 0:
        raise RuntimeError("decode reported an error during warm-up")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        step(i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if c.status(stream) != 0:
        raise RuntimeError("decode reported an error in the timed region")
    # per-stage kernel times: the same steps again with the library's HIP
    # events around every launch (about 5 us per stage of their own, so they
    # stay out of the timed run above)
    stages = {}
    if profile:
        c.profile(True)
        for i in range(steps):
            step(i)
        torch.cuda.synchronize()
        stages = c.profile_read()
        c.profile(False)
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    # reconstruction of chunk 0 for the PSNR comparison
    _, n0 = c.encode(chunks[0], out=bufs[0], stream=stream)
    rec = c.decode(bufs[0], n0, H, W, stream=stream).clone()
    freq, _, _ = c.tables()
    sym = c.buffer(ufvc.BUF_SYM, H, W).reshape(-1)
    idx = c.buffer(ufvc.BUF_IDX, H, W).reshape(-1)
    zs = c.buffer(ufvc.BUF_ZSYM, H, W).reshape(-1)
    f = freq.astype(np.float64)
    ideal = float(np.sum(16 - np.log2(f[idx, sym])) + np.sum(16 - np.log2(f[22, zs])))
    tuning = c.tuning(H, W)
    head = bufs[0][:28].cpu().numpy()
    n_seg_z, n_seg_y = (int(v) for v in head[20:28].view("<u4"))
    table = bufs[0][28:28 + 4 * (n_seg_z + n_seg_y)].cpu().numpy().view("<u4")
    c.close()
    return dict(seconds=t1 - t0, lat=lat, stages=stages, rec=rec, bytes=n0, ideal_bits=ideal,
                n_sym=int(sym.size + zs.size), tuning=tuning, z_bytes=int(table[:n_seg_z].sum()),
                y_bytes=int(table[n_seg_z:].sum()))


def run_pipelined(torch, ufvc, weights, prec, chunks, H, W, steps, warmup, seg_log2, seg_log2_z,
                  lanes=2):
    """The same step (encode one chunk, then decode its stream) with `lanes`
    chunks in flight: one codec context, HIP stream and host thread per lane,
    so one chunk's latency-bound entropy coding overlaps another's convs."""
    import threading
    T = chunks[0].shape[0]
    codecs = [ufvc.Codec(T, 128, weights, precision=prec, seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                         model_tag=0x0800_1080, autotune=True) for _ in range(lanes)]
    streams = [torch.cuda.Stream() for _ in range(lanes)]
    cap = codecs[0].max_bitstream_bytes(H, W)
    bufs = [[torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in chunks] for _ in range(lanes)]
    outs = [torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda") for _ in range(lanes)]
    per = steps // lanes
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(per)] for _ in range(lanes)]

    def lane(li, n, timed):
        c, st = codecs[li], streams[li]
        for i in range(n):
            k = (li + i * lanes) % len(chunks)
            if timed:
                ev[li][i][0].record(st)
            _, nb = c.encode(chunks[k], out=bufs[li][k], stream=st)
            c.decode(bufs[li][k], nb, H, W, out=outs[li], stream=st, check=False)
            if timed:
                ev[li][i][1].record(st)

    def run(n, timed):
        ths = [threading.Thread(target=lane, args=(li, n, timed)) for li in range(lanes)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()

    run(max(1, warmup), False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(per, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for li, c in enumerate(codecs):
        if c.status(streams[li]) != 0:
            raise RuntimeError("decode reported an error in the pipelined run")
    lat = np.array([a.elapsed_time(b) for lv in ev for a, b in lv])
    for c in codecs:
        c.close()
    return dict(seconds=t1 - t0, steps=per * lanes, lat=lat)


C3_MIX = [(16, 832, 480), (16, 1280, 720), (12, 1920, 1088), (4, 3840, 2160)]


def run_batch_c3(torch, ufvc, steps, seg_log2, seg_log2_z):
    """48 uneven chunks (T drawn from {4, 8}) encoded and decoded as one batch:
    one launch per stage and tile configuration, decode replayed from a graph."""
    from synthetic import stand_in_weights, video_chunk
    C = 128
    rng = np.random.default_rng(2)
    spec = []
    for count, W, H in C3_MIX:
        for _ in range(count):
            spec.append((int(rng.choice([4, 8])), H, W))
    models = {T: ufvc.Codec(T, C, stand_in_weights(T, C), precision="bf16", seg_log2=seg_log2,
                            seg_log2_z=seg_log2_z, model_tag=0x0C30_0000 + T, autotune=True)
              for T in (4, 8)}
    midx = {4: 0, 8: 1}
    batch = ufvc.Batch([models[4], models[8]])
    cache = {}
    frames = []
    for i, (T, H, W) in enumerate(spec):
        key = (T, H, W, i % 2)
        if key not in cache:
            cache[key] = torch.from_numpy(video_chunk(T, H, W, 16, seed=3, chunk_id=len(cache))).cuda()
        frames.append(cache[key])
    outs = [torch.empty(models[T].max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
            for (T, H, W) in spec]
    recs = [torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda") for (T, H, W) in spec]
    enc_items = [(midx[T], fr, o) for (T, H, W), fr, o in zip(spec, frames, outs)]
    lens = batch.encode(enc_items)                      # plans, tunes buckets
    dec_items = [(midx[T], o, n, H, W, r) for (T, H, W), o, n, r in zip(spec, outs, lens, recs)]
    batch.decode(dec_items, graph=False)
    st, code = batch.decode(dec_items, graph=True)      # captures the graph
    if code != 0:
        raise RuntimeError(f"batch decode status {st}")
    torch.cuda.synchronize()
    frames_total = sum(T for T, _, _ in spec)
    per_policy = {}
    for policy in (0, 1):
        batch.set_policy(policy)
        batch.encode(enc_items)                          # plans for this policy
        batch.decode(dec_items, graph=True)
        torch.cuda.synchronize()
        te = td = 0.0
        for _ in range(steps):
            t0 = time.perf_counter()
            lens = batch.encode(enc_items)
            t1 = time.perf_counter()
            batch.decode(dec_items, graph=True, check=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            te += t1 - t0
            td += t2 - t1
        st, code = batch.sync_status()
        if code != 0:
            raise RuntimeError(f"batch decode status {st}")
        bst = batch.stats()
        per_policy[policy] = {"value": round(frames_total * steps / (te + td), 2),
                              "enc_ms_per_batch": round(1e3 * te / steps, 3),
                              "dec_ms_per_batch": round(1e3 * td / steps, 3),
                              "conv_stages": int(bst["conv_stages"]),
                              "conv_launches": int(bst["conv_launches"])}
    best = max(per_policy, key=lambda k: per_policy[k]["value"])
    te = per_policy[best]["enc_ms_per_batch"] * steps / 1e3
    td = per_policy[best]["dec_ms_per_batch"] * steps / 1e3
    tuning = {f"{W}x{H}": {f"T{T}": models[T].tuning(H, W)["k1"] for T in (4, 8)}
              for _, W, H in C3_MIX}
    res = {"chunks": len(spec), "frames_per_batch": frames_total,
           "value": round(frames_total * steps / (te + td), 2), "unit": "frames/s",
           "enc_ms_per_batch": round(1e3 * te / steps, 3),
           "dec_ms_per_batch": round(1e3 * td / steps, 3), "steps": steps,
           "decode": "hipGraph replay", "k1_tile_per_bucket": tuning,
           "launch_policy": {"chosen": "one launch per stage" if best == 1 else
                             "one launch per tile configuration",
                             "per_tile_configuration": per_policy[0], "one_per_stage": per_policy[1]},
           "mix": "16x832x480, 16x1280x720, 12x1920x1088, 4x3840x2160; T from {4,8} (seed 2)"}
    batch.close()
    for m in models.values():
        m.close()
    return res


def run_quadtree(torch, ufvc, chunks, H, W, steps, warmup, seg_log2, seg_log2_z, lanes,
                 autotune=True):
    """The quadtree model (four-step progressive means): the headline's
    workload and step, one chunk at a time (with the mean steps' HIP-event
    times) and with `lanes` chunks in flight."""
    from synthetic import stand_in_weights
    T, C = chunks[0].shape[0], 128
    wq = stand_in_weights(T, C, quadtree=True)
    r = run_codec(torch, ufvc, wq, "bf16", chunks, H, W, steps, warmup, seg_log2, seg_log2_z,
                  profile=True, autotune=autotune)
    rp = run_pipelined(torch, ufvc, wq, "bf16", chunks, H, W, steps, warmup, seg_log2,
                       seg_log2_z, lanes=lanes)
    h, w = -(-H // 16) * 2, -(-W // 16) * 2
    fl = mean_step_flops(C, h, w)
    st = r["stages"]
    out = {"value": round(T * rp["steps"] / rp["seconds"], 2), "unit": "frames/s",
           "chunks_in_flight": lanes,
           "sequential": round(T * steps / r["seconds"], 2),
           "latency_ms_p99": round(float(np.percentile(rp["lat"], 99)), 4),
           "bytes": r["bytes"]}
    for side in ("enc", "dec"):
        k = f"mean_steps_{side}"
        if k in st:
            ms = st[k][0] / steps
            out[f"{k}_ms"] = round(ms, 4)
            out[f"{k}_tflops"] = round(fl / (ms * 1e-3) / 1e12, 2)
    if "mean_steps_dec_ms" in out:
        a = out["mean_steps_dec_tflops"]
        out["roofline"] = {"kernel": "mean_step_kernel (3 launches per side)", "bound": "mfma",
                           "achieved": a, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                           "frac": round(a / PEAK_TFLOPS["fp32"], 4),
                           "flop_per_side": fl}
    out["note"] = ("bf16 convs; partitions 1-3 refined by 3 float32 MFMA mean steps per side "
                   "(Sec. 3.4 quadtree means); same 1080p T=8 chunks and step as the headline")
    return out


def run_seg_sweep(torch, ufvc, weights, chunks, H, W, steps, warmup, lanes, sizes=(11, 12, 13, 14)):
    """y segment size (symbols per rANS segment = 2^seg_log2) against speed
    and stream size on the headline workload: per size, the y decode and
    encode kernel times (HIP events, one chunk at a time), the stream bytes,
    and the enc+dec rates one chunk at a time and with `lanes` in flight."""
    out = {}
    for sl in sizes:
        r = run_codec(torch, ufvc, weights, "bf16", chunks, H, W, steps, warmup, sl, 10,
                      profile=True, autotune=True)
        rp = run_pipelined(torch, ufvc, weights, "bf16", chunks, H, W, steps, warmup, sl, 10,
                           lanes=lanes)
        T = chunks[0].shape[0]
        st = r["stages"]
        out[str(sl)] = {"y_segments": -(-((H + 15) // 16 * 2) * ((W + 15) // 16 * 2) * 128 // (1 << sl)),
                        "rans_decode_y_us": round(1e3 * st["rans_decode_y"][0] / steps, 1),
                        "rans_encode_us": round(1e3 * st["rans_encode"][0] / steps, 1),
                        "bytes": r["bytes"],
                        "sequential_fps": round(T * steps / r["seconds"], 1),
                        "pipelined_fps": round(T * rp["steps"] / rp["seconds"], 1)}
    return out


def run_temporal(torch, ufvc, chunks, H, W, steps, warmup, seg_log2, seg_log2_z, lanes):
    """The temporal-context model: each lane codes one stream of 1080p T=8
    chunks in order (its encoder and decoder stream objects carry the
    context), one chunk's encode + decode per step; one lane, then `lanes`
    streams in flight on their own HIP streams and host threads."""
    import threading
    from synthetic import stand_in_weights
    T, C = chunks[0].shape[0], 128
    wt = stand_in_weights(T, C, temporal=True)

    def run(n_lanes, n_steps, profile):
        codecs = [ufvc.Codec(T, C, wt, precision="bf16", seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                             model_tag=0x7E00_1080, autotune=True) for _ in range(n_lanes)]
        encs = [ufvc.Stream(c, H, W) for c in codecs]
        decs = [ufvc.Stream(c, H, W) for c in codecs]
        hs = [torch.cuda.Stream() for _ in range(n_lanes)]
        cap = codecs[0].max_bitstream_bytes(H, W)
        bufs = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in range(n_lanes)]
        outs = [torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda") for _ in range(n_lanes)]
        sizes = [[] for _ in range(n_lanes)]

        def lane(li, n, off):
            for i in range(n):
                _, nb = encs[li].encode(chunks[(off + i * n_lanes + li) % len(chunks)], out=bufs[li],
                                        stream=hs[li])
                sizes[li].append(nb)
                decs[li].decode(bufs[li], nb, out=outs[li], stream=hs[li], check=False)

        def go(n, off):
            ths = [threading.Thread(target=lane, args=(li, n, off)) for li in range(n_lanes)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()

        go(warmup, 0)
        torch.cuda.synchronize()
        if profile:
            codecs[0].profile(True)
        per = n_steps // n_lanes
        t0 = time.perf_counter()
        go(per, warmup)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = codecs[0].profile_read() if profile else {}
        for li, c in enumerate(codecs):
            if c.status(hs[li]) != 0:
                raise RuntimeError("temporal decode reported an error")
            if not np.array_equal(encs[li].context().view(np.uint32), decs[li].context().view(np.uint32)):
                raise RuntimeError("encoder and decoder contexts differ")
        for o in encs + decs + codecs:
            o.close()
        return T * per * n_lanes / dt, st, int(np.mean(sizes[0][warmup:]))

    seq, st, nbytes = run(1, steps, True)
    pipe, _, _ = run(lanes, steps, False)
    extra = {k: round(v[0] / steps, 4) for k, v in st.items()
             if k.startswith("context") or k == "chunk_decoder_enc"}
    return {"value": round(pipe, 2), "unit": "frames/s", "chunks_in_flight": lanes,
            "sequential": round(seq, 2), "mean_bytes": nbytes, "context_stage_ms": extra,
            "note": "bf16; each step encodes the stream's next 1080p T=8 chunk with its context "
                    "and decodes it (the encoder also runs the chunk decoder and the context "
                    "network); encoder and decoder contexts checked equal after the run"}


def run_color(torch, ufvc, chunks, H, W, steps, seg_log2, seg_log2_z):
    """Format conversions around the YUV444 interface (BT.709 RGB, 4:2:0) on
    the headline's 1080p T=8 frames: each kernel's HBM rate (HIP events on the
    stream it runs on; algorithmic bytes = every value read once and written
    once), and the RGB-in / RGB-out codec step one chunk at a time."""
    T = chunks[0].shape[0]
    px = T * H * W
    nbytes = {"rgb_to_yuv444": 24.0 * px, "yuv444_to_rgb": 24.0 * px,
              "yuv420_to_444": 18.0 * px, "yuv444_to_420": 18.0 * px}
    src = {"rgb_to_yuv444": ("rgb", "yuv444"), "yuv444_to_rgb": ("yuv444", "rgb"),
           "yuv420_to_444": ("yuv420", "yuv444"), "yuv444_to_420": ("yuv444", "yuv420")}
    yuv = ufvc.convert_frames(chunks[0], "rgb", "yuv444", T, H, W)
    f420 = ufvc.convert_frames(yuv, "yuv444", "yuv420", T, H, W)
    inputs = {"rgb": chunks[0], "yuv444": yuv, "yuv420": f420}
    stream = torch.cuda.current_stream()
    out = {}
    reps = 20
    for k, (a, b) in src.items():
        dst = ufvc.convert_frames(inputs[a], a, b, T, H, W)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            ufvc.convert_frames(inputs[a], a, b, T, H, W, out=dst)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes[k] / (ms * 1e-3) / 1e9
        out[k] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
                  "bytes": nbytes[k]}
    from synthetic import stand_in_weights
    c = ufvc.Codec(T, 128, stand_in_weights(T, 128), precision="bf16", seg_log2=seg_log2,
                   seg_log2_z=seg_log2_z, model_tag=0x0800_1080, autotune=True)
    bs = torch.empty(c.max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
    rgb_out = torch.empty_like(chunks[0])
    yuv_in = torch.empty_like(chunks[0])
    yuv_out = torch.empty_like(chunks[0])

    def step(i):
        ufvc.convert_frames(chunks[i % len(chunks)], "rgb", "yuv444", T, H, W, out=yuv_in)
        _, n = c.encode(yuv_in, out=bs)
        c.decode(bs, n, H, W, out=yuv_out, check=False)
        ufvc.convert_frames(yuv_out, "yuv444", "rgb", T, H, W, out=rgb_out)

    for i in range(3):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if c.status() != 0:
        raise RuntimeError("decode reported an error in the rgb run")
    c.close()
    return {"kernels": out, "rgb_codec_sequential": {"value": round(T * steps / dt, 2),
                                                      "unit": "frames/s", "steps": steps},
            "note": "RGB in and out (BT.709 to and from YUV444 on the GPU), one chunk at a time"}


def run_dc_block(torch, ufvc, h, w, C=128, reps=50):
    """One fused DC block on the 1080p latent (h x w x C, bf16): HIP-event
    time per launch on the stream it runs on, against the bf16 matrix-core
    peak (algorithmic FLOPs: 2 (6 C^2 + 9 C) per position) and HBM (input
    read and output written once, plus the weights)."""
    from synthetic import dc_block_weights, feature_map
    blk = ufvc.DcBlock(C, dc_block_weights(C, seed=1))
    x = torch.from_numpy(np.ascontiguousarray(np.transpose(feature_map(C, h, w, seed=3), (1, 2, 0))))
    x = x.to(torch.bfloat16).cuda()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        blk.run(x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        blk.run(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    blk.close()
    ms = e0.elapsed_time(e1) / reps
    npos = h * w
    flop = 2.0 * (6 * C * C + 9 * C) * npos
    nbytes = 4.0 * C * npos + 12.0 * C * C + 36.0 * C
    tf = flop / (ms * 1e-3) / 1e12
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"latent": f"{h}x{w}x{C}", "ms": round(ms, 4),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK_TFLOPS["bf16"],
                         "unit": "TFLOP/s", "frac": round(tf / PEAK_TFLOPS["bf16"], 4),
                         "flop_per_launch": flop},
            "hbm": {"achieved_gbs": round(gbs, 1), "frac": round(gbs / PEAK_HBM_GBS, 4),
                    "bytes_per_launch": nbytes},
            "note": "fused DC block (pw1, depth-wise 3x3, pw2, pw3, pw4 with residuals), "
                    "bf16 in and out; intensity 2 (6C + 9) / 4 FLOP per byte"}


def run_fp8_c4(torch, ufvc, steps, seg_log2, seg_log2_z, n_chunks=16, n_oracle=2):
    """16 chunks of 1920x1088, T = 8: analysis convs BF16, synthesis convs FP8
    E4M3 (per-output-channel weight scales), entropy params FP32, tables FP64
    on the GPU; encoded and decoded as one batch.  Reports throughput, the
    bit-stream size against the FP32 path, PSNR against the source next to
    the FP32 and BF16 paths, and for the first n_oracle chunks the max abs
    and PSNR of the FP8 and BF16 frames against the float64 oracle's
    synthesis of the same y_hat (a bounded sample: about 5 s of host work per
    chunk and precision)."""
    from synthetic import stand_in_weights, video_chunk
    T, H, W, C = 8, 1088, 1920, 128
    w = stand_in_weights(T, C)
    frames = [torch.from_numpy(video_chunk(T, H, W, 16, seed=4, chunk_id=k)).cuda()
              for k in range(n_chunks)]
    codecs = {p: ufvc.Codec(T, C, w, precision=p, seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                            model_tag=0x0C40_1080, autotune=True)
              for p in ("bf16_fp8", "bf16", "fp32")}
    per = {p: [] for p in codecs}
    sizes = {p: [] for p in codecs}
    vs_oracle = {p: [] for p in ("bf16_fp8", "bf16")}
    from oracle import nets
    for p, c in codecs.items():
        for k, fr in enumerate(frames):
            bs, n = c.encode(fr)
            sizes[p].append(n)
            rec = c.decode(bs, n, H, W)
            per[p].append(psnr_t(torch, fr, rec))
            if p in vs_oracle and k < n_oracle:
                # the float64 oracle's synthesis of this chunk's own y_hat
                sym = c.buffer(ufvc.BUF_SYM, H, W).astype(np.float64)
                mu = c.buffer(ufvc.BUF_PARAMS, H, W)[..., :C].astype(np.float64)
                ref = nets.synthesis(np.transpose(sym - 32 + mu, (2, 0, 1)), w, T, H, W)
                err = np.abs(rec.cpu().numpy().astype(np.float64) - ref)
                mse = float(np.mean(err ** 2))
                vs_oracle[p].append({"chunk": k, "max_abs": round(float(err.max()), 5),
                                     "mean_abs": round(float(err.mean()), 6),
                                     "psnr_db": round(10 * np.log10(1 / mse), 3)})
    batch = ufvc.Batch([codecs["bf16_fp8"]])
    outs = [torch.empty(codecs["bf16_fp8"].max_bitstream_bytes(H, W), dtype=torch.uint8,
                        device="cuda") for _ in frames]
    recs = [torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda") for _ in frames]
    enc_items = [(0, fr, o) for fr, o in zip(frames, outs)]
    lens = batch.encode(enc_items)
    dec_items = [(0, o, n, H, W, r) for o, n, r in zip(outs, lens, recs)]
    st, code = batch.decode(dec_items, graph=True)
    if code != 0:
        raise RuntimeError(f"fp8 batch decode status {st}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lens = batch.encode(enc_items)
        batch.decode(dec_items, graph=True, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st, code = batch.sync_status()
    if code != 0:
        raise RuntimeError(f"fp8 batch decode status {st}")
    same = all(int(lens[i]) == sizes["bf16_fp8"][i] for i in range(len(frames)))
    # one chunk at a time: the synthesis convs' HIP-event times, FP8 next to BF16
    synth = ("d1_conv", "d2_conv", "d3_conv", "k1_conv", "k2_conv", "k3_conv")
    one_chunk = {}
    for p in ("bf16_fp8", "bf16"):
        c = codecs[p]
        torch.cuda.synchronize()
        c.profile(True)
        reps = 5
        for _ in range(reps):
            bs, n = c.encode(frames[0])
            c.decode(bs, n, H, W, check=False)
        torch.cuda.synchronize()
        stg = c.profile_read()
        c.profile(False)
        one_chunk[p] = {k: round(v[0] / reps, 4) for k, v in stg.items() if k in synth}
        one_chunk[p]["synthesis"] = round(sum(v[0] for k, v in stg.items() if k in synth) / reps, 4)
    d8 = np.array(per["bf16_fp8"]) - np.array(per["fp32"])
    d16 = np.array(per["bf16"]) - np.array(per["fp32"])
    dsize = np.array(sizes["bf16_fp8"], np.float64) / np.array(sizes["fp32"]) - 1
    res = {"chunks": len(frames), "value": round(T * len(frames) * steps / dt, 2),
           "unit": "frames/s", "steps": steps, "ms_per_batch": round(1e3 * dt / steps, 3),
           "batch_lengths_equal_single": same,
           "psnr_delta_fp8_vs_fp32_db": {"min": round(float(d8.min()), 4),
                                         "max": round(float(d8.max()), 4),
                                         "mean": round(float(d8.mean()), 4)},
           "psnr_delta_bf16_vs_fp32_db_mean": round(float(d16.mean()), 4),
           "bitstream_size_delta_vs_fp32": {"min": round(float(dsize.min()), 6),
                                            "max": round(float(dsize.max()), 6)},
           "per_chunk_psnr_db": {p: [round(x, 3) for x in v] for p, v in per.items()},
           "vs_fp64_oracle": {"sample": f"chunks 0-{n_oracle - 1} of {len(frames)}", **vs_oracle},
           "one_chunk_synthesis_ms": one_chunk,
           "precision": "analysis bf16, synthesis fp8 e4m3 (d1 bf16), params fp32, tables fp64"}
    batch.close()
    for c in codecs.values():
        c.close()
    return res


C5_MIX = [(21, 832, 480), (21, 1280, 720), (16, 1920, 1088), (6, 3840, 2160)]


def run_serving(torch, ufvc, prec, mix, seconds, rate, seg_log2, seg_log2_z, seed=5,
                lanes=2, max_batch=8, small_pixels=1920 * 1088):
    """Open-loop serving: 64 streams (resolution mix), Poisson arrivals of
    `rate` chunk requests/s for `seconds`, 70% decode / 30% encode, T = 8,
    C = 128.  Inputs and bit-streams are resident in HBM before the clock
    starts; the server admits requests within a 64 GiB footprint; lane 0
    prefers requests of at most 1920x1088.  Its frames/s is bound by the
    arrival rate; `capacity` is a closed-loop run of the same request mix
    (all submitted at once) that measures what the server sustains."""
    import threading
    from synthetic import stand_in_weights, video_chunk
    T, C = 8, 128
    codec = ufvc.Codec(T, C, stand_in_weights(T, C), precision=prec, seg_log2=seg_log2,
                       seg_log2_z=seg_log2_z, model_tag=0x0C50_0000, autotune=True)
    streams = [(W, H) for count, W, H in mix for _ in range(count)]
    res = sorted(set(streams))
    src, bits = {}, {}
    for k, (W, H) in enumerate(res):
        fr = torch.from_numpy(video_chunk(T, H, W, 16, seed=seed, chunk_id=k)).cuda()
        bs, n = codec.encode(fr)              # also tunes this size's tiles
        codec.decode(bs, n, H, W)
        src[(W, H)], bits[(W, H)] = fr, (bs[:n].clone(), n)
    enc_out = [torch.empty(codec.max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
               for (W, H) in streams]
    dec_out = [torch.empty((T, 3, H, W), dtype=torch.float32, device="cuda") for (W, H) in streams]
    srv = ufvc.Server([codec], hbm_budget=64 << 30, lanes=lanes, max_batch=max_batch, graph=True,
                      small_pixels=small_pixels)

    def submit(i, kind):
        W, H = streams[i]
        if kind == "enc":
            return srv.submit_encode(0, src[(W, H)], enc_out[i], tag=i)
        bs, n = bits[(W, H)]
        return srv.submit_decode(0, bs, n, H, W, dec_out[i], tag=i)

    # warm-up burst: plans and arenas for the common compositions
    warm = [submit(i % len(streams), "dec" if i % 3 else "enc") for i in range(4 * max_batch)]
    got = 0
    while got < len(warm):
        got += len(srv.poll(64, 200))
    rng = np.random.default_rng(seed)
    n_req = int(rng.poisson(rate * seconds))
    t_arr = np.sort(rng.uniform(0.0, seconds, n_req))
    who = rng.integers(0, len(streams), n_req)
    kinds = np.where(rng.uniform(size=n_req) < 0.7, "dec", "enc")
    comps = []

    def poller():
        while len(comps) < n_req:
            comps.extend(srv.poll(256, 200))

    th = threading.Thread(target=poller)
    st0 = srv.stats()
    th.start()
    t0 = time.perf_counter()
    for k in range(n_req):
        dt = t0 + t_arr[k] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        submit(int(who[k]), kinds[k])
    th.join()
    st = srv.stats()
    # closed loop: the same number of requests, all queued at once
    n_cap = min(n_req, 600)
    t_c = time.perf_counter()
    for k in range(n_cap):
        submit(int(who[k]), kinds[k])
    got = 0
    while got < n_cap:
        got += len(srv.poll(256, 200))
    cap_s = time.perf_counter() - t_c
    st_cap = srv.stats()
    srv.close()
    codec.close()
    bad = sum(1 for c in comps if c["status"] != 0)
    if bad:
        raise RuntimeError(f"{bad} serving requests failed")
    lat = np.array([(c["t_done_us"] - c["t_submit_us"]) / 1e3 for c in comps])
    first = min(c["t_submit_us"] for c in comps)
    last = max(c["t_done_us"] for c in comps)
    pix = {i: streams[i][0] * streams[i][1] for i in range(len(streams))}
    frames = T * n_req
    by_res = {}
    for (W, H) in res:
        lr = np.array([(c["t_done_us"] - c["t_submit_us"]) / 1e3 for c in comps
                       if streams[int(c["tag"])] == (W, H)])
        if lr.size:
            by_res[f"{W}x{H}"] = {"requests": int(lr.size), "p50": round(float(np.percentile(lr, 50)), 3),
                                  "p99": round(float(np.percentile(lr, 99)), 3),
                                  "max": round(float(lr.max()), 3)}
    return {"precision": prec, "requests": n_req, "seconds": seconds, "rate_req_s": rate,
            "value": round(frames / ((last - first) / 1e6), 2), "unit": "frames/s",
            "value_note": "arrival-bound: the open-loop rate times T, not the server's capacity",
            "capacity": {"value": round(T * n_cap / cap_s, 2), "unit": "frames/s",
                         "requests": n_cap, "mean_batch": round(
                             (st_cap["completed"] - st["completed"]) /
                             max(1, st_cap["batches"] - st["batches"]), 2)},
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "max": round(float(lat.max()), 3)},
            "latency_ms_by_resolution": by_res,
            "plan_builds_in_timed_window": int(st["plans_built"] - st0["plans_built"]),
            "small_first_lane_pixels": small_pixels,
            "decode_share": round(float(np.mean(kinds == "dec")), 3),
            "mean_batch": round(float(np.mean([c["batch_size"] for c in comps])), 2),
            "batches": int(st["batches"]), "lanes": lanes, "max_batch": max_batch,
            "peak_footprint_gib": round(st["peak_footprint"] / 2 ** 30, 3),
            "budget_gib": round(st["budget"] / 2 ** 30, 1),
            "mpix_per_s": round(sum(pix[int(i)] for i in who) * T / ((last - first) / 1e6) / 1e6, 1)}


def bitstream_report(r, h, w, C, sl, slz):
    """Stream size against the ideal code length: the literal reading (whole
    stream within 0.5%) and the per-segment reading (payload within 0.5% plus
    the 32 flushed 32-bit lane states of every segment)."""
    ny, nz = h * w * C, ((h + 1) // 2) * ((w + 1) // 2) * 32
    n_seg = -(-ny // (1 << sl)) + -(-nz // (1 << slz))
    payload_bits = 8 * (r["bytes"] - 28 - 4 * n_seg)
    ideal = r["ideal_bits"]
    return {"bytes": r["bytes"], "segments": n_seg,
            "bits_per_symbol": round(8 * r["bytes"] / r["n_sym"], 4),
            "overhead_vs_ideal": round(8 * r["bytes"] / ideal - 1, 5),
            "overhead_excluding_lane_flush": round((payload_bits - 1024 * n_seg) / ideal - 1, 5),
            "within_0p5pct_literal": bool(8 * r["bytes"] - ideal <= 0.005 * ideal),
            "within_0p5pct_plus_flush": bool(0 <= payload_bits - ideal <= 0.005 * ideal + 1024 * n_seg)}


def psnr_t(torch, a, b):
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def precision_report(torch, ufvc, weights, chunk_np, H, W, seg_log2, seg_log2_z):
    """Every precision's error against the float64 oracle on chunk 0 of the
    headline workload (T=8, 1080p, C=128), each stage on the GPU's own input:
    y against the oracle's analysis of the frames; scale indices and symbols
    against the oracle's entropy model of the GPU's z_hat and y, and against
    the FP32 GPU path; frames against the oracle synthesis of the GPU's own
    y_hat (what the decoder decodes), as max abs and PSNR; and the BF16 / FP8
    reconstruction against the FP32 one directly.  About 20 s of host float64
    work."""
    from oracle import entropy, nets
    T, C = chunk_np.shape[0], 128
    o_y = np.transpose(nets.analysis(chunk_np, weights), (1, 2, 0))
    h, w = o_y.shape[0], o_y.shape[1]
    res, gpu = {}, {}
    frames = torch.from_numpy(chunk_np).cuda()
    for p in ("fp32", "bf16", "bf16_fp8"):
        c = ufvc.Codec(T, C, weights, precision=p, seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                       model_tag=0x0800_1080, autotune=True)
        bs, n = c.encode(frames)
        g_y = c.buffer(ufvc.BUF_Y, H, W).astype(np.float64)
        g_z = c.buffer(ufvc.BUF_ZSYM, H, W).astype(np.float64) - 32
        g_P = c.buffer(ufvc.BUF_PARAMS, H, W).astype(np.float64)
        g_idx = c.buffer(ufvc.BUF_IDX, H, W)
        g_sym = c.buffer(ufvc.BUF_SYM, H, W)
        rec = c.decode(bs, n, H, W).cpu().numpy().astype(np.float64)
        c.close()
        mu, sigma = nets.params(np.transpose(g_z, (2, 0, 1)), weights, h, w)
        o_idx = np.transpose(entropy.scale_index(sigma), (1, 2, 0))
        o_sym = np.clip(np.rint(g_y - np.transpose(mu, (1, 2, 0))), -32, 32) + 32
        y_hat = np.transpose(g_sym.astype(np.float64) - 32 + g_P[..., :C], (2, 0, 1))
        ref = nets.synthesis(y_hat, weights, T, H, W)
        err = np.abs(rec - ref)
        mse = float(np.mean(err ** 2))
        gpu[p] = (g_idx, g_sym, rec, n)
        res[p] = {"y_max_abs_vs_oracle": float(np.abs(g_y - o_y).max()),
                  "y_max_abs_over_max_y": float(np.abs(g_y - o_y).max() / np.abs(o_y).max()),
                  "idx_agree_oracle": float(np.mean(g_idx == o_idx)),
                  "sym_agree_oracle": float(np.mean(g_sym == o_sym)),
                  "frames_vs_oracle_synthesis": {"max_abs": float(err.max()),
                                                 "psnr_db": round(10 * np.log10(1 / mse), 3)
                                                 if mse > 0 else None},
                  "bytes": int(n)}
    for p in ("bf16", "bf16_fp8"):
        i32, s32, r32, n32 = gpu["fp32"]
        ip, sp_, rp, npb = gpu[p]
        mse = float(np.mean((rp - r32) ** 2))
        res[p]["idx_agree_fp32"] = float(np.mean(ip == i32))
        res[p]["sym_agree_fp32"] = float(np.mean(sp_ == s32))
        res[p]["recon_psnr_vs_fp32_db"] = round(10 * np.log10(1 / mse), 3) if mse > 0 else None
        res[p]["bytes_vs_fp32"] = round(npb / n32 - 1, 6)
    res["note"] = ("chunk 0 of the 1080p T=8 workload; every stage on the GPU's own input; "
                   "frames against the float64 oracle's synthesis of the GPU's own y_hat")
    return res


def cpu_baseline(T, H, W, C, n_chunks=3, seg_log2=13, seg_log2_z=10):
    """The oracle, untouched, on `n_chunks` full chunks of the same workload
    (about 10-30 s of host work)."""
    from oracle import codec as ocodec
    from synthetic import stand_in_weights, video_chunk
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = 1
    w = stand_in_weights(T, C)
    frames = [video_chunk(T, H, W, 16, seed=1, chunk_id=k) for k in range(n_chunks)]
    t0 = time.perf_counter()
    for fr in frames:
        bs, _ = ocodec.encode_chunk(fr, w, seg_log2=seg_log2, seg_log2_z=seg_log2_z,
                                    model_tag=0x0800_1080)
        ocodec.decode_chunk(bs, w)
    dt = time.perf_counter() - t0
    return {"value": T * n_chunks / dt, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_chunks} {W}x{H} T={T} chunks (generator chunks 0-{n_chunks - 1}): "
                      f"float64 oracle encode + decode at segment sizes 2^{seg_log2} / "
                      f"2^{seg_log2_z} (the GPU line's), {dt:.1f} s; BLAS threads {threads}, "
                      f"rANS loop single-threaded, host cpus {len(os.sched_getaffinity(0))}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp32-steps", type=int, default=10)
    ap.add_argument("--seg-log2", type=int, default=None, help="default: the package's")
    ap.add_argument("--seg-log2-z", type=int, default=None, help="default: the package's")
    ap.add_argument("--chunks", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 leg (profiling runs)")
    ap.add_argument("--no-t1", action="store_true", help="skip the one-frame-chunk leg")
    ap.add_argument("--no-quadtree", action="store_true", help="skip the quadtree-means leg")
    ap.add_argument("--no-color", action="store_true", help="skip the format-conversion leg")
    ap.add_argument("--no-dcblock", action="store_true", help="skip the DC-block leg")
    ap.add_argument("--no-temporal", action="store_true", help="skip the temporal-context leg")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the per-precision errors against the oracle (about 20 s of host work)")
    ap.add_argument("--seg-sweep", action="store_true",
                    help="add the y segment-size sweep (2^11 .. 2^14) to the line")
    ap.add_argument("--lanes", type=int, default=2, help="chunks in flight for the headline run")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="finish with three plain device copies of this many MB (counter scaling)")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--batch-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: it measures the single-GPU hot path "
              "(whole chunks shard across GPUs with no exchange between them).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2606_04410_amd as ufvc
    from synthetic import stand_in_weights, video_chunk
    if args.seg_log2 is None:
        args.seg_log2 = ufvc.DEFAULT_SEG_LOG2
    if args.seg_log2_z is None:
        args.seg_log2_z = ufvc.DEFAULT_SEG_LOG2_Z

    T, H, W, C = 8, 1080, 1920, 128
    log(f"bench: generating {args.chunks} chunks T={T} {W}x{H}")
    chunks_np = [video_chunk(T, H, W, 16, seed=1, chunk_id=k) for k in range(args.chunks)]
    chunks = [torch.from_numpy(x).cuda() for x in chunks_np]
    weights = stand_in_weights(T, C)
    Hp = -(-H // 16) * 16
    h, w = Hp // 8, W // 8

    log("bench: bf16 timed region")
    r16 = run_codec(torch, ufvc, weights, "bf16", chunks, H, W, args.steps, args.warmup,
                    args.seg_log2, args.seg_log2_z, profile=True, autotune=not args.no_autotune)
    r32 = None
    if not args.no_fp32:
        log("bench: fp32 timed region")
        r32 = run_codec(torch, ufvc, weights, "fp32", chunks, H, W, args.fp32_steps, 2,
                        args.seg_log2, args.seg_log2_z, profile=True, autotune=not args.no_autotune)

    log(f"bench: bf16 pipelined ({args.lanes} chunks in flight)")
    rp = run_pipelined(torch, ufvc, weights, "bf16", chunks, H, W, args.steps, args.warmup,
                       args.seg_log2, args.seg_log2_z, lanes=args.lanes)
    fps16 = T * args.steps / r16["seconds"]
    fps_pipe = T * rp["steps"] / rp["seconds"]
    src0 = chunks[0]
    p16 = psnr_t(torch, src0, r16["rec"])

    flops = conv_flops(T, C, h, w)
    hbm = stage_bytes(h, w, C, r16)
    st = r16["stages"]
    dom = max(st, key=lambda k: st[k][0])
    avg_ms = st[dom][0] / st[dom][1]
    if dom in flops:
        achieved = flops[dom] / (avg_ms * 1e-3) / 1e12
        traffic = None
        tile = r16["tuning"].get(dom.replace("_conv", ""))
        if tile and conv_sources_sha256() == TRAFFIC_SHA256:
            rw = TRAFFIC.get((dom, tile[0]))
            if rw:
                alg = (a1_algorithmic_bytes(T, C, H, W, h, w) if dom == "a1_conv"
                       else k3_algorithmic_bytes(T, C, H, W, h, w))
                traffic = {"read_bytes": rw[0], "write_bytes": rw[1], "bytes": rw[0] + rw[1],
                           "algorithmic_bytes": alg, "tile_config": tile[0],
                           "source": "rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated"}
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2),
                "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS["bf16"], 4), "traffic": traffic,
                "avg_launch_ms": round(avg_ms, 4), "flop_per_launch": flops[dom]}
    else:
        achieved = hbm.get(dom, 0.0) / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 5), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": hbm.get(dom)}
    hbm_gbs = {k: round(hbm[k] / (st[k][0] / st[k][1] * 1e-3) / 1e9, 1) for k in hbm if k in st}
    conv_ms = sum(v[0] for k, v in st.items() if k in flops) / args.steps
    conv_flop = sum(flops.values())
    stage_ms = {k: round(v[0] / args.steps, 4) for k, v in sorted(st.items(), key=lambda kv: -kv[1][0])}
    enc_stages = ("a1_conv", "a2_conv", "a3_conv", "hyper_conv", "params_conv_enc",
                  "params_epilogue_enc", "rans_encode", "compact")
    enc_ms = sum(v for k, v in stage_ms.items() if k in enc_stages)
    dec_ms = sum(v for k, v in stage_ms.items() if k not in enc_stages)

    result = {
        "metric": METRIC, "value": round(fps_pipe, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": rp["steps"], "warmup": args.warmup,
        "ms_per_step": round(1e3 * rp["seconds"] / rp["steps"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"1080p chunk codec: T={T} frames {W}x{H} (padded {Hp}), C={C}, "
                               f"encode+decode per step, {args.lanes} chunks in flight", "T": T,
                   "H": H, "W": W, "C": C, "chunks_in_flight": args.lanes,
                   "seg_log2": args.seg_log2, "seg_log2_z": args.seg_log2_z,
                   "chunks_cycled": args.chunks, "precision": "bf16 convs, fp32 entropy params, "
                                                          "fp64 tables"},
        "latency_ms": {"p50": round(float(np.percentile(rp["lat"], 50)), 4),
                       "p99": round(float(np.percentile(rp["lat"], 99)), 4)},
        "sequential": {"value": round(fps16, 2), "unit": "frames/s", "steps": args.steps,
                       "ms_per_step": round(1e3 * r16["seconds"] / args.steps, 4),
                       "latency_ms": {"p50": round(float(np.percentile(r16["lat"], 50)), 4),
                                      "p99": round(float(np.percentile(r16["lat"], 99)), 4)},
                       "note": "one chunk at a time on one stream (the paper's chunk-by-chunk "
                               "order), timed without per-stage events; the per-stage timings "
                               "(stage_ms, roofline) come from the same steps run again with the "
                               "library's HIP events around every launch"},
        "roofline": roof,
        "entropy_gbs": hbm_gbs,
        "conv_stack": {"tflop_per_step": round(conv_flop / 1e12, 4), "ms_per_step": round(conv_ms, 4),
                       "achieved_tflops": round(conv_flop / (conv_ms * 1e-3) / 1e12, 2),
                       "frac_bf16_peak": round(conv_flop / (conv_ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"], 4)},
        "enc_ms": round(enc_ms, 4), "dec_ms": round(dec_ms, 4),
        "stage_ms": stage_ms,
        "tile_configs": {k: (v[1:] if v else None) for k, v in r16["tuning"].items()},
        "bitstream": bitstream_report(r16, h, w, C, args.seg_log2, args.seg_log2_z),
    }
    if r32 is not None:
        fps32 = T * args.fp32_steps / r32["seconds"]
        p32 = psnr_t(torch, src0, r32["rec"])
        result["fp32"] = {"value": round(fps32, 2), "unit": "frames/s", "steps": args.fp32_steps,
                          "ms_per_step": round(1e3 * r32["seconds"] / args.fp32_steps, 4),
                          "latency_ms_p99": round(float(np.percentile(r32["lat"], 99)), 4)}
        result["bf16_speedup_vs_fp32"] = round(fps16 / fps32, 3)
        result["psnr_db"] = {"bf16": round(p16, 4), "fp32": round(p32, 4),
                             "delta": round(p16 - p32, 4),
                             "bf16_vs_fp32_recon": round(psnr_t(torch, r32["rec"], r16["rec"]), 3)}
        result["fp32_stage_ms"] = {k: round(v[0] / args.fp32_steps, 4)
                                   for k, v in r32["stages"].items()}
    if not args.no_t1:
        # one-frame chunks: the chunk size of the paper's low-delay mode (its
        # temporal context is not built), same stand-in net with T = 1
        log("bench: one-frame chunks (T=1)")
        c1_np = [video_chunk(1, H, W, 16, seed=3, chunk_id=k) for k in range(args.chunks)]
        c1 = [torch.from_numpy(x).cuda() for x in c1_np]
        w1 = stand_in_weights(1, C)
        r1 = run_codec(torch, ufvc, w1, "bf16", c1, H, W, args.steps, args.warmup,
                       args.seg_log2, args.seg_log2_z, profile=False, autotune=not args.no_autotune)
        p1 = run_pipelined(torch, ufvc, w1, "bf16", c1, H, W, args.steps, args.warmup,
                           args.seg_log2, args.seg_log2_z, lanes=args.lanes)
        result["one_frame_chunks"] = {
            "value": round(args.steps / r1["seconds"], 2), "unit": "frames/s",
            "latency_ms": {"p50": round(float(np.percentile(r1["lat"], 50)), 4),
                           "p99": round(float(np.percentile(r1["lat"], 99)), 4)},
            "in_flight": {"chunks": args.lanes, "value": round(p1["steps"] / p1["seconds"], 2),
                          "latency_ms_p99": round(float(np.percentile(p1["lat"], 99)), 4)},
            "psnr_db": round(psnr_t(torch, c1[0], r1["rec"]), 4),
            "note": "T=1 chunks of 1920x1080 (the low-delay mode's chunk size; its temporal "
                    "context is not built), bf16, encode+decode per frame, one frame at a time"}
    if not args.no_quadtree:
        log("bench: quadtree progressive means")
        result["quadtree"] = run_quadtree(torch, ufvc, chunks, H, W, args.steps, args.warmup,
                                          args.seg_log2, args.seg_log2_z, args.lanes,
                                          autotune=not args.no_autotune)
    if not args.no_color:
        log("bench: format conversions (BT.709 RGB, 4:2:0)")
        result["color"] = run_color(torch, ufvc, chunks, H, W, 20, args.seg_log2, args.seg_log2_z)
    if not args.no_precision:
        log("bench: per-precision errors against the oracle (chunk 0)")
        result["precision_vs_oracle"] = precision_report(torch, ufvc, weights, chunks_np[0], H, W,
                                                         args.seg_log2, args.seg_log2_z)
    if args.seg_sweep:
        log("bench: segment-size sweep")
        result["seg_sweep"] = run_seg_sweep(torch, ufvc, weights, chunks, H, W, args.steps,
                                            args.warmup, args.lanes)
    if not args.no_temporal:
        log("bench: temporal context")
        result["temporal"] = run_temporal(torch, ufvc, chunks, H, W, args.steps, args.warmup,
                                          args.seg_log2, args.seg_log2_z, args.lanes)
    if not args.no_dcblock:
        log("bench: DC block")
        result["dc_block"] = run_dc_block(torch, ufvc, h, w, C)
    if not args.no_batch:
        log("bench: 48-chunk batch")
        result["batch_c3"] = run_batch_c3(torch, ufvc, args.batch_steps, args.seg_log2,
                                          args.seg_log2_z)
    if not args.no_fp8:
        log("bench: fp8 synthesis, 16 chunks")
        result["fp8_c4"] = run_fp8_c4(torch, ufvc, args.batch_steps, args.seg_log2,
                                      args.seg_log2_z)
    if not args.no_serve:
        serving = {}
        for name, mix in (("mix", C5_MIX), ("all_1080p", [(64, 1920, 1088)])):
            for prec in ("bf16", "fp32"):
                log(f"bench: serving {name} {prec}")
                serving[f"{name}_{prec}"] = run_serving(torch, ufvc, prec, mix, args.serve_seconds,
                                                        240.0, args.seg_log2, args.seg_log2_z)
        result["serving"] = serving
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(T, H, W, C, seg_log2=args.seg_log2,
                                              seg_log2_z=args.seg_log2_z)
    if args.calib_copy_mb:
        # plain copies of a known size, for scaling hardware byte counters
        n = args.calib_copy_mb * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
