"""Batched launches: each chunk's result is the same alone and in a batch of
uneven chunks (two models, T = 4 and T = 8), and graph-captured decode
replays equal eager decode."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from synthetic import stand_in_weights, video_chunk  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["bf16", "fp32", "bf16_fp8"])
def test_batch_equals_single_and_graph_equals_eager(prec):
    import paper_2606_04410_amd as u
    C = 64
    models = [u.Codec(4, C, stand_in_weights(4, C), precision=prec, seg_log2=11, seg_log2_z=9,
                      model_tag=41, autotune=True),
              u.Codec(8, C, stand_in_weights(8, C), precision=prec, seg_log2=11, seg_log2_z=9,
                      model_tag=81, autotune=True)]
    shapes = [(0, 64, 64), (1, 96, 128), (0, 136, 80), (1, 64, 64), (0, 48, 200)]
    say(f"batch {prec}: {shapes}")
    frames = [torch.from_numpy(video_chunk(models[m].T, H, W, 3, seed=7, chunk_id=i)).cuda()
              for i, (m, H, W) in enumerate(shapes)]
    # single-chunk reference
    ref_bs, ref_fr = [], []
    for (m, H, W), fr in zip(shapes, frames):
        bs, n = models[m].encode(fr)
        ref_bs.append(bs[:n].cpu().numpy().tobytes())
        ref_fr.append(models[m].decode(bs, n, H, W).cpu().numpy())
    batch = u.Batch(models)
    outs = [torch.empty(models[m].max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
            for (m, H, W) in shapes]
    lens = batch.encode([(m, fr, o) for (m, _, _), fr, o in zip(shapes, frames, outs)])
    for i in range(len(shapes)):
        assert outs[i][:lens[i]].cpu().numpy().tobytes() == ref_bs[i], i
    rec = [torch.empty((models[m].T, 3, H, W), dtype=torch.float32, device="cuda")
           for (m, H, W) in shapes]
    items = [(m, o, n, H, W, r) for (m, H, W), o, n, r in zip(shapes, outs, lens, rec)]
    st, code = batch.decode(items, graph=False)
    assert code == 0 and all(x == 0 for x in st)
    for i in range(len(shapes)):
        np.testing.assert_array_equal(rec[i].cpu().numpy(), ref_fr[i])
    # graph replays, with eager work and synchronisation in between
    for rep in range(3):
        for r in rec:
            r.fill_(-1.0)
        st, code = batch.decode(items, graph=True)
        assert code == 0 and all(x == 0 for x in st), (rep, st)
        for i in range(len(shapes)):
            np.testing.assert_array_equal(rec[i].cpu().numpy(), ref_fr[i])
        models[0].encode(frames[0])
        torch.cuda.synchronize()
    # a corrupted stream is reported for its chunk only
    bad = outs[2].clone()
    bad[lens[2] // 2] ^= 0x55
    items2 = list(items)
    items2[2] = (shapes[2][0], bad, lens[2], shapes[2][1], shapes[2][2], rec[2])
    st, code = batch.decode(items2, graph=True)
    assert st[2] == -3 and all(st[i] == 0 for i in range(len(st)) if i != 2)
    batch.close()
    for m in models:
        m.close()


C3_BUCKETS = [(480, 832), (720, 1280), (1088, 1920), (2160, 3840)]


@pytest.mark.parametrize("prec", ["bf16", "bf16_fp8"])
def test_batch_c3_buckets_at_c128(prec):
    """One chunk per bucket of the 48-chunk batch mix (832x480, 1280x720,
    1920x1088, 3840x2160), each at T = 4 and T = 8, C = 128, default segment
    sizes and autotuned tiles (the batch benchmark's configuration): batch
    results equal single-chunk results bit for bit, and graph replays equal
    eager decode."""
    import paper_2606_04410_amd as u
    C = 128
    models = [u.Codec(T, C, stand_in_weights(T, C), precision=prec, model_tag=0x0C30_0000 + T,
                      autotune=True) for T in (4, 8)]
    shapes = [(m, H, W) for H, W in C3_BUCKETS for m in (0, 1)]
    say(f"batch C3 buckets {prec}: {shapes}")
    frames = [torch.from_numpy(video_chunk(models[m].T, H, W, 16, seed=3, chunk_id=i)).cuda()
              for i, (m, H, W) in enumerate(shapes)]
    ref_bs, ref_fr = [], []
    for (m, H, W), fr in zip(shapes, frames):
        bs, n = models[m].encode(fr)
        ref_bs.append(bs[:n].clone())
        ref_fr.append(models[m].decode(bs, n, H, W).clone())
    torch.cuda.synchronize()
    batch = u.Batch(models)
    launches = {}
    # both launch policies: one launch per tile configuration, one per stage
    for policy in (0, 1):
        batch.set_policy(policy)
        outs = [torch.zeros(models[m].max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
                for (m, H, W) in shapes]
        lens = batch.encode([(m, fr, o) for (m, _, _), fr, o in zip(shapes, frames, outs)])
        for i in range(len(shapes)):
            assert lens[i] == ref_bs[i].numel() and torch.equal(outs[i][:lens[i]], ref_bs[i]), i
        rec = [torch.full((models[m].T, 3, H, W), -1.0, device="cuda") for (m, H, W) in shapes]
        items = [(m, o, n, H, W, r) for (m, H, W), o, n, r in zip(shapes, outs, lens, rec)]
        st, code = batch.decode(items, graph=False)
        assert code == 0 and all(x == 0 for x in st)
        for i in range(len(shapes)):
            assert torch.equal(rec[i], ref_fr[i]), i
        for rep in range(3):
            for r in rec:
                r.fill_(-1.0)
            st, code = batch.decode(items, graph=True)
            assert code == 0 and all(x == 0 for x in st), (rep, st)
            for i in range(len(shapes)):
                assert torch.equal(rec[i], ref_fr[i]), (rep, i)
            models[1].encode(frames[1])
            torch.cuda.synchronize()
        stt = batch.stats()
        launches[policy] = (stt["conv_launches"], stt["conv_stages"])
    assert launches[1][0] == launches[1][1]          # one launch per conv stage
    assert launches[1][0] <= launches[0][0]
    say(f"  {len(shapes)} chunks: batch == single, graph x3 == eager, both policies; "
        f"conv launches / stages {launches}; "
        f"k1 tiles {[models[m].tuning(H, W)['k1'] for m, H, W in shapes]}")
    batch.close()
    for m in models:
        m.close()


def test_batch_plan_cache_is_bounded():
    """More compositions than the plan cache holds: the least recently used
    plans are evicted, and an evicted composition is rebuilt with the same
    results."""
    import paper_2606_04410_amd as u
    C = 64
    m = u.Codec(1, C, stand_in_weights(1, C), precision="bf16", seg_log2=10, seg_log2_z=8,
                model_tag=7, autotune=False)
    widths = [16 + 8 * k for k in range(34)]
    frames = {W: torch.from_numpy(video_chunk(1, 16, W, 3, seed=2, chunk_id=W)).cuda() for W in widths}
    ref = {}
    for W in widths:
        bs, n = m.encode(frames[W])
        ref[W] = bs[:n].cpu().numpy().tobytes()
    batch = u.Batch([m])
    for W in widths + widths[:2]:
        out = torch.zeros(m.max_bitstream_bytes(16, W), dtype=torch.uint8, device="cuda")
        (n,) = batch.encode([(0, frames[W], out)])
        assert out[:n].cpu().numpy().tobytes() == ref[W], W
    st = batch.stats()
    say(f"  plan cache: {st}")
    assert st["plans_cached"] <= 32 and st["plans_evicted"] >= 2 and st["plans_built"] == 36
    assert st["policy"] == 1                          # one launch per stage by default
    batch.close()
    m.close()
