"""Request server: each result is the same alone and in the mix (bitwise),
requests that arrive together are batched and overlap on two lanes, a
corrupt stream fails only its own request, and admission keeps the admitted
HBM footprint within the budget."""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from synthetic import stand_in_weights, video_chunk  # noqa: E402

SHAPES = [(0, 64, 64), (1, 96, 128), (0, 136, 80), (1, 64, 64), (0, 48, 200), (1, 128, 96)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pkg():
    import paper_2606_04410_amd as p
    return p


def models(prec):
    u = pkg()
    C = 64
    return [u.Codec(4, C, stand_in_weights(4, C), precision=prec, seg_log2=11, seg_log2_z=9,
                    model_tag=41, autotune=True),
            u.Codec(8, C, stand_in_weights(8, C), precision=prec, seg_log2=11, seg_log2_z=9,
                    model_tag=81, autotune=True)]


def collect(srv, n, timeout_s=60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < n:
        assert time.time() < t_end, f"only {len(got)} of {n} completions"
        for c in srv.poll(64, 200):
            got[c["ticket"]] = c
    return got


def references(ms, frames):
    ref_bs, ref_fr = [], []
    for (m, H, W), fr in zip(SHAPES, frames):
        bs, n = ms[m].encode(fr)
        ref_bs.append(bs[:n].clone())
        ref_fr.append(ms[m].decode(bs, n, H, W).clone())
    torch.cuda.synchronize()
    return ref_bs, ref_fr


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_server_results_equal_alone_and_in_the_mix(prec):
    u = pkg()
    ms = models(prec)
    frames = [torch.from_numpy(video_chunk(ms[m].T, H, W, 3, seed=11, chunk_id=i)).cuda()
              for i, (m, H, W) in enumerate(SHAPES)]
    ref_bs, ref_fr = references(ms, frames)
    say(f"server {prec}: {len(SHAPES)} encodes + {len(SHAPES)} decodes + 1 corrupt, 2 lanes")
    srv = u.Server(ms, lanes=2, max_batch=4, graph=True)
    enc_out = [torch.zeros(ms[m].max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
               for (m, H, W) in SHAPES]
    dec_out = [torch.full((ms[m].T, 3, H, W), -1.0, device="cuda") for (m, H, W) in SHAPES]
    bad = ref_bs[2].clone()
    bad[bad.numel() // 2] ^= 0x55
    bad_out = torch.zeros_like(ref_fr[2])
    tickets = {}
    for i, (m, H, W) in enumerate(SHAPES):   # interleaved kinds, submitted back to back
        tickets[srv.submit_encode(m, frames[i], enc_out[i], tag=i)] = ("enc", i)
        tickets[srv.submit_decode(m, ref_bs[i], ref_bs[i].numel(), H, W, dec_out[i], tag=100 + i)] = ("dec", i)
    tickets[srv.submit_decode(SHAPES[2][0], bad, bad.numel(), SHAPES[2][1], SHAPES[2][2], bad_out,
                              tag=999)] = ("bad", 2)
    got = collect(srv, len(tickets))
    sizes = []
    for t, (kind, i) in tickets.items():
        c = got[t]
        sizes.append(c["batch_size"])
        assert c["t_submit_us"] <= c["t_admit_us"] <= c["t_done_us"]
        if kind == "enc":
            assert c["status"] == 0 and c["len"] == ref_bs[i].numel()
            assert torch.equal(enc_out[i][:c["len"]], ref_bs[i]), i
        elif kind == "dec":
            assert c["status"] == 0
            assert torch.equal(dec_out[i], ref_fr[i]), i
        else:
            assert c["status"] == -3
    st = srv.stats()
    say(f"  batch sizes {sorted(sizes)}; stats {st}")
    assert max(sizes) > 1 and st["completed"] == len(tickets)
    assert st["peak_footprint"] <= st["budget"]
    srv.close()
    for m in ms:
        m.close()


def test_server_admission_by_hbm_footprint():
    u = pkg()
    ms = models("bf16")
    m, H, W = SHAPES[1]
    fr = torch.from_numpy(video_chunk(ms[m].T, H, W, 3, seed=12)).cuda()
    bs, n = ms[m].encode(fr)
    ref = ms[m].decode(bs, n, H, W).clone()
    # footprint of one such request, from a server with room to spare
    probe = u.Server(ms, lanes=1, max_batch=1)
    out = torch.empty_like(ref)
    probe.submit_decode(m, bs, n, H, W, out)
    collect(probe, 1)
    one = probe.stats()["peak_footprint"]
    probe.close()
    # a budget for one and a half requests: they are admitted one at a time
    srv = u.Server(ms, hbm_budget=int(1.5 * one), lanes=1, max_batch=8)
    outs = [torch.full_like(ref, -1.0) for _ in range(6)]
    ts = [srv.submit_decode(m, bs, n, H, W, o) for o in outs]
    got = collect(srv, len(ts))
    st = srv.stats()
    say(f"  one request {one} B, budget {st['budget']} B, peak {st['peak_footprint']} B, "
        f"batch sizes {[got[t]['batch_size'] for t in ts]}")
    assert st["peak_footprint"] <= st["budget"]
    assert all(got[t]["batch_size"] == 1 and got[t]["status"] == 0 for t in ts)
    for o in outs:
        assert torch.equal(o, ref)
    # a request that can never fit is refused at submission
    big = torch.empty((ms[1].T, 3, 512, 512), device="cuda")
    big_bs = torch.empty(ms[1].max_bitstream_bytes(512, 512), dtype=torch.uint8, device="cuda")
    with pytest.raises(u.UfvcError) as e:
        srv.submit_encode(1, big, big_bs)
    assert e.value.code == -2
    srv.close()
    for mm in ms:
        mm.close()


def test_server_c128_two_resolutions():
    """C = 128, T = 8, default segment sizes (the serving benchmark's
    configuration), two resolutions of the mix: every result is bitwise the
    single-chunk call's, alone and in the mix."""
    u = pkg()
    T, C = 8, 128
    codec = u.Codec(T, C, stand_in_weights(T, C), precision="bf16", model_tag=0x0C50_0000,
                    autotune=True)
    sizes = [(480, 832), (1088, 1920), (480, 832), (1088, 1920)]
    frames = [torch.from_numpy(video_chunk(T, H, W, 16, seed=13, chunk_id=i)).cuda()
              for i, (H, W) in enumerate(sizes)]
    ref_bs, ref_fr = [], []
    for (H, W), fr in zip(sizes, frames):
        bs, n = codec.encode(fr)
        ref_bs.append(bs[:n].clone())
        ref_fr.append(codec.decode(bs, n, H, W).clone())
    torch.cuda.synchronize()
    say(f"server C=128: {len(sizes)} encodes + {len(sizes)} decodes, {sizes}, lane 0 small-first")
    srv = u.Server([codec], lanes=2, max_batch=4, graph=True, small_pixels=832 * 480)
    enc_out = [torch.zeros(codec.max_bitstream_bytes(H, W), dtype=torch.uint8, device="cuda")
               for (H, W) in sizes]
    dec_out = [torch.full((T, 3, H, W), -1.0, device="cuda") for (H, W) in sizes]
    tickets = {}
    for rnd in range(2):      # the second round reuses the cached plans
        for i, (H, W) in enumerate(sizes):
            tickets[srv.submit_encode(0, frames[i], enc_out[i], tag=i)] = ("enc", i)
            tickets[srv.submit_decode(0, ref_bs[i], ref_bs[i].numel(), H, W, dec_out[i],
                                      tag=100 + i)] = ("dec", i)
        got = collect(srv, len(tickets), timeout_s=120.0)
        for t, (kind, i) in tickets.items():
            c = got[t]
            assert c["status"] == 0
            if kind == "enc":
                assert c["len"] == ref_bs[i].numel() and torch.equal(enc_out[i][:c["len"]], ref_bs[i])
            else:
                assert torch.equal(dec_out[i], ref_fr[i])
        say(f"  round {rnd}: batch sizes {sorted(got[t]['batch_size'] for t in tickets)}")
        for o in dec_out:
            o.fill_(-1.0)
        for o in enc_out:
            o.zero_()
        tickets = {}
    st = srv.stats()
    say(f"  stats {st}")
    assert st["peak_footprint"] <= st["budget"]
    assert st["arena_bytes"] == st["budget"]       # both lane arenas reserved up front
    srv.close()
    codec.close()
