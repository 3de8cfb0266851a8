"""The allocation-free rANS encoder (ufvc_rans_encode_noalloc) against the
allocating one (ufvc_rans_encode): same kernels, same bytes.

Two calls in a row, the second on a smaller input, so the second reads a
scratch array that still holds the first call's contents; then an input past
the fixed scratch, which must be refused without enqueuing work.  Both
streams are also checked against the oracle's coding of the same symbols."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import entropy, rans  # noqa: E402
from synthetic import stand_in_weights  # noqa: E402

FREQ, CUM = entropy.cdf_tables()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_bare(sym, idx, sl):
    segs = rans.encode(sym, idx, FREQ, CUM, 1 << sl)
    table = np.array([len(s) for s in segs], dtype="<u4").tobytes()
    return np.frombuffer(table + b"".join(segs), np.uint8)


def gauss_symbols(n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 64, n).astype(np.uint8)
    s = entropy.scales()[idx]
    sym = (np.clip(np.rint(rng.standard_normal(n) * s), -32, 32) + 32).astype(np.uint8)
    return sym, idx


def test_noalloc_encode_matches_allocating_encode():
    import paper_2606_04410_amd as ufvc
    c = ufvc.Codec(4, 64, stand_in_weights(4, 64), precision="fp32", seg_log2=13, seg_log2_z=10)
    try:
        for n, sl, seed in ((1_500_000, 13, 3), (70_001, 11, 4)):
            say(f"noalloc rans encode n={n} seg_log2={sl}")
            sym, idx = gauss_symbols(n, seed)
            dsym = torch.from_numpy(sym).cuda()
            didx = torch.from_numpy(idx).cuda()
            want = c.rans_encode(dsym, didx, sl).cpu().numpy()
            got = c.rans_encode_noalloc(dsym, didx, sl).cpu().numpy()
            assert got.size == want.size
            np.testing.assert_array_equal(got, want)
            if n < 100_000:
                np.testing.assert_array_equal(got, oracle_bare(sym, idx, sl))
            back = c.rans_decode(torch.from_numpy(got).cuda(), didx, sl)
            assert c.status() == 0
            np.testing.assert_array_equal(back.cpu().numpy(), sym)
        # past the fixed scratch: refused before any work is enqueued
        n = 20_000_000
        big = torch.full((n,), 32, dtype=torch.uint8, device="cuda")
        with pytest.raises(ufvc.UfvcError) as e:
            c.rans_encode_noalloc(big, big, 13)
        assert e.value.code == -7
    finally:
        c.close()
